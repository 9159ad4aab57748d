"""GPU perturbation-pressure step and Courant numbers against the oracle
(paper section 3.1, the remark after Table 3 on rescaling the pressure a
priori; section 3.2 on small or adaptive time steps).

Inputs from the seeded generators; expected values from the oracle's
perturbation step (oracle.split_step_pert), whose pins are in
test_oracle_pert.py.  Bar: relative L2 per field <= 1e-11 on the state and on
its change from U^n (here p holds p - p_bar, so the p bar is on the
perturbation itself, far stricter than on the full pressure).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_common import compare
from paper_2004_13887_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-11
FIELDS = ("p", "ur", "ut", "uf", "T")
ROT_GAS = I.MaterialSpec(cp=1000.0, cv=713.0, pi_inf=2.0e4, mu=2.0, prandtl=0.71, omega=5.0e-3,
                         g_r=9.80665)
CASES = {
    "parity": I.WORKLOADS["parity"],
    "sector-ragged": I.Workload("sector-ragged", I.sector(13, 29, 37, math.radians(25) / 29,
                                                          math.radians(31) / 37),
                                mach=1e-2, amplitude=0.5, steps=1, K=3, seed=77),
    "sphere-rot-gas": I.Workload("sphere-rot-gas", I.full_sphere(6, 12, 16), mach=1e-2,
                                 amplitude=0.5, steps=1, K=3, seed=85, material=ROT_GAS),
    "sector-low-mach": I.Workload("sector-low-mach", I.sector(8, 10, 12, 4e-4, 5e-4), mach=1e-6,
                                  amplitude=0.5, steps=1, K=3, seed=87),
    # 16384 (r, theta) slots: the phi pass as two launches, the r sweep
    # partitioned in two launches, as on the global grid
    "sphere-split": I.Workload("sphere-split", I.full_sphere(128, 128, 32), mach=1e-4,
                               amplitude=0.5, steps=1, K=3, seed=86),
}


@pytest.fixture(scope="module")
def dsw():
    from paper_2004_13887_amd import dsw as D
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    D.lib()
    return D


def _pert_state(w):
    U0, tau = I.initial_state(w)
    pbar, Tbar = I.reference_column(w.grid, w.material, I.T0)
    Up = dict(U0)
    Up["p"] = np.ascontiguousarray(U0["p"] - pbar[:, None, None])
    return U0, Up, pbar, Tbar, tau


@pytest.mark.parametrize("name", list(CASES))
def test_perturbation_step_parity(name, dsw):
    w = CASES[name]
    print(f"[pert] {name} {w.grid.nr}x{w.grid.nt}x{w.grid.np} M={w.mach}", flush=True)
    _, Up, pbar, Tbar, tau = _pert_state(w)
    og, om = oracle.Grid(*w.grid.args()), oracle.Material(*w.material.astuple())
    ref = oracle.split_step_pert(og, om, Up, pbar, Tbar, tau, w.K)
    gg = dsw.Grid.from_spec(w.grid, w.material)
    gg.set_reference(pbar, Tbar)
    d0, d1 = dsw.to_device(Up), gg.empty()
    gg.split_step_pert(d0, d1, tau, w.K)
    torch.cuda.synchronize()
    gg.get_status()
    e = compare(f"[pert] {name}", dsw.to_host(d1), ref, base=Up)
    assert max(e[k] for k in FIELDS) <= TOL
    assert max(e[k + "_change"] for k in FIELDS) <= TOL


def test_perturbation_step_equals_plain_step(dsw):
    """the same scheme: p' + p_bar after the step equals the plain step's p
    to rounding of the plain form"""
    w = CASES["sphere-rot-gas"]
    U0, Up, pbar, Tbar, tau = _pert_state(w)
    gg = dsw.Grid.from_spec(w.grid, w.material)
    gg.set_reference(pbar, Tbar)
    a, b = gg.empty(), gg.empty()
    gg.split_step(dsw.to_device(U0), a, tau, w.K)
    gg.split_step_pert(dsw.to_device(Up), b, tau, w.K)
    torch.cuda.synchronize()
    A, B = dsw.to_host(a), dsw.to_host(b)
    for k in FIELDS:
        full = B[k] + (pbar[:, None, None] if k == "p" else 0.0)
        d, ch = np.abs(full - A[k]).max(), np.abs(A[k] - U0[k]).max()
        print(f"[pert] plain vs perturbation {k}: {d:.3e} (change {ch:.3e})", flush=True)
        assert d <= 1e-10 * ch + 4 * np.spacing(np.abs(A[k]).max()), k


def test_rest_state_kept_bit_for_bit(dsw):
    w = CASES["parity"]
    g = w.grid
    _, tau = I.initial_state(w)
    pbar, Tbar = I.reference_column(g, w.material, I.T0)
    sh = g.shapes()
    rest = {k: np.zeros(sh[k]) for k in FIELDS}
    rest["T"] = np.full(sh["T"], I.T0)
    gg = dsw.Grid.from_spec(g, w.material)
    gg.set_reference(pbar, Tbar)
    out = gg.empty()
    gg.split_step_pert(dsw.to_device(rest), out, tau, 3)
    torch.cuda.synchronize()
    O = dsw.to_host(out)
    for k in FIELDS:
        assert np.array_equal(O[k], rest[k]), k


def test_reference_checks(dsw):
    w = CASES["parity"]
    gg = dsw.Grid.from_spec(w.grid, w.material)
    U0, Up, pbar, Tbar, tau = _pert_state(w)
    with pytest.raises(dsw.DswError):  # no reference yet
        gg.split_step_pert(dsw.to_device(Up), gg.empty(), tau, 3)
    bad = Tbar.copy()
    bad[3] = -1.0
    with pytest.raises(dsw.DswError):
        gg.set_reference(pbar, bad)
    with pytest.raises(ValueError):
        gg.set_reference(pbar[:-1], Tbar[:-1])


@pytest.mark.parametrize("name", ["parity", "sphere-rot-gas", "sector-ragged"])
def test_courant_parity(name, dsw):
    w = CASES[name]
    U0, tau = I.initial_state(w)
    og, om = oracle.Grid(*w.grid.args()), oracle.Material(*w.material.astuple())
    ref = oracle.courant(og, om, U0, tau)
    gg = dsw.Grid.from_spec(w.grid, w.material)
    got = gg.courant(dsw.to_device(U0), tau)
    print(f"[courant] {name}: gpu {got} oracle {ref}", flush=True)
    for a, b in zip(got, ref):
        assert math.isclose(a, b, rel_tol=1e-14)
    # the acoustic number is the workload's CFL where T peaks at the
    # smallest spacing's cell... at least it never exceeds it
    assert got[1] <= w.cfl * (1 + 1e-12)


def test_adaptive_step_holds_the_advective_courant_number(dsw):
    """A time-step controller on the Courant numbers (paper section 3.2):
    tau_{n+1} = min(tau_max, tau_n * target / C_adv(U^{n+1}, tau_n)).  As a
    warm bubble accelerates the step shrinks; every step taken starts at an
    advective Courant number at most the target."""
    # 4 km x 4 km x 10 km, 250 m horizontal cells, a 5 K bubble
    w = I.Workload("adaptive", I.sector(16, 16, 16, 250.0 / I.EARTH_R1, 250.0 / I.EARTH_R1),
                   mach=1e-3, amplitude=5.0, steps=1, K=3, seed=91)
    U0, tau_ac = I.initial_state(w)
    gg = dsw.Grid.from_spec(w.grid, w.material)
    target, tau_max = 0.05, 4.0 * tau_ac
    a, b = dsw.to_device(U0), gg.empty()
    tau = min(tau_max, target / gg.courant(a, 1.0)[0])
    taus = []
    for n in range(6):
        c0 = gg.courant(a, tau)[0]
        assert c0 <= target * (1 + 1e-12)
        gg.split_step(a, b, tau, 3)
        gg.get_status()
        taus.append(tau)
        c1 = gg.courant(b, tau)[0]
        tau = min(tau_max, tau * target / c1)
        a, b = b, a
    print(f"[adaptive] taus {['%.3g' % t for t in taus]}", flush=True)
    assert all(t > 0 for t in taus)
    assert taus[-1] < 0.5 * taus[0]  # the bubble accelerates: the step shrinks
