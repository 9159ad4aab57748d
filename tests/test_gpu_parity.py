"""GPU parity of every C-ABI entry point against the CPU oracle.

Inputs come from the seeded generators only; expected values from the oracle
only.  Bar: relative L2 per field <= 1e-11 for the time step (FP64 end to
end); the intermediate residual and sweep outputs are held to the same bar.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import compare, small_cases
from paper_2004_13887_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-11


def residual_errors(tag, got, ref, tau, w):
    """Relative L2 of R per field.  The u_r row of F_h subtracts the
    hydrostatic pressure gradient from gravity, two terms of size g that cancel
    to the (much smaller) buoyancy; its FP64 rounding error therefore scales
    with tau*g, so that row is measured against max(|R|, tau g sqrt(n))."""
    out = {}
    for k in ("p", "ur", "ut", "uf", "T"):
        d = np.linalg.norm(got[k] - ref[k])
        s = np.linalg.norm(ref[k])
        if k == "ur":
            s = max(s, tau * abs(w.material.g_r) * np.sqrt(ref[k].size))
        out[k] = float(d / s) if s > 0 else float(d)
        print(f"{tag} R {k}: rel err={out[k]:.3e}", flush=True)
    return out


@pytest.fixture(scope="module")
def dsw():
    from paper_2004_13887_amd import dsw as D
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    D.lib()
    return D


def _setup(w, dsw):
    U0, tau = I.initial_state(w)
    og = oracle.Grid(*w.grid.args())
    om = oracle.Material(*w.material.astuple())
    gg = dsw.Grid.from_spec(w.grid, w.material)
    return U0, tau, og, om, gg


CASES = small_cases()
# every material term the atmospheric cases leave at zero: rotation about the
# polar axis (Coriolis), a stiffened gas (pi_inf) and a larger viscosity
ROT_GAS = I.MaterialSpec(cp=1000.0, cv=713.0, pi_inf=2.0e4, mu=2.0, prandtl=0.71, omega=5.0e-3,
                         g_r=9.80665)
CASES["sector-rot-gas"] = I.Workload("sector-rot-gas", I.sector(7, 12, 17, 4e-4, 5e-4), mach=1e-2,
                                     amplitude=0.5, steps=1, K=3, seed=84, material=ROT_GAS)
# 16384 (r, theta) slots: the phi pass runs as the two launches (block lines,
# then scalar lines) that the global grid takes
CASES["sphere-split"] = I.Workload("sphere-split", I.full_sphere(128, 128, 32), mach=1e-4,
                                   amplitude=0.5, steps=1, K=3, seed=86)
CASES["sphere-rot-gas"] = I.Workload("sphere-rot-gas", I.full_sphere(6, 12, 16), mach=1e-2,
                                     amplitude=0.5, steps=1, K=3, seed=85, material=ROT_GAS)


@pytest.mark.parametrize("name", list(CASES))
def test_residual_parity(name, dsw):
    w = CASES[name]
    print(f"[residual] {name} {w.grid.nr}x{w.grid.nt}x{w.grid.np}", flush=True)
    U0, tau, og, om, gg = _setup(w, dsw)
    Uk = I.random_fields(w.grid, 5, base=U0, scale=1e-3 * w.mach * 347.0)
    Uk["p"] = U0["p"] * (1.0 + 1e-6 * I.random_fields(w.grid, 6)["p"])
    Uk["T"] = np.ascontiguousarray(U0["T"] + 1e-3 * I.random_fields(w.grid, 7)["T"])
    R_o, Ub_o = oracle.residual(og, om, U0, Uk, tau)
    dUn, dUk = dsw.to_device(U0), dsw.to_device(Uk)
    R, Ub = gg.empty(), gg.empty()
    gg.residual(dUn, dUk, tau, R, Ub)
    torch.cuda.synchronize()
    gg.get_status()
    e1 = residual_errors(name, dsw.to_host(R), R_o, tau, w)
    e2 = compare(f"{name} Ubar", dsw.to_host(Ub), Ub_o)
    assert max(e1.values()) <= TOL and max(e2.values()) <= TOL


# (direction, r/theta solver): 4 the partitioned solver (the default), 0 the
# two-ended one; the phi sweep has its own
SOLVERS = [(0, 4), (0, 0), (1, 4), (1, 0), (2, 4)]


@pytest.mark.parametrize("d,rt", SOLVERS)
@pytest.mark.parametrize("name", list(CASES))
def test_line_solve_parity(name, d, rt, dsw):
    w = CASES[name]
    print(f"[line_solve d={d} rt={rt}] {name}", flush=True)
    U0, tau, og, om, gg = _setup(w, dsw)
    gg.set_config(rows_per_thread_r=rt, rows_per_thread_theta=rt)
    rhs = I.random_fields(w.grid, 11 + d)
    x_o = oracle.line_solve(og, om, U0, tau, d, rhs)
    x = gg.empty()
    for v in x.values():
        v.fill_(123.0)  # boundary faces must be overwritten with 0
    gg.line_solve(d, dsw.to_device(U0), tau, dsw.to_device(rhs), x)
    torch.cuda.synchronize()
    gg.get_status()
    e = compare(f"{name} x{d}", dsw.to_host(x), x_o)
    assert max(e.values()) <= TOL


@pytest.mark.parametrize("rt", [4, 0])
@pytest.mark.parametrize("name", list(CASES))
def test_split_step_parity(name, rt, dsw):
    w = CASES[name]
    print(f"[split_step rt={rt}] {name} K={w.K}", flush=True)
    U0, tau, og, om, gg = _setup(w, dsw)
    gg.set_config(rows_per_thread_r=rt, rows_per_thread_theta=rt)
    U1_o = oracle.split_step(og, om, U0, tau, w.K)
    dU0 = dsw.to_device(U0)
    dU1 = gg.empty()
    gg.split_step(dU0, dU1, tau, w.K)
    torch.cuda.synchronize()
    gg.get_status()
    U1 = dsw.to_host(dU1)
    e = compare(f"{name} U1", U1, U1_o, base=U0)
    assert max(e[k] for k in ("p", "ur", "ut", "uf", "T")) <= TOL
    # the change from U^n too: at low Mach the full p field cannot see it
    assert max(e[k + "_change"] for k in ("p", "ur", "ut", "uf", "T")) <= TOL
    # input untouched
    for k, v in dsw.to_host(dU0).items():
        assert np.array_equal(v, U0[k])


def test_split_step_bitwise_reproducible(dsw):
    w = CASES["sphere-ragged"]
    U0, tau, og, om, gg = _setup(w, dsw)
    dU0 = dsw.to_device(U0)
    a, b = gg.empty(), gg.empty()
    gg.split_step(dU0, a, tau, 3)
    gg.split_step(dU0, b, tau, 3)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k
