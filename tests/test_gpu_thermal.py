"""The paper's "Thermal 1" rising bubble (section "Rising thermal bubble") on
the GPU: 100 x 200 x 200 cells over 10 km x 20 km x 20 km, dry air at rest at
constant potential temperature 300 K (discretely hydrostatic), a 2 K
cos^2 bubble of radius 2 km centred 2 km above the ground, run to t = 500 s.
Self-consistency only (the paper shows isolines, no numbers).  The claims
the paper makes about its figure "bub1" are checked:

* tau = 1 s: the bubble rises and keeps its mirror symmetry in theta and phi;
* tau = 0.2 s gives the same solution as tau = 1 s;
* a viscosity 1000 times that of air has almost no effect;
* tau = 50 s with K = 2 dissipates the bubble and slows it; K = 50 at
  tau = 50 s compensates part of that.

A reduced copy (10 x 20 x 20 cells) is checked against the oracle first.

"Thermal 2": 200^3 cells over a 1 km cube, a (1 + cos pi L)/4 K bubble of
radius 250 m centred 260 m above the ground; tau = 0.25 s and 1 s with K = 2
and 10, to t = 300 s (the paper does not state its final time).  Its claim:
the larger time step smooths the solution, and raising K removes most of
that.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
from gpu_common import compare
from paper_2004_13887_amd import inputs as I

pytestmark = pytest.mark.gpu

T_END = 500.0


@pytest.fixture(scope="module")
def dsw():
    from paper_2004_13887_amd import dsw as D
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    D.lib()
    return D


def test_thermal1_reduced_parity(dsw):
    g = I.thermal1_grid(10, 20, 20)
    U0 = I.thermal1_state(g)
    og, om = oracle.Grid(*g.args()), oracle.Material(*I.AIR.astuple())
    gg = dsw.Grid.from_spec(g, I.AIR)
    U = U0
    A, B = dsw.to_device(U0), gg.empty()
    for _ in range(3):
        U = oracle.split_step(og, om, U, 1.0, 2)
        gg.split_step(A, B, 1.0, 2)
        A, B = B, A
    torch.cuda.synchronize()
    gg.get_status()
    e = compare("thermal1 10x20x20, 3 steps", dsw.to_host(A), U, base=U0)
    assert max(e[k] for k in ("p", "ur", "ut", "uf", "T")) <= 1e-11


_runs = {}


def run(dsw, name, tau, K, mu=None):
    if name in _runs:
        return _runs[name]
    g = I.thermal1_grid()
    mat = I.AIR if mu is None else replace(I.AIR, mu=mu)
    gg = dsw.Grid.from_spec(g, mat)
    n = int(round(T_END / tau))
    print(f"[thermal1 {name}] tau={tau} K={K} mu={mat.mu} steps={n}", flush=True)
    A, B = dsw.to_device(I.thermal1_state(g)), gg.empty()
    for q in range(n):
        gg.split_step(A, B, tau, K)
        A, B = B, A
        if (q + 1) % 500 == 0:
            torch.cuda.synchronize()
            print(f"  step {q + 1}/{n}", flush=True)
    torch.cuda.synchronize()
    gg.get_status()
    U = dsw.to_host(A)
    dth = I.potential_temperature_excess(g, U)
    c = I.coords(g)
    z = (c["rc"] - g.r1)[:, None, None]
    m = dth > 0.1
    out = {"dth": dth, "max": float(dth.max()), "zc": float((dth * z)[m].sum() / dth[m].sum()),
           "wmax": float(U["ur"].max())}
    print(f"  max dTheta {out['max']:.4f} K, centroid height {out['zc']:.1f} m, max u_r {out['wmax']:.3f} m/s",
          flush=True)
    _runs[name] = out
    return out


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_thermal1_rises_symmetric(dsw):
    base = run(dsw, "tau1", 1.0, 2)
    dth = base["dth"]
    sym_t = rel(dth[:, ::-1, :], dth)
    sym_p = rel(dth[:, :, ::-1], dth)
    print(f"  mirror asymmetry: theta {sym_t:.2e}, phi {sym_p:.2e}", flush=True)
    assert base["zc"] > 3.5e3 and base["wmax"] > 5.0  # from 2 km at rest (measured 4.4 km, 16 m/s)
    assert sym_t < 1e-9 and sym_p < 1e-9


def test_thermal1_small_tau_same(dsw):
    base, fine = run(dsw, "tau1", 1.0, 2), run(dsw, "tau0.2", 0.2, 2)
    d = rel(fine["dth"], base["dth"])
    print(f"  tau 0.2 vs 1: dTheta rel L2 {d:.3e}, centroid {fine['zc']:.1f} vs {base['zc']:.1f} m", flush=True)
    assert d < 0.06 and abs(fine["zc"] - base["zc"]) < 50.0


def test_thermal1_viscosity_no_effect(dsw):
    base, visc = run(dsw, "tau1", 1.0, 2), run(dsw, "mu1e-2", 1.0, 2, mu=1.846e-2)
    d = rel(visc["dth"], base["dth"])
    print(f"  mu x1000 vs air: dTheta rel L2 {d:.3e}, centroid {visc['zc']:.1f} vs {base['zc']:.1f} m", flush=True)
    assert d < 0.02 and abs(visc["zc"] - base["zc"]) < 20.0


def test_thermal1_large_tau_dissipates(dsw):
    base = run(dsw, "tau1", 1.0, 2)
    big = run(dsw, "tau50K2", 50.0, 2)
    bigk = run(dsw, "tau50K50", 50.0, 50)
    d2, d50 = rel(big["dth"], base["dth"]), rel(bigk["dth"], base["dth"])
    print(f"  tau 50: K=2 max {big['max']:.3f} centroid {big['zc']:.1f} (rel {d2:.3f}); "
          f"K=50 max {bigk['max']:.3f} centroid {bigk['zc']:.1f} (rel {d50:.3f}); "
          f"tau 1: max {base['max']:.3f} centroid {base['zc']:.1f}", flush=True)
    # K = 2: dissipated and slowed down
    assert big["max"] < 0.85 * base["max"] and big["zc"] < base["zc"] - 1.0e3
    # K = 50: part of that recovered, still different from tau = 1
    assert bigk["zc"] > big["zc"] + 1.0e3 and d50 < d2 and d50 > 0.1


_runs2 = {}


def run2(dsw, tau, K, t_end=300.0):
    key = (tau, K)
    if key in _runs2:
        return _runs2[key]
    g = I.thermal2_grid()
    gg = dsw.Grid.from_spec(g, I.AIR)
    n = int(round(t_end / tau))
    print(f"[thermal2] tau={tau} K={K} steps={n}", flush=True)
    A, B = dsw.to_device(I.thermal2_state(g)), gg.empty()
    for q in range(n):
        gg.split_step(A, B, tau, K)
        A, B = B, A
        if (q + 1) % 400 == 0:
            torch.cuda.synchronize()
            print(f"  step {q + 1}/{n}", flush=True)
    torch.cuda.synchronize()
    gg.get_status()
    U = dsw.to_host(A)
    dth = I.potential_temperature_excess(g, U)
    c = I.coords(g)
    z = (c["rc"] - g.r1)[:, None, None]
    m = dth > 0.02
    out = {"dth": dth, "max": float(dth.max()), "zc": float((dth * z)[m].sum() / dth[m].sum()),
           "wmax": float(U["ur"].max())}
    print(f"  max dTheta {out['max']:.4f} K, centroid height {out['zc']:.1f} m, max u_r {out['wmax']:.3f} m/s",
          flush=True)
    _runs2[key] = out
    return out


def test_thermal2_time_step_and_iterations(dsw):
    ref = run2(dsw, 0.25, 2)
    k2 = run2(dsw, 1.0, 2)
    k10 = run2(dsw, 1.0, 10)
    d2, d10 = rel(k2["dth"], ref["dth"]), rel(k10["dth"], ref["dth"])
    print(f"  tau 1 vs 0.25: K=2 rel {d2:.3e} (max {k2['max']:.4f}), K=10 rel {d10:.3e} "
          f"(max {k10['max']:.4f}); tau 0.25 max {ref['max']:.4f}, centroid {ref['zc']:.1f} m", flush=True)
    assert ref["zc"] > 350.0  # risen from 260 m
    assert k2["max"] < 0.9 * ref["max"]  # smoothed by the larger step
    assert d10 < 0.4 * d2 and k10["max"] > k2["max"]  # mostly restored by K = 10
