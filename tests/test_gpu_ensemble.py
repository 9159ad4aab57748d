"""Batched ensembles of uneven grids: one launch per pass over all members,
replayed from a HIP graph, against the oracle and against per-member
dsw_split_step calls.  The batched and the per-member kernels run the same
per-point code, built with multiply-adds fused only within one source
expression, so the two give the same bits; replays of one graph too."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_common import compare
from paper_2004_13887_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-11
K = 3
FIELDS = ("p", "ur", "ut", "uf", "T")


@pytest.fixture(scope="module")
def dsw():
    from paper_2004_13887_amd import dsw as D
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    D.lib()
    return D


def small_members():
    """sectors and full spheres of uneven sizes; the last sphere's phi lines
    (12 cells, 3 chunks of 4) fall back to one thread per line, so the phi
    pass of the batch has two launches"""
    def sec(nr, nt, np_, seed):
        return I.Workload(f"sec{seed}", I.sector(nr, nt, np_, math.radians(20) / nt,
                                                 math.radians(24) / np_),
                          mach=1e-2, amplitude=0.5, steps=1, K=K, seed=seed)

    def sph(nr, nt, np_, seed):
        return I.Workload(f"sph{seed}", I.full_sphere(nr, nt, np_), mach=1e-3, amplitude=0.5,
                          steps=1, K=K, seed=seed)

    return [sec(5, 7, 9, 301), sph(4, 6, 8, 302), sec(4, 6, 12, 303), sph(5, 8, 12, 304),
            sec(3, 9, 5, 305), sph(6, 10, 16, 306)]


def _make(dsw, ws):
    E = dsw.Ensemble([w.grid for w in ws], [w.material for w in ws])
    states = [I.initial_state(w) for w in ws]
    U0 = [s[0] for s in states]
    taus = [s[1] for s in states]
    return E, U0, taus


def _per_member(E, dU0, taus):
    out = []
    for m, g in enumerate(E.members):
        o = g.empty()
        g.split_step(dU0[m], o, taus[m], K)
        out.append(o)
    return out


SAME = 1e-13


def _assert_same(a, b, tag):
    """bitwise equal (the relative L2 is printed first, to show the size of
    any difference)"""
    for m, (x, y) in enumerate(zip(a, b)):
        for k in x:
            d = float(torch.linalg.vector_norm(x[k] - y[k]))
            n = float(torch.linalg.vector_norm(y[k]))
            r = d / n if n > 0 else d
            assert r <= SAME, f"{tag}: member {m} field {k}: rel L2 {r:.3e}"
            assert torch.equal(x[k], y[k]), f"{tag}: member {m} field {k}: rel L2 {r:.3e}, not bitwise"


def _assert_bitwise(a, b, tag):
    for m, (x, y) in enumerate(zip(a, b)):
        for k in x:
            assert torch.equal(x[k], y[k]), f"{tag}: member {m} field {k}"


def test_ensemble_matches_oracle_and_member_steps(dsw):
    ws = small_members()
    print("[ensemble] members:", [(w.grid.nr, w.grid.nt, w.grid.np, w.grid.periodic) for w in ws],
          flush=True)
    E, U0, taus = _make(dsw, ws)
    dU0 = [dsw.to_device(u) for u in U0]
    out = [g.empty() for g in E.members]
    E.ensemble_step(dU0, out, taus, K)
    torch.cuda.synchronize()
    E.get_status()
    ref = _per_member(E, dU0, taus)
    torch.cuda.synchronize()
    _assert_same(out, ref, "ensemble vs split_step")
    for m, w in enumerate(ws):
        og = oracle.Grid(*w.grid.args())
        om = oracle.Material(*w.material.astuple())
        U1_o = oracle.split_step(og, om, U0[m], taus[m], K)
        e = compare(f"member {m}", dsw.to_host(out[m]), U1_o, base=U0[m])
        assert max(e[k] for k in FIELDS) <= TOL


def test_members_whose_theta_sweeps_plan_different_passes(dsw):
    """theta lines of 256 rows take the two-ended solver with the scalar
    lines in a partitioned pass of their own; 200 rows, the two-ended solver
    in one pass (its chunks would not fill a workgroup); 64 rows, the
    partitioned solver.  The members' passes stay aligned in the batched
    plan: bitwise equal to their own steps, and against the oracle."""
    def sec(nr, nt, np_, seed):
        return I.Workload(f"sec{seed}", I.sector(nr, nt, np_, math.radians(20) / nt,
                                                 math.radians(24) / np_),
                          mach=1e-2, amplitude=0.5, steps=1, K=K, seed=seed)

    ws = [sec(4, 200, 6, 312), sec(4, 256, 8, 311), sec(5, 64, 10, 313)]
    print("[ensemble] theta passes:", [(w.grid.nr, w.grid.nt, w.grid.np) for w in ws], flush=True)
    E, U0, taus = _make(dsw, ws)
    dU0 = [dsw.to_device(u) for u in U0]
    out = [g.empty() for g in E.members]
    E.ensemble_step(dU0, out, taus, K)
    torch.cuda.synchronize()
    E.get_status()
    ref = _per_member(E, dU0, taus)
    torch.cuda.synchronize()
    _assert_same(out, ref, "ensemble vs split_step")
    for m, w in enumerate(ws):
        og = oracle.Grid(*w.grid.args())
        om = oracle.Material(*w.material.astuple())
        U1_o = oracle.split_step(og, om, U0[m], taus[m], K)
        e = compare(f"member {m}", dsw.to_host(out[m]), U1_o, base=U0[m])
        assert max(e[k] for k in FIELDS) <= TOL


def test_graph_replays_and_ping_pong(dsw):
    """replay the captured graph several times with eager work and
    synchronisations in between; alternate two pointer sets (two graphs)"""
    ws = small_members()
    E, U0, taus = _make(dsw, ws)
    A = [dsw.to_device(u) for u in U0]
    B = [g.empty() for g in E.members]
    refA = [{k: v.clone() for k, v in a.items()} for a in A]
    refB = [g.empty() for g in E.members]
    first = None
    for step in range(4):
        src, dst = (A, B) if step % 2 == 0 else (B, A)
        rsrc, rdst = (refA, refB) if step % 2 == 0 else (refB, refA)
        E.ensemble_step(src, dst, taus, K)
        torch.cuda.synchronize()
        if step == 0:
            first = [{k: v.clone() for k, v in d.items()} for d in dst]
        junk = torch.randn(1 << 16, device="cuda", dtype=torch.float64).sum()  # eager work
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for m, g in enumerate(E.members):
            g.split_step(rsrc[m], rdst[m], taus[m], K)
        torch.cuda.synchronize()
        print(f"[ensemble] replay step {step}", flush=True)
        _assert_same(dst, rdst, f"step {step}")
    # replay the first graph once more from the original input: same bits
    A0 = [dsw.to_device(u) for u in U0]
    B0 = [g.empty() for g in E.members]
    E.ensemble_step(A0, B0, taus, K)
    for m in range(len(A)):
        for k in A[m]:
            A[m][k].copy_(A0[m][k])
    E.ensemble_step(A, B, taus, K)
    torch.cuda.synchronize()
    _assert_bitwise(B0, first, "graph for new pointers vs first graph")
    _assert_bitwise(B, first, "replay of the first graph")
    E.get_status()


def test_configs_give_oracle_parity(dsw):
    """every launch shape the autotuner may pick, on a single grid"""
    ws = small_members()
    for cfg in ((64, 128, 128, 4, 4, 4), (128, 64, 256, 2, 4, 0), (256, 256, 64, 0, 0, 4),
                (64, 256, 128, 4, 0, 0), (128, 128, 128, 4, -1, -1)):
        for m in (1, 3, 2):
            w = ws[m]
            g = dsw.Grid.from_spec(w.grid, w.material)
            g.set_config(*cfg)
            assert g.get_config() == cfg
            U0, tau = I.initial_state(w)
            d0, d1 = dsw.to_device(U0), g.empty()
            g.split_step(d0, d1, tau, K)
            torch.cuda.synchronize()
            g.get_status()
            og = oracle.Grid(*w.grid.args())
            om = oracle.Material(*w.material.astuple())
            U1_o = oracle.split_step(og, om, U0, tau, K)
            e = compare(f"cfg {cfg} member {m}", dsw.to_host(d1), U1_o, base=U0)
            assert max(e[k] for k in FIELDS) <= TOL


def test_bad_config_rejected(dsw):
    w = small_members()[0]
    g = dsw.Grid.from_spec(w.grid, w.material)
    with pytest.raises(dsw.DswError):
        g.set_config(96, 128, 128, 4)
    with pytest.raises(dsw.DswError):
        g.set_config(64, 128, 128, 3)
    with pytest.raises(dsw.DswError):
        g.set_config(64, 128, 128, 4, 2, 4)
    with pytest.raises(dsw.DswError):
        g.set_config(64, 128, 128, 4, 4, 8)
    with pytest.raises(dsw.DswError):
        g.set_config(64, 128, 128, 4, 8, 0)
    assert g.get_config() == (64, 256, 256, 4, -1, -1)


def test_autotuner_then_bitwise_member_equality(dsw):
    ws = small_members()
    E, U0, taus = _make(dsw, ws)
    dU0 = [dsw.to_device(u) for u in U0]
    out = [g.empty() for g in E.members]
    cfg = E.ensemble_tune(dU0, out, taus, K, reps=1)
    print("[ensemble] tuned config", cfg, flush=True)
    assert cfg[0] in (64, 128, 256) and cfg[1] in (64, 128, 256) and cfg[2] in (64, 128, 256)
    assert cfg[3] in (0, 2, 4) and cfg[4] in (-1, 0, 4) and cfg[5] in (-1, 0, 4)
    assert E.get_config() == cfg
    assert all(g.get_config() == cfg for g in E.members)
    E.ensemble_step(dU0, out, taus, K)
    ref = _per_member(E, dU0, taus)
    torch.cuda.synchronize()
    E.get_status()
    _assert_same(out, ref, "tuned ensemble vs split_step")
    w = ws[3]
    og = oracle.Grid(*w.grid.args())
    om = oracle.Material(*w.material.astuple())
    U1_o = oracle.split_step(og, om, U0[3], taus[3], K)
    e = compare("tuned member 3", dsw.to_host(out[3]), U1_o, base=U0[3])
    assert max(e[k] for k in FIELDS) <= TOL


def test_recipe_members_full_size(dsw):
    """three members of the 64-member ensemble recipe at their real sizes:
    batched step equal to per-member split_step calls to rounding"""
    ws = I.ensemble_members()[:3]
    print("[ensemble] recipe members:", [(w.grid.nr, w.grid.nt, w.grid.np) for w in ws], flush=True)
    E, U0, taus = _make(dsw, ws)
    dU0 = [dsw.to_device(u) for u in U0]
    del U0
    out = [g.empty() for g in E.members]
    E.ensemble_step(dU0, out, taus, K)
    ref = _per_member(E, dU0, taus)
    torch.cuda.synchronize()
    E.get_status()
    _assert_same(out, ref, "recipe members")
    for m in range(len(ws)):
        assert all(bool(torch.isfinite(v).all()) for v in out[m].values())
        assert not all(torch.equal(out[m][k], dU0[m][k]) for k in out[m])


def test_bad_ensemble_arguments(dsw):
    ws = small_members()[:2]
    E, U0, taus = _make(dsw, ws)
    dU0 = [dsw.to_device(u) for u in U0]
    out = [g.empty() for g in E.members]
    with pytest.raises(dsw.DswError):
        E.ensemble_step(dU0, dU0, taus, K)           # Unp1 aliases Un
    with pytest.raises(dsw.DswError):
        E.ensemble_step(dU0, [out[0], out[0]], taus, K)  # two members, one output
    with pytest.raises(dsw.DswError):
        E.ensemble_step(dU0, out, [taus[0], -1.0], K)


def test_graph_on_a_caller_stream(dsw):
    """the two-lane graph launched on a stream of the caller's: work queued on
    that stream right after the launch (a copy of the outputs) sees the whole
    step"""
    ws = small_members()
    E, U0, taus = _make(dsw, ws)
    dU0 = [dsw.to_device(u) for u in U0]
    ref = _per_member(E, dU0, taus)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        out = [g.empty() for g in E.members]
        for rep in range(2):  # capture, then a replay
            E.ensemble_step(dU0, out, taus, K, stream=s)
            cp = [{k: v.clone() for k, v in o.items()} for o in out]
            for o in out:
                for v in o.values():
                    v.fill_(7.0)
    torch.cuda.synchronize()
    E.get_status()
    _assert_same(cp, ref, "graph on a caller stream")
