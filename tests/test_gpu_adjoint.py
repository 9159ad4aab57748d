"""GPU adjoint of the split step against the complex-step oracle.

The complex-step oracle gives exact Jacobian-vector products J v of the
oracle's own step (pinned in test_oracle_adjoint.py); the GPU adjoint gives
J^T lam.  Every piece is checked by the identity <J^T lam, v> = <lam, J v> on
random lam and v, and on tiny grids the whole transposed Jacobian is built
column by column and compared entry by entry.  Bar: 1e-10 relative."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import small_cases
from paper_2004_13887_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-10
FIELDS = ("p", "ur", "ut", "uf", "T")
SCALE = {"p": 1.0, "ur": 1e-2, "ut": 1e-2, "uf": 1e-2, "T": 1e-2}
CASES = small_cases()
NAMES = ["parity", "sector-ragged", "sphere-ragged", "sphere-chunks16", "sector-min", "sphere-min"]


@pytest.fixture(scope="module")
def dsw():
    from paper_2004_13887_amd import dsw as D
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    D.lib()
    return D


def direction(spec, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return {k: SCALE[k] * rng.uniform(-1.0, 1.0, s) for k, s in spec.shapes().items()}


def cotangent(spec, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return {k: rng.uniform(-1.0, 1.0, s) / SCALE[k] for k, s in spec.shapes().items()}


def dot(a, b):
    return float(sum(np.dot(np.ravel(a[k]), np.ravel(b[k])) for k in FIELDS))


def check_dot(tag, lhs, rhs):
    e = abs(lhs - rhs) / max(abs(lhs), abs(rhs), 1e-300)
    print(f"{tag}: <J^T lam, v> = {lhs:.15e}  <lam, J v> = {rhs:.15e}  rel {e:.2e}", flush=True)
    assert e <= TOL


def _setup(name, dsw):
    w = CASES[name]
    U0, tau = I.initial_state(w)
    og = oracle.Grid(*w.grid.args())
    om = oracle.Material(*w.material.astuple())
    gg = dsw.Grid.from_spec(w.grid, w.material)
    return w, U0, tau, og, om, gg


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("name", NAMES)
def test_transposed_line_solve(name, d, dsw):
    print(f"[line_solve_T d={d}] {name}", flush=True)
    w, U0, tau, og, om, gg = _setup(name, dsw)
    b = I.random_fields(w.grid, 21 + d)
    y = cotangent(w.grid, 31 + d)
    xb = oracle.line_solve(og, om, U0, tau, d, b)
    xT = gg.empty()
    gg.line_solve_T(d, dsw.to_device(U0), tau, dsw.to_device(y), xT)
    torch.cuda.synchronize()
    gg.get_status()
    check_dot(f"{name} M_{d}^-T", dot(dsw.to_host(xT), b), dot(y, xb))


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("name", NAMES)
def test_line_operator_vjp(name, d, dsw):
    print(f"[line_vjp d={d}] {name}", flush=True)
    w, U0, tau, og, om, gg = _setup(name, dsw)
    X = I.random_fields(w.grid, 41 + d, scale=1e-3)
    mu = cotangent(w.grid, 51 + d)
    V = direction(w.grid, 61 + d)
    _, dy = oracle.jvp_line_matvec(og, om, U0, V, tau, d, X)
    acc = gg.empty()
    gg.line_vjp(d, dsw.to_device(U0), tau, dsw.to_device(X), dsw.to_device(mu), acc)
    torch.cuda.synchronize()
    gg.get_status()
    check_dot(f"{name} dM_{d}", dot(dsw.to_host(acc), V), dot(mu, dy))


@pytest.mark.parametrize("name", NAMES)
def test_residual_vjp(name, dsw):
    print(f"[residual_vjp] {name}", flush=True)
    w, U0, tau, og, om, gg = _setup(name, dsw)
    mu = cotangent(w.grid, 71)
    V = direction(w.grid, 72)
    _, dR = oracle.jvp_residual(og, om, U0, V, tau)
    acc = gg.empty()
    gg.residual_vjp(dsw.to_device(U0), tau, dsw.to_device(mu), acc)
    torch.cuda.synchronize()
    gg.get_status()
    check_dot(f"{name} dR", dot(dsw.to_host(acc), V), dot(mu, dR))


@pytest.mark.parametrize("name", NAMES)
def test_adjoint_step_dot_product(name, dsw):
    print(f"[adjoint_step] {name}", flush=True)
    w, U0, tau, og, om, gg = _setup(name, dsw)
    lam = cotangent(w.grid, 81)
    V = direction(w.grid, 82)
    _, dU1 = oracle.jvp_split_step(og, om, U0, V, tau, w.K)
    out = gg.empty()
    gg.adjoint_step(dsw.to_device(U0), tau, w.K, dsw.to_device(lam), out)
    torch.cuda.synchronize()
    gg.get_status()
    check_dot(f"{name} J^T (K={w.K})", dot(dsw.to_host(out), V), dot(lam, dU1))


@pytest.mark.parametrize("phi", [0, 2])
@pytest.mark.parametrize("name", ["sector-ragged", "sphere-chunks16", "sphere-chunks2"])
def test_adjoint_step_other_phi_solvers(name, phi, dsw):
    """the adjoint with the phi lines solved one thread per line (0) or
    partitioned with 2 rows per thread"""
    print(f"[adjoint_step phi={phi}] {name}", flush=True)
    w, U0, tau, og, om, gg = _setup(name, dsw)
    gg.set_config(64, 128, 128, phi)
    lam = cotangent(w.grid, 83)
    V = direction(w.grid, 84)
    _, dU1 = oracle.jvp_split_step(og, om, U0, V, tau, w.K)
    out = gg.empty()
    gg.adjoint_step(dsw.to_device(U0), tau, w.K, dsw.to_device(lam), out)
    torch.cuda.synchronize()
    gg.get_status()
    check_dot(f"{name} J^T phi={phi}", dot(dsw.to_host(out), V), dot(lam, dU1))


@pytest.mark.parametrize("name", ["sector-min", "sphere-min", "sphere-chunks2"])
def test_adjoint_step_dense_tiny(name, dsw):
    """the whole transposed Jacobian on a tiny grid, entry by entry: 3x3x3
    sector and sphere, and a 4x5x8 full sphere whose phi lines go through the
    partitioned transposed solver (two chunks, cyclic reduction)"""
    print(f"[adjoint dense] {name}", flush=True)
    w, U0, tau, og, om, gg = _setup(name, dsw)
    shapes = w.grid.shapes()
    sizes = [int(np.prod(shapes[k])) for k in FIELDS]
    n = sum(sizes)
    J = np.zeros((n, n))
    col = 0
    for q, k in enumerate(FIELDS):
        for e in range(sizes[q]):
            V = {kk: np.zeros(shapes[kk]) for kk in FIELDS}
            V[k].reshape(-1)[e] = 1.0
            _, d = oracle.jvp_split_step(og, om, U0, V, tau, w.K)
            J[:, col] = np.concatenate([d[kk].ravel() for kk in FIELDS])
            col += 1
    lam = cotangent(w.grid, 91)
    ref = J.T @ np.concatenate([lam[k].ravel() for k in FIELDS])
    out = gg.empty()
    gg.adjoint_step(dsw.to_device(U0), tau, w.K, dsw.to_device(lam), out)
    torch.cuda.synchronize()
    got = np.concatenate([dsw.to_host(out)[k].ravel() for k in FIELDS])
    e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"{name}: {n} unknowns, rel L2 of J^T lam = {e:.2e}", flush=True)
    assert e <= TOL


def test_autograd_function(dsw):
    """torch.autograd through SplitStep: the gradient of <w, U^{n+1}> is the
    adjoint step applied to w"""
    w, U0, tau, og, om, gg = _setup("sphere-ragged", dsw)
    Ud = {k: v.clone().requires_grad_(True) for k, v in dsw.to_device(U0).items()}
    wt = cotangent(w.grid, 101)
    U1 = dsw.split_step_fn(gg, Ud, tau, w.K)
    loss = sum((U1[k] * torch.as_tensor(wt[k], device="cuda")).sum() for k in FIELDS)
    loss.backward()
    V = direction(w.grid, 102)
    _, dU1 = oracle.jvp_split_step(og, om, U0, V, tau, w.K)
    grad = {k: Ud[k].grad.cpu().numpy() for k in FIELDS}
    check_dot("autograd", dot(grad, V), dot(wt, dU1))


@pytest.mark.parametrize("name", ["parity", "sphere-ragged", "sector-min"])
def test_taped_step_and_adjoint(name, dsw):
    """dsw_split_step_taped computes what dsw_split_step computes (the same
    kernels: bitwise) and fills the tape; dsw_adjoint_step_taped from it
    gives the adjoint of dsw_adjoint_step (up to the order of the atomic
    sums) and passes the oracle's dot-product check"""
    print(f"[taped] {name}", flush=True)
    w, U0, tau, og, om, gg = _setup(name, dsw)
    per = sum(int(np.prod(s)) for s in w.grid.shapes().values())
    assert gg.tape_bytes(w.K) == 4 * w.K * per * 8
    Ud = dsw.to_device(U0)
    plain, taped = gg.empty(), gg.empty()
    tape = gg.new_tape(w.K)
    gg.split_step(Ud, plain, tau, w.K)
    gg.split_step_taped(Ud, taped, tau, w.K, tape)
    lam = cotangent(w.grid, 111)
    a1, a2 = gg.empty(), gg.empty()
    gg.adjoint_step(Ud, tau, w.K, dsw.to_device(lam), a1)
    gg.adjoint_step_taped(Ud, tau, w.K, tape, dsw.to_device(lam), a2)
    torch.cuda.synchronize()
    gg.get_status()
    for k in FIELDS:
        assert torch.equal(plain[k], taped[k]), k
    h1, h2 = dsw.to_host(a1), dsw.to_host(a2)
    e = max(np.linalg.norm(h1[k] - h2[k]) / max(np.linalg.norm(h1[k]), 1e-300) for k in FIELDS)
    print(f"{name}: taped vs recomputed adjoint rel L2 {e:.2e}", flush=True)
    assert e <= 1e-12
    V = direction(w.grid, 112)
    _, dU1 = oracle.jvp_split_step(og, om, U0, V, tau, w.K)
    check_dot(f"{name} taped J^T", dot(h2, V), dot(lam, dU1))


def test_autograd_taped(dsw):
    """SplitStep with taped=True: the same gradient as with the recompute"""
    w, U0, tau, og, om, gg = _setup("sphere-ragged", dsw)
    wt = cotangent(w.grid, 121)
    grads = []
    for taped in (False, True):
        Ud = {k: v.clone().requires_grad_(True) for k, v in dsw.to_device(U0).items()}
        U1 = dsw.split_step_fn(gg, Ud, tau, w.K, taped=taped)
        U2 = dsw.split_step_fn(gg, U1, tau, w.K, taped=taped)  # two steps: two tapes
        loss = sum((U2[k] * torch.as_tensor(wt[k], device="cuda")).sum() for k in FIELDS)
        loss.backward()
        grads.append({k: Ud[k].grad.cpu().numpy() for k in FIELDS})
    e = max(np.linalg.norm(grads[0][k] - grads[1][k]) / np.linalg.norm(grads[0][k]) for k in FIELDS)
    print(f"autograd taped vs recomputed: rel L2 {e:.2e}", flush=True)
    assert e <= 1e-12


@pytest.mark.parametrize("name,nsteps", [("parity", 3), ("sphere-ragged", 3), ("sector-min", 1)])
def test_adjoint_trajectory(name, nsteps, dsw):
    """dsw_adjoint_trajectory over N steps from per-step checkpoints: the
    oracle's dot-product identity <lam_0, V> = <lam_end, J_{N-1} ... J_0 V>
    (the checkpoints are the oracle's own states, the J V products its
    complex-step JVPs), and N chained dsw_adjoint_step calls up to the order
    of the atomic sums; a second call gives the same result"""
    print(f"[trajectory] {name} N={nsteps}", flush=True)
    w, U0, tau, og, om, gg = _setup(name, dsw)
    V = direction(w.grid, 131)
    states, dU = [U0], V
    for _ in range(nsteps):
        U1, dU = oracle.jvp_split_step(og, om, states[-1], dU, tau, w.K)
        states.append(U1)
    ck = [dsw.to_device(u) for u in states[:-1]]
    lam = cotangent(w.grid, 132)
    lam_d = dsw.to_device(lam)
    t1, t2 = gg.empty(), gg.empty()
    gg.adjoint_trajectory(ck, tau, w.K, lam_d, t1)
    gg.adjoint_trajectory(ck, tau, w.K, lam_d, t2)
    chained = lam_d
    for n in range(nsteps - 1, -1, -1):
        nxt = gg.empty()
        gg.adjoint_step(ck[n], tau, w.K, chained, nxt)
        chained = nxt
    torch.cuda.synchronize()
    gg.get_status()
    h1, h2, hc = dsw.to_host(t1), dsw.to_host(t2), dsw.to_host(chained)
    for other, tag in ((hc, "chained adjoint_step"), (h2, "second call")):
        e = max(np.linalg.norm(h1[k] - other[k]) / max(np.linalg.norm(other[k]), 1e-300) for k in FIELDS)
        print(f"{name}: trajectory vs {tag} rel L2 {e:.2e}", flush=True)
        assert e <= 1e-12
    check_dot(f"{name} trajectory J^T (N={nsteps}, K={w.K})", dot(h1, V), dot(lam, dU))


def test_adjoint_trajectory_bad_args(dsw):
    w, U0, tau, og, om, gg = _setup("sector-min", dsw)
    ck = [dsw.to_device(U0)]
    lam, out = dsw.to_device(cotangent(w.grid, 141)), gg.empty()
    for tag, call in (("no checkpoints", lambda: gg.adjoint_trajectory([], tau, w.K, lam, out)),
                      ("lam_0 is a checkpoint", lambda: gg.adjoint_trajectory(ck, tau, w.K, lam, ck[0])),
                      ("K=0", lambda: gg.adjoint_trajectory(ck, tau, 0, lam, out)),
                      ("lam_0 is lam_end", lambda: gg.adjoint_trajectory(ck, tau, w.K, lam, lam))):
        with pytest.raises(dsw.DswError) as ei:
            call()
        assert ei.value.code == dsw.DSW_EINVAL, tag
        print(f"{tag}: {ei.value}", flush=True)


def test_adjoint_on_a_caller_stream(dsw):
    """dsw_adjoint_step and dsw_adjoint_trajectory on a stream of the
    caller's: their second-stream work is ordered before the caller's next
    work on that stream (a copy queued right after each call sees the whole
    result)"""
    w, U0, tau, og, om, gg = _setup("parity", dsw)
    Ud = dsw.to_device(U0)
    lam = dsw.to_device(cotangent(w.grid, 151))
    nxt = gg.empty()
    gg.split_step(Ud, nxt, tau, w.K)
    ck = [Ud, nxt]
    ref, tref = gg.empty(), gg.empty()
    gg.adjoint_step(Ud, tau, w.K, lam, ref)
    gg.adjoint_trajectory(ck, tau, w.K, lam, tref)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        a, t = gg.empty(), gg.empty()
        gg.adjoint_step(Ud, tau, w.K, lam, a, stream=s)
        a_cp = {k: v.clone() for k, v in a.items()}
        gg.adjoint_trajectory(ck, tau, w.K, lam, t, stream=s)
        t_cp = {k: v.clone() for k, v in t.items()}
    torch.cuda.synchronize()
    gg.get_status()
    for got, want, tag in ((a_cp, ref, "adjoint_step"), (t_cp, tref, "adjoint_trajectory")):
        e = max(float(torch.linalg.norm(got[k] - want[k]) / torch.linalg.norm(want[k])) for k in FIELDS)
        print(f"{tag} on a caller stream: rel L2 {e:.2e}", flush=True)
        assert e <= 1e-12
