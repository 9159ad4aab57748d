"""Pins of the oracle's line systems and line solvers (CPU only).

* block / scalar / cyclic Thomas agree with dense LU (numpy) on random
  diagonally dominant systems and on the oracle's own assembled lines
  (paper, end of section 2: block-tridiagonal Thomas per line);
* the assembled line matrices equal I + tau/2 N_d(Ubar; .) applied by the
  operator form (the line matrices are the direction-d part of the operator,
  eqs. (dr), (dtheta), (dphi)), including wall ghosts, poles and the periodic
  wrap.
"""
import numpy as np
import pytest

import oracle
from helpers import AIR, grid_of, random_state, random_wall, rel, small_sector, small_sphere
from paper_2004_13887_amd import inputs as I


def dense_from_blocks(L, D, U, cyclic):
    n, bs = D.shape[0], D.shape[1]
    A = np.zeros((n * bs, n * bs))
    for i in range(n):
        A[i * bs:(i + 1) * bs, i * bs:(i + 1) * bs] = D[i]
        if i > 0 or cyclic:
            j = (i - 1) % n
            A[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] += L[i]
        if i < n - 1 or cyclic:
            j = (i + 1) % n
            A[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] += U[i]
    return A


@pytest.mark.parametrize("bs", [1, 3])
@pytest.mark.parametrize("cyclic", [False, True])
@pytest.mark.parametrize("n", [3, 4, 7, 16])
def test_block_solvers_vs_dense_lu(bs, cyclic, n):
    rng = np.random.Generator(np.random.PCG64(1000 * n + 10 * bs + cyclic))
    L = rng.uniform(-1, 1, (n, bs, bs))
    U = rng.uniform(-1, 1, (n, bs, bs))
    D = rng.uniform(-1, 1, (n, bs, bs)) + np.eye(bs) * (2.5 * bs + 1.0)
    b = rng.uniform(-1, 1, (n, bs))
    x = oracle.block_solve(L, D, U, b, cyclic=cyclic)
    A = dense_from_blocks(L, D, U, cyclic)
    xd = np.linalg.solve(A, b.ravel())
    assert np.max(np.abs(x.ravel() - xd)) <= 1e-13 * max(1.0, np.max(np.abs(xd)))


def _line_cases(spec):
    """(d, kind, a, b) for a few lines of every family, including boundary ones"""
    nr, nt, np_ = spec.nr, spec.nt, spec.np
    kf = [0, np_ // 2, np_ - 1] if spec.periodic else [1, np_ // 2, np_ - 1]
    cases = []
    for (j, k) in [(0, 0), (nt // 2, np_ // 2), (nt - 1, np_ - 1)]:
        cases.append((0, -1, j, k))
    for (f, k) in [(1, 0), (nt - 1, np_ - 1)]:
        cases.append((0, 2, f, k))
    for f in kf:
        cases.append((0, 3, 0, f))
    for (i, k) in [(0, 0), (nr - 1, np_ // 2)]:
        cases.append((1, -1, i, k))
    for (f, k) in [(1, 0), (nr - 1, np_ - 1)]:
        cases.append((1, 1, f, k))
    for f in kf:
        cases.append((1, 3, nr - 1, f))
    for (i, j) in [(0, 0), (nr - 1, nt - 1), (nr // 2, nt // 2)]:
        cases.append((2, -1, i, j))
    for (f, j) in [(1, 0), (nr - 1, nt - 1)]:
        cases.append((2, 1, f, j))
    for (i, f) in [(0, 1), (nr - 1, nt - 1)]:
        cases.append((2, 2, i, f))
    return cases


@pytest.mark.parametrize("which", ["sector", "sphere"])
def test_assembled_lines_vs_dense_lu(which):
    spec = small_sector() if which == "sector" else small_sphere()
    g = grid_of(spec)
    U, tau = random_state(spec, 11)
    wall = random_wall(spec, 12, 0.3) if which == "sector" else None
    rhs = I.random_fields(spec, 13, scale=1.0)
    for d in range(3):
        x = oracle.line_solve(g, AIR, U, tau, d, rhs, wall=wall)
        for (dd, kind, a, b) in _line_cases(spec):
            if dd != d:
                continue
            L, D, Uu, idx, fid, cyc = oracle.line_blocks(g, AIR, U, tau, d, kind, a, b, wall=wall)
            A = dense_from_blocks(L, D, Uu, cyc)
            names = oracle.FIELDS
            bvec = np.array([rhs[names[f]].ravel()[i] if i >= 0 else 0.0 for f, i in zip(fid, idx)])
            xd = np.linalg.solve(A, bvec)
            xo = np.array([x[names[f]].ravel()[i] if i >= 0 else 0.0 for f, i in zip(fid, idx)])
            scale = np.maximum(np.abs(xd), 1e-300)
            assert np.max(np.abs(xo - xd) / np.maximum(scale, np.max(np.abs(xd)) * 1e-3)) < 1e-10, \
                (d, kind, a, b)


@pytest.mark.parametrize("which", ["sector", "sphere"])
def test_line_matrices_are_direction_operators(which):
    """(I + tau/2 D_d) x from the assembled blocks == x + tau/2 N_d(Ubar; x)."""
    spec = small_sector() if which == "sector" else small_sphere()
    g = grid_of(spec)
    U, tau = random_state(spec, 21)
    wall = random_wall(spec, 22, 0.3) if which == "sector" else None
    x = I.random_fields(spec, 23)
    for d, mask in enumerate((oracle.MASK_R, oracle.MASK_T, oracle.MASK_F)):
        y = oracle.line_matvec(g, AIR, U, tau, d, x, wall=wall)
        N = oracle.apply(g, AIR, U, x, mask, wall_u=wall, wall_v=None)
        for k in oracle.FIELDS:
            ref = x[k] + 0.5 * tau * N[k]
            from helpers import unknown_mask
            m = unknown_mask(spec, k)
            assert rel(y[k][m], ref[m]) < 1e-13, (which, d, k)


def test_line_solve_inverts_line_matvec():
    spec = small_sphere(5, 6, 9)
    g = grid_of(spec)
    U, tau = random_state(spec, 31)
    rhs = I.random_fields(spec, 32)
    for d in range(3):
        x = oracle.line_solve(g, AIR, U, tau, d, rhs)
        y = oracle.line_matvec(g, AIR, U, tau, d, x)
        for k in oracle.FIELDS:
            assert rel(y[k], rhs[k]) < 1e-12, (d, k)


def _all_lines(g, d):
    """every line of direction d as (kind, a, b): block lines (kind -1), then
    the two scalar families (kind = the field id), as the full solve has them"""
    FR, FT, FF = 1, 2, 3
    kf = range(0, g.np) if g.periodic else range(1, g.np)
    if d == 0:
        out = [(-1, j, k) for j in range(g.nt) for k in range(g.np)]
        out += [(FT, f, k) for f in range(1, g.nt) for k in range(g.np)]
        out += [(FF, j, f) for j in range(g.nt) for f in kf]
    elif d == 1:
        out = [(-1, i, k) for i in range(g.nr) for k in range(g.np)]
        out += [(FR, f, k) for f in range(1, g.nr) for k in range(g.np)]
        out += [(FF, i, f) for i in range(g.nr) for f in kf]
    else:
        out = [(-1, i, j) for i in range(g.nr) for j in range(g.nt)]
        out += [(FR, f, j) for f in range(1, g.nr) for j in range(g.nt)]
        out += [(FT, i, f) for i in range(g.nr) for f in range(1, g.nt)]
    return np.array(out, dtype=np.int64).T


@pytest.mark.parametrize("which", ["sector", "sphere"])
def test_sampled_residual_equals_the_full_residual(which):
    """residual_at, the point-sample checker of the full-size GPU tests, gives
    the full residual's value at every point of every field, bit for bit
    (boundary-normal faces included, where both are 0)"""
    spec = small_sector() if which == "sector" else small_sphere()
    g = grid_of(spec)
    Un, tau = random_state(spec, 91, mach=0.05)
    rng = np.random.Generator(np.random.PCG64(92))
    Uk = {k: v + 1e-3 * np.abs(v).mean() * rng.uniform(-1, 1, v.shape) for k, v in Un.items()}
    wall = random_wall(spec, 93) if which == "sector" else None
    R, Ub = oracle.residual(g, AIR, Un, Uk, tau, wall=wall)
    for k, fid in oracle.FID.items():
        idx = np.arange(R[k].size)
        got = oracle.residual_at(g, AIR, Un, Uk, Ub, tau, np.full(idx.size, fid), idx, wall=wall)
        assert np.array_equal(got, R[k].ravel()), k


@pytest.mark.parametrize("which", ["sector", "sphere"])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_line_solve_of_some_lines_equals_the_full_solve(which, d):
    """line_solve_some, the line-sample checker of the full-size GPU tests,
    solves every line of the full solve, bit for bit, and writes nothing
    outside the lines it is given"""
    spec = small_sector() if which == "sector" else small_sphere()
    g = grid_of(spec)
    Ub, tau = random_state(spec, 94, mach=0.05)
    rng = np.random.Generator(np.random.PCG64(95))
    rhs = {k: rng.uniform(-1, 1, s) for k, s in g.shapes().items()}
    for k in ("ur", "ut", "uf"):
        rhs[k][~oracle_unknowns(g, k)] = 0.0
    wall = random_wall(spec, 96) if which == "sector" else None
    full = oracle.line_solve(g, AIR, Ub, tau, d, rhs, wall=wall)
    kinds, a, b = _all_lines(g, d)
    some = oracle.line_solve_some(g, AIR, Ub, tau, d, kinds, a, b, rhs, wall=wall)
    for k in full:
        m = oracle_unknowns(g, k)
        assert np.array_equal(some[k][m], full[k][m]), k
    # half of the lines: the other half's unknowns stay untouched (NaN)
    half = slice(0, None, 2)
    part = oracle.line_solve_some(g, AIR, Ub, tau, d, kinds[half], a[half], b[half], rhs, wall=wall)
    touched = sum(int(np.sum(~np.isnan(v))) for v in part.values())
    total = sum(int(np.sum(oracle_unknowns(g, k))) for k in full)
    assert 0 < touched < total
    for k in full:
        ok = ~np.isnan(part[k])
        assert np.array_equal(part[k][ok], full[k][ok]), k


def oracle_unknowns(g, key):
    """points that are unknowns (not boundary-normal faces)"""
    sh = g.shapes()[key]
    m = np.ones(sh, dtype=bool)
    if key == "ur":
        m[0] = m[-1] = False
    if key == "ut":
        m[:, 0] = m[:, -1] = False
    if key == "uf" and not g.periodic:
        m[:, :, 0] = m[:, :, -1] = False
    return m
