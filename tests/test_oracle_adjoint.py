"""Pins of the complex-step oracle that the GPU adjoint is checked against.

The complex-step build is the same C source compiled with a complex state
type.  Its real part must reproduce the FP64 oracle bit for bit, and its
imaginary part (the directional derivative) must agree with central finite
differences of the FP64 oracle and be linear in the direction."""
import numpy as np
import pytest

import oracle
from helpers import AIR, grid_of, random_state, small_sector, small_sphere
from paper_2004_13887_amd import inputs as I

FIELDS = ("p", "ur", "ut", "uf", "T")
SCALE = {"p": 1.0, "ur": 1e-2, "ut": 1e-2, "uf": 1e-2, "T": 1e-2}


def direction(spec, seed):
    """a random direction with physical scales per field, boundary faces
    included"""
    rng = np.random.Generator(np.random.PCG64(seed))
    return {k: SCALE[k] * rng.uniform(-1.0, 1.0, s) for k, s in spec.shapes().items()}


def rel(a, b):
    num = sum(np.linalg.norm(a[k] - b[k]) ** 2 for k in FIELDS) ** 0.5
    den = sum(np.linalg.norm(b[k]) ** 2 for k in FIELDS) ** 0.5
    return num / den


@pytest.mark.parametrize("spec", [small_sector(), small_sphere()], ids=["sector", "sphere"])
def test_real_part_is_the_fp64_oracle(spec):
    g = grid_of(spec)
    U, tau = random_state(spec, 3)
    V = direction(spec, 4)
    U1, _ = oracle.jvp_split_step(g, AIR, U, V, tau, 3)
    ref = oracle.split_step(g, AIR, U, tau, 3)
    for k in FIELDS:
        assert np.array_equal(U1[k], ref[k]), k
    R, _ = oracle.jvp_residual(g, AIR, U, V, tau)
    Rref, _ = oracle.residual(g, AIR, U, U, tau)
    for k in FIELDS:
        assert np.array_equal(R[k], Rref[k]), k
    X = I.random_fields(spec, 5)
    for d in range(3):
        y, _ = oracle.jvp_line_matvec(g, AIR, U, V, tau, d, X)
        yref = oracle.line_matvec(g, AIR, U, tau, d, X)
        for k in FIELDS:
            assert np.array_equal(y[k], yref[k]), (d, k)


def _fd(fn, U, V, eps):
    """fourth-order central difference along V"""
    f = {s: fn({k: U[k] + s * eps * V[k] for k in FIELDS}) for s in (-2, -1, 1, 2)}
    return {k: (f[-2][k] - 8.0 * f[-1][k] + 8.0 * f[1][k] - f[2][k]) / (12.0 * eps) for k in FIELDS}


def _best_fd_error(fn, U, V, exact):
    """smallest error of the fourth-order difference over step sizes spanning
    the trade-off between truncation and rounding"""
    return min(rel(_fd(fn, U, V, eps), exact) for eps in (1e-3, 1e-2, 1e-1))


@pytest.mark.parametrize("spec", [small_sector(), small_sphere()], ids=["sector", "sphere"])
def test_derivatives_match_central_differences(spec):
    g = grid_of(spec)
    U, tau = random_state(spec, 6)
    V = direction(spec, 7)
    _, dU1 = oracle.jvp_split_step(g, AIR, U, V, tau, 3)
    e = _best_fd_error(lambda W: oracle.split_step(g, AIR, W, tau, 3), U, V, dU1)
    print("split step: complex step vs central difference", e)
    assert e < 1e-9
    _, dR = oracle.jvp_residual(g, AIR, U, V, tau)
    e = _best_fd_error(lambda W: oracle.residual(g, AIR, W, W, tau)[0], U, V, dR)
    print("residual:", e)
    assert e < 1e-9
    X = I.random_fields(spec, 8)
    for d in range(3):
        _, dy = oracle.jvp_line_matvec(g, AIR, U, V, tau, d, X)
        e = _best_fd_error(lambda W: oracle.line_matvec(g, AIR, W, tau, d, X), U, V, dy)
        print(f"line operator d={d}:", e)
        assert e < 1e-9


def test_derivative_is_linear_in_the_direction():
    spec = small_sphere()
    g = grid_of(spec)
    U, tau = random_state(spec, 9)
    V1, V2 = direction(spec, 10), direction(spec, 11)
    V3 = {k: 2.0 * V1[k] - 3.0 * V2[k] for k in FIELDS}
    _, d1 = oracle.jvp_split_step(g, AIR, U, V1, tau, 2)
    _, d2 = oracle.jvp_split_step(g, AIR, U, V2, tau, 2)
    _, d3 = oracle.jvp_split_step(g, AIR, U, V3, tau, 2)
    comb = {k: 2.0 * d1[k] - 3.0 * d2[k] for k in FIELDS}
    assert rel(d3, comb) < 1e-12


def test_boundary_faces_pass_through():
    """U^{n+1} copies the boundary-normal faces of U^n: the derivative along
    a direction that moves only those faces is that direction there"""
    spec = small_sector()
    g = grid_of(spec)
    U, tau = random_state(spec, 12)
    V = {k: np.zeros(s) for k, s in spec.shapes().items()}
    V["ur"][0] = 1.0
    V["ur"][-1] = -2.0
    _, d = oracle.jvp_split_step(g, AIR, U, V, tau, 2)
    assert np.array_equal(d["ur"][0], V["ur"][0]) and np.array_equal(d["ur"][-1], V["ur"][-1])
