"""Gradient of a ten-step objective through the GPU adjoint, checked against
central finite differences of the GPU forward step (the adjoint workload:
64 x 128 x 256 cells, 100 m horizontal spacing, Mach 1e-2, checkpoint every
step).

Objective: J = sum over the cells of a 5 x 5 x 2 km box around the bubble of
Theta * V_cell at the final time, Theta = T / (p / p00)^(R/c_p).  Gradient
with respect to the initial cell-centred Theta0 (T0 = Theta0 (p0/p00)^(R/c_p),
p0 fixed), by torch.autograd through the SplitStep function (backward =
dsw_adjoint_step).  Each of 32 seeded directions v is checked:
(J(Theta0 + e v) - J(Theta0 - e v)) / 2e, differenced cell by cell before the
sum, against <dJ/dTheta0, v>; the best of e = 1e-2, 1e-3, 1e-4 K must agree
to 1e-6."""
import numpy as np
import pytest
import torch

from paper_2004_13887_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("p", "ur", "ut", "uf", "T")


@pytest.fixture(scope="module")
def dsw():
    from paper_2004_13887_amd import dsw as D
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    D.lib()
    return D


def test_adjoint_gradient_matches_finite_differences(dsw):
    w = I.WORKLOADS["adjoint"]
    mat = w.material
    U0, tau = I.initial_state(w)
    print(f"[adjoint fd] {w.grid.np}x{w.grid.nt}x{w.grid.nr}, {w.steps} steps, tau={tau:.4f}",
          flush=True)
    grid = dsw.Grid.from_spec(w.grid, mat)
    dev = dsw.to_device(U0)
    wts = torch.as_tensor(I.adjoint_box_weights(w), device="cuda")
    ex0 = torch.as_tensor(I.exner(U0["p"], mat), device="cuda")
    theta0 = dev["T"] / ex0

    def run(th, grad=False):
        U = dict(dev)
        U["T"] = th * ex0
        for _ in range(w.steps):
            U = dsw.split_step_fn(grid, U, tau, w.K) if grad else _step(U)
        return U

    def _step(U):
        out = grid.empty()
        grid.split_step(U, out, tau, w.K)
        return out

    def theta(U):
        return U["T"] / ((U["p"] / I.P00) ** (mat.R / mat.cp))

    th = theta0.clone().requires_grad_(True)
    UT = run(th, grad=True)
    J = (wts * theta(UT)).sum()
    J.backward()
    grad = th.grad.detach()
    grid.get_status()
    print(f"[adjoint fd] J = {float(J):.6e}", flush=True)
    worst = 0.0
    with torch.no_grad():
        for jd, v in enumerate(I.adjoint_directions(theta0.shape)):
            vt = torch.as_tensor(v, device="cuda")
            ad = float((grad * vt).sum())
            errs = []
            for eps in (1e-2, 1e-3, 1e-4):
                tp, tm = theta(run(theta0 + eps * vt)), theta(run(theta0 - eps * vt))
                fd = float((wts * (tp - tm)).sum()) / (2.0 * eps)
                errs.append(abs(fd - ad) / abs(ad))
            best = min(errs)
            worst = max(worst, best)
            print(f"[adjoint fd] direction {jd:2d}: <grad, v> = {ad:.10e}, best rel err {best:.2e}",
                  flush=True)
            assert best <= 1e-6
    print(f"[adjoint fd] worst over 32 directions: {worst:.2e}", flush=True)


def test_trajectory_matches_autograd(dsw):
    """dsw_adjoint_trajectory over the workload's ten checkpoints, started
    from lam_N = dJ/dU^N, gives the gradient of J with respect to every field
    of U^0 that the autograd function (one dsw_adjoint_step per step) gives,
    up to the order of the atomic sums"""
    w = I.WORKLOADS["adjoint"]
    mat = w.material
    U0, tau = I.initial_state(w)
    grid = dsw.Grid.from_spec(w.grid, mat)
    wts = torch.as_tensor(I.adjoint_box_weights(w), device="cuda")

    def objective(U):
        return (wts * (U["T"] / ((U["p"] / I.P00) ** (mat.R / mat.cp)))).sum()

    leaf = {k: v.clone().requires_grad_(True) for k, v in dsw.to_device(U0).items()}
    U = leaf
    for _ in range(w.steps):
        U = dsw.split_step_fn(grid, U, tau, w.K)
    objective(U).backward()
    ref = {k: leaf[k].grad.detach() for k in FIELDS}
    ck = [dsw.to_device(U0)]
    for _ in range(w.steps):
        nxt = grid.empty()
        grid.split_step(ck[-1], nxt, tau, w.K)
        ck.append(nxt)
    UN = {k: v.clone().requires_grad_(True) for k, v in ck[-1].items()}
    objective(UN).backward()
    lam_end = {k: (UN[k].grad.detach().contiguous() if UN[k].grad is not None else torch.zeros_like(UN[k]))
               for k in FIELDS}
    lam0 = grid.empty()
    grid.adjoint_trajectory(ck[:-1], tau, w.K, lam_end, lam0)
    torch.cuda.synchronize()
    grid.get_status()
    for k in FIELDS:
        nr = float(torch.linalg.norm(ref[k]))
        e = float(torch.linalg.norm(lam0[k] - ref[k])) / max(nr, 1e-300)
        print(f"[trajectory] {k}: |grad| {nr:.3e}, rel L2 vs autograd {e:.2e}", flush=True)
        assert e <= 1e-12 or nr == 0.0
