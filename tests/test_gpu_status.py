"""Device status words through the C-ABI: a finite non-positive temperature
is DSW_ENONPHYS, a NaN or an infinity in the state (or an iteration that
diverged) gives a non-finite residual, DSW_EDIVERGED; reading the status
clears it.  The planted values are ordinary FP64 inputs: every kernel runs
to its end, the status words record what it met."""
import math

import pytest
import torch

from paper_2004_13887_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dsw():
    from paper_2004_13887_amd import dsw as D
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    D.lib()
    return D


W = I.WORKLOADS["parity"]


def _step(dsw, U, K=2):
    gg = dsw.Grid.from_spec(W.grid, W.material)
    _, tau = I.initial_state(W)
    out = gg.empty()
    gg.split_step(dsw.to_device(U), out, tau, K)
    torch.cuda.synchronize()
    return gg, out, tau


@pytest.mark.parametrize("field,index,value,code", [
    ("T", (3, 7, 9), -1.0, "DSW_ENONPHYS"),
    ("ur", (5, 7, 9), math.nan, "DSW_EDIVERGED"),
    ("uf", (8, 20, 11), math.inf, "DSW_EDIVERGED"),
    ("p", (0, 0, 0), math.nan, "DSW_EDIVERGED"),
])
def test_status_reports_the_planted_value(field, index, value, code, dsw):
    print(f"[status] {field}{index} = {value} -> {code}", flush=True)
    U0, _ = I.initial_state(W)
    U = {k: v.copy() for k, v in U0.items()}
    U[field][index] = value
    gg, _, tau = _step(dsw, U)
    with pytest.raises(dsw.DswError) as ei:
        gg.get_status()
    assert ei.value.code == getattr(dsw, code), str(ei.value)
    # read and cleared: a clean step on the same handle reports nothing
    out = gg.empty()
    gg.split_step(dsw.to_device(U0), out, tau, 2)
    torch.cuda.synchronize()
    assert gg.get_status() == dsw.DSW_OK
    assert all(bool(torch.isfinite(v).all()) for v in out.values())


def test_ensemble_status_names_the_member_error(dsw):
    specs = [W.grid, I.sector(8, 12, 16, 0.004, 0.004)]
    E = dsw.Ensemble(specs, [W.material, W.material])
    U, taus = [], []
    for q, g in enumerate(specs):
        u, tau = I.initial_state(I.Workload(f"m{q}", g, mach=1e-2, amplitude=0.5, steps=1, K=2,
                                            seed=900 + q))
        U.append(dsw.to_device(u))
        taus.append(tau)
    U[1]["ut"][3, 5, 7] = float("nan")
    out = [g.empty() for g in E.members]
    E.ensemble_step(U, out, taus, 2)
    torch.cuda.synchronize()
    with pytest.raises(dsw.DswError) as ei:
        E.get_status()
    assert ei.value.code == dsw.DSW_EDIVERGED
    assert E.get_status() == dsw.DSW_OK
