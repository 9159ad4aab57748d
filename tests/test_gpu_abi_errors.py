"""Error paths of the C-ABI (include/dsw.h): every invalid descriptor,
material or argument is refused with DSW_EINVAL and a message from
dsw_last_error, before any kernel is launched; a refused call leaves its
outputs untouched."""
import ctypes as C
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


GOOD = I.sector(4, 5, 6, 0.01, 0.01)


def _desc(**kw):
    a = dict(nr=GOOD.nr, nt=GOOD.nt, np_=GOOD.np, r1=GOOD.r1, r2=GOOD.r2, t1=GOOD.t1, t2=GOOD.t2,
             p1=GOOD.p1, p2=GOOD.p2, periodic=False)
    a.update(kw)
    return a


@pytest.mark.parametrize("bad", [
    {"nr": 2}, {"nt": 0}, {"np_": -1},
    {"r1": 0.0}, {"r2": GOOD.r1},
    {"t1": -0.1}, {"t2": GOOD.t1}, {"t2": math.pi + 0.1},
    {"p2": GOOD.p1},
    {"periodic": True},  # periodic needs phi2 - phi1 = 2 pi
    {"nr": 2000, "nt": 2000, "np_": 1000},  # 4e9 cells: past the 32-bit line counts, refused before allocating
], ids=lambda b: ",".join(f"{k}={v}" for k, v in b.items()))
def test_bad_descriptor(bad, dsw):
    a = _desc(**bad)
    with pytest.raises(dsw.DswError) as ei:
        dsw.Grid(a["nr"], a["nt"], a["np_"], a["r1"], a["r2"], a["t1"], a["t2"], a["p1"], a["p2"],
                 a["periodic"], I.AIR.astuple())
    assert ei.value.code == dsw.DSW_EINVAL
    assert dsw.lib().dsw_last_error().decode()


@pytest.mark.parametrize("bad", [{"cp": 700.0}, {"cv": 0.0}, {"mu": -1.0}, {"prandtl": 0.0}],
                         ids=lambda b: ",".join(f"{k}={v}" for k, v in b.items()))
def test_bad_material(bad, dsw):
    m = dict(zip(("cp", "cv", "pi_inf", "mu", "prandtl", "omega", "g_r"), I.AIR.astuple()))
    m.update(bad)
    with pytest.raises(dsw.DswError) as ei:
        dsw.Grid(*GOOD.args(), tuple(m.values()))
    assert ei.value.code == dsw.DSW_EINVAL


def test_bad_call_arguments(dsw):
    gg = dsw.Grid.from_spec(GOOD, I.AIR)
    U0, tau = I.initial_state(I.Workload("t", GOOD, mach=1e-2, amplitude=0.5, steps=1, K=2, seed=5))
    U = dsw.to_device(U0)
    out, R, Ub, x = gg.empty(), gg.empty(), gg.empty(), gg.empty()
    for v in out.values():
        v.fill_(7.0)
    calls = {
        "split_step K=0": lambda: gg.split_step(U, out, tau, 0),
        "split_step tau=0": lambda: gg.split_step(U, out, 0.0, 2),
        "split_step tau=nan": lambda: gg.split_step(U, out, float("nan"), 2),
        "split_step alias": lambda: gg.split_step(U, U, tau, 2),
        "line_solve alias": lambda: gg.line_solve(1, U, tau, R, R),
        "line_solve tau<0": lambda: gg.line_solve(2, U, -tau, R, x),
        "adjoint alias": lambda: gg.adjoint_step(U, tau, 2, R, R),
        "adjoint K=0": lambda: gg.adjoint_step(U, tau, 0, R, x),
    }
    for name, call in calls.items():
        with pytest.raises(dsw.DswError) as ei:
            call()
        assert ei.value.code == dsw.DSW_EINVAL, name
        print(f"{name}: {ei.value}", flush=True)
    torch.cuda.synchronize()
    for k, v in out.items():  # refused calls wrote nothing
        assert bool((v == 7.0).all()), k
    assert gg.get_status() == dsw.DSW_OK


def test_null_field_pointer(dsw):
    gg = dsw.Grid.from_spec(GOOD, I.AIR)
    U0, tau = I.initial_state(I.Workload("t", GOOD, mach=1e-2, amplitude=0.5, steps=1, K=2, seed=6))
    U = dsw.to_device(U0)
    out = gg.empty()
    f_in, f_out = dsw._fields(U), dsw._fields(out)
    f_in.uf = None
    rc = dsw.lib().dsw_split_step(gg._h, C.byref(f_in), C.byref(f_out), float(tau), 2, None)
    assert rc == dsw.DSW_EINVAL
    assert b"null field pointer" in dsw.lib().dsw_last_error()
    assert dsw.lib().dsw_split_step(None, C.byref(dsw._fields(U)), C.byref(f_out), float(tau), 2,
                                    None) == dsw.DSW_EINVAL
