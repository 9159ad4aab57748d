"""Python binding of libdsw.so (the C-ABI in include/dsw.h).

Argument marshalling only: every step of the time step runs in the HIP
kernels of the library.  PyTorch supplies device memory and the stream.  The
library must have been built (``__graft_entry__.build()`` or
``python paper_2004_13887_amd/build.py``); importing this module without it
raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsw.so")
FIELDS = ("p", "ur", "ut", "uf", "T")

DSW_OK, DSW_EINVAL, DSW_ENOMEM, DSW_EHIP, DSW_ENONPHYS, DSW_ESINGULAR, DSW_EDIVERGED = (
    0, -1, -2, -3, -4, -5, -6)
_NAMES = {DSW_EINVAL: "DSW_EINVAL", DSW_ENOMEM: "DSW_ENOMEM", DSW_EHIP: "DSW_EHIP",
          DSW_ENONPHYS: "DSW_ENONPHYS", DSW_ESINGULAR: "DSW_ESINGULAR", DSW_EDIVERGED: "DSW_EDIVERGED"}

# every extern "C" symbol the header declares
SYMBOLS = ("dsw_init_grid", "dsw_free_grid", "dsw_layout", "dsw_residual", "dsw_line_solve_r",
           "dsw_line_solve_theta", "dsw_line_solve_phi", "dsw_split_step", "dsw_set_timing",
           "dsw_read_timing", "dsw_get_status", "dsw_set_config", "dsw_get_config",
           "dsw_ensemble_create", "dsw_ensemble_free", "dsw_ensemble_member", "dsw_ensemble_step",
           "dsw_ensemble_tune", "dsw_ensemble_set_config", "dsw_ensemble_get_config",
           "dsw_ensemble_get_status", "dsw_adjoint_step", "dsw_line_solve_T_r",
           "dsw_line_solve_T_theta", "dsw_line_solve_T_phi", "dsw_line_vjp_r", "dsw_line_vjp_theta",
           "dsw_line_vjp_phi", "dsw_residual_vjp", "dsw_split_step_forced", "dsw_tape_bytes", "dsw_split_step_taped",
           "dsw_adjoint_step_taped", "dsw_adjoint_trajectory", "dsw_split_step_noalloc",
           "dsw_set_reference", "dsw_split_step_pert", "dsw_courant", "dsw_last_error")
TIMING_KINDS = ("residual", "sweep_r", "sweep_theta", "sweep_phi_update", "boundary_copy")


class DswError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_theta", C.c_int32), ("n_phi", C.c_int32),
                ("periodic_phi", C.c_int32), ("r1", C.c_double), ("r2", C.c_double),
                ("theta1", C.c_double), ("theta2", C.c_double), ("phi1", C.c_double),
                ("phi2", C.c_double)]


class Material(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("cp", "cv", "pi_inf", "mu", "prandtl", "omega", "g_r")]


class Fields(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in FIELDS]


WALLS = ("ur_t1", "ur_t2", "ur_p1", "ur_p2", "ut_r1", "ut_r2", "ut_p1", "ut_p2",
         "uf_r1", "uf_r2", "uf_t1", "uf_t2")


class Wall(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in WALLS]


class Config(C.Structure):
    _fields_ = [("residual_block", C.c_int32), ("sweep_block_r", C.c_int32),
                ("sweep_block_theta", C.c_int32), ("phi_rows_per_thread", C.c_int32),
                ("rows_per_thread_r", C.c_int32), ("rows_per_thread_theta", C.c_int32)]

    def astuple(self):
        return (self.residual_block, self.sweep_block_r, self.sweep_block_theta,
                self.phi_rows_per_thread, self.rows_per_thread_r, self.rows_per_thread_theta)


class LayoutInfo(C.Structure):
    _fields_ = [("shape", (C.c_int64 * 3) * 5), ("count", C.c_int64 * 5),
                ("bytes_per_state", C.c_int64)]


_lib = None


def lib():
    """Load libdsw.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        P, D, I = C.c_void_p, C.c_double, C.c_int32
        FP = C.POINTER(Fields)
        L.dsw_init_grid.argtypes = [C.POINTER(GridDesc), C.POINTER(Material), C.POINTER(C.c_void_p)]
        L.dsw_free_grid.argtypes = [P]
        L.dsw_layout.argtypes = [P, C.POINTER(LayoutInfo)]
        L.dsw_residual.argtypes = [P, FP, FP, D, FP, FP, P]
        for n in ("dsw_line_solve_r", "dsw_line_solve_theta", "dsw_line_solve_phi"):
            getattr(L, n).argtypes = [P, FP, D, FP, FP, P]
        L.dsw_split_step.argtypes = [P, FP, FP, D, I, P]
        L.dsw_split_step_noalloc.argtypes = [P, FP, FP, D, I, P]
        L.dsw_set_reference.argtypes = [P, C.c_void_p, C.c_void_p]
        L.dsw_split_step_pert.argtypes = [P, FP, FP, D, I, P]
        L.dsw_courant.argtypes = [P, FP, D, C.c_void_p, P]
        L.dsw_get_status.argtypes = [P, P]
        L.dsw_set_timing.argtypes = [P, I]
        L.dsw_read_timing.argtypes = [P, P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        CP = C.POINTER(Config)
        L.dsw_set_config.argtypes = [P, CP]
        L.dsw_get_config.argtypes = [P, CP]
        L.dsw_ensemble_create.argtypes = [C.POINTER(GridDesc), C.POINTER(Material), I,
                                          C.POINTER(C.c_void_p)]
        L.dsw_ensemble_free.argtypes = [P]
        L.dsw_ensemble_member.argtypes = [P, I, C.POINTER(C.c_void_p)]
        L.dsw_ensemble_step.argtypes = [P, FP, FP, C.POINTER(C.c_double), I, P]
        L.dsw_ensemble_tune.argtypes = [P, FP, FP, C.POINTER(C.c_double), I, I, P, CP]
        L.dsw_ensemble_set_config.argtypes = [P, CP]
        L.dsw_ensemble_get_config.argtypes = [P, CP]
        L.dsw_ensemble_get_status.argtypes = [P, P]
        L.dsw_adjoint_step.argtypes = [P, FP, D, I, FP, FP, P]
        for n in ("dsw_line_solve_T_r", "dsw_line_solve_T_theta", "dsw_line_solve_T_phi"):
            getattr(L, n).argtypes = [P, FP, D, FP, FP, P]
        for n in ("dsw_line_vjp_r", "dsw_line_vjp_theta", "dsw_line_vjp_phi"):
            getattr(L, n).argtypes = [P, FP, D, FP, FP, FP, P]
        L.dsw_residual_vjp.argtypes = [P, FP, D, FP, FP, P]
        L.dsw_split_step_forced.argtypes = [P, FP, FP, D, I, FP, C.POINTER(Wall), C.POINTER(Wall), FP, P]
        L.dsw_tape_bytes.argtypes = [P, I, C.POINTER(C.c_int64)]
        L.dsw_split_step_taped.argtypes = [P, FP, FP, D, I, P, P]
        L.dsw_adjoint_step_taped.argtypes = [P, FP, D, I, P, FP, FP, P]
        L.dsw_adjoint_trajectory.argtypes = [P, FP, I, D, I, FP, FP, P]
        L.dsw_last_error.restype = C.c_char_p
        for n in SYMBOLS[:-1]:
            getattr(L, n).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != DSW_OK:
        raise DswError(rc, lib().dsw_last_error().decode())


def _fields(d) -> Fields:
    f = Fields()
    for n in FIELDS:
        t = d[n]
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError(f"field {n}: need a contiguous float64 device tensor")
        setattr(f, n, t.data_ptr())
    return f


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Grid:
    """Handle of dsw_init_grid; methods are the C-ABI calls of the same names."""

    def __init__(self, nr, nt, np_, r1, r2, t1, t2, p1, p2, periodic, material, _borrowed=None):
        self.desc = GridDesc(int(nr), int(nt), int(np_), 1 if periodic else 0, float(r1), float(r2),
                             float(t1), float(t2), float(p1), float(p2))
        self.mat = Material(*(float(x) for x in material))
        if _borrowed is not None:  # member handle owned by an Ensemble
            self._h, self._owned, self._owner = _borrowed[0], False, _borrowed[1]
            return
        h = C.c_void_p()
        _check(lib().dsw_init_grid(C.byref(self.desc), C.byref(self.mat), C.byref(h)))
        # kept on the object: at interpreter exit the module's globals may be
        # gone before the finaliser runs
        self._free = lib().dsw_free_grid
        self._h, self._owned = h, True

    @classmethod
    def from_spec(cls, spec, material):
        return cls(*spec.args(), material.astuple())

    def free_grid(self):
        if getattr(self, "_h", None) and getattr(self, "_owned", False):
            self._free(self._h)
        self._h = None

    __del__ = free_grid

    def layout(self):
        info = LayoutInfo()
        _check(lib().dsw_layout(self._h, C.byref(info)))
        return {n: tuple(int(x) for x in info.shape[q]) for q, n in enumerate(FIELDS)}

    def empty(self, device="cuda"):
        return {n: torch.zeros(s, dtype=torch.float64, device=device) for n, s in self.layout().items()}

    def residual(self, Un, Uk, tau, R, Ubar, stream=None):
        _check(lib().dsw_residual(self._h, C.byref(_fields(Un)), C.byref(_fields(Uk)), float(tau),
                                  C.byref(_fields(R)), C.byref(_fields(Ubar)), _stream(stream)))

    def line_solve_r(self, Ubar, tau, rhs, x, stream=None):
        _check(lib().dsw_line_solve_r(self._h, C.byref(_fields(Ubar)), float(tau),
                                      C.byref(_fields(rhs)), C.byref(_fields(x)), _stream(stream)))

    def line_solve_theta(self, Ubar, tau, rhs, x, stream=None):
        _check(lib().dsw_line_solve_theta(self._h, C.byref(_fields(Ubar)), float(tau),
                                          C.byref(_fields(rhs)), C.byref(_fields(x)), _stream(stream)))

    def line_solve_phi(self, Ubar, tau, rhs, x, stream=None):
        _check(lib().dsw_line_solve_phi(self._h, C.byref(_fields(Ubar)), float(tau),
                                        C.byref(_fields(rhs)), C.byref(_fields(x)), _stream(stream)))

    def line_solve(self, d, Ubar, tau, rhs, x, stream=None):
        (self.line_solve_r, self.line_solve_theta, self.line_solve_phi)[d](Ubar, tau, rhs, x, stream)

    def adjoint_step(self, Un, tau, K, lam_np1, lam_n, stream=None):
        _check(lib().dsw_adjoint_step(self._h, C.byref(_fields(Un)), float(tau), int(K),
                                      C.byref(_fields(lam_np1)), C.byref(_fields(lam_n)),
                                      _stream(stream)))

    def adjoint_trajectory(self, ckpts, tau, K, lam_end, lam_0, stream=None):
        """lam_0 = J(U^0)^T ... J(U^{N-1})^T lam_end over the N steps whose
        starting states ckpts holds (a list of field dicts, U^0 first)."""
        arr = (Fields * len(ckpts))(*[_fields(u) for u in ckpts])
        _check(lib().dsw_adjoint_trajectory(self._h, arr, len(ckpts), float(tau), int(K),
                                            C.byref(_fields(lam_end)), C.byref(_fields(lam_0)),
                                            _stream(stream)))

    def line_solve_T(self, d, Ubar, tau, rhs, x, stream=None):
        fn = ("dsw_line_solve_T_r", "dsw_line_solve_T_theta", "dsw_line_solve_T_phi")[d]
        _check(getattr(lib(), fn)(self._h, C.byref(_fields(Ubar)), float(tau), C.byref(_fields(rhs)),
                                  C.byref(_fields(x)), _stream(stream)))

    def line_vjp(self, d, Ubar, tau, X, mu, acc, stream=None):
        fn = ("dsw_line_vjp_r", "dsw_line_vjp_theta", "dsw_line_vjp_phi")[d]
        _check(getattr(lib(), fn)(self._h, C.byref(_fields(Ubar)), float(tau), C.byref(_fields(X)),
                                  C.byref(_fields(mu)), C.byref(_fields(acc)), _stream(stream)))

    def residual_vjp(self, Ubar, tau, mu, acc, stream=None):
        _check(lib().dsw_residual_vjp(self._h, C.byref(_fields(Ubar)), float(tau),
                                      C.byref(_fields(mu)), C.byref(_fields(acc)), _stream(stream)))

    def split_step(self, Un, Unp1, tau, K, stream=None):
        _check(lib().dsw_split_step(self._h, C.byref(_fields(Un)), C.byref(_fields(Unp1)),
                                    float(tau), int(K), _stream(stream)))

    def split_step_noalloc(self, Un, Unp1, tau, K, stream=None):
        """dsw_split_step_noalloc: the same step on the library's static
        workspace (no device allocation; grids up to DSW_NOALLOC_BYTES of
        workspace)"""
        _check(lib().dsw_split_step_noalloc(self._h, C.byref(_fields(Un)), C.byref(_fields(Unp1)),
                                            float(tau), int(K), _stream(stream)))

    def set_reference(self, p_ref, T_ref):
        """dsw_set_reference: the reference column (n_r values each) of the
        perturbation-pressure form"""
        nr = int(self.desc.n_r)
        pr, tr = [float(x) for x in p_ref], [float(x) for x in T_ref]
        if len(pr) != nr or len(tr) != nr:
            raise ValueError("p_ref and T_ref need n_r values each")
        _check(lib().dsw_set_reference(self._h, (C.c_double * nr)(*pr), (C.c_double * nr)(*tr)))

    def split_step_pert(self, Un, Unp1, tau, K, stream=None):
        """dsw_split_step_pert: the split step on states whose p holds p - p_ref"""
        _check(lib().dsw_split_step_pert(self._h, C.byref(_fields(Un)), C.byref(_fields(Unp1)),
                                         float(tau), int(K), _stream(stream)))

    def courant(self, U, tau, stream=None):
        """dsw_courant: (advective, acoustic) Courant numbers of U for the step tau"""
        out = (C.c_double * 2)()
        _check(lib().dsw_courant(self._h, C.byref(_fields(U)), float(tau), out, _stream(stream)))
        return float(out[0]), float(out[1])

    def tape_bytes(self, K):
        n = C.c_int64()
        _check(lib().dsw_tape_bytes(self._h, int(K), C.byref(n)))
        return int(n.value)

    def new_tape(self, K, device="cuda"):
        """a device buffer for dsw_split_step_taped (8-byte aligned)"""
        return torch.empty(self.tape_bytes(K) // 8, dtype=torch.float64, device=device)

    def split_step_taped(self, Un, Unp1, tau, K, tape, stream=None):
        _check(lib().dsw_split_step_taped(self._h, C.byref(_fields(Un)), C.byref(_fields(Unp1)),
                                          float(tau), int(K), C.c_void_p(tape.data_ptr()),
                                          _stream(stream)))

    def adjoint_step_taped(self, Un, tau, K, tape, lam_np1, lam_n, stream=None):
        _check(lib().dsw_adjoint_step_taped(self._h, C.byref(_fields(Un)), float(tau), int(K),
                                            C.c_void_p(tape.data_ptr()), C.byref(_fields(lam_np1)),
                                            C.byref(_fields(lam_n)), _stream(stream)))

    def split_step_forced(self, Un, Unp1, tau, K, src=None, wall0=None, wall1=None, bnd=None,
                          stream=None):
        """dsw_split_step_forced: src (dict of five device arrays, a missing
        one is zero), wall0 / wall1 (dicts of the WALLS arrays at t^n and
        t^{n+1}, a missing one is zero), bnd (dict whose ur, ut, uf
        boundary-normal faces hold the Dirichlet data of t^{n+1})."""
        def wall_struct(wall):
            w = Wall()
            for n in WALLS:
                t = wall.get(n)
                if t is not None:
                    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                        raise ValueError(f"wall {n}: need a contiguous float64 device tensor")
                    setattr(w, n, t.data_ptr())
            return w
        w0 = wall_struct(wall0) if wall0 is not None else None
        w1 = wall_struct(wall1) if wall1 is not None else None
        fs = None
        if src is not None:
            fs = Fields()
            for n in FIELDS:
                t = src.get(n)
                if t is not None:
                    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                        raise ValueError(f"src {n}: need a contiguous float64 device tensor")
                    setattr(fs, n, t.data_ptr())
        fb = None
        if bnd is not None:
            fb = Fields()
            for n in ("ur", "ut", "uf"):
                t = bnd[n]
                if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                    raise ValueError(f"bnd {n}: need a contiguous float64 device tensor")
                setattr(fb, n, t.data_ptr())
        _check(lib().dsw_split_step_forced(
            self._h, C.byref(_fields(Un)), C.byref(_fields(Unp1)), float(tau), int(K),
            C.byref(fs) if fs is not None else None, C.byref(w0) if w0 is not None else None,
            C.byref(w1) if w1 is not None else None,
            C.byref(fb) if fb is not None else None, _stream(stream)))

    def set_timing(self, enable=True):
        _check(lib().dsw_set_timing(self._h, 1 if enable else 0))

    def read_timing(self, stream=None):
        """{kind: (total ms, launches)} since the last read."""
        ms = (C.c_double * len(TIMING_KINDS))()
        n = (C.c_int64 * len(TIMING_KINDS))()
        _check(lib().dsw_read_timing(self._h, _stream(stream), ms, n))
        return {k: (float(ms[q]), int(n[q])) for q, k in enumerate(TIMING_KINDS)}

    def get_status(self, stream=None):
        """DSW_OK, or raises DswError(DSW_ENONPHYS / DSW_EDIVERGED / DSW_ESINGULAR)."""
        _check(lib().dsw_get_status(self._h, _stream(stream)))
        return DSW_OK

    def set_config(self, residual_block=64, sweep_block_r=256, sweep_block_theta=256,
                   phi_rows_per_thread=4, rows_per_thread_r=None, rows_per_thread_theta=None):
        """dsw_set_config; the r / theta solver choices left as None keep the
        grid's current ones"""
        cur = self.get_config()
        rr = cur[4] if rows_per_thread_r is None else rows_per_thread_r
        rt = cur[5] if rows_per_thread_theta is None else rows_per_thread_theta
        c = Config(residual_block, sweep_block_r, sweep_block_theta, phi_rows_per_thread, rr, rt)
        _check(lib().dsw_set_config(self._h, C.byref(c)))

    def get_config(self):
        c = Config()
        _check(lib().dsw_get_config(self._h, C.byref(c)))
        return c.astuple()


def _field_array(states):
    arr = (Fields * len(states))()
    for q, d in enumerate(states):
        arr[q] = _fields(d)
    return arr


class Ensemble:
    """Handle of dsw_ensemble_create: n grids stepped by batched launches
    replayed from one HIP graph."""

    def __init__(self, specs, materials):
        n = len(specs)
        descs = (GridDesc * n)()
        mats = (Material * n)()
        for q, (g, m) in enumerate(zip(specs, materials)):
            nr, nt, np_, r1, r2, t1, t2, p1, p2, periodic = g.args()
            descs[q] = GridDesc(nr, nt, np_, 1 if periodic else 0, r1, r2, t1, t2, p1, p2)
            mats[q] = Material(*m.astuple())
        h = C.c_void_p()
        _check(lib().dsw_ensemble_create(descs, mats, n, C.byref(h)))
        self._free = lib().dsw_ensemble_free  # as for Grid
        self._h = h
        self.n = n
        self.members = []
        for q, (g, m) in enumerate(zip(specs, materials)):
            gh = C.c_void_p()
            _check(lib().dsw_ensemble_member(self._h, q, C.byref(gh)))
            self.members.append(Grid(*g.args(), m.astuple(), _borrowed=(gh, self)))

    def ensemble_free(self):
        if getattr(self, "_h", None):
            for g in self.members:
                g._h = None
            self._free(self._h)
            self._h = None

    __del__ = ensemble_free

    def ensemble_step(self, Un, Unp1, tau, K, stream=None):
        taus = (C.c_double * self.n)(*[float(t) for t in tau])
        _check(lib().dsw_ensemble_step(self._h, _field_array(Un), _field_array(Unp1), taus, int(K),
                                       _stream(stream)))

    def ensemble_tune(self, Un, Unp1, tau, K, reps=2, stream=None):
        taus = (C.c_double * self.n)(*[float(t) for t in tau])
        c = Config()
        _check(lib().dsw_ensemble_tune(self._h, _field_array(Un), _field_array(Unp1), taus, int(K),
                                       int(reps), _stream(stream), C.byref(c)))
        return c.astuple()

    def set_config(self, residual_block=64, sweep_block_r=256, sweep_block_theta=256,
                   phi_rows_per_thread=4, rows_per_thread_r=None, rows_per_thread_theta=None):
        """dsw_ensemble_set_config; solver choices left as None keep the
        ensemble's current ones"""
        cur = self.get_config()
        rr = cur[4] if rows_per_thread_r is None else rows_per_thread_r
        rt = cur[5] if rows_per_thread_theta is None else rows_per_thread_theta
        c = Config(residual_block, sweep_block_r, sweep_block_theta, phi_rows_per_thread, rr, rt)
        _check(lib().dsw_ensemble_set_config(self._h, C.byref(c)))

    def get_config(self):
        c = Config()
        _check(lib().dsw_ensemble_get_config(self._h, C.byref(c)))
        return c.astuple()

    def get_status(self, stream=None):
        _check(lib().dsw_ensemble_get_status(self._h, _stream(stream)))
        return DSW_OK


class SplitStep(torch.autograd.Function):
    """U^{n+1} = split_step(U^n) as a differentiable function of the five
    fields (in the order p, ur, ut, uf, T).  The forward keeps U^n as the
    checkpoint; the backward calls dsw_adjoint_step, which recomputes the
    step from it.  With taped=True the forward also keeps a tape of the step
    (dsw_split_step_taped; 4K states of device memory per step) and the
    backward skips the recompute (dsw_adjoint_step_taped)."""

    @staticmethod
    def forward(ctx, grid, tau, K, taped, p, ur, ut, uf, T):
        Un = {"p": p.detach().contiguous(), "ur": ur.detach().contiguous(),
              "ut": ut.detach().contiguous(), "uf": uf.detach().contiguous(),
              "T": T.detach().contiguous()}
        out = grid.empty(device=p.device)
        tape = None
        if taped:
            tape = grid.new_tape(K, device=p.device)
            grid.split_step_taped(Un, out, tau, K, tape)
        else:
            grid.split_step(Un, out, tau, K)
        ctx.grid, ctx.tau, ctx.K, ctx.tape = grid, tau, K, tape
        ctx.save_for_backward(*(Un[k] for k in FIELDS))
        return tuple(out[k] for k in FIELDS)

    @staticmethod
    def backward(ctx, *grads):
        Un = dict(zip(FIELDS, ctx.saved_tensors))
        lam = {k: (g if g is not None else torch.zeros_like(Un[k])).contiguous()
               for k, g in zip(FIELDS, grads)}
        out = ctx.grid.empty(device=Un["p"].device)
        if ctx.tape is not None:
            ctx.grid.adjoint_step_taped(Un, ctx.tau, ctx.K, ctx.tape, lam, out)
            ctx.tape = None
        else:
            ctx.grid.adjoint_step(Un, ctx.tau, ctx.K, lam, out)
        return (None, None, None, None) + tuple(out[k] for k in FIELDS)


def split_step_fn(grid, U, tau, K, taped=False):
    """differentiable split step on a dict of fields"""
    outs = SplitStep.apply(grid, tau, K, taped, *(U[k] for k in FIELDS))
    return dict(zip(FIELDS, outs))


def to_device(fields, device="cuda"):
    return {k: torch.as_tensor(v).to(device=device, dtype=torch.float64).contiguous()
            for k, v in fields.items()}


def to_host(fields):
    return {k: v.detach().cpu().numpy() for k, v in fields.items()}
