"""Python wrapper of the plain FP64 CPU oracle (``dsw_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product path never imports
it.  It shares no code with the HIP path; only the seeded input generators
(``paper_2004_13887_amd.inputs``) feed both.

The oracle follows the direction-split nonlinear iteration of the paper
(section "Discretization", eqs. (chapter3mainsd), (splitting2), (spl1)-(spl3))
with the spatial operators of Appendix B; see ``dsw_oracle.c`` for the detailed
statement.  Fields are numpy float64 arrays in C order:

    p, T : [nr][nt][np]       (cell centres)
    ur   : [nr+1][nt][np]     (r faces)
    ut   : [nr][nt+1][np]     (theta faces)
    uf   : [nr][nt][npf]      (phi faces; npf = np if periodic else np+1)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dsw_oracle.c")
_LIB = os.path.join(_HERE, "libdsw_oracle.so")
_LIB_CS = os.path.join(_HERE, "libdsw_oracle_cs.so")  # complex-step build

MASK_R, MASK_T, MASK_F, MASK_M, MASK_ALL = 1, 2, 4, 8, 15
FIELDS = ("p", "ur", "ut", "uf", "T")
FID = {"p": 0, "ur": 1, "ut": 2, "uf": 3, "T": 4}


def _build_one(out, defs, force):
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared"] + defs + ["-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math): the FP64
    library and its complex-step twin (same source, complex state type)."""
    _build_one(_LIB_CS, ["-DORC_COMPLEX_STEP"], force)
    return _build_one(_LIB, [], force)


_LIB_BENCH = os.path.join(_HERE, "libdsw_oracle_bench.so")  # this host's CPU only


def lib_bench():
    """The FP64 oracle built for timing on this host: -O3 -march=native, still
    without FMA contraction or fast-math (the same results as the test build).
    Built where it runs, every time, since -march=native code is not portable."""
    tmp = _LIB_BENCH + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-std=gnu11", "-fopenmp", "-ffp-contract=off",
                           "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_BENCH)
    L_ = _load(_LIB_BENCH)
    L_.orc_set_threads.argtypes = [C.c_int]
    L_.orc_max_threads.restype = C.c_int
    return L_


class _Mat(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("cp", "cv", "pi_inf", "mu", "prandtl", "omega", "g_r")]


class _Fields(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_double)) for n in FIELDS]


_WALL_NAMES = ("ur_t1", "ur_t2", "ur_p1", "ur_p2", "ut_r1", "ut_r2", "ut_p1", "ut_p2",
               "uf_r1", "uf_r2", "uf_t1", "uf_t2")


class _Wall(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_double)) for n in _WALL_NAMES]


_lib = None
_lib_cs = None


def _load(path):
    L_ = C.CDLL(path)
    P, D, I, L = C.c_void_p, C.c_double, C.c_int, C.c_long
    L_.orc_grid_new.restype = P
    L_.orc_grid_new.argtypes = [I, I, I, D, D, D, D, D, D, I]
    L_.orc_grid_free.argtypes = [P]
    FP = C.POINTER(_Fields)
    MP = C.POINTER(_Mat)
    WP = C.POINTER(_Wall)
    L_.orc_apply.argtypes = [P, MP, FP, WP, FP, WP, I, FP]
    L_.orc_residual.argtypes = [P, MP, FP, FP, WP, FP, D, FP, FP]
    L_.orc_line_solve.argtypes = [P, MP, FP, WP, D, I, FP, FP]
    L_.orc_line_matvec.argtypes = [P, MP, FP, WP, D, I, FP, FP]
    L_.orc_line_blocks.argtypes = [P, MP, FP, WP, D, I, I, I, I, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]
    L_.orc_split_step.argtypes = [P, MP, FP, FP, D, I, WP, WP, FP, FP]
    L_.orc_residual_at.argtypes = [P, MP, FP, FP, FP, WP, D, L, C.c_void_p, C.c_void_p,
                                     C.c_void_p]
    L_.orc_line_solve_some.argtypes = [P, MP, FP, WP, D, I, L, C.c_void_p, C.c_void_p,
                                         C.c_void_p, FP, FP]
    L_.orc_block_solve.argtypes = [I, I, I, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L_.orc_split_step_pert.argtypes = [P, MP, C.c_void_p, C.c_void_p, FP, FP, D, I]
    for f in ("orc_block_solve", "orc_apply", "orc_residual", "orc_line_solve", "orc_line_matvec",
              "orc_line_blocks", "orc_split_step", "orc_residual_at", "orc_line_solve_some",
              "orc_split_step_pert"):
        getattr(L_, f).restype = I
    if hasattr(L_, "orc_courant"):
        L_.orc_courant.argtypes = [P, MP, FP, D, C.c_void_p]
        L_.orc_courant.restype = None
    return L_


def lib():
    global _lib
    if _lib is None:
        _lib = _load(build())
    return _lib


def lib_cs():
    """the complex-step build (state type double complex)"""
    global _lib_cs
    if _lib_cs is None:
        build()
        _lib_cs = _load(_LIB_CS)
    return _lib_cs


@dataclass(frozen=True)
class Material:
    cp: float
    cv: float
    pi_inf: float
    mu: float
    prandtl: float
    omega: float
    g_r: float

    def c(self) -> _Mat:
        return _Mat(self.cp, self.cv, self.pi_inf, self.mu, self.prandtl, self.omega, self.g_r)


class Grid:
    """MAC grid on the sector [r1,r2] x [t1,t2] x [p1,p2] (paper section 2.1)."""

    def __init__(self, nr, nt, np_, r1, r2, t1, t2, p1, p2, periodic=False):
        self.nr, self.nt, self.np = int(nr), int(nt), int(np_)
        self.r1, self.r2, self.t1, self.t2, self.p1, self.p2 = map(float, (r1, r2, t1, t2, p1, p2))
        self.periodic = bool(periodic)
        self.npf = self.np if self.periodic else self.np + 1
        h = lib().orc_grid_new(self.nr, self.nt, self.np, self.r1, self.r2, self.t1, self.t2,
                               self.p1, self.p2, int(self.periodic))
        if not h:
            raise ValueError("invalid grid description")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_grid_free(h)
            self._h = None

    def shapes(self):
        nr, nt, np_, npf = self.nr, self.nt, self.np, self.npf
        return {"p": (nr, nt, np_), "ur": (nr + 1, nt, np_), "ut": (nr, nt + 1, np_),
                "uf": (nr, nt, npf), "T": (nr, nt, np_)}

    def zeros(self):
        return {k: np.zeros(s) for k, s in self.shapes().items()}

    def coords(self):
        """Centre and face coordinates (for tests / manufactured solutions)."""
        dr = (self.r2 - self.r1) / self.nr
        dt = (self.t2 - self.t1) / self.nt
        dp = (self.p2 - self.p1) / self.np
        return {
            "rc": self.r1 + (np.arange(self.nr) + 0.5) * dr,
            "rf": self.r1 + np.arange(self.nr + 1) * dr,
            "tc": self.t1 + (np.arange(self.nt) + 0.5) * dt,
            "tf": self.t1 + np.arange(self.nt + 1) * dt,
            "pc": self.p1 + (np.arange(self.np) + 0.5) * dp,
            "pf": self.p1 + np.arange(self.npf) * dp,
            "dr": dr, "dt": dt, "dp": dp,
        }


def _fields(g: Grid, d, keep):
    """dict of arrays -> ctypes struct; arrays are checked and kept alive."""
    sh = g.shapes()
    f = _Fields()
    for n in FIELDS:
        a = d[n]
        if a.dtype != np.float64 or not a.flags.c_contiguous or a.shape != sh[n]:
            raise ValueError(f"field {n}: need C-contiguous float64 of shape {sh[n]}")
        keep.append(a)
        setattr(f, n, a.ctypes.data_as(C.POINTER(C.c_double)))
    return C.byref(f)


def _wall(g: Grid, w, keep):
    if w is None:
        return None
    s = _Wall()
    for n in _WALL_NAMES:
        a = w.get(n)
        if a is not None:
            a = np.ascontiguousarray(a, dtype=np.float64)
            keep.append(a)
            setattr(s, n, a.ctypes.data_as(C.POINTER(C.c_double)))
    return C.byref(s)


def _copy(d):
    return {k: np.ascontiguousarray(v, dtype=np.float64).copy() for k, v in d.items()}


def apply(g: Grid, mat: Material, u, v, mask=MASK_ALL, wall_u=None, wall_v=None):
    """N(u; v) restricted to the direction tags in ``mask`` (0 on boundary faces)."""
    keep = []
    out = g.zeros()
    m = mat.c()
    rc = lib().orc_apply(g._h, C.byref(m), _fields(g, u, keep), _wall(g, wall_u, keep),
                         _fields(g, v, keep), _wall(g, wall_v, keep), int(mask),
                         _fields(g, out, keep))
    assert rc == 0
    return out


def residual(g: Grid, mat: Material, Un, Uk, tau, wall=None, src=None):
    """(R, Ubar): R = -(Uk-Un) - tau (F_h(Ubar) - src), Ubar = (Uk+Un)/2."""
    keep = []
    R, Ub = g.zeros(), g.zeros()
    m = mat.c()
    rc = lib().orc_residual(g._h, C.byref(m), _fields(g, Un, keep), _fields(g, Uk, keep),
                            _wall(g, wall, keep), _fields(g, src, keep) if src else None,
                            float(tau), _fields(g, R, keep), _fields(g, Ub, keep))
    assert rc == 0
    return R, Ub


def line_solve(g: Grid, mat: Material, Ubar, tau, d, rhs, wall=None):
    """x solving (I + tau/2 D_d(Ubar)) x = rhs; d = 0 (r), 1 (theta), 2 (phi)."""
    keep = []
    x = g.zeros()
    m = mat.c()
    rc = lib().orc_line_solve(g._h, C.byref(m), _fields(g, Ubar, keep), _wall(g, wall, keep),
                              float(tau), int(d), _fields(g, rhs, keep), _fields(g, x, keep))
    if rc != 0:
        raise ArithmeticError("zero pivot in a line solve")
    return x


def line_matvec(g: Grid, mat: Material, Ubar, tau, d, x, wall=None):
    keep = []
    y = g.zeros()
    m = mat.c()
    rc = lib().orc_line_matvec(g._h, C.byref(m), _fields(g, Ubar, keep), _wall(g, wall, keep),
                               float(tau), int(d), _fields(g, x, keep), _fields(g, y, keep))
    assert rc == 0
    return y


def line_blocks(g: Grid, mat: Material, Ubar, tau, d, kind, a, b, wall=None):
    """Blocks of one line: (L, D, U, flat_idx, field_id, cyclic).  kind = -1 for
    the (p, T, normal-velocity) block line, else the scalar family's field id."""
    n = (g.nr, g.nt, g.np)[d]
    bs = 3 if kind < 0 else 1
    Lo = np.zeros((n, bs, bs)); Do = np.zeros((n, bs, bs)); Uo = np.zeros((n, bs, bs))
    idx = np.zeros(n * bs, dtype=np.int64); fid = np.zeros(n * bs, dtype=np.int32)
    keep = []
    m = mat.c()
    cyc = lib().orc_line_blocks(g._h, C.byref(m), _fields(g, Ubar, keep), _wall(g, wall, keep),
                                float(tau), int(d), int(kind), int(a), int(b),
                                Lo.ctypes.data, Do.ctypes.data, Uo.ctypes.data,
                                idx.ctypes.data, fid.ctypes.data)
    return Lo, Do, Uo, idx, fid, bool(cyc)


def split_step(g: Grid, mat: Material, Un, tau, K, wall0=None, wall1=None, src=None, bnd=None):
    """One direction-split time step U^{n+1} from U^n with K iterations.
    wall0, wall1: tangential wall velocities at t^n and t^{n+1} (None: zero);
    bnd: fields whose boundary-normal faces hold the Dirichlet data at t^{n+1}
    (None: Un's); src: the midpoint source.  The change of the boundary data
    enters the first iteration's increments as inhomogeneous Dirichlet data
    (see orc_split_step)."""
    keep = []
    out = g.zeros()
    m = mat.c()
    rc = lib().orc_split_step(g._h, C.byref(m), _fields(g, Un, keep), _fields(g, out, keep),
                              float(tau), int(K), _wall(g, wall0, keep), _wall(g, wall1, keep),
                              _fields(g, src, keep) if src else None,
                              _fields(g, bnd, keep) if bnd else None)
    if rc != 0:
        raise ArithmeticError("zero pivot in a line solve")
    return out


def split_step_pert(g: Grid, mat: Material, Un, pbar, Tbar, tau, K):
    """The split step on the perturbation-pressure state: Un["p"] holds
    p - pbar(r) for the discretely hydrostatic reference column (pbar, Tbar)
    at the cell centres (see orc_split_step_pert); returns the same form."""
    keep = []
    out = g.zeros()
    m = mat.c()
    pb = np.ascontiguousarray(pbar, dtype=np.float64)
    tb = np.ascontiguousarray(Tbar, dtype=np.float64)
    assert pb.shape == (g.nr,) and tb.shape == (g.nr,)
    rc = lib().orc_split_step_pert(g._h, C.byref(m), pb.ctypes.data, tb.ctypes.data,
                                   _fields(g, Un, keep), _fields(g, out, keep), float(tau), int(K))
    if rc != 0:
        raise ArithmeticError("zero pivot in a line solve")
    return out


def courant(g: Grid, mat: Material, U, tau):
    """(advective, acoustic) Courant numbers of U for the step tau (see
    orc_courant)."""
    keep = []
    m = mat.c()
    out = np.zeros(2)
    lib().orc_courant(g._h, C.byref(m), _fields(g, U, keep), float(tau), out.ctypes.data)
    return float(out[0]), float(out[1])


def residual_at(g: Grid, mat: Material, Un, Uk, Ubar, tau, fids, idx, wall=None):
    """R at sample points (fids: field ids, idx: flat indices), Ubar given."""
    fids = np.ascontiguousarray(fids, dtype=np.int32)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(len(idx))
    keep = []
    m = mat.c()
    lib().orc_residual_at(g._h, C.byref(m), _fields(g, Un, keep), _fields(g, Uk, keep),
                          _fields(g, Ubar, keep), _wall(g, wall, keep), float(tau), len(idx),
                          fids.ctypes.data, idx.ctypes.data, out.ctypes.data)
    return out


def line_solve_some(g: Grid, mat: Material, Ubar, tau, d, kinds, as_, bs_, rhs, wall=None):
    """Solve only the listed lines; returns fields that hold the solution on
    those lines and NaN elsewhere."""
    kinds = np.ascontiguousarray(kinds, dtype=np.int32)
    as_ = np.ascontiguousarray(as_, dtype=np.int32)
    bs_ = np.ascontiguousarray(bs_, dtype=np.int32)
    x = {k: np.full(s, np.nan) for k, s in g.shapes().items()}
    keep = []
    m = mat.c()
    rc = lib().orc_line_solve_some(g._h, C.byref(m), _fields(g, Ubar, keep), _wall(g, wall, keep),
                                   float(tau), int(d), len(kinds), kinds.ctypes.data,
                                   as_.ctypes.data, bs_.ctypes.data, _fields(g, rhs, keep),
                                   _fields(g, x, keep))
    if rc != 0:
        raise ArithmeticError("zero pivot in a line solve")
    return x


def block_solve(L, D, U, b, cyclic=False):
    """Solve a block-tridiagonal system (blocks n x bs x bs, b n x bs)."""
    L, D, U = (np.ascontiguousarray(a, dtype=np.float64) for a in (L, D, U))
    n, bs = D.shape[0], D.shape[1]
    x = np.ascontiguousarray(b, dtype=np.float64).reshape(n, bs).copy()
    rc = lib().orc_block_solve(n, bs, int(cyclic), L.ctypes.data, D.ctypes.data, U.ctypes.data,
                               x.ctypes.data)
    if rc != 0:
        raise ArithmeticError("zero pivot")
    return x


# ---------------------------------------------------------- complex step --
#
# The complex-step build evaluates the same oracle on complex states.  At
# U + i h V with h = 1e-30 every output equals its real value plus i h times
# its directional derivative along V, with no subtraction of nearby values,
# so Im(.)/h is the Jacobian-vector product exact to rounding.  A grid handle
# of the FP64 build serves both builds (the grid struct holds only FP64
# geometry).

CS_H = 1e-30


def _cfields(g: Grid, d, keep):
    sh = g.shapes()
    f = _Fields()
    for n in FIELDS:
        a = d[n]
        if a.dtype != np.complex128 or not a.flags.c_contiguous or a.shape != sh[n]:
            raise ValueError(f"field {n}: need C-contiguous complex128 of shape {sh[n]}")
        keep.append(a)
        setattr(f, n, a.ctypes.data_as(C.POINTER(C.c_double)))
    return C.byref(f)


def _czeros(g: Grid):
    return {k: np.zeros(s, dtype=np.complex128) for k, s in g.shapes().items()}


def _probe(U, V, h):
    return {k: np.ascontiguousarray(np.asarray(U[k], dtype=np.float64)
                                    + 1j * h * np.asarray(V[k], dtype=np.float64))
            for k in FIELDS}


def _split(Z, h):
    return ({k: np.ascontiguousarray(v.real) for k, v in Z.items()},
            {k: np.ascontiguousarray(v.imag / h) for k, v in Z.items()})


def jvp_residual(g: Grid, mat: Material, Ubar, V, tau, h=CS_H):
    """(R, dR) for Un = Uk = Ubar + e V at e = 0: R = -tau F_h(Ubar) and
    dR = -tau J_F(Ubar) V (complex step)."""
    keep = []
    Z = _probe(Ubar, V, h)
    R, Ub = _czeros(g), _czeros(g)
    m = mat.c()
    rc = lib_cs().orc_residual(g._h, C.byref(m), _cfields(g, Z, keep), _cfields(g, Z, keep), None,
                               None, float(tau), _cfields(g, R, keep), _cfields(g, Ub, keep))
    assert rc == 0
    return _split(R, h)


def jvp_line_matvec(g: Grid, mat: Material, Ubar, V, tau, d, X, h=CS_H):
    """(y, dy): y = (I + tau/2 D_d(Ubar)) X and its derivative along Ubar -> V."""
    keep = []
    Z = _probe(Ubar, V, h)
    Xc = _probe(X, {k: np.zeros_like(X[k]) for k in FIELDS}, h)
    y = _czeros(g)
    m = mat.c()
    rc = lib_cs().orc_line_matvec(g._h, C.byref(m), _cfields(g, Z, keep), None, float(tau), int(d),
                                  _cfields(g, Xc, keep), _cfields(g, y, keep))
    assert rc == 0
    return _split(y, h)


def jvp_split_step(g: Grid, mat: Material, Un, V, tau, K, h=CS_H):
    """(U^{n+1}, dU^{n+1}): one split step from Un + e V and its derivative
    at e = 0 (complex step)."""
    keep = []
    Z = _probe(Un, V, h)
    out = _czeros(g)
    m = mat.c()
    rc = lib_cs().orc_split_step(g._h, C.byref(m), _cfields(g, Z, keep), _cfields(g, out, keep),
                                 float(tau), int(K), None, None, None, None)
    if rc != 0:
        raise ArithmeticError("zero pivot in a line solve")
    return _split(out, h)
