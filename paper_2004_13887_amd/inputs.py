"""Seeded synthetic workloads: grids, materials and initial states.

This module generates inputs only.  It contains none of the time-stepping
method's arithmetic and imports nothing else from this package, so the CPU
oracle's tests and the GPU path can both draw their inputs from it.

Workloads (shapes of the paper's own test problems; the paper uses no public
dataset):

* ``parity``    32 (phi) x 32 (theta) x 16 (r) regional sector, 30 x 30 deg,
                Mach 1e-2, 1 step, K = 3.
* ``global``    512 x 256 x 128 full sphere (phi periodic, theta in [0, pi]),
                Mach 1e-4, 10 steps, K = 3; bubble at 45 deg latitude.
* ``sweeps``    1024 x 512 x 64 regional sector with 100 m horizontal spacing,
                Mach 1e-6, 5 steps, K = 3.
* ``ensemble``  64 regional members, each size uniform in [64, 256] per
                direction, 10 steps, K = 3.
* ``adjoint``   256 x 128 x 64 sector, 100 m horizontal, 10 steps.

Initial data (paper section "Rising thermal bubble" for the physical constants
of dry air and the potential temperature / Exner relation):

* isothermal T0 = 300 K background in discrete hydrostatic balance: the radial
  momentum equation at rest, (1/rho_face)(p_i - p_{i-1})/dr + g = 0 with
  rho_face the mean of the two cell densities, is integrated upward from
  p_0 = p00 exp(-g dr / (2 R T0)), p00 = 1e5 Pa;
* a Gaussian potential-temperature bubble dTheta = A exp(-(L/R_b)^2), L the
  chord distance from the bubble centre, T = T0 + dTheta (p/p00)^{R/c_p};
* face velocities u = M c0 xi, xi ~ U[-1, 1] i.i.d. (u_r array first, then
  u_theta, then u_phi, each in C order), c0 = sqrt(gamma R T0); Dirichlet
  (boundary-normal) faces set to 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

EARTH_R1 = 6371.0e3
SHELL_DEPTH = 10.0e3
P00 = 1.0e5
T0 = 300.0
SEED_BASE = 200413887


@dataclass(frozen=True)
class MaterialSpec:
    cp: float
    cv: float
    pi_inf: float
    mu: float
    prandtl: float
    omega: float
    g_r: float

    @property
    def gamma(self) -> float:
        return self.cp / self.cv

    @property
    def R(self) -> float:
        return self.cp - self.cv

    def astuple(self):
        return (self.cp, self.cv, self.pi_inf, self.mu, self.prandtl, self.omega, self.g_r)


# dry air at about 300 K, as in the paper's bubble tests
AIR = MaterialSpec(cp=1000.0, cv=713.0, pi_inf=0.0, mu=1.846e-5, prandtl=0.71, omega=0.0,
                   g_r=9.80665)
# manufactured-solution test: gamma = 1.6, mu = Pr = 1, no rotation, no gravity
# (c_v = 1 and pi_inf = 0 are not printed in the paper; rho = 1 with
# T = p / (c_v (gamma-1)) requires pi_inf = 0)
MMS = MaterialSpec(cp=1.6, cv=1.0, pi_inf=0.0, mu=1.0, prandtl=1.0, omega=0.0, g_r=0.0)


@dataclass(frozen=True)
class GridSpec:
    nr: int
    nt: int
    np: int
    r1: float
    r2: float
    t1: float
    t2: float
    p1: float
    p2: float
    periodic: bool = False

    @property
    def npf(self) -> int:
        return self.np if self.periodic else self.np + 1

    @property
    def ncells(self) -> int:
        return self.nr * self.nt * self.np

    def shapes(self):
        nr, nt, np_, npf = self.nr, self.nt, self.np, self.npf
        return {"p": (nr, nt, np_), "ur": (nr + 1, nt, np_), "ut": (nr, nt + 1, np_),
                "uf": (nr, nt, npf), "T": (nr, nt, np_)}

    def args(self):
        return (self.nr, self.nt, self.np, self.r1, self.r2, self.t1, self.t2, self.p1, self.p2,
                self.periodic)

    @property
    def pole_lo(self) -> bool:
        return self.t1 == 0.0

    @property
    def pole_hi(self) -> bool:
        return abs(self.t2 - math.pi) <= 1e-12


@dataclass(frozen=True)
class Workload:
    name: str
    grid: GridSpec
    mach: float
    amplitude: float
    steps: int
    K: int
    seed: object
    bubble_theta: float = math.pi / 2
    bubble_phi: float = math.pi
    bubble_height: float = 2.0e3
    bubble_radius: float = 2.0e3
    material: MaterialSpec = AIR
    cfl: float = 5.0


def sector(nr, nt, np_, dtheta, dphi, theta_c=math.pi / 2, phi_c=math.pi):
    return GridSpec(nr, nt, np_, EARTH_R1, EARTH_R1 + SHELL_DEPTH,
                    theta_c - 0.5 * nt * dtheta, theta_c + 0.5 * nt * dtheta,
                    phi_c - 0.5 * np_ * dphi, phi_c + 0.5 * np_ * dphi, False)


def full_sphere(nr, nt, np_):
    return GridSpec(nr, nt, np_, EARTH_R1, EARTH_R1 + SHELL_DEPTH, 0.0, math.pi, 0.0,
                    2.0 * math.pi, True)


H100 = 100.0 / EARTH_R1  # 100 m of arc at r1

WORKLOADS = {
    "parity": Workload("parity", sector(16, 32, 32, math.radians(30) / 32, math.radians(30) / 32),
                       mach=1e-2, amplitude=0.5, steps=1, K=3, seed=SEED_BASE + 1),
    "global": Workload("global", full_sphere(128, 256, 512), mach=1e-4, amplitude=0.5, steps=10,
                       K=3, seed=SEED_BASE + 2, bubble_theta=math.pi / 4),
    "sweeps": Workload("sweeps", sector(64, 512, 1024, H100, H100), mach=1e-6, amplitude=0.5,
                       steps=5, K=3, seed=SEED_BASE + 3),
    "adjoint": Workload("adjoint", sector(64, 128, 256, H100, H100), mach=1e-2, amplitude=0.5,
                        steps=10, K=3, seed=SEED_BASE + 5),
}


def scaled(w: Workload, nr: int, nt: int, np_: int, name: str | None = None) -> Workload:
    """Same recipe on a different grid size (keeps the extents)."""
    g = replace(w.grid, nr=nr, nt=nt, np=np_)
    return replace(w, grid=g, name=name or f"{w.name}-{np_}x{nt}x{nr}")


def ensemble_members(n=64, steps=10, K=3):
    """Uneven regional members: sizes U{64..256} per direction, amplitude
    U[0.1, 1] K, log10 Mach U[-6, -2]; member m drawn from PCG64([200413891, m])
    in the order sizes -> amplitude -> Mach (velocities are drawn later from
    the same generator by ``initial_state``)."""
    out = []
    for m in range(n):
        rng = np.random.Generator(np.random.PCG64([SEED_BASE + 4, m]))
        nphi, nth, nr = (int(x) for x in rng.integers(64, 257, 3))
        amp = float(rng.uniform(0.1, 1.0))
        mach = float(10.0 ** rng.uniform(-6.0, -2.0))
        g = sector(nr, nth, nphi, H100, H100)
        out.append(Workload(f"member{m}", g, mach=mach, amplitude=amp, steps=steps, K=K,
                            seed=("member", m)))
    return out


def _rng(w: Workload):
    if isinstance(w.seed, tuple) and w.seed[0] == "member":
        rng = np.random.Generator(np.random.PCG64([SEED_BASE + 4, w.seed[1]]))
        rng.integers(64, 257, 3)  # replay the draws that fixed the member
        rng.uniform(0.1, 1.0)
        rng.uniform(-6.0, -2.0)
        return rng
    return np.random.Generator(np.random.PCG64(w.seed))


def coords(g: GridSpec):
    dr = (g.r2 - g.r1) / g.nr
    dt = (g.t2 - g.t1) / g.nt
    dp = (g.p2 - g.p1) / g.np
    return {
        "rc": g.r1 + (np.arange(g.nr) + 0.5) * dr, "rf": g.r1 + np.arange(g.nr + 1) * dr,
        "tc": g.t1 + (np.arange(g.nt) + 0.5) * dt, "tf": g.t1 + np.arange(g.nt + 1) * dt,
        "pc": g.p1 + (np.arange(g.np) + 0.5) * dp, "pf": g.p1 + np.arange(g.npf) * dp,
        "dr": dr, "dt": dt, "dp": dp,
    }


def hydrostatic_pressure(g: GridSpec, mat: MaterialSpec, T_bg: float = T0):
    """Discretely balanced isothermal column p_i (cell centres)."""
    dr = (g.r2 - g.r1) / g.nr
    a = mat.g_r * dr / (2.0 * mat.R * T_bg)
    p = np.empty(g.nr)
    p[0] = P00 * math.exp(-a)
    for i in range(1, g.nr):
        p[i] = p[i - 1] * (1.0 - a) / (1.0 + a)
    return p


def reference_column(g: GridSpec, mat: MaterialSpec, T_bar, p_top=None):
    """A discretely hydrostatic reference column (p_bar, T_bar) at the cell
    centres for the perturbation-pressure form: the radial momentum row at
    rest, (p_i - p_{i-1}) / dr + g (rho_{i-1} + rho_i) / 2 = 0 with
    rho = (p + pi_inf) / (R T), solved upward for p_i from
    p_0 = p00 exp(-g dr / (2 R T_0)) (or p_top given for the first centre).
    T_bar: a scalar or nr values."""
    dr = (g.r2 - g.r1) / g.nr
    T = np.broadcast_to(np.asarray(T_bar, dtype=np.float64), (g.nr,)).copy()
    a = mat.g_r * dr / (2.0 * mat.R * T)
    p = np.empty(g.nr)
    p[0] = P00 * math.exp(-a[0]) if p_top is None else float(p_top)
    for i in range(1, g.nr):
        p[i] = (p[i - 1] * (1.0 - a[i - 1]) - mat.pi_inf * (a[i - 1] + a[i])) / (1.0 + a[i])
    return p, T


def time_step(w: Workload, T_max: float) -> float:
    """tau at the workload's acoustic CFL number: cfl * d_min / c_max, with
    d_min = min(dr, r1 dtheta, r1 sin(theta_min) dphi) over cell centres."""
    g, mat = w.grid, w.material
    c = coords(g)
    smin = float(np.min(np.sin(c["tc"])))
    dmin = min(c["dr"], g.r1 * c["dt"], g.r1 * smin * c["dp"])
    cmax = math.sqrt(mat.gamma * mat.R * T_max)
    return w.cfl * dmin / cmax


def initial_state(w: Workload):
    """(fields, tau) for a workload; fields is a dict of C-contiguous float64."""
    g, mat = w.grid, w.material
    rng = _rng(w)
    c = coords(g)
    sh = g.shapes()
    pcol = hydrostatic_pressure(g, mat)
    p = np.broadcast_to(pcol[:, None, None], sh["p"]).copy()
    # bubble: chord distance from the centre, 2 km above r1 (separable in
    # r, theta, phi: trigonometry on the 1-D coordinates, then broadcast)
    rb = g.r1 + w.bubble_height
    xb = rb * np.sin(w.bubble_theta) * np.cos(w.bubble_phi)
    yb = rb * np.sin(w.bubble_theta) * np.sin(w.bubble_phi)
    zb = rb * np.cos(w.bubble_theta)
    r3 = c["rc"][:, None, None]
    st, ct = np.sin(c["tc"])[None, :, None], np.cos(c["tc"])[None, :, None]
    sp, cp = np.sin(c["pc"])[None, None, :], np.cos(c["pc"])[None, None, :]
    x = r3 * st * cp - xb
    y = r3 * st * sp - yb
    z = r3 * ct - zb
    L2 = (x * x + y * y + z * z) / (w.bubble_radius ** 2)
    del x, y, z
    # exp(-L2) is exactly 0 in FP64 beyond L2 = 746: evaluate it only nearer
    near = L2 < 750.0
    dtheta = np.zeros(sh["p"])
    dtheta[near] = w.amplitude * np.exp(-L2[near])
    exner = ((pcol / P00) ** (mat.R / mat.cp))[:, None, None]
    T = T0 + dtheta * exner
    c0 = math.sqrt(mat.gamma * mat.R * T0)
    scale = w.mach * c0
    ur = scale * rng.uniform(-1.0, 1.0, sh["ur"])
    ut = scale * rng.uniform(-1.0, 1.0, sh["ut"])
    uf = scale * rng.uniform(-1.0, 1.0, sh["uf"])
    ur[0] = 0.0
    ur[-1] = 0.0
    ut[:, 0] = 0.0
    ut[:, -1] = 0.0
    if not g.periodic:
        uf[:, :, 0] = 0.0
        uf[:, :, -1] = 0.0
    fields = {"p": p, "ur": ur, "ut": ut, "uf": uf, "T": np.ascontiguousarray(T)}
    fields = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in fields.items()}
    tau = time_step(w, float(T.max()))
    return fields, tau


# ------------------------------------------------ rising thermal bubble --

def thermal1_grid(nr=100, nt=200, np_=200) -> GridSpec:
    """The paper's "Thermal 1" domain (section "Rising thermal bubble"):
    r in [6371, 6381] km, theta in pi/2 +- 10/6371, phi in pi +- 10/6371
    (20 km x 20 km x 10 km); 100 x 200 x 200 MAC cells by default."""
    half = 10.0e3 / EARTH_R1
    return GridSpec(nr, nt, np_, EARTH_R1, EARTH_R1 + SHELL_DEPTH, math.pi / 2 - half,
                    math.pi / 2 + half, math.pi - half, math.pi + half, False)


def exner_column(g: GridSpec, mat: MaterialSpec, theta0: float = T0):
    """Discretely hydrostatic column at constant potential temperature
    theta0: centre pressures p_i with T_i = theta0 (p_i / p00)^(R/c_p) and
    p_i (1 + g dr / (2 R T_i)) = p_{i-1} (1 - g dr / (2 R T_{i-1})) (the u_r
    equation at rest with the face density the mean of the two centres); the
    first centre from the continuous profile pi = 1 - g z / (c_p theta0) half a
    cell above r1, where p = p00.  Returns (p, T) of the column."""
    dr = (g.r2 - g.r1) / g.nr
    kap = mat.R / mat.cp
    c = mat.g_r * dr / (2.0 * mat.R)
    p = np.empty(g.nr)
    T = np.empty(g.nr)
    p[0] = P00 * (1.0 - mat.g_r * 0.5 * dr / (mat.cp * theta0)) ** (1.0 / kap)
    T[0] = theta0 * (p[0] / P00) ** kap
    for i in range(1, g.nr):
        top = p[i - 1] * (1.0 - c / T[i - 1])
        pi_ = top / (1.0 + c / T[i - 1])
        for _ in range(50):  # fixed point in T_i (contraction factor ~ g dr / (R T))
            Ti = theta0 * (pi_ / P00) ** kap
            nxt = top / (1.0 + c / Ti)
            if nxt == pi_:
                break
            pi_ = nxt
        p[i] = pi_
        T[i] = theta0 * (p[i] / P00) ** kap
    return p, T


def thermal1_state(g: GridSpec, mat: MaterialSpec = AIR, theta0: float = T0, amplitude: float = 2.0,
                   radius: float = 2.0e3, height: float = 2.0e3, theta_c: float = math.pi / 2,
                   phi_c: float = math.pi):
    """Thermal 1 initial state: fluid at rest in the column of exner_column,
    the potential temperature raised by 2 cos^2(pi L / 2) where L (the chord
    distance to the centre, 2 km above r1, over R = 2 km) is <= 1, the
    pressure unchanged (T = (theta0 + dTheta) (p / p00)^(R/c_p))."""
    c = coords(g)
    sh = g.shapes()
    pcol, _ = exner_column(g, mat, theta0)
    rb = g.r1 + height
    xb = rb * math.sin(theta_c) * math.cos(phi_c)
    yb = rb * math.sin(theta_c) * math.sin(phi_c)
    zb = rb * math.cos(theta_c)
    r3 = c["rc"][:, None, None]
    st, ct = np.sin(c["tc"])[None, :, None], np.cos(c["tc"])[None, :, None]
    sp, cp = np.sin(c["pc"])[None, None, :], np.cos(c["pc"])[None, None, :]
    L = np.sqrt((r3 * st * cp - xb) ** 2 + (r3 * st * sp - yb) ** 2 + (r3 * ct - zb) ** 2) / radius
    dth = np.where(L <= 1.0, amplitude * np.cos(0.5 * math.pi * L) ** 2, 0.0)
    exner = ((pcol / P00) ** (mat.R / mat.cp))[:, None, None]
    fields = {"p": np.broadcast_to(pcol[:, None, None], sh["p"]), "ur": np.zeros(sh["ur"]),
              "ut": np.zeros(sh["ut"]), "uf": np.zeros(sh["uf"]), "T": (theta0 + dth) * exner}
    return {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in fields.items()}


def thermal2_grid(nr=200, nt=200, np_=200) -> GridSpec:
    """The paper's "Thermal 2" domain (section "Rising thermal bubble"): a
    1 km cube, theta in pi/2 +- 0.5/6371, phi in pi +- 0.5/6371, r from
    6371 km up by 1 km (the printed radial interval is garbled; 1 km is the
    span the cube and the bubble imply); 200^3 MAC cells by default."""
    half = 0.5e3 / EARTH_R1
    return GridSpec(nr, nt, np_, EARTH_R1, EARTH_R1 + 1.0e3, math.pi / 2 - half, math.pi / 2 + half,
                    math.pi - half, math.pi + half, False)


def thermal2_state(g: GridSpec, mat: MaterialSpec = AIR, theta0: float = T0):
    """Thermal 2 initial state: as thermal1_state with the perturbation
    (1 + cos(pi L)) / 4 K for L <= 1, R = 250 m, centred 260 m above r1."""
    c = coords(g)
    sh = g.shapes()
    pcol, _ = exner_column(g, mat, theta0)
    rb = g.r1 + 260.0
    xb, yb, zb = -rb, 0.0, 0.0  # theta = pi/2, phi = pi
    r3 = c["rc"][:, None, None]
    st, ct = np.sin(c["tc"])[None, :, None], np.cos(c["tc"])[None, :, None]
    sp, cp = np.sin(c["pc"])[None, None, :], np.cos(c["pc"])[None, None, :]
    L = np.sqrt((r3 * st * cp - xb) ** 2 + (r3 * st * sp - yb) ** 2 + (r3 * ct - zb) ** 2) / 250.0
    dth = np.where(L <= 1.0, 0.25 * (1.0 + np.cos(math.pi * L)), 0.0)
    exner = ((pcol / P00) ** (mat.R / mat.cp))[:, None, None]
    fields = {"p": np.broadcast_to(pcol[:, None, None], sh["p"]), "ur": np.zeros(sh["ur"]),
              "ut": np.zeros(sh["ut"]), "uf": np.zeros(sh["uf"]), "T": (theta0 + dth) * exner}
    return {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in fields.items()}


def potential_temperature_excess(g: GridSpec, U, mat: MaterialSpec = AIR, theta0: float = T0):
    """Theta - theta0 at the cell centres, Theta = T / (p / p00)^(R/c_p)."""
    return U["T"] / (U["p"] / P00) ** (mat.R / mat.cp) - theta0


def random_fields(g: GridSpec, seed: int, base=None, scale=1.0):
    """Random perturbation fields (for line-solve tests): base + scale * U[-1,1]
    at every unknown, 0 on boundary-normal faces."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {}
    for k, s in g.shapes().items():
        a = scale * rng.uniform(-1.0, 1.0, s)
        if base is not None:
            a = a + base[k]
        out[k] = np.ascontiguousarray(a)
    out["ur"][0] = 0.0
    out["ur"][-1] = 0.0
    out["ut"][:, 0] = 0.0
    out["ut"][:, -1] = 0.0
    if not g.periodic:
        out["uf"][:, :, 0] = 0.0
        out["uf"][:, :, -1] = 0.0
    return out


# ------------------------------------------------- adjoint-check workload --

def adjoint_box_weights(w: Workload, half_width=2.5e3, r_lo=1.0e3, r_hi=3.0e3):
    """Cell volumes of the cells whose centre lies in the box of the adjoint
    check (zero elsewhere), shape (nr, nt, np): horizontally within
    +-half_width of the bubble centre, measured as arc length at r1, and
    radially in [r1 + r_lo, r1 + r_hi].  Exact spherical cell volumes
    (r^3/3) dcos(theta) dphi."""
    g = w.grid
    c = coords(g)
    vol_r = (c["rf"][1:] ** 3 - c["rf"][:-1] ** 3) / 3.0
    vol_t = np.cos(c["tf"][:-1]) - np.cos(c["tf"][1:])
    vol = vol_r[:, None, None] * vol_t[None, :, None] * c["dp"]
    in_r = (c["rc"] >= g.r1 + r_lo) & (c["rc"] <= g.r1 + r_hi)
    in_t = np.abs(c["tc"] - w.bubble_theta) * g.r1 <= half_width
    in_p = np.abs(c["pc"] - w.bubble_phi) * g.r1 <= half_width
    mask = in_r[:, None, None] & in_t[None, :, None] & in_p[None, None, :]
    return np.where(mask, vol, 0.0)


def exner(p, mat: MaterialSpec):
    """(p / p00)^(R / c_p): potential temperature Theta = T / exner(p)"""
    return (p / P00) ** (mat.R / mat.cp)


def adjoint_directions(shape, n=32):
    """seeded perturbation directions of Theta0 (K per cell), N(0, 1)"""
    return [np.random.Generator(np.random.PCG64([SEED_BASE + 5, 1000 + j])).standard_normal(shape)
            for j in range(n)]
