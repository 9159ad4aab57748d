"""Manufactured solution of the paper (section "Well-prepared manufactured
solution", eq. (man_sol)) and its source terms.

The sources are computed independently of any spherical discretisation: the
exact fields are pushed to Cartesian coordinates, the continuous equations
(nonconservmass), (nonconservmom), (nonconservener) with the stress tensor and
equation of state of section 2.1 are evaluated there by automatic
differentiation (torch.func, float64, CPU), and the momentum residual is
projected back onto the local spherical unit vectors.  No curvature term is
written by hand, so this pins every metric term of the oracle's F_h.

Test infrastructure only.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from torch.func import jacfwd, vmap

torch.set_default_dtype(torch.float64)

P0 = 6250.0
RHO0 = 1.0
DOMAIN = (1.0, 2.0, math.pi / 4, 3 * math.pi / 4, math.pi / 4, 7 * math.pi / 4)


class MMS:
    def __init__(self, mach, mat):
        self.mat = mat
        self.gamma = mat.cp / mat.cv
        self.c0 = math.sqrt(self.gamma * P0 / RHO0)
        self.u0 = mach * self.c0

    # ------------------------------------------------------------ exact --
    def sph(self, r, th, ph, t):
        """exact (p, u_r, u_theta, u_phi, T) in spherical components"""
        u0, c0 = self.u0, self.c0
        p = P0 + u0 ** 2 * (1 + torch.sin(5 * t) + torch.cos(math.pi * r) ** 2 *
                            torch.cos(4 * ph) ** 2 * torch.cos(4 * th) ** 2)
        ur = u0 * (1 + torch.sin(t)) / (2 * r ** 2) + u0 ** 2 / c0 * (
            1 + torch.sin(4 * t) + torch.sin(r ** 2) * torch.cos(th) ** 3 * torch.sin(ph) ** 2)
        ut = u0 * (1 + torch.cos(3 * t + 2)) / (2 * torch.sin(th)) + u0 ** 2 / c0 * (
            1 + torch.sin(t) + torch.cos(r ** 2) ** 3 * torch.cos(th) ** 2 * torch.sin(ph) ** 3)
        uf = u0 * (1 + torch.sin(6 + t)) / 2 + u0 ** 2 / c0 * (
            1 + torch.cos(2 + t) + torch.cos(r) * torch.sin(th) ** 3 * torch.sin(ph) ** 2)
        T = p / (self.mat.cv * (self.gamma - 1.0))
        return p, ur, ut, uf, T

    @staticmethod
    def _sph_of(x):
        r = torch.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
        th = torch.acos(x[2] / r)
        ph = math.pi + torch.atan2(-x[1], -x[0])  # branch cut at phi = 0 (outside the domain)
        return r, th, ph

    @staticmethod
    def _basis(th, ph):
        er = torch.stack([torch.sin(th) * torch.cos(ph), torch.sin(th) * torch.sin(ph), torch.cos(th)])
        et = torch.stack([torch.cos(th) * torch.cos(ph), torch.cos(th) * torch.sin(ph), -torch.sin(th)])
        ef = torch.stack([-torch.sin(ph), torch.cos(ph), torch.zeros_like(ph)])
        return er, et, ef

    def _cart(self, xt):
        """xt = (x, y, z, t) -> (p, u_x, u_y, u_z, T)"""
        x, t = xt[:3], xt[3]
        r, th, ph = self._sph_of(x)
        p, ur, ut, uf, T = self.sph(r, th, ph, t)
        er, et, ef = self._basis(th, ph)
        u = ur * er + ut * et + uf * ef
        return torch.stack([p, u[0], u[1], u[2], T])

    # --------------------------------------------------------- operator --
    def _residual_point(self, xt):
        """continuous dU/dt + F(U) at one point, momentum in Cartesian comps"""
        m = self.mat
        gam = self.gamma
        kap = m.mu * m.cp / m.prandtl
        f = self._cart
        V = f(xt)
        J1 = jacfwd(f)(xt)                # 5 x 4
        H = jacfwd(jacfwd(f))(xt)         # 5 x 4 x 4
        p, u, T = V[0], V[1:4], V[4]
        dpdt, dudt, dTdt = J1[0, 3], J1[1:4, 3], J1[4, 3]
        gp, gT = J1[0, :3], J1[4, :3]
        J = J1[1:4, :3]                   # J[a, b] = d u_a / d x_b
        div = J[0, 0] + J[1, 1] + J[2, 2]
        lapT = H[4, 0, 0] + H[4, 1, 1] + H[4, 2, 2]
        lapu = torch.stack([H[1 + a, 0, 0] + H[1 + a, 1, 1] + H[1 + a, 2, 2] for a in range(3)])
        graddiv = torch.stack([H[1, 0, b] + H[2, 1, b] + H[3, 2, b] for b in range(3)])
        eye = torch.eye(3)
        sig = m.mu * (J + J.T - (2.0 / 3.0) * div * eye)
        Phi = (J * sig).sum()
        P = p + m.pi_inf
        rho = P / (m.cv * (gam - 1.0) * T)
        Fp = u @ gp + gam * P * div - (gam - 1.0) * kap * lapT - (gam - 1.0) * Phi
        chi = (gam - 1.0) * T / P
        FT = u @ gT + (gam - 1.0) * T * div - chi * (kap * lapT + Phi)
        r, th, ph = self._sph_of(xt[:3])
        er, et, ef = self._basis(th, ph)
        ez = torch.tensor([0.0, 0.0, 1.0])
        cor = 2.0 * m.omega * torch.linalg.cross(ez, u)
        Fu = J @ u + gp / rho - (m.mu / rho) * (lapu + graddiv / 3.0) + m.g_r * er + cor
        Su = dudt + Fu
        return torch.stack([dpdt + Fp, Su @ er, Su @ et, Su @ ef, dTdt + FT])

    def _points(self, r, th, ph, t):
        r, th, ph = (torch.as_tensor(np.asarray(a, dtype=np.float64)) for a in (r, th, ph))
        x = torch.stack([r * torch.sin(th) * torch.cos(ph), r * torch.sin(th) * torch.sin(ph),
                         r * torch.cos(th), torch.full_like(r, float(t))], dim=-1)
        return x

    def residual_at(self, r, th, ph, t, chunk=20000):
        """dU/dt + F(U) (spherical comps) at arrays of points: (5, n)"""
        x = self._points(np.ravel(r), np.ravel(th), np.ravel(ph), t)
        outs = []
        fn = vmap(self._residual_point)
        for s in range(0, x.shape[0], chunk):
            outs.append(fn(x[s:s + chunk]))
        return torch.cat(outs).T.numpy()

    # ------------------------------------------------ discrete sampling --
    def _locs(self, g):
        c = g.coords()
        def mesh(a, b, cc):
            return np.meshgrid(a, b, cc, indexing="ij")
        return {
            "p": mesh(c["rc"], c["tc"], c["pc"]), "T": mesh(c["rc"], c["tc"], c["pc"]),
            "ur": mesh(c["rf"], c["tc"], c["pc"]), "ut": mesh(c["rc"], c["tf"], c["pc"]),
            "uf": mesh(c["rc"], c["tc"], c["pf"]),
        }

    def fields(self, g, t):
        """exact solution sampled at the MAC locations"""
        out = {}
        comp = {"p": 0, "ur": 1, "ut": 2, "uf": 3, "T": 4}
        for k, (r, th, ph) in self._locs(g).items():
            vals = self.sph(torch.as_tensor(r), torch.as_tensor(th), torch.as_tensor(ph),
                            torch.tensor(float(t)))
            out[k] = np.ascontiguousarray(vals[comp[k]].numpy())
        return out

    def sources(self, g, t):
        """S = dU/dt + F(U) at the MAC locations"""
        out = {}
        comp = {"p": 0, "ur": 1, "ut": 2, "uf": 3, "T": 4}
        for k, (r, th, ph) in self._locs(g).items():
            res = self.residual_at(r, th, ph, t)
            out[k] = np.ascontiguousarray(res[comp[k]].reshape(r.shape))
        return out

    def wall(self, g, t):
        """tangential wall velocities at the wall points (ghost data)"""
        c = g.coords()
        r1, r2, t1, t2, p1, p2 = g.r1, g.r2, g.t1, g.t2, g.p1, g.p2
        tt = torch.tensor(float(t))

        def ev(comp, r, th, ph):
            r, th, ph = np.broadcast_arrays(r, th, ph)
            v = self.sph(torch.as_tensor(np.array(r, dtype=float)), torch.as_tensor(np.array(th, dtype=float)),
                         torch.as_tensor(np.array(ph, dtype=float)), tt)[comp]
            return np.ascontiguousarray(v.numpy())

        rf, tc, pc, tf, rc, pf = c["rf"], c["tc"], c["pc"], c["tf"], c["rc"], c["pf"]
        return {
            "ur_t1": ev(1, rf[:, None], t1, pc[None, :]), "ur_t2": ev(1, rf[:, None], t2, pc[None, :]),
            "ur_p1": ev(1, rf[:, None], tc[None, :], p1), "ur_p2": ev(1, rf[:, None], tc[None, :], p2),
            "ut_r1": ev(2, r1, tf[:, None], pc[None, :]), "ut_r2": ev(2, r2, tf[:, None], pc[None, :]),
            "ut_p1": ev(2, rc[:, None], tf[None, :], p1), "ut_p2": ev(2, rc[:, None], tf[None, :], p2),
            "uf_r1": ev(3, r1, tc[:, None], pf[None, :]), "uf_r2": ev(3, r2, tc[:, None], pf[None, :]),
            "uf_t1": ev(3, rc[:, None], t1, pf[None, :]), "uf_t2": ev(3, rc[:, None], t2, pf[None, :]),
        }


def sources_interpolator(M, g, t0, t1, nodes=7):
    """S(t) on [t0, t1] by polynomial interpolation of the exact sources at
    Chebyshev nodes"""
    k = np.arange(nodes)
    ts = 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * np.cos((2 * k + 1) * np.pi / (2 * nodes))
    Ss = [M.sources(g, t) for t in ts]

    def S(t):
        w = np.array([np.prod([(t - ts[m]) / (ts[j] - ts[m]) for m in range(nodes) if m != j])
                      for j in range(nodes)])
        return {f: sum(w[j] * Ss[j][f] for j in range(nodes)) for f in Ss[0]}
    return S


def region_mask(g, key, frac=0.25):
    """points whose coordinates lie in the middle of the box (a fixed physical
    region, so that errors at different resolutions are comparable)"""
    c = g.coords()
    names = {"p": ("rc", "tc", "pc"), "T": ("rc", "tc", "pc"), "ur": ("rf", "tc", "pc"),
             "ut": ("rc", "tf", "pc"), "uf": ("rc", "tc", "pf")}[key]
    lims = ((g.r1, g.r2), (g.t1, g.t2), (g.p1, g.p2))
    m = np.ones(g.shapes()[key], dtype=bool)
    for ax, (nm, (lo, hi)) in enumerate(zip(names, lims)):
        x = c[nm]
        w = hi - lo
        sel = (x >= lo + frac * w - 1e-12) & (x <= hi - frac * w + 1e-12)
        shape = [1, 1, 1]
        shape[ax] = len(x)
        m &= sel.reshape(shape)
    return m


def interior_mask(g, key, margin):
    """boolean mask of points at least ``margin`` cells away from every wall"""
    sh = g.shapes()[key]
    m = np.ones(sh, dtype=bool)
    for ax in range(3):
        n = sh[ax]
        idx = np.arange(n)
        face_ax = {"ur": 0, "ut": 1, "uf": 2}.get(key) == ax
        lo = margin + (1 if face_ax else 0)
        hi = n - margin - (1 if face_ax else 0)
        sel = (idx >= lo) & (idx < hi)
        shape = [1, 1, 1]
        shape[ax] = n
        m &= sel.reshape(shape)
    return m


def unknown_mask(g, key):
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


class AxisymmetricField(MMS):
    """A smooth field on the full sphere for pinning the pole rules: symmetric
    about the polar axis and smooth there as a Cartesian field (u_r and the
    scalars functions of cos theta, u_theta and u_phi sin theta times such
    functions), so that across a pole u_r, p and T are even, u_phi is odd and
    u_theta vanishes on the axis, which are the ghost rules of the full-sphere
    reading.  p and T have zero normal derivative on the walls r = 1, 2 (the
    cos^2(pi r) factor), as the boundary conditions require.  The same source
    machinery (Cartesian automatic differentiation of
    the continuous equations) gives F(U)."""

    def sph(self, r, th, ph, t):
        u0, c0 = self.u0, self.c0
        c, s = torch.cos(th), torch.sin(th)
        p = P0 + u0 ** 2 * (1 + torch.sin(t) + torch.cos(math.pi * r) ** 2 * (1 + 0.5 * c + c ** 2))
        ur = u0 * (1 + 0.3 * torch.cos(2 * t)) * (0.2 + torch.sin(r) * c * (1 + c))
        ut = u0 * (1 + 0.2 * torch.sin(t)) * s * torch.cos(r) * (1 + 0.7 * c)
        uf = u0 * (1 + 0.4 * torch.cos(t)) * s * r * (1 - 0.3 * c ** 2)
        T = p / (self.mat.cv * (self.gamma - 1.0)) * (1 + 0.01 * c)
        return p, ur, ut, uf, T


class ZonalShear(MMS):
    """A zonal shear flow u_phi = u0 r^2 sin theta (smooth across the polar
    axis, divergence-free) with uniform p and T: the pressure row of F is then
    the viscous heating -(gamma - 1) grad u : sigma, whose strain component
    S_theta phi = (1/r) d u_phi / d theta - u_phi cot(theta) / r vanishes
    exactly; next to a pole its centred difference reads the u_phi ghost
    across the axis, so this row pins that ghost's sign."""

    def sph(self, r, th, ph, t):
        u0 = self.u0
        z = torch.zeros_like(r * th * ph)
        p = P0 + z + 0.0 * t
        uf = u0 * (1 + 0.5 * torch.sin(t)) * r ** 2 * torch.sin(th)
        T = p / (self.mat.cv * (self.gamma - 1.0))
        return p, z, z, uf, T
