"""Continuous direction operators D_r, D_theta, D_phi of the paper's
Appendix B (eqs. (dr), (dtheta), (dphi) with the operators A1..C3 listed
there), evaluated by automatic differentiation in spherical coordinates.

Used to check that the oracle's discrete direction split converges to the
paper's continuous one.  Readings of the appendix: operators act on the
operand v (the appendix writes B2^{theta,phi} on u); A2^phi and C2^phi carry
no 2 G_phiphi cot(theta) v_phi / r term (no such term arises from
grad(u):sigma(v), whose v_phi-only parts are -v_phi/r in G_phi r and
-v_phi cot(theta)/r in G_phi theta).

Test infrastructure only.
"""
import torch
from torch.func import jacfwd, vmap

torch.set_default_dtype(torch.float64)


def direction_ops(fields_fn, mat, q):
    """fields_fn(q) -> (p, ur, ut, uf, T) at q = (r, theta, phi);
    returns a (3, 5) tensor: rows d = r, theta, phi; cols p, ur, ut, uf, T
    of D_d(U) U at q."""
    gam = mat.cp / mat.cv
    mu = mat.mu
    kap = mat.mu * mat.cp / mat.prandtl
    F = fields_fn
    V = F(q)
    J = jacfwd(F)(q)
    r, th = q[0], q[1]
    s, c = torch.sin(th), torch.cos(th)
    ct = c / s
    p, ur, ut, uf, T = V
    P = p + mat.pi_inf
    rho = P / ((mat.cp - mat.cv) * T)
    chi = (gam - 1.0) * T / P
    # velocity gradient (physical components)
    Grr = J[1, 0]
    Gtt = J[2, 1] / r + ur / r
    Gff = J[3, 2] / (r * s) + ur / r + ut * ct / r
    Grt = J[2, 0]
    Gtr = J[1, 1] / r - ut / r
    Grf = J[3, 0]
    Gfr = J[1, 2] / (r * s) - uf / r
    Gtf = J[3, 1] / r
    Gft = J[2, 2] / (r * s) - uf * ct / r
    tr = Grr + Gtt + Gff

    def d_(fn, axis):
        return jacfwd(fn)(q)[axis]

    # pieces as functions of q so that they can be differentiated again
    div_r = d_(lambda x: x[0] ** 2 * F(x)[1], 0) / r ** 2
    div_t = d_(lambda x: torch.sin(x[1]) * F(x)[2], 1) / (r * s)
    div_f = J[3, 2] / (r * s)
    lap_r = lambda comp: d_(lambda x: x[0] ** 2 * jacfwd(F)(x)[comp, 0], 0) / r ** 2
    lap_t = lambda comp: d_(lambda x: torch.sin(x[1]) * jacfwd(F)(x)[comp, 1], 1) / (r ** 2 * s)
    lap_f = lambda comp: d_(lambda x: jacfwd(F)(x)[comp, 2], 2) / (r ** 2 * s ** 2)

    def gd_r():  # d/dr of (1/r^2) d/dr (r^2 v_r)
        return d_(lambda x: jacfwd(lambda y: y[0] ** 2 * F(y)[1])(x)[0] / x[0] ** 2, 0)

    def gd_t():  # (1/r) d/dtheta of (1/(r sin)) d/dtheta (sin v_theta)
        return d_(lambda x: jacfwd(lambda y: torch.sin(y[1]) * F(y)[2])(x)[1] /
                  (x[0] * torch.sin(x[1])), 1) / r

    def gd_f():  # (1/(r sin)) d/dphi of (1/(r sin)) d/dphi v_phi
        return d_(lambda x: jacfwd(F)(x)[3, 2] / (x[0] * torch.sin(x[1])), 2) / (r * s)

    out = []
    # ---- r
    A2 = (gam * P + 2 * mu * (gam - 1) / 3 * tr) * div_r - 2 * mu * (gam - 1) * Grr * J[1, 0] \
        - 2 * mu * (gam - 1) * (Gtt + Gff) * ur / r
    C2 = ((gam - 1) * T + 2 * mu * chi / 3 * tr) * div_r - 2 * mu * chi * Grr * J[1, 0] \
        - 2 * mu * chi * (Gtt + Gff) * ur / r
    out.append(torch.stack([
        ur * J[0, 0] + A2 - (gam - 1) * kap * lap_r(4),
        J[0, 0] / rho + ur * J[1, 0] - mu / rho * lap_r(1) - mu / (3 * rho) * gd_r(),
        ur * J[2, 0] - mu / rho * lap_r(2),
        ur * J[3, 0] - mu / rho * lap_r(3),
        C2 + ur * J[4, 0] - chi * kap * lap_r(4),
    ]))
    # ---- theta
    A2 = (gam * P + 2 * mu * (gam - 1) / 3 * tr) * div_t - 2 * mu * (gam - 1) * Gtt / r * J[2, 1] \
        - mu * (gam - 1) * (2 * Gff * ct - Grt - Gtr) * ut / r
    C2 = ((gam - 1) * T + 2 * mu * chi / 3 * tr) * div_t - 2 * mu * chi * Gtt / r * J[2, 1] \
        - mu * chi * (2 * Gff * ct - Grt - Gtr) * ut / r
    out.append(torch.stack([
        ut / r * J[0, 1] + A2 - (gam - 1) * kap * lap_t(4),
        ut / r * J[1, 1] - mu / rho * lap_t(1),
        J[0, 1] / (rho * r) + ut / r * J[2, 1] - mu / rho * lap_t(2) - mu / (3 * rho) * gd_t(),
        ut / r * J[3, 1] - mu / rho * lap_t(3),
        C2 + ut / r * J[4, 1] - chi * kap * lap_t(4),
    ]))
    # ---- phi
    A2 = (gam * P + 2 * mu * (gam - 1) / 3 * (Grr + Gtt - 2 * Gff)) * div_f \
        - mu * (gam - 1) * (-(Gft + Gtf) * ct - Grf - Gfr) * uf / r
    C2 = ((gam - 1) * T + 2 * mu * chi / 3 * (Grr + Gtt - 2 * Gff)) * div_f \
        - mu * chi * (-(Gft + Gtf) * ct - Grf - Gfr) * uf / r
    out.append(torch.stack([
        uf / (r * s) * J[0, 2] + A2 - (gam - 1) * kap * lap_f(4),
        uf / (r * s) * J[1, 2] - mu / rho * lap_f(1),
        uf / (r * s) * J[2, 2] - mu / rho * lap_f(2),
        J[0, 2] / (rho * r * s) + uf / (r * s) * J[3, 2] - mu / rho * lap_f(3) - mu / (3 * rho) * gd_f(),
        C2 + uf / (r * s) * J[4, 2] - chi * kap * lap_f(4),
    ]))
    return torch.stack(out)


def direction_ops_at(fields_fn, mat, r, th, ph):
    q = torch.stack([torch.as_tensor(r).ravel(), torch.as_tensor(th).ravel(),
                     torch.as_tensor(ph).ravel()], dim=-1)
    fn = vmap(lambda x: direction_ops(fields_fn, mat, x))
    outs = [fn(q[s:s + 8000]) for s in range(0, q.shape[0], 8000)]
    return torch.cat(outs).numpy()  # (n, 3, 5)
