// residual.hip -- right-hand side of the first split sweep (paper eq. (spl1)):
//   R = -(Uk - Un) - tau * F_h(Ubar),  Ubar = (Uk + Un)/2,
// F_h(V) = (D + D_M)(V) V + G is the full discrete operator of the
// non-conservative system (nonconservmass)-(nonconservener) in spherical
// components (Appendix B): advection with curvature terms, pressure gradient,
// compressibility terms, vector Laplacian + grad-div viscosity, viscous
// heating, heat conduction, Coriolis and gravity.
//
// One thread per point of the extended index space (nr+1) x (nt+1) x npf; a
// thread owns the centre (i,j,k) and the three faces with the same indices.
// The midpoint state is formed on the fly from Un and Uk (both read through
// the caches), so the pass reads Un, Uk and writes Ubar, R once each.
#include "dsw_common.hpp"
#include "dsw_internal.hpp"

namespace dsw {

template <class S>
__device__ double F_p_T(const Geo &g, const Mat &m, const S &s, int i, int j, int k, double *FT) {
  Cent c;
  centre(g, m, s, i, j, k, c);
  const double r = g.rc[i], sn = g.sc[j];
  double advp = c.ur * (gC(g, s, F_P, i + 1, j, k) - gC(g, s, F_P, i - 1, j, k)) / (2.0 * g.dr) +
                c.ut / r * (gC(g, s, F_P, i, j + 1, k) - gC(g, s, F_P, i, j - 1, k)) / (2.0 * g.dt) +
                c.uf / (r * sn) * (gC(g, s, F_P, i, j, k + 1) - gC(g, s, F_P, i, j, k - 1)) / (2.0 * g.dp);
  double advT = c.ur * (gC(g, s, F_T, i + 1, j, k) - gC(g, s, F_T, i - 1, j, k)) / (2.0 * g.dr) +
                c.ut / r * (gC(g, s, F_T, i, j + 1, k) - gC(g, s, F_T, i, j - 1, k)) / (2.0 * g.dt) +
                c.uf / (r * sn) * (gC(g, s, F_T, i, j, k + 1) - gC(g, s, F_T, i, j, k - 1)) / (2.0 * g.dp);
  const double T0 = c.T;
  double lap =
      (g.rf[i + 1] * g.rf[i + 1] * (gC(g, s, F_T, i + 1, j, k) - T0) -
       g.rf[i] * g.rf[i] * (T0 - gC(g, s, F_T, i - 1, j, k))) / (r * r * g.dr * g.dr) +
      (g.sf[j + 1] * (gC(g, s, F_T, i, j + 1, k) - T0) - g.sf[j] * (T0 - gC(g, s, F_T, i, j - 1, k))) /
          (r * r * sn * g.dt * g.dt) +
      (gC(g, s, F_T, i, j, k + 1) - 2.0 * T0 + gC(g, s, F_T, i, j, k - 1)) / (r * r * sn * sn * g.dp * g.dp);
  double phi = m.mu * (2.0 * (c.Grr * c.Grr + c.Gtt * c.Gtt + c.Gff * c.Gff) + c.Srt * c.Srt +
                       c.Srf * c.Srf + c.Stf * c.Stf - (2.0 / 3.0) * c.tr * c.div);
  *FT = advT + (m.gam - 1.0) * c.T * c.div - c.chi * phi - c.chi * m.kap * lap;
  return advp + m.gam * c.P * c.div - (m.gam - 1.0) * phi - (m.gam - 1.0) * m.kap * lap;
}

template <class S>
__device__ double F_ur(const Geo &g, const Mat &m, const S &s, int f, int j, int k) {
  const double rF = g.rf[f], sn = g.sc[j];
  const double rho = 0.5 * (rho_at(g, m, s, f - 1, j, k) + rho_at(g, m, s, f, j, k));
  const double nu = m.mu / rho;
  const double un = gR(g, s, f, j, k);
  const double ua = 0.25 * (gT(g, s, f - 1, j, k) + gT(g, s, f - 1, j + 1, k) + gT(g, s, f, j, k) +
                            gT(g, s, f, j + 1, k));
  const double ub = 0.25 * (gF(g, s, f - 1, j, k) + gF(g, s, f - 1, j, k + 1) + gF(g, s, f, j, k) +
                            gF(g, s, f, j, k + 1));
  const double xp = gR(g, s, f + 1, j, k), xm = gR(g, s, f - 1, j, k);
  const double yp = gR(g, s, f, j + 1, k), ym = gR(g, s, f, j - 1, k);
  const double zp = gR(g, s, f, j, k + 1), zm = gR(g, s, f, j, k - 1);
  double N = (gC(g, s, F_P, f, j, k) - gC(g, s, F_P, f - 1, j, k)) / (rho * g.dr);
  N += un * (xp - xm) / (2.0 * g.dr) + ua / rF * (yp - ym) / (2.0 * g.dt) +
       ub / (rF * sn) * (zp - zm) / (2.0 * g.dp) - (ua * ua + ub * ub) / rF;
  double vis = (g.rc[f] * g.rc[f] * (xp - un) - g.rc[f - 1] * g.rc[f - 1] * (un - xm)) / (rF * rF * g.dr * g.dr) +
               (g.sf[j + 1] * (yp - un) - g.sf[j] * (un - ym)) / (rF * rF * sn * g.dt * g.dt) +
               (zp - 2.0 * un + zm) / (rF * rF * sn * sn * g.dp * g.dp);
  const double dth = 0.5 *
                     ((g.sf[j + 1] * gT(g, s, f - 1, j + 1, k) - g.sf[j] * gT(g, s, f - 1, j, k)) +
                      (g.sf[j + 1] * gT(g, s, f, j + 1, k) - g.sf[j] * gT(g, s, f, j, k))) / g.dt;
  const double dph = 0.5 *
                     ((gF(g, s, f - 1, j, k + 1) - gF(g, s, f - 1, j, k)) +
                      (gF(g, s, f, j, k + 1) - gF(g, s, f, j, k))) / g.dp;
  vis += -2.0 * un / (rF * rF) - 2.0 / (rF * rF * sn) * dth - 2.0 / (rF * rF * sn) * dph;
  const double gd = (divc(g, s, f, j, k) - divc(g, s, f - 1, j, k)) / g.dr;
  N += -2.0 * m.omega * sn * ub;
  return N - nu * vis - nu / 3.0 * gd + m.g_r;
}

template <class S>
__device__ double F_ut(const Geo &g, const Mat &m, const S &s, int i, int f, int k) {
  const double r = g.rc[i], sF = g.sf[f], ctF = g.cf[f] / g.sf[f];
  const int j0 = f - 1, j1 = f;
  const double rho = 0.5 * (rho_at(g, m, s, i, j0, k) + rho_at(g, m, s, i, j1, k));
  const double nu = m.mu / rho;
  const double un = gT(g, s, i, f, k);
  const double ua = 0.25 * (gR(g, s, i, j0, k) + gR(g, s, i, j1, k) + gR(g, s, i + 1, j0, k) +
                            gR(g, s, i + 1, j1, k));
  const double ub = 0.25 * (gF(g, s, i, j0, k) + gF(g, s, i, j0, k + 1) + gF(g, s, i, j1, k) +
                            gF(g, s, i, j1, k + 1));
  const double xp = gT(g, s, i + 1, f, k), xm = gT(g, s, i - 1, f, k);
  const double yp = gT(g, s, i, f + 1, k), ym = gT(g, s, i, f - 1, k);
  const double zp = gT(g, s, i, f, k + 1), zm = gT(g, s, i, f, k - 1);
  double N = (gC(g, s, F_P, i, j1, k) - gC(g, s, F_P, i, j0, k)) / (rho * r * g.dt);
  N += ua * (xp - xm) / (2.0 * g.dr) + un / r * (yp - ym) / (2.0 * g.dt) +
       ub / (r * sF) * (zp - zm) / (2.0 * g.dp) + (un * ua - ub * ub * ctF) / r;
  double vis = (g.rf[i + 1] * g.rf[i + 1] * (xp - un) - g.rf[i] * g.rf[i] * (un - xm)) / (r * r * g.dr * g.dr) +
               (g.sc[j1] * (yp - un) - g.sc[j0] * (un - ym)) / (r * r * sF * g.dt * g.dt) +
               (zp - 2.0 * un + zm) / (r * r * sF * sF * g.dp * g.dp);
  const double dthr = 0.5 * ((gR(g, s, i, j1, k) - gR(g, s, i, j0, k)) + (gR(g, s, i + 1, j1, k) - gR(g, s, i + 1, j0, k))) / g.dt;
  const double dphf = 0.5 * ((gF(g, s, i, j0, k + 1) - gF(g, s, i, j0, k)) + (gF(g, s, i, j1, k + 1) - gF(g, s, i, j1, k))) / g.dp;
  vis += -un / (r * r * sF * sF) + 2.0 / (r * r) * dthr - 2.0 * ctF / (r * r * sF) * dphf;
  const double gd = (divc(g, s, i, j1, k) - divc(g, s, i, j0, k)) / (r * g.dt);
  N += -2.0 * m.omega * g.cf[f] * ub;
  return N - nu * vis - nu / 3.0 * gd;
}

template <class S>
__device__ double F_uf(const Geo &g, const Mat &m, const S &s, int i, int j, int f) {
  const double r = g.rc[i], sn = g.sc[j], ct = g.cc[j] / g.sc[j];
  const int k0 = g.periodic ? wrapk(g, f - 1) : f - 1, k1 = g.periodic ? wrapk(g, f) : f;
  const double rho = 0.5 * (rho_at(g, m, s, i, j, k0) + rho_at(g, m, s, i, j, k1));
  const double nu = m.mu / rho;
  const double un = gF(g, s, i, j, f);
  const double ua = 0.25 * (gR(g, s, i, j, k0) + gR(g, s, i, j, k1) + gR(g, s, i + 1, j, k0) +
                            gR(g, s, i + 1, j, k1));
  const double ub = 0.25 * (gT(g, s, i, j, k0) + gT(g, s, i, j, k1) + gT(g, s, i, j + 1, k0) +
                            gT(g, s, i, j + 1, k1));
  const double xp = gF(g, s, i + 1, j, f), xm = gF(g, s, i - 1, j, f);
  const double yp = gF(g, s, i, j + 1, f), ym = gF(g, s, i, j - 1, f);
  const double zp = gF(g, s, i, j, f + 1), zm = gF(g, s, i, j, f - 1);
  double N = (gC(g, s, F_P, i, j, k1) - gC(g, s, F_P, i, j, k0)) / (rho * r * sn * g.dp);
  N += ua * (xp - xm) / (2.0 * g.dr) + ub / r * (yp - ym) / (2.0 * g.dt) +
       un / (r * sn) * (zp - zm) / (2.0 * g.dp) + un * (ua + ub * ct) / r;
  double vis = (g.rf[i + 1] * g.rf[i + 1] * (xp - un) - g.rf[i] * g.rf[i] * (un - xm)) / (r * r * g.dr * g.dr) +
               (g.sf[j + 1] * (yp - un) - g.sf[j] * (un - ym)) / (r * r * sn * g.dt * g.dt) +
               (zp - 2.0 * un + zm) / (r * r * sn * sn * g.dp * g.dp);
  const double dphr = 0.5 * ((gR(g, s, i, j, k1) - gR(g, s, i, j, k0)) + (gR(g, s, i + 1, j, k1) - gR(g, s, i + 1, j, k0))) / g.dp;
  const double dpht = 0.5 * ((gT(g, s, i, j, k1) - gT(g, s, i, j, k0)) + (gT(g, s, i, j + 1, k1) - gT(g, s, i, j + 1, k0))) / g.dp;
  vis += -un / (r * r * sn * sn) + 2.0 / (r * r * sn) * dphr + 2.0 * ct / (r * r * sn) * dpht;
  const double gd = (divc(g, s, i, j, k1) - divc(g, s, i, j, k0)) / (r * sn * g.dp);
  N += 2.0 * m.omega * (g.cc[j] * ub + sn * ua);
  return N - nu * vis - nu / 3.0 * gd;
}

__global__ void __launch_bounds__(256) k_residual(Geo g, Mat m, SrcMid s, double tau, Fields R,
                                                  Fields Ub, int *status) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int i = blockIdx.z;
  if (k >= g.npf) return;
  const bool kc = k < g.np;
  // cell centre
  if (i < g.nr && j < g.nt && kc) {
    const long x = idx_c(g, i, j, k);
    const double ubp = s.ld(F_P, x), ubT = s.ld(F_T, x);
    Ub.p[x] = ubp;
    Ub.T[x] = ubT;
    if (!(ubT > 0.0) || !(ubp + m.pinf > 0.0)) status[ST_NONPHYS] = 1; // plain vector store
    double FT;
    const double Fp = F_p_T(g, m, s, i, j, k, &FT);
    R.p[x] = -(s.k[F_P][x] - s.n[F_P][x]) - tau * Fp;
    R.T[x] = -(s.k[F_T][x] - s.n[F_T][x]) - tau * FT;
  }
  // r face i
  if (j < g.nt && kc) {
    const long x = idx_r(g, i, j, k);
    Ub.ur[x] = s.ld(F_UR, x);
    R.ur[x] = (i >= 1 && i < g.nr) ? -(s.k[F_UR][x] - s.n[F_UR][x]) - tau * F_ur(g, m, s, i, j, k) : 0.0;
  }
  // theta face j
  if (i < g.nr && kc) {
    const long x = idx_t(g, i, j, k);
    Ub.ut[x] = s.ld(F_UT, x);
    R.ut[x] = (j >= 1 && j < g.nt) ? -(s.k[F_UT][x] - s.n[F_UT][x]) - tau * F_ut(g, m, s, i, j, k) : 0.0;
  }
  // phi face k
  if (i < g.nr && j < g.nt) {
    const long x = idx_f(g, i, j, k);
    Ub.uf[x] = s.ld(F_UF, x);
    const bool interior = g.periodic || (k >= 1 && k < g.np);
    R.uf[x] = interior ? -(s.k[F_UF][x] - s.n[F_UF][x]) - tau * F_uf(g, m, s, i, j, k) : 0.0;
  }
}

void launch_residual(const Geo &g, const Mat &m, const Fields &Un, const Fields &Uk, double tau,
                     const Fields &R, const Fields &Ub, int *status, hipStream_t st) {
  SrcMid s;
  s.n[F_P] = Un.p; s.n[F_UR] = Un.ur; s.n[F_UT] = Un.ut; s.n[F_UF] = Un.uf; s.n[F_T] = Un.T;
  s.k[F_P] = Uk.p; s.k[F_UR] = Uk.ur; s.k[F_UT] = Uk.ut; s.k[F_UF] = Uk.uf; s.k[F_T] = Uk.T;
  dim3 block(64, 1, 1);
  dim3 grid((g.npf + 63) / 64, g.nt + 1, g.nr + 1);
  hipLaunchKernelGGL(k_residual, grid, block, 0, st, g, m, s, tau, R, Ub, status);
}

} // namespace dsw
