// residual.hip -- right-hand side of the first split sweep (paper eq. (spl1)):
//   R = -(Uk - Un) - tau * F_h(Ubar),  Ubar = (Uk + Un)/2,
// F_h(V) = (D + D_M)(V) V + G is the full discrete operator of the
// non-conservative system (nonconservmass)-(nonconservener) in spherical
// components (Appendix B): advection with curvature terms, pressure gradient,
// compressibility terms, viscosity, viscous heating, heat conduction,
// Coriolis and gravity.
//
// Viscosity: -(mu/rho) (Lap u + grad div u / 3) = -(mu/rho) V with
// V = (4/3) grad(div u) - curl(curl u) on the MAC complex: the divergence at
// cell centres, the vorticity at cell edges (circulation round the dual face
// over its area), its curl at a face (circulation round the face over the
// face area).  Then div(curl) vanishes identically and a discretely
// solenoidal velocity field keeps a solenoidal viscous update.  A radial
// circulation r_a u_a - r_b u_b over centres r_a = r_f + dr/2, r_b = r_f - dr/2
// is formed as r_f (u_a - u_b) + dr (u_a + u_b) / 2 (the same value, without
// the cancellation of two products of size r).  The phi rows next to a pole
// keep the component form (the edge vorticity on the polar axis is one value
// for the whole ring).
//
// One thread per point of the extended index space (nr+1) x (nt+1) x npf; a
// thread owns the centre (i,j,k) and the three faces with the same indices.
// Two variants:
//   * the C-ABI call forms the midpoint on the fly from Un and Uk and writes it;
//   * inside a split step the midpoint is already resident (written by the
//     previous iteration's last sweep, or U^n itself at the first iteration),
//     so every neighbour read is a single load.
#include <algorithm>
#include <type_traits>

#include "dsw_common.hpp"
#include "dsw_internal.hpp"

namespace dsw {

template <class S>
__device__ __forceinline__ double F_p_T(const Geo &g, const Mat &m, const S &s, int i, int j, int k, double *FT) {
  Cent c;
  centre(g, m, s, i, j, k, c);
  const double ir = g.irc[i], is = g.isc[j];
  const double hr = 0.5 * g.idr, ht = 0.5 * ir * g.idt, hp = 0.5 * ir * is * g.idp;
  double dpr = gC(g, s, F_P, i + 1, j, k) - gC(g, s, F_P, i - 1, j, k);
  // perturbation form: the reference column's gradient joins the r difference
  if constexpr (S::PERT) dpr += s.pref[min(i + 1, g.nr - 1)] - s.pref[max(i - 1, 0)];
  const double advp = c.ur * dpr * hr +
                      c.ut * (gC(g, s, F_P, i, j + 1, k) - gC(g, s, F_P, i, j - 1, k)) * ht +
                      c.uf * (gC(g, s, F_P, i, j, k + 1) - gC(g, s, F_P, i, j, k - 1)) * hp;
  const double Tim = gC(g, s, F_T, i - 1, j, k), Tip = gC(g, s, F_T, i + 1, j, k);
  const double Tjm = gC(g, s, F_T, i, j - 1, k), Tjp = gC(g, s, F_T, i, j + 1, k);
  const double Tkm = gC(g, s, F_T, i, j, k - 1), Tkp = gC(g, s, F_T, i, j, k + 1);
  const double advT = c.ur * (Tip - Tim) * hr + c.ut * (Tjp - Tjm) * ht + c.uf * (Tkp - Tkm) * hp;
  const double T0 = c.T, ir2 = ir * ir;
  const double lap =
      (g.rf[i + 1] * g.rf[i + 1] * (Tip - T0) - g.rf[i] * g.rf[i] * (T0 - Tim)) * (ir2 * g.idr * g.idr) +
      (g.sf[j + 1] * (Tjp - T0) - g.sf[j] * (T0 - Tjm)) * (ir2 * is * g.idt * g.idt) +
      (Tkp - 2.0 * T0 + Tkm) * (ir2 * is * is * g.idp * g.idp);
  const double phi = m.mu * (2.0 * (c.Grr * c.Grr + c.Gtt * c.Gtt + c.Gff * c.Gff) + c.Srt * c.Srt +
                             c.Srf * c.Srf + c.Stf * c.Stf - (2.0 / 3.0) * c.tr * c.div);
  *FT = advT + (m.gam - 1.0) * c.T * c.div - c.chi * phi - c.chi * m.kap * lap;
  return advp + m.gam * c.P * c.div - (m.gam - 1.0) * phi - (m.gam - 1.0) * m.kap * lap;
}

template <class S>
__device__ __forceinline__ double F_ur(const Geo &g, const Mat &m, const S &s, int f, int j, int k) {
  const double irF = g.irf[f], is = g.isc[j];
  const double irho = irho_mean(g, m, s, f - 1, j, k, f, j, k);
  const double nu = m.mu * irho;
  const double un = gR(g, s, f, j, k);
  const double ua = 0.25 * (gT(g, s, f - 1, j, k) + gT(g, s, f - 1, j + 1, k) + gT(g, s, f, j, k) +
                            gT(g, s, f, j + 1, k));
  const double ub = 0.25 * (gF(g, s, f - 1, j, k) + gF(g, s, f - 1, j, k + 1) + gF(g, s, f, j, k) +
                            gF(g, s, f, j, k + 1));
  const double xp = gR(g, s, f + 1, j, k), xm = gR(g, s, f - 1, j, k);
  const double yp = gR(g, s, f, j + 1, k), ym = gR(g, s, f, j - 1, k);
  const double zp = gR(g, s, f, j, k + 1), zm = gR(g, s, f, j, k - 1);
  double N = (gC(g, s, F_P, f, j, k) - gC(g, s, F_P, f - 1, j, k)) * (irho * g.idr);
  N += un * (xp - xm) * (0.5 * g.idr) + ua * (yp - ym) * (0.5 * irF * g.idt) +
       ub * (zp - zm) * (0.5 * irF * is * g.idp) - (ua * ua + ub * ub) * irF;
  const double gd = (divc(g, s, f, j, k) - divc(g, s, f - 1, j, k)) * g.idr;
  // vorticity: omega_phi at the edges (f, j) and (f, j + 1), omega_theta at
  // the edges (f, k) and (f, k + 1); C = (curl omega)_r
  const double T00 = gT(g, s, f - 1, j, k), T01 = gT(g, s, f - 1, j + 1, k);
  const double T10 = gT(g, s, f, j, k), T11 = gT(g, s, f, j + 1, k);
  const double F00 = gF(g, s, f - 1, j, k), F01 = gF(g, s, f - 1, j, k + 1);
  const double F10 = gF(g, s, f, j, k), F11 = gF(g, s, f, j, k + 1);
  const double wp0 = (T10 - T00) * g.idr + 0.5 * (T10 + T00) * irF - (un - ym) * (irF * g.idt);
  const double wp1 = (T11 - T01) * g.idr + 0.5 * (T11 + T01) * irF - (yp - un) * (irF * g.idt);
  const double wt0 = (un - zm) * (irF * is * g.idp) - (F10 - F00) * g.idr - 0.5 * (F10 + F00) * irF;
  const double wt1 = (zp - un) * (irF * is * g.idp) - (F11 - F01) * g.idr - 0.5 * (F11 + F01) * irF;
  const double C = ((g.sf[j + 1] * wp1 - g.sf[j] * wp0) * g.idt - (wt1 - wt0) * g.idp) * (irF * is);
  const double vis = gd - C;  // nu (vis + gd / 3) = nu ((4/3) gd - C)
  N += -2.0 * m.omega * g.sc[j] * ub;
  if constexpr (S::PERT) {
    // perturbation form: the gradient of p' above, and gravity less the
    // reference column's balanced gradient, g (rho_f - rhobar_f) / rho_f,
    // with rho - rhobar = (p' Tbar - (pbar + pi_inf)(T - Tbar)) / (R T Tbar)
    const double Ta = gC(g, s, F_T, f - 1, j, k), Tb = gC(g, s, F_T, f, j, k);
    const double ta = s.tref[f - 1], tb = s.tref[f];
    const double da = (gC(g, s, F_P, f - 1, j, k) * ta - (s.pref[f - 1] + m.pinf) * (Ta - ta)) / (m.Rg * Ta * ta);
    const double db = (gC(g, s, F_P, f, j, k) * tb - (s.pref[f] + m.pinf) * (Tb - tb)) / (m.Rg * Tb * tb);
    return N - nu * vis - nu * (1.0 / 3.0) * gd + m.g_r * (0.5 * (da + db)) * irho;
  } else {
    return N - nu * vis - nu * (1.0 / 3.0) * gd + m.g_r;
  }
}

template <class S>
__device__ __forceinline__ double F_ut(const Geo &g, const Mat &m, const S &s, int i, int f, int k) {
  const double ir = g.irc[i], isF = g.isf[f], ctF = g.ctf[f];
  const int j0 = f - 1, j1 = f;
  const double irho = irho_mean(g, m, s, i, j0, k, i, j1, k);
  const double nu = m.mu * irho;
  const double un = gT(g, s, i, f, k);
  const double ua = 0.25 * (gR(g, s, i, j0, k) + gR(g, s, i, j1, k) + gR(g, s, i + 1, j0, k) +
                            gR(g, s, i + 1, j1, k));
  const double ub = 0.25 * (gF(g, s, i, j0, k) + gF(g, s, i, j0, k + 1) + gF(g, s, i, j1, k) +
                            gF(g, s, i, j1, k + 1));
  const double xp = gT(g, s, i + 1, f, k), xm = gT(g, s, i - 1, f, k);
  const double yp = gT(g, s, i, f + 1, k), ym = gT(g, s, i, f - 1, k);
  const double zp = gT(g, s, i, f, k + 1), zm = gT(g, s, i, f, k - 1);
  double N = (gC(g, s, F_P, i, j1, k) - gC(g, s, F_P, i, j0, k)) * (irho * ir * g.idt);
  N += ua * (xp - xm) * (0.5 * g.idr) + un * (yp - ym) * (0.5 * ir * g.idt) +
       ub * (zp - zm) * (0.5 * ir * isF * g.idp) + (un * ua - ub * ub * ctF) * ir;
  const double gd = (divc(g, s, i, j1, k) - divc(g, s, i, j0, k)) * (ir * g.idt);
  // vorticity: omega_r at the edges (f, k) and (f, k + 1), omega_phi at the
  // edges (i, f) and (i + 1, f); C = (curl omega)_theta
  const double R00 = gR(g, s, i, j0, k), R01 = gR(g, s, i, j1, k);
  const double R10 = gR(g, s, i + 1, j0, k), R11 = gR(g, s, i + 1, j1, k);
  const double F00 = gF(g, s, i, j0, k), F01 = gF(g, s, i, j0, k + 1);
  const double F10 = gF(g, s, i, j1, k), F11 = gF(g, s, i, j1, k + 1);
  const double wr0 = ((g.sc[j1] * F10 - g.sc[j0] * F00) * g.idt - (un - zm) * g.idp) * (ir * isF);
  const double wr1 = ((g.sc[j1] * F11 - g.sc[j0] * F01) * g.idt - (zp - un) * g.idp) * (ir * isF);
  const double ira = g.irf[i], irb = g.irf[i + 1];
  const double wp0 = (un - xm) * g.idr + 0.5 * (un + xm) * ira - (R01 - R00) * (ira * g.idt);
  const double wp1 = (xp - un) * g.idr + 0.5 * (xp + un) * irb - (R11 - R10) * (irb * g.idt);
  const double C = (wr1 - wr0) * (ir * isF * g.idp) - (g.rf[i + 1] * wp1 - g.rf[i] * wp0) * (ir * g.idr);
  const double vis = gd - C;
  N += -2.0 * m.omega * g.cf[f] * ub;
  return N - nu * vis - nu * (1.0 / 3.0) * gd;
}

template <class S>
__device__ __forceinline__ double F_uf(const Geo &g, const Mat &m, const S &s, int i, int j, int f) {
  const double ir = g.irc[i], is = g.isc[j], ct = g.ctc[j], ir2 = ir * ir;
  const int k0 = g.periodic ? wrapk(g, f - 1) : f - 1, k1 = g.periodic ? wrapk(g, f) : f;
  const double irho = irho_mean(g, m, s, i, j, k0, i, j, k1);
  const double nu = m.mu * irho;
  const double un = gF(g, s, i, j, f);
  const double ua = 0.25 * (gR(g, s, i, j, k0) + gR(g, s, i, j, k1) + gR(g, s, i + 1, j, k0) +
                            gR(g, s, i + 1, j, k1));
  const double ub = 0.25 * (gT(g, s, i, j, k0) + gT(g, s, i, j, k1) + gT(g, s, i, j + 1, k0) +
                            gT(g, s, i, j + 1, k1));
  const double xp = gF(g, s, i + 1, j, f), xm = gF(g, s, i - 1, j, f);
  const double yp = gF(g, s, i, j + 1, f), ym = gF(g, s, i, j - 1, f);
  const double zp = gF(g, s, i, j, f + 1), zm = gF(g, s, i, j, f - 1);
  double N = (gC(g, s, F_P, i, j, k1) - gC(g, s, F_P, i, j, k0)) * (irho * ir * is * g.idp);
  N += ua * (xp - xm) * (0.5 * g.idr) + ub * (yp - ym) * (0.5 * ir * g.idt) +
       un * (zp - zm) * (0.5 * ir * is * g.idp) + un * (ua + ub * ct) * ir;
  const double gd = (divc(g, s, i, j, k1) - divc(g, s, i, j, k0)) * (ir * is * g.idp);
  const double R00 = gR(g, s, i, j, k0), R01 = gR(g, s, i, j, k1);
  const double R10 = gR(g, s, i + 1, j, k0), R11 = gR(g, s, i + 1, j, k1);
  const double T00 = gT(g, s, i, j, k0), T01 = gT(g, s, i, j, k1);
  const double T10 = gT(g, s, i, j + 1, k0), T11 = gT(g, s, i, j + 1, k1);
  double vis;
  if (!S::INTERIOR && ((j == 0 && g.pole_lo) || (j == g.nt - 1 && g.pole_hi))) {
    // next to a pole: component form, scalar Laplacians and curvature terms
    vis = (g.rf[i + 1] * g.rf[i + 1] * (xp - un) - g.rf[i] * g.rf[i] * (un - xm)) * (ir2 * g.idr * g.idr) +
          (g.sf[j + 1] * (yp - un) - g.sf[j] * (un - ym)) * (ir2 * is * g.idt * g.idt) +
          (zp - 2.0 * un + zm) * (ir2 * is * is * g.idp * g.idp);
    const double dphr = 0.5 * ((R01 - R00) + (R11 - R10)) * g.idp;
    const double dpht = 0.5 * ((T01 - T00) + (T11 - T10)) * g.idp;
    vis += -un * ir2 * is * is + 2.0 * ir2 * is * dphr + 2.0 * ct * ir2 * is * dpht;
  } else {
    // vorticity: omega_theta at the edges (i, f) and (i + 1, f), omega_r at
    // the edges (j, f) and (j + 1, f); C = (curl omega)_phi
    const double ira = g.irf[i], irb = g.irf[i + 1];
    const double wt0 = (R01 - R00) * (ira * is * g.idp) - (un - xm) * g.idr - 0.5 * (un + xm) * ira;
    const double wt1 = (R11 - R10) * (irb * is * g.idp) - (xp - un) * g.idr - 0.5 * (xp + un) * irb;
    const double wr0 = ((g.scx[j + 1] * un - g.scx[j] * ym) * g.idt - (T01 - T00) * g.idp) * (ir * g.isf[j]);
    const double wr1 = ((g.scx[j + 2] * yp - g.scx[j + 1] * un) * g.idt - (T11 - T10) * g.idp) * (ir * g.isf[j + 1]);
    const double C = (g.rf[i + 1] * wt1 - g.rf[i] * wt0) * (ir * g.idr) - (wr1 - wr0) * (ir * g.idt);
    vis = gd - C;
  }
  N += 2.0 * m.omega * (g.cc[j] * ub + g.sc[j] * ua);
  return N - nu * vis - nu * (1.0 / 3.0) * gd;
}

// F_h at an unknown, less the source term of a forced state (manufactured
// solutions: the residual takes -(F_h - S))
template <class S>
__device__ __forceinline__ double forced(const S &s, int fid, long x, double F) {
  if constexpr (S::WALL) return s.f[fid] ? F - s.f[fid][x] : F;
  else return F;
}

// residual at the centre (i,j,k) and the three faces with the same indices
template <class S, bool WRITE_UB>
__device__ __forceinline__ void residual_point(const Geo &g, const Mat &m, const S &s, const Diff &dU,
                                               double tau, const Fields &R, const Fields &Ub,
                                               int *status, int i, int j, int k) {
  if (k >= g.npf) return;
  const bool kc = k < g.np;
  double chk = 0.0; // the sum of this point's residuals: non-finite iff one of them is
  if (i < g.nr && j < g.nt && kc) { // cell centre
    const long x = idx_c(g, i, j, k);
    const double ubp = s.ld(F_P, x), ubT = s.ld(F_T, x);
    if (WRITE_UB) { Ub.p[x] = ubp; Ub.T[x] = ubT; }
    // finite and non-positive; a NaN or an infinity shows as a non-finite
    // residual below
    double pfull = ubp;
    if constexpr (S::PERT) pfull += s.pref[i];
    if (ubT <= 0.0 || pfull + m.pinf <= 0.0) status[ST_NONPHYS] = 1; // plain vector store
    double FT;
    const double Fp = F_p_T(g, m, s, i, j, k, &FT);
    const double rp = -dU.at(F_P, x) - tau * forced(s, F_P, x, Fp);
    const double rT = -dU.at(F_T, x) - tau * forced(s, F_T, x, FT);
    R.p[x] = rp;
    R.T[x] = rT;
    chk = rp + rT;
  }
  if (j < g.nt && kc) { // r face i
    const long x = idx_r(g, i, j, k);
    if (WRITE_UB) Ub.ur[x] = s.ld(F_UR, x);
    const double r = (i >= 1 && i < g.nr) ? -dU.at(F_UR, x) - tau * forced(s, F_UR, x, F_ur(g, m, s, i, j, k)) : 0.0;
    R.ur[x] = r;
    chk += r;
  }
  if (i < g.nr && kc) { // theta face j
    const long x = idx_t(g, i, j, k);
    if (WRITE_UB) Ub.ut[x] = s.ld(F_UT, x);
    const double r = (j >= 1 && j < g.nt) ? -dU.at(F_UT, x) - tau * forced(s, F_UT, x, F_ut(g, m, s, i, j, k)) : 0.0;
    R.ut[x] = r;
    chk += r;
  }
  if (i < g.nr && j < g.nt) { // phi face k
    const long x = idx_f(g, i, j, k);
    if (WRITE_UB) Ub.uf[x] = s.ld(F_UF, x);
    const bool interior = g.periodic || (k >= 1 && k < g.np);
    const double r = interior ? -dU.at(F_UF, x) - tau * forced(s, F_UF, x, F_uf(g, m, s, i, j, k)) : 0.0;
    R.uf[x] = r;
    chk += r;
  }
  if (!isfinite(chk)) status[ST_DIVERGED] = 1; // plain vector store
}

// public form: midpoint formed from Un and Uk and written out; 3-D grid
__global__ void __launch_bounds__(256) k_residual_mid(Geo g, Mat m, SrcMid s, Diff dU, double tau,
                                                      Fields R, Fields Ub, int *status) {
  residual_point<SrcMid, true>(g, m, s, dU, tau, R, Ub, status, blockIdx.z, blockIdx.y,
                               blockIdx.x * blockDim.x + threadIdx.x);
}

// split-step form: the midpoint is resident; flat grid of workgroups over
// (phi block, theta index, r index).  B: a batch of grids, each workgroup
// reads its grid's arguments from the batch table; else one grid by value.
// The split-step residual runs as two launches.  The interior launch covers
// the workgroups whose points and all their stencil neighbours lie inside the
// arrays in r and theta (1 <= i <= nr-2, 1 <= j <= nt-2), every phi block;
// its accessors apply the phi ghost rules without branches and use 32-bit
// indices, which roughly halves its registers.  The general launch covers
// the whole index space and leaves those workgroups at once.
__host__ __device__ inline bool res_interior_ok(const Geo &g) {
  return (long)(g.nr + 1) * (g.nt + 1) * g.npf < 0x7fffffffL;
}
__host__ __device__ inline int res_nk(const Geo &g, int bs) { return (g.npf + bs - 1) / bs; }
__host__ __device__ inline unsigned res_interior_blocks(const Geo &g, int bs) {
  if (!res_interior_ok(g) || g.nr < 3 || g.nt < 3) return 0;
  return (unsigned)res_nk(g, bs) * (unsigned)(g.nt - 2) * (unsigned)(g.nr - 2);
}

// The (i, j) pairs the general launch takes when the interior launch runs:
// the shell around the interior, i in {0, nr-1, nr} for every j, then j in
// {0, nt-1, nt} for 1 <= i <= nr-2; else every pair.  Workgroups per pair:
// the phi blocks.
__host__ __device__ inline unsigned res_shell_pairs(const Geo &g) {
  return 3u * (unsigned)(g.nt + 1) + 3u * (unsigned)(g.nr - 2);
}
__host__ __device__ inline unsigned res_general_blocks(const Geo &g, int bs) {
  const unsigned pairs = res_interior_blocks(g, bs) ? res_shell_pairs(g) : (unsigned)(g.nt + 1) * (unsigned)(g.nr + 1);
  return (unsigned)res_nk(g, bs) * pairs;
}

// W: a forced pass (wall velocities and source term); PT: the
// perturbation-pressure form
template <bool W = false, bool PT = false>
__device__ __forceinline__ void residual_body(const PassArgs &a, unsigned w) {
  const Geo &g = a.g;
  const int bs = (int)blockDim.x;
  const unsigned nkb = (unsigned)res_nk(g, bs);
  const unsigned kb = w % nkb, rest = w / nkb;
  int i, j;
  if (res_interior_blocks(g, bs) > 0) {  // the shell (the interior launch does the rest)
    const unsigned na = 3u * (unsigned)(g.nt + 1);
    if (rest < na) {
      const unsigned ia = rest / (unsigned)(g.nt + 1);
      j = (int)(rest % (unsigned)(g.nt + 1));
      i = ia == 0 ? 0 : (ia == 1 ? g.nr - 1 : g.nr);
    } else {
      const unsigned r2 = rest - na;
      if (r2 >= 3u * (unsigned)(g.nr - 2)) return;
      const unsigned jb = r2 % 3u;
      i = 1 + (int)(r2 / 3u);
      j = jb == 0 ? 0 : (jb == 1 ? g.nt - 1 : g.nt);
    }
  } else {
    j = (int)(rest % (g.nt + 1));
    i = (int)(rest / (g.nt + 1));
  }
  decltype(auto) s = SrcSel<W, PT>::get(a);
  residual_point<std::decay_t<decltype(s)>, false>(g, a.m, s, a.d, a.tau, a.R, Fields{}, a.status, i, j,
                                                   (int)(kb * blockDim.x + threadIdx.x));
}

// residual_point for the interior launch (1 <= i <= nr-2, 1 <= j <= nt-2,
// so that every r and theta row exists): every row is evaluated before any
// is stored, and none under a branch except the phi face of a bounded line,
// so that the loads of all four rows can be in flight together (a store of R
// between two rows would hold the next row's loads back until the previous
// row's arithmetic is done, since R may alias the state).  On a bounded phi
// line the lane k = np has no centre: its centre rows are evaluated at
// np - 1 and not stored.  Measured on the 512 x 256 x 128 sphere: 1.40 ->
// 1.00 ms per residual, at 2 waves per SIMD (227 VGPRs) against 4 for the
// row-by-row form; results bitwise unchanged.  Capping the registers for 3
// or 4 waves spills and is slower.
template <class S>
__device__ __forceinline__ void residual_point_in(const Geo &g, const Mat &m, const S &s, const Diff &dU,
                                                  double tau, const Fields &R, int *status, int i, int j,
                                                  int k) {
  if (k >= g.npf) return;
  const bool kc = S::PERIODIC || k < g.np;
  const int kk = S::PERIODIC ? k : min(k, g.np - 1);
  const long xc = idx_c(g, i, j, kk), xr = idx_r(g, i, j, kk), xt = idx_t(g, i, j, kk);
  const double ubp = s.ld(F_P, xc), ubT = s.ld(F_T, xc);
  double pfull = ubp;
  if constexpr (S::PERT) pfull += s.pref[i];
  const bool nonphys = ubT <= 0.0 || pfull + m.pinf <= 0.0;
  double FT;
  const double Fp = F_p_T(g, m, s, i, j, kk, &FT);
  const double rp = -dU.at(F_P, xc) - tau * forced(s, F_P, xc, Fp);
  const double rT = -dU.at(F_T, xc) - tau * forced(s, F_T, xc, FT);
  const double rr = -dU.at(F_UR, xr) - tau * forced(s, F_UR, xr, F_ur(g, m, s, i, j, kk));
  const double rt = -dU.at(F_UT, xt) - tau * forced(s, F_UT, xt, F_ut(g, m, s, i, j, kk));
  const long xf = idx_f(g, i, j, k);
  double rf = 0.0;
  if (S::PERIODIC || (k >= 1 && k < g.np))
    rf = -dU.at(F_UF, xf) - tau * forced(s, F_UF, xf, F_uf(g, m, s, i, j, k));
  if (kc) {
    R.p[xc] = rp;
    R.T[xc] = rT;
    R.ur[xr] = rr;
    R.ut[xt] = rt;
  }
  R.uf[xf] = rf;
  double chk = rf;  // the sum of this point's residuals: non-finite iff one of them is
  if (kc) chk += rp + rT + rr + rt;
  if (kc && nonphys) status[ST_NONPHYS] = 1;  // plain vector store
  if (!isfinite(chk)) status[ST_DIVERGED] = 1;  // plain vector store
}

template <class SI>
__device__ __forceinline__ void residual_at_in(const PassArgs &a, unsigned kb, int j, int i) {
  const Geo &g = a.g;
  SI s;
#pragma unroll
  for (int q = 0; q < 5; q++) s.a[q] = a.u.a[q];
  if constexpr (SI::WALL) {
    s.w = a.wall;
    s.f[F_P] = a.fsrc.p; s.f[F_UR] = a.fsrc.ur; s.f[F_UT] = a.fsrc.ut; s.f[F_UF] = a.fsrc.uf;
    s.f[F_T] = a.fsrc.T;
  }
  if constexpr (SI::PERT) {
    s.pref = a.pref;
    s.tref = a.tref;
  }
  residual_point_in<SI>(g, a.m, s, a.d, a.tau, a.R, a.status, i, j, (int)(kb * blockDim.x + threadIdx.x));
}

// workgroup w of a one-dimensional launch: phi block fastest, then j, then i
template <class SI>
__device__ __forceinline__ void residual_body_in(const PassArgs &a, unsigned w) {
  const Geo &g = a.g;
  const int bs = (int)blockDim.x;
  const unsigned nkin = (unsigned)res_nk(g, bs);
  const unsigned kb = w % nkin, rest = w / nkin;
  const int j = 1 + (int)(rest % (unsigned)(g.nt - 2)), i = 1 + (int)(rest / (unsigned)(g.nt - 2));
  residual_at_in<SI>(a, kb, j, i);
}

template <bool B>
__global__ void __launch_bounds__(256) DSW_OCC(DSW_WAVES_RES) k_residual(PassArgs a, Batch bt) {
  if constexpr (B) {
    const int mb = batch_member(bt, blockIdx.x);
    residual_body(batch_args(bt, mb), blockIdx.x - bt.woff[mb]);
  } else {
    residual_body(a, blockIdx.x);
  }
}

// forced split step, one grid: the interior workgroups (P: periodic), then
// the rest
template <bool P>
__global__ void __launch_bounds__(256) k_residual_in_forced(PassArgs a) {
  residual_body_in<SrcInW<P>>(a, blockIdx.x);
}
__global__ void __launch_bounds__(256) k_residual_forced(PassArgs a) { residual_body<true>(a, blockIdx.x); }

void launch_residual_forced(const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st) {
  const unsigned nin = res_interior_blocks(a.g, (int)threads);
  if (nin) {
    if (a.g.periodic) hipLaunchKernelGGL(k_residual_in_forced<true>, dim3(nin), dim3(threads), 0, st, a);
    else hipLaunchKernelGGL(k_residual_in_forced<false>, dim3(nin), dim3(threads), 0, st, a);
  }
  hipLaunchKernelGGL(k_residual_forced, dim3(blocks), dim3(threads), 0, st, a);
}

// perturbation-pressure form, one grid: the interior workgroups (P:
// periodic), then the rest
template <bool P>
__global__ void __launch_bounds__(256) k_residual_in_pert(PassArgs a) {
  residual_body_in<SrcPert<SrcOneT<true, P>>>(a, blockIdx.x);
}
__global__ void __launch_bounds__(256) k_residual_pert(PassArgs a) { residual_body<false, true>(a, blockIdx.x); }

void launch_residual_pert(const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st) {
  const unsigned nin = res_interior_blocks(a.g, (int)threads);
  if (nin) {
    if (a.g.periodic) hipLaunchKernelGGL(k_residual_in_pert<true>, dim3(nin), dim3(threads), 0, st, a);
    else hipLaunchKernelGGL(k_residual_in_pert<false>, dim3(nin), dim3(threads), 0, st, a);
  }
  hipLaunchKernelGGL(k_residual_pert, dim3(blocks), dim3(threads), 0, st, a);
}

// P: the grids of the launch are periodic in phi (full sphere)
template <bool B, bool P>
__global__ void __launch_bounds__(256) k_residual_in(PassArgs a, Batch bt) {
  using SI = SrcOneT<true, P>;
  if constexpr (B) {
    const int mb = batch_member(bt, blockIdx.x);
    const PassArgs am = batch_args(bt, mb);  // loaded once, before any store
    residual_body_in<SI>(am, blockIdx.x - bt.woff[mb]);
  } else {
    // one grid: a three-dimensional launch (phi block, j - 1, i - 1), so the
    // workgroup's indices need no integer division (on this GPU a division
    // of even uniform integers runs on the vector unit)
    residual_at_in<SI>(a, blockIdx.x, 1 + (int)blockIdx.y, 1 + (int)blockIdx.z);
  }
}

unsigned residual_interior_blocks(const Geo &g, int bs) { return res_interior_blocks(g, bs); }
unsigned residual_general_blocks(const Geo &g, int bs) { return res_general_blocks(g, bs); }

static void set5(const double **dst, const Fields &f) {
  dst[F_P] = f.p; dst[F_UR] = f.ur; dst[F_UT] = f.ut; dst[F_UF] = f.uf; dst[F_T] = f.T;
}

void launch_residual(const Geo &g, const Mat &m, const Fields &Un, const Fields &Uk, double tau,
                     const Fields &R, const Fields &Ub, int *status, hipStream_t st) {
  SrcMid s;
  set5(s.n, Un);
  set5(s.k, Uk);
  Diff d;
  set5(d.n, Un);
  set5(d.k, Uk);
  d.same = 0;
  dim3 block(64, 1, 1);
  dim3 grid((g.npf + 63) / 64, g.nt + 1, g.nr + 1);
  hipLaunchKernelGGL(k_residual_mid, grid, block, 0, st, g, m, s, d, tau, R, Ub, status);
}

void launch_residual_pass(const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                          hipStream_t st) {
  if (b.tab) hipLaunchKernelGGL(k_residual<true>, dim3(blocks), dim3(threads), 0, st, a, b);
  else hipLaunchKernelGGL(k_residual<false>, dim3(blocks), dim3(threads), 0, st, a, b);
}

void launch_residual_in_pass(bool periodic, const PassArgs &a, const Batch &b, unsigned blocks,
                             unsigned threads, hipStream_t st) {
  const dim3 bl(threads);
  // a batch numbers its members' workgroups in one dimension; one grid takes
  // the same workgroups, in the same order, as (phi block, j - 1, i - 1)
  const dim3 gr = b.tab ? dim3(blocks)
                        : dim3((unsigned)res_nk(a.g, (int)threads), (unsigned)(a.g.nt - 2), (unsigned)(a.g.nr - 2));
  if (periodic) {
    if (b.tab) hipLaunchKernelGGL((k_residual_in<true, true>), gr, bl, 0, st, a, b);
    else hipLaunchKernelGGL((k_residual_in<false, true>), gr, bl, 0, st, a, b);
  } else {
    if (b.tab) hipLaunchKernelGGL((k_residual_in<true, false>), gr, bl, 0, st, a, b);
    else hipLaunchKernelGGL((k_residual_in<false, false>), gr, bl, 0, st, a, b);
  }
}

// Courant numbers of a state for the step tau (for a time-step controller):
// at every centre, with the centre-averaged velocity and the spacings
// h_r = dr, h_t = r dtheta, h_f = r sin(theta) dphi, the advective number
// tau (|u_r| / h_r + |u_theta| / h_t + |u_phi| / h_f) and the acoustic one
// tau c max(1/h_r, 1/h_t, 1/h_f), c = sqrt(gamma R T); their maxima over the
// grid.  Non-negative doubles order as their bit patterns, so the maxima are
// unsigned 64-bit atomic maxima (vector atomics) into out[0], out[1].
__global__ void __launch_bounds__(256) k_courant(Geo g, Mat m, Fields U, double tau, unsigned long long *out) {
  const long n = (long)g.nr * g.nt * g.np;
  double ca = 0.0, cs = 0.0;
  for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (long)gridDim.x * blockDim.x) {
    const int k = (int)(x % g.np), j = (int)((x / g.np) % g.nt), i = (int)(x / ((long)g.np * g.nt));
    const double hr = g.dr, ht = g.rc[i] * g.dt, hf = g.rc[i] * g.sc[j] * g.dp;
    const double ur = 0.5 * (U.ur[idx_r(g, i, j, k)] + U.ur[idx_r(g, i + 1, j, k)]);
    const double ut = 0.5 * (U.ut[idx_t(g, i, j, k)] + U.ut[idx_t(g, i, j + 1, k)]);
    const int k1 = g.periodic ? wrapk(g, k + 1) : k + 1;
    const double uf = 0.5 * (U.uf[idx_f(g, i, j, k)] + U.uf[idx_f(g, i, j, k1)]);
    const double a = tau * (fabs(ur) / hr + fabs(ut) / ht + fabs(uf) / hf);
    double ih = 1.0 / hr;
    if (1.0 / ht > ih) ih = 1.0 / ht;
    if (1.0 / hf > ih) ih = 1.0 / hf;
    const double c = tau * sqrt(m.gam * m.Rg * U.T[x]) * ih;
    if (a > ca) ca = a;
    if (c > cs) cs = c;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double a = __shfl_xor(ca, o), c = __shfl_xor(cs, o);
    if (a > ca) ca = a;
    if (c > cs) cs = c;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(ca));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(cs));
  }
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

void launch_courant(const Geo &g, const Mat &m, const Fields &U, double tau, unsigned long long *out,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, out, 2);
  const long n = (long)g.nr * g.nt * g.np;
  const unsigned blocks = (unsigned)std::min<long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_courant, dim3(blocks), dim3(256), 0, st, g, m, U, tau, out);
}

} // namespace dsw
