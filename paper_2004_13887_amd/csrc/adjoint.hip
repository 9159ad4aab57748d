// adjoint.hip -- reverse-mode (transposed Jacobian) kernels of the split step
// (paper eqs. (spl1)-(spl3) iterated K times; operators of Appendix B).
//
// For the midpoint state Ubar every forward output is a local function of
// Ubar: the residual rows -tau F_h(Ubar) and the entries of the line matrices
// I + tau/2 D_d(Ubar).  The kernels here apply the transposes of their
// Jacobians:
//   k_residual_vjp   acc += (d(-tau F_h)/dUbar)^T mu
//   k_line_vjp<D>    acc += (d(M_d(Ubar) X)/dUbar)^T mu,  M_d = I + tau/2 D_d
// Each thread recomputes its outputs' intermediates, runs the statements of
// the forward evaluation backwards, and adds every partial into the
// cotangent array at the place the forward value was loaded from, through
// the same ghost mapping as the load (sign included).  The adds are FP64
// atomics (several outputs read each input), so the summation order, and the
// last bits of the result, may differ from run to run.
#include "dsw_common.hpp"
#include "dsw_internal.hpp"
#include "rows.hpp"

namespace dsw {

#ifndef DSW_ADJ_JT
#define DSW_ADJ_JT 4   // theta rows per workgroup of the column-tiled reverse
#endif
#ifndef DSW_ADJ_SEG
#define DSW_ADJ_SEG 8  // r planes per workgroup of the column-tiled reverse
#endif

// Scatter targets.  add(g, fid, i, j, k, v) adds v to array fid at its own
// index triple (cells: centre (i, j, k); r faces: (face, j, k); theta faces:
// (i, face, k); phi faces: (i, j, face)), ghost-mapped except for the
// periodic phi wrap: on a periodic grid k may be -1 or np, and add wraps it.
// GAcc: FP64 atomics straight into the global arrays.
struct GAcc {
  Fields A;
  __device__ __forceinline__ void add(const Geo &g, int fid, int i, int j, int k, double v) const {
    if (g.periodic) k = wrapk(g, k);
    double *p;
    if (fid == F_P) p = A.p + idx_c(g, i, j, k);
    else if (fid == F_T) p = A.T + idx_c(g, i, j, k);
    else if (fid == F_UR) p = A.ur + idx_r(g, i, j, k);
    else if (fid == F_UT) p = A.ut + idx_t(g, i, j, k);
    else p = A.uf + idx_f(g, i, j, k);
    unsafeAtomicAdd(p, v);
  }
};

// ----------------------------------------------- reverse of the ghost loads --

template <class Acc>
__device__ __forceinline__ void sC(const Geo &g, const Acc &A, int fid, int i, int j, int k, double v) {
  i = clampi(i, 0, g.nr - 1);
  j = clampi(j, 0, g.nt - 1);
  if (!g.periodic) k = clampi(k, 0, g.np - 1);
  A.add(g, fid, i, j, k, v);
}
template <class Acc>
__device__ __forceinline__ void sR(const Geo &g, const Acc &A, int f, int j, int k, double v) {
  double sg = 1.0;
  if (!g.periodic && (k < 0 || k >= g.np)) { sg = -sg; k = k < 0 ? 0 : g.np - 1; }
  if (j < 0) { if (!g.pole_lo) sg = -sg; j = 0; }
  else if (j >= g.nt) { if (!g.pole_hi) sg = -sg; j = g.nt - 1; }
  A.add(g, F_UR, f, j, k, sg * v);
}
template <class Acc>
__device__ __forceinline__ void sT(const Geo &g, const Acc &A, int i, int f, int k, double v) {
  double sg = 1.0;
  if (!g.periodic && (k < 0 || k >= g.np)) { sg = -sg; k = k < 0 ? 0 : g.np - 1; }
  if (i < 0) { sg = -sg; i = 0; }
  else if (i >= g.nr) { sg = -sg; i = g.nr - 1; }
  A.add(g, F_UT, i, f, k, sg * v);
}
template <class Acc>
__device__ __forceinline__ void sF(const Geo &g, const Acc &A, int i, int j, int f, double v) {
  double sg = 1.0;
  if (j < 0) { sg = -sg; j = 0; }
  else if (j >= g.nt) { sg = -sg; j = g.nt - 1; }
  if (i < 0) { sg = -sg; i = 0; }
  else if (i >= g.nr) { sg = -sg; i = g.nr - 1; }
  A.add(g, F_UF, i, j, f, sg * v);
}

// centre averages (avgR / avgT / avgF of dsw_common.hpp), reversed
template <class Acc>
__device__ __forceinline__ void avgR_rev(const Geo &g, const Acc &A, int i, int j, int k, double a) {
  sR(g, A, i, j, k, 0.5 * a);
  sR(g, A, i + 1, j, k, 0.5 * a);
}
template <class Acc>
__device__ __forceinline__ void avgT_rev(const Geo &g, const Acc &A, int i, int j, int k, double a) {
  sT(g, A, i, j, k, 0.5 * a);
  sT(g, A, i, j + 1, k, 0.5 * a);
}
template <class Acc>
__device__ __forceinline__ void avgF_rev(const Geo &g, const Acc &A, int i, int j, int k, double a) {
  sF(g, A, i, j, k, 0.5 * a);
  sF(g, A, i, j, k + 1, 0.5 * a);
}

// rho = (p + pi_inf) / (R T) at a (ghost-mapped) centre, reversed
template <class S, class Acc>
__device__ __forceinline__ void rho_rev(const Geo &g, const Mat &m, const S &s, const Acc &A, int i,
                                        int j, int k, double rb) {
  const double P = gC(g, s, F_P, i, j, k) + m.pinf, T = gC(g, s, F_T, i, j, k);
  const double iRT = 1.0 / (m.Rg * T);
  sC(g, A, F_P, i, j, k, rb * iRT);
  sC(g, A, F_T, i, j, k, -rb * P * iRT / T);
}

// divc (compact divergence at a centre), reversed
template <class Acc>
__device__ __forceinline__ void divc_rev(const Geo &g, const Acc &A, int i, int j, int k, double a) {
  const double ir = g.irc[i], irs = ir * g.isc[j];
  const double cr = ir * ir * g.idr * a, ct = irs * g.idt * a, cp = irs * g.idp * a;
  sR(g, A, i + 1, j, k, g.rf[i + 1] * g.rf[i + 1] * cr);
  sR(g, A, i, j, k, -g.rf[i] * g.rf[i] * cr);
  sT(g, A, i, j + 1, k, g.sf[j + 1] * ct);
  sT(g, A, i, j, k, -g.sf[j] * ct);
  sF(g, A, i, j, k + 1, cp);
  sF(g, A, i, j, k, -cp);
}

// centre() reversed: cb holds the adjoints of the Cent fields, c the values
template <class S, class Acc>
__device__ __forceinline__ void centre_rev(const Geo &g, const Mat &m, const S &s, int i, int j, int k, const Cent &c,
                           const Cent &cb, const Acc &A) {
  const double ir = g.irc[i], is = g.isc[j], ct = g.ctc[j], irs = ir * is;
  const double Grr = cb.Grr + cb.tr, Gtt = cb.Gtt + cb.tr, Gff = cb.Gff + cb.tr;
  double ur = cb.ur, ut = cb.ut, uf = cb.uf;
  double r0 = 0.0, r1 = 0.0, t0 = 0.0, t1 = 0.0, f0 = 0.0, f1 = 0.0;
  {  // div
    const double dr_ = ir * ir * g.idr * cb.div, dt_ = irs * g.idt * cb.div, dp_ = irs * g.idp * cb.div;
    r1 += g.rf[i + 1] * g.rf[i + 1] * dr_;
    r0 -= g.rf[i] * g.rf[i] * dr_;
    t1 += g.sf[j + 1] * dt_;
    t0 -= g.sf[j] * dt_;
    f1 += dp_;
    f0 -= dp_;
  }
  {  // Stf
    const double a = 0.5 * ir * g.idt * cb.Stf, b = 0.5 * irs * g.idp * cb.Stf;
    avgF_rev(g, A, i, j + 1, k, a);
    avgF_rev(g, A, i, j - 1, k, -a);
    avgT_rev(g, A, i, j, k + 1, b);
    avgT_rev(g, A, i, j, k - 1, -b);
    uf -= ct * ir * cb.Stf;
  }
  {  // Srf
    const double a = 0.5 * g.idr * cb.Srf, b = 0.5 * irs * g.idp * cb.Srf;
    avgF_rev(g, A, i + 1, j, k, a);
    avgF_rev(g, A, i - 1, j, k, -a);
    avgR_rev(g, A, i, j, k + 1, b);
    avgR_rev(g, A, i, j, k - 1, -b);
    uf -= ir * cb.Srf;
  }
  {  // Srt
    const double a = 0.5 * g.idr * cb.Srt, b = 0.5 * ir * g.idt * cb.Srt;
    avgT_rev(g, A, i + 1, j, k, a);
    avgT_rev(g, A, i - 1, j, k, -a);
    avgR_rev(g, A, i, j + 1, k, b);
    avgR_rev(g, A, i, j - 1, k, -b);
    ut -= ir * cb.Srt;
  }
  f1 += irs * g.idp * Gff;  // Gff
  f0 -= irs * g.idp * Gff;
  ur += ir * Gff;
  ut += ct * ir * Gff;
  t1 += ir * g.idt * Gtt;  // Gtt
  t0 -= ir * g.idt * Gtt;
  ur += ir * Gtt;
  r1 += g.idr * Grr;  // Grr
  r0 -= g.idr * Grr;
  // chi = (gamma - 1) T / P
  sC(g, A, F_P, i, j, k, cb.P - c.chi / c.P * cb.chi);
  sC(g, A, F_T, i, j, k, cb.T + (m.gam - 1.0) / c.P * cb.chi);
  r0 += 0.5 * ur; r1 += 0.5 * ur;
  t0 += 0.5 * ut; t1 += 0.5 * ut;
  f0 += 0.5 * uf; f1 += 0.5 * uf;
  sR(g, A, i, j, k, r0);
  sR(g, A, i + 1, j, k, r1);
  sT(g, A, i, j, k, t0);
  sT(g, A, i, j + 1, k, t1);
  sF(g, A, i, j, k, f0);
  sF(g, A, i, j, k + 1, f1);
}

// ------------------------------------------------ residual rows, reversed --

// pressure and temperature rows at a centre (F_p_T of residual.hip);
// wp, wT: adjoints of F_p and F_T
template <class S, class Acc>
__device__ __forceinline__ void F_p_T_rev_cb(const Geo &g, const Mat &m, const S &s, int i, int j, int k, const Cent &c,
                             double wp, double wT, Cent &cb, const Acc &A) {
  const double ir = g.irc[i], is = g.isc[j], ir2 = ir * ir;
  const double hr = 0.5 * g.idr, ht = 0.5 * ir * g.idt, hp = 0.5 * ir * is * g.idp;
  const double pim = gC(g, s, F_P, i - 1, j, k), pip = gC(g, s, F_P, i + 1, j, k);
  const double pjm = gC(g, s, F_P, i, j - 1, k), pjp = gC(g, s, F_P, i, j + 1, k);
  const double pkm = gC(g, s, F_P, i, j, k - 1), pkp = gC(g, s, F_P, i, j, k + 1);
  const double Tim = gC(g, s, F_T, i - 1, j, k), Tip = gC(g, s, F_T, i + 1, j, k);
  const double Tjm = gC(g, s, F_T, i, j - 1, k), Tjp = gC(g, s, F_T, i, j + 1, k);
  const double Tkm = gC(g, s, F_T, i, j, k - 1), Tkp = gC(g, s, F_T, i, j, k + 1);
  const double T0 = c.T;
  const double Ar = ir2 * g.idr * g.idr, At = ir2 * is * g.idt * g.idt, Ap = ir2 * is * is * g.idp * g.idp;
  const double rp2 = g.rf[i + 1] * g.rf[i + 1], rm2 = g.rf[i] * g.rf[i];
  const double lap = (rp2 * (Tip - T0) - rm2 * (T0 - Tim)) * Ar +
                     (g.sf[j + 1] * (Tjp - T0) - g.sf[j] * (T0 - Tjm)) * At + (Tkp - 2.0 * T0 + Tkm) * Ap;
  const double phi = m.mu * (2.0 * (c.Grr * c.Grr + c.Gtt * c.Gtt + c.Gff * c.Gff) + c.Srt * c.Srt +
                             c.Srf * c.Srf + c.Stf * c.Stf - (2.0 / 3.0) * c.tr * c.div);
  const double g1 = m.gam - 1.0;
  cb.P += m.gam * c.div * wp;
  cb.div += m.gam * c.P * wp + g1 * c.T * wT;
  cb.T += g1 * c.div * wT;
  const double phib = -g1 * wp - c.chi * wT;
  cb.chi += -(phi + m.kap * lap) * wT;
  const double lapb = -g1 * m.kap * wp - c.chi * m.kap * wT;
  cb.Grr += 4.0 * m.mu * c.Grr * phib;
  cb.Gtt += 4.0 * m.mu * c.Gtt * phib;
  cb.Gff += 4.0 * m.mu * c.Gff * phib;
  cb.Srt += 2.0 * m.mu * c.Srt * phib;
  cb.Srf += 2.0 * m.mu * c.Srf * phib;
  cb.Stf += 2.0 * m.mu * c.Stf * phib;
  cb.tr += -(2.0 / 3.0) * m.mu * c.div * phib;
  cb.div += -(2.0 / 3.0) * m.mu * c.tr * phib;
  double Tipb = rp2 * Ar * lapb, Timb = rm2 * Ar * lapb;
  double Tjpb = g.sf[j + 1] * At * lapb, Tjmb = g.sf[j] * At * lapb;
  double Tkpb = Ap * lapb, Tkmb = Ap * lapb;
  cb.T += -((rp2 + rm2) * Ar + (g.sf[j + 1] + g.sf[j]) * At + 2.0 * Ap) * lapb;
  // advection of T (seed wT) and of p (seed wp)
  cb.ur += (Tip - Tim) * hr * wT + (pip - pim) * hr * wp;
  cb.ut += (Tjp - Tjm) * ht * wT + (pjp - pjm) * ht * wp;
  cb.uf += (Tkp - Tkm) * hp * wT + (pkp - pkm) * hp * wp;
  Tipb += c.ur * hr * wT; Timb -= c.ur * hr * wT;
  Tjpb += c.ut * ht * wT; Tjmb -= c.ut * ht * wT;
  Tkpb += c.uf * hp * wT; Tkmb -= c.uf * hp * wT;
  sC(g, A, F_T, i + 1, j, k, Tipb);
  sC(g, A, F_T, i - 1, j, k, Timb);
  sC(g, A, F_T, i, j + 1, k, Tjpb);
  sC(g, A, F_T, i, j - 1, k, Tjmb);
  sC(g, A, F_T, i, j, k + 1, Tkpb);
  sC(g, A, F_T, i, j, k - 1, Tkmb);
  sC(g, A, F_P, i + 1, j, k, c.ur * hr * wp);
  sC(g, A, F_P, i - 1, j, k, -c.ur * hr * wp);
  sC(g, A, F_P, i, j + 1, k, c.ut * ht * wp);
  sC(g, A, F_P, i, j - 1, k, -c.ut * ht * wp);
  sC(g, A, F_P, i, j, k + 1, c.uf * hp * wp);
  sC(g, A, F_P, i, j, k - 1, -c.uf * hp * wp);
}

template <class S, class Acc>
__device__ __forceinline__ void F_p_T_rev(const Geo &g, const Mat &m, const S &s, int i, int j, int k, double wp,
                          double wT, const Acc &A) {
  Cent c, cb{};
  centre(g, m, s, i, j, k, c);
  F_p_T_rev_cb(g, m, s, i, j, k, c, wp, wT, cb, A);
  centre_rev(g, m, s, i, j, k, c, cb, A);
}

// The three momentum rows reversed.  Contributions that land on the same
// load are summed before the one atomic add of that load.  Extra inputs
// (from the two scalar line rows through the same face, which read the same
// face density and the same transverse averages): rfx, the adjoint of the
// face density rho_f = (rho_a + rho_b)/2; uax, ubx, of the two transverse
// averages ua, ub.

// radial momentum row at interior r-face (f, j, k) (F_ur of residual.hip)
template <class S, class Acc>
__device__ __forceinline__ void F_ur_rev(const Geo &g, const Mat &m, const S &s, int f, int j, int k, double w,
                         const Acc &A, double rfx = 0.0, double uax = 0.0, double ubx = 0.0) {
  const double irF = g.irf[f], is = g.isc[j];
  const double Pa = gC(g, s, F_P, f, j, k) + m.pinf, Ta = gC(g, s, F_T, f, j, k);
  const double Pb_ = gC(g, s, F_P, f - 1, j, k) + m.pinf, Tb_ = gC(g, s, F_T, f - 1, j, k);
  const double rho_a = Pa / (m.Rg * Ta), rho_b = Pb_ / (m.Rg * Tb_);
  const double irho = 1.0 / (0.5 * (rho_b + rho_a));
  const double nu = m.mu * irho;
  const double un = gR(g, s, f, j, k);
  const double T00 = gT(g, s, f - 1, j, k), T01 = gT(g, s, f - 1, j + 1, k);
  const double T10 = gT(g, s, f, j, k), T11 = gT(g, s, f, j + 1, k);
  const double F00 = gF(g, s, f - 1, j, k), F01 = gF(g, s, f - 1, j, k + 1);
  const double F10 = gF(g, s, f, j, k), F11 = gF(g, s, f, j, k + 1);
  const double ua = 0.25 * (T00 + T01 + T10 + T11);
  const double ub = 0.25 * (F00 + F01 + F10 + F11);
  const double xp = gR(g, s, f + 1, j, k), xm = gR(g, s, f - 1, j, k);
  const double yp = gR(g, s, f, j + 1, k), ym = gR(g, s, f, j - 1, k);
  const double zp = gR(g, s, f, j, k + 1), zm = gR(g, s, f, j, k - 1);
  const double pa = Pa - m.pinf, pb = Pb_ - m.pinf;
  const double gd = (divc(g, s, f, j, k) - divc(g, s, f - 1, j, k)) * g.idr;
  const double wp0 = (T10 - T00) * g.idr + 0.5 * (T10 + T00) * irF - (un - ym) * (irF * g.idt);
  const double wp1 = (T11 - T01) * g.idr + 0.5 * (T11 + T01) * irF - (yp - un) * (irF * g.idt);
  const double wt0 = (un - zm) * (irF * is * g.idp) - (F10 - F00) * g.idr - 0.5 * (F10 + F00) * irF;
  const double wt1 = (zp - un) * (irF * is * g.idp) - (F11 - F01) * g.idr - 0.5 * (F11 + F01) * irF;
  const double C = ((g.sf[j + 1] * wp1 - g.sf[j] * wp0) * g.idt - (wt1 - wt0) * g.idp) * (irF * is);
  const double vis = gd - C;
  // reverse of F = N - nu vis - nu/3 gd + g_r, vis = gd - C
  const double Nb = w, visb = -nu * w, gdb = -nu / 3.0 * w + visb, nub = -(vis + gd / 3.0) * w;
  double uab = uax, ubb = ubx - 2.0 * m.omega * g.sc[j] * Nb, unb = 0.0;
  double aT00 = 0.0, aT01 = 0.0, aT10 = 0.0, aT11 = 0.0, aF00 = 0.0, aF01 = 0.0, aF10 = 0.0, aF11 = 0.0;
  double aRf = 0.0, aRfp = 0.0, aRfm = 0.0;
  {  // divergences at cells f (+) and f - 1 (-)
    const double a1 = g.idr * gdb, a0 = -g.idr * gdb;
    const double ir1 = g.irc[f], ir0 = g.irc[f - 1];
    const double c1r = ir1 * ir1 * g.idr * a1, c1t = ir1 * is * g.idt * a1, c1p = ir1 * is * g.idp * a1;
    const double c0r = ir0 * ir0 * g.idr * a0, c0t = ir0 * is * g.idt * a0, c0p = ir0 * is * g.idp * a0;
    aRfp += g.rf[f + 1] * g.rf[f + 1] * c1r;
    aRf += -g.rf[f] * g.rf[f] * c1r + g.rf[f] * g.rf[f] * c0r;
    aRfm += -g.rf[f - 1] * g.rf[f - 1] * c0r;
    aT11 += g.sf[j + 1] * c1t; aT10 -= g.sf[j] * c1t;
    aT01 += g.sf[j + 1] * c0t; aT00 -= g.sf[j] * c0t;
    aF11 += c1p; aF10 -= c1p;
    aF01 += c0p; aF00 -= c0p;
  }
  double xpb = 0.0, xmb = 0.0, ypb, ymb, zpb, zmb;
  {  // C = (curl omega)_r, reversed
    const double q = -visb * (irF * is);
    const double wp1b = g.sf[j + 1] * g.idt * q, wp0b = -g.sf[j] * g.idt * q;
    const double wt1b = -g.idp * q, wt0b = g.idp * q;
    const double c1 = g.idr + 0.5 * irF, c0 = -g.idr + 0.5 * irF;
    aT10 += c1 * wp0b; aT00 += c0 * wp0b;
    aT11 += c1 * wp1b; aT01 += c0 * wp1b;
    aF10 -= c1 * wt0b; aF00 -= c0 * wt0b;
    aF11 -= c1 * wt1b; aF01 -= c0 * wt1b;
    const double ht_ = irF * g.idt, hp_ = irF * is * g.idp;
    unb += ht_ * (wp1b - wp0b) + hp_ * (wt0b - wt1b);
    ymb = ht_ * wp0b; ypb = -ht_ * wp1b;
    zmb = -hp_ * wt0b; zpb = hp_ * wt1b;
  }
  const double hr = 0.5 * g.idr, ht = 0.5 * irF * g.idt, hp = 0.5 * irF * is * g.idp;
  double irhob = (pa - pb) * g.idr * Nb;
  double aPa = irho * g.idr * Nb, aPb = -irho * g.idr * Nb;
  unb += (xp - xm) * hr * Nb; xpb += un * hr * Nb; xmb -= un * hr * Nb;
  uab += (yp - ym) * ht * Nb; ypb += ua * ht * Nb; ymb -= ua * ht * Nb;
  ubb += (zp - zm) * hp * Nb; zpb += ub * hp * Nb; zmb -= ub * hp * Nb;
  uab += -2.0 * ua * irF * Nb;
  ubb += -2.0 * ub * irF * Nb;
  irhob += m.mu * nub;
  const double rhob = 0.5 * (rfx - irho * irho * irhob); // each of the two cells
  aPa += rhob / (m.Rg * Ta);
  aPb += rhob / (m.Rg * Tb_);
  const double aTa = -rhob * rho_a / Ta, aTb = -rhob * rho_b / Tb_;
  aT00 += 0.25 * uab; aT01 += 0.25 * uab; aT10 += 0.25 * uab; aT11 += 0.25 * uab;
  aF00 += 0.25 * ubb; aF01 += 0.25 * ubb; aF10 += 0.25 * ubb; aF11 += 0.25 * ubb;
  sR(g, A, f, j, k, unb + aRf);
  sR(g, A, f + 1, j, k, xpb + aRfp);
  sR(g, A, f - 1, j, k, xmb + aRfm);
  sR(g, A, f, j + 1, k, ypb);
  sR(g, A, f, j - 1, k, ymb);
  sR(g, A, f, j, k + 1, zpb);
  sR(g, A, f, j, k - 1, zmb);
  sT(g, A, f - 1, j, k, aT00);
  sT(g, A, f - 1, j + 1, k, aT01);
  sT(g, A, f, j, k, aT10);
  sT(g, A, f, j + 1, k, aT11);
  sF(g, A, f - 1, j, k, aF00);
  sF(g, A, f - 1, j, k + 1, aF01);
  sF(g, A, f, j, k, aF10);
  sF(g, A, f, j, k + 1, aF11);
  sC(g, A, F_P, f, j, k, aPa);
  sC(g, A, F_P, f - 1, j, k, aPb);
  sC(g, A, F_T, f, j, k, aTa);
  sC(g, A, F_T, f - 1, j, k, aTb);
}

// colatitudinal momentum row at interior theta-face (i, f, k) (F_ut)
template <class S, class Acc>
__device__ __forceinline__ void F_ut_rev(const Geo &g, const Mat &m, const S &s, int i, int f, int k, double w,
                         const Acc &A, double rfx = 0.0, double uax = 0.0, double ubx = 0.0) {
  const double ir = g.irc[i], isF = g.isf[f], ctF = g.ctf[f];
  const int j0 = f - 1, j1 = f;
  const double P1 = gC(g, s, F_P, i, j1, k) + m.pinf, T1 = gC(g, s, F_T, i, j1, k);
  const double P0 = gC(g, s, F_P, i, j0, k) + m.pinf, T0 = gC(g, s, F_T, i, j0, k);
  const double rho1 = P1 / (m.Rg * T1), rho0 = P0 / (m.Rg * T0);
  const double irho = 1.0 / (0.5 * (rho0 + rho1));
  const double nu = m.mu * irho;
  const double un = gT(g, s, i, f, k);
  const double R00 = gR(g, s, i, j0, k), R01 = gR(g, s, i, j1, k);
  const double R10 = gR(g, s, i + 1, j0, k), R11 = gR(g, s, i + 1, j1, k);
  const double F00 = gF(g, s, i, j0, k), F01 = gF(g, s, i, j0, k + 1);
  const double F10 = gF(g, s, i, j1, k), F11 = gF(g, s, i, j1, k + 1);
  const double ua = 0.25 * (R00 + R01 + R10 + R11);
  const double ub = 0.25 * (F00 + F01 + F10 + F11);
  const double xp = gT(g, s, i + 1, f, k), xm = gT(g, s, i - 1, f, k);
  const double yp = gT(g, s, i, f + 1, k), ym = gT(g, s, i, f - 1, k);
  const double zp = gT(g, s, i, f, k + 1), zm = gT(g, s, i, f, k - 1);
  const double p1 = P1 - m.pinf, p0 = P0 - m.pinf;
  const double gd = (divc(g, s, i, j1, k) - divc(g, s, i, j0, k)) * (ir * g.idt);
  const double wr0 = ((g.sc[j1] * F10 - g.sc[j0] * F00) * g.idt - (un - zm) * g.idp) * (ir * isF);
  const double wr1 = ((g.sc[j1] * F11 - g.sc[j0] * F01) * g.idt - (zp - un) * g.idp) * (ir * isF);
  const double ira = g.irf[i], irb = g.irf[i + 1];
  const double wp0 = (un - xm) * g.idr + 0.5 * (un + xm) * ira - (R01 - R00) * (ira * g.idt);
  const double wp1 = (xp - un) * g.idr + 0.5 * (xp + un) * irb - (R11 - R10) * (irb * g.idt);
  const double C = (wr1 - wr0) * (ir * isF * g.idp) - (g.rf[i + 1] * wp1 - g.rf[i] * wp0) * (ir * g.idr);
  const double vis = gd - C;
  const double Nb = w, visb = -nu * w, gdb = -nu / 3.0 * w + visb, nub = -(vis + gd / 3.0) * w;
  double uab = uax, ubb = ubx - 2.0 * m.omega * g.cf[f] * Nb, unb = 0.0;
  double aR00 = 0.0, aR01 = 0.0, aR10 = 0.0, aR11 = 0.0, aF00 = 0.0, aF01 = 0.0, aF10 = 0.0, aF11 = 0.0;
  double aTf = 0.0, aTfp = 0.0, aTfm = 0.0;
  {  // divergences at cells (i, j1) (+) and (i, j0) (-)
    const double a1 = ir * g.idt * gdb, a0 = -ir * g.idt * gdb;
    const double is1 = g.isc[j1], is0 = g.isc[j0];
    const double c1r = ir * ir * g.idr * a1, c1t = ir * is1 * g.idt * a1, c1p = ir * is1 * g.idp * a1;
    const double c0r = ir * ir * g.idr * a0, c0t = ir * is0 * g.idt * a0, c0p = ir * is0 * g.idp * a0;
    aR11 += g.rf[i + 1] * g.rf[i + 1] * c1r; aR01 -= g.rf[i] * g.rf[i] * c1r;
    aR10 += g.rf[i + 1] * g.rf[i + 1] * c0r; aR00 -= g.rf[i] * g.rf[i] * c0r;
    aTfp += g.sf[j1 + 1] * c1t;
    aTf += -g.sf[j1] * c1t + g.sf[j0 + 1] * c0t;
    aTfm += -g.sf[j0] * c0t;
    aF11 += c1p; aF10 -= c1p;
    aF01 += c0p; aF00 -= c0p;
  }
  double xpb, xmb, ypb = 0.0, ymb = 0.0, zpb, zmb;
  {  // C = (curl omega)_theta, reversed
    const double Cb = -visb;
    const double wr1b = ir * isF * g.idp * Cb, wr0b = -wr1b;
    const double wp1b = -g.rf[i + 1] * ir * g.idr * Cb, wp0b = g.rf[i] * ir * g.idr * Cb;
    const double e = ir * isF;
    aF10 += g.sc[j1] * g.idt * e * wr0b; aF00 -= g.sc[j0] * g.idt * e * wr0b;
    aF11 += g.sc[j1] * g.idt * e * wr1b; aF01 -= g.sc[j0] * g.idt * e * wr1b;
    unb += g.idp * e * (wr1b - wr0b);
    zmb = g.idp * e * wr0b; zpb = -g.idp * e * wr1b;
    unb += (g.idr + 0.5 * ira) * wp0b + (-g.idr + 0.5 * irb) * wp1b;
    xmb = (-g.idr + 0.5 * ira) * wp0b; xpb = (g.idr + 0.5 * irb) * wp1b;
    aR01 -= ira * g.idt * wp0b; aR00 += ira * g.idt * wp0b;
    aR11 -= irb * g.idt * wp1b; aR10 += irb * g.idt * wp1b;
  }
  const double hr = 0.5 * g.idr, ht = 0.5 * ir * g.idt, hp = 0.5 * ir * isF * g.idp;
  double irhob = (p1 - p0) * ir * g.idt * Nb;
  double aP1 = irho * ir * g.idt * Nb, aP0 = -irho * ir * g.idt * Nb;
  uab += (xp - xm) * hr * Nb; xpb += ua * hr * Nb; xmb -= ua * hr * Nb;
  unb += (yp - ym) * ht * Nb; ypb += un * ht * Nb; ymb -= un * ht * Nb;
  ubb += (zp - zm) * hp * Nb; zpb += ub * hp * Nb; zmb -= ub * hp * Nb;
  unb += ua * ir * Nb;
  uab += un * ir * Nb;
  ubb += -2.0 * ub * ctF * ir * Nb;
  irhob += m.mu * nub;
  const double rhob = 0.5 * (rfx - irho * irho * irhob);
  aP1 += rhob / (m.Rg * T1);
  aP0 += rhob / (m.Rg * T0);
  const double aT1 = -rhob * rho1 / T1, aT0 = -rhob * rho0 / T0;
  aR00 += 0.25 * uab; aR01 += 0.25 * uab; aR10 += 0.25 * uab; aR11 += 0.25 * uab;
  aF00 += 0.25 * ubb; aF01 += 0.25 * ubb; aF10 += 0.25 * ubb; aF11 += 0.25 * ubb;
  sT(g, A, i, f, k, unb + aTf);
  sT(g, A, i + 1, f, k, xpb);
  sT(g, A, i - 1, f, k, xmb);
  sT(g, A, i, f + 1, k, ypb + aTfp);
  sT(g, A, i, f - 1, k, ymb + aTfm);
  sT(g, A, i, f, k + 1, zpb);
  sT(g, A, i, f, k - 1, zmb);
  sR(g, A, i, j0, k, aR00);
  sR(g, A, i, j1, k, aR01);
  sR(g, A, i + 1, j0, k, aR10);
  sR(g, A, i + 1, j1, k, aR11);
  sF(g, A, i, j0, k, aF00);
  sF(g, A, i, j0, k + 1, aF01);
  sF(g, A, i, j1, k, aF10);
  sF(g, A, i, j1, k + 1, aF11);
  sC(g, A, F_P, i, j1, k, aP1);
  sC(g, A, F_P, i, j0, k, aP0);
  sC(g, A, F_T, i, j1, k, aT1);
  sC(g, A, F_T, i, j0, k, aT0);
}

// azimuthal momentum row at phi-face (i, j, f) (F_uf)
template <class S, class Acc>
__device__ __forceinline__ void F_uf_rev(const Geo &g, const Mat &m, const S &s, int i, int j, int f, double w,
                         const Acc &A, double rfx = 0.0, double uax = 0.0, double ubx = 0.0) {
  const double ir = g.irc[i], is = g.isc[j], ct = g.ctc[j], ir2 = ir * ir;
  const int k0 = g.periodic ? wrapk(g, f - 1) : f - 1, k1 = g.periodic ? wrapk(g, f) : f;
  const double P1 = gC(g, s, F_P, i, j, k1) + m.pinf, T1 = gC(g, s, F_T, i, j, k1);
  const double P0 = gC(g, s, F_P, i, j, k0) + m.pinf, T0 = gC(g, s, F_T, i, j, k0);
  const double rho1 = P1 / (m.Rg * T1), rho0 = P0 / (m.Rg * T0);
  const double irho = 1.0 / (0.5 * (rho0 + rho1));
  const double nu = m.mu * irho;
  const double un = gF(g, s, i, j, f);
  const double R00 = gR(g, s, i, j, k0), R01 = gR(g, s, i, j, k1);
  const double R10 = gR(g, s, i + 1, j, k0), R11 = gR(g, s, i + 1, j, k1);
  const double T00 = gT(g, s, i, j, k0), T01 = gT(g, s, i, j, k1);
  const double T10 = gT(g, s, i, j + 1, k0), T11 = gT(g, s, i, j + 1, k1);
  const double ua = 0.25 * (R00 + R01 + R10 + R11);
  const double ub = 0.25 * (T00 + T01 + T10 + T11);
  const double xp = gF(g, s, i + 1, j, f), xm = gF(g, s, i - 1, j, f);
  const double yp = gF(g, s, i, j + 1, f), ym = gF(g, s, i, j - 1, f);
  const double zp = gF(g, s, i, j, f + 1), zm = gF(g, s, i, j, f - 1);
  const double p1 = P1 - m.pinf, p0 = P0 - m.pinf;
  const double gd = (divc(g, s, i, j, k1) - divc(g, s, i, j, k0)) * (ir * is * g.idp);
  const bool pole_row = !S::INTERIOR && ((j == 0 && g.pole_lo) || (j == g.nt - 1 && g.pole_hi));
  double vis;
  double xpb = 0.0, xmb = 0.0, ypb = 0.0, ymb = 0.0, zpb = 0.0, zmb = 0.0, unb = 0.0;
  double aR00 = 0.0, aR01 = 0.0, aR10 = 0.0, aR11 = 0.0, aT00 = 0.0, aT01 = 0.0, aT10 = 0.0, aT11 = 0.0;
  const double visb = -nu * w;
  if (pole_row) {
    // next to a pole: component form (scalar Laplacians and curvature terms)
    const double Cr = ir2 * g.idr * g.idr, Ct = ir2 * is * g.idt * g.idt, Cp = ir2 * is * is * g.idp * g.idp;
    const double rp2 = g.rf[i + 1] * g.rf[i + 1], rm2 = g.rf[i] * g.rf[i];
    vis = (rp2 * (xp - un) - rm2 * (un - xm)) * Cr + (g.sf[j + 1] * (yp - un) - g.sf[j] * (un - ym)) * Ct +
          (zp - 2.0 * un + zm) * Cp;
    const double dphr = 0.5 * ((R01 - R00) + (R11 - R10)) * g.idp;
    const double dpht = 0.5 * ((T01 - T00) + (T11 - T10)) * g.idp;
    vis += -un * ir2 * is * is + 2.0 * ir2 * is * dphr + 2.0 * ct * ir2 * is * dpht;
    unb += -ir2 * is * is * visb;
    const double dphrb = 2.0 * ir2 * is * visb, dphtb = 2.0 * ct * ir2 * is * visb;
    aR01 += 0.5 * g.idp * dphrb; aR00 -= 0.5 * g.idp * dphrb;
    aR11 += 0.5 * g.idp * dphrb; aR10 -= 0.5 * g.idp * dphrb;
    aT01 += 0.5 * g.idp * dphtb; aT00 -= 0.5 * g.idp * dphtb;
    aT11 += 0.5 * g.idp * dphtb; aT10 -= 0.5 * g.idp * dphtb;
    xpb = rp2 * Cr * visb; xmb = rm2 * Cr * visb;
    ypb = g.sf[j + 1] * Ct * visb; ymb = g.sf[j] * Ct * visb;
    zpb = Cp * visb; zmb = Cp * visb;
    unb -= ((rp2 + rm2) * Cr + (g.sf[j + 1] + g.sf[j]) * Ct + 2.0 * Cp) * visb;
  } else {
    const double ira = g.irf[i], irb = g.irf[i + 1];
    const double wt0 = (R01 - R00) * (ira * is * g.idp) - (un - xm) * g.idr - 0.5 * (un + xm) * ira;
    const double wt1 = (R11 - R10) * (irb * is * g.idp) - (xp - un) * g.idr - 0.5 * (xp + un) * irb;
    const double wr0 = ((g.scx[j + 1] * un - g.scx[j] * ym) * g.idt - (T01 - T00) * g.idp) * (ir * g.isf[j]);
    const double wr1 = ((g.scx[j + 2] * yp - g.scx[j + 1] * un) * g.idt - (T11 - T10) * g.idp) * (ir * g.isf[j + 1]);
    const double C = (g.rf[i + 1] * wt1 - g.rf[i] * wt0) * (ir * g.idr) - (wr1 - wr0) * (ir * g.idt);
    vis = gd - C;
    // C = (curl omega)_phi, reversed
    const double Cb = -visb;
    const double wt1b = g.rf[i + 1] * ir * g.idr * Cb, wt0b = -g.rf[i] * ir * g.idr * Cb;
    const double wr1b = -ir * g.idt * Cb, wr0b = -wr1b;
    aR01 += ira * is * g.idp * wt0b; aR00 -= ira * is * g.idp * wt0b;
    aR11 += irb * is * g.idp * wt1b; aR10 -= irb * is * g.idp * wt1b;
    unb += (-g.idr - 0.5 * ira) * wt0b + (g.idr - 0.5 * irb) * wt1b;
    xmb = (g.idr - 0.5 * ira) * wt0b; xpb = (-g.idr - 0.5 * irb) * wt1b;
    const double e0 = ir * g.isf[j] * wr0b, e1 = ir * g.isf[j + 1] * wr1b;
    unb += g.scx[j + 1] * g.idt * (e0 - e1);
    ymb = -g.scx[j] * g.idt * e0; ypb = g.scx[j + 2] * g.idt * e1;
    aT01 -= g.idp * e0; aT00 += g.idp * e0;
    aT11 -= g.idp * e1; aT10 += g.idp * e1;
  }
  // reverse of F = N - nu vis - nu/3 gd, vis = gd - C off the poles
  const double Nb = w, gdb = -nu / 3.0 * w + (pole_row ? 0.0 : visb), nub = -(vis + gd / 3.0) * w;
  double ubb = ubx + 2.0 * m.omega * g.cc[j] * Nb, uab = uax + 2.0 * m.omega * g.sc[j] * Nb;
  double aFf = 0.0, aFfp = 0.0, aFfm = 0.0;
  {  // divergences at cells (i, j, k1) (+) and (i, j, k0) (-); their phi
     // faces k1 + 1 = f + 1, k1 = f, k0 + 1 = f, k0 = f - 1 (wrapped alike)
    const double a1 = ir * is * g.idp * gdb, a0 = -ir * is * g.idp * gdb;
    const double cr = ir * ir * g.idr, irs = ir * is;
    aR11 += g.rf[i + 1] * g.rf[i + 1] * cr * a1; aR01 -= g.rf[i] * g.rf[i] * cr * a1;
    aR10 += g.rf[i + 1] * g.rf[i + 1] * cr * a0; aR00 -= g.rf[i] * g.rf[i] * cr * a0;
    aT11 += g.sf[j + 1] * irs * g.idt * a1; aT01 -= g.sf[j] * irs * g.idt * a1;
    aT10 += g.sf[j + 1] * irs * g.idt * a0; aT00 -= g.sf[j] * irs * g.idt * a0;
    aFfp += irs * g.idp * a1;
    aFf += -irs * g.idp * a1 + irs * g.idp * a0;
    aFfm += -irs * g.idp * a0;
  }
  const double hr = 0.5 * g.idr, ht = 0.5 * ir * g.idt, hp = 0.5 * ir * is * g.idp;
  double irhob = (p1 - p0) * ir * is * g.idp * Nb;
  double aP1 = irho * ir * is * g.idp * Nb, aP0 = -irho * ir * is * g.idp * Nb;
  uab += (xp - xm) * hr * Nb; xpb += ua * hr * Nb; xmb -= ua * hr * Nb;
  ubb += (yp - ym) * ht * Nb; ypb += ub * ht * Nb; ymb -= ub * ht * Nb;
  unb += (zp - zm) * hp * Nb; zpb += un * hp * Nb; zmb -= un * hp * Nb;
  unb += (ua + ub * ct) * ir * Nb;
  uab += un * ir * Nb;
  ubb += un * ct * ir * Nb;
  irhob += m.mu * nub;
  const double rhob = 0.5 * (rfx - irho * irho * irhob);
  aP1 += rhob / (m.Rg * T1);
  aP0 += rhob / (m.Rg * T0);
  const double aT1 = -rhob * rho1 / T1, aT0 = -rhob * rho0 / T0;
  aR00 += 0.25 * uab; aR01 += 0.25 * uab; aR10 += 0.25 * uab; aR11 += 0.25 * uab;
  aT00 += 0.25 * ubb; aT01 += 0.25 * ubb; aT10 += 0.25 * ubb; aT11 += 0.25 * ubb;
  sF(g, A, i, j, f, unb + aFf);
  sF(g, A, i + 1, j, f, xpb);
  sF(g, A, i - 1, j, f, xmb);
  sF(g, A, i, j + 1, f, ypb);
  sF(g, A, i, j - 1, f, ymb);
  sF(g, A, i, j, f + 1, zpb + aFfp);
  sF(g, A, i, j, f - 1, zmb + aFfm);
  // scatter with the unwrapped cell indices f - 1, f
  sR(g, A, i, j, f - 1, aR00);
  sR(g, A, i, j, f, aR01);
  sR(g, A, i + 1, j, f - 1, aR10);
  sR(g, A, i + 1, j, f, aR11);
  sT(g, A, i, j, f - 1, aT00);
  sT(g, A, i, j, f, aT01);
  sT(g, A, i, j + 1, f - 1, aT10);
  sT(g, A, i, j + 1, f, aT11);
  sC(g, A, F_P, i, j, f, aP1);
  sC(g, A, F_P, i, j, f - 1, aP0);
  sC(g, A, F_T, i, j, f, aT1);
  sC(g, A, F_T, i, j, f - 1, aT0);
}

// acc += (d(-tau F_h(Ubar))/dUbar)^T mu over every unknown row (the rows of the
// boundary-normal faces are constant); index space as k_residual.  One
// launch per kind of row (PART 0: p and T at centres, 1: r faces, 2: theta
// faces, 3: phi faces), which keeps each kernel's registers in bounds.
template <int PART>
__global__ void __launch_bounds__(256) k_residual_vjp(Geo g, Mat m, SrcOne u, double tau, Fields mu,
                                                      Fields A) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, i = blockIdx.z;
  if (k >= g.npf) return;
  const bool kc = k < g.np;
  const GAcc ga{A};
  if (PART == 0 && i < g.nr && j < g.nt && kc) {
    const long x = idx_c(g, i, j, k);
    F_p_T_rev(g, m, u, i, j, k, -tau * mu.p[x], -tau * mu.T[x], ga);
  }
  if (PART == 1 && j < g.nt && kc && i >= 1 && i < g.nr)
    F_ur_rev(g, m, u, i, j, k, -tau * mu.ur[idx_r(g, i, j, k)], ga);
  if (PART == 2 && i < g.nr && kc && j >= 1 && j < g.nt)
    F_ut_rev(g, m, u, i, j, k, -tau * mu.ut[idx_t(g, i, j, k)], ga);
  if (PART == 3 && i < g.nr && j < g.nt && (g.periodic || (k >= 1 && k < g.np)))
    F_uf_rev(g, m, u, i, j, k, -tau * mu.uf[idx_f(g, i, j, k)], ga);
}

void launch_residual_vjp(const Geo &g, const Mat &m, const Fields &Ub, double tau, const Fields &mu,
                         const Fields &acc_, hipStream_t st) {
  SrcOne u;
  u.a[F_P] = Ub.p; u.a[F_UR] = Ub.ur; u.a[F_UT] = Ub.ut; u.a[F_UF] = Ub.uf; u.a[F_T] = Ub.T;
  const dim3 grid((g.npf + 63) / 64, g.nt + 1, g.nr + 1), block(64);
  hipLaunchKernelGGL(k_residual_vjp<0>, grid, block, 0, st, g, m, u, tau, mu, acc_);
  hipLaunchKernelGGL(k_residual_vjp<1>, grid, block, 0, st, g, m, u, tau, mu, acc_);
  hipLaunchKernelGGL(k_residual_vjp<2>, grid, block, 0, st, g, m, u, tau, mu, acc_);
  hipLaunchKernelGGL(k_residual_vjp<3>, grid, block, 0, st, g, m, u, tau, mu, acc_);
}

// ------------------------------------------------- line rows, reversed --

// Reverse of block_row<D> (rows.hpp) for the coefficient entries: EL, ED, EU
// are the adjoints of the final (scaled) L, D, U blocks of row s.
template <int D, class Acc>
__device__ __forceinline__ void block_row_rev_cb(const Geo &g, const Mat &m, const SrcOne &u, int a, int b, int s, int n,
                                 int cyc, double hs, const double *EL, const double *ED, const double *EU,
                                 const Cent &c, Cent &cb, const Acc &A) {
  int i, j, k;
  if (D == 0) { i = s; j = a; k = b; }
  else if (D == 1) { i = a; j = s; k = b; }
  else { i = a; j = b; k = s; }
  const double ir = g.irc[i], is = g.isc[j], ir2 = ir * ir;
  double hadv, dp_, dm_, lp, lm;
  if (D == 0) {
    hadv = 0.5 * g.idr;
    dp_ = g.rf[i + 1] * g.rf[i + 1] * (ir2 * g.idr);
    dm_ = -g.rf[i] * g.rf[i] * (ir2 * g.idr);
    lp = g.rf[i + 1] * g.rf[i + 1] * (ir2 * g.idr * g.idr);
    lm = g.rf[i] * g.rf[i] * (ir2 * g.idr * g.idr);
  } else if (D == 1) {
    hadv = 0.5 * ir * g.idt;
    dp_ = g.sf[j + 1] * (ir * is * g.idt);
    dm_ = -g.sf[j] * (ir * is * g.idt);
    lp = g.sf[j + 1] * (ir2 * is * g.idt * g.idt);
    lm = g.sf[j] * (ir2 * is * g.idt * g.idt);
  } else {
    hadv = 0.5 * ir * is * g.idp;
    dp_ = ir * is * g.idp;
    dm_ = -dp_;
    lp = ir2 * is * is * g.idp * g.idp;
    lm = lp;
  }
  const bool first = !cyc && s == 0, last = !cyc && s == n - 1;
  if (first) lm = 0.0;
  if (last) lp = 0.0;
  const bool w_unknown = cyc || s < n - 1;
  double ap, am;
  if (D == 0) {
    const double gg = (c.Gtt + c.Gff) * ir;
    ap = m.mu * (2.0 * c.Grr * g.idr + gg - (2.0 / 3.0) * c.tr * dp_);
    am = m.mu * (-2.0 * c.Grr * g.idr + gg - (2.0 / 3.0) * c.tr * dm_);
  } else if (D == 1) {
    const double gg = c.Gff * g.ctc[j] * ir - 0.5 * c.Srt * ir;
    ap = m.mu * (2.0 * c.Gtt * (ir * g.idt) + gg - (2.0 / 3.0) * c.tr * dp_);
    am = m.mu * (-2.0 * c.Gtt * (ir * g.idt) + gg - (2.0 / 3.0) * c.tr * dm_);
  } else {
    const double gg = -0.5 * (c.Srf + c.Stf * g.ctc[j]) * ir;
    ap = m.mu * (2.0 * c.Gff * dp_ + gg - (2.0 / 3.0) * c.tr * dp_);
    am = m.mu * (-2.0 * c.Gff * dp_ + gg - (2.0 / 3.0) * c.tr * dm_);
  }
  // adjoints of the unscaled entries; entries that end up constant or zero
  // carry none
  double L[9], Dg[9], U[9];
#pragma unroll
  for (int q = 0; q < 9; q++) {
    L[q] = first ? 0.0 : hs * EL[q];
    Dg[q] = hs * ED[q];
    U[q] = hs * EU[q];
  }
  if (last) { U[0] = 0.0; U[4] = 0.0; }
  if (!w_unknown) { Dg[2] = 0.0; Dg[5] = 0.0; }
  const double g1 = m.gam - 1.0;
  double advb = -L[0] + U[0] - L[4] + U[4];
  if (first) advb -= Dg[0] + Dg[4];
  if (last) advb += Dg[0] + Dg[4];
  double chib = m.kap * (-lm * L[4] + (lp + lm) * Dg[4] - lp * U[4]);
  double Pb = m.gam * (dm_ * L[2] + dp_ * Dg[2]);
  double Tb = g1 * (dm_ * L[5] + dp_ * Dg[5]);
  const double amb = -g1 * L[2] - c.chi * L[5], apb = -g1 * Dg[2] - c.chi * Dg[5];
  chib += -(am * L[5] + ap * Dg[5]);
  cb.P += Pb;
  cb.T += Tb;
  cb.chi += chib;
  const double ggb = m.mu * (apb + amb);
  cb.tr += -(2.0 / 3.0) * m.mu * (dp_ * apb + dm_ * amb);
  if (D == 0) {
    cb.ur += hadv * advb;
    cb.Grr += 2.0 * m.mu * g.idr * (apb - amb);
    cb.Gtt += ir * ggb;
    cb.Gff += ir * ggb;
  } else if (D == 1) {
    cb.ut += hadv * advb;
    cb.Gtt += 2.0 * m.mu * ir * g.idt * (apb - amb);
    cb.Gff += g.ctc[j] * ir * ggb;
    cb.Srt += -0.5 * ir * ggb;
  } else {
    cb.uf += hadv * advb;
    cb.Gff += 2.0 * m.mu * dp_ * (apb - amb);
    cb.Srf += -0.5 * ir * ggb;
    cb.Stf += -0.5 * g.ctc[j] * ir * ggb;
  }
  if (!w_unknown) return;
  // w row: gp = irho * G, cp / c0 / cm linear in un and nu = mu irho
  const double U8 = (!cyc && s == n - 2) ? 0.0 : U[8];
  double G, hc, ap_, a0_, am_;
  int i1 = i, j1 = j, k1 = k;
  int wf, wi = i, wj = j, wk = k; // the row's face unknown w
  if (D == 0) {
    const int f = i + 1;
    const double irF2 = g.irf[f] * g.irf[f], d2 = g.idr * g.idr, rF2 = g.rf[f] * g.rf[f];
    const double ra2 = g.rc[i] * g.rc[i], rb2 = g.rc[i + 1] * g.rc[i + 1];
    const double ira2 = g.irc[i] * g.irc[i], irb2 = g.irc[i + 1] * g.irc[i + 1];
    G = g.idr;
    hc = 0.5 * g.idr;
    ap_ = -rb2 * irF2 * d2 - g.rf[i + 2] * g.rf[i + 2] * irb2 * d2 / 3.0;
    a0_ = (rb2 + ra2) * irF2 * d2 + rF2 * (irb2 + ira2) * d2 / 3.0;
    am_ = -ra2 * irF2 * d2 - g.rf[i] * g.rf[i] * ira2 * d2 / 3.0;
    i1 = i + 1;
    wf = F_UR; wi = f;
  } else if (D == 1) {
    const int f = j + 1;
    const double sF_ = g.sf[f], isF = g.isf[f], r2d2 = ir2 * g.idt * g.idt;
    const double sa = g.sc[j], sb = g.sc[j + 1], isa = g.isc[j], isb = g.isc[j + 1];
    G = ir * g.idt;
    hc = 0.5 * ir * g.idt;
    ap_ = -sb * r2d2 * isF - g.sf[j + 2] * r2d2 * isb / 3.0;
    a0_ = (sb + sa) * r2d2 * isF + sF_ * (isb + isa) * r2d2 / 3.0;
    am_ = -sa * r2d2 * isF - g.sf[j] * r2d2 * isa / 3.0;
    j1 = j + 1;
    wf = F_UT; wj = f;
  } else {
    const double q2 = ir2 * is * is * g.idp * g.idp;
    G = ir * is * g.idp;
    hc = 0.5 * ir * is * g.idp;
    ap_ = -4.0 * q2 / 3.0;
    a0_ = 8.0 * q2 / 3.0;
    am_ = -4.0 * q2 / 3.0;
    k1 = k + 1;
    wf = F_UF; wk = k + 1; // unwrapped
  }
  const double irho = 1.0 / (0.5 * (rho_at(g, m, u, i, j, k) + rho_at(g, m, u, i1, j1, k1)));
  double irhob = G * (U[6] - Dg[6]);
  const double unb = hc * (U8 - L[8]);
  const double nub = ap_ * U8 + a0_ * Dg[8] + am_ * L[8];
  irhob += m.mu * nub;
  const double rhob = -0.5 * irho * irho * irhob;
  rho_rev(g, m, u, A, i, j, k, rhob);
  rho_rev(g, m, u, A, i1, j1, k1, rhob);
  A.add(g, wf, wi, wj, wk, unb);
}

template <int D, class Acc>
__device__ __forceinline__ void block_row_rev(const Geo &g, const Mat &m, const SrcOne &u, int a, int b, int s, int n,
                              int cyc, double hs, const double *EL, const double *ED, const double *EU,
                              const Acc &A) {
  int i, j, k;
  if (D == 0) { i = s; j = a; k = b; }
  else if (D == 1) { i = a; j = s; k = b; }
  else { i = a; j = b; k = s; }
  Cent c, cb{};
  centre(g, m, u, i, j, k, c);
  block_row_rev_cb<D>(g, m, u, a, b, s, n, cyc, hs, EL, ED, EU, c, cb, A);
  centre_rev(g, m, u, i, j, k, c, cb, A);
}

// Reverse of scalar_row<D, FAM> for its entries: ea, eb, ec are the adjoints
// of the final a, b, c of row s.
// The reverse is returned as rfb, the adjoint of the face density
// rho_f = (rho_c0 + rho_c1)/2, and uab, that of the transverse average
// (scalar_row_parts); scalar_row_rev also scatters them into A.
template <int D, int FAM>
__device__ __forceinline__ void scalar_row_parts(const Geo &g, const Mat &m, const SrcOne &u, int a, int b, int s, int n,
                                 int cyc, double hs, double ea, double eb, double ec, double &rfb,
                                 double &uab, int *cells, long *ix, int &bfid) {
  double h, qa, qb, qc, sglo = -1.0, sghi = -1.0;
  int ci0, cj0, ck0, ci1, cj1, ck1; // the two cells of the face density
  if (D == 0) {
    const int i = s;
    const double ir = g.irc[i], r2d2 = ir * ir * g.idr * g.idr;
    const double fp = g.rf[i + 1] * g.rf[i + 1], fm = g.rf[i] * g.rf[i];
    h = 0.5 * g.idr; qa = fm * r2d2; qb = (fp + fm) * r2d2; qc = fp * r2d2;
    bfid = F_UR;
    if (FAM == 0) {
      const int jf = a, k = b;
      ix[0] = idx_r(g, i, jf - 1, k); ix[1] = idx_r(g, i, jf, k);
      ix[2] = idx_r(g, i + 1, jf - 1, k); ix[3] = idx_r(g, i + 1, jf, k);
      ci0 = i; cj0 = jf - 1; ck0 = k; ci1 = i; cj1 = jf; ck1 = k;
    } else {
      const int j = a, kf = b;
      const int k0 = g.periodic ? wrapk(g, kf - 1) : kf - 1, k1 = g.periodic ? wrapk(g, kf) : kf;
      ix[0] = idx_r(g, i, j, k0); ix[1] = idx_r(g, i, j, k1);
      ix[2] = idx_r(g, i + 1, j, k0); ix[3] = idx_r(g, i + 1, j, k1);
      ci0 = i; cj0 = j; ck0 = k0; ci1 = i; cj1 = j; ck1 = k1;
    }
  } else if (D == 1) {
    const int j = s;
    const double is = g.isc[j];
    double irr;
    bfid = F_UT;
    if (FAM == 0) {
      const int fr = a, k = b;
      irr = g.irf[fr];
      ix[0] = idx_t(g, fr - 1, j, k); ix[1] = idx_t(g, fr - 1, j + 1, k);
      ix[2] = idx_t(g, fr, j, k); ix[3] = idx_t(g, fr, j + 1, k);
      ci0 = fr - 1; cj0 = j; ck0 = k; ci1 = fr; cj1 = j; ck1 = k;
      sglo = g.pole_lo ? 1.0 : -1.0;
      sghi = g.pole_hi ? 1.0 : -1.0;
    } else {
      const int i = a, kf = b;
      irr = g.irc[i];
      const int k0 = g.periodic ? wrapk(g, kf - 1) : kf - 1, k1 = g.periodic ? wrapk(g, kf) : kf;
      ix[0] = idx_t(g, i, j, k0); ix[1] = idx_t(g, i, j, k1);
      ix[2] = idx_t(g, i, j + 1, k0); ix[3] = idx_t(g, i, j + 1, k1);
      ci0 = i; cj0 = j; ck0 = k0; ci1 = i; cj1 = j; ck1 = k1;
    }
    const double q = irr * irr * is * g.idt * g.idt;
    h = 0.5 * irr * g.idt; qa = g.sf[j] * q; qb = (g.sf[j + 1] + g.sf[j]) * q; qc = g.sf[j + 1] * q;
  } else {
    const int k = s;
    const int kp = g.periodic ? wrapk(g, k + 1) : k + 1;
    double irr, iss;
    bfid = F_UF;
    if (FAM == 0) {
      const int fr = a, j = b;
      irr = g.irf[fr]; iss = g.isc[j];
      ix[0] = idx_f(g, fr - 1, j, k); ix[1] = idx_f(g, fr - 1, j, kp);
      ix[2] = idx_f(g, fr, j, k); ix[3] = idx_f(g, fr, j, kp);
      ci0 = fr - 1; cj0 = j; ck0 = k; ci1 = fr; cj1 = j; ck1 = k;
    } else {
      const int i = a, ft = b;
      irr = g.irc[i]; iss = g.isf[ft];
      ix[0] = idx_f(g, i, ft - 1, k); ix[1] = idx_f(g, i, ft - 1, kp);
      ix[2] = idx_f(g, i, ft, k); ix[3] = idx_f(g, i, ft, kp);
      ci0 = i; cj0 = ft - 1; ck0 = k; ci1 = i; cj1 = ft; ck1 = k;
    }
    const double q = irr * irr * iss * iss * g.idp * g.idp;
    h = 0.5 * irr * iss * g.idp; qa = q; qb = 2.0 * q; qc = q;
  }
  const bool first = !cyc && s == 0, last = !cyc && s == n - 1;
  const double cab = first ? hs * sglo * eb : hs * ea;
  const double cbb = hs * eb;
  const double ccb = last ? hs * sghi * eb : hs * ec;
  uab = h * (ccb - cab);
  const double nub = -qa * cab + qb * cbb - qc * ccb;
  const double rho = 0.5 * (rho_at(g, m, u, ci0, cj0, ck0) + rho_at(g, m, u, ci1, cj1, ck1));
  rfb = -m.mu / (rho * rho) * nub;
  cells[0] = ci0; cells[1] = cj0; cells[2] = ck0; cells[3] = ci1; cells[4] = cj1; cells[5] = ck1;
}

template <int D, int FAM>
__device__ __forceinline__ void scalar_row_rev(const Geo &g, const Mat &m, const SrcOne &u, int a, int b, int s, int n,
                               int cyc, double hs, double ea, double eb, double ec, const GAcc &A) {
  double rfb, uab;
  int c[6], bfid;
  long ix[4];
  scalar_row_parts<D, FAM>(g, m, u, a, b, s, n, cyc, hs, ea, eb, ec, rfb, uab, c, ix, bfid);
  rho_rev(g, m, u, A, c[0], c[1], c[2], 0.5 * rfb);
  rho_rev(g, m, u, A, c[3], c[4], c[5], 0.5 * rfb);
  double *base = fsel(A.A, bfid);
#pragma unroll
  for (int q = 0; q < 4; q++) unsafeAtomicAdd(base + ix[q], 0.25 * uab);
}

// the three unknowns (p, T, w) of block s of a line, 0 outside a non-cyclic
// line and for the boundary face that closes it
template <int D>
__device__ __forceinline__ void load3(const Geo &g, const Fields &X, int a, int b, int s, int n, int cyc,
                                      double *v) {
  v[0] = v[1] = v[2] = 0.0;
  if (!cyc && (s < 0 || s >= n)) return;
  if (cyc) s = s < 0 ? s + n : (s >= n ? s - n : s);
  int i, j, k;
  if (D == 0) { i = s; j = a; k = b; }
  else if (D == 1) { i = a; j = s; k = b; }
  else { i = a; j = b; k = s; }
  const long xc = idx_c(g, i, j, k);
  v[0] = X.p[xc];
  v[1] = X.T[xc];
  if (!cyc && s == n - 1) return;
  if (D == 0) v[2] = X.ur[idx_r(g, i + 1, j, k)];
  else if (D == 1) v[2] = X.ut[idx_t(g, i, j + 1, k)];
  else v[2] = X.uf[idx_f(g, i, j, g.periodic ? wrapk(g, k + 1) : k + 1)];
}

template <int D, int FAM>
__device__ __forceinline__ double load1(const Geo &g, const Fields &X, int a, int b, int s, int n, int cyc) {
  if (!cyc && (s < 0 || s >= n)) return 0.0;
  if (cyc) s = s < 0 ? s + n : (s >= n ? s - n : s);
  long x;
  const double *arr;
  if (D == 0) { x = FAM == 0 ? idx_t(g, s, a, b) : idx_f(g, s, a, b); arr = FAM == 0 ? X.ut : X.uf; }
  else if (D == 1) { x = FAM == 0 ? idx_r(g, a, s, b) : idx_f(g, a, s, b); arr = FAM == 0 ? X.ur : X.uf; }
  else { x = FAM == 0 ? idx_r(g, a, b, s) : idx_t(g, a, b, s); arr = FAM == 0 ? X.ur : X.ut; }
  return arr[x];
}

// acc += (d(M_d(Ubar) X)/dUbar)^T mu: one thread per row of every line of
// direction D, numbered so that neighbouring lanes touch neighbouring phi
// positions (r and theta lines: rows outer, lines inner; phi lines: lines
// outer, rows inner)
template <int D>
__global__ void __launch_bounds__(256) k_line_vjp(Geo g, Mat m, SrcOne u, double hs, Fields X,
                                                  Fields mu, Fields Aout) {
  const GAcc A{Aout};
  const Families F = families(g, D);
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = F.n, cyc = F.cyclic;
  const int nkf = g.periodic ? g.np : g.np - 1, kf0 = g.periodic ? 0 : 1;
  const long nbr = (long)F.nb * n, nar = (long)F.na * n, nbbr = (long)F.nbb * n;
  if (t < nbr) {
    const long line = D == 2 ? t / n : t % F.nb;
    const int s = D == 2 ? (int)(t % n) : (int)(t / F.nb);
    int p, q;
    if (D == 2) { p = (int)(line / g.nt); q = (int)(line % g.nt); }
    else { p = (int)(line / g.np); q = (int)(line % g.np); }
    double mv[3], xm[3], x0[3], xp[3], EL[9], ED[9], EU[9];
    load3<D>(g, mu, p, q, s, n, cyc, mv);
    load3<D>(g, X, p, q, s - 1, n, cyc, xm);
    load3<D>(g, X, p, q, s, n, cyc, x0);
    load3<D>(g, X, p, q, s + 1, n, cyc, xp);
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
      for (int c = 0; c < 3; c++) {
        EL[r * 3 + c] = mv[r] * xm[c];
        ED[r * 3 + c] = mv[r] * x0[c];
        EU[r * 3 + c] = mv[r] * xp[c];
      }
    block_row_rev<D>(g, m, u, p, q, s, n, cyc, hs, EL, ED, EU, A);
    return;
  }
  long t2 = t - nbr;
  if (t2 < nar) {
    const long line = D == 2 ? t2 / n : t2 % F.na;
    const int s = D == 2 ? (int)(t2 % n) : (int)(t2 / F.na);
    int p, q;
    if (D == 2) { p = 1 + (int)(line / g.nt); q = (int)(line % g.nt); }
    else { p = 1 + (int)(line / g.np); q = (int)(line % g.np); }
    const double mv = load1<D, 0>(g, mu, p, q, s, n, cyc);
    scalar_row_rev<D, 0>(g, m, u, p, q, s, n, cyc, hs, mv * load1<D, 0>(g, X, p, q, s - 1, n, cyc),
                         mv * load1<D, 0>(g, X, p, q, s, n, cyc), mv * load1<D, 0>(g, X, p, q, s + 1, n, cyc), A);
    return;
  }
  t2 -= nar;
  if (t2 < nbbr) {
    const long line = D == 2 ? t2 / n : t2 % F.nbb;
    const int s = D == 2 ? (int)(t2 % n) : (int)(t2 / F.nbb);
    int p, q;
    if (D == 2) { p = (int)(line / (g.nt - 1)); q = 1 + (int)(line % (g.nt - 1)); }
    else { p = (int)(line / nkf); q = kf0 + (int)(line % nkf); }
    const double mv = load1<D, 1>(g, mu, p, q, s, n, cyc);
    scalar_row_rev<D, 1>(g, m, u, p, q, s, n, cyc, hs, mv * load1<D, 1>(g, X, p, q, s - 1, n, cyc),
                         mv * load1<D, 1>(g, X, p, q, s, n, cyc), mv * load1<D, 1>(g, X, p, q, s + 1, n, cyc), A);
  }
}

void launch_line_vjp(int d, const Geo &g, const Mat &m, const Fields &Ub, double tau, const Fields &X,
                     const Fields &mu, const Fields &acc_, hipStream_t st) {
  SrcOne u;
  u.a[F_P] = Ub.p; u.a[F_UR] = Ub.ur; u.a[F_UT] = Ub.ut; u.a[F_UF] = Ub.uf; u.a[F_T] = Ub.T;
  const Families F = families(g, d);
  const long rows = ((long)F.nb + F.na + F.nbb) * F.n;
  const dim3 grid((unsigned)((rows + 127) / 128)), block(128);
  const double hs = 0.5 * tau;
  if (d == 0) hipLaunchKernelGGL(k_line_vjp<0>, grid, block, 0, st, g, m, u, hs, X, mu, acc_);
  else if (d == 1) hipLaunchKernelGGL(k_line_vjp<1>, grid, block, 0, st, g, m, u, hs, X, mu, acc_);
  else hipLaunchKernelGGL(k_line_vjp<2>, grid, block, 0, st, g, m, u, hs, X, mu, acc_);
}

// ------------------------------------------ fused reverse of one iteration --

// For dsw_adjoint_step: acc += (d(-tau F_h)/dUbar)^T mu[0]
//                              - sum_d (d(M_d(Ubar) X[d])/dUbar)^T mu[d]
// (d = 0 r, 1 theta, 2 phi).  PART 0: every cell, with the p and T rows and
// the three block rows through the cell sharing one evaluation of the centre
// coefficients and one reverse of it; PART 1, 2, 3: the r, theta, phi faces,
// each with its momentum row and the two scalar rows through it.
struct AdjIn {
  Fields X[3], mu[3];
};

template <int D, class Acc>
__device__ __forceinline__ void cell_block_row(const Geo &g, const Mat &m, const SrcOne &u, double hs,
                                               const AdjIn &in, int i, int j, int k, const Cent &c,
                                               Cent &cb, const Acc &A) {
  int a, b, s, n;
  if (D == 0) { a = j; b = k; s = i; n = g.nr; }
  else if (D == 1) { a = i; b = k; s = j; n = g.nt; }
  else { a = i; b = j; s = k; n = g.np; }
  const int cyc = (D == 2 && g.periodic) ? 1 : 0;
  double mv[3], xm[3], x0[3], xp[3], EL[9], ED[9], EU[9];
  load3<D>(g, in.mu[D], a, b, s, n, cyc, mv);
  load3<D>(g, in.X[D], a, b, s - 1, n, cyc, xm);
  load3<D>(g, in.X[D], a, b, s, n, cyc, x0);
  load3<D>(g, in.X[D], a, b, s + 1, n, cyc, xp);
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int q = 0; q < 3; q++) {
      EL[r * 3 + q] = -mv[r] * xm[q];
      ED[r * 3 + q] = -mv[r] * x0[q];
      EU[r * 3 + q] = -mv[r] * xp[q];
    }
  block_row_rev_cb<D>(g, m, u, a, b, s, n, cyc, hs, EL, ED, EU, c, cb, A);
}

// the scalar row of family FAM in direction D through a face: adds the
// adjoints of the face density and of the transverse average it reads to
// rfb, uab (the momentum row of the face reads the same ones)
template <int D, int FAM>
__device__ __forceinline__ void face_scalar_row(const Geo &g, const Mat &m, const SrcOne &u, double hs,
                                                const AdjIn &in, int a, int b, int s, double &rfb,
                                                double &uab) {
  const int n = D == 0 ? g.nr : (D == 1 ? g.nt : g.np);
  const int cyc = (D == 2 && g.periodic) ? 1 : 0;
  const double mv = load1<D, FAM>(g, in.mu[D], a, b, s, n, cyc);
  double r, ua;
  int c[6], bfid;
  long ix[4];
  scalar_row_parts<D, FAM>(g, m, u, a, b, s, n, cyc, hs, -mv * load1<D, FAM>(g, in.X[D], a, b, s - 1, n, cyc),
                           -mv * load1<D, FAM>(g, in.X[D], a, b, s, n, cyc),
                           -mv * load1<D, FAM>(g, in.X[D], a, b, s + 1, n, cyc), r, ua, c, ix, bfid);
  rfb += r;
  uab += ua;
}

// the reverse at one index (i, j, k) of the rows of one kind (PART 0: the
// cell, 1: r-face i, 2: theta-face j, 3: phi-face k), when that row exists
template <int PART, class Acc>
__device__ __forceinline__ void adj_point(const Geo &g, const Mat &m, const SrcOne &u, double tau,
                                          const AdjIn &in, int i, int j, int k, const Acc &A) {
  const double hs = 0.5 * tau;
  const Fields &mu1 = in.mu[0];
  const bool kc = k < g.np;
  if (PART == 0 && i < g.nr && j < g.nt && kc) {
    Cent c, cb{};
    centre(g, m, u, i, j, k, c);
    const long x = idx_c(g, i, j, k);
    F_p_T_rev_cb(g, m, u, i, j, k, c, -tau * mu1.p[x], -tau * mu1.T[x], cb, A);
    cell_block_row<0>(g, m, u, hs, in, i, j, k, c, cb, A);
    cell_block_row<1>(g, m, u, hs, in, i, j, k, c, cb, A);
    cell_block_row<2>(g, m, u, hs, in, i, j, k, c, cb, A);
    centre_rev(g, m, u, i, j, k, c, cb, A);
  }
  double rfb = 0.0, uab = 0.0, ubb = 0.0;
  if (PART == 1 && j < g.nt && kc && i >= 1 && i < g.nr) {
    face_scalar_row<1, 0>(g, m, u, hs, in, i, k, j, rfb, uab); // u_r along theta: reads ua (u_theta)
    face_scalar_row<2, 0>(g, m, u, hs, in, i, j, k, rfb, ubb); // u_r along phi: reads ub (u_phi)
    F_ur_rev(g, m, u, i, j, k, -tau * mu1.ur[idx_r(g, i, j, k)], A, rfb, uab, ubb);
  }
  if (PART == 2 && i < g.nr && kc && j >= 1 && j < g.nt) {
    face_scalar_row<0, 0>(g, m, u, hs, in, j, k, i, rfb, uab); // u_theta along r: ua (u_r)
    face_scalar_row<2, 1>(g, m, u, hs, in, i, j, k, rfb, ubb); // u_theta along phi: ub (u_phi)
    F_ut_rev(g, m, u, i, j, k, -tau * mu1.ut[idx_t(g, i, j, k)], A, rfb, uab, ubb);
  }
  if (PART == 3 && i < g.nr && j < g.nt && (g.periodic || (k >= 1 && k < g.np))) {
    face_scalar_row<0, 1>(g, m, u, hs, in, j, k, i, rfb, uab); // u_phi along r: ua (u_r)
    face_scalar_row<1, 1>(g, m, u, hs, in, i, k, j, rfb, ubb); // u_phi along theta: ub (u_theta)
    F_uf_rev(g, m, u, i, j, k, -tau * mu1.uf[idx_f(g, i, j, k)], A, rfb, uab, ubb);
  }
}

// The cell rows in four pieces, each with its own evaluation of the centre
// coefficients and its own reverse of them (centre_rev is linear in the
// adjoints, so the pieces add up to the fused form): P = 0 the p and T rows,
// P = 1, 2, 3 the block rows of the r, theta, phi lines.  Fewer values live at
// once than in the fused form.
template <int P, class Acc>
__device__ __forceinline__ void adj_cell_piece(const Geo &g, const Mat &m, const SrcOne &u, double tau,
                                               const AdjIn &in, int i, int j, int k, const Acc &A) {
  if (!(i < g.nr && j < g.nt && k < g.np)) return;
  const double hs = 0.5 * tau;
  Cent c, cb{};
  centre(g, m, u, i, j, k, c);
  if constexpr (P == 0) {
    const long x = idx_c(g, i, j, k);
    F_p_T_rev_cb(g, m, u, i, j, k, c, -tau * in.mu[0].p[x], -tau * in.mu[0].T[x], cb, A);
  } else {
    cell_block_row<P - 1>(g, m, u, hs, in, i, j, k, c, cb, A);
  }
  centre_rev(g, m, u, i, j, k, c, cb, A);
}

// One thread per index, FP64 atomics straight into the global arrays.
template <int PART>
__global__ void __launch_bounds__(256) k_adj_local(Geo g, Mat m, SrcOne u, double tau, AdjIn in,
                                                   Fields A) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, i = blockIdx.z;
  if (k >= g.npf) return;
  adj_point<PART>(g, m, u, tau, in, i, j, k, GAcc{A});
}

// Column-tiled variant: a workgroup owns 64 (phi) x JT (theta) indices and
// walks a segment of r planes, doing all four kinds of rows at each plane.
// Every scatter target lies within one index of the source in each direction
// (in its own array's index space), so the adds go into an LDS window of
// three r planes x (JT + 2) x 66 per field (phi indices unwrapped, so a
// periodic neighbour across phi = 0 stays in the window); after plane i is
// done, plane i - 1 can receive nothing more from this workgroup and is added
// to the global arrays (one atomic per non-zero window entry) and cleared for
// plane i + 2.  Global atomics drop from ~100 per cell to ~10.
constexpr int ACOL_K = 64;
constexpr int ACOL_W = ACOL_K + 2;

template <int JT>
struct TileAcc {
  Fields A;
  double *lds;         // [5 fields][3 slots][JT + 2][ACOL_W]
  int i0, j0, k0;      // current plane, first theta row and phi column of the tile
  int sl0, sl1, sl2;   // LDS slots of planes i0 - 1, i0, i0 + 1
  __device__ __forceinline__ void add(const Geo &, int fid, int i, int j, int k, double v) const {
    // in the window by construction; the clamps only keep LDS addresses in
    // bounds
    const int di = min(max(i - i0 + 1, 0), 2), jj = min(max(j - j0 + 1, 0), JT + 1);
    const int kk = min(max(k - k0 + 1, 0), ACOL_W - 1);
    const int sl = di == 0 ? sl0 : (di == 1 ? sl1 : sl2);
    __hip_atomic_fetch_add(&lds[((fid * 3 + sl) * (JT + 2) + jj) * ACOL_W + kk], v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

// add LDS slot sl (plane p) to the global arrays and clear it
template <int JT>
__device__ __forceinline__ void acol_flush(const Geo &g, const Fields &A, double *lds, int sl, int p, int j0,
                                           int k0, int tid, int nth) {
  constexpr int PER = (JT + 2) * ACOL_W;
  for (int e = tid; e < 5 * PER; e += nth) {
    const int fid = e / PER, r = e - fid * PER, jj = r / ACOL_W, kk = r - jj * ACOL_W;
    double *q = &lds[(fid * 3 + sl) * PER + r];
    const double v = *q;
    *q = 0.0;
    if (v == 0.0) continue;
    const int j = j0 - 1 + jj;
    int k = k0 - 1 + kk;
    if (g.periodic) k = wrapk(g, k);
    const int ni = fid == F_UR ? g.nr + 1 : g.nr, nj = fid == F_UT ? g.nt + 1 : g.nt;
    const int nk = fid == F_UF ? g.npf : g.np;
    if (p >= 0 && p < ni && j >= 0 && j < nj && k >= 0 && k < nk) GAcc{A}.add(g, fid, p, j, k, v);
  }
}

template <int JT>
__global__ void __launch_bounds__(64 * JT) k_adj_col(Geo g, Mat m, SrcOne u, double tau, AdjIn in,
                                                     Fields A, int seg) {
  __shared__ double lds[5 * 3 * (JT + 2) * ACOL_W];
  const int tid = threadIdx.y * ACOL_K + threadIdx.x, nth = ACOL_K * JT;
  const int k0 = blockIdx.x * ACOL_K, j0 = blockIdx.y * JT;
  // one wave per theta row (blockDim.x is the wave size): j is wave-uniform
  const int k = k0 + threadIdx.x, j = __builtin_amdgcn_readfirstlane(j0 + (int)threadIdx.y);
  const int ib = blockIdx.z * seg, ie = min(g.nr, ib + seg);
  for (int e = tid; e < 5 * 3 * (JT + 2) * ACOL_W; e += nth) lds[e] = 0.0;
  __syncthreads();
  // plane p lives in slot (p - ib + 1) % 3
  TileAcc<JT> ta{A, lds, 0, j0, k0, 0, 0, 0};
  const bool on = j < g.nt && k < g.np;
#pragma nounroll
  for (int i = ib; i < ie; i++) {
    ta.i0 = i;
    ta.sl0 = (i - ib) % 3;
    ta.sl1 = (i - ib + 1) % 3;
    ta.sl2 = (i - ib + 2) % 3;
    if (on) {
      // the indices pass through an empty asm before each piece, so that
      // nothing derived from them is hoisted out of the loop or shared
      // between pieces (either keeps hundreds of registers live)
      int jv, kv;
#define DSW_ACOL_PIECE(CALL)                  \
      jv = j; kv = k;                         \
      asm volatile("" : "+s"(jv), "+v"(kv));  \
      CALL;
      DSW_ACOL_PIECE((adj_cell_piece<0>(g, m, u, tau, in, i, jv, kv, ta)))
      DSW_ACOL_PIECE((adj_cell_piece<1>(g, m, u, tau, in, i, jv, kv, ta)))
      DSW_ACOL_PIECE((adj_cell_piece<2>(g, m, u, tau, in, i, jv, kv, ta)))
      DSW_ACOL_PIECE((adj_cell_piece<3>(g, m, u, tau, in, i, jv, kv, ta)))
      DSW_ACOL_PIECE((adj_point<1>(g, m, u, tau, in, i, jv, kv, ta)))
      DSW_ACOL_PIECE((adj_point<2>(g, m, u, tau, in, i, jv, kv, ta)))
      DSW_ACOL_PIECE((adj_point<3>(g, m, u, tau, in, i, jv, kv, ta)))
#undef DSW_ACOL_PIECE
    }
    __syncthreads();
    if (i - 1 >= 0) acol_flush<JT>(g, A, lds, (i - ib) % 3, i - 1, j0, k0, tid, nth);
    __syncthreads();
  }
  acol_flush<JT>(g, A, lds, (ie - ib) % 3, ie - 1, j0, k0, tid, nth);
  if (ie <= g.nr) acol_flush<JT>(g, A, lds, (ie - ib + 1) % 3, ie, j0, k0, tid, nth);
}

void launch_adj_local(const Geo &g, const Mat &m, const Fields &Ub, double tau, const Fields *X,
                      const Fields *mu, const Fields &acc_, hipStream_t st) {
  SrcOne u;
  u.a[F_P] = Ub.p; u.a[F_UR] = Ub.ur; u.a[F_UT] = Ub.ut; u.a[F_UF] = Ub.uf; u.a[F_T] = Ub.T;
  AdjIn in;
  for (int d = 0; d < 3; d++) { in.X[d] = X[d]; in.mu[d] = mu[d]; }
#ifndef DSW_ADJ_ATOMIC
  constexpr int JT = DSW_ADJ_JT;
  const int seg = DSW_ADJ_SEG;
  const dim3 grid((g.np + ACOL_K - 1) / ACOL_K, (g.nt + JT - 1) / JT, (g.nr + seg - 1) / seg),
      block(ACOL_K, JT);
  hipLaunchKernelGGL(k_adj_col<JT>, grid, block, 0, st, g, m, u, tau, in, acc_, seg);
#else
  const dim3 grid((g.npf + 63) / 64, g.nt + 1, g.nr + 1), block(64);
  hipLaunchKernelGGL(k_adj_local<0>, grid, block, 0, st, g, m, u, tau, in, acc_);
  hipLaunchKernelGGL(k_adj_local<1>, grid, block, 0, st, g, m, u, tau, in, acc_);
  hipLaunchKernelGGL(k_adj_local<2>, grid, block, 0, st, g, m, u, tau, in, acc_);
  hipLaunchKernelGGL(k_adj_local<3>, grid, block, 0, st, g, m, u, tau, in, acc_);
#endif
}

// --------------------------------------------------- elementwise helpers --

// out = a*x + b*y + c*z over the five arrays (n doubles each, given per
// field); y or z may be null; x is not read when a = 0
__global__ void __launch_bounds__(256) k_axpy3(long n0, long n1, long n2, long n3, long n4, double a,
                                               Fields x, double b, Fields y, double c, Fields z, Fields out) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long ns[5] = {n0, n1, n2, n3, n4};
  int f = 0;
  while (f < 5 && t >= ns[f]) { t -= ns[f]; f++; }
  if (f >= 5) return;
  double v = a != 0.0 ? a * fsel(x, f)[t] : 0.0;
  if (y.p) v += b * fsel(y, f)[t];
  if (z.p) v += c * fsel(z, f)[t];
  fsel(out, f)[t] = v;
}

void launch_axpy3(const long *cnt, double a, const Fields &x, double b, const Fields &y, double c,
                  const Fields &z, const Fields &out, hipStream_t st) {
  const long tot = cnt[0] + cnt[1] + cnt[2] + cnt[3] + cnt[4];
  hipLaunchKernelGGL(k_axpy3, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, cnt[0], cnt[1], cnt[2],
                     cnt[3], cnt[4], a, x, b, y, c, z, out);
}

// One reverse iteration's bookkeeping (boundary-normal faces of every
// iterate are copies of those of U^n):
//   Lnew = (bnd ? 0 : L) - mu1 + ub/2,   lam_n += (bnd ? L : 0) + mu1 + ub/2,
// and ub = 0 for the next iteration's accumulation.  fold (the first
// iteration, whose U^{n+1,0} is U^n): lam_n += Lnew as well, i.e.
// lam_n += L + ub, and Lnew is not written.  first (the last iteration,
// which the reverse takes first): lam_n is written, not accumulated.
__global__ void __launch_bounds__(256) k_adj_mix(Geo g, long n0, long n1, long n2, long n3, long n4,
                                                 Fields L, Fields mu1, Fields ubb, Fields Lnew, Fields lam,
                                                 int fold, int first) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long ns[5] = {n0, n1, n2, n3, n4};
  int f = 0;
  while (f < 5 && t >= ns[f]) { t -= ns[f]; f++; }
  if (f >= 5) return;
  bool bnd = false;
  if (f == F_UR) { const long fr = t / ((long)g.nt * g.np); bnd = fr == 0 || fr == g.nr; }
  else if (f == F_UT) { const long ft = (t / g.np) % (g.nt + 1); bnd = ft == 0 || ft == g.nt; }
  else if (f == F_UF && !g.periodic) { const long ff = t % g.npf; bnd = ff == 0 || ff == g.np; }
  const double l = fsel(L, f)[t], ub = fsel(ubb, f)[t];
  fsel(ubb, f)[t] = 0.0;
  const double prev = first ? 0.0 : fsel(lam, f)[t];
  if (fold) {
    fsel(lam, f)[t] = prev + (l + ub);
    return;
  }
  const double m1 = fsel(mu1, f)[t], hb = 0.5 * ub;
  fsel(Lnew, f)[t] = (bnd ? 0.0 : l) - m1 + hb;
  fsel(lam, f)[t] = prev + ((bnd ? l : 0.0) + m1 + hb);
}

void launch_adj_mix(const Geo &g, const long *cnt, const Fields &L, const Fields &mu1, const Fields &ubb,
                    const Fields &Lnew, const Fields &lam, bool fold, bool first, hipStream_t st) {
  const long tot = cnt[0] + cnt[1] + cnt[2] + cnt[3] + cnt[4];
  hipLaunchKernelGGL(k_adj_mix, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, g, cnt[0], cnt[1],
                     cnt[2], cnt[3], cnt[4], L, mu1, ubb, Lnew, lam, fold ? 1 : 0,
                     first ? 1 : 0);
}

} // namespace dsw
