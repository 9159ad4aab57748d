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

__device__ __forceinline__ void acc(double *p, double v) { unsafeAtomicAdd(p, v); }

// ----------------------------------------------- reverse of the ghost loads --

__device__ __forceinline__ void sC(const Geo &g, const Fields &A, int fid, int i, int j, int k,
                                   double v) {
  i = clampi(i, 0, g.nr - 1);
  j = clampi(j, 0, g.nt - 1);
  k = g.periodic ? wrapk(g, k) : clampi(k, 0, g.np - 1);
  acc((fid == F_P ? A.p : A.T) + idx_c(g, i, j, k), v);
}
__device__ __forceinline__ void sR(const Geo &g, const Fields &A, int f, int j, int k, double v) {
  double sg = 1.0;
  if (k < 0 || k >= g.np) {
    if (g.periodic) k = wrapk(g, k);
    else { sg = -sg; k = k < 0 ? 0 : g.np - 1; }
  }
  if (j < 0) { if (!g.pole_lo) sg = -sg; j = 0; }
  else if (j >= g.nt) { if (!g.pole_hi) sg = -sg; j = g.nt - 1; }
  acc(A.ur + idx_r(g, f, j, k), sg * v);
}
__device__ __forceinline__ void sT(const Geo &g, const Fields &A, int i, int f, int k, double v) {
  double sg = 1.0;
  if (k < 0 || k >= g.np) {
    if (g.periodic) k = wrapk(g, k);
    else { sg = -sg; k = k < 0 ? 0 : g.np - 1; }
  }
  if (i < 0) { sg = -sg; i = 0; }
  else if (i >= g.nr) { sg = -sg; i = g.nr - 1; }
  acc(A.ut + idx_t(g, i, f, k), sg * v);
}
__device__ __forceinline__ void sF(const Geo &g, const Fields &A, int i, int j, int f, double v) {
  double sg = 1.0;
  if (g.periodic) f = wrapk(g, f);
  if (j < 0) { sg = -sg; j = 0; }
  else if (j >= g.nt) { sg = -sg; j = g.nt - 1; }
  if (i < 0) { sg = -sg; i = 0; }
  else if (i >= g.nr) { sg = -sg; i = g.nr - 1; }
  acc(A.uf + idx_f(g, i, j, f), sg * v);
}

// centre averages (avgR / avgT / avgF of dsw_common.hpp), reversed
__device__ __forceinline__ void avgR_rev(const Geo &g, const Fields &A, int i, int j, int k, double a) {
  sR(g, A, i, j, k, 0.5 * a);
  sR(g, A, i + 1, j, k, 0.5 * a);
}
__device__ __forceinline__ void avgT_rev(const Geo &g, const Fields &A, int i, int j, int k, double a) {
  sT(g, A, i, j, k, 0.5 * a);
  sT(g, A, i, j + 1, k, 0.5 * a);
}
__device__ __forceinline__ void avgF_rev(const Geo &g, const Fields &A, int i, int j, int k, double a) {
  sF(g, A, i, j, k, 0.5 * a);
  sF(g, A, i, j, k + 1, 0.5 * a);
}

// rho = (p + pi_inf) / (R T) at a (ghost-mapped) centre, reversed
template <class S>
__device__ __forceinline__ void rho_rev(const Geo &g, const Mat &m, const S &s, const Fields &A, int i,
                                        int j, int k, double rb) {
  const double P = gC(g, s, F_P, i, j, k) + m.pinf, T = gC(g, s, F_T, i, j, k);
  const double iRT = 1.0 / (m.Rg * T);
  sC(g, A, F_P, i, j, k, rb * iRT);
  sC(g, A, F_T, i, j, k, -rb * P * iRT / T);
}

// divc (compact divergence at a centre), reversed
__device__ __forceinline__ void divc_rev(const Geo &g, const Fields &A, int i, int j, int k, double a) {
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
template <class S>
__device__ void centre_rev(const Geo &g, const Mat &m, const S &s, int i, int j, int k, const Cent &c,
                           const Cent &cb, const Fields &A) {
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
template <class S>
__device__ void F_p_T_rev(const Geo &g, const Mat &m, const S &s, int i, int j, int k, double wp,
                          double wT, const Fields &A) {
  Cent c;
  centre(g, m, s, i, j, k, c);
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
  Cent cb{};
  cb.P = m.gam * c.div * wp;
  cb.div = m.gam * c.P * wp + g1 * c.T * wT;
  cb.T = g1 * c.div * wT;
  const double phib = -g1 * wp - c.chi * wT;
  cb.chi = -(phi + m.kap * lap) * wT;
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
  centre_rev(g, m, s, i, j, k, c, cb, A);
}

// radial momentum row at interior r-face (f, j, k) (F_ur of residual.hip)
template <class S>
__device__ void F_ur_rev(const Geo &g, const Mat &m, const S &s, int f, int j, int k, double w,
                         const Fields &A) {
  const double irF = g.irf[f], is = g.isc[j], irF2 = irF * irF;
  const double irho = 1.0 / (0.5 * (rho_at(g, m, s, f - 1, j, k) + rho_at(g, m, s, f, j, k)));
  const double nu = m.mu * irho;
  const double un = gR(g, s, f, j, k);
  const double ua = 0.25 * (gT(g, s, f - 1, j, k) + gT(g, s, f - 1, j + 1, k) + gT(g, s, f, j, k) +
                            gT(g, s, f, j + 1, k));
  const double ub = 0.25 * (gF(g, s, f - 1, j, k) + gF(g, s, f - 1, j, k + 1) + gF(g, s, f, j, k) +
                            gF(g, s, f, j, k + 1));
  const double xp = gR(g, s, f + 1, j, k), xm = gR(g, s, f - 1, j, k);
  const double yp = gR(g, s, f, j + 1, k), ym = gR(g, s, f, j - 1, k);
  const double zp = gR(g, s, f, j, k + 1), zm = gR(g, s, f, j, k - 1);
  const double pa = gC(g, s, F_P, f, j, k), pb = gC(g, s, F_P, f - 1, j, k);
  const double Cr = irF2 * g.idr * g.idr, Ct = irF2 * is * g.idt * g.idt, Cp = irF2 * is * is * g.idp * g.idp;
  const double ra2 = g.rc[f] * g.rc[f], rb2 = g.rc[f - 1] * g.rc[f - 1];
  double vis = (ra2 * (xp - un) - rb2 * (un - xm)) * Cr + (g.sf[j + 1] * (yp - un) - g.sf[j] * (un - ym)) * Ct +
               (zp - 2.0 * un + zm) * Cp;
  const double dth = 0.5 *
                     ((g.sf[j + 1] * gT(g, s, f - 1, j + 1, k) - g.sf[j] * gT(g, s, f - 1, j, k)) +
                      (g.sf[j + 1] * gT(g, s, f, j + 1, k) - g.sf[j] * gT(g, s, f, j, k))) * g.idt;
  const double dph = 0.5 *
                     ((gF(g, s, f - 1, j, k + 1) - gF(g, s, f - 1, j, k)) +
                      (gF(g, s, f, j, k + 1) - gF(g, s, f, j, k))) * g.idp;
  vis += -2.0 * un * irF2 - 2.0 * irF2 * is * dth - 2.0 * irF2 * is * dph;
  const double gd = (divc(g, s, f, j, k) - divc(g, s, f - 1, j, k)) * g.idr;
  // reverse of F = N - nu vis - nu/3 gd + g_r
  const double Nb = w, visb = -nu * w, gdb = -nu / 3.0 * w, nub = -(vis + gd / 3.0) * w;
  double ubb = -2.0 * m.omega * g.sc[j] * Nb, uab = 0.0, unb = 0.0;
  divc_rev(g, A, f, j, k, g.idr * gdb);
  divc_rev(g, A, f - 1, j, k, -g.idr * gdb);
  unb += -2.0 * irF2 * visb;
  const double dthb = -2.0 * irF2 * is * visb, dphb = -2.0 * irF2 * is * visb;
  sF(g, A, f - 1, j, k + 1, 0.5 * g.idp * dphb);
  sF(g, A, f - 1, j, k, -0.5 * g.idp * dphb);
  sF(g, A, f, j, k + 1, 0.5 * g.idp * dphb);
  sF(g, A, f, j, k, -0.5 * g.idp * dphb);
  sT(g, A, f - 1, j + 1, k, 0.5 * g.idt * g.sf[j + 1] * dthb);
  sT(g, A, f - 1, j, k, -0.5 * g.idt * g.sf[j] * dthb);
  sT(g, A, f, j + 1, k, 0.5 * g.idt * g.sf[j + 1] * dthb);
  sT(g, A, f, j, k, -0.5 * g.idt * g.sf[j] * dthb);
  double xpb = ra2 * Cr * visb, xmb = rb2 * Cr * visb;
  double ypb = g.sf[j + 1] * Ct * visb, ymb = g.sf[j] * Ct * visb;
  double zpb = Cp * visb, zmb = Cp * visb;
  unb -= ((ra2 + rb2) * Cr + (g.sf[j + 1] + g.sf[j]) * Ct + 2.0 * Cp) * visb;
  // N
  const double hr = 0.5 * g.idr, ht = 0.5 * irF * g.idt, hp = 0.5 * irF * is * g.idp;
  double irhob = (pa - pb) * g.idr * Nb;
  sC(g, A, F_P, f, j, k, irho * g.idr * Nb);
  sC(g, A, F_P, f - 1, j, k, -irho * g.idr * Nb);
  unb += (xp - xm) * hr * Nb; xpb += un * hr * Nb; xmb -= un * hr * Nb;
  uab += (yp - ym) * ht * Nb; ypb += ua * ht * Nb; ymb -= ua * ht * Nb;
  ubb += (zp - zm) * hp * Nb; zpb += ub * hp * Nb; zmb -= ub * hp * Nb;
  uab += -2.0 * ua * irF * Nb;
  ubb += -2.0 * ub * irF * Nb;
  irhob += m.mu * nub;
  const double rhob = -0.5 * irho * irho * irhob;
  rho_rev(g, m, s, A, f - 1, j, k, rhob);
  rho_rev(g, m, s, A, f, j, k, rhob);
  sR(g, A, f, j, k, unb);
  sR(g, A, f + 1, j, k, xpb);
  sR(g, A, f - 1, j, k, xmb);
  sR(g, A, f, j + 1, k, ypb);
  sR(g, A, f, j - 1, k, ymb);
  sR(g, A, f, j, k + 1, zpb);
  sR(g, A, f, j, k - 1, zmb);
  sT(g, A, f - 1, j, k, 0.25 * uab);
  sT(g, A, f - 1, j + 1, k, 0.25 * uab);
  sT(g, A, f, j, k, 0.25 * uab);
  sT(g, A, f, j + 1, k, 0.25 * uab);
  sF(g, A, f - 1, j, k, 0.25 * ubb);
  sF(g, A, f - 1, j, k + 1, 0.25 * ubb);
  sF(g, A, f, j, k, 0.25 * ubb);
  sF(g, A, f, j, k + 1, 0.25 * ubb);
}

// colatitudinal momentum row at interior theta-face (i, f, k) (F_ut)
template <class S>
__device__ void F_ut_rev(const Geo &g, const Mat &m, const S &s, int i, int f, int k, double w,
                         const Fields &A) {
  const double ir = g.irc[i], isF = g.isf[f], ctF = g.ctf[f], ir2 = ir * ir;
  const int j0 = f - 1, j1 = f;
  const double irho = 1.0 / (0.5 * (rho_at(g, m, s, i, j0, k) + rho_at(g, m, s, i, j1, k)));
  const double nu = m.mu * irho;
  const double un = gT(g, s, i, f, k);
  const double ua = 0.25 * (gR(g, s, i, j0, k) + gR(g, s, i, j1, k) + gR(g, s, i + 1, j0, k) +
                            gR(g, s, i + 1, j1, k));
  const double ub = 0.25 * (gF(g, s, i, j0, k) + gF(g, s, i, j0, k + 1) + gF(g, s, i, j1, k) +
                            gF(g, s, i, j1, k + 1));
  const double xp = gT(g, s, i + 1, f, k), xm = gT(g, s, i - 1, f, k);
  const double yp = gT(g, s, i, f + 1, k), ym = gT(g, s, i, f - 1, k);
  const double zp = gT(g, s, i, f, k + 1), zm = gT(g, s, i, f, k - 1);
  const double p1 = gC(g, s, F_P, i, j1, k), p0 = gC(g, s, F_P, i, j0, k);
  const double Cr = ir2 * g.idr * g.idr, Ct = ir2 * isF * g.idt * g.idt, Cp = ir2 * isF * isF * g.idp * g.idp;
  const double rp2 = g.rf[i + 1] * g.rf[i + 1], rm2 = g.rf[i] * g.rf[i];
  double vis = (rp2 * (xp - un) - rm2 * (un - xm)) * Cr + (g.sc[j1] * (yp - un) - g.sc[j0] * (un - ym)) * Ct +
               (zp - 2.0 * un + zm) * Cp;
  const double dthr = 0.5 * ((gR(g, s, i, j1, k) - gR(g, s, i, j0, k)) + (gR(g, s, i + 1, j1, k) - gR(g, s, i + 1, j0, k))) * g.idt;
  const double dphf = 0.5 * ((gF(g, s, i, j0, k + 1) - gF(g, s, i, j0, k)) + (gF(g, s, i, j1, k + 1) - gF(g, s, i, j1, k))) * g.idp;
  vis += -un * ir2 * isF * isF + 2.0 * ir2 * dthr - 2.0 * ctF * ir2 * isF * dphf;
  const double gd = (divc(g, s, i, j1, k) - divc(g, s, i, j0, k)) * (ir * g.idt);
  const double Nb = w, visb = -nu * w, gdb = -nu / 3.0 * w, nub = -(vis + gd / 3.0) * w;
  double ubb = -2.0 * m.omega * g.cf[f] * Nb, uab = 0.0, unb = 0.0;
  divc_rev(g, A, i, j1, k, ir * g.idt * gdb);
  divc_rev(g, A, i, j0, k, -ir * g.idt * gdb);
  unb += -ir2 * isF * isF * visb;
  const double dthrb = 2.0 * ir2 * visb, dphfb = -2.0 * ctF * ir2 * isF * visb;
  sR(g, A, i, j1, k, 0.5 * g.idt * dthrb);
  sR(g, A, i, j0, k, -0.5 * g.idt * dthrb);
  sR(g, A, i + 1, j1, k, 0.5 * g.idt * dthrb);
  sR(g, A, i + 1, j0, k, -0.5 * g.idt * dthrb);
  sF(g, A, i, j0, k + 1, 0.5 * g.idp * dphfb);
  sF(g, A, i, j0, k, -0.5 * g.idp * dphfb);
  sF(g, A, i, j1, k + 1, 0.5 * g.idp * dphfb);
  sF(g, A, i, j1, k, -0.5 * g.idp * dphfb);
  double xpb = rp2 * Cr * visb, xmb = rm2 * Cr * visb;
  double ypb = g.sc[j1] * Ct * visb, ymb = g.sc[j0] * Ct * visb;
  double zpb = Cp * visb, zmb = Cp * visb;
  unb -= ((rp2 + rm2) * Cr + (g.sc[j1] + g.sc[j0]) * Ct + 2.0 * Cp) * visb;
  const double hr = 0.5 * g.idr, ht = 0.5 * ir * g.idt, hp = 0.5 * ir * isF * g.idp;
  double irhob = (p1 - p0) * ir * g.idt * Nb;
  sC(g, A, F_P, i, j1, k, irho * ir * g.idt * Nb);
  sC(g, A, F_P, i, j0, k, -irho * ir * g.idt * Nb);
  uab += (xp - xm) * hr * Nb; xpb += ua * hr * Nb; xmb -= ua * hr * Nb;
  unb += (yp - ym) * ht * Nb; ypb += un * ht * Nb; ymb -= un * ht * Nb;
  ubb += (zp - zm) * hp * Nb; zpb += ub * hp * Nb; zmb -= ub * hp * Nb;
  unb += ua * ir * Nb;
  uab += un * ir * Nb;
  ubb += -2.0 * ub * ctF * ir * Nb;
  irhob += m.mu * nub;
  const double rhob = -0.5 * irho * irho * irhob;
  rho_rev(g, m, s, A, i, j0, k, rhob);
  rho_rev(g, m, s, A, i, j1, k, rhob);
  sT(g, A, i, f, k, unb);
  sT(g, A, i + 1, f, k, xpb);
  sT(g, A, i - 1, f, k, xmb);
  sT(g, A, i, f + 1, k, ypb);
  sT(g, A, i, f - 1, k, ymb);
  sT(g, A, i, f, k + 1, zpb);
  sT(g, A, i, f, k - 1, zmb);
  sR(g, A, i, j0, k, 0.25 * uab);
  sR(g, A, i, j1, k, 0.25 * uab);
  sR(g, A, i + 1, j0, k, 0.25 * uab);
  sR(g, A, i + 1, j1, k, 0.25 * uab);
  sF(g, A, i, j0, k, 0.25 * ubb);
  sF(g, A, i, j0, k + 1, 0.25 * ubb);
  sF(g, A, i, j1, k, 0.25 * ubb);
  sF(g, A, i, j1, k + 1, 0.25 * ubb);
}

// azimuthal momentum row at phi-face (i, j, f) (F_uf)
template <class S>
__device__ void F_uf_rev(const Geo &g, const Mat &m, const S &s, int i, int j, int f, double w,
                         const Fields &A) {
  const double ir = g.irc[i], is = g.isc[j], ct = g.ctc[j], ir2 = ir * ir;
  const int k0 = g.periodic ? wrapk(g, f - 1) : f - 1, k1 = g.periodic ? wrapk(g, f) : f;
  const double irho = 1.0 / (0.5 * (rho_at(g, m, s, i, j, k0) + rho_at(g, m, s, i, j, k1)));
  const double nu = m.mu * irho;
  const double un = gF(g, s, i, j, f);
  const double ua = 0.25 * (gR(g, s, i, j, k0) + gR(g, s, i, j, k1) + gR(g, s, i + 1, j, k0) +
                            gR(g, s, i + 1, j, k1));
  const double ub = 0.25 * (gT(g, s, i, j, k0) + gT(g, s, i, j, k1) + gT(g, s, i, j + 1, k0) +
                            gT(g, s, i, j + 1, k1));
  const double xp = gF(g, s, i + 1, j, f), xm = gF(g, s, i - 1, j, f);
  const double yp = gF(g, s, i, j + 1, f), ym = gF(g, s, i, j - 1, f);
  const double zp = gF(g, s, i, j, f + 1), zm = gF(g, s, i, j, f - 1);
  const double p1 = gC(g, s, F_P, i, j, k1), p0 = gC(g, s, F_P, i, j, k0);
  const double Cr = ir2 * g.idr * g.idr, Ct = ir2 * is * g.idt * g.idt, Cp = ir2 * is * is * g.idp * g.idp;
  const double rp2 = g.rf[i + 1] * g.rf[i + 1], rm2 = g.rf[i] * g.rf[i];
  double vis = (rp2 * (xp - un) - rm2 * (un - xm)) * Cr + (g.sf[j + 1] * (yp - un) - g.sf[j] * (un - ym)) * Ct +
               (zp - 2.0 * un + zm) * Cp;
  const double dphr = 0.5 * ((gR(g, s, i, j, k1) - gR(g, s, i, j, k0)) + (gR(g, s, i + 1, j, k1) - gR(g, s, i + 1, j, k0))) * g.idp;
  const double dpht = 0.5 * ((gT(g, s, i, j, k1) - gT(g, s, i, j, k0)) + (gT(g, s, i, j + 1, k1) - gT(g, s, i, j + 1, k0))) * g.idp;
  vis += -un * ir2 * is * is + 2.0 * ir2 * is * dphr + 2.0 * ct * ir2 * is * dpht;
  const double gd = (divc(g, s, i, j, k1) - divc(g, s, i, j, k0)) * (ir * is * g.idp);
  const double Nb = w, visb = -nu * w, gdb = -nu / 3.0 * w, nub = -(vis + gd / 3.0) * w;
  double ubb = 2.0 * m.omega * g.cc[j] * Nb, uab = 2.0 * m.omega * g.sc[j] * Nb, unb = 0.0;
  divc_rev(g, A, i, j, k1, ir * is * g.idp * gdb);
  divc_rev(g, A, i, j, k0, -ir * is * g.idp * gdb);
  unb += -ir2 * is * is * visb;
  const double dphrb = 2.0 * ir2 * is * visb, dphtb = 2.0 * ct * ir2 * is * visb;
  sR(g, A, i, j, k1, 0.5 * g.idp * dphrb);
  sR(g, A, i, j, k0, -0.5 * g.idp * dphrb);
  sR(g, A, i + 1, j, k1, 0.5 * g.idp * dphrb);
  sR(g, A, i + 1, j, k0, -0.5 * g.idp * dphrb);
  sT(g, A, i, j, k1, 0.5 * g.idp * dphtb);
  sT(g, A, i, j, k0, -0.5 * g.idp * dphtb);
  sT(g, A, i, j + 1, k1, 0.5 * g.idp * dphtb);
  sT(g, A, i, j + 1, k0, -0.5 * g.idp * dphtb);
  double xpb = rp2 * Cr * visb, xmb = rm2 * Cr * visb;
  double ypb = g.sf[j + 1] * Ct * visb, ymb = g.sf[j] * Ct * visb;
  double zpb = Cp * visb, zmb = Cp * visb;
  unb -= ((rp2 + rm2) * Cr + (g.sf[j + 1] + g.sf[j]) * Ct + 2.0 * Cp) * visb;
  const double hr = 0.5 * g.idr, ht = 0.5 * ir * g.idt, hp = 0.5 * ir * is * g.idp;
  double irhob = (p1 - p0) * ir * is * g.idp * Nb;
  sC(g, A, F_P, i, j, k1, irho * ir * is * g.idp * Nb);
  sC(g, A, F_P, i, j, k0, -irho * ir * is * g.idp * Nb);
  uab += (xp - xm) * hr * Nb; xpb += ua * hr * Nb; xmb -= ua * hr * Nb;
  ubb += (yp - ym) * ht * Nb; ypb += ub * ht * Nb; ymb -= ub * ht * Nb;
  unb += (zp - zm) * hp * Nb; zpb += un * hp * Nb; zmb -= un * hp * Nb;
  unb += (ua + ub * ct) * ir * Nb;
  uab += un * ir * Nb;
  ubb += un * ct * ir * Nb;
  irhob += m.mu * nub;
  const double rhob = -0.5 * irho * irho * irhob;
  rho_rev(g, m, s, A, i, j, k0, rhob);
  rho_rev(g, m, s, A, i, j, k1, rhob);
  sF(g, A, i, j, f, unb);
  sF(g, A, i + 1, j, f, xpb);
  sF(g, A, i - 1, j, f, xmb);
  sF(g, A, i, j + 1, f, ypb);
  sF(g, A, i, j - 1, f, ymb);
  sF(g, A, i, j, f + 1, zpb);
  sF(g, A, i, j, f - 1, zmb);
  sR(g, A, i, j, k0, 0.25 * uab);
  sR(g, A, i, j, k1, 0.25 * uab);
  sR(g, A, i + 1, j, k0, 0.25 * uab);
  sR(g, A, i + 1, j, k1, 0.25 * uab);
  sT(g, A, i, j, k0, 0.25 * ubb);
  sT(g, A, i, j, k1, 0.25 * ubb);
  sT(g, A, i, j + 1, k0, 0.25 * ubb);
  sT(g, A, i, j + 1, k1, 0.25 * ubb);
}

// acc += (d(-tau F_h(Ubar))/dUbar)^T mu over every unknown row (the rows of the
// boundary-normal faces are constant); index space as k_residual
__global__ void __launch_bounds__(256) k_residual_vjp(Geo g, Mat m, SrcOne u, double tau, Fields mu,
                                                      Fields A) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, i = blockIdx.z;
  if (k >= g.npf) return;
  const bool kc = k < g.np;
  if (i < g.nr && j < g.nt && kc) {
    const long x = idx_c(g, i, j, k);
    F_p_T_rev(g, m, u, i, j, k, -tau * mu.p[x], -tau * mu.T[x], A);
  }
  if (j < g.nt && kc && i >= 1 && i < g.nr) F_ur_rev(g, m, u, i, j, k, -tau * mu.ur[idx_r(g, i, j, k)], A);
  if (i < g.nr && kc && j >= 1 && j < g.nt) F_ut_rev(g, m, u, i, j, k, -tau * mu.ut[idx_t(g, i, j, k)], A);
  if (i < g.nr && j < g.nt && (g.periodic || (k >= 1 && k < g.np)))
    F_uf_rev(g, m, u, i, j, k, -tau * mu.uf[idx_f(g, i, j, k)], A);
}

void launch_residual_vjp(const Geo &g, const Mat &m, const Fields &Ub, double tau, const Fields &mu,
                         const Fields &acc_, hipStream_t st) {
  SrcOne u;
  u.a[F_P] = Ub.p; u.a[F_UR] = Ub.ur; u.a[F_UT] = Ub.ut; u.a[F_UF] = Ub.uf; u.a[F_T] = Ub.T;
  dim3 grid((g.npf + 63) / 64, g.nt + 1, g.nr + 1);
  hipLaunchKernelGGL(k_residual_vjp, grid, dim3(64), 0, st, g, m, u, tau, mu, acc_);
}

// ------------------------------------------------- line rows, reversed --

// Reverse of block_row<D> (rows.hpp) for the coefficient entries: EL, ED, EU
// are the adjoints of the final (scaled) L, D, U blocks of row s.
template <int D>
__device__ void block_row_rev(const Geo &g, const Mat &m, const SrcOne &u, int a, int b, int s, int n,
                              int cyc, double hs, const double *EL, const double *ED, const double *EU,
                              const Fields &A) {
  int i, j, k;
  if (D == 0) { i = s; j = a; k = b; }
  else if (D == 1) { i = a; j = s; k = b; }
  else { i = a; j = b; k = s; }
  Cent c;
  centre(g, m, u, i, j, k, c);
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
  Cent cb{};
  cb.P = Pb;
  cb.T = Tb;
  cb.chi = chib;
  const double ggb = m.mu * (apb + amb);
  cb.tr = -(2.0 / 3.0) * m.mu * (dp_ * apb + dm_ * amb);
  if (D == 0) {
    cb.ur = hadv * advb;
    cb.Grr = 2.0 * m.mu * g.idr * (apb - amb);
    cb.Gtt = ir * ggb;
    cb.Gff = ir * ggb;
  } else if (D == 1) {
    cb.ut = hadv * advb;
    cb.Gtt = 2.0 * m.mu * ir * g.idt * (apb - amb);
    cb.Gff = g.ctc[j] * ir * ggb;
    cb.Srt = -0.5 * ir * ggb;
  } else {
    cb.uf = hadv * advb;
    cb.Gff = 2.0 * m.mu * dp_ * (apb - amb);
    cb.Srf = -0.5 * ir * ggb;
    cb.Stf = -0.5 * g.ctc[j] * ir * ggb;
  }
  centre_rev(g, m, u, i, j, k, c, cb, A);
  if (!w_unknown) return;
  // w row: gp = irho * G, cp / c0 / cm linear in un and nu = mu irho
  const double U8 = (!cyc && s == n - 2) ? 0.0 : U[8];
  double G, hc, ap_, a0_, am_;
  int i1 = i, j1 = j, k1 = k;
  double *up;
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
    up = A.ur + idx_r(g, f, j, k);
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
    up = A.ut + idx_t(g, i, f, k);
  } else {
    const int f = g.periodic ? wrapk(g, k + 1) : k + 1;
    const double q2 = ir2 * is * is * g.idp * g.idp;
    G = ir * is * g.idp;
    hc = 0.5 * ir * is * g.idp;
    ap_ = -4.0 * q2 / 3.0;
    a0_ = 8.0 * q2 / 3.0;
    am_ = -4.0 * q2 / 3.0;
    k1 = k + 1;
    up = A.uf + idx_f(g, i, j, f);
  }
  const double irho = 1.0 / (0.5 * (rho_at(g, m, u, i, j, k) + rho_at(g, m, u, i1, j1, k1)));
  double irhob = G * (U[6] - Dg[6]);
  const double unb = hc * (U8 - L[8]);
  const double nub = ap_ * U8 + a0_ * Dg[8] + am_ * L[8];
  irhob += m.mu * nub;
  const double rhob = -0.5 * irho * irho * irhob;
  rho_rev(g, m, u, A, i, j, k, rhob);
  rho_rev(g, m, u, A, i1, j1, k1, rhob);
  acc(up, unb);
}

// Reverse of scalar_row<D, FAM> for its entries: ea, eb, ec are the adjoints
// of the final a, b, c of row s.
template <int D, int FAM>
__device__ void scalar_row_rev(const Geo &g, const Mat &m, const SrcOne &u, int a, int b, int s, int n,
                               int cyc, double hs, double ea, double eb, double ec, const Fields &A) {
  double h, qa, qb, qc, sglo = -1.0, sghi = -1.0;
  int ci0, cj0, ck0, ci1, cj1, ck1; // the two cells of the face density
  long ix[4];                        // the four loads of the transverse average
  double *base;
  if (D == 0) {
    const int i = s;
    const double ir = g.irc[i], r2d2 = ir * ir * g.idr * g.idr;
    const double fp = g.rf[i + 1] * g.rf[i + 1], fm = g.rf[i] * g.rf[i];
    h = 0.5 * g.idr; qa = fm * r2d2; qb = (fp + fm) * r2d2; qc = fp * r2d2;
    base = A.ur;
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
    base = A.ut;
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
    base = A.uf;
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
  const double uab = h * (ccb - cab);
  const double nub = -qa * cab + qb * cbb - qc * ccb;
  const double rho = 0.5 * (rho_at(g, m, u, ci0, cj0, ck0) + rho_at(g, m, u, ci1, cj1, ck1));
  const double rhob = -m.mu / (rho * rho) * nub;
  rho_rev(g, m, u, A, ci0, cj0, ck0, 0.5 * rhob);
  rho_rev(g, m, u, A, ci1, cj1, ck1, 0.5 * rhob);
#pragma unroll
  for (int q = 0; q < 4; q++) acc(base + ix[q], 0.25 * uab);
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
// direction D (rows s outer, lines inner, so that lanes read neighbouring
// phi positions)
template <int D>
__global__ void __launch_bounds__(256) k_line_vjp(Geo g, Mat m, SrcOne u, double hs, Fields X,
                                                  Fields mu, Fields A) {
  const Families F = families(g, D);
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = F.n, cyc = F.cyclic;
  const int nkf = g.periodic ? g.np : g.np - 1, kf0 = g.periodic ? 0 : 1;
  const long nbr = (long)F.nb * n, nar = (long)F.na * n, nbbr = (long)F.nbb * n;
  if (t < nbr) {
    const long line = t % F.nb;
    const int s = (int)(t / F.nb);
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
    const long line = t2 % F.na;
    const int s = (int)(t2 / F.na);
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
    const long line = t2 % F.nbb;
    const int s = (int)(t2 / F.nbb);
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

// --------------------------------------------------- elementwise helpers --

// out = a*x + b*y + c*z over the five arrays (n doubles each, given per
// field); y or z may be null
__global__ void __launch_bounds__(256) k_axpy3(long n0, long n1, long n2, long n3, long n4, double a,
                                               Fields x, double b, Fields y, double c, Fields z, Fields out) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long ns[5] = {n0, n1, n2, n3, n4};
  int f = 0;
  while (f < 5 && t >= ns[f]) { t -= ns[f]; f++; }
  if (f >= 5) return;
  double v = a * fsel(x, f)[t];
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
//   Lnew = (bnd ? 0 : L) - mu1 + ub/2,   lam_n += (bnd ? L : 0) + mu1 + ub/2
__global__ void __launch_bounds__(256) k_adj_mix(Geo g, long n0, long n1, long n2, long n3, long n4,
                                                 Fields L, Fields mu1, Fields ubb, Fields Lnew, Fields lam) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long ns[5] = {n0, n1, n2, n3, n4};
  int f = 0;
  while (f < 5 && t >= ns[f]) { t -= ns[f]; f++; }
  if (f >= 5) return;
  bool bnd = false;
  if (f == F_UR) { const long fr = t / ((long)g.nt * g.np); bnd = fr == 0 || fr == g.nr; }
  else if (f == F_UT) { const long ft = (t / g.np) % (g.nt + 1); bnd = ft == 0 || ft == g.nt; }
  else if (f == F_UF && !g.periodic) { const long ff = t % g.npf; bnd = ff == 0 || ff == g.np; }
  const double l = fsel(L, f)[t], m1 = fsel(mu1, f)[t], hb = 0.5 * fsel(ubb, f)[t];
  fsel(Lnew, f)[t] = (bnd ? 0.0 : l) - m1 + hb;
  fsel(lam, f)[t] += (bnd ? l : 0.0) + m1 + hb;
}

void launch_adj_mix(const Geo &g, const long *cnt, const Fields &L, const Fields &mu1, const Fields &ubb,
                    const Fields &Lnew, const Fields &lam, hipStream_t st) {
  const long tot = cnt[0] + cnt[1] + cnt[2] + cnt[3] + cnt[4];
  hipLaunchKernelGGL(k_adj_mix, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, g, cnt[0], cnt[1],
                     cnt[2], cnt[3], cnt[4], L, mu1, ubb, Lnew, lam);
}

} // namespace dsw
