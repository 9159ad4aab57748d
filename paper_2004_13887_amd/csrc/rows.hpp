// rows.hpp -- assembly of one row of the line systems (I + tau/2 D_d(Ubar))
// of the three split sweeps (paper eqs. (spl1)-(spl3); direction operators
// of Appendix B, eqs. (dr), (dtheta), (dphi)), and 3x3 helpers.  Shared by the
// thread-per-line and the partitioned line solvers.
#pragma once

#include "dsw_common.hpp"
#include "dsw_internal.hpp"

namespace dsw {

struct BRow {
  double L[9], D[9], U[9], b[3];
};

// The coupling of a line's end rows to values beyond its ends, scaled by
// tau/2, as the line assembly drops or folds it for homogeneous increment
// data: lo[0..2] the p, T and w rows of block 0 on the boundary face before
// it; hi[0..1] the p and T rows of block n-1 on the boundary face that closes
// the line, hiw the w row of block n-2 on that face; slo, shi the scalar rows
// 0 and n-1 on their ghost values.  Filled only where a row asks for it.
struct Edge {
  double lo[3], hi[2], hiw, slo, shi;
};

// X = A^{-1} (3x3); returns whether A is singular (a zero or non-finite
// determinant)
__device__ __forceinline__ bool inv3q(const double *A, double *X) {
  const double c00 = A[4] * A[8] - A[5] * A[7];
  const double c01 = A[5] * A[6] - A[3] * A[8];
  const double c02 = A[3] * A[7] - A[4] * A[6];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  const double id = rcp_nr(det);
  X[0] = c00 * id;
  X[1] = (A[2] * A[7] - A[1] * A[8]) * id;
  X[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  X[3] = c01 * id;
  X[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  X[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  X[6] = c02 * id;
  X[7] = (A[1] * A[6] - A[0] * A[7]) * id;
  X[8] = (A[0] * A[4] - A[1] * A[3]) * id;
  return !(det != 0.0) || !isfinite(det);
}

__device__ __forceinline__ void inv3(const double *A, double *X, int *status) {
  if (inv3q(A, X)) status[ST_SINGULAR] = 1;
}

// C = A * B (3x3)
__device__ __forceinline__ void mm3(const double *A, const double *B, double *C) {
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int c = 0; c < 3; c++) C[r * 3 + c] = A[r * 3] * B[c] + A[r * 3 + 1] * B[3 + c] + A[r * 3 + 2] * B[6 + c];
}
// y = A * x (3x3 . 3)
__device__ __forceinline__ void mv3(const double *A, const double *x, double *y) {
#pragma unroll
  for (int r = 0; r < 3; r++) y[r] = A[r * 3] * x[0] + A[r * 3 + 1] * x[1] + A[r * 3 + 2] * x[2];
}

// B -= A * P and y -= A * x, each product rounded as mm3 / mv3 round it;
// A <- -(A * P) in place, a row at a time.  The reductions use these to keep
// few registers live beside the rows they carry.
__device__ __forceinline__ void mm3_sub(const double *A, const double *P, double *B) {
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int c = 0; c < 3; c++) B[r * 3 + c] -= A[r * 3] * P[c] + A[r * 3 + 1] * P[3 + c] + A[r * 3 + 2] * P[6 + c];
}
__device__ __forceinline__ void mv3_sub(const double *A, const double *x, double *y) {
#pragma unroll
  for (int r = 0; r < 3; r++) y[r] -= A[r * 3] * x[0] + A[r * 3 + 1] * x[1] + A[r * 3 + 2] * x[2];
}
__device__ __forceinline__ void mm3_neg_inplace(double *A, const double *P) {
#pragma unroll
  for (int r = 0; r < 3; r++) {
    double t[3];
#pragma unroll
    for (int c = 0; c < 3; c++) t[c] = A[r * 3] * P[c] + A[r * 3 + 1] * P[3 + c] + A[r * 3 + 2] * P[6 + c];
#pragma unroll
    for (int c = 0; c < 3; c++) A[r * 3 + c] = -t[c];
  }
}

// Structural non-zeros of the blocks that block_row assembles: bit 3r + c is
// set where entry (r, c) can be non-zero (unknowns p, T, w).  The lower block
// couples the p and T rows to p, T and w of the row before, the w row to w
// only; the upper block couples p to p and T, T to T, and w to p and w.  The
// zeros are computed as 0 * tau/2, which the compiler may not fold, so the
// full products spend a third or more of their FMAs on them.
constexpr unsigned NZ_ALL = 0x1FFu;
constexpr unsigned NZ_L = 0x137u;  // (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)
constexpr unsigned NZ_U = 0x153u;  // (0,0) (0,1) (1,1) (2,0) (2,2)
// mask of the transposed block
__host__ __device__ constexpr unsigned nz_tr(unsigned m) {
  unsigned t = 0;
  for (int r = 0; r < 3; r++)
    for (int c = 0; c < 3; c++)
      if ((m >> (r * 3 + c)) & 1u) t |= 1u << (c * 3 + r);
  return t;
}

// a0 b0 + a1 b1 + a2 b2 over the terms present (p0, p1, p2), rounded as
// mm3 and mv3 round the full sum under FMA contraction,
// fma(a2, b2, fma(a0, b0, a1 b1)): dropping a term whose factor is zero
// leaves every finite result unchanged.
__device__ __forceinline__ double dot3m(bool p0, bool p1, bool p2, double a0, double b0, double a1,
                                        double b1, double a2, double b2) {
  double s = 0.0;
  if (p1) s = a1 * b1;
  if (p0) s = p1 ? __builtin_fma(a0, b0, s) : a0 * b0;
  if (p2) s = (p0 || p1) ? __builtin_fma(a2, b2, s) : a2 * b2;
  return s;
}
// C = A * B (3x3) for A, B with the structural non-zeros MA, MB
template <unsigned MA, unsigned MB>
__device__ __forceinline__ void mm3m(const double *A, const double *B, double *C) {
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int c = 0; c < 3; c++)
      C[r * 3 + c] = dot3m((MA >> (r * 3)) & (MB >> c) & 1u, (MA >> (r * 3 + 1)) & (MB >> (3 + c)) & 1u,
                           (MA >> (r * 3 + 2)) & (MB >> (6 + c)) & 1u, A[r * 3], B[c], A[r * 3 + 1],
                           B[3 + c], A[r * 3 + 2], B[6 + c]);
}
// y = A * x for A with the structural non-zeros MA
template <unsigned MA>
__device__ __forceinline__ void mv3m(const double *A, const double *x, double *y) {
#pragma unroll
  for (int r = 0; r < 3; r++)
    y[r] = dot3m((MA >> (r * 3)) & 1u, (MA >> (r * 3 + 1)) & 1u, (MA >> (r * 3 + 2)) & 1u, A[r * 3], x[0],
                 A[r * 3 + 1], x[1], A[r * 3 + 2], x[2]);
}

// ------------------------------------------------------------------ lines --

// number of lines per family: block, scalar A, scalar B
struct Families {
  int nb, na, nbb, n, cyclic;
};

__host__ __device__ inline Families families(const Geo &g, int d) {
  Families f;
  const int nkf = g.periodic ? g.np : g.np - 1; // interior phi faces
  if (d == 0) { f.nb = g.nt * g.np; f.na = (g.nt - 1) * g.np; f.nbb = g.nt * nkf; f.n = g.nr; }
  else if (d == 1) { f.nb = g.nr * g.np; f.na = (g.nr - 1) * g.np; f.nbb = g.nr * nkf; f.n = g.nt; }
  else { f.nb = g.nr * g.nt; f.na = (g.nr - 1) * g.nt; f.nbb = g.nr * (g.nt - 1); f.n = g.np; }
  f.cyclic = (d == 2 && g.periodic) ? 1 : 0;
  return f;
}

// ------------------------------------------------------------ block rows --

// Assemble block row s of (I + tau/2 D_d) on block line (a, b).  hs = tau/2.
// Unknown order within a block: p, T, w.
template <int D, class S>
__device__ __forceinline__ void block_row(const Geo &g, const Mat &m, const S &u, const Fields &rhs, int a,
                          int b, int s, int n, int cyc, double hs, BRow &R, Edge *e = nullptr) {
  int i, j, k;
  if (D == 0) { i = s; j = a; k = b; }
  else if (D == 1) { i = a; j = s; k = b; }
  else { i = a; j = b; k = s; }
  Cent c;
  centre(g, m, u, i, j, k, c);
  const double ir = g.irc[i], is = g.isc[j], ir2 = ir * ir;
  double adv, dp_, dm_, ap, am, lp, lm;
  if (D == 0) {
    adv = c.ur * (0.5 * g.idr);
    dp_ = g.rf[i + 1] * g.rf[i + 1] * (ir2 * g.idr);
    dm_ = -g.rf[i] * g.rf[i] * (ir2 * g.idr);
    const double gg = (c.Gtt + c.Gff) * ir;
    ap = m.mu * (2.0 * c.Grr * g.idr + gg - (2.0 / 3.0) * c.tr * dp_);
    am = m.mu * (-2.0 * c.Grr * g.idr + gg - (2.0 / 3.0) * c.tr * dm_);
    lp = g.rf[i + 1] * g.rf[i + 1] * (ir2 * g.idr * g.idr);
    lm = g.rf[i] * g.rf[i] * (ir2 * g.idr * g.idr);
  } else if (D == 1) {
    const double ct = g.ctc[j];
    adv = c.ut * (0.5 * ir * g.idt);
    dp_ = g.sf[j + 1] * (ir * is * g.idt);
    dm_ = -g.sf[j] * (ir * is * g.idt);
    const double gg = c.Gff * ct * ir - 0.5 * c.Srt * ir;
    ap = m.mu * (2.0 * c.Gtt * (ir * g.idt) + gg - (2.0 / 3.0) * c.tr * dp_);
    am = m.mu * (-2.0 * c.Gtt * (ir * g.idt) + gg - (2.0 / 3.0) * c.tr * dm_);
    lp = g.sf[j + 1] * (ir2 * is * g.idt * g.idt);
    lm = g.sf[j] * (ir2 * is * g.idt * g.idt);
  } else {
    const double ct = g.ctc[j];
    adv = c.uf * (0.5 * ir * is * g.idp);
    dp_ = ir * is * g.idp;
    dm_ = -dp_;
    const double gg = -0.5 * (c.Srf + c.Stf * ct) * ir;
    ap = m.mu * (2.0 * c.Gff * dp_ + gg - (2.0 / 3.0) * c.tr * dp_);
    am = m.mu * (-2.0 * c.Gff * dp_ + gg - (2.0 / 3.0) * c.tr * dm_);
    lp = ir2 * is * is * g.idp * g.idp;
    lm = lp;
  }
  const bool first = !cyc && s == 0, last = !cyc && s == n - 1;
  if (first) lm = 0.0; // zero flux through the boundary (copy ghost)
  if (last) lp = 0.0;
  const double g1 = m.gam - 1.0;
  const double kp = g1 * m.kap, kT = c.chi * m.kap;
#pragma unroll
  for (int q = 0; q < 9; q++) { R.L[q] = 0.0; R.D[q] = 0.0; R.U[q] = 0.0; }
  // p row
  R.L[0] = -adv; R.U[0] = adv;
  R.L[1] = -kp * lm; R.D[1] = kp * (lp + lm); R.U[1] = -kp * lp;
  R.L[2] = m.gam * c.P * dm_ - g1 * am;
  R.D[2] = m.gam * c.P * dp_ - g1 * ap;
  // T row
  R.L[4] = -adv - kT * lm; R.D[4] = kT * (lp + lm); R.U[4] = adv - kT * lp;
  R.L[5] = g1 * c.T * dm_ - c.chi * am;
  R.D[5] = g1 * c.T * dp_ - c.chi * ap;
  if (first) { R.D[0] += R.L[0]; R.D[4] += -adv; } // advection ghost p_{-1} = p_0
  if (last) { R.D[0] += R.U[0]; R.U[0] = 0.0; R.D[4] += adv; R.U[4] = 0.0; }
  if (first) { R.L[0] = 0.0; R.L[4] = 0.0; }
  // w row (face after cell s)
  const bool w_unknown = cyc || s < n - 1;
  double gp = 0.0, cm = 0.0, c0 = 0.0, cp = 0.0;
  if (w_unknown) {
    if (D == 0) {
      const int f = i + 1;
      const double irho = irho_mean(g, m, u, i, j, k, i + 1, j, k);
      const double nu = m.mu * irho, un = u.ld(F_UR, idx_r(g, f, j, k));
      const double irF2 = g.irf[f] * g.irf[f], d2 = g.idr * g.idr, rF2 = g.rf[f] * g.rf[f];
      const double ra2 = g.rc[i] * g.rc[i], rb2 = g.rc[i + 1] * g.rc[i + 1];
      const double ira2 = g.irc[i] * g.irc[i], irb2 = g.irc[i + 1] * g.irc[i + 1];
      gp = irho * g.idr;
      cp = un * (0.5 * g.idr) - nu * rb2 * irF2 * d2 - nu * (1.0 / 3.0) * g.rf[i + 2] * g.rf[i + 2] * irb2 * d2;
      c0 = nu * (rb2 + ra2) * irF2 * d2 + nu * (1.0 / 3.0) * rF2 * (irb2 + ira2) * d2;
      cm = -un * (0.5 * g.idr) - nu * ra2 * irF2 * d2 - nu * (1.0 / 3.0) * g.rf[i] * g.rf[i] * ira2 * d2;
    } else if (D == 1) {
      const int f = j + 1;
      const double irho = irho_mean(g, m, u, i, j, k, i, j + 1, k);
      const double nu = m.mu * irho, un = u.ld(F_UT, idx_t(g, i, f, k));
      const double sF = g.sf[f], isF = g.isf[f], r2d2 = ir2 * g.idt * g.idt;
      const double sa = g.sc[j], sb = g.sc[j + 1], isa = g.isc[j], isb = g.isc[j + 1];
      gp = irho * ir * g.idt;
      cp = un * (0.5 * ir * g.idt) - nu * sb * r2d2 * isF - nu * (1.0 / 3.0) * g.sf[j + 2] * r2d2 * isb;
      c0 = nu * (sb + sa) * r2d2 * isF + nu * (1.0 / 3.0) * sF * (isb + isa) * r2d2;
      cm = -un * (0.5 * ir * g.idt) - nu * sa * r2d2 * isF - nu * (1.0 / 3.0) * g.sf[j] * r2d2 * isa;
    } else {
      const int f = g.periodic ? wrapk(g, k + 1) : k + 1;
      const double irho = irho_mean(g, m, u, i, j, k, i, j, k + 1);
      const double nu = m.mu * irho, un = u.ld(F_UF, idx_f(g, i, j, f));
      const double q2 = ir2 * is * is * g.idp * g.idp;
      gp = irho * ir * is * g.idp;
      cp = un * (0.5 * ir * is * g.idp) - nu * (4.0 / 3.0) * q2;
      c0 = nu * (8.0 / 3.0) * q2;
      cm = -un * (0.5 * ir * is * g.idp) - nu * (4.0 / 3.0) * q2;
    }
    R.D[6] = -gp; R.U[6] = gp;
    R.L[8] = cm; R.D[8] = c0; R.U[8] = cp;
    if (e && !cyc && s == n - 2) e->hiw = hs * cp;
    if (!cyc && s == n - 2) R.U[8] = 0.0; // w_{s+1} is the boundary face
  }
  if (e && !w_unknown) { e->hi[0] = hs * R.D[2]; e->hi[1] = hs * R.D[5]; }
  if (!w_unknown) { R.D[2] = 0.0; R.D[5] = 0.0; } // w_{n-1} is the boundary face
  if (e && first) { e->lo[0] = hs * R.L[2]; e->lo[1] = hs * R.L[5]; e->lo[2] = hs * R.L[8]; }
  if (first) { // no row before the first one: the L block couples to nothing
#pragma unroll
    for (int q = 0; q < 9; q++) R.L[q] = 0.0;
  }
  // scale and add the identity
#pragma unroll
  for (int q = 0; q < 9; q++) { R.L[q] *= hs; R.D[q] *= hs; R.U[q] *= hs; }
  R.D[0] += 1.0; R.D[4] += 1.0; R.D[8] += 1.0;
  if (!w_unknown) { R.L[6] = R.L[7] = R.L[8] = 0.0; R.D[6] = R.D[7] = 0.0; R.D[8] = 1.0; R.U[6] = R.U[7] = R.U[8] = 0.0; }
  // right-hand side
  const long xc = idx_c(g, i, j, k);
  R.b[0] = rhs.p[xc];
  R.b[1] = rhs.T[xc];
  if (w_unknown) {
    if (D == 0) R.b[2] = rhs.ur[idx_r(g, i + 1, j, k)];
    else if (D == 1) R.b[2] = rhs.ut[idx_t(g, i, j + 1, k)];
    else R.b[2] = rhs.uf[idx_f(g, i, j, g.periodic ? wrapk(g, k + 1) : k + 1)];
  } else {
    R.b[2] = 0.0;
  }
}

// ----------------------------------------------------------- scalar rows --

struct SRow {
  double a, b, c, r;
};

// Scalar line of family FAM (0: A, 1: B) in direction D, transverse coords
// (a, b); row s.  Ghost folding at non-cyclic ends: walls -1, poles (u_r
// along theta) +1.
template <int D, int FAM, class S>
__device__ __forceinline__ void scalar_row(const Geo &g, const Mat &m, const S &u, const Fields &rhs, int a,
                           int b, int s, int n, int cyc, double hs, SRow &R, long &xi,
                           double *&arr, Edge *e = nullptr) {
  double ca, cb, cc_, sglo = -1.0, sghi = -1.0;
  if (D == 0) {
    const int i = s;
    const double ir = g.irc[i], r2d2 = ir * ir * g.idr * g.idr;
    double ua, irho;
    if (FAM == 0) { // u_theta at theta-face (jf, k)
      const int jf = a, k = b;
      ua = 0.25 * (u.ld(F_UR, idx_r(g, i, jf - 1, k)) + u.ld(F_UR, idx_r(g, i, jf, k)) +
                   u.ld(F_UR, idx_r(g, i + 1, jf - 1, k)) + u.ld(F_UR, idx_r(g, i + 1, jf, k)));
      irho = irho_mean(g, m, u, i, jf - 1, k, i, jf, k);
      xi = idx_t(g, i, jf, k); arr = rhs.ut;
    } else { // u_phi at phi-face (j, kf)
      const int j = a, kf = b;
      const int k0 = g.periodic ? wrapk(g, kf - 1) : kf - 1, k1 = g.periodic ? wrapk(g, kf) : kf;
      ua = 0.25 * (u.ld(F_UR, idx_r(g, i, j, k0)) + u.ld(F_UR, idx_r(g, i, j, k1)) +
                   u.ld(F_UR, idx_r(g, i + 1, j, k0)) + u.ld(F_UR, idx_r(g, i + 1, j, k1)));
      irho = irho_mean(g, m, u, i, j, k0, i, j, k1);
      xi = idx_f(g, i, j, kf); arr = rhs.uf;
    }
    const double nu = m.mu * irho;
    const double fp = g.rf[i + 1] * g.rf[i + 1], fm = g.rf[i] * g.rf[i];
    ca = -ua * (0.5 * g.idr) - nu * fm * r2d2;
    cb = nu * (fp + fm) * r2d2;
    cc_ = ua * (0.5 * g.idr) - nu * fp * r2d2;
  } else if (D == 1) {
    const int j = s;
    const double is = g.isc[j];
    double ua, irho, irr;
    if (FAM == 0) { // u_r at r-face (fr, k)
      const int fr = a, k = b;
      irr = g.irf[fr];
      ua = 0.25 * (u.ld(F_UT, idx_t(g, fr - 1, j, k)) + u.ld(F_UT, idx_t(g, fr - 1, j + 1, k)) +
                   u.ld(F_UT, idx_t(g, fr, j, k)) + u.ld(F_UT, idx_t(g, fr, j + 1, k)));
      irho = irho_mean(g, m, u, fr - 1, j, k, fr, j, k);
      xi = idx_r(g, fr, j, k); arr = rhs.ur;
      sglo = g.pole_lo ? 1.0 : -1.0;
      sghi = g.pole_hi ? 1.0 : -1.0;
    } else { // u_phi at phi-face (i, kf)
      const int i = a, kf = b;
      irr = g.irc[i];
      const int k0 = g.periodic ? wrapk(g, kf - 1) : kf - 1, k1 = g.periodic ? wrapk(g, kf) : kf;
      ua = 0.25 * (u.ld(F_UT, idx_t(g, i, j, k0)) + u.ld(F_UT, idx_t(g, i, j, k1)) +
                   u.ld(F_UT, idx_t(g, i, j + 1, k0)) + u.ld(F_UT, idx_t(g, i, j + 1, k1)));
      irho = irho_mean(g, m, u, i, j, k0, i, j, k1);
      xi = idx_f(g, i, j, kf); arr = rhs.uf;
    }
    const double nu = m.mu * irho, q = irr * irr * is * g.idt * g.idt;
    ca = -ua * (0.5 * irr * g.idt) - nu * g.sf[j] * q;
    cb = nu * (g.sf[j + 1] + g.sf[j]) * q;
    cc_ = ua * (0.5 * irr * g.idt) - nu * g.sf[j + 1] * q;
  } else {
    const int k = s;
    double ua, irho, irr, iss;
    if (FAM == 0) { // u_r at r-face (fr, j)
      const int fr = a, j = b;
      irr = g.irf[fr]; iss = g.isc[j];
      const int kp = g.periodic ? wrapk(g, k + 1) : k + 1;
      ua = 0.25 * (u.ld(F_UF, idx_f(g, fr - 1, j, k)) + u.ld(F_UF, idx_f(g, fr - 1, j, kp)) +
                   u.ld(F_UF, idx_f(g, fr, j, k)) + u.ld(F_UF, idx_f(g, fr, j, kp)));
      irho = irho_mean(g, m, u, fr - 1, j, k, fr, j, k);
      xi = idx_r(g, fr, j, k); arr = rhs.ur;
    } else { // u_theta at theta-face (i, ft)
      const int i = a, ft = b;
      irr = g.irc[i]; iss = g.isf[ft];
      const int kp = g.periodic ? wrapk(g, k + 1) : k + 1;
      ua = 0.25 * (u.ld(F_UF, idx_f(g, i, ft - 1, k)) + u.ld(F_UF, idx_f(g, i, ft - 1, kp)) +
                   u.ld(F_UF, idx_f(g, i, ft, k)) + u.ld(F_UF, idx_f(g, i, ft, kp)));
      irho = irho_mean(g, m, u, i, ft - 1, k, i, ft, k);
      xi = idx_t(g, i, ft, k); arr = rhs.ut;
    }
    const double nu = m.mu * irho, q = irr * irr * iss * iss * g.idp * g.idp;
    ca = -ua * (0.5 * irr * iss * g.idp) - nu * q;
    cb = 2.0 * nu * q;
    cc_ = ua * (0.5 * irr * iss * g.idp) - nu * q;
  }
  if (e && !cyc && s == 0) e->slo = hs * ca;
  if (e && !cyc && s == n - 1) e->shi = hs * cc_;
  if (!cyc && s == 0) { cb += sglo * ca; ca = 0.0; }
  if (!cyc && s == n - 1) { cb += sghi * cc_; cc_ = 0.0; }
  R.a = hs * ca;
  R.b = 1.0 + hs * cb;
  R.c = hs * cc_;
  R.r = arr[xi];
}


// Forward elimination of one chunk of a scalar line (partitioned solvers):
// rows a0 .. a0 + len - 2 with the left spike, x_q = Y_q - C_q x_{q+1} -
// E_q x_left, and the chunk's last row (the separator) into S.  Every row of
// the chunk is assembled first, without a branch (rows past the chunk's end
// repeat its last row, clamped into the line; their results are not used),
// so that the loads of all its rows are in flight together: a row assembled
// under a branch on the chunk length waits for the previous row's
// elimination before its loads issue.  row(s, R) assembles row s.  Returns
// whether an eliminated row had a zero pivot.
template <int PM, class RowFn>
__device__ __forceinline__ bool scalar_chunk_fwd(const RowFn &row, int a0, int len, int n, double *Cm,
                                                 double *Em, double *Ym, SRow &S) {
  const int rl = min(a0 + max(len - 1, 0), n - 1);
  SRow R[PM];
#pragma unroll
  for (int q = 0; q < PM; q++) row(min(a0 + q, rl), R[q]);
  bool sing = false;
#pragma unroll
  for (int q = 0; q < PM - 1; q++) {
    double dp = R[q].b, rr = R[q].r, lx = R[q].a;
    if (q > 0) { dp -= R[q].a * Cm[q - 1]; rr -= R[q].a * Ym[q - 1]; lx = -R[q].a * Em[q - 1]; }
    sing |= q < len - 1 && !(dp != 0.0);
    const double id = rcp_nr(dp);
    Cm[q] = R[q].c * id;
    Ym[q] = rr * id;
    Em[q] = lx * id;
  }
#pragma unroll
  for (int q = 0; q < PM; q++)
    if (q == len - 1) S = R[q];
  return sing;
}

// Row s of the line system, or of its transpose (TR): the transposed row s
// has lower block U_{s-1}^T, diagonal D_s^T and upper block L_{s+1}^T, and
// the right-hand side read at row s's unknowns.
__device__ __forceinline__ void tr3(const double *A, double *B) {
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int c = 0; c < 3; c++) B[c * 3 + r] = A[r * 3 + c];
}

template <int D, bool TR>
__device__ __forceinline__ void get_brow(const Geo &g, const Mat &m, const SrcOne &u,
                                         const Fields &rhs, int a, int b, int s, int n, int cyc,
                                         double hs, BRow &R) {
  block_row<D>(g, m, u, rhs, a, b, s, n, cyc, hs, R);
  if (!TR) return;
  double t9[9];
  tr3(R.D, t9);
#pragma unroll
  for (int q = 0; q < 9; q++) R.D[q] = t9[q];
  const bool has_m = cyc || s > 0, has_p = cyc || s < n - 1;
  BRow Q;
  if (has_m) {
    block_row<D>(g, m, u, rhs, a, b, s > 0 ? s - 1 : n - 1, n, cyc, hs, Q);
    tr3(Q.U, R.L);
  } else {
#pragma unroll
    for (int q = 0; q < 9; q++) R.L[q] = 0.0;
  }
  if (has_p) {
    block_row<D>(g, m, u, rhs, a, b, s < n - 1 ? s + 1 : 0, n, cyc, hs, Q);
    tr3(Q.L, R.U);
  } else {
#pragma unroll
    for (int q = 0; q < 9; q++) R.U[q] = 0.0;
  }
}

// The rows of the transposed line in increasing order s0, s0 + 1, ...,
// assembling each row of the line once: the walker keeps U_{s-1}, D_s, U_s
// and b_s, and next() assembles row s + 1 for L_{s+1}.
template <int D>
struct TrWalk {
  double Up[9], Dc[9], Uc[9], bc[3];
  int s;
  __device__ __forceinline__ void init(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                       int a, int b, int s0, int n, int cyc, double hs) {
    BRow R;
    if (cyc || s0 > 0) {
      block_row<D>(g, m, u, rhs, a, b, s0 > 0 ? s0 - 1 : n - 1, n, cyc, hs, R);
#pragma unroll
      for (int q = 0; q < 9; q++) Up[q] = R.U[q];
    } else {
#pragma unroll
      for (int q = 0; q < 9; q++) Up[q] = 0.0;
    }
    block_row<D>(g, m, u, rhs, a, b, s0, n, cyc, hs, R);
#pragma unroll
    for (int q = 0; q < 9; q++) { Dc[q] = R.D[q]; Uc[q] = R.U[q]; }
#pragma unroll
    for (int q = 0; q < 3; q++) bc[q] = R.b[q];
    s = s0;
  }
  // transposed row s into T, then advance to s + 1
  __device__ __forceinline__ void next(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                       int a, int b, int n, int cyc, double hs, BRow &T) {
    BRow R;
    const bool has_p = cyc || s < n - 1;
    if (has_p) {
      block_row<D>(g, m, u, rhs, a, b, s < n - 1 ? s + 1 : 0, n, cyc, hs, R);
    } else {
#pragma unroll
      for (int q = 0; q < 9; q++) { R.L[q] = 0.0; R.D[q] = 0.0; R.U[q] = 0.0; }
#pragma unroll
      for (int q = 0; q < 3; q++) R.b[q] = 0.0;
    }
    tr3(Up, T.L);
    tr3(Dc, T.D);
    tr3(R.L, T.U);
#pragma unroll
    for (int q = 0; q < 3; q++) T.b[q] = bc[q];
#pragma unroll
    for (int q = 0; q < 9; q++) { Up[q] = Uc[q]; Dc[q] = R.D[q]; Uc[q] = R.U[q]; }
#pragma unroll
    for (int q = 0; q < 3; q++) bc[q] = R.b[q];
    s++;
  }
};

template <int D, int FAM, bool TR>
__device__ __forceinline__ void get_srow(const Geo &g, const Mat &m, const SrcOne &u,
                                         const Fields &rhs, int a, int b, int s, int n, int cyc,
                                         double hs, SRow &R, long &xi, double *&arr) {
  scalar_row<D, FAM>(g, m, u, rhs, a, b, s, n, cyc, hs, R, xi, arr);
  if (!TR) return;
  SRow Q;
  long xq;
  double *aq;
  double lo = 0.0, up = 0.0;
  if (cyc || s > 0) {
    scalar_row<D, FAM>(g, m, u, rhs, a, b, s > 0 ? s - 1 : n - 1, n, cyc, hs, Q, xq, aq);
    lo = Q.c;
  }
  if (cyc || s < n - 1) {
    scalar_row<D, FAM>(g, m, u, rhs, a, b, s < n - 1 ? s + 1 : 0, n, cyc, hs, Q, xq, aq);
    up = Q.a;
  }
  R.a = lo;
  R.c = up;
}

// The scalar counterpart of TrWalk: transposed row s is (c_{s-1}, b_s,
// a_{s+1}) with the right-hand side r_s.
template <int D, int FAM>
struct TrWalkS {
  double cp, bc, cc, rc;
  int s;
  __device__ __forceinline__ void init(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                       int a, int b, int s0, int n, int cyc, double hs) {
    SRow Q;
    long xq;
    double *aq;
    cp = 0.0;
    if (cyc || s0 > 0) {
      scalar_row<D, FAM>(g, m, u, rhs, a, b, s0 > 0 ? s0 - 1 : n - 1, n, cyc, hs, Q, xq, aq);
      cp = Q.c;
    }
    scalar_row<D, FAM>(g, m, u, rhs, a, b, s0, n, cyc, hs, Q, xq, aq);
    bc = Q.b; cc = Q.c; rc = Q.r;
    s = s0;
  }
  __device__ __forceinline__ void next(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                       int a, int b, int n, int cyc, double hs, SRow &T) {
    SRow Q{0.0, 0.0, 0.0, 0.0};
    long xq;
    double *aq;
    if (cyc || s < n - 1) scalar_row<D, FAM>(g, m, u, rhs, a, b, s < n - 1 ? s + 1 : 0, n, cyc, hs, Q, xq, aq);
    T.a = cp; T.b = bc; T.c = Q.a; T.r = rc;
    cp = cc; bc = Q.b; cc = Q.c; rc = Q.r;
    s++;
  }
};

__device__ __forceinline__ double *fsel(const Fields &f, int fid) {
  return fid == F_P ? f.p : fid == F_UR ? f.ur : fid == F_UT ? f.ut : fid == F_UF ? f.uf : f.T;
}

// store one solution value at (field, flat index) according to the sweep's
// destination mode
__device__ __forceinline__ void put(const Out &o, int fid, long idx, double v) {
  if (o.mode == 0) {
    fsel(o.x, fid)[idx] = v;
    return;
  }
  const double nv = fsel(o.base, fid)[idx] + v;
  fsel(o.x, fid)[idx] = nv;
  if (o.ub.p) fsel(o.ub, fid)[idx] = 0.5 * (nv + fsel(o.un, fid)[idx]);
  if (o.raw.p) fsel(o.raw, fid)[idx] = v;
}

template <int D>
__device__ __forceinline__ void block_store(const Geo &g, const Out &o, int a, int b, int s,
                                            const double *v) {
  int i, j, k;
  if (D == 0) { i = s; j = a; k = b; }
  else if (D == 1) { i = a; j = s; k = b; }
  else { i = a; j = b; k = s; }
  const long xc = idx_c(g, i, j, k);
  put(o, F_P, xc, v[0]);
  put(o, F_T, xc, v[1]);
  if (D == 0) put(o, F_UR, idx_r(g, i + 1, j, k), v[2]);
  else if (D == 1) put(o, F_UT, idx_t(g, i, j + 1, k), v[2]);
  else put(o, F_UF, idx_f(g, i, j, g.periodic ? wrapk(g, k + 1) : k + 1), v[2]);
}

// zero the boundary-normal faces of x that no line of this sweep writes:
// every block line owns a short piece of them
template <int D>
__device__ __forceinline__ void zero_bnd(const Geo &g, const Fields &x, int a, int b) {
  if (D == 0) { // line (j,k): ur faces 0 (nr written as last block); ut faces 0/nt; uf faces 0/np
    const int j = a, k = b;
    x.ur[idx_r(g, 0, j, k)] = 0.0;
    for (int i = 0; i < g.nr; i++) {
      if (j == 0) x.ut[idx_t(g, i, 0, k)] = 0.0;
      if (j == g.nt - 1) x.ut[idx_t(g, i, g.nt, k)] = 0.0;
      if (!g.periodic && k == 0) x.uf[idx_f(g, i, j, 0)] = 0.0;
      if (!g.periodic && k == g.np - 1) x.uf[idx_f(g, i, j, g.np)] = 0.0;
    }
  } else if (D == 1) { // line (i,k)
    const int i = a, k = b;
    x.ut[idx_t(g, i, 0, k)] = 0.0;
    for (int j = 0; j < g.nt; j++) {
      if (i == 0) x.ur[idx_r(g, 0, j, k)] = 0.0;
      if (i == g.nr - 1) x.ur[idx_r(g, g.nr, j, k)] = 0.0;
      if (!g.periodic && k == 0) x.uf[idx_f(g, i, j, 0)] = 0.0;
      if (!g.periodic && k == g.np - 1) x.uf[idx_f(g, i, j, g.np)] = 0.0;
    }
  } else { // line (i,j)
    const int i = a, j = b;
    if (!g.periodic) x.uf[idx_f(g, i, j, 0)] = 0.0;
    for (int k = 0; k < g.np; k++) {
      if (i == 0) x.ur[idx_r(g, 0, j, k)] = 0.0;
      if (i == g.nr - 1) x.ur[idx_r(g, g.nr, j, k)] = 0.0;
      if (j == 0) x.ut[idx_t(g, i, 0, k)] = 0.0;
      if (j == g.nt - 1) x.ut[idx_t(g, i, g.nt, k)] = 0.0;
    }
  }
}

template <int D, int FAM>
__device__ __forceinline__ long scalar_index(const Geo &g, int a, int b, int s) {
  if (D == 0) return FAM == 0 ? idx_t(g, s, a, b) : idx_f(g, s, a, b);
  if (D == 1) return FAM == 0 ? idx_r(g, a, s, b) : idx_f(g, a, s, b);
  return FAM == 0 ? idx_r(g, a, b, s) : idx_t(g, a, b, s);
}

} // namespace dsw
