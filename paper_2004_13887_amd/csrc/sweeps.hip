// sweeps.hip -- the three one-dimensional implicit sweeps of the split step
// (paper eqs. (spl1), (spl2), (spl3)):  (I + tau/2 D_d(Ubar)) x = rhs.
//
// In sweep direction d every line carries
//   * one 3x3-block tridiagonal system in (p_s, T_s, w_s), w_s the velocity
//     component normal to the d-faces on the face after cell s (rows of
//     D_r / D_theta / D_phi, Appendix B eqs. (dr)-(dphi): A1^d, A2^d, A3^d,
//     B1^d, B2^{d,d}, C2^d, C3^d), and
//   * one scalar tridiagonal system per transverse velocity component
//     (B2^{d,c}, c != d).
// The matrix rows are assembled on the fly from the midpoint state and solved
// with the block Thomas algorithm (no pivoting between blocks; the paper's
// end of section 2); lines that close on themselves (phi on the full sphere)
// use bordered elimination of the last block.
//
// One thread per line.  Forward-elimination intermediates go to a scratch
// array laid out [position][quantity][line] so that a wavefront's accesses
// are contiguous across lines.
#include "dsw_common.hpp"
#include "dsw_internal.hpp"

namespace dsw {

struct BRow {
  double L[9], D[9], U[9], b[3];
};

__device__ __forceinline__ void inv3(const double *A, double *X, int *status) {
  const double c00 = A[4] * A[8] - A[5] * A[7];
  const double c01 = A[5] * A[6] - A[3] * A[8];
  const double c02 = A[3] * A[7] - A[4] * A[6];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  if (!(det != 0.0) || !isfinite(det)) status[ST_SINGULAR] = 1;
  const double id = 1.0 / det;
  X[0] = c00 * id;
  X[1] = (A[2] * A[7] - A[1] * A[8]) * id;
  X[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  X[3] = c01 * id;
  X[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  X[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  X[6] = c02 * id;
  X[7] = (A[1] * A[6] - A[0] * A[7]) * id;
  X[8] = (A[0] * A[4] - A[1] * A[3]) * id;
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
template <int D>
__device__ void block_row(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs, int a,
                          int b, int s, int n, int cyc, double hs, BRow &R) {
  int i, j, k;
  if (D == 0) { i = s; j = a; k = b; }
  else if (D == 1) { i = a; j = s; k = b; }
  else { i = a; j = b; k = s; }
  Cent c;
  centre(g, m, u, i, j, k, c);
  const double r = g.rc[i], sn = g.sc[j];
  double adv, dp_, dm_, ap, am, lp, lm;
  if (D == 0) {
    adv = c.ur / (2.0 * g.dr);
    dp_ = g.rf[i + 1] * g.rf[i + 1] / (r * r * g.dr);
    dm_ = -g.rf[i] * g.rf[i] / (r * r * g.dr);
    const double gg = (c.Gtt + c.Gff) / r;
    ap = m.mu * (2.0 * c.Grr / g.dr + gg - (2.0 / 3.0) * c.tr * dp_);
    am = m.mu * (-2.0 * c.Grr / g.dr + gg - (2.0 / 3.0) * c.tr * dm_);
    lp = g.rf[i + 1] * g.rf[i + 1] / (r * r * g.dr * g.dr);
    lm = g.rf[i] * g.rf[i] / (r * r * g.dr * g.dr);
  } else if (D == 1) {
    const double ct = g.cc[j] / sn;
    adv = c.ut / (r * 2.0 * g.dt);
    dp_ = g.sf[j + 1] / (r * sn * g.dt);
    dm_ = -g.sf[j] / (r * sn * g.dt);
    const double gg = c.Gff * ct / r - 0.5 * c.Srt / r;
    ap = m.mu * (2.0 * c.Gtt / (r * g.dt) + gg - (2.0 / 3.0) * c.tr * dp_);
    am = m.mu * (-2.0 * c.Gtt / (r * g.dt) + gg - (2.0 / 3.0) * c.tr * dm_);
    lp = g.sf[j + 1] / (r * r * sn * g.dt * g.dt);
    lm = g.sf[j] / (r * r * sn * g.dt * g.dt);
  } else {
    const double ct = g.cc[j] / sn;
    adv = c.uf / (r * sn * 2.0 * g.dp);
    dp_ = 1.0 / (r * sn * g.dp);
    dm_ = -1.0 / (r * sn * g.dp);
    const double gg = -0.5 * (c.Srf + c.Stf * ct) / r;
    ap = m.mu * (2.0 * c.Gff / (r * sn * g.dp) + gg - (2.0 / 3.0) * c.tr * dp_);
    am = m.mu * (-2.0 * c.Gff / (r * sn * g.dp) + gg - (2.0 / 3.0) * c.tr * dm_);
    lp = 1.0 / (r * r * sn * sn * g.dp * g.dp);
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
      const double rho = 0.5 * (rho_at(g, m, u, i, j, k) + rho_at(g, m, u, i + 1, j, k));
      const double nu = m.mu / rho, un = u.ld(F_UR, idx_r(g, f, j, k));
      const double rF2 = g.rf[f] * g.rf[f], d2 = g.dr * g.dr;
      const double ra2 = g.rc[i] * g.rc[i], rb2 = g.rc[i + 1] * g.rc[i + 1];
      gp = 1.0 / (rho * g.dr);
      cp = un / (2.0 * g.dr) - nu * rb2 / (rF2 * d2) - nu / 3.0 * g.rf[i + 2] * g.rf[i + 2] / (rb2 * d2);
      c0 = nu * (rb2 + ra2) / (rF2 * d2) + nu / 3.0 * rF2 * (1.0 / rb2 + 1.0 / ra2) / d2;
      cm = -un / (2.0 * g.dr) - nu * ra2 / (rF2 * d2) - nu / 3.0 * g.rf[i] * g.rf[i] / (ra2 * d2);
    } else if (D == 1) {
      const int f = j + 1;
      const double rho = 0.5 * (rho_at(g, m, u, i, j, k) + rho_at(g, m, u, i, j + 1, k));
      const double nu = m.mu / rho, un = u.ld(F_UT, idx_t(g, i, f, k));
      const double sF = g.sf[f], r2d2 = r * r * g.dt * g.dt;
      const double sa = g.sc[j], sb = g.sc[j + 1];
      gp = 1.0 / (rho * r * g.dt);
      cp = un / (2.0 * r * g.dt) - nu * sb / (r2d2 * sF) - nu / 3.0 * g.sf[j + 2] / (r2d2 * sb);
      c0 = nu * (sb + sa) / (r2d2 * sF) + nu / 3.0 * sF * (1.0 / sb + 1.0 / sa) / r2d2;
      cm = -un / (2.0 * r * g.dt) - nu * sa / (r2d2 * sF) - nu / 3.0 * g.sf[j] / (r2d2 * sa);
    } else {
      const int f = g.periodic ? wrapk(g, k + 1) : k + 1;
      const double rho = 0.5 * (rho_at(g, m, u, i, j, k) + rho_at(g, m, u, i, j, k + 1));
      const double nu = m.mu / rho, un = u.ld(F_UF, idx_f(g, i, j, f));
      const double q2 = r * r * sn * sn * g.dp * g.dp;
      gp = 1.0 / (rho * r * sn * g.dp);
      cp = un / (2.0 * r * sn * g.dp) - 4.0 * nu / 3.0 / q2;
      c0 = 8.0 * nu / 3.0 / q2;
      cm = -un / (2.0 * r * sn * g.dp) - 4.0 * nu / 3.0 / q2;
    }
    R.D[6] = -gp; R.U[6] = gp;
    R.L[8] = cm; R.D[8] = c0; R.U[8] = cp;
    if (!cyc && s == n - 2) R.U[8] = 0.0; // w_{s+1} is the boundary face
  }
  if (!w_unknown) { R.D[2] = 0.0; R.D[5] = 0.0; } // w_{n-1} is the boundary face
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

template <int D>
__device__ __forceinline__ void block_store(const Geo &g, const Fields &x, int a, int b, int s,
                                            const double *v, bool accum) {
  int i, j, k;
  if (D == 0) { i = s; j = a; k = b; }
  else if (D == 1) { i = a; j = s; k = b; }
  else { i = a; j = b; k = s; }
  const long xc = idx_c(g, i, j, k);
  long xw;
  double *w;
  if (D == 0) { xw = idx_r(g, i + 1, j, k); w = x.ur; }
  else if (D == 1) { xw = idx_t(g, i, j + 1, k); w = x.ut; }
  else { xw = idx_f(g, i, j, g.periodic ? wrapk(g, k + 1) : k + 1); w = x.uf; }
  if (accum) {
    x.p[xc] += v[0];
    x.T[xc] += v[1];
    w[xw] += v[2];
  } else {
    x.p[xc] = v[0];
    x.T[xc] = v[1];
    w[xw] = v[2];
  }
}

// zero the boundary-normal faces of x that no line of this sweep writes:
// every block line owns a short piece of them
template <int D>
__device__ void zero_bnd(const Geo &g, const Fields &x, int a, int b) {
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

template <int D>
__device__ void solve_block_line(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                 const Fields &x, double *sc, long nl, long line, int a, int b,
                                 int n, double hs, bool accum, int *status) {
  // scratch: [s][q][line], q < 12: C (9), y (3)
#define SC(s, q) sc[((long)(s) * 12 + (q)) * nl + line]
  BRow R;
  double C[9], y[3], Ap[9], Ai[9], t9[9], t3[3];
  for (int s = 0; s < n; s++) {
    block_row<D>(g, m, u, rhs, a, b, s, n, 0, hs, R);
    if (s == 0) {
#pragma unroll
      for (int q = 0; q < 9; q++) Ap[q] = R.D[q];
#pragma unroll
      for (int q = 0; q < 3; q++) t3[q] = R.b[q];
    } else {
      mm3(R.L, C, t9);
#pragma unroll
      for (int q = 0; q < 9; q++) Ap[q] = R.D[q] - t9[q];
      double ly[3];
      mv3(R.L, y, ly);
#pragma unroll
      for (int q = 0; q < 3; q++) t3[q] = R.b[q] - ly[q];
    }
    inv3(Ap, Ai, status);
    mm3(Ai, R.U, C);
    mv3(Ai, t3, y);
    if (s < n - 1) {
#pragma unroll
      for (int q = 0; q < 9; q++) SC(s, q) = C[q];
#pragma unroll
      for (int q = 0; q < 3; q++) SC(s, 9 + q) = y[q];
    }
  }
  // back substitution: x_{n-1} = y_{n-1}
  double xn[3] = {y[0], y[1], y[2]};
  block_store<D>(g, x, a, b, n - 1, xn, accum);
  for (int s = n - 2; s >= 0; s--) {
#pragma unroll
    for (int q = 0; q < 9; q++) C[q] = SC(s, q);
    double cx[3];
    mv3(C, xn, cx);
#pragma unroll
    for (int q = 0; q < 3; q++) xn[q] = SC(s, 9 + q) - cx[q];
    block_store<D>(g, x, a, b, s, xn, accum);
  }
#undef SC
}

// cyclic block line: bordered elimination of the last block
template <int D>
__device__ void solve_block_cyclic(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                   const Fields &x, double *sc, long nl, long line, int a, int b,
                                   int n, double hs, bool accum, int *status) {
  // scratch: [s][q][line], q < 21: C (9), y (3), Z (9)
#define SC(s, q) sc[((long)(s) * 21 + (q)) * nl + line]
  BRow R;
  double C[9], y[3], Z[9], Ap[9], Ai[9], t9[9], t3[3], E[9];
  for (int s = 0; s < n - 1; s++) {
    block_row<D>(g, m, u, rhs, a, b, s, n, 1, hs, R);
#pragma unroll
    for (int q = 0; q < 9; q++) E[q] = 0.0;
    if (s == 0) {
#pragma unroll
      for (int q = 0; q < 9; q++) { E[q] = R.L[q]; Ap[q] = R.D[q]; }
#pragma unroll
      for (int q = 0; q < 3; q++) t3[q] = R.b[q];
    } else {
      mm3(R.L, C, t9);
#pragma unroll
      for (int q = 0; q < 9; q++) Ap[q] = R.D[q] - t9[q];
      double ly[3];
      mv3(R.L, y, ly);
#pragma unroll
      for (int q = 0; q < 3; q++) t3[q] = R.b[q] - ly[q];
      mm3(R.L, Z, t9);
#pragma unroll
      for (int q = 0; q < 9; q++) E[q] = -t9[q];
    }
    if (s == n - 2) {
#pragma unroll
      for (int q = 0; q < 9; q++) { E[q] += R.U[q]; R.U[q] = 0.0; }
    }
    inv3(Ap, Ai, status);
    mm3(Ai, R.U, C);
    mv3(Ai, t3, y);
    mm3(Ai, E, Z);
#pragma unroll
    for (int q = 0; q < 9; q++) { SC(s, q) = C[q]; SC(s, 12 + q) = Z[q]; }
#pragma unroll
    for (int q = 0; q < 3; q++) SC(s, 9 + q) = y[q];
  }
  // backward: y_s -= C_s y_{s+1}, Z_s -= C_s Z_{s+1}; keep y, Z of rows n-2 and 0
  double yl[3], Zl[9];
#pragma unroll
  for (int q = 0; q < 3; q++) yl[q] = y[q];
#pragma unroll
  for (int q = 0; q < 9; q++) Zl[q] = Z[q];
  for (int s = n - 3; s >= 0; s--) {
#pragma unroll
    for (int q = 0; q < 9; q++) C[q] = SC(s, q);
    double cy[3];
    mv3(C, y, cy);
    mm3(C, Z, t9);
#pragma unroll
    for (int q = 0; q < 3; q++) { y[q] = SC(s, 9 + q) - cy[q]; SC(s, 9 + q) = y[q]; }
#pragma unroll
    for (int q = 0; q < 9; q++) { Z[q] = SC(s, 12 + q) - t9[q]; SC(s, 12 + q) = Z[q]; }
  }
  // last row: (D - L Z_{n-2} - U Z_0) x = b - L y_{n-2} - U y_0
  block_row<D>(g, m, u, rhs, a, b, n - 1, n, 1, hs, R);
  double LZ[9], UZ[9], Ly[3], Uy[3], xl[3];
  mm3(R.L, Zl, LZ);
  mm3(R.U, Z, UZ);
  mv3(R.L, yl, Ly);
  mv3(R.U, y, Uy);
#pragma unroll
  for (int q = 0; q < 9; q++) Ap[q] = R.D[q] - LZ[q] - UZ[q];
#pragma unroll
  for (int q = 0; q < 3; q++) t3[q] = R.b[q] - Ly[q] - Uy[q];
  inv3(Ap, Ai, status);
  mv3(Ai, t3, xl);
  block_store<D>(g, x, a, b, n - 1, xl, accum);
  for (int s = 0; s < n - 1; s++) {
    double v[3];
#pragma unroll
    for (int q = 0; q < 9; q++) Z[q] = SC(s, 12 + q);
    mv3(Z, xl, v);
#pragma unroll
    for (int q = 0; q < 3; q++) v[q] = SC(s, 9 + q) - v[q];
    block_store<D>(g, x, a, b, s, v, accum);
  }
#undef SC
}

// ----------------------------------------------------------- scalar rows --

struct SRow {
  double a, b, c, r;
};

// Scalar line of family FAM (0: A, 1: B) in direction D, transverse coords
// (a, b); row s.  Ghost folding at non-cyclic ends: walls -1, poles (u_r
// along theta) +1.
template <int D, int FAM>
__device__ void scalar_row(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs, int a,
                           int b, int s, int n, int cyc, double hs, SRow &R, long &xi,
                           double *&arr) {
  double ca, cb, cc_, sglo = -1.0, sghi = -1.0;
  if (D == 0) {
    const int i = s;
    const double r = g.rc[i], r2d2 = r * r * g.dr * g.dr;
    double ua, rho;
    if (FAM == 0) { // u_theta at theta-face (jf, k)
      const int jf = a, k = b;
      ua = 0.25 * (u.ld(F_UR, idx_r(g, i, jf - 1, k)) + u.ld(F_UR, idx_r(g, i, jf, k)) +
                   u.ld(F_UR, idx_r(g, i + 1, jf - 1, k)) + u.ld(F_UR, idx_r(g, i + 1, jf, k)));
      rho = 0.5 * (rho_at(g, m, u, i, jf - 1, k) + rho_at(g, m, u, i, jf, k));
      xi = idx_t(g, i, jf, k); arr = rhs.ut;
    } else { // u_phi at phi-face (j, kf)
      const int j = a, kf = b;
      const int k0 = g.periodic ? wrapk(g, kf - 1) : kf - 1, k1 = g.periodic ? wrapk(g, kf) : kf;
      ua = 0.25 * (u.ld(F_UR, idx_r(g, i, j, k0)) + u.ld(F_UR, idx_r(g, i, j, k1)) +
                   u.ld(F_UR, idx_r(g, i + 1, j, k0)) + u.ld(F_UR, idx_r(g, i + 1, j, k1)));
      rho = 0.5 * (rho_at(g, m, u, i, j, k0) + rho_at(g, m, u, i, j, k1));
      xi = idx_f(g, i, j, kf); arr = rhs.uf;
    }
    const double nu = m.mu / rho;
    const double fp = g.rf[i + 1] * g.rf[i + 1], fm = g.rf[i] * g.rf[i];
    ca = -ua / (2.0 * g.dr) - nu * fm / r2d2;
    cb = nu * (fp + fm) / r2d2;
    cc_ = ua / (2.0 * g.dr) - nu * fp / r2d2;
  } else if (D == 1) {
    const int j = s;
    const double sn = g.sc[j];
    double ua, rho, rr;
    if (FAM == 0) { // u_r at r-face (fr, k)
      const int fr = a, k = b;
      rr = g.rf[fr];
      ua = 0.25 * (u.ld(F_UT, idx_t(g, fr - 1, j, k)) + u.ld(F_UT, idx_t(g, fr - 1, j + 1, k)) +
                   u.ld(F_UT, idx_t(g, fr, j, k)) + u.ld(F_UT, idx_t(g, fr, j + 1, k)));
      rho = 0.5 * (rho_at(g, m, u, fr - 1, j, k) + rho_at(g, m, u, fr, j, k));
      xi = idx_r(g, fr, j, k); arr = rhs.ur;
      sglo = g.pole_lo ? 1.0 : -1.0;
      sghi = g.pole_hi ? 1.0 : -1.0;
    } else { // u_phi at phi-face (i, kf)
      const int i = a, kf = b;
      rr = g.rc[i];
      const int k0 = g.periodic ? wrapk(g, kf - 1) : kf - 1, k1 = g.periodic ? wrapk(g, kf) : kf;
      ua = 0.25 * (u.ld(F_UT, idx_t(g, i, j, k0)) + u.ld(F_UT, idx_t(g, i, j, k1)) +
                   u.ld(F_UT, idx_t(g, i, j + 1, k0)) + u.ld(F_UT, idx_t(g, i, j + 1, k1)));
      rho = 0.5 * (rho_at(g, m, u, i, j, k0) + rho_at(g, m, u, i, j, k1));
      xi = idx_f(g, i, j, kf); arr = rhs.uf;
    }
    const double nu = m.mu / rho, q = rr * rr * sn * g.dt * g.dt;
    ca = -ua / (2.0 * rr * g.dt) - nu * g.sf[j] / q;
    cb = nu * (g.sf[j + 1] + g.sf[j]) / q;
    cc_ = ua / (2.0 * rr * g.dt) - nu * g.sf[j + 1] / q;
  } else {
    const int k = s;
    double ua, rho, rr, ss;
    if (FAM == 0) { // u_r at r-face (fr, j)
      const int fr = a, j = b;
      rr = g.rf[fr]; ss = g.sc[j];
      const int kp = g.periodic ? wrapk(g, k + 1) : k + 1;
      ua = 0.25 * (u.ld(F_UF, idx_f(g, fr - 1, j, k)) + u.ld(F_UF, idx_f(g, fr - 1, j, kp)) +
                   u.ld(F_UF, idx_f(g, fr, j, k)) + u.ld(F_UF, idx_f(g, fr, j, kp)));
      rho = 0.5 * (rho_at(g, m, u, fr - 1, j, k) + rho_at(g, m, u, fr, j, k));
      xi = idx_r(g, fr, j, k); arr = rhs.ur;
    } else { // u_theta at theta-face (i, ft)
      const int i = a, ft = b;
      rr = g.rc[i]; ss = g.sf[ft];
      const int kp = g.periodic ? wrapk(g, k + 1) : k + 1;
      ua = 0.25 * (u.ld(F_UF, idx_f(g, i, ft - 1, k)) + u.ld(F_UF, idx_f(g, i, ft - 1, kp)) +
                   u.ld(F_UF, idx_f(g, i, ft, k)) + u.ld(F_UF, idx_f(g, i, ft, kp)));
      rho = 0.5 * (rho_at(g, m, u, i, ft - 1, k) + rho_at(g, m, u, i, ft, k));
      xi = idx_t(g, i, ft, k); arr = rhs.ut;
    }
    const double nu = m.mu / rho, q = rr * rr * ss * ss * g.dp * g.dp;
    ca = -ua / (2.0 * rr * ss * g.dp) - nu / q;
    cb = 2.0 * nu / q;
    cc_ = ua / (2.0 * rr * ss * g.dp) - nu / q;
  }
  if (!cyc && s == 0) { cb += sglo * ca; ca = 0.0; }
  if (!cyc && s == n - 1) { cb += sghi * cc_; cc_ = 0.0; }
  R.a = hs * ca;
  R.b = 1.0 + hs * cb;
  R.c = hs * cc_;
  R.r = arr[xi];
}

template <int D, int FAM>
__device__ __forceinline__ long scalar_index(const Geo &g, int a, int b, int s) {
  if (D == 0) return FAM == 0 ? idx_t(g, s, a, b) : idx_f(g, s, a, b);
  if (D == 1) return FAM == 0 ? idx_r(g, a, s, b) : idx_f(g, a, s, b);
  return FAM == 0 ? idx_r(g, a, b, s) : idx_t(g, a, b, s);
}

template <int D, int FAM>
__device__ void solve_scalar_line(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                  const Fields &x, double *sc, long nl, long line, int a, int b,
                                  int n, int cyc, double hs, bool accum, int *status) {
  // output array of this family
  double *out;
  if (D == 0) out = FAM == 0 ? x.ut : x.uf;
  else if (D == 1) out = FAM == 0 ? x.ur : x.uf;
  else out = FAM == 0 ? x.ur : x.ut;
  SRow R;
  long xi;
  double *arr;
  if (!cyc) {
#define SC(s, q) sc[((long)(s) * 2 + (q)) * nl + line]
    double cpv = 0.0, yv = 0.0;
    for (int s = 0; s < n; s++) {
      scalar_row<D, FAM>(g, m, u, rhs, a, b, s, n, 0, hs, R, xi, arr);
      const double den = R.b - R.a * cpv;
      if (!(den != 0.0)) status[ST_SINGULAR] = 1;
      const double id = 1.0 / den;
      cpv = R.c * id;
      yv = (R.r - R.a * yv) * id;
      if (s < n - 1) { SC(s, 0) = cpv; SC(s, 1) = yv; }
    }
    double xv = yv;
    if (accum) out[xi] += xv; else out[xi] = xv;
    for (int s = n - 2; s >= 0; s--) {
      xv = SC(s, 1) - SC(s, 0) * xv;
      const long xs = scalar_index<D, FAM>(g, a, b, s);
      if (accum) out[xs] += xv; else out[xs] = xv;
    }
#undef SC
  } else {
#define SC(s, q) sc[((long)(s) * 3 + (q)) * nl + line]
    // bordered elimination of the last unknown
    double cpv = 0.0, yv = 0.0, zv = 0.0;
    for (int s = 0; s < n - 1; s++) {
      scalar_row<D, FAM>(g, m, u, rhs, a, b, s, n, 1, hs, R, xi, arr);
      double e = 0.0, c = R.c, den;
      if (s == 0) { e = R.a; den = R.b; }
      else { den = R.b - R.a * cpv; e = -R.a * zv; }
      if (s == n - 2) { e += c; c = 0.0; }
      if (!(den != 0.0)) status[ST_SINGULAR] = 1;
      const double id = 1.0 / den;
      yv = (s == 0 ? R.r : R.r - R.a * yv) * id;
      cpv = c * id;
      zv = e * id;
      SC(s, 0) = cpv; SC(s, 1) = yv; SC(s, 2) = zv;
    }
    double yl = yv, zl = zv;
    for (int s = n - 3; s >= 0; s--) {
      const double cs = SC(s, 0);
      yv = SC(s, 1) - cs * yv;
      zv = SC(s, 2) - cs * zv;
      SC(s, 1) = yv; SC(s, 2) = zv;
    }
    scalar_row<D, FAM>(g, m, u, rhs, a, b, n - 1, n, 1, hs, R, xi, arr);
    const double den = R.b - R.a * zl - R.c * zv;
    if (!(den != 0.0)) status[ST_SINGULAR] = 1;
    const double xl = (R.r - R.a * yl - R.c * yv) / den;
    if (accum) out[xi] += xl; else out[xi] = xl;
    for (int s = 0; s < n - 1; s++) {
      const double xv = SC(s, 1) - SC(s, 2) * xl;
      const long xs = scalar_index<D, FAM>(g, a, b, s);
      if (accum) out[xs] += xv; else out[xs] = xv;
    }
#undef SC
  }
}

// ----------------------------------------------------------------- kernel --

template <int D>
__global__ void __launch_bounds__(128) k_sweep(Geo g, Mat m, SrcOne u, double hs, Fields rhs,
                                               Fields x, double *scb, double *scs, int accum,
                                               int *status) {
  const Families F = families(g, D);
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nkf = g.periodic ? g.np : g.np - 1, kf0 = g.periodic ? 0 : 1;
  if (t < F.nb) {
    int a, b;
    if (D == 0) { a = (int)(t / g.np); b = (int)(t % g.np); }
    else if (D == 1) { a = (int)(t / g.np); b = (int)(t % g.np); }
    else { a = (int)(t / g.nt); b = (int)(t % g.nt); }
    if (!accum) zero_bnd<D>(g, x, a, b);
    if (F.cyclic) solve_block_cyclic<D>(g, m, u, rhs, x, scb, F.nb, t, a, b, F.n, hs, accum != 0, status);
    else solve_block_line<D>(g, m, u, rhs, x, scb, F.nb, t, a, b, F.n, hs, accum != 0, status);
    return;
  }
  long t2 = t - F.nb;
  const long ns = (long)F.na + F.nbb;
  if (t2 < F.na) {
    int a, b;
    if (D == 0) { a = 1 + (int)(t2 / g.np); b = (int)(t2 % g.np); }
    else if (D == 1) { a = 1 + (int)(t2 / g.np); b = (int)(t2 % g.np); }
    else { a = 1 + (int)(t2 / g.nt); b = (int)(t2 % g.nt); }
    solve_scalar_line<D, 0>(g, m, u, rhs, x, scs, ns, t2, a, b, F.n, F.cyclic, hs, accum != 0, status);
    return;
  }
  t2 -= F.na;
  if (t2 < F.nbb) {
    int a, b;
    if (D == 0) { a = (int)(t2 / nkf); b = kf0 + (int)(t2 % nkf); }
    else if (D == 1) { a = (int)(t2 / nkf); b = kf0 + (int)(t2 % nkf); }
    else { a = (int)(t2 / (g.nt - 1)); b = 1 + (int)(t2 % (g.nt - 1)); }
    solve_scalar_line<D, 1>(g, m, u, rhs, x, scs, ns, F.na + t2, a, b, F.n, F.cyclic, hs, accum != 0, status);
  }
}

void sweep_scratch_size(const Geo &g, long *blk, long *sca) {
  long b = 0, s = 0;
  for (int d = 0; d < 3; d++) {
    const Families F = families(g, d);
    const long per = F.cyclic ? 21 : 12, pers = F.cyclic ? 3 : 2;
    b = b > per * F.n * (long)F.nb ? b : per * F.n * (long)F.nb;
    const long ss = pers * F.n * ((long)F.na + F.nbb);
    s = s > ss ? s : ss;
  }
  *blk = b;
  *sca = s;
}

void launch_sweep(int d, const Geo &g, const Mat &m, const Fields &Ub, double tau,
                  const Fields &rhs, const Fields &x, const Scratch &sc, int *status,
                  hipStream_t st, bool accum) {
  SrcOne u;
  u.a[F_P] = Ub.p; u.a[F_UR] = Ub.ur; u.a[F_UT] = Ub.ut; u.a[F_UF] = Ub.uf; u.a[F_T] = Ub.T;
  const Families F = families(g, d);
  const long nt = (long)F.nb + F.na + F.nbb;
  const int bs = 128;
  dim3 grid((unsigned)((nt + bs - 1) / bs));
  const double hs = 0.5 * tau;
  if (d == 0) hipLaunchKernelGGL(k_sweep<0>, grid, dim3(bs), 0, st, g, m, u, hs, rhs, x, sc.blk, sc.sca, accum ? 1 : 0, status);
  else if (d == 1) hipLaunchKernelGGL(k_sweep<1>, grid, dim3(bs), 0, st, g, m, u, hs, rhs, x, sc.blk, sc.sca, accum ? 1 : 0, status);
  else hipLaunchKernelGGL(k_sweep<2>, grid, dim3(bs), 0, st, g, m, u, hs, rhs, x, sc.blk, sc.sca, accum ? 1 : 0, status);
}

} // namespace dsw
