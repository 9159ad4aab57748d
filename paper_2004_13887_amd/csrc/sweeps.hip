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
#include "rows.hpp"

namespace dsw {

template <int D, bool TR>
__device__ __forceinline__ void solve_block_line(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                 const Out &o, double *sc, long nl, long line, int a, int b,
                                 int n, double hs, int *status) {
  // scratch: [s][q][line], q < 12: C (9), y (3)
#define SC(s, q) sc[((long)(s) * 12 + (q)) * nl + line]
  BRow R;
  double C[9], y[3], Ap[9], Ai[9], t9[9], t3[3];
  for (int s = 0; s < n; s++) {
    get_brow<D, TR>(g, m, u, rhs, a, b, s, n, 0, hs, R);
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
  block_store<D>(g, o, a, b, n - 1, xn);
  for (int s = n - 2; s >= 0; s--) {
#pragma unroll
    for (int q = 0; q < 9; q++) C[q] = SC(s, q);
    double cx[3];
    mv3(C, xn, cx);
#pragma unroll
    for (int q = 0; q < 3; q++) xn[q] = SC(s, 9 + q) - cx[q];
    block_store<D>(g, o, a, b, s, xn);
  }
#undef SC
}

// Transposed non-cyclic block line, M^T x = y, from the block LU factors of
// M that the forward recurrence builds (M = L U: L has the pivots
// Ap_s = D_s - A_s C'_{s-1} on its diagonal and the lower blocks A_s below it,
// U is unit upper with C'_s = Ap_s^{-1} C_s): first U^T z = y,
// z_s = y_s - C'_{s-1}^T z_{s-1}, alongside the factorisation; then L^T x = z,
// x_s = Ap_s^{-T} (z_s - A_{s+1}^T x_{s+1}).  Each row is assembled once.
// scratch [s][q][line], q < 21: Ap^{-1} (9), A (9), z (3)
template <int D>
__device__ __forceinline__ void solve_block_line_T(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                   const Out &o, double *sc, long nl, long line, int a, int b, int n,
                                   double hs, int *status) {
#define SC(s, q) sc[((long)(s) * 21 + (q)) * nl + line]
  BRow R;
  double C[9], z[3], Ap[9], Ai[9], t9[9], t3[3];
  for (int s = 0; s < n; s++) {
    block_row<D>(g, m, u, rhs, a, b, s, n, 0, hs, R);
    if (s == 0) {
#pragma unroll
      for (int q = 0; q < 9; q++) Ap[q] = R.D[q];
#pragma unroll
      for (int q = 0; q < 3; q++) z[q] = R.b[q];
    } else {
      mm3(R.L, C, t9);
#pragma unroll
      for (int q = 0; q < 9; q++) Ap[q] = R.D[q] - t9[q];
#pragma unroll
      for (int q = 0; q < 3; q++) t3[q] = R.b[q] - (C[q] * z[0] + C[3 + q] * z[1] + C[6 + q] * z[2]);
#pragma unroll
      for (int q = 0; q < 3; q++) z[q] = t3[q];
    }
    inv3(Ap, Ai, status);
    mm3(Ai, R.U, C);
    if (s < n - 1) {
#pragma unroll
      for (int q = 0; q < 9; q++) { SC(s, q) = Ai[q]; SC(s, 9 + q) = R.L[q]; }
#pragma unroll
      for (int q = 0; q < 3; q++) SC(s, 18 + q) = z[q];
    }
  }
  // x_{n-1} = Ap_{n-1}^{-T} z_{n-1}
  double x[3], An[9];
#pragma unroll
  for (int q = 0; q < 3; q++) x[q] = Ai[q] * z[0] + Ai[3 + q] * z[1] + Ai[6 + q] * z[2];
#pragma unroll
  for (int q = 0; q < 9; q++) An[q] = R.L[q];
  block_store<D>(g, o, a, b, n - 1, x);
  for (int s = n - 2; s >= 0; s--) {
    double w[3];
#pragma unroll
    for (int q = 0; q < 3; q++)
      w[q] = SC(s, 18 + q) - (An[q] * x[0] + An[3 + q] * x[1] + An[6 + q] * x[2]);
#pragma unroll
    for (int q = 0; q < 9; q++) { Ai[q] = SC(s, q); An[q] = SC(s, 9 + q); }
#pragma unroll
    for (int q = 0; q < 3; q++) x[q] = Ai[q] * w[0] + Ai[3 + q] * w[1] + Ai[6 + q] * w[2];
    block_store<D>(g, o, a, b, s, x);
  }
#undef SC
}

// cyclic block line: bordered elimination of the last block
template <int D, bool TR>
__device__ __forceinline__ void solve_block_cyclic(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                   const Out &o, double *sc, long nl, long line, int a, int b,
                                   int n, double hs, int *status) {
  // scratch: [s][q][line], q < 21: C (9), y (3), Z (9)
#define SC(s, q) sc[((long)(s) * 21 + (q)) * nl + line]
  BRow R;
  double C[9], y[3], Z[9], Ap[9], Ai[9], t9[9], t3[3], E[9];
  for (int s = 0; s < n - 1; s++) {
    get_brow<D, TR>(g, m, u, rhs, a, b, s, n, 1, hs, R);
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
  get_brow<D, TR>(g, m, u, rhs, a, b, n - 1, n, 1, hs, R);
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
  block_store<D>(g, o, a, b, n - 1, xl);
  for (int s = 0; s < n - 1; s++) {
    double v[3];
#pragma unroll
    for (int q = 0; q < 9; q++) Z[q] = SC(s, 12 + q);
    mv3(Z, xl, v);
#pragma unroll
    for (int q = 0; q < 3; q++) v[q] = SC(s, 9 + q) - v[q];
    block_store<D>(g, o, a, b, s, v);
  }
#undef SC
}


template <int D, int FAM, bool TR>
__device__ __forceinline__ void solve_scalar_line(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                  const Out &o, double *sc, long nl, long line, int a, int b,
                                  int n, int cyc, double hs, int *status) {
  // output field of this family
  int ofid;
  if (D == 0) ofid = FAM == 0 ? F_UT : F_UF;
  else if (D == 1) ofid = FAM == 0 ? F_UR : F_UF;
  else ofid = FAM == 0 ? F_UR : F_UT;
  SRow R;
  long xi;
  double *arr;
  if (!cyc && TR) {
    // transposed, from the LU factors of the forward recurrence:
    // z_s = y_s - c'_{s-1} z_{s-1}; x_s = (z_s - a_{s+1} x_{s+1}) / den_s
#define SC(s, q) sc[((long)(s) * 3 + (q)) * nl + line]
    double cpv = 0.0, zv = 0.0, av = 0.0, id = 1.0;
    for (int s = 0; s < n; s++) {
      scalar_row<D, FAM>(g, m, u, rhs, a, b, s, n, 0, hs, R, xi, arr);
      const double den = R.b - R.a * cpv;
      if (!(den != 0.0)) status[ST_SINGULAR] = 1;
      id = rcp_nr(den);
      zv = R.r - cpv * zv;
      cpv = R.c * id;
      av = R.a;
      if (s < n - 1) { SC(s, 0) = id; SC(s, 1) = R.a; SC(s, 2) = zv; }
    }
    double xv = id * zv;
    put(o, ofid, xi, xv);
    for (int s = n - 2; s >= 0; s--) {
      xv = SC(s, 0) * (SC(s, 2) - av * xv);
      av = SC(s, 1);
      put(o, ofid, scalar_index<D, FAM>(g, a, b, s), xv);
    }
#undef SC
  } else if (!cyc) {
#define SC(s, q) sc[((long)(s) * 2 + (q)) * nl + line]
    double cpv = 0.0, yv = 0.0;
    for (int s = 0; s < n; s++) {
      get_srow<D, FAM, TR>(g, m, u, rhs, a, b, s, n, 0, hs, R, xi, arr);
      const double den = R.b - R.a * cpv;
      if (!(den != 0.0)) status[ST_SINGULAR] = 1;
      const double id = rcp_nr(den);
      cpv = R.c * id;
      yv = (R.r - R.a * yv) * id;
      if (s < n - 1) { SC(s, 0) = cpv; SC(s, 1) = yv; }
    }
    double xv = yv;
    put(o, ofid, xi, xv);
    for (int s = n - 2; s >= 0; s--) {
      xv = SC(s, 1) - SC(s, 0) * xv;
      const long xs = scalar_index<D, FAM>(g, a, b, s);
      put(o, ofid, xs, xv);
    }
#undef SC
  } else {
#define SC(s, q) sc[((long)(s) * 3 + (q)) * nl + line]
    // bordered elimination of the last unknown
    double cpv = 0.0, yv = 0.0, zv = 0.0;
    for (int s = 0; s < n - 1; s++) {
      get_srow<D, FAM, TR>(g, m, u, rhs, a, b, s, n, 1, hs, R, xi, arr);
      double e = 0.0, c = R.c, den;
      if (s == 0) { e = R.a; den = R.b; }
      else { den = R.b - R.a * cpv; e = -R.a * zv; }
      if (s == n - 2) { e += c; c = 0.0; }
      if (!(den != 0.0)) status[ST_SINGULAR] = 1;
      const double id = rcp_nr(den);
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
    get_srow<D, FAM, TR>(g, m, u, rhs, a, b, n - 1, n, 1, hs, R, xi, arr);
    const double den = R.b - R.a * zl - R.c * zv;
    if (!(den != 0.0)) status[ST_SINGULAR] = 1;
    const double xl = (R.r - R.a * yl - R.c * yv) * rcp_nr(den);
    put(o, ofid, xi, xl);
    for (int s = 0; s < n - 1; s++) {
      const double xv = SC(s, 1) - SC(s, 2) * xl;
      const long xs = scalar_index<D, FAM>(g, a, b, s);
      put(o, ofid, xs, xv);
    }
#undef SC
  }
}

// ----------------------------------------------------------------- kernel --

// one thread per line: the block lines first, then the two scalar families;
// one grid or a batch of grids (flat grid of workgroups)
template <int D, bool TR>
__device__ __forceinline__ void sweep_body(const PassArgs &a, unsigned w) {
  const Geo &g = a.g;
  const Families F = families(g, D);
  const long t = (long)w * blockDim.x + threadIdx.x;
  const int nkf = g.periodic ? g.np : g.np - 1, kf0 = g.periodic ? 0 : 1;
  const double hs = a.tau;
  if (t < F.nb) {
    int p, q;
    if (D == 0) { p = (int)(t / g.np); q = (int)(t % g.np); }
    else if (D == 1) { p = (int)(t / g.np); q = (int)(t % g.np); }
    else { p = (int)(t / g.nt); q = (int)(t % g.nt); }
    if (a.o.mode == 0) zero_bnd<D>(g, a.o.x, p, q);
    if (F.cyclic) solve_block_cyclic<D, TR>(g, a.m, a.u, a.rhs, a.o, a.scb, F.nb, t, p, q, F.n, hs, a.status);
    else if (TR) solve_block_line_T<D>(g, a.m, a.u, a.rhs, a.o, a.scb, F.nb, t, p, q, F.n, hs, a.status);
    else solve_block_line<D, false>(g, a.m, a.u, a.rhs, a.o, a.scb, F.nb, t, p, q, F.n, hs, a.status);
    return;
  }
  long t2 = t - F.nb;
  const long ns = (long)F.na + F.nbb;
  if (t2 < F.na) {
    int p, q;
    if (D == 0) { p = 1 + (int)(t2 / g.np); q = (int)(t2 % g.np); }
    else if (D == 1) { p = 1 + (int)(t2 / g.np); q = (int)(t2 % g.np); }
    else { p = 1 + (int)(t2 / g.nt); q = (int)(t2 % g.nt); }
    solve_scalar_line<D, 0, TR>(g, a.m, a.u, a.rhs, a.o, a.scs, ns, t2, p, q, F.n, F.cyclic, hs, a.status);
    return;
  }
  t2 -= F.na;
  if (t2 < F.nbb) {
    int p, q;
    if (D == 0) { p = (int)(t2 / nkf); q = kf0 + (int)(t2 % nkf); }
    else if (D == 1) { p = (int)(t2 / nkf); q = kf0 + (int)(t2 % nkf); }
    else { p = (int)(t2 / (g.nt - 1)); q = 1 + (int)(t2 % (g.nt - 1)); }
    solve_scalar_line<D, 1, TR>(g, a.m, a.u, a.rhs, a.o, a.scs, ns, F.na + t2, p, q, F.n, F.cyclic, hs,
                            a.status);
  }
}

// B: a batch of grids (arguments from the batch table), else one grid
template <int D, bool B>
__global__ void __launch_bounds__(256) DSW_OCC(DSW_WAVES_SWEEP) k_sweep(PassArgs a, Batch bt) {
  if constexpr (B) {
    const int mb = batch_member(bt, blockIdx.x);
    sweep_body<D, false>(batch_args(bt, mb), blockIdx.x - bt.woff[mb]);
  } else {
    sweep_body<D, false>(a, blockIdx.x);
  }
}

// transposed systems (adjoint): (I + tau/2 D_d(Ubar))^T x = rhs, one grid
template <int D>
__global__ void __launch_bounds__(256) k_sweep_T(PassArgs a) {
  sweep_body<D, true>(a, blockIdx.x);
}

void launch_sweep_T(int d, const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st) {
  const dim3 gr(blocks), bl(threads);
  if (d == 0) hipLaunchKernelGGL(k_sweep_T<0>, gr, bl, 0, st, a);
  else if (d == 1) hipLaunchKernelGGL(k_sweep_T<1>, gr, bl, 0, st, a);
  else hipLaunchKernelGGL(k_sweep_T<2>, gr, bl, 0, st, a);
}

// ------------------------------------------------ two-ended block lines --

// The elimination and substitution loops of the theta lines are unrolled by
// two: the next row's loads issue while the current row is eliminated.  The
// theta sweep runs at two waves per SIMD whatever its register count, so the
// extra registers cost no occupancy (the r sweep's would: three waves to two).
// Not for the forced sweep (wall-aware sources), which then spills.
//
// Twisted block factorisation of a non-cyclic block line by two threads: the
// top thread eliminates rows 0 .. m-1 downwards (C'_s = Ap_s^{-1} U_s,
// y_s = Ap_s^{-1}(b_s - L_s y_{s-1}), Ap_s = D_s - L_s C'_{s-1}), the bottom
// thread rows n-1 .. m+1 upwards (E'_s = Bp_s^{-1} L_s,
// z_s = Bp_s^{-1}(b_s - U_s z_{s+1}), Bp_s = D_s - U_s E'_{s+1}); the top
// thread then solves the middle row
//   (D_m - L_m C'_{m-1} - U_m E'_{m+1}) x_m = b_m - L_m y_{m-1} - U_m z_{m+1}
// and each substitutes back over its half (x_s = y_s - C'_s x_{s+1} above,
// x_s = z_s - E'_s x_{s-1} below).  Same arithmetic and scratch as one thread
// per line, twice the threads.  Lane l of the top half and lane l of the
// bottom half of a workgroup share a line; the middle data pass through LDS.
template <int D, class S>
__device__ __forceinline__ void twisted_block_line(const Geo &g, const Mat &m, const S &u, const Fields &rhs,
                                   const Out &o, double *__restrict__ sc, long nl, long line, bool act, bool top,
                                   int a, int b, int n, double hs, double *lds, int lane, int *status) {
#define SC(s, q) sc[((long)(s) * 12 + (q)) * nl + line]
  constexpr int UNR = (D == 1 && !S::WALL) ? 2 : 1;  // theta lines: unrolled twice
  const int mid = n / 2;
  BRow R;
  double C[9], y[3], Ap[9], Ai[9], t9[9], t3[3];
  double *my = lds + (long)lane * 15;  // E'_{m+1} (9), z_{m+1} (3), x_m (3)
  // A zero pivot is recorded once, after the elimination: a store (or a
  // branch) inside the loop would hold the next row's loads back until the
  // row before is done; so would the scratch stores, were the scratch array
  // not declared unaliased.
  bool sing = false;
  if (act) {
    if (top) {
      #pragma unroll UNR
      for (int s = 0; s < mid; s++) {
        block_row<D>(g, m, u, rhs, a, b, s, n, 0, hs, R);
        if (s == 0) {
#pragma unroll
          for (int q = 0; q < 9; q++) Ap[q] = R.D[q];
#pragma unroll
          for (int q = 0; q < 3; q++) t3[q] = R.b[q];
        } else {
          mm3m<NZ_L, NZ_ALL>(R.L, C, t9);
#pragma unroll
          for (int q = 0; q < 9; q++) Ap[q] = R.D[q] - t9[q];
          double ly[3];
          mv3m<NZ_L>(R.L, y, ly);
#pragma unroll
          for (int q = 0; q < 3; q++) t3[q] = R.b[q] - ly[q];
        }
        sing |= inv3q(Ap, Ai);
        mm3m<NZ_ALL, NZ_U>(Ai, R.U, C);
        mv3(Ai, t3, y);
#pragma unroll
        for (int q = 0; q < 9; q++) SC(s, q) = C[q];
#pragma unroll
        for (int q = 0; q < 3; q++) SC(s, 9 + q) = y[q];
      }
    } else {
      #pragma unroll UNR
      for (int s = n - 1; s > mid; s--) {
        block_row<D>(g, m, u, rhs, a, b, s, n, 0, hs, R);
        if (s == n - 1) {
#pragma unroll
          for (int q = 0; q < 9; q++) Ap[q] = R.D[q];
#pragma unroll
          for (int q = 0; q < 3; q++) t3[q] = R.b[q];
        } else {
          mm3m<NZ_U, NZ_ALL>(R.U, C, t9);
#pragma unroll
          for (int q = 0; q < 9; q++) Ap[q] = R.D[q] - t9[q];
          double uz[3];
          mv3m<NZ_U>(R.U, y, uz);
#pragma unroll
          for (int q = 0; q < 3; q++) t3[q] = R.b[q] - uz[q];
        }
        sing |= inv3q(Ap, Ai);
        mm3m<NZ_ALL, NZ_L>(Ai, R.L, C);  // E'_s
        mv3(Ai, t3, y);   // z_s
#pragma unroll
        for (int q = 0; q < 9; q++) SC(s, q) = C[q];
#pragma unroll
        for (int q = 0; q < 3; q++) SC(s, 9 + q) = y[q];
      }
#pragma unroll
      for (int q = 0; q < 9; q++) my[q] = C[q];
#pragma unroll
      for (int q = 0; q < 3; q++) my[9 + q] = y[q];
    }
  }
  if (sing) status[ST_SINGULAR] = 1;
  __syncthreads();
  if (act && top) {  // middle row
    block_row<D>(g, m, u, rhs, a, b, mid, n, 0, hs, R);
    double Ub[9], t9b[9], uz[3], ly[3];
    mm3m<NZ_U, NZ_ALL>(R.U, my, Ub);  // U_m E'_{m+1}
    mv3m<NZ_U>(R.U, my + 9, uz);
    if (mid > 0) {
      mm3m<NZ_L, NZ_ALL>(R.L, C, t9b);
      mv3m<NZ_L>(R.L, y, ly);
    } else {
#pragma unroll
      for (int q = 0; q < 9; q++) t9b[q] = 0.0;
#pragma unroll
      for (int q = 0; q < 3; q++) ly[q] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < 9; q++) Ap[q] = R.D[q] - t9b[q] - Ub[q];
#pragma unroll
    for (int q = 0; q < 3; q++) t3[q] = R.b[q] - ly[q] - uz[q];
    inv3(Ap, Ai, status);
    double xm[3];
    mv3(Ai, t3, xm);
    block_store<D>(g, o, a, b, mid, xm);
#pragma unroll
    for (int q = 0; q < 3; q++) my[12 + q] = xm[q];
  }
  __syncthreads();
  if (!act) return;
  double x[3] = {my[12], my[13], my[14]};
  if (top) {
    #pragma unroll UNR
    for (int s = mid - 1; s >= 0; s--) {
#pragma unroll
      for (int q = 0; q < 9; q++) C[q] = SC(s, q);
      double cx[3];
      mv3(C, x, cx);
#pragma unroll
      for (int q = 0; q < 3; q++) x[q] = SC(s, 9 + q) - cx[q];
      block_store<D>(g, o, a, b, s, x);
    }
  } else {
    #pragma unroll UNR
    for (int s = mid + 1; s < n; s++) {
#pragma unroll
      for (int q = 0; q < 9; q++) C[q] = SC(s, q);
      double ex[3];
      mv3(C, x, ex);
#pragma unroll
      for (int q = 0; q < 3; q++) x[q] = SC(s, 9 + q) - ex[q];
      block_store<D>(g, o, a, b, s, x);
    }
  }
#undef SC
}

// The same two-ended elimination for the transposed line M^T x = b (adjoint).
// Row s of M^T is (U_{s-1}^T, D_s^T, L_{s+1}^T) with the right-hand side read
// at row s's unknowns.  Each thread keeps a window of the rows of M around
// the row it is at, so every row of M is assembled once per thread (plus one
// row for the middle), not three times.  Lines have n >= 3, so 1 <= m < n - 1.
template <int D>
__device__ __forceinline__ void twisted_block_line_T(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                     const Out &o, double *__restrict__ sc, long nl, long line, bool act, bool top,
                                     int a, int b, int n, double hs, double *lds, int lane, int *status) {
#define SC(s, q) sc[((long)(s) * 12 + (q)) * nl + line]
  const int mid = n / 2;
  BRow R;
  double C[9], y[3], Ap[9], Ai[9], t9[9], t3[3], Lt[9], Dt[9], Ut[9];
  double Wa[9], Wd[9], Wb[9], wb[3]; // window (see each half)
  double *my = lds + (long)lane * 15;
#pragma unroll
  for (int q = 0; q < 9; q++) C[q] = 0.0;
#pragma unroll
  for (int q = 0; q < 3; q++) y[q] = 0.0;
  bool sing = false;  // a zero pivot, recorded once after the elimination
  if (act) {
    if (top) {
      // window: Wa = U_{s-1}, Wd = D_s, Wb = U_s, wb = b_s
      block_row<D>(g, m, u, rhs, a, b, 0, n, 0, hs, R);
#pragma unroll
      for (int q = 0; q < 9; q++) { Wa[q] = 0.0; Wd[q] = R.D[q]; Wb[q] = R.U[q]; }
#pragma unroll
      for (int q = 0; q < 3; q++) wb[q] = R.b[q];
      for (int s = 0; s < mid; s++) {
        block_row<D>(g, m, u, rhs, a, b, s + 1, n, 0, hs, R);
        tr3(Wa, Lt);
        tr3(Wd, Dt);
        tr3(R.L, Ut);
        if (s == 0) {
#pragma unroll
          for (int q = 0; q < 9; q++) Ap[q] = Dt[q];
#pragma unroll
          for (int q = 0; q < 3; q++) t3[q] = wb[q];
        } else {
          mm3(Lt, C, t9);
#pragma unroll
          for (int q = 0; q < 9; q++) Ap[q] = Dt[q] - t9[q];
          double ly[3];
          mv3(Lt, y, ly);
#pragma unroll
          for (int q = 0; q < 3; q++) t3[q] = wb[q] - ly[q];
        }
        sing |= inv3q(Ap, Ai);
        mm3(Ai, Ut, C);
        mv3(Ai, t3, y);
#pragma unroll
        for (int q = 0; q < 9; q++) SC(s, q) = C[q];
#pragma unroll
        for (int q = 0; q < 3; q++) SC(s, 9 + q) = y[q];
#pragma unroll
        for (int q = 0; q < 9; q++) { Wa[q] = Wb[q]; Wd[q] = R.D[q]; Wb[q] = R.U[q]; }
#pragma unroll
        for (int q = 0; q < 3; q++) wb[q] = R.b[q];
      }
    } else {
      // window: Wa = L_{s+1}, Wd = D_s, Wb = L_s, wb = b_s
      block_row<D>(g, m, u, rhs, a, b, n - 1, n, 0, hs, R);
#pragma unroll
      for (int q = 0; q < 9; q++) { Wa[q] = 0.0; Wd[q] = R.D[q]; Wb[q] = R.L[q]; }
#pragma unroll
      for (int q = 0; q < 3; q++) wb[q] = R.b[q];
      for (int s = n - 1; s > mid; s--) {
        block_row<D>(g, m, u, rhs, a, b, s - 1, n, 0, hs, R);
        tr3(R.U, Lt);
        tr3(Wd, Dt);
        tr3(Wa, Ut);
        if (s == n - 1) {
#pragma unroll
          for (int q = 0; q < 9; q++) Ap[q] = Dt[q];
#pragma unroll
          for (int q = 0; q < 3; q++) t3[q] = wb[q];
        } else {
          mm3(Ut, C, t9);
#pragma unroll
          for (int q = 0; q < 9; q++) Ap[q] = Dt[q] - t9[q];
          double uz[3];
          mv3(Ut, y, uz);
#pragma unroll
          for (int q = 0; q < 3; q++) t3[q] = wb[q] - uz[q];
        }
        sing |= inv3q(Ap, Ai);
        mm3(Ai, Lt, C);  // E'_s
        mv3(Ai, t3, y);  // z_s
#pragma unroll
        for (int q = 0; q < 9; q++) SC(s, q) = C[q];
#pragma unroll
        for (int q = 0; q < 3; q++) SC(s, 9 + q) = y[q];
#pragma unroll
        for (int q = 0; q < 9; q++) { Wa[q] = Wb[q]; Wd[q] = R.D[q]; Wb[q] = R.L[q]; }
#pragma unroll
        for (int q = 0; q < 3; q++) wb[q] = R.b[q];
      }
#pragma unroll
      for (int q = 0; q < 9; q++) my[q] = C[q];
#pragma unroll
      for (int q = 0; q < 3; q++) my[9 + q] = y[q];
    }
  }
  if (sing) status[ST_SINGULAR] = 1;
  __syncthreads();
  if (act && top) {  // middle row: the top window now holds U_{m-1}, D_m, U_m, b_m
    block_row<D>(g, m, u, rhs, a, b, mid + 1, n, 0, hs, R);
    tr3(Wa, Lt);
    tr3(Wd, Dt);
    tr3(R.L, Ut);
    double Ub[9], t9b[9], uz[3], ly[3];
    mm3(Ut, my, Ub);
    mv3(Ut, my + 9, uz);
    mm3(Lt, C, t9b);
    mv3(Lt, y, ly);
#pragma unroll
    for (int q = 0; q < 9; q++) Ap[q] = Dt[q] - t9b[q] - Ub[q];
#pragma unroll
    for (int q = 0; q < 3; q++) t3[q] = wb[q] - ly[q] - uz[q];
    inv3(Ap, Ai, status);
    double xm[3];
    mv3(Ai, t3, xm);
    block_store<D>(g, o, a, b, mid, xm);
#pragma unroll
    for (int q = 0; q < 3; q++) my[12 + q] = xm[q];
  }
  __syncthreads();
  if (!act) return;
  double x[3] = {my[12], my[13], my[14]};
  if (top) {
    for (int s = mid - 1; s >= 0; s--) {
#pragma unroll
      for (int q = 0; q < 9; q++) C[q] = SC(s, q);
      double cx[3];
      mv3(C, x, cx);
#pragma unroll
      for (int q = 0; q < 3; q++) x[q] = SC(s, 9 + q) - cx[q];
      block_store<D>(g, o, a, b, s, x);
    }
  } else {
    for (int s = mid + 1; s < n; s++) {
#pragma unroll
      for (int q = 0; q < 9; q++) C[q] = SC(s, q);
      double ex[3];
      mv3(C, x, ex);
#pragma unroll
      for (int q = 0; q < 3; q++) x[q] = SC(s, 9 + q) - ex[q];
      block_store<D>(g, o, a, b, s, x);
    }
  }
#undef SC
}

// Two-ended elimination of a non-cyclic scalar line by two threads, as for
// the block lines: the top thread runs the Thomas recurrence down rows
// 0 .. m-1 (c'_s, y_s), the bottom thread up rows n-1 .. m+1
// (e'_s = a_s / den_s, z_s = (r_s - c_s z_{s+1}) / den_s,
// den_s = b_s - c_s e'_{s+1}); the top thread solves the middle row
//   (b_m - a_m c'_{m-1} - c_m e'_{m+1}) x_m = r_m - a_m y_{m-1} - c_m z_{m+1}
// and both substitute back over their halves.  LDS per lane: e'_{m+1},
// z_{m+1}, x_m.
template <int D, int FAM, class S>
__device__ __forceinline__ void twisted_scalar_line(const Geo &g, const Mat &m, const S &u, const Fields &rhs,
                                    const Out &o, double *__restrict__ sc, long nl, long line, bool act, bool top,
                                    int a, int b, int n, double hs, double *lds, int lane, int *status) {
#define SC(s, q) sc[((long)(s) * 2 + (q)) * nl + line]
  int ofid;
  if (D == 0) ofid = FAM == 0 ? F_UT : F_UF;
  else ofid = FAM == 0 ? F_UR : F_UF;
  constexpr int UNR = (D == 1 && !S::WALL) ? 2 : 1;
  const int mid = n / 2;
  double *my = lds + (long)lane * 15;
  SRow R;
  long xi;
  double *arr;
  double cv = 0.0, yv = 0.0;
  bool sing = false;  // recorded once, after the elimination (as for the block lines)
  if (act) {
    if (top) {
      #pragma unroll UNR
      for (int s = 0; s < mid; s++) {
        scalar_row<D, FAM>(g, m, u, rhs, a, b, s, n, 0, hs, R, xi, arr);
        const double den = R.b - R.a * cv;
        sing |= !(den != 0.0);
        const double id = rcp_nr(den);
        yv = (R.r - R.a * yv) * id;
        cv = R.c * id;
        SC(s, 0) = cv;
        SC(s, 1) = yv;
      }
    } else {
      #pragma unroll UNR
      for (int s = n - 1; s > mid; s--) {
        scalar_row<D, FAM>(g, m, u, rhs, a, b, s, n, 0, hs, R, xi, arr);
        const double den = R.b - R.c * cv;
        sing |= !(den != 0.0);
        const double id = rcp_nr(den);
        yv = (R.r - R.c * yv) * id;
        cv = R.a * id;
        SC(s, 0) = cv;
        SC(s, 1) = yv;
      }
      my[0] = cv;
      my[1] = yv;
    }
  }
  if (sing) status[ST_SINGULAR] = 1;
  __syncthreads();
  if (act && top) { // middle row
    scalar_row<D, FAM>(g, m, u, rhs, a, b, mid, n, 0, hs, R, xi, arr);
    const double den = R.b - R.a * cv - R.c * my[0];
    if (!(den != 0.0)) status[ST_SINGULAR] = 1;
    const double xm = (R.r - R.a * yv - R.c * my[1]) * rcp_nr(den);
    put(o, ofid, xi, xm);
    my[2] = xm;
  }
  __syncthreads();
  if (!act) return;
  double x = my[2];
  if (top) {
    #pragma unroll UNR
    for (int s = mid - 1; s >= 0; s--) {
      x = SC(s, 1) - SC(s, 0) * x;
      put(o, ofid, scalar_index<D, FAM>(g, a, b, s), x);
    }
  } else {
    #pragma unroll UNR
    for (int s = mid + 1; s < n; s++) {
      x = SC(s, 1) - SC(s, 0) * x;
      put(o, ofid, scalar_index<D, FAM>(g, a, b, s), x);
    }
  }
#undef SC
}

// The same for the transposed scalar line: row s of M^T is
// (c_{s-1}, b_s, a_{s+1}) with the right-hand side r_s.  Each thread keeps a
// window of the rows of M around its position (top: c_{s-1}, b_s, c_s, r_s;
// bottom: a_{s+1}, b_s, a_s, r_s), so every row is assembled once.
template <int D, int FAM>
__device__ __forceinline__ void twisted_scalar_line_T(const Geo &g, const Mat &m, const SrcOne &u, const Fields &rhs,
                                      const Out &o, double *__restrict__ sc, long nl, long line, bool act, bool top,
                                      int a, int b, int n, double hs, double *lds, int lane, int *status) {
#define SC(s, q) sc[((long)(s) * 2 + (q)) * nl + line]
  int ofid;
  if (D == 0) ofid = FAM == 0 ? F_UT : F_UF;
  else ofid = FAM == 0 ? F_UR : F_UF;
  const int mid = n / 2;
  double *my = lds + (long)lane * 15;
  SRow R;
  long xi;
  double *arr;
  double cv = 0.0, yv = 0.0;
  double w0 = 0.0, wb = 0.0, w1 = 0.0, wr = 0.0; // window
  bool sing = false;  // a zero pivot, recorded once after the elimination
  if (act) {
    if (top) {
      // w0 = c_{s-1}, wb = b_s, w1 = c_s, wr = r_s
      scalar_row<D, FAM>(g, m, u, rhs, a, b, 0, n, 0, hs, R, xi, arr);
      wb = R.b; w1 = R.c; wr = R.r;
      for (int s = 0; s < mid; s++) {
        scalar_row<D, FAM>(g, m, u, rhs, a, b, s + 1, n, 0, hs, R, xi, arr);
        const double at = w0, bt = wb, ct = R.a, rt = wr; // transposed row s
        const double den = bt - at * cv;
        sing |= !(den != 0.0);
        const double id = rcp_nr(den);
        yv = (rt - at * yv) * id;
        cv = ct * id;
        SC(s, 0) = cv;
        SC(s, 1) = yv;
        w0 = w1; wb = R.b; w1 = R.c; wr = R.r;
      }
    } else {
      // w0 = a_{s+1}, wb = b_s, w1 = a_s, wr = r_s
      scalar_row<D, FAM>(g, m, u, rhs, a, b, n - 1, n, 0, hs, R, xi, arr);
      wb = R.b; w1 = R.a; wr = R.r;
      for (int s = n - 1; s > mid; s--) {
        scalar_row<D, FAM>(g, m, u, rhs, a, b, s - 1, n, 0, hs, R, xi, arr);
        const double at = R.c, bt = wb, ct = w0, rt = wr; // transposed row s
        const double den = bt - ct * cv;
        sing |= !(den != 0.0);
        const double id = rcp_nr(den);
        yv = (rt - ct * yv) * id;
        cv = at * id;
        SC(s, 0) = cv;
        SC(s, 1) = yv;
        w0 = w1; wb = R.b; w1 = R.a; wr = R.r;
      }
      my[0] = cv;
      my[1] = yv;
    }
  }
  if (sing) status[ST_SINGULAR] = 1;
  __syncthreads();
  if (act && top) { // middle row (c_{m-1}, b_m, a_{m+1}): the top window holds c_{m-1}, b_m, r_m
    scalar_row<D, FAM>(g, m, u, rhs, a, b, mid + 1, n, 0, hs, R, xi, arr);
    const double at = w0, bt = wb, ct = R.a, rt = wr;
    const double den = bt - at * cv - ct * my[0];
    if (!(den != 0.0)) status[ST_SINGULAR] = 1;
    const double xm = (rt - at * yv - ct * my[1]) * rcp_nr(den);
    put(o, ofid, scalar_index<D, FAM>(g, a, b, mid), xm);
    my[2] = xm;
  }
  __syncthreads();
  if (!act) return;
  double x = my[2];
  if (top) {
    for (int s = mid - 1; s >= 0; s--) {
      x = SC(s, 1) - SC(s, 0) * x;
      put(o, ofid, scalar_index<D, FAM>(g, a, b, s), x);
    }
  } else {
    for (int s = mid + 1; s < n; s++) {
      x = SC(s, 1) - SC(s, 0) * x;
      put(o, ofid, scalar_index<D, FAM>(g, a, b, s), x);
    }
  }
#undef SC
}

// r and theta sweeps: workgroups [0, nbw) take the block lines, two threads
// per line (blockDim/2 lines per workgroup), the rest one scalar line per
// thread
__host__ __device__ inline unsigned twisted_block_wgs(const Geo &g, int d, unsigned bs) {
  const Families F = families(g, d);
  const unsigned lpw = bs / 2;
  return (unsigned)((F.nb + lpw - 1) / lpw);
}

// W: a forced pass (the coefficients see the wall velocities); PT: the
// perturbation-pressure form
template <int D, bool TR = false, bool W = false, bool PT = false>
__device__ __forceinline__ void sweep2_body(const PassArgs &a, unsigned w, double *lds) {
  const Geo &g = a.g;
  decltype(auto) u = SrcSel<W, PT>::get(a);
  const Families F = families(g, D);
  const double hs = a.tau;
  const unsigned nbw = twisted_block_wgs(g, D, blockDim.x);
  if (w < nbw) {
    const unsigned lpw = blockDim.x / 2;
    const unsigned lane = threadIdx.x % lpw;
    const bool top = threadIdx.x < lpw;
    const long line = (long)w * lpw + lane;
    const bool act = line < F.nb;
    int p = 0, q = 0;
    if (act) { p = (int)(line / g.np); q = (int)(line % g.np); }
    if (act && top && a.o.mode == 0) zero_bnd<D>(g, a.o.x, p, q);
    if constexpr (TR)
      twisted_block_line_T<D>(g, a.m, a.u, a.rhs, a.o, a.scb, F.nb, line, act, top, p, q, F.n, hs, lds,
                              (int)lane, a.status);
    else
      twisted_block_line<D>(g, a.m, u, a.rhs, a.o, a.scb, F.nb, line, act, top, p, q, F.n, hs, lds,
                            (int)lane, a.status);
    return;
  }
  // scalar lines two-ended too: blockDim/2 lines per workgroup, each
  // workgroup within one family (so its barriers are uniform)
  const long ns = (long)F.na + F.nbb;
  const int nkf = g.periodic ? g.np : g.np - 1, kf0 = g.periodic ? 0 : 1;
  const unsigned lpw = blockDim.x / 2;
  const unsigned lane = threadIdx.x % lpw;
  const bool top = threadIdx.x < lpw;
  const unsigned nwa = (unsigned)((F.na + lpw - 1) / lpw);
  // this grid's scalar workgroups, numbered XCD-contiguously (lines of
  // neighbouring families share cells): r sweep 1.46 -> 1.42 ms on the
  // global grid; the transposed sweeps of the adjoint gain a little too
  const unsigned nws = nwa + (unsigned)((F.nbb + lpw - 1) / lpw);
  const unsigned w2 = xcd_contiguous(w - nbw, nws);
  if (w2 < nwa) {
    const long line = (long)w2 * lpw + lane;
    const bool act = line < F.na;
    int p = 1, q = 0;
    if (act) { p = 1 + (int)(line / g.np); q = (int)(line % g.np); }
    if constexpr (TR)
      twisted_scalar_line_T<D, 0>(g, a.m, a.u, a.rhs, a.o, a.scs, ns, line, act, top, p, q, F.n, hs, lds,
                                  (int)lane, a.status);
    else
      twisted_scalar_line<D, 0>(g, a.m, u, a.rhs, a.o, a.scs, ns, line, act, top, p, q, F.n, hs, lds,
                                (int)lane, a.status);
  } else {
    const long l3 = (long)(w2 - nwa) * lpw + lane;
    const bool act = l3 < F.nbb;
    int p = 0, q = kf0;
    if (act) { p = (int)(l3 / nkf); q = kf0 + (int)(l3 % nkf); }
    if constexpr (TR)
      twisted_scalar_line_T<D, 1>(g, a.m, a.u, a.rhs, a.o, a.scs, ns, F.na + l3, act, top, p, q, F.n, hs, lds,
                                  (int)lane, a.status);
    else
      twisted_scalar_line<D, 1>(g, a.m, u, a.rhs, a.o, a.scs, ns, F.na + l3, act, top, p, q, F.n, hs, lds,
                                (int)lane, a.status);
  }
}

template <int D, bool B>
__global__ void __launch_bounds__(256) DSW_OCC(DSW_WAVES_SWEEP) k_sweep2(PassArgs a, Batch bt) {
  __shared__ double lds[128 * 15];
  if constexpr (B) {
    const int mb = batch_member(bt, blockIdx.x);
    sweep2_body<D>(batch_args(bt, mb), blockIdx.x - bt.woff[mb], lds);
  } else {
    sweep2_body<D>(a, blockIdx.x, lds);
  }
}

// forced split step, one grid
template <int D>
__global__ void __launch_bounds__(256) DSW_OCC(DSW_WAVES_SWEEP) k_sweep2F(PassArgs a) {
  __shared__ double lds[128 * 15];
  sweep2_body<D, false, true>(a, blockIdx.x, lds);
}

// perturbation-pressure form, one grid
template <int D>
__global__ void __launch_bounds__(256) DSW_OCC(DSW_WAVES_SWEEP) k_sweep2P(PassArgs a) {
  __shared__ double lds[128 * 15];
  sweep2_body<D, false, false, true>(a, blockIdx.x, lds);
}

void launch_sweep2_pert(int d, const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st) {
  if (d == 0) hipLaunchKernelGGL(k_sweep2P<0>, dim3(blocks), dim3(threads), 0, st, a);
  else hipLaunchKernelGGL(k_sweep2P<1>, dim3(blocks), dim3(threads), 0, st, a);
}

void launch_sweep2_forced(int d, const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st) {
  if (d == 0) hipLaunchKernelGGL(k_sweep2F<0>, dim3(blocks), dim3(threads), 0, st, a);
  else hipLaunchKernelGGL(k_sweep2F<1>, dim3(blocks), dim3(threads), 0, st, a);
}

// transposed systems (adjoint), one grid
template <int D>
__global__ void __launch_bounds__(256) k_sweep2T(PassArgs a) {
  __shared__ double lds[128 * 15];
  sweep2_body<D, true>(a, blockIdx.x, lds);
}

void launch_sweep2_T(int d, const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st) {
  if (d == 0) hipLaunchKernelGGL(k_sweep2T<0>, dim3(blocks), dim3(threads), 0, st, a);
  else hipLaunchKernelGGL(k_sweep2T<1>, dim3(blocks), dim3(threads), 0, st, a);
}

// workgroups of a two-ended r or theta sweep: the block lines, then the
// scalar lines of each family, two threads per line
unsigned sweep2_block_blocks(const Geo &g, int d, unsigned bs) { return twisted_block_wgs(g, d, bs); }

unsigned sweep2_blocks(const Geo &g, int d, unsigned bs) {
  const Families F = families(g, d);
  const long lpw = bs / 2;
  return twisted_block_wgs(g, d, bs) + (unsigned)((F.na + lpw - 1) / lpw) + (unsigned)((F.nbb + lpw - 1) / lpw);
}

void launch_sweep2_pass(int d, const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                        hipStream_t st) {
  const dim3 gr(blocks), bl(threads);
  if (b.tab) {
    if (d == 0) hipLaunchKernelGGL((k_sweep2<0, true>), gr, bl, 0, st, a, b);
    else hipLaunchKernelGGL((k_sweep2<1, true>), gr, bl, 0, st, a, b);
  } else {
    if (d == 0) hipLaunchKernelGGL((k_sweep2<0, false>), gr, bl, 0, st, a, b);
    else hipLaunchKernelGGL((k_sweep2<1, false>), gr, bl, 0, st, a, b);
  }
}

void sweep_scratch_size(const Geo &g, long *blk, long *sca) {
  long b = 0, s = 0;
  for (int d = 0; d < 3; d++) {
    const Families F = families(g, d);
    const long per = 21, pers = 3; // transposed and cyclic solvers need the most
    b = b > per * F.n * (long)F.nb ? b : per * F.n * (long)F.nb;
    const long ss = pers * F.n * ((long)F.na + F.nbb);
    s = s > ss ? s : ss;
  }
  *blk = b;
  *sca = s;
}

unsigned sweep_lines(const Geo &g, int d) {
  const Families F = families(g, d);
  return (unsigned)((long)F.nb + F.na + F.nbb);
}

void launch_sweep_pass(int d, const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                       hipStream_t st) {
  const dim3 gr(blocks), bl(threads);
  if (b.tab) {
    if (d == 0) hipLaunchKernelGGL((k_sweep<0, true>), gr, bl, 0, st, a, b);
    else if (d == 1) hipLaunchKernelGGL((k_sweep<1, true>), gr, bl, 0, st, a, b);
    else hipLaunchKernelGGL((k_sweep<2, true>), gr, bl, 0, st, a, b);
  } else {
    if (d == 0) hipLaunchKernelGGL((k_sweep<0, false>), gr, bl, 0, st, a, b);
    else if (d == 1) hipLaunchKernelGGL((k_sweep<1, false>), gr, bl, 0, st, a, b);
    else hipLaunchKernelGGL((k_sweep<2, false>), gr, bl, 0, st, a, b);
  }
}

// boundary-normal faces: u_r on r = r1, r2; u_theta on the theta boundaries;
// u_phi on the phi walls (sector only).  FORCED: d0 takes the Dirichlet data
// of the new time level (rhs; src's own when rhs is unset), d1 and d2 the
// midpoint of src's and those
template <bool FORCED = false>
__device__ __forceinline__ void bnd_body(const PassArgs &a, unsigned w) {
  const Geo &g = a.g;
  const long t = (long)w * blockDim.x + threadIdx.x;
  const long nr_ = (long)g.nt * g.np, nt_ = (long)g.nr * g.np, nf_ = g.periodic ? 0 : (long)g.nr * g.nt;
  long idx;
  int fid;
  if (t < 2 * nr_) {
    const long q = t % nr_;
    idx = idx_r(g, t < nr_ ? 0 : g.nr, (int)(q / g.np), (int)(q % g.np));
    fid = F_UR;
  } else if (t < 2 * nr_ + 2 * nt_) {
    const long u = t - 2 * nr_, q = u % nt_;
    idx = idx_t(g, (int)(q / g.np), u < nt_ ? 0 : g.nt, (int)(q % g.np));
    fid = F_UT;
  } else if (t < 2 * nr_ + 2 * nt_ + 2 * nf_) {
    const long u = t - 2 * nr_ - 2 * nt_, q = u % nf_;
    idx = idx_f(g, (int)(q / g.nt), (int)(q % g.nt), u < nf_ ? 0 : g.np);
    fid = F_UF;
  } else {
    return;
  }
  const double v = fsel(a.src, fid)[idx];
  if constexpr (FORCED) {
    const double vb = a.rhs.ur ? fsel(a.rhs, fid)[idx] : v, mid = 0.5 * (vb + v);
    fsel(a.d0, fid)[idx] = vb;
    fsel(a.d1, fid)[idx] = mid;
    fsel(a.d2, fid)[idx] = mid;
    return;
  }
  if (a.d0.p) fsel(a.d0, fid)[idx] = v;
  if (a.d1.p) fsel(a.d1, fid)[idx] = v;
  if (a.d2.p) fsel(a.d2, fid)[idx] = v;
}


// ------------------------------------------------ lifted boundary data --

// The first iteration of a forced step starts from U^n, old boundary data
// included; the change of the data to the new time level enters the
// increment solve of direction D as inhomogeneous Dirichlet data on the walls
// normal to D.  With X = X_0 + X_b (X_b zero but on those walls), X_0 solves
// the homogeneous line systems with the right-hand side rhs - tau/2 D_D X_b.
// This kernel subtracts that term in place (a.rhs) on the rows that see X_b:
// the end blocks of each block line, through the boundary faces of the
// normal velocity (X_b = a.d0 - a.src there: the new data less U^n's), and
// the end rows of each scalar line that ends on a wall, through the ghost
// value 2 dw - x of the tangential velocity (dw: the change of the wall
// velocity).  Rows next to a pole see no data.  One thread per line; the
// coefficients come from Ubar (a.u, wall data a.wall) as in the sweeps.
template <int D, int FAM>
__device__ __forceinline__ void lift_scalar(const PassArgs &a, const SrcW &u, const Wall &dw, int p, int q,
                                            int n, double hs) {
  const Geo &g = a.g;
  double dlo = 0.0, dhi = 0.0;
  if (D == 0 && FAM == 0) { dlo = wallv(dw.ut_r1, (long)p * g.np + q); dhi = wallv(dw.ut_r2, (long)p * g.np + q); }
  if (D == 0 && FAM == 1) { dlo = wallv(dw.uf_r1, (long)p * g.npf + q); dhi = wallv(dw.uf_r2, (long)p * g.npf + q); }
  if (D == 1 && FAM == 0) {
    if (!g.pole_lo) dlo = wallv(dw.ur_t1, (long)p * g.np + q);
    if (!g.pole_hi) dhi = wallv(dw.ur_t2, (long)p * g.np + q);
  }
  if (D == 1 && FAM == 1) {
    if (!g.pole_lo) dlo = wallv(dw.uf_t1, (long)p * g.npf + q);
    if (!g.pole_hi) dhi = wallv(dw.uf_t2, (long)p * g.npf + q);
  }
  if (D == 2 && FAM == 0) { dlo = wallv(dw.ur_p1, (long)p * g.nt + q); dhi = wallv(dw.ur_p2, (long)p * g.nt + q); }
  if (D == 2 && FAM == 1) { dlo = wallv(dw.ut_p1, (long)p * (g.nt + 1) + q); dhi = wallv(dw.ut_p2, (long)p * (g.nt + 1) + q); }
  SRow R;
  long xi;
  double *arr;
  Edge e;
  if (dlo != 0.0) {
    scalar_row<D, FAM>(g, a.m, u, a.rhs, p, q, 0, n, 0, hs, R, xi, arr, &e);
    arr[xi] -= 2.0 * e.slo * dlo;
  }
  if (dhi != 0.0) {
    scalar_row<D, FAM>(g, a.m, u, a.rhs, p, q, n - 1, n, 0, hs, R, xi, arr, &e);
    arr[xi] -= 2.0 * e.shi * dhi;
  }
}

template <int D>
__global__ void __launch_bounds__(256) k_lift(PassArgs a, Wall dw) {
  const Geo &g = a.g;
  const Families F = families(g, D);
  if (F.cyclic) return;  // no walls normal to a periodic direction
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nkf = g.periodic ? g.np : g.np - 1, kf0 = g.periodic ? 0 : 1;
  const double hs = a.tau;
  const SrcW u = SrcSel<true>::get(a);
  const int n = F.n;
  if (t < F.nb) {
    if (!a.d0.ur) return;  // the normal data keep U^n's
    int p, q;
    if (D == 2) { p = (int)(t / g.nt); q = (int)(t % g.nt); }
    else { p = (int)(t / g.np); q = (int)(t % g.np); }
    auto cell = [&](int s) { return D == 0 ? idx_c(g, s, p, q) : (D == 1 ? idx_c(g, p, s, q) : idx_c(g, p, q, s)); };
    auto face = [&](int f) { return D == 0 ? idx_r(g, f, p, q) : (D == 1 ? idx_t(g, p, f, q) : idx_f(g, p, q, f)); };
    const int wf = D == 0 ? F_UR : (D == 1 ? F_UT : F_UF);
    const double *nw = fsel(a.d0, wf), *od = fsel(a.src, wf);
    double *rw = fsel(a.rhs, wf);
    const double dlo = nw[face(0)] - od[face(0)], dhi = nw[face(n)] - od[face(n)];
    BRow R;
    Edge e;
    if (dlo != 0.0) {
      block_row<D>(g, a.m, u, a.rhs, p, q, 0, n, 0, hs, R, &e);
      a.rhs.p[cell(0)] -= e.lo[0] * dlo;
      a.rhs.T[cell(0)] -= e.lo[1] * dlo;
      rw[face(1)] -= e.lo[2] * dlo;
    }
    if (dhi != 0.0) {
      block_row<D>(g, a.m, u, a.rhs, p, q, n - 1, n, 0, hs, R, &e);
      a.rhs.p[cell(n - 1)] -= e.hi[0] * dhi;
      a.rhs.T[cell(n - 1)] -= e.hi[1] * dhi;
      block_row<D>(g, a.m, u, a.rhs, p, q, n - 2, n, 0, hs, R, &e);
      rw[face(n - 1)] -= e.hiw * dhi;
    }
    return;
  }
  long t2 = t - F.nb;
  if (t2 < F.na) {
    const int p = 1 + (int)(t2 / (D == 2 ? g.nt : g.np)), q = (int)(t2 % (D == 2 ? g.nt : g.np));
    lift_scalar<D, 0>(a, u, dw, p, q, n, hs);
    return;
  }
  t2 -= F.na;
  if (t2 < F.nbb) {
    int p, q;
    if (D == 2) { p = (int)(t2 / (g.nt - 1)); q = 1 + (int)(t2 % (g.nt - 1)); }
    else { p = (int)(t2 / nkf); q = kf0 + (int)(t2 % nkf); }
    lift_scalar<D, 1>(a, u, dw, p, q, n, hs);
  }
}

void launch_lift(int d, const PassArgs &a, const Wall &dw, hipStream_t st) {
  const unsigned lines = sweep_lines(a.g, d);
  const dim3 gr((lines + 255) / 256), bl(256);
  if (d == 0) hipLaunchKernelGGL(k_lift<0>, gr, bl, 0, st, a, dw);
  else if (d == 1) hipLaunchKernelGGL(k_lift<1>, gr, bl, 0, st, a, dw);
  else hipLaunchKernelGGL(k_lift<2>, gr, bl, 0, st, a, dw);
}

// the mean and the change of two sets of wall velocities (a null array is zero)
__global__ void __launch_bounds__(256) k_wall_mix(WallMix w) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= w.off[12]) return;
  int q = 0;
  while (t >= w.off[q + 1]) q++;
  const long e = t - w.off[q];
  const double x = w.a[q] ? w.a[q][e] : 0.0, y = w.b[q] ? w.b[q][e] : 0.0;
  w.mid[q][e] = 0.5 * (x + y);
  w.dw[q][e] = y - x;
}

void launch_wall_mix(const WallMix &w, hipStream_t st) {
  if (w.off[12] > 0) hipLaunchKernelGGL(k_wall_mix, dim3((unsigned)((w.off[12] + 255) / 256)), dim3(256), 0, st, w);
}

__global__ void __launch_bounds__(256) k_bnd_forced(PassArgs a) { bnd_body<true>(a, blockIdx.x); }

void launch_bnd_forced(const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st) {
  hipLaunchKernelGGL(k_bnd_forced, dim3(blocks), dim3(threads), 0, st, a);
}

template <bool B>
__global__ void __launch_bounds__(256) k_bnd_copy(PassArgs a, Batch bt) {
  if constexpr (B) {
    const int mb = batch_member(bt, blockIdx.x);
    bnd_body(batch_args(bt, mb), blockIdx.x - bt.woff[mb]);
  } else {
    bnd_body(a, blockIdx.x);
  }
}

unsigned bnd_points(const Geo &g) {
  return (unsigned)(2L * g.nt * g.np + 2L * g.nr * g.np + (g.periodic ? 0 : 2L * g.nr * g.nt));
}

void launch_bnd_pass(const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                     hipStream_t st) {
  if (b.tab) hipLaunchKernelGGL(k_bnd_copy<true>, dim3(blocks), dim3(threads), 0, st, a, b);
  else hipLaunchKernelGGL(k_bnd_copy<false>, dim3(blocks), dim3(threads), 0, st, a, b);
}

} // namespace dsw
