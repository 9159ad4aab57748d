// phi_part.hip -- partitioned line solver for the phi sweep (paper eq. (spl3),
// operator D_phi of Appendix B eq. (dphi)).
//
// One workgroup per line slot (i, j).  It solves the 3x3-block line in
// (p, T, u_phi) and the two scalar lines (u_r on r-face i, u_theta on
// theta-face j) that share that slot.  Thread t owns rows [4t, 4t + 4):
//   1. it assembles its rows (consecutive threads read consecutive phi cells:
//      contiguous loads) and eliminates its interior rows with the block
//      Thomas recurrence, carrying the dependence on the previous chunk's last
//      row ("spike"), then sweeps back so that every interior row reads
//      x_q = g_q + V_q x_left + W_q x_sep;
//   2. the chunks' last rows ("separators") form a block-tridiagonal system
//      (cyclic when phi is periodic) that is solved in LDS by parallel cyclic
//      reduction, log2(#chunks) steps;
//   3. interior rows are filled in from the separators.
// All intermediates stay in registers and LDS: no scratch traffic.
#include <algorithm>

#include "rows.hpp"

namespace dsw {

constexpr int PT_MAX = 256;  // chunks per line (lines up to PM * 256 cells)

template <int PM>
__host__ __device__ inline int part_chunks(int n) { return (n + PM - 1) / PM; }

// ---------------------------------------------------------- 3x3 helpers --
__device__ __forceinline__ void mm3s(const double *A, const double *B, double *C, double s) {
  mm3(A, B, C);
#pragma unroll
  for (int q = 0; q < 9; q++) C[q] *= s;
}

// ------------------------------------------------------- block: PCR step --
// Solve the T separator rows A x_{t-1} + B x_t + C x_{t+1} = r (t < T) held
// in registers of threads t < T; returns x_t.  Each step, every row
// publishes B^{-1} A, B^{-1} C and B^{-1} r (LDS: 21 T doubles) and
// eliminates its neighbours h rows away from them.
__device__ __forceinline__ void pcr_block(int t, int T, int cyc, double *A, double *B, double *C, double *r,
                          double *lds, double *x, int *status) {
  double *sPA = lds, *sPC = lds + 9 * T, *sPr = lds + 18 * T;
  const bool act = t < T;
  for (int h = 1; h < T; h *= 2) {
    if (act) {
      double Bi[9];
      inv3(B, Bi, status);
      mm3(Bi, A, &sPA[t * 9]);
      mm3(Bi, C, &sPC[t * 9]);
      mv3(Bi, r, &sPr[t * 3]);
    }
    __syncthreads();
    if (act) {
      int lo = t - h, hi = t + h;
      bool has_lo = lo >= 0, has_hi = hi < T;
      if (cyc) { lo &= T - 1; hi &= T - 1; has_lo = has_hi = true; }  // cyclic: T a power of two
      // B' = B - A P_C(lo) - C P_A(hi), r' alike, A' = -A P_A(lo),
      // C' = -C P_C(hi) (P = B^{-1} times the published row)
      if (has_lo) { mm3_sub(A, &sPC[lo * 9], B); mv3_sub(A, &sPr[lo * 3], r); }
      if (has_hi) { mm3_sub(C, &sPA[hi * 9], B); mv3_sub(C, &sPr[hi * 3], r); }
      if (has_lo) mm3_neg_inplace(A, &sPA[lo * 9]);
      else {
#pragma unroll
        for (int q = 0; q < 9; q++) A[q] = 0.0;
      }
      if (has_hi) mm3_neg_inplace(C, &sPC[hi * 9]);
      else {
#pragma unroll
        for (int q = 0; q < 9; q++) C[q] = 0.0;
      }
    }
    __syncthreads();
  }
  if (act) {
    // every remaining coupling points at x_t itself (cyclic) or is zero
    double S[9], Si[9];
#pragma unroll
    for (int q = 0; q < 9; q++) S[q] = A[q] + B[q] + C[q];
    inv3(S, Si, status);
    mv3(Si, r, x);
  }
}

__device__ __forceinline__ void pcr_scalar(int t, int T, int cyc, double &A, double &B, double &C, double &r,
                           double *lds, double &x, int *status) {
  double *sA = lds, *sC = lds + T, *sR = lds + 2 * T, *sB = lds + 3 * T;
  const bool act = t < T;
  for (int h = 1; h < T; h *= 2) {
    if (act) { sA[t] = A; sC[t] = C; sR[t] = r; sB[t] = B; }
    __syncthreads();
    if (act) {
      int lo = t - h, hi = t + h;
      bool has_lo = lo >= 0, has_hi = hi < T;
      if (cyc) { lo &= T - 1; hi &= T - 1; has_lo = has_hi = true; }  // cyclic: T a power of two
      double nA = 0.0, nC = 0.0, nB = B, nr = r;
      if (has_lo) {
        const double al = -A * rcp_nr(sB[lo]);
        nA = al * sA[lo];
        nB += al * sC[lo];
        nr += al * sR[lo];
      }
      if (has_hi) {
        const double be = -C * rcp_nr(sB[hi]);
        nC = be * sC[hi];
        nB += be * sA[hi];
        nr += be * sR[hi];
      }
      A = nA; B = nB; C = nC; r = nr;
    }
    __syncthreads();
  }
  if (act) {
    const double S = A + B + C;
    if (!(S != 0.0)) status[ST_SINGULAR] = 1;
    x = r * rcp_nr(S);
  }
}

// Two independent scalar systems of the same size T, reduced side by side:
// the steps of pcr_scalar for each, under one set of barriers.  LDS: system
// f at lds + 4 T f (8 T doubles).
__device__ __forceinline__ void pcr_scalar2(int t, int T, int cyc, double *A, double *B, double *C, double *r,
                                            double *lds, double *x, int *status) {
  const bool act = t < T;
  for (int h = 1; h < T; h *= 2) {
    if (act) {
#pragma unroll
      for (int f = 0; f < 2; f++) {
        double *L = lds + 4 * T * f;
        L[t] = A[f]; L[T + t] = C[f]; L[2 * T + t] = r[f]; L[3 * T + t] = B[f];
      }
    }
    __syncthreads();
    if (act) {
      int lo = t - h, hi = t + h;
      bool has_lo = lo >= 0, has_hi = hi < T;
      if (cyc) { lo &= T - 1; hi &= T - 1; has_lo = has_hi = true; }  // cyclic: T a power of two
#pragma unroll
      for (int f = 0; f < 2; f++) {
        const double *sA = lds + 4 * T * f, *sC = sA + T, *sR = sA + 2 * T, *sB = sA + 3 * T;
        double nA = 0.0, nC = 0.0, nB = B[f], nr = r[f];
        if (has_lo) {
          const double al = -A[f] * rcp_nr(sB[lo]);
          nA = al * sA[lo];
          nB += al * sC[lo];
          nr += al * sR[lo];
        }
        if (has_hi) {
          const double be = -C[f] * rcp_nr(sB[hi]);
          nC = be * sC[hi];
          nB += be * sA[hi];
          nr += be * sR[hi];
        }
        A[f] = nA; B[f] = nB; C[f] = nC; r[f] = nr;
      }
    }
    __syncthreads();
  }
  if (act) {
#pragma unroll
    for (int f = 0; f < 2; f++) {
      const double S = A[f] + B[f] + C[f];
      if (!(S != 0.0)) status[ST_SINGULAR] = 1;
      x[f] = r[f] * rcp_nr(S);
    }
  }
}

// ------------------------------------------------------------ block line --
template <int PM, bool TR, class US>
__device__ __forceinline__ void part_block_line(const Geo &g, const Mat &m, const US &u, const Fields &rhs,
                                const Out &o, int i, int j, double hs, double *lds, int *status) {
  const int N = g.np, T = part_chunks<PM>(N), cyc = g.periodic;
  const int t = threadIdx.x;
  const bool act = t < T;
  const int a0 = t * PM;
  const int len = act ? min(PM, N - a0) : 0;
  double Cm[PM - 1][9], Em[PM - 1][9], Ym[PM - 1][3];
  // structural non-zeros of the row blocks (transposed rows: L = U^T, U = L^T)
  constexpr unsigned mL = TR ? nz_tr(NZ_U) : NZ_L, mU = TR ? nz_tr(NZ_L) : NZ_U;
  BRow R;
  TrWalk<2> tw; // transposed rows: each row of the line assembled once
  if constexpr (TR) {
    if (act) tw.init(g, m, u, rhs, i, j, a0, N, cyc, hs);
  }
  // a zero pivot is recorded after the loop: a store inside it would hold
  // the next row's loads back
  bool sing = false;
  // 1. forward elimination over interior rows with the left spike
#pragma unroll
  for (int q = 0; q < PM - 1; q++) {
    if (q < len - 1) {
      if constexpr (TR) tw.next(g, m, u, rhs, i, j, N, cyc, hs, R);
      else block_row<2>(g, m, u, rhs, i, j, a0 + q, N, cyc, hs, R);
      double Dp[9], rr[3], Lx[9], Ai[9];
      if (q == 0) {
#pragma unroll
        for (int z = 0; z < 9; z++) Dp[z] = R.D[z];
#pragma unroll
        for (int z = 0; z < 3; z++) rr[z] = R.b[z];
      } else {
        double t9[9], t3[3];
        mm3m<mL, NZ_ALL>(R.L, Cm[q - 1], t9);
#pragma unroll
        for (int z = 0; z < 9; z++) Dp[z] = R.D[z] - t9[z];
        mv3m<mL>(R.L, Ym[q - 1], t3);
#pragma unroll
        for (int z = 0; z < 3; z++) rr[z] = R.b[z] - t3[z];
        mm3m<mL, NZ_ALL>(R.L, Em[q - 1], Lx);
#pragma unroll
        for (int z = 0; z < 9; z++) Lx[z] *= -1.0;
      }
      sing |= inv3q(Dp, Ai);
      mm3m<NZ_ALL, mU>(Ai, R.U, Cm[q]);
      mv3(Ai, rr, Ym[q]);
      if (q == 0) mm3m<NZ_ALL, mL>(Ai, R.L, Em[q]);
      else mm3(Ai, Lx, Em[q]);
    }
  }
  if (sing) status[ST_SINGULAR] = 1;
  // separator row (last row of the chunk)
  BRow S;
  if (act) {
    if constexpr (TR) tw.next(g, m, u, rhs, i, j, N, cyc, hs, S);
    else block_row<2>(g, m, u, rhs, i, j, a0 + len - 1, N, cyc, hs, S);
  }
  // backward sweep: (Y, E, C) -> (g, V, W), x_q = g_q + V_q x_left + W_q x_sep
#pragma unroll
  for (int q = PM - 2; q >= 0; q--) {
    if (q == len - 2) {
#pragma unroll
      for (int z = 0; z < 9; z++) { Em[q][z] = -Em[q][z]; Cm[q][z] = -Cm[q][z]; }
    } else if (q < len - 2) {
      double t9[9], t3[3];
      mv3(Cm[q], Ym[q + 1], t3);
#pragma unroll
      for (int z = 0; z < 3; z++) Ym[q][z] -= t3[z];
      mm3(Cm[q], Em[q + 1], t9);
#pragma unroll
      for (int z = 0; z < 9; z++) Em[q][z] = -Em[q][z] - t9[z];
      mm3s(Cm[q], Cm[q + 1], t9, -1.0);
#pragma unroll
      for (int z = 0; z < 9; z++) Cm[q][z] = t9[z];
    }
  }
  // 2. exchange the first interior row of each chunk with its left neighbour
  double *sG = lds, *sV = lds + 3 * T, *sW = lds + 12 * T, *sL = lds + 21 * T;
  if (act) {
    sL[t] = (double)len;
    if (len >= 2) {
#pragma unroll
      for (int z = 0; z < 3; z++) sG[t * 3 + z] = Ym[0][z];
#pragma unroll
      for (int z = 0; z < 9; z++) { sV[t * 9 + z] = Em[0][z]; sW[t * 9 + z] = Cm[0][z]; }
    }
  }
  __syncthreads();
  double A[9], B[9], Cc[9], r[3];
  if (act) {
    int nt_ = t + 1;
    bool has_next = nt_ < T;
    if (cyc) { nt_ %= T; has_next = true; }
    const int nlen = has_next ? (int)sL[nt_] : 0;
    // last interior row of this chunk
    double Gl[3] = {0, 0, 0}, Vl[9], Wl[9];
#pragma unroll
    for (int z = 0; z < 9; z++) { Vl[z] = 0.0; Wl[z] = 0.0; }
#pragma unroll
    for (int q = 0; q < PM - 1; q++)
      if (q == len - 2) {
#pragma unroll
        for (int z = 0; z < 3; z++) Gl[z] = Ym[q][z];
#pragma unroll
        for (int z = 0; z < 9; z++) { Vl[z] = Em[q][z]; Wl[z] = Cm[q][z]; }
      }
    double t9[9], t3[3];
#pragma unroll
    for (int z = 0; z < 9; z++) B[z] = S.D[z];
#pragma unroll
    for (int z = 0; z < 3; z++) r[z] = S.b[z];
    if (len >= 2) {
      mm3m<mL, NZ_ALL>(S.L, Vl, A);
      mm3m<mL, NZ_ALL>(S.L, Wl, t9);
#pragma unroll
      for (int z = 0; z < 9; z++) B[z] += t9[z];
      mv3m<mL>(S.L, Gl, t3);
#pragma unroll
      for (int z = 0; z < 3; z++) r[z] -= t3[z];
    } else {
#pragma unroll
      for (int z = 0; z < 9; z++) A[z] = S.L[z];
    }
    if (nlen >= 2) {
      mm3m<mU, NZ_ALL>(S.U, &sV[nt_ * 9], t9);
#pragma unroll
      for (int z = 0; z < 9; z++) B[z] += t9[z];
      mm3m<mU, NZ_ALL>(S.U, &sW[nt_ * 9], Cc);
      mv3m<mU>(S.U, &sG[nt_ * 3], t3);
#pragma unroll
      for (int z = 0; z < 3; z++) r[z] -= t3[z];
    } else {
#pragma unroll
      for (int z = 0; z < 9; z++) Cc[z] = S.U[z];
    }
  }
  __syncthreads(); // exchange area is reused by the reduction
  double xs[3] = {0, 0, 0};
  pcr_block(t, T, cyc, A, B, Cc, r, lds, xs, status);
  // 3. fill in the interior rows
  double *sX = lds + 21 * T;
  if (act) {
#pragma unroll
    for (int z = 0; z < 3; z++) sX[t * 3 + z] = xs[z];
  }
  __syncthreads();
  double val[PM][3];
  if (act) {
    double xl[3] = {0, 0, 0};
    if (t > 0 || cyc) {
      const int lt = t > 0 ? t - 1 : T - 1;
#pragma unroll
      for (int z = 0; z < 3; z++) xl[z] = sX[lt * 3 + z];
    }
#pragma unroll
    for (int q = 0; q < PM - 1; q++) {
      if (q < len - 1) {
        double t3[3];
        mv3(Em[q], xl, val[q]);
        mv3(Cm[q], xs, t3);
#pragma unroll
        for (int z = 0; z < 3; z++) val[q][z] += Ym[q][z] + t3[z];
      }
    }
  }
  __syncthreads(); // every thread has read the separators: the LDS is free
  // stage the solution in LDS and store it row-contiguously (whole lines
  // per store instruction instead of a 4-row stride across lanes)
  double *sP = lds, *sT_ = lds + N, *sWv = lds + 2 * N;
  if (act) {
#pragma unroll
    for (int q = 0; q < PM - 1; q++)
      if (q < len - 1) { sP[a0 + q] = val[q][0]; sT_[a0 + q] = val[q][1]; sWv[a0 + q] = val[q][2]; }
    sP[a0 + len - 1] = xs[0]; sT_[a0 + len - 1] = xs[1]; sWv[a0 + len - 1] = xs[2];
  }
  __syncthreads();
  for (int r = t; r < N; r += blockDim.x) {
    const double v[3] = {sP[r], sT_[r], sWv[r]};
    block_store<2>(g, o, i, j, r, v);
  }
  __syncthreads();
}

// ----------------------------------------------------------- scalar line --
template <int PM, int FAM, bool TR, class US>
__device__ __forceinline__ void part_scalar_line(const Geo &g, const Mat &m, const US &u, const Fields &rhs,
                                 const Out &o, int a, int b, double hs, double *lds, int *status) {
  const int N = g.np, T = part_chunks<PM>(N), cyc = g.periodic;
  const int t = threadIdx.x;
  const bool act = t < T;
  const int a0 = t * PM;
  const int len = act ? min(PM, N - a0) : 0;
  const int ofid = FAM == 0 ? F_UR : F_UT;
  double Cm[PM - 1], Em[PM - 1], Ym[PM - 1];
  SRow R;
  long xi;
  double *arr;
  TrWalkS<2, FAM> tw; // transposed rows: each row of the line assembled once
  if constexpr (TR) {
    if (act) tw.init(g, m, u, rhs, a, b, a0, N, cyc, hs);
  }
  SRow S{0, 1, 0, 0};
  if constexpr (TR) {
#pragma unroll
    for (int q = 0; q < PM - 1; q++) {
      if (q < len - 1) {
        tw.next(g, m, u, rhs, a, b, N, cyc, hs, R);
        double dp = R.b, rr = R.r, lx = R.a;
        if (q > 0) { dp -= R.a * Cm[q - 1]; rr -= R.a * Ym[q - 1]; lx = -R.a * Em[q - 1]; }
        if (!(dp != 0.0)) status[ST_SINGULAR] = 1;
        const double id = rcp_nr(dp);
        Cm[q] = R.c * id;
        Ym[q] = rr * id;
        Em[q] = lx * id;
      }
    }
    if (act) tw.next(g, m, u, rhs, a, b, N, cyc, hs, S);
  } else {
    const auto row = [&](int s, SRow &Q) { scalar_row<2, FAM>(g, m, u, rhs, a, b, s, N, cyc, hs, Q, xi, arr); };
    if (scalar_chunk_fwd<PM>(row, a0, len, N, Cm, Em, Ym, S)) status[ST_SINGULAR] = 1;
  }
#pragma unroll
  for (int q = PM - 2; q >= 0; q--) {
    if (q == len - 2) { Em[q] = -Em[q]; Cm[q] = -Cm[q]; }
    else if (q < len - 2) {
      Ym[q] -= Cm[q] * Ym[q + 1];
      Em[q] = -Em[q] - Cm[q] * Em[q + 1];
      Cm[q] = -Cm[q] * Cm[q + 1];
    }
  }
  double *sG = lds, *sV = lds + T, *sW = lds + 2 * T, *sL = lds + 3 * T;
  if (act) {
    sL[t] = (double)len;
    if (len >= 2) { sG[t] = Ym[0]; sV[t] = Em[0]; sW[t] = Cm[0]; }
  }
  __syncthreads();
  double A = 0.0, B = 1.0, C = 0.0, r = 0.0;
  if (act) {
    int nt_ = t + 1;
    bool has_next = nt_ < T;
    if (cyc) { nt_ %= T; has_next = true; }
    const int nlen = has_next ? (int)sL[nt_] : 0;
    double Gl = 0.0, Vl = 0.0, Wl = 0.0;
#pragma unroll
    for (int q = 0; q < PM - 1; q++)
      if (q == len - 2) { Gl = Ym[q]; Vl = Em[q]; Wl = Cm[q]; }
    B = S.b;
    r = S.r;
    if (len >= 2) { A = S.a * Vl; B += S.a * Wl; r -= S.a * Gl; }
    else A = S.a;
    if (nlen >= 2) { B += S.c * sV[nt_]; C = S.c * sW[nt_]; r -= S.c * sG[nt_]; }
    else C = S.c;
  }
  __syncthreads();
  double xs = 0.0;
  pcr_scalar(t, T, cyc, A, B, C, r, lds, xs, status);
  double *sX = lds + 4 * T;
  if (act) sX[t] = xs;
  __syncthreads();
  double val[PM];
  if (act) {
    double xl = 0.0;
    if (t > 0 || cyc) xl = sX[t > 0 ? t - 1 : T - 1];
#pragma unroll
    for (int q = 0; q < PM - 1; q++)
      if (q < len - 1) val[q] = Ym[q] + Em[q] * xl + Cm[q] * xs;
  }
  __syncthreads(); // the LDS is free: stage the line, store it contiguously
  if (act) {
#pragma unroll
    for (int q = 0; q < PM - 1; q++)
      if (q < len - 1) lds[a0 + q] = val[q];
    lds[a0 + len - 1] = xs;
  }
  __syncthreads();
  for (int r = t; r < N; r += blockDim.x)
    put(o, ofid, FAM == 0 ? idx_r(g, a, b, r) : idx_t(g, a, b, r), lds[r]);
  __syncthreads();
}

// Both scalar lines of slot (i, j) at once (u_r on r-face i, u_theta on
// theta-face j; both must exist, as at the interior slots): the steps of
// part_scalar_line for each line, with the rows of both lines assembled
// before either is eliminated and one set of barriers for the two
// reductions, so that each line's load and barrier latency overlaps the
// other's.  LDS: 10 doubles per chunk (line f's exchange and reduction at
// 4 T f, its separators at 8 T + T f; the staged lines at N f).
template <int PM, class US>
__device__ __forceinline__ void part_scalar_lines2(const Geo &g, const Mat &m, const US &u, const Fields &rhs,
                                                   const Out &o, int i, int j, double hs, double *lds,
                                                   int *status) {
  const int N = g.np, T = part_chunks<PM>(N), cyc = g.periodic;
  const int t = threadIdx.x;
  const bool act = t < T;
  const int a0 = t * PM;
  const int len = act ? min(PM, N - a0) : 0;
  double Cm[2][PM - 1], Em[2][PM - 1], Ym[2][PM - 1];
  SRow S[2] = {{0, 1, 0, 0}, {0, 1, 0, 0}};
  {
    long xi;
    double *arr;
    const auto row0 = [&](int s, SRow &Q) { scalar_row<2, 0>(g, m, u, rhs, i, j, s, N, cyc, hs, Q, xi, arr); };
    const auto row1 = [&](int s, SRow &Q) { scalar_row<2, 1>(g, m, u, rhs, i, j, s, N, cyc, hs, Q, xi, arr); };
    const bool s0 = scalar_chunk_fwd<PM>(row0, a0, len, N, Cm[0], Em[0], Ym[0], S[0]);
    const bool s1 = scalar_chunk_fwd<PM>(row1, a0, len, N, Cm[1], Em[1], Ym[1], S[1]);
    if (s0 || s1) status[ST_SINGULAR] = 1;
  }
#pragma unroll
  for (int f = 0; f < 2; f++) {
#pragma unroll
    for (int q = PM - 2; q >= 0; q--) {
      if (q == len - 2) { Em[f][q] = -Em[f][q]; Cm[f][q] = -Cm[f][q]; }
      else if (q < len - 2) {
        Ym[f][q] -= Cm[f][q] * Ym[f][q + 1];
        Em[f][q] = -Em[f][q] - Cm[f][q] * Em[f][q + 1];
        Cm[f][q] = -Cm[f][q] * Cm[f][q + 1];
      }
    }
  }
  if (act) {
#pragma unroll
    for (int f = 0; f < 2; f++) {
      double *sG = lds + 4 * T * f, *sV = sG + T, *sW = sG + 2 * T, *sL = sG + 3 * T;
      sL[t] = (double)len;
      if (len >= 2) { sG[t] = Ym[f][0]; sV[t] = Em[f][0]; sW[t] = Cm[f][0]; }
    }
  }
  __syncthreads();
  double A[2] = {0.0, 0.0}, B[2] = {1.0, 1.0}, C[2] = {0.0, 0.0}, r[2] = {0.0, 0.0};
  if (act) {
    int nt_ = t + 1;
    bool has_next = nt_ < T;
    if (cyc) { nt_ %= T; has_next = true; }
#pragma unroll
    for (int f = 0; f < 2; f++) {
      const double *sG = lds + 4 * T * f, *sV = sG + T, *sW = sG + 2 * T, *sL = sG + 3 * T;
      const int nlen = has_next ? (int)sL[nt_] : 0;
      double Gl = 0.0, Vl = 0.0, Wl = 0.0;
#pragma unroll
      for (int q = 0; q < PM - 1; q++)
        if (q == len - 2) { Gl = Ym[f][q]; Vl = Em[f][q]; Wl = Cm[f][q]; }
      B[f] = S[f].b;
      r[f] = S[f].r;
      if (len >= 2) { A[f] = S[f].a * Vl; B[f] += S[f].a * Wl; r[f] -= S[f].a * Gl; }
      else A[f] = S[f].a;
      if (nlen >= 2) { B[f] += S[f].c * sV[nt_]; C[f] = S[f].c * sW[nt_]; r[f] -= S[f].c * sG[nt_]; }
      else C[f] = S[f].c;
    }
  }
  __syncthreads();
  double xs[2] = {0.0, 0.0};
  pcr_scalar2(t, T, cyc, A, B, C, r, lds, xs, status);
  if (act) {
    lds[8 * T + t] = xs[0];
    lds[9 * T + t] = xs[1];
  }
  __syncthreads();
  double val[2][PM];
  if (act) {
#pragma unroll
    for (int f = 0; f < 2; f++) {
      double xl = 0.0;
      if (t > 0 || cyc) xl = lds[(8 + f) * T + (t > 0 ? t - 1 : T - 1)];
#pragma unroll
      for (int q = 0; q < PM - 1; q++)
        if (q < len - 1) val[f][q] = Ym[f][q] + Em[f][q] * xl + Cm[f][q] * xs[f];
    }
  }
  __syncthreads(); // the LDS is free: stage both lines, store them contiguously
  if (act) {
#pragma unroll
    for (int f = 0; f < 2; f++) {
#pragma unroll
      for (int q = 0; q < PM - 1; q++)
        if (q < len - 1) lds[f * N + a0 + q] = val[f][q];
      lds[f * N + a0 + len - 1] = xs[f];
    }
  }
  __syncthreads();
  for (int s = t; s < N; s += blockDim.x) {
    put(o, F_UR, idx_r(g, i, j, s), lds[s]);
    put(o, F_UT, idx_t(g, i, j, s), lds[N + s]);
  }
  __syncthreads();
}

// one workgroup per (i, j): block line (i, j), u_r line on r-face i (i >= 1),
// u_theta line on theta-face j (j >= 1).  Flat grid of nr * nt workgroups per
// grid; one grid or a batch of grids.  The workgroup may be wider than the
// chunk count: threads past it only join the barriers.  PART 0: the block
// line; 1: the two scalar lines; 2: all three.  On large launches the
// forward sweep runs parts 0 and 1 as two launches: the scalar lines need far
// fewer registers (about 55 against 256) and on their own run at a much
// higher occupancy; on small ones the second launch costs more than that
// gains.
// MAP: 0 every slot, w = i * nt + j; 1 the interior slots
// (1 <= i <= nr - 2, 1 <= j <= nt - 2), whose rows read no ghost across an
// r or theta boundary, with the interior source (32-bit indices, ghosts in
// phi only; P: periodic phi); 2 the other slots, with the general source.
template <int PM, bool TR, int PART = 2, bool W = false, int MAP = 0, bool P = false, bool PT = false>
__device__ __forceinline__ void phi_body(const PassArgs &a, unsigned w, double *lds) {
  const Geo &g = a.g;
  int i, j;
  if constexpr (MAP == 1) {
    j = 1 + (int)(w % (unsigned)(g.nt - 2));
    i = 1 + (int)(w / (unsigned)(g.nt - 2));
  } else if constexpr (MAP == 2) {
    if (w < 2u * (unsigned)g.nr) {
      i = (int)(w >> 1);
      j = (w & 1u) ? g.nt - 1 : 0;
    } else {
      const unsigned w2 = w - 2u * (unsigned)g.nr;
      j = 1 + (int)(w2 >> 1);
      i = (w2 & 1u) ? g.nr - 1 : 0;
    }
  } else {
    j = (int)(w % g.nt);
    i = (int)(w / g.nt);
  }
  const int t = threadIdx.x;
  const Out &o = a.o;
  if (PART != 1 && o.mode == 0) { // boundary-normal faces of x that no phi line owns
    const Fields &x = o.x;
    for (int k = t; k < g.np; k += blockDim.x) {
      if (i == 0) x.ur[idx_r(g, 0, j, k)] = 0.0;
      if (i == g.nr - 1) x.ur[idx_r(g, g.nr, j, k)] = 0.0;
      if (j == 0) x.ut[idx_t(g, i, 0, k)] = 0.0;
      if (j == g.nt - 1) x.ut[idx_t(g, i, g.nt, k)] = 0.0;
    }
    if (!g.periodic && t == 0) x.uf[idx_f(g, i, j, 0)] = 0.0;
  }
  if constexpr (MAP == 1) {
    const auto u = SrcSelIn<W, PT, P>::get(a);
    if (PART != 1) part_block_line<PM, TR>(g, a.m, u, a.rhs, o, i, j, a.tau, lds, a.status);
    if (PART != 0) {
      if constexpr (TR) {
        part_scalar_line<PM, 0, TR>(g, a.m, u, a.rhs, o, i, j, a.tau, lds, a.status);
        part_scalar_line<PM, 1, TR>(g, a.m, u, a.rhs, o, i, j, a.tau, lds, a.status);
      } else {
        part_scalar_lines2<PM>(g, a.m, u, a.rhs, o, i, j, a.tau, lds, a.status);
      }
    }
  } else {
    // W: forced pass (wall velocities); PT: perturbation-pressure form
    decltype(auto) u = SrcSel<W, PT>::get(a);
    if (PART != 1) part_block_line<PM, TR>(g, a.m, u, a.rhs, o, i, j, a.tau, lds, a.status);
    if (PART != 0) {
      if (i >= 1) part_scalar_line<PM, 0, TR>(g, a.m, u, a.rhs, o, i, j, a.tau, lds, a.status);
      if (j >= 1) part_scalar_line<PM, 1, TR>(g, a.m, u, a.rhs, o, i, j, a.tau, lds, a.status);
    }
  }
}

// The scalar lines of slot (i, j) read the cells of slots (i - 1, j) and
// (i, j - 1) too: the scalar launch numbers its slots XCD-contiguously.
// Measured on the global grid: the phi pass 1.93 -> 1.87 ms; renumbering the
// block launch as well is slower.
template <int PM, bool B, int PART>
__global__ void __launch_bounds__(256) DSW_OCC(DSW_WAVES_PHI) k_phi_part(PassArgs a, Batch bt) {
  extern __shared__ double lds[];
  const unsigned w = PART == 1 ? xcd_contiguous(blockIdx.x, gridDim.x) : blockIdx.x;
  if constexpr (B) {
    const int mb = batch_member(bt, w);
    phi_body<PM, false, PART>(batch_args(bt, mb), w - bt.woff[mb], lds);
  } else {
    phi_body<PM, false, PART>(a, w, lds);
  }
}

// perturbation-pressure form, one grid (as the plain pass of one grid)
template <int PM, int PART>
__global__ void __launch_bounds__(256) DSW_OCC(DSW_WAVES_PHI) k_phi_partP(PassArgs a) {
  extern __shared__ double lds[];
  const unsigned w = PART == 1 ? xcd_contiguous(blockIdx.x, gridDim.x) : blockIdx.x;
  phi_body<PM, false, PART, false, 0, false, true>(a, w, lds);
}

// one grid, every slot: the boundary ring's slots (MAP 2, the general
// source) in workgroups [0, ring), then the interior slots (MAP 1, the
// interior source; P: periodic phi); PT: perturbation-pressure form.  One
// launch instead of one per slot set: the ring's few hundred workgroups fill
// the interior launch's tail instead of running as a launch of their own.
template <int PM, int PART, bool P, bool PT>
__global__ void __launch_bounds__(256) DSW_OCC(DSW_WAVES_PHI) k_phi_partC(PassArgs a) {
  extern __shared__ double lds[];
  const unsigned w = PART == 1 ? xcd_contiguous(blockIdx.x, gridDim.x) : blockIdx.x;
  const unsigned ring = 2u * (unsigned)a.g.nr + 2u * (unsigned)(a.g.nt - 2);
  if (w < ring) phi_body<PM, false, PART, false, 2, false, PT>(a, w, lds);
  else phi_body<PM, false, PART, false, 1, P, PT>(a, w - ring, lds);
}

// a batch of grids with an interior (P: periodic phi): member m's workgroups
// take its boundary ring's slots first, then its interior slots, as
// k_phi_partC does for one grid
template <int PM, int PART, bool P>
__global__ void __launch_bounds__(256) DSW_OCC(DSW_WAVES_PHI) k_phi_partCB(PassArgs a, Batch bt) {
  extern __shared__ double lds[];
  const unsigned w = PART == 1 ? xcd_contiguous(blockIdx.x, gridDim.x) : blockIdx.x;
  const int mb = batch_member(bt, w);
  const PassArgs &am = batch_args(bt, mb);
  const unsigned wl = w - bt.woff[mb];
  const unsigned ring = 2u * (unsigned)am.g.nr + 2u * (unsigned)(am.g.nt - 2);
  if (wl < ring) phi_body<PM, false, PART, false, 2>(am, wl, lds);
  else phi_body<PM, false, PART, false, 1, P>(am, wl - ring, lds);
}

// forced split step, one grid: as the plain sweep, all three lines of a slot
// in one launch, or from PHI_SPLIT_SLOTS slots on the block lines and the
// scalar lines as two
template <int PM, int PART, int MAP, bool P = false>
__global__ void __launch_bounds__(256) DSW_OCC(DSW_WAVES_PHI) k_phi_partF(PassArgs a) {
  extern __shared__ double lds[];
  phi_body<PM, false, PART, true, MAP, P>(a, blockIdx.x, lds);
}

// transposed systems (adjoint), one grid: each chunk walks the rows of the
// line once and forms the transposed rows from them (TrWalk, TrWalkS)
template <int PM, int PART>
__global__ void __launch_bounds__(256) k_phi_part_T(PassArgs a) {
  extern __shared__ double lds[];
  // the scalar launch numbered XCD-contiguously, as in the forward sweep
  phi_body<PM, true, PART>(a, PART == 1 ? xcd_contiguous(blockIdx.x, gridDim.x) : blockIdx.x, lds);
}

// block lines, then scalar lines, as two launches: the scalar launch holds a
// fraction of the block launch's registers and runs at higher occupancy
void launch_phi_T(int pm, const PassArgs &a, unsigned blocks, unsigned threads, size_t lds,
                  hipStream_t st) {
  const size_t lds_s = sizeof(double) * (size_t)(pm > 5 ? pm : 5) * threads;
  if (pm == 2) {
    hipLaunchKernelGGL((k_phi_part_T<2, 0>), dim3(blocks), dim3(threads), lds, st, a);
    hipLaunchKernelGGL((k_phi_part_T<2, 1>), dim3(blocks), dim3(threads), lds_s, st, a);
  } else {
    hipLaunchKernelGGL((k_phi_part_T<4, 0>), dim3(blocks), dim3(threads), lds, st, a);
    hipLaunchKernelGGL((k_phi_part_T<4, 1>), dim3(blocks), dim3(threads), lds_s, st, a);
  }
}

bool phi_part_supported(const Geo &g, int pm) {
  if (pm != 2 && pm != 4) return false;
  const int T = (g.np + pm - 1) / pm;
  if (T > PT_MAX) return false;
  if (g.periodic) { // cyclic reduction needs a power-of-two number of equal chunks
    if (g.np % pm != 0) return false;
    if (T & (T - 1)) return false;
  }
  return true;
}

unsigned phi_part_threads(const Geo &g, int pm) {
  const int T = (g.np + pm - 1) / pm;
  return (unsigned)(((T + 63) / 64) * 64);
}

size_t phi_part_lds(const Geo &g, int pm) {
  const int T = (g.np + pm - 1) / pm;
  return sizeof(double) * 24 * (size_t)T;
}

// From this many line slots on, the block and the scalar lines run as two
// launches (measured: 1.99 -> 1.93 ms on 32768 slots of 512 cells, 0.27 ->
// 0.31 ms on 8192 slots of 256 cells).
constexpr unsigned PHI_SPLIT_SLOTS = 16384;

// Whether a split pass of one grid takes the interior slots with the
// interior source: the slots' 32-bit indices reach, and the grid has an
// interior.  The interior source drops the ghost code across r and theta
// boundaries and forms 32-bit indices: measured on the 512 x 256 x 128
// sphere, the phi pass 1.83 -> 1.78 ms, results bitwise unchanged.
bool phi_interior_split(const Geo &g) {
  return g.nr >= 3 && g.nt >= 3 && (long)(g.nr + 1) * (g.nt + 1) * g.npf < 0x7fffffffL;
}

// one grid, split: the block lines of every slot (ring, then interior), then
// their scalar lines (at the interior slots both lines of a slot at once: 10
// doubles of LDS per thread)
template <int PM, bool PT>
static void launch_phi_in(const PassArgs &a, unsigned threads, size_t lds, size_t lds_s, hipStream_t st) {
  const Geo &g = a.g;
  (void)lds_s;
  const size_t lds_s2 = sizeof(double) * 10 * (size_t)threads;
  const dim3 gall((unsigned)(g.nr - 2) * (unsigned)(g.nt - 2) + 2u * (unsigned)g.nr + 2u * (unsigned)(g.nt - 2));
  const dim3 bl(threads);
  if (g.periodic) {
    hipLaunchKernelGGL((k_phi_partC<PM, 0, true, PT>), gall, bl, lds, st, a);
    hipLaunchKernelGGL((k_phi_partC<PM, 1, true, PT>), gall, bl, lds_s2, st, a);
  } else {
    hipLaunchKernelGGL((k_phi_partC<PM, 0, false, PT>), gall, bl, lds, st, a);
    hipLaunchKernelGGL((k_phi_partC<PM, 1, false, PT>), gall, bl, lds_s2, st, a);
  }
}

// the block lines, then the scalar lines (their LDS: the exchange and
// reduction arrays, 5 doubles per chunk, or the staged line, PM per chunk),
// or all in one launch
void launch_phi_pass(int pm, const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                     size_t lds, hipStream_t st) {
  const dim3 gr(blocks), bl(threads);
  const size_t lds_s = sizeof(double) * (size_t)(pm > 5 ? pm : 5) * threads;
  if (!b.tab && blocks >= PHI_SPLIT_SLOTS && phi_interior_split(a.g)) {
    if (pm == 2) launch_phi_in<2, false>(a, threads, lds, lds_s, st);
    else launch_phi_in<4, false>(a, threads, lds, lds_s, st);
    return;
  }
  if (blocks < PHI_SPLIT_SLOTS) {
    if (b.tab) {
      if (pm == 2) hipLaunchKernelGGL((k_phi_part<2, true, 2>), gr, bl, lds, st, a, b);
      else hipLaunchKernelGGL((k_phi_part<4, true, 2>), gr, bl, lds, st, a, b);
    } else {
      if (pm == 2) hipLaunchKernelGGL((k_phi_part<2, false, 2>), gr, bl, lds, st, a, b);
      else hipLaunchKernelGGL((k_phi_part<4, false, 2>), gr, bl, lds, st, a, b);
    }
    return;
  }
  if (b.tab) {
    if (pm == 2) {
      hipLaunchKernelGGL((k_phi_part<2, true, 0>), gr, bl, lds, st, a, b);
      hipLaunchKernelGGL((k_phi_part<2, true, 1>), gr, bl, lds_s, st, a, b);
    } else {
      hipLaunchKernelGGL((k_phi_part<4, true, 0>), gr, bl, lds, st, a, b);
      hipLaunchKernelGGL((k_phi_part<4, true, 1>), gr, bl, lds_s, st, a, b);
    }
  } else {
    if (pm == 2) {
      hipLaunchKernelGGL((k_phi_part<2, false, 0>), gr, bl, lds, st, a, b);
      hipLaunchKernelGGL((k_phi_part<2, false, 1>), gr, bl, lds_s, st, a, b);
    } else {
      hipLaunchKernelGGL((k_phi_part<4, false, 0>), gr, bl, lds, st, a, b);
      hipLaunchKernelGGL((k_phi_part<4, false, 1>), gr, bl, lds_s, st, a, b);
    }
  }
}

template <int PM, bool P>
static void launch_phi_cb(const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads, size_t lds,
                          hipStream_t st) {
  const dim3 gr(blocks), bl(threads);
  if (blocks < PHI_SPLIT_SLOTS) {
    hipLaunchKernelGGL((k_phi_partCB<PM, 2, P>), gr, bl, lds, st, a, b);
    return;
  }
  const size_t lds_s2 = sizeof(double) * 10 * (size_t)threads;  // both scalar lines of a slot at once
  hipLaunchKernelGGL((k_phi_partCB<PM, 0, P>), gr, bl, lds, st, a, b);
  hipLaunchKernelGGL((k_phi_partCB<PM, 1, P>), gr, bl, lds_s2, st, a, b);
}

void launch_phi_pass_c(int pm, bool periodic, const PassArgs &a, const Batch &b, unsigned blocks,
                       unsigned threads, size_t lds, hipStream_t st) {
  if (!b.tab) {  // one grid: as any partitioned phi pass
    launch_phi_pass(pm, a, b, blocks, threads, lds, st);
    return;
  }
  if (pm == 2) {
    if (periodic) launch_phi_cb<2, true>(a, b, blocks, threads, lds, st);
    else launch_phi_cb<2, false>(a, b, blocks, threads, lds, st);
  } else {
    if (periodic) launch_phi_cb<4, true>(a, b, blocks, threads, lds, st);
    else launch_phi_cb<4, false>(a, b, blocks, threads, lds, st);
  }
}

void launch_phi_pert(int pm, const PassArgs &a, unsigned blocks, unsigned threads, size_t lds,
                     hipStream_t st) {
  const dim3 gr(blocks), bl(threads);
  const size_t lds_s = sizeof(double) * (size_t)(pm > 5 ? pm : 5) * threads;
  if (blocks >= PHI_SPLIT_SLOTS && phi_interior_split(a.g)) {
    if (pm == 2) launch_phi_in<2, true>(a, threads, lds, lds_s, st);
    else launch_phi_in<4, true>(a, threads, lds, lds_s, st);
    return;
  }
  if (blocks < PHI_SPLIT_SLOTS) {
    if (pm == 2) hipLaunchKernelGGL((k_phi_partP<2, 2>), gr, bl, lds, st, a);
    else hipLaunchKernelGGL((k_phi_partP<4, 2>), gr, bl, lds, st, a);
    return;
  }
  if (pm == 2) {
    hipLaunchKernelGGL((k_phi_partP<2, 0>), gr, bl, lds, st, a);
    hipLaunchKernelGGL((k_phi_partP<2, 1>), gr, bl, lds_s, st, a);
  } else {
    hipLaunchKernelGGL((k_phi_partP<4, 0>), gr, bl, lds, st, a);
    hipLaunchKernelGGL((k_phi_partP<4, 1>), gr, bl, lds_s, st, a);
  }
}

// one launch of the forced phi pass over a slot set (MAP) and a part
template <int PM, int MAP>
static void launch_phi_forced_map(const PassArgs &a, unsigned blocks, unsigned threads, size_t lds,
                                  size_t lds_s, bool split, hipStream_t st) {
  if (!blocks) return;
  // the interior slots solve both scalar lines at once: 10 doubles per thread
  if (MAP == 1) lds_s = std::max(lds_s, sizeof(double) * 10 * (size_t)threads);
  const dim3 gr(blocks), bl(threads);
  if constexpr (MAP == 1) {
    if (a.g.periodic) {
      if (!split) hipLaunchKernelGGL((k_phi_partF<PM, 2, MAP, true>), gr, bl, lds, st, a);
      else {
        hipLaunchKernelGGL((k_phi_partF<PM, 0, MAP, true>), gr, bl, lds, st, a);
        hipLaunchKernelGGL((k_phi_partF<PM, 1, MAP, true>), gr, bl, lds_s, st, a);
      }
      return;
    }
  }
  if (!split) {
    hipLaunchKernelGGL((k_phi_partF<PM, 2, MAP>), gr, bl, lds, st, a);
  } else {
    hipLaunchKernelGGL((k_phi_partF<PM, 0, MAP>), gr, bl, lds, st, a);
    hipLaunchKernelGGL((k_phi_partF<PM, 1, MAP>), gr, bl, lds_s, st, a);
  }
}

// The interior slots with the interior source, the rest with the general
// one (its ghost code across r and theta walls costs the block kernel a
// wave per SIMD); every slot with the general one when 32-bit indices do
// not reach.
void launch_phi_forced(int pm, const PassArgs &a, unsigned blocks, unsigned threads, size_t lds,
                       hipStream_t st) {
  const Geo &g = a.g;
  const size_t lds_s = sizeof(double) * (size_t)(pm > 5 ? pm : 5) * threads;
  const bool split = blocks >= PHI_SPLIT_SLOTS;
  const bool in32 = (long)(g.nr + 1) * (g.nt + 1) * g.npf < 0x7fffffffL;
  if (!in32) {
    if (pm == 2) launch_phi_forced_map<2, 0>(a, blocks, threads, lds, lds_s, split, st);
    else launch_phi_forced_map<4, 0>(a, blocks, threads, lds, lds_s, split, st);
    return;
  }
  const unsigned nin = (unsigned)(g.nr - 2) * (unsigned)(g.nt - 2);
  const unsigned nbd = 2u * (unsigned)g.nr + 2u * (unsigned)(g.nt - 2);
  if (pm == 2) {
    launch_phi_forced_map<2, 1>(a, nin, threads, lds, lds_s, split, st);
    launch_phi_forced_map<2, 2>(a, nbd, threads, lds, lds_s, split, st);
  } else {
    launch_phi_forced_map<4, 1>(a, nin, threads, lds, lds_s, split, st);
    launch_phi_forced_map<4, 2>(a, nbd, threads, lds, lds_s, split, st);
  }
}

} // namespace dsw
