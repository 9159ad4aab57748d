// rt_part.hip -- partitioned line solver for the r and theta sweeps (paper
// eqs. (spl1), (spl2); operators D_r and D_theta of Appendix B, eqs. (dr),
// (dtheta)).
//
// A workgroup takes L neighbouring lines of one family (consecutive phi
// index: the lanes that read one row of their lines read contiguous memory)
// and splits every line into T chunks of PM rows; thread t = c * L + l holds
// chunk c of line l.  As in the phi solver:
//   1. each thread assembles its rows and eliminates the interior ones with
//      the block Thomas recurrence, carrying the dependence on the last row
//      of the chunk before ("spike"), then sweeps back so that every interior
//      row reads x_q = g_q + V_q x_left + W_q x_sep;
//   2. the chunks' last rows ("separators") of each line form a
//      block-tridiagonal system, solved in LDS by parallel cyclic reduction
//      (log2 T steps);
//   3. the interior rows are filled in from the separators and stored.
// Every intermediate stays in registers and LDS: no scratch array, so the
// pass moves one read of its inputs and one write of its result.
#include "rows.hpp"

namespace dsw {

constexpr int RT_PMS = 8;  // rows per thread, scalar lines

// chunks of PM rows on a line of n rows
template <int PM>
__host__ __device__ inline int rt_chunks(int n) { return (n + PM - 1) / PM; }

// --------------------------------------------------- reduction over lines --
// Parallel cyclic reduction of the separator rows A x_{c-1} + B x_c +
// C x_{c+1} = r of every line of the workgroup; separator (l, c) is held by
// thread c * L + l (act: a separator of a real line).  Each step, every
// separator publishes B^{-1} A, B^{-1} C and B^{-1} r (21 doubles of LDS per
// thread) and folds in its neighbours h chunks away.  Non-cyclic lines: the
// couplings past either end are zero from the start and stay zero.
__device__ __forceinline__ void rt_pcr_block(int c, int l, int T, int L, bool act, double *A, double *B,
                                             double *C, double *r, double *lds, double *x, int *status) {
  const int nt = T * L, t = c * L + l;
  double *sA = lds, *sC = lds + 9 * nt, *sR = lds + 18 * nt;
  for (int h = 1; h < T; h *= 2) {
    if (act) {
      double Bi[9];
      inv3(B, Bi, status);
      mm3(Bi, A, &sA[t * 9]);
      mm3(Bi, C, &sC[t * 9]);
      mv3(Bi, r, &sR[t * 3]);
    }
    __syncthreads();
    if (act) {
      // x_{c-h} = R' - A' x_{c-2h} - C' x_c and x_{c+h} alike: B' = B -
      // A C'(c-h) - C A'(c+h), r' alike, A' = -A A'(c-h), C' = -C C'(c+h)
      const bool has_lo = c - h >= 0, has_hi = c + h < T;
      const int ul = (c - h) * L + l, uh = (c + h) * L + l;
      if (has_lo) { mm3_sub(A, &sC[ul * 9], B); mv3_sub(A, &sR[ul * 3], r); }
      if (has_hi) { mm3_sub(C, &sA[uh * 9], B); mv3_sub(C, &sR[uh * 3], r); }
      if (has_lo) mm3_neg_inplace(A, &sA[ul * 9]);
      else {
#pragma unroll
        for (int q = 0; q < 9; q++) A[q] = 0.0;
      }
      if (has_hi) mm3_neg_inplace(C, &sC[uh * 9]);
      else {
#pragma unroll
        for (int q = 0; q < 9; q++) C[q] = 0.0;
      }
    }
    __syncthreads();
  }
  if (act) {
    double Bi[9];
    inv3(B, Bi, status);
    mv3(Bi, r, x);
  }
}

__device__ __forceinline__ void rt_pcr_scalar(int c, int l, int T, int L, bool act, double &A, double &B,
                                              double &C, double &r, double *lds, double &x, int *status) {
  const int nt = T * L, t = c * L + l;
  double *sA = lds, *sC = lds + nt, *sR = lds + 2 * nt;
  for (int h = 1; h < T; h *= 2) {
    if (act) {
      if (!(B != 0.0)) status[ST_SINGULAR] = 1;
      const double ib = rcp_nr(B);
      sA[t] = A * ib;
      sC[t] = C * ib;
      sR[t] = r * ib;
    }
    __syncthreads();
    if (act) {
      double nA = 0.0, nC = 0.0;
      if (c - h >= 0) {
        const int u = (c - h) * L + l;
        nA = -A * sA[u];
        B -= A * sC[u];
        r -= A * sR[u];
      }
      if (c + h < T) {
        const int u = (c + h) * L + l;
        nC = -C * sC[u];
        B -= C * sA[u];
        r -= C * sR[u];
      }
      A = nA;
      C = nC;
    }
    __syncthreads();
  }
  if (act) {
    if (!(B != 0.0)) status[ST_SINGULAR] = 1;
    x = r * rcp_nr(B);
  }
}

// ------------------------------------------------------------ block lines --
// The block lines [line0, line0 + L) of sweep D (line = a * np + b); LDS
// 24 doubles per thread.
// TR: the transposed system (adjoint): each chunk walks its rows once and
// forms the transposed rows from them (TrWalk; u is then the plain source).
template <int D, int PM, bool TR, class US>
__device__ __forceinline__ void rt_block_lines(const Geo &g, const Mat &m, const US &u, const Fields &rhs,
                                               const Out &o, long line0, double hs, double *lds,
                                               int *status) {
  const Families F = families(g, D);
  const int n = F.n, T = rt_chunks<PM>(n), L = (int)blockDim.x / T;
  const int t = threadIdx.x, c = t / L, l = t % L;
  const long line = line0 + l;
  const bool act = c < T && line < F.nb;
  int pa = 0, pb = 0;
  if (act) { pa = (int)(line / g.np); pb = (int)(line % g.np); }
  if (act && c == 0 && o.mode == 0) zero_bnd<D>(g, o.x, pa, pb);
  const int a0 = c * PM;
  const int len = act ? min(PM, n - a0) : 0;
  double Cm[PM - 1][9], Em[PM - 1][9], Ym[PM - 1][3];
  // structural non-zeros of the row blocks (transposed rows: L = U^T, U = L^T)
  constexpr unsigned mL = TR ? nz_tr(NZ_U) : NZ_L, mU = TR ? nz_tr(NZ_L) : NZ_U;
  TrWalk<D> tw;
  if constexpr (TR) {
    if (act) tw.init(g, m, u, rhs, pa, pb, a0, n, 0, hs);
  }
  // a zero pivot is recorded after the loop: a store inside it would hold
  // the next row's loads back
  bool sing = false;
  // 1. forward elimination over the interior rows with the left spike
#pragma unroll
  for (int q = 0; q < PM - 1; q++) {
    if (q < len - 1) {
      BRow R;
      if constexpr (TR) tw.next(g, m, u, rhs, pa, pb, n, 0, hs, R);
      else block_row<D>(g, m, u, rhs, pa, pb, a0 + q, n, 0, hs, R);
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
        mm3m<mL, NZ_ALL>(R.L, Em[q - 1], t9);
#pragma unroll
        for (int z = 0; z < 9; z++) Lx[z] = -t9[z];
      }
      sing |= inv3q(Dp, Ai);
      mm3m<NZ_ALL, mU>(Ai, R.U, Cm[q]);
      mv3(Ai, rr, Ym[q]);
      if (q == 0) mm3m<NZ_ALL, mL>(Ai, R.L, Em[q]);
      else mm3(Ai, Lx, Em[q]);
    }
  }
  if (sing) status[ST_SINGULAR] = 1;
  BRow S;  // separator row (last row of the chunk)
  if (act) {
    if constexpr (TR) tw.next(g, m, u, rhs, pa, pb, n, 0, hs, S);
    else block_row<D>(g, m, u, rhs, pa, pb, a0 + len - 1, n, 0, hs, S);
  }
  // backward sweep: (Y, E, C) -> (g, V, W)
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
      mm3(Cm[q], Cm[q + 1], t9);
#pragma unroll
      for (int z = 0; z < 9; z++) Cm[q][z] = -t9[z];
    }
  }
  // 2. the first interior row of every chunk to the chunk before it
  const int nt = T * L;
  double *sG = lds, *sV = lds + 3 * nt, *sW = lds + 12 * nt, *sL = lds + 21 * nt;
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
    const int tn = t + L;  // chunk c + 1 of the same line
    const int nlen = c + 1 < T ? (int)sL[tn] : 0;
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
      mm3m<mU, NZ_ALL>(S.U, &sV[tn * 9], t9);
#pragma unroll
      for (int z = 0; z < 9; z++) B[z] += t9[z];
      mm3m<mU, NZ_ALL>(S.U, &sW[tn * 9], Cc);
      mv3m<mU>(S.U, &sG[tn * 3], t3);
#pragma unroll
      for (int z = 0; z < 3; z++) r[z] -= t3[z];
    } else {
#pragma unroll
      for (int z = 0; z < 9; z++) Cc[z] = S.U[z];
    }
  }
  __syncthreads();  // the exchange area is reused by the reduction
  double xs[3] = {0, 0, 0};
  rt_pcr_block(c, l, T, L, act, A, B, Cc, r, lds, xs, status);
  // 3. fill in the interior rows from the separators on either side
  double *sX = lds + 21 * nt;
  if (act) {
#pragma unroll
    for (int z = 0; z < 3; z++) sX[t * 3 + z] = xs[z];
  }
  __syncthreads();
  if (!act) return;
  double xl[3] = {0, 0, 0};
  if (c > 0) {
#pragma unroll
    for (int z = 0; z < 3; z++) xl[z] = sX[(t - L) * 3 + z];
  }
#pragma unroll
  for (int q = 0; q < PM - 1; q++) {
    if (q < len - 1) {
      double v[3], t3[3];
      mv3(Em[q], xl, v);
      mv3(Cm[q], xs, t3);
#pragma unroll
      for (int z = 0; z < 3; z++) v[z] += Ym[q][z] + t3[z];
      block_store<D>(g, o, pa, pb, a0 + q, v);
    }
  }
  block_store<D>(g, o, pa, pb, a0 + len - 1, xs);
}

// ----------------------------------------------------------- scalar lines --
// Lines [line0, line0 + L) of scalar family FAM of sweep D; LDS 4 doubles
// per thread.
template <int D, int FAM, int PM, bool TR, class US>
__device__ __forceinline__ void rt_scalar_lines(const Geo &g, const Mat &m, const US &u, const Fields &rhs,
                                                const Out &o, long line0, double hs, double *lds,
                                                int *status) {
  const Families F = families(g, D);
  const int n = F.n, T = rt_chunks<PM>(n), L = (int)blockDim.x / T;
  const int t = threadIdx.x, c = t / L, l = t % L;
  const long line = line0 + l;
  const long nl = FAM == 0 ? F.na : F.nbb;
  const bool act = c < T && line < nl;
  const int nkf = g.periodic ? g.np : g.np - 1, kf0 = g.periodic ? 0 : 1;
  int pa = FAM == 0 ? 1 : 0, pb = FAM == 0 ? 0 : kf0;
  if (act) {
    if (FAM == 0) { pa = 1 + (int)(line / g.np); pb = (int)(line % g.np); }
    else { pa = (int)(line / nkf); pb = kf0 + (int)(line % nkf); }
  }
  int ofid;
  if (D == 0) ofid = FAM == 0 ? F_UT : F_UF;
  else ofid = FAM == 0 ? F_UR : F_UF;
  const int a0 = c * PM;
  const int len = act ? min(PM, n - a0) : 0;
  double Cm[PM - 1], Em[PM - 1], Ym[PM - 1];
  long xi;
  double *arr;
  TrWalkS<D, FAM> tw;
  if constexpr (TR) {
    if (act) tw.init(g, m, u, rhs, pa, pb, a0, n, 0, hs);
  }
#pragma unroll
  for (int q = 0; q < PM - 1; q++) {
    if (q < len - 1) {
      SRow R;
      if constexpr (TR) tw.next(g, m, u, rhs, pa, pb, n, 0, hs, R);
      else scalar_row<D, FAM>(g, m, u, rhs, pa, pb, a0 + q, n, 0, hs, R, xi, arr);
      double dp = R.b, rr = R.r, lx = R.a;
      if (q > 0) { dp -= R.a * Cm[q - 1]; rr -= R.a * Ym[q - 1]; lx = -R.a * Em[q - 1]; }
      if (!(dp != 0.0)) status[ST_SINGULAR] = 1;
      const double id = rcp_nr(dp);
      Cm[q] = R.c * id;
      Ym[q] = rr * id;
      Em[q] = lx * id;
    }
  }
  SRow S{0, 1, 0, 0};
  if (act) {
    if constexpr (TR) tw.next(g, m, u, rhs, pa, pb, n, 0, hs, S);
    else scalar_row<D, FAM>(g, m, u, rhs, pa, pb, a0 + len - 1, n, 0, hs, S, xi, arr);
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
  const int nt = T * L;
  double *sG = lds, *sV = lds + nt, *sW = lds + 2 * nt, *sL = lds + 3 * nt;
  if (act) {
    sL[t] = (double)len;
    if (len >= 2) { sG[t] = Ym[0]; sV[t] = Em[0]; sW[t] = Cm[0]; }
  }
  __syncthreads();
  double A = 0.0, B = 1.0, C = 0.0, r = 0.0;
  if (act) {
    const int tn = t + L;
    const int nlen = c + 1 < T ? (int)sL[tn] : 0;
    double Gl = 0.0, Vl = 0.0, Wl = 0.0;
#pragma unroll
    for (int q = 0; q < PM - 1; q++)
      if (q == len - 2) { Gl = Ym[q]; Vl = Em[q]; Wl = Cm[q]; }
    B = S.b;
    r = S.r;
    if (len >= 2) { A = S.a * Vl; B += S.a * Wl; r -= S.a * Gl; }
    else A = S.a;
    if (nlen >= 2) { B += S.c * sV[tn]; C = S.c * sW[tn]; r -= S.c * sG[tn]; }
    else C = S.c;
  }
  __syncthreads();
  double xs = 0.0;
  rt_pcr_scalar(c, l, T, L, act, A, B, C, r, lds, xs, status);
  double *sX = lds + 3 * nt;
  if (act) sX[t] = xs;
  __syncthreads();
  if (!act) return;
  const double xl = c > 0 ? sX[t - L] : 0.0;
#pragma unroll
  for (int q = 0; q < PM - 1; q++)
    if (q < len - 1) put(o, ofid, scalar_index<D, FAM>(g, pa, pb, a0 + q), Ym[q] + Em[q] * xl + Cm[q] * xs);
  put(o, ofid, scalar_index<D, FAM>(g, pa, pb, a0 + len - 1), xs);
}

// ------------------------------------------------------------ the passes --

// pm: rows per thread on the block lines
__host__ __device__ inline int rt_block_chunks(int n, int pm) { return (n + pm - 1) / pm; }
__host__ __device__ inline unsigned rt_block_wgs(const Geo &g, int d, unsigned bs, int pm) {
  const Families F = families(g, d);
  const unsigned L = bs / (unsigned)rt_block_chunks(F.n, pm);
  return (unsigned)((F.nb + L - 1) / L);
}

// workgroups of scalar family A, and of both families
__host__ __device__ inline unsigned rt_scalar_wgs_a(const Geo &g, int d, unsigned bs) {
  const Families F = families(g, d);
  const unsigned L = bs / (unsigned)rt_chunks<RT_PMS>(F.n);
  return (unsigned)((F.na + L - 1) / L);
}
__host__ __device__ inline unsigned rt_scalar_wgs(const Geo &g, int d, unsigned bs) {
  const Families F = families(g, d);
  const unsigned L = bs / (unsigned)rt_chunks<RT_PMS>(F.n);
  return rt_scalar_wgs_a(g, d, bs) + (unsigned)((F.nbb + L - 1) / L);
}

// PART 0: block lines only; 1: scalar lines only; 2: block lines in
// workgroups [0, nbw), then the scalar lines.  COMB: workgroups numbered as
// for PART 2 whatever the part (a batched launch's member table counts both
// kinds), those of the other part leaving at once; else PART 1 numbers the
// scalar workgroups from 0.  W: a forced pass.
template <int D, int PM, int PART, bool W = false, bool TR = false, bool PT = false, bool COMB = false>
__device__ __forceinline__ void rt_body(const PassArgs &a, unsigned w, double *lds) {
  const Geo &g = a.g;
  decltype(auto) u = SrcSel<W, PT>::get(a);  // the plain source when TR
  const unsigned bs = blockDim.x;
  const unsigned nbw = (PART == 1 && !COMB) ? 0u : rt_block_wgs(g, D, bs, PM);
  if (w < nbw) {
    if constexpr (PART != 1) {
      const unsigned L = bs / (unsigned)rt_chunks<PM>(families(g, D).n);
      rt_block_lines<D, PM, TR>(g, a.m, u, a.rhs, a.o, (long)w * L, a.tau, lds, a.status);
    }
    return;
  }
  if constexpr (PART != 0) {
    const unsigned w2 = w - nbw;
    const unsigned L = bs / (unsigned)rt_chunks<RT_PMS>(families(g, D).n);
    const unsigned nwa = rt_scalar_wgs_a(g, D, bs);
    if (w2 < nwa) rt_scalar_lines<D, 0, RT_PMS, TR>(g, a.m, u, a.rhs, a.o, (long)w2 * L, a.tau, lds, a.status);
    else rt_scalar_lines<D, 1, RT_PMS, TR>(g, a.m, u, a.rhs, a.o, (long)(w2 - nwa) * L, a.tau, lds, a.status);
  }
}

// Workgroups are numbered XCD-contiguously within a launch, so that the
// neighbouring lines of neighbouring workgroups (which share cache lines and
// neighbour cells) meet in one L2.
template <int D, int PM, int PART, bool B>
__global__ void __launch_bounds__(256) k_rt_part(PassArgs a, Batch bt) {
  extern __shared__ double lds[];
  if constexpr (B) {
    const int mb = batch_member(bt, blockIdx.x);
    rt_body<D, PM, PART, false, false, false, true>(batch_args(bt, mb), blockIdx.x - bt.woff[mb], lds);
  } else {
    rt_body<D, PM, PART>(a, xcd_contiguous(blockIdx.x, gridDim.x), lds);
  }
}

template <int D, int PM, int PART>
__global__ void __launch_bounds__(256) k_rt_partF(PassArgs a) {
  extern __shared__ double lds[];
  rt_body<D, PM, PART, true>(a, xcd_contiguous(blockIdx.x, gridDim.x), lds);
}

// perturbation-pressure form, one grid
template <int D, int PM, int PART>
__global__ void __launch_bounds__(256) k_rt_partP(PassArgs a) {
  extern __shared__ double lds[];
  rt_body<D, PM, PART, false, false, true>(a, xcd_contiguous(blockIdx.x, gridDim.x), lds);
}

// transposed systems (adjoint), one grid
template <int D, int PM, int PART>
__global__ void __launch_bounds__(256) k_rt_partT(PassArgs a) {
  extern __shared__ double lds[];
  rt_body<D, PM, PART, false, true>(a, xcd_contiguous(blockIdx.x, gridDim.x), lds);
}

// From this many workgroups on, one grid's block and scalar lines run as two
// launches (the scalar lines need a fraction of the block lines' registers
// and run at a higher occupancy on their own).  Measured on the 256 x 128 x 64
// sector (4084 workgroups): r 0.22 -> 0.16 ms, theta 0.28 -> 0.19 ms; the
// same from 256 to 1024.
constexpr unsigned RT_SPLIT_WGS = 1024;

bool rt_part_supported(const Geo &g, int d, unsigned bs, int pm) {
  const Families F = families(g, d);
  return d < 2 && pm == 4 && bs <= 256 && rt_block_chunks(F.n, pm) <= (int)bs &&
         rt_chunks<RT_PMS>(F.n) <= (int)bs;
}

unsigned rt_part_blocks(const Geo &g, int d, unsigned bs, int pm) {
  return rt_block_wgs(g, d, bs, pm) + rt_scalar_wgs(g, d, bs);
}

size_t rt_part_lds(unsigned bs) { return sizeof(double) * 24 * (size_t)bs; }

template <int D, int PM>
static void launch_rt_d(const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads, hipStream_t st) {
  const size_t lds = rt_part_lds(threads), lds_s = sizeof(double) * 4 * (size_t)threads;
  if (b.tab) {
    // a batch: the members' block and scalar workgroups as two launches over
    // the same table (each leaves the other kind's workgroups at once)
    if (blocks < RT_SPLIT_WGS) {
      hipLaunchKernelGGL((k_rt_part<D, PM, 2, true>), dim3(blocks), dim3(threads), lds, st, a, b);
    } else {
      hipLaunchKernelGGL((k_rt_part<D, PM, 0, true>), dim3(blocks), dim3(threads), lds, st, a, b);
      hipLaunchKernelGGL((k_rt_part<D, PM, 1, true>), dim3(blocks), dim3(threads), lds_s, st, a, b);
    }
    return;
  }
  if (blocks < RT_SPLIT_WGS) {
    hipLaunchKernelGGL((k_rt_part<D, PM, 2, false>), dim3(blocks), dim3(threads), lds, st, a, b);
    return;
  }
  const unsigned nbw = rt_block_wgs(a.g, D, threads, PM), nsw = rt_scalar_wgs(a.g, D, threads);
  hipLaunchKernelGGL((k_rt_part<D, PM, 0, false>), dim3(nbw), dim3(threads), lds, st, a, b);
  hipLaunchKernelGGL((k_rt_part<D, PM, 1, false>), dim3(nsw), dim3(threads), lds_s, st, a, b);
}

void launch_rt_pass(int d, int pm, const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                    hipStream_t st) {
  (void)pm;  // 4: the only chunk size built (8 measured slower: one wave per SIMD)
  if (d == 0) launch_rt_d<0, 4>(a, b, blocks, threads, st);
  else launch_rt_d<1, 4>(a, b, blocks, threads, st);
}

template <int D, int PM>
static void launch_rt_T_d(const PassArgs &a, unsigned threads, hipStream_t st) {
  const size_t lds = rt_part_lds(threads), lds_s = sizeof(double) * 4 * (size_t)threads;
  const unsigned nbw = rt_block_wgs(a.g, D, threads, PM), nsw = rt_scalar_wgs(a.g, D, threads);
  if (nbw + nsw < RT_SPLIT_WGS) {
    hipLaunchKernelGGL((k_rt_partT<D, PM, 2>), dim3(nbw + nsw), dim3(threads), lds, st, a);
    return;
  }
  hipLaunchKernelGGL((k_rt_partT<D, PM, 0>), dim3(nbw), dim3(threads), lds, st, a);
  hipLaunchKernelGGL((k_rt_partT<D, PM, 1>), dim3(nsw), dim3(threads), lds_s, st, a);
}

template <int D, int PM>
static void launch_rt_pert_d(const PassArgs &a, unsigned threads, hipStream_t st) {
  const size_t lds = rt_part_lds(threads), lds_s = sizeof(double) * 4 * (size_t)threads;
  const unsigned nbw = rt_block_wgs(a.g, D, threads, PM), nsw = rt_scalar_wgs(a.g, D, threads);
  if (nbw + nsw < RT_SPLIT_WGS) {
    hipLaunchKernelGGL((k_rt_partP<D, PM, 2>), dim3(nbw + nsw), dim3(threads), lds, st, a);
    return;
  }
  hipLaunchKernelGGL((k_rt_partP<D, PM, 0>), dim3(nbw), dim3(threads), lds, st, a);
  hipLaunchKernelGGL((k_rt_partP<D, PM, 1>), dim3(nsw), dim3(threads), lds_s, st, a);
}

void launch_rt_pert(int d, const PassArgs &a, unsigned threads, hipStream_t st) {
  if (d == 0) launch_rt_pert_d<0, 4>(a, threads, st);
  else launch_rt_pert_d<1, 4>(a, threads, st);
}

void launch_rt_T(int d, const PassArgs &a, unsigned threads, hipStream_t st) {
  (void)d;  // r only: see the transposed solve's launcher in the host code
  launch_rt_T_d<0, 4>(a, threads, st);
}

// Where the scalar lines of a two-ended sweep run apart, by the partitioned
// solver: lines whose chunks are all full and fill the workgroup (n a
// multiple of the rows per thread, a chunk count dividing the workgroup).
// Measured: theta on the 512 x 256 x 128 sphere (256 rows) 1.53 -> 1.43 ms;
// on 64 uneven sectors (lines of 64 to 256 rows) the ragged chunks and idle
// lanes made the two passes slower than the one two-ended launch.
bool rt_scalar_supported(const Geo &g, int d, unsigned bs) {
  if (d > 1 || bs > 256) return false;
  const int n = families(g, d).n, T = rt_chunks<RT_PMS>(n);
  return n % RT_PMS == 0 && T <= (int)bs && bs % (unsigned)T == 0 && rt_scalar_wgs(g, d, bs) > 0;
}

unsigned rt_scalar_blocks(const Geo &g, int d, unsigned bs) { return rt_scalar_wgs(g, d, bs); }

size_t rt_scalar_lds(unsigned bs) { return sizeof(double) * 4 * (size_t)bs; }

// The scalar lines of an r or theta sweep alone (after a two-ended solve of
// its block lines): one grid (workgroups numbered XCD-contiguously) or a
// batch (each member's scalar workgroups from 0).  Without the scalar lines
// the two-ended solve's scratch traffic drops by a sixth: theta on the
// 512 x 256 x 128 sphere 1.53 -> 1.43 ms.
template <int D, bool B>
__global__ void __launch_bounds__(256) k_rt_scal(PassArgs a, Batch bt) {
  extern __shared__ double lds[];
  if constexpr (B) {
    const int mb = batch_member(bt, blockIdx.x);
    rt_body<D, 4, 1>(batch_args(bt, mb), blockIdx.x - bt.woff[mb], lds);
  } else {
    rt_body<D, 4, 1>(a, xcd_contiguous(blockIdx.x, gridDim.x), lds);
  }
}

void launch_rt_scalar_pass(int d, const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                           hipStream_t st) {
  const size_t lds = rt_scalar_lds(threads);
  const dim3 gr(blocks), bl(threads);
  if (b.tab) {
    if (d == 0) hipLaunchKernelGGL((k_rt_scal<0, true>), gr, bl, lds, st, a, b);
    else hipLaunchKernelGGL((k_rt_scal<1, true>), gr, bl, lds, st, a, b);
  } else {
    if (d == 0) hipLaunchKernelGGL((k_rt_scal<0, false>), gr, bl, lds, st, a, b);
    else hipLaunchKernelGGL((k_rt_scal<1, false>), gr, bl, lds, st, a, b);
  }
}

// the solver a grid takes by default: partitioned where a block line
// splits into at most 32 chunks (L >= 8 neighbouring lines per 256-thread
// workgroup), else two-ended.  Measured: partitioned r 0.16 / theta 0.19 ms
// against 0.20 / 0.31 ms two-ended on the 256 x 128 x 64 sector (64 and 128
// rows); theta on the 512 x 256 x 128 sphere (256 rows, 64 chunks) 1.74
// against 1.63 ms.
int rt_default_pm(const Geo &g, int d) {
  return rt_part_supported(g, d, 256, 4) && rt_block_chunks(families(g, d).n, 4) <= 32 ? 4 : 0;
}

template <int D, int PM>
static void launch_rt_forced_d(const PassArgs &a, unsigned threads, hipStream_t st) {
  const size_t lds = rt_part_lds(threads), lds_s = sizeof(double) * 4 * (size_t)threads;
  const unsigned nbw = rt_block_wgs(a.g, D, threads, PM), nsw = rt_scalar_wgs(a.g, D, threads);
  if (nbw + nsw < RT_SPLIT_WGS) {
    hipLaunchKernelGGL((k_rt_partF<D, PM, 2>), dim3(nbw + nsw), dim3(threads), lds, st, a);
    return;
  }
  hipLaunchKernelGGL((k_rt_partF<D, PM, 0>), dim3(nbw), dim3(threads), lds, st, a);
  hipLaunchKernelGGL((k_rt_partF<D, PM, 1>), dim3(nsw), dim3(threads), lds_s, st, a);
}

void launch_rt_forced(int d, int pm, const PassArgs &a, unsigned threads, hipStream_t st) {
  (void)pm;
  if (d == 0) launch_rt_forced_d<0, 4>(a, threads, st);
  else launch_rt_forced_d<1, 4>(a, threads, st);
}

} // namespace dsw
