// dsw_internal.hpp -- declarations shared by the host API and the kernel
// translation units of libdsw (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "dsw_common.hpp"

namespace dsw {

// Occupancy targets (waves per SIMD) of the hot kernels: the compiler then
// keeps their registers within 512 / target.  0 leaves the choice to it.
#ifndef DSW_WAVES_RES
#define DSW_WAVES_RES 0
#endif
#ifndef DSW_WAVES_SWEEP
#define DSW_WAVES_SWEEP 0
#endif
#ifndef DSW_WAVES_PHI
#define DSW_WAVES_PHI 0
#endif
#define DSW_OCC(w) __attribute__((amdgpu_waves_per_eu((w) > 0 ? (w) : 1)))

// device status words, each set by plain stores of 1 (no atomics)
enum { ST_NONPHYS = 0, ST_SINGULAR = 1, ST_DIVERGED = 2, ST_WORDS = 3 };

struct Fields {
  double *p, *ur, *ut, *uf, *T;
};

// Destination of a sweep.  mode 0: x = solution (boundary-normal faces of x
// are zeroed).  mode 1: x = base + solution at every unknown (x may alias
// base); when ub.p is set, also ub = (x + un)/2 there (the midpoint state of
// the next iteration); when raw.p is set, also raw = solution there.
struct Out {
  Fields x, base, ub, un, raw;
  int mode;
};

// -(Uk - Un) at a point; zero when the two states are the same array
struct Diff {
  const double *k[5], *n[5];
  int same;
  __device__ __forceinline__ double at(int f, long x) const { return same ? 0.0 : k[f][x] - n[f][x]; }
};

// workspace of the line solvers: intermediates of the forward elimination
struct Scratch {
  double *blk;   // block lines
  double *sca;   // scalar lines
  long blk_len;  // doubles available
  long sca_len;
};

// Everything one pass (one kernel) needs for one grid.  Fields a pass does
// not use are left zero.
struct PassArgs {
  Geo g;
  Mat m;
  SrcOne u;          // midpoint state: residual operand / sweep coefficients
  Diff d;            // residual: -(Uk - Un)
  double tau;        // residual: tau; sweeps: tau/2
  Fields rhs;        // sweeps: right-hand side
  Fields R;          // residual: output
  Out o;             // sweeps: destination
  double *scb, *scs; // sweeps: scratch of block and scalar lines
  int *status;
  Fields src, d0, d1, d2; // boundary-face copy: src -> d0, d1, d2
  Wall wall;              // forced passes: tangential wall velocities
  Fields fsrc;            // forced residual: source term (null entries: none)
  const double *pref, *tref; // perturbation-pressure passes: reference column [nr]
};

// The state source of a pass: the plain midpoint (zero wall velocities),
// for a forced pass (W) the midpoint with the wall velocities and the
// source, for a perturbation-pressure pass (PT) the midpoint with the
// reference column.
template <bool W, bool PT = false>
struct SrcSel {
  __device__ static __forceinline__ const SrcOne &get(const PassArgs &a) { return a.u; }
};
template <>
struct SrcSel<false, true> {
  __device__ static __forceinline__ SrcPert<SrcOne> get(const PassArgs &a) {
    SrcPert<SrcOne> s;
#pragma unroll
    for (int q = 0; q < 5; q++) s.a[q] = a.u.a[q];
    s.pref = a.pref;
    s.tref = a.tref;
    return s;
  }
};
template <>
struct SrcSel<true, false> {
  __device__ static __forceinline__ SrcW get(const PassArgs &a) {
    SrcW s;
#pragma unroll
    for (int q = 0; q < 5; q++) s.a[q] = a.u.a[q];
    s.w = a.wall;
    s.f[F_P] = a.fsrc.p; s.f[F_UR] = a.fsrc.ur; s.f[F_UT] = a.fsrc.ut; s.f[F_UF] = a.fsrc.uf;
    s.f[F_T] = a.fsrc.T;
    return s;
  }
};

// The interior sources of a pass over slots whose stencils read no ghost
// across an r or theta boundary (32-bit indices; P: periodic phi): plain,
// perturbation-pressure form (PT) or forced (W).
template <bool W, bool PT, bool P>
struct SrcSelIn {
  __device__ static __forceinline__ SrcOneT<true, P> get(const PassArgs &a) {
    SrcOneT<true, P> s;
#pragma unroll
    for (int q = 0; q < 5; q++) s.a[q] = a.u.a[q];
    return s;
  }
};
template <bool P>
struct SrcSelIn<false, true, P> {
  __device__ static __forceinline__ SrcPert<SrcOneT<true, P>> get(const PassArgs &a) {
    SrcPert<SrcOneT<true, P>> s;
#pragma unroll
    for (int q = 0; q < 5; q++) s.a[q] = a.u.a[q];
    s.pref = a.pref;
    s.tref = a.tref;
    return s;
  }
};
template <bool P>
struct SrcSelIn<true, false, P> {
  __device__ static __forceinline__ SrcInW<P> get(const PassArgs &a) {
    SrcInW<P> s;
#pragma unroll
    for (int q = 0; q < 5; q++) s.a[q] = a.u.a[q];
    s.w = a.wall;
    s.f[F_P] = a.fsrc.p; s.f[F_UR] = a.fsrc.ur; s.f[F_UT] = a.fsrc.ut; s.f[F_UF] = a.fsrc.uf;
    s.f[F_T] = a.fsrc.T;
    return s;
  }
};

// One launch over several grids.  Workgroup w belongs to member m with
// woff[m] <= w < woff[m+1] (woff has n+1 entries, woff[0] = 0); tab[m] is
// that member's PassArgs.  tab == nullptr: a single grid, passed by value.
// In device code the table is seen through the constant address space: the
// kernels never write it, and so its loads stay scalar (a generic pointer
// would turn every use of a member's arguments into a vector load, reloaded
// after every store).
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) PassArgs CPassArgs;
#else
typedef const PassArgs CPassArgs;
#endif
struct Batch {
  CPassArgs *tab;
  const unsigned *woff;
  int n;
};

// member m's arguments, as a reference the pass bodies take
__device__ __forceinline__ const PassArgs &batch_args(const Batch &b, int m) {
  return (const PassArgs &)b.tab[m];
}

// Launch shapes (the tunable parameters).
struct Cfg {
  int res_bs;      // residual: threads per workgroup along phi (64, 128, 256)
  int sweep_bs[2]; // r and theta sweeps: lines per workgroup (64, 128, 256)
  int phi_pm;      // phi sweep: 0 = one thread per line, 2 or 4 = partitioned
                   // with that many rows per thread
  int rt_pm[2];    // r and theta sweeps: 0 = two threads per line, 4 =
                   // partitioned (4 rows per thread on the block lines)
};

// PK_SW0T / PK_SW1T: a two-ended r / theta sweep over every line; where the
// partitioned scalar-line solver takes the grid it runs as two passes, the
// block lines two-ended (PK_SW0B / PK_SW1B) and then the scalar lines
// partitioned (PK_SW0S / PK_SW1S).  PK_NONE: a pass that launches nothing
// (it keeps the passes of different grids' steps aligned).
enum PassKind { PK_BND = 0, PK_RES = 1, PK_SW0 = 2, PK_SW1 = 3, PK_SW2_LINE = 4, PK_SW2_PART = 5,
                PK_RES_IN = 6, PK_SW0T = 7, PK_SW1T = 8, PK_RES_INP = 9, PK_SW0P = 10, PK_SW1P = 11,
                PK_SW0B = 12, PK_SW1B = 13, PK_SW0S = 14, PK_SW1S = 15, PK_NONE = 16,
                PK_SW2_CP = 17, PK_SW2_CN = 18 };
// PK_SW2_CP / PK_SW2_CN: the partitioned phi pass of a grid with an interior
// (periodic / bounded phi); in a batch, each member's ring slots and then its
// interior slots (the interior ones through the interior source).

// forced split step (source term, wall velocities, Dirichlet data at the new
// time level): one grid, the general residual over every point, the
// two-ended r and theta sweeps and the partitioned phi solver
void launch_bnd_forced(const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st);
void launch_residual_forced(const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st);
void launch_sweep2_forced(int d, const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st);
// first iteration of a forced step: rhs -= tau/2 D_d(Ubar) X_b for the change
// X_b of the boundary data (a.d0 - a.src on the boundary-normal faces, dw on
// the walls), in place on a.rhs
void launch_lift(int d, const PassArgs &a, const Wall &dw, hipStream_t st);
// mean and change of two sets of the twelve wall arrays
struct WallMix {
  const double *a[12], *b[12];
  double *mid[12], *dw[12];
  long off[13];  // prefix sums of the array lengths
};
void launch_wall_mix(const WallMix &w, hipStream_t st);
void launch_phi_forced(int pm, const PassArgs &a, unsigned blocks, unsigned threads, size_t lds,
                       hipStream_t st);
void launch_rt_forced(int d, int pm, const PassArgs &a, unsigned threads, hipStream_t st);
// transposed r systems (adjoint) by the partitioned solver (d = 0 only)
void launch_rt_T(int d, const PassArgs &a, unsigned threads, hipStream_t st);
// the scalar lines of an r or theta sweep alone, partitioned (one grid or a
// batch; workgroups numbered from 0 per grid)
bool rt_scalar_supported(const Geo &g, int d, unsigned bs);
unsigned rt_scalar_blocks(const Geo &g, int d, unsigned bs);
size_t rt_scalar_lds(unsigned bs);
void launch_rt_scalar_pass(int d, const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                           hipStream_t st);
// the r / theta solver a grid takes by default (4 partitioned, 0 two-ended)
int rt_default_pm(const Geo &g, int d);

// r and theta sweeps take two threads per line (two-ended elimination) on
// grids with fewer block lines than this; measured faster than one thread
// per line on every grid tried (2^12 .. 2^17 block lines of 64 .. 256 rows)
constexpr long TWIST_LINES = 1L << 24;

// kernel launchers of the passes: by value for one grid (b.tab == nullptr), or
// over a batch (blocks = sum over the members, threads and lds = maxima)
void launch_residual_pass(const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                          hipStream_t st);
void launch_residual_in_pass(bool periodic, const PassArgs &a, const Batch &b, unsigned blocks,
                             unsigned threads, hipStream_t st);
unsigned residual_interior_blocks(const Geo &g, int bs); // workgroups of the interior launch
// workgroups of the general residual launch (the shell when the interior
// launch runs, else every point)
unsigned residual_general_blocks(const Geo &g, int bs);
void launch_sweep_pass(int d, const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                       hipStream_t st);
void launch_phi_pass(int pm, const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                     size_t lds, hipStream_t st);
void launch_bnd_pass(const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                     hipStream_t st);
unsigned sweep_lines(const Geo &g, int d);   // lines of all families of sweep d
// r and theta sweeps with two threads per block line (twisted factorisation)
void launch_sweep2_pass(int d, const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                        hipStream_t st);
unsigned sweep2_blocks(const Geo &g, int d, unsigned bs);
// the block-line workgroups alone of a two-ended r or theta sweep
unsigned sweep2_block_blocks(const Geo &g, int d, unsigned bs);
// r and theta sweeps, partitioned: workgroups of bs threads, each on a few
// neighbouring lines split into chunks (block lines, then scalar lines)
// (pm rows per thread on the block lines: 4)
bool rt_part_supported(const Geo &g, int d, unsigned bs, int pm);
unsigned rt_part_blocks(const Geo &g, int d, unsigned bs, int pm);
size_t rt_part_lds(unsigned bs);
void launch_rt_pass(int d, int pm, const PassArgs &a, const Batch &b, unsigned blocks, unsigned threads,
                    hipStream_t st);
unsigned bnd_points(const Geo &g);           // boundary-normal faces
unsigned phi_part_threads(const Geo &g, int pm);
size_t phi_part_lds(const Geo &g, int pm);

// adjoint pieces: transposed line solves (one thread per line), the
// transposed Jacobians of the residual and of the line operators (both
// accumulate into acc), and elementwise helpers
void launch_sweep_T(int d, const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st);
void launch_sweep2_T(int d, const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st);
void launch_phi_T(int pm, const PassArgs &a, unsigned blocks, unsigned threads, size_t lds,
                  hipStream_t st);
void launch_residual_vjp(const Geo &g, const Mat &m, const Fields &Ub, double tau, const Fields &mu,
                         const Fields &acc, hipStream_t st);
void launch_line_vjp(int d, const Geo &g, const Mat &m, const Fields &Ub, double tau, const Fields &X,
                     const Fields &mu, const Fields &acc, hipStream_t st);
// one reverse iteration's local functions at once (cells, then r, theta, phi
// faces): acc += (d(-tau F_h)/dUbar)^T mu[0] - sum_d (d(M_d X[d])/dUbar)^T mu[d]
void launch_adj_local(const Geo &g, const Mat &m, const Fields &Ub, double tau, const Fields *X,
                      const Fields *mu, const Fields &acc, hipStream_t st);
void launch_axpy3(const long *cnt, double a, const Fields &x, double b, const Fields &y, double c,
                  const Fields &z, const Fields &out, hipStream_t st);
void launch_adj_mix(const Geo &g, const long *cnt, const Fields &L, const Fields &mu1, const Fields &ubb,
                    const Fields &Lnew, const Fields &lam, bool fold, bool first, hipStream_t st);

// perturbation-pressure split step (one grid): the residual (interior and
// general launches), the partitioned r / theta solver, the two-ended
// r / theta solver and the partitioned phi solver with the reference column
// (a.pref, a.tref) of the state's pressure
void launch_residual_pert(const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st);
void launch_rt_pert(int d, const PassArgs &a, unsigned threads, hipStream_t st);
void launch_sweep2_pert(int d, const PassArgs &a, unsigned blocks, unsigned threads, hipStream_t st);
void launch_phi_pert(int pm, const PassArgs &a, unsigned blocks, unsigned threads, size_t lds, hipStream_t st);

// Courant numbers (advective, acoustic) of a state for the step tau into
// out[0], out[1] (device, as the bit patterns of non-negative doubles)
void launch_courant(const Geo &g, const Mat &m, const Fields &U, double tau, unsigned long long *out,
                    hipStream_t st);

// public residual: forms the midpoint on the fly from Un and Uk and writes it
void launch_residual(const Geo &g, const Mat &m, const Fields &Un, const Fields &Uk, double tau,
                     const Fields &R, const Fields &Ub, int *status, hipStream_t st);

// partitioned phi solver: whether a grid's phi lines fit it
bool phi_part_supported(const Geo &g, int pm);

// doubles of scratch needed by the sweeps of a grid
void sweep_scratch_size(const Geo &g, long *blk, long *sca);

// the kind of the phi pass of a grid under a configuration
// whether a grid's phi pass can take its interior slots through the
// interior source (it has an interior, and 32-bit indices reach)
bool phi_interior_split(const Geo &g);
// a batch of grids that all have an interior (P: periodic phi): each
// member's boundary ring, then its interior slots
void launch_phi_pass_c(int pm, bool periodic, const PassArgs &a, const Batch &b, unsigned blocks,
                       unsigned threads, size_t lds, hipStream_t st);
inline int phi_kind(const Geo &g, const Cfg &c) {
  if (!(c.phi_pm > 0 && phi_part_supported(g, c.phi_pm))) return PK_SW2_LINE;
  if (phi_interior_split(g)) return g.periodic ? PK_SW2_CP : PK_SW2_CN;
  return PK_SW2_PART;
}

// Workgroups go to the chip's 8 XCDs in turn (w mod 8), and each XCD has an
// L2 of its own.  Renumbered by this bijection of [0, n), every XCD takes one
// contiguous range of n work items, so that items next to each other, which
// read each other's neighbour data, share an L2.  Used where that pays: the
// scalar lines of the three sweeps (bandwidth-bound); the block lines and the
// residual keep the round-robin order, which spreads every moment's accesses
// over the whole grid and measured faster for them.
__device__ __forceinline__ unsigned xcd_contiguous(unsigned w, unsigned n) {
  const unsigned x = w & 7u, i = w >> 3, q = n >> 3, r = n & 7u;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// member lookup of a batched launch (binary search over the offsets)
__device__ __forceinline__ int batch_member(const Batch &b, unsigned w) {
  int lo = 0, hi = b.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.woff[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

} // namespace dsw
