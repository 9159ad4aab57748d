// dsw_internal.hpp -- declarations shared by the host API and the kernel
// translation units of libdsw (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "dsw_common.hpp"

namespace dsw {

// device status words, each set by plain stores of 1 (no atomics)
enum { ST_NONPHYS = 0, ST_SINGULAR = 1, ST_WORDS = 2 };

struct Fields {
  double *p, *ur, *ut, *uf, *T;
};

// Destination of a sweep.  mode 0: x = solution (boundary-normal faces of x
// are zeroed).  mode 1: x = base + solution at every unknown (x may alias
// base); when ub.p is set, also ub = (x + un)/2 there (the midpoint state of
// the next iteration).
struct Out {
  Fields x, base, ub, un;
  int mode;
};

// workspace of the line solvers: intermediates of the forward elimination
struct Scratch {
  double *blk;   // block lines
  double *sca;   // scalar lines
  long blk_len;  // doubles available
  long sca_len;
};

void launch_residual(const Geo &g, const Mat &m, const Fields &Un, const Fields &Uk, double tau,
                     const Fields &R, const Fields &Ub, int *status, hipStream_t st);

// d = 0 (r), 1 (theta), 2 (phi).  If upd is non-null (phi sweep of a split
// step), the solution is added to upd instead of being stored in x.
void launch_sweep(int d, const Geo &g, const Mat &m, const Fields &Ub, double tau,
                  const Fields &rhs, const Out &o, const Scratch &sc, int *status, hipStream_t st);

// residual with the midpoint state already resident (split-step internal);
// Uk may be the same arrays as Un (first iteration: no difference term)
void launch_residual_given_mid(const Geo &g, const Mat &m, const Fields &Un, const Fields &Uk,
                               const Fields &Ub, double tau, const Fields &R, int *status,
                               hipStream_t st);

// copy the boundary-normal faces of src into dst (skipped where dst.p is null)
void launch_bnd_copy(const Geo &g, const Fields &src, const Fields &d0, const Fields &d1,
                     const Fields &d2, hipStream_t st);

// partitioned phi solver (one workgroup per line slot), when the line fits
bool phi_part_supported(const Geo &g);
void launch_phi_part(const Geo &g, const Mat &m, const Fields &Ub, double tau, const Fields &rhs,
                     const Out &o, int *status, hipStream_t st);

// doubles of scratch needed by the sweeps of a grid
void sweep_scratch_size(const Geo &g, long *blk, long *sca);

} // namespace dsw
