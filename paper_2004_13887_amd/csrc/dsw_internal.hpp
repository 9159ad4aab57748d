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
                  const Fields &rhs, const Fields &x, const Scratch &sc, int *status,
                  hipStream_t st, bool accum);

// partitioned phi solver (one workgroup per line slot), when the line fits
bool phi_part_supported(const Geo &g);
void launch_phi_part(const Geo &g, const Mat &m, const Fields &Ub, double tau, const Fields &rhs,
                     const Fields &x, int *status, hipStream_t st, bool accum);

// doubles of scratch needed by the sweeps of a grid
void sweep_scratch_size(const Geo &g, long *blk, long *sca);

} // namespace dsw
