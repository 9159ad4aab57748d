// dsw_common.hpp -- device-side geometry, ghost rules and coefficient fields
// shared by the residual and line-solve kernels of libdsw (gfx950, FP64).
//
// MAC grid (paper section 2.2, "standard central differences on the MAC
// stencil"): p, T at cell centres, u_r / u_theta / u_phi on the r / theta /
// phi faces; arrays are C-order with phi fastest.  Ghost values outside the
// grid: p, T copy the interior value (zero normal gradient); a velocity
// component tangential to a wall takes minus the interior value (no-slip);
// across a pole u_r is copied and u_phi negated; phi wraps when periodic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsw {

enum { F_P = 0, F_UR = 1, F_UT = 2, F_UF = 3, F_T = 4 };

struct Geo {
  int nr, nt, np, npf;
  int periodic, pole_lo, pole_hi;
  double dr, dt, dp;
  double idr, idt, idp;    // reciprocals of the spacings
  const double *rc, *rf;   // centre radii [nr], face radii [nr+1]
  const double *sc, *cc;   // sin, cos of theta at centres [nt]
  const double *sf, *cf;   // sin, cos of theta at faces [nt+1]
  const double *irc, *irf; // 1/rc, 1/rf
  const double *isc, *ctc; // 1/sin, cot at centres
  const double *isf, *ctf; // 1/sin, cot at faces (0 at a pole face: never used there)
  const double *scx;       // sin of theta at centres j = -1 .. nt (ghosts included), at scx[j + 1]
};

struct Mat {
  double gam, Rg, pinf, mu, kap, omega, g_r;
};

__device__ __forceinline__ long idx_c(const Geo &g, int i, int j, int k) {
  return ((long)i * g.nt + j) * g.np + k;
}
__device__ __forceinline__ long idx_r(const Geo &g, int f, int j, int k) {
  return ((long)f * g.nt + j) * g.np + k;
}
__device__ __forceinline__ long idx_t(const Geo &g, int i, int f, int k) {
  return ((long)i * (g.nt + 1) + f) * g.np + k;
}
__device__ __forceinline__ long idx_f(const Geo &g, int i, int j, int f) {
  return ((long)i * g.nt + j) * g.npf + f;
}
__device__ __forceinline__ int wrapk(const Geo &g, int k) {
  return k < 0 ? k + g.np : (k >= g.np ? k - g.np : k);
}
__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// State sources: a single array set, or the midpoint of two.  INTERIOR: the
// caller guarantees that every neighbour a stencil reads lies inside the
// arrays in r and theta; the ghost rules in phi (wrap when periodic, else the
// zero-gradient copy for p, T and the no-slip sign for u_r, u_theta) are
// applied without branches, and indices are 32-bit.
template <bool I, bool P = false>
struct SrcOneT {
  const double *a[5];
  static constexpr bool INTERIOR = I;
  static constexpr bool PERIODIC = P; // interior sources: phi periodic (known at compile time)
  static constexpr bool WALL = false;  // tangential wall velocities are zero
  static constexpr bool PERT = false;  // p holds the full pressure
  __device__ __forceinline__ double ld(int f, long x) const { return a[f][x]; }
};
using SrcOne = SrcOneT<false>;
using SrcInN = SrcOneT<true, false>; // interior, phi bounded by walls
using SrcInP = SrcOneT<true, true>;  // interior, phi periodic
struct SrcMid {
  const double *n[5], *k[5];
  static constexpr bool INTERIOR = false;
  static constexpr bool PERIODIC = false;
  static constexpr bool WALL = false;
  static constexpr bool PERT = false;
  __device__ __forceinline__ double ld(int f, long x) const { return 0.5 * (k[f][x] + n[f][x]); }
};

// Tangential velocities on the non-periodic walls (device arrays; a null
// entry is a zero wall velocity).  A ghost value across a wall is 2 g - u of
// the interior neighbour.  Shapes:
//   ur_t1, ur_t2 [nr+1][np]   u_r on the theta walls   ur_p1, ur_p2 [nr+1][nt]   on the phi walls
//   ut_r1, ut_r2 [nt+1][np]   u_theta on the r walls   ut_p1, ut_p2 [nr][nt+1]   on the phi walls
//   uf_r1, uf_r2 [nt][npf]    u_phi on the r walls     uf_t1, uf_t2 [nr][npf]    on the theta walls
struct Wall {
  const double *ur_t1, *ur_t2, *ur_p1, *ur_p2;
  const double *ut_r1, *ut_r2, *ut_p1, *ut_p2;
  const double *uf_r1, *uf_r2, *uf_t1, *uf_t2;
};
__device__ __forceinline__ double wallv(const double *w, long x) { return w ? w[x] : 0.0; }

// A forced source: the state with wall velocities, plus a source term that
// the residual adds to -F_h (paper section 3.1, manufactured solutions)
struct SrcW {
  const double *a[5];
  Wall w;
  const double *f[5]; // source at the midpoint time; null: none
  static constexpr bool INTERIOR = false;
  static constexpr bool PERIODIC = false;
  static constexpr bool WALL = true;
  static constexpr bool PERT = false;
  __device__ __forceinline__ double ld(int fid, long x) const { return a[fid][x]; }
};

// A forced source for the interior residual launch (every r and theta
// neighbour inside the arrays): ghosts only across phi walls (P: periodic)
template <bool P>
struct SrcInW {
  const double *a[5];
  Wall w;
  const double *f[5];
  static constexpr bool INTERIOR = true;
  static constexpr bool PERIODIC = P;
  static constexpr bool WALL = true;
  static constexpr bool PERT = false;
  __device__ __forceinline__ double ld(int fid, long x) const { return a[fid][x]; }
};

// The perturbation-pressure form of a plain source (dsw_split_step_pert):
// the state's p holds p - pref(r) for a discretely hydrostatic reference
// column (pref, tref) at the centres.  Where the pressure enters as a
// coefficient (density, P), rho_at and centre add pref back; differences of
// p stay differences of p' (pref depends on r only, and the r terms that
// see it are written out in the residual).
template <class B>
struct SrcPert : B {
  const double *pref, *tref;  // [nr]
  static constexpr bool PERT = true;
};

// Velocity ghosts of a forced source: across a wall 2 g - u (g the wall's
// tangential velocity), the phi wall first, then the theta or r wall; across
// a pole the symmetry ghosts of the plain rules.
template <class S>
__device__ __forceinline__ double gR_wall(const Geo &g, const S &s, int f, int j, int k) {
  double sg = 1.0, add = 0.0;
  if (k < 0 || k >= g.np) {
    if (g.periodic) k = wrapk(g, k);
    else {
      add = 2.0 * wallv(k < 0 ? s.w.ur_p1 : s.w.ur_p2, (long)f * g.nt + clampi(j, 0, g.nt - 1));
      sg = -sg; k = k < 0 ? 0 : g.np - 1;
    }
  }
  if (j < 0) {
    if (!g.pole_lo) { add += sg * 2.0 * wallv(s.w.ur_t1, (long)f * g.np + k); sg = -sg; }
    j = 0;
  } else if (j >= g.nt) {
    if (!g.pole_hi) { add += sg * 2.0 * wallv(s.w.ur_t2, (long)f * g.np + k); sg = -sg; }
    j = g.nt - 1;
  }
  return add + sg * s.ld(F_UR, idx_r(g, f, j, k));
}
template <class S>
__device__ __forceinline__ double gT_wall(const Geo &g, const S &s, int i, int f, int k) {
  double sg = 1.0, add = 0.0;
  if (k < 0 || k >= g.np) {
    if (g.periodic) k = wrapk(g, k);
    else {
      add = 2.0 * wallv(k < 0 ? s.w.ut_p1 : s.w.ut_p2, (long)clampi(i, 0, g.nr - 1) * (g.nt + 1) + f);
      sg = -sg; k = k < 0 ? 0 : g.np - 1;
    }
  }
  if (i < 0) { add += sg * 2.0 * wallv(s.w.ut_r1, (long)f * g.np + k); sg = -sg; i = 0; }
  else if (i >= g.nr) { add += sg * 2.0 * wallv(s.w.ut_r2, (long)f * g.np + k); sg = -sg; i = g.nr - 1; }
  return add + sg * s.ld(F_UT, idx_t(g, i, f, k));
}
template <class S>
__device__ __forceinline__ double gF_wall(const Geo &g, const S &s, int i, int j, int f) {
  double sg = 1.0, add = 0.0;
  if (g.periodic) f = wrapk(g, f);
  if (j < 0 || j >= g.nt) {
    const bool pole = j < 0 ? g.pole_lo : g.pole_hi;
    if (!pole) add = 2.0 * wallv(j < 0 ? s.w.uf_t1 : s.w.uf_t2, (long)clampi(i, 0, g.nr - 1) * g.npf + f);
    sg = -sg; j = j < 0 ? 0 : g.nt - 1;
  }
  if (i < 0) { add += sg * 2.0 * wallv(s.w.uf_r1, (long)j * g.npf + f); sg = -sg; i = 0; }
  else if (i >= g.nr) { add += sg * 2.0 * wallv(s.w.uf_r2, (long)j * g.npf + f); sg = -sg; i = g.nr - 1; }
  return add + sg * s.ld(F_UF, idx_f(g, i, j, f));
}

// p or T at a (possibly ghost) centre
template <class S>
__device__ __forceinline__ double gC(const Geo &g, const S &s, int fid, int i, int j, int k) {
  if constexpr (S::INTERIOR) {
    const int kk = S::PERIODIC ? wrapk(g, k) : clampi(k, 0, g.np - 1);
    return s.ld(fid, (i * g.nt + j) * g.np + kk);
  }
  i = clampi(i, 0, g.nr - 1);
  j = clampi(j, 0, g.nt - 1);
  k = g.periodic ? wrapk(g, k) : clampi(k, 0, g.np - 1);
  return s.ld(fid, idx_c(g, i, j, k));
}
// u_r at r-face f (0..nr), ghosts across theta and phi boundaries
template <class S>
__device__ __forceinline__ double gR(const Geo &g, const S &s, int f, int j, int k) {
  if constexpr (S::INTERIOR) {
    if constexpr (S::PERIODIC) return s.ld(F_UR, (f * g.nt + j) * g.np + wrapk(g, k));
    const int kk = clampi(k, 0, g.np - 1);
    const double v = s.ld(F_UR, (f * g.nt + j) * g.np + kk);
    if constexpr (S::WALL) return kk == k ? v : 2.0 * wallv(k < 0 ? s.w.ur_p1 : s.w.ur_p2, (long)f * g.nt + j) - v;
    return kk == k ? v : -v;
  }
  if constexpr (S::WALL) return gR_wall(g, s, f, j, k);
  double sg = 1.0;
  if (k < 0 || k >= g.np) {
    if (g.periodic) k = wrapk(g, k);
    else { sg = -sg; k = k < 0 ? 0 : g.np - 1; }
  }
  if (j < 0) { if (!g.pole_lo) sg = -sg; j = 0; }
  else if (j >= g.nt) { if (!g.pole_hi) sg = -sg; j = g.nt - 1; }
  return sg * s.ld(F_UR, idx_r(g, f, j, k));
}
// u_theta at theta-face f (0..nt), ghosts across r and phi boundaries
template <class S>
__device__ __forceinline__ double gT(const Geo &g, const S &s, int i, int f, int k) {
  if constexpr (S::INTERIOR) {
    if constexpr (S::PERIODIC) return s.ld(F_UT, (i * (g.nt + 1) + f) * g.np + wrapk(g, k));
    const int kk = clampi(k, 0, g.np - 1);
    const double v = s.ld(F_UT, (i * (g.nt + 1) + f) * g.np + kk);
    if constexpr (S::WALL) return kk == k ? v : 2.0 * wallv(k < 0 ? s.w.ut_p1 : s.w.ut_p2, (long)i * (g.nt + 1) + f) - v;
    return kk == k ? v : -v;
  }
  if constexpr (S::WALL) return gT_wall(g, s, i, f, k);
  double sg = 1.0;
  if (k < 0 || k >= g.np) {
    if (g.periodic) k = wrapk(g, k);
    else { sg = -sg; k = k < 0 ? 0 : g.np - 1; }
  }
  if (i < 0) { sg = -sg; i = 0; }
  else if (i >= g.nr) { sg = -sg; i = g.nr - 1; }
  return sg * s.ld(F_UT, idx_t(g, i, f, k));
}
// u_phi at phi-face f, ghosts across r and theta boundaries (poles included)
template <class S>
__device__ __forceinline__ double gF(const Geo &g, const S &s, int i, int j, int f) {
  if constexpr (S::INTERIOR) return s.ld(F_UF, (i * g.nt + j) * g.npf + (S::PERIODIC ? wrapk(g, f) : f));
  if constexpr (S::WALL) return gF_wall(g, s, i, j, f);
  double sg = 1.0;
  if (g.periodic) f = wrapk(g, f);
  if (j < 0) { sg = -sg; j = 0; }
  else if (j >= g.nt) { sg = -sg; j = g.nt - 1; }
  if (i < 0) { sg = -sg; i = 0; }
  else if (i >= g.nr) { sg = -sg; i = g.nr - 1; }
  return sg * s.ld(F_UF, idx_f(g, i, j, f));
}

// the pressure at a (possibly ghost) centre as a coefficient: the stored
// value, plus the reference column's (ghost rows copy the nearest) in the
// perturbation form
template <class S>
__device__ __forceinline__ double pcoef(const Geo &g, const S &s, int i, int j, int k) {
  double p = gC(g, s, F_P, i, j, k);
  if constexpr (S::PERT) p += s.pref[clampi(i, 0, g.nr - 1)];
  return p;
}

// 1 / x from the hardware reciprocal estimate refined by two Newton-Raphson
// steps (e = 1 - x r, r <- r + r e): within an ulp of the rounded quotient
// for normal x, with half the instructions of the IEEE division sequence;
// x = 0 or a non-finite x gives a non-finite result.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

template <class S>
__device__ __forceinline__ double rho_at(const Geo &g, const Mat &m, const S &s, int i, int j, int k) {
  return (pcoef(g, s, i, j, k) + m.pinf) / (m.Rg * gC(g, s, F_T, i, j, k));
}

// 1 / (0.5 (rho_a + rho_b)), the inverse mean density of two cells, with one
// reciprocal instead of three divisions: 2 R T_a T_b / ((p_a + pi_inf) T_b + (p_b + pi_inf) T_a)
template <class S>
__device__ __forceinline__ double irho_mean(const Geo &g, const Mat &m, const S &s, int ia, int ja, int ka,
                                            int ib, int jb, int kb) {
  const double pa = pcoef(g, s, ia, ja, ka) + m.pinf, pb = pcoef(g, s, ib, jb, kb) + m.pinf;
  const double ta = gC(g, s, F_T, ia, ja, ka), tb = gC(g, s, F_T, ib, jb, kb);
  return 2.0 * m.Rg * ta * tb * rcp_nr(pa * tb + pb * ta);
}

// Coefficient fields at a centre: centre-averaged velocities, thermodynamic
// factors and the velocity gradient (physical spherical components; only the
// symmetric off-diagonal sums S_ab = G_ab + G_ba are needed).
struct Cent {
  double ur, ut, uf, P, T, chi;
  double Grr, Gtt, Gff, Srt, Srf, Stf, tr, div;
};

template <class S>
__device__ __forceinline__ double avgR(const Geo &g, const S &s, int i, int j, int k) {
  return 0.5 * (gR(g, s, i, j, k) + gR(g, s, i + 1, j, k));
}
template <class S>
__device__ __forceinline__ double avgT(const Geo &g, const S &s, int i, int j, int k) {
  return 0.5 * (gT(g, s, i, j, k) + gT(g, s, i, j + 1, k));
}
template <class S>
__device__ __forceinline__ double avgF(const Geo &g, const S &s, int i, int j, int k) {
  return 0.5 * (gF(g, s, i, j, k) + gF(g, s, i, j, k + 1));
}

template <class S>
__device__ __forceinline__ void centre(const Geo &g, const Mat &m, const S &s, int i, int j, int k,
                                       Cent &c) {
  const double ir = g.irc[i], is = g.isc[j], ct = g.ctc[j], irs = ir * is;
  const double r0 = gR(g, s, i, j, k), r1 = gR(g, s, i + 1, j, k);
  const double t0 = gT(g, s, i, j, k), t1 = gT(g, s, i, j + 1, k);
  const double f0 = gF(g, s, i, j, k), f1 = gF(g, s, i, j, k + 1);
  c.ur = 0.5 * (r0 + r1);
  c.ut = 0.5 * (t0 + t1);
  c.uf = 0.5 * (f0 + f1);
  c.P = pcoef(g, s, i, j, k) + m.pinf;
  c.T = gC(g, s, F_T, i, j, k);
  c.chi = (m.gam - 1.0) * c.T * rcp_nr(c.P);
  c.Grr = (r1 - r0) * g.idr;
  c.Gtt = (t1 - t0) * (ir * g.idt) + c.ur * ir;
  c.Gff = (f1 - f0) * (irs * g.idp) + c.ur * ir + c.ut * ct * ir;
  c.Srt = (avgT(g, s, i + 1, j, k) - avgT(g, s, i - 1, j, k)) * (0.5 * g.idr) +
          (avgR(g, s, i, j + 1, k) - avgR(g, s, i, j - 1, k)) * (0.5 * ir * g.idt) - c.ut * ir;
  c.Srf = (avgF(g, s, i + 1, j, k) - avgF(g, s, i - 1, j, k)) * (0.5 * g.idr) +
          (avgR(g, s, i, j, k + 1) - avgR(g, s, i, j, k - 1)) * (0.5 * irs * g.idp) - c.uf * ir;
  c.Stf = (avgF(g, s, i, j + 1, k) - avgF(g, s, i, j - 1, k)) * (0.5 * ir * g.idt) +
          (avgT(g, s, i, j, k + 1) - avgT(g, s, i, j, k - 1)) * (0.5 * irs * g.idp) - c.uf * ct * ir;
  c.tr = c.Grr + c.Gtt + c.Gff;
  c.div = (g.rf[i + 1] * g.rf[i + 1] * r1 - g.rf[i] * g.rf[i] * r0) * (ir * ir * g.idr) +
          (g.sf[j + 1] * t1 - g.sf[j] * t0) * (irs * g.idt) + (f1 - f0) * (irs * g.idp);
}

// full compact divergence at a centre (for the grad-div term of the momentum
// equations at the faces between two cells)
template <class S>
__device__ __forceinline__ double divc(const Geo &g, const S &s, int i, int j, int k) {
  const double ir = g.irc[i], irs = ir * g.isc[j];
  return (g.rf[i + 1] * g.rf[i + 1] * gR(g, s, i + 1, j, k) - g.rf[i] * g.rf[i] * gR(g, s, i, j, k)) *
             (ir * ir * g.idr) +
         (g.sf[j + 1] * gT(g, s, i, j + 1, k) - g.sf[j] * gT(g, s, i, j, k)) * (irs * g.idt) +
         (gF(g, s, i, j, k + 1) - gF(g, s, i, j, k)) * (irs * g.idp);
}

} // namespace dsw
