/*
 * dsw_oracle.c -- plain, slow, obviously-correct FP64 CPU reference of one
 * direction-split time step of Frolov, Minev & Takhirov, "An efficient
 * algorithm for weakly compressible flows in spherical geometries"
 * (arXiv 2004.13887).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  The product path (HIP kernels behind
 * the C-ABI) shares no code, header, table or constant with it.
 *
 * What is computed (paper section "Discretization", eqs. (chapter3mainsd),
 * (splitting2) and (spl1)-(spl3); operators of Appendix B):
 *
 *   U^{n+1,0} = U^n (boundary-normal faces take their Dirichlet data at t^{n+1})
 *   for k = 0..K-1:
 *     Ubar = (U^{n+1,k} + U^n)/2
 *     R    = -(U^{n+1,k} - U^n) - tau*(F_h(Ubar) - Sbar)            (a)
 *     (I + tau/2 D_r(Ubar))     X1 = R
 *     (I + tau/2 D_theta(Ubar)) X2 = X1
 *     (I + tau/2 D_phi(Ubar))   X3 = X2
 *     U^{n+1,k+1} = U^{n+1,k} + X3
 *
 * (a) is the right-hand side of (spl1) rearranged: every D(.) is linear in its
 * operand and frozen at Ubar, so -(I + tau/2 D)(U^k - U^n) - tau D U^n - tau G
 * - tau/2 D_M (U^k + U^n) = -(U^k - U^n) - tau [(D + D_M)(Ubar) Ubar + G].
 *
 * The spatial operator is written once, as a form N(u; v) that is linear in the
 * operand v with coefficients taken from u; every term carries the direction
 * tag the paper's Appendix B gives it (r, theta, phi, or the explicit
 * remainder M).  Then F_h(U) = N(U; U) + G, and D_d(Ubar) X = N_d(Ubar; X).
 * The line matrices are obtained by probing N_d with unit operands, so they
 * are I + tau/2 D_d by construction.  Line systems are solved by the block
 * Thomas algorithm without inter-block pivoting (paper, end of section 2); the
 * periodic (cyclic) lines by bordered elimination of the last block.
 *
 * Discrete conventions (the paper says only "standard central differences on
 * the MAC stencil"): compact flux-form divergence at centres; face gradients
 * of centre scalars; centre-averaged velocities for advection of centre
 * scalars and 4-point averages for the transverse advecting velocity at a
 * face; conservative 3-point second differences with metric factors at the
 * half points; face 1/rho from the mean of the two centre densities; velocity
 * gradient at centres with compact diagonal and 4-point-averaged off-diagonal
 * entries; grad-div at a face from the two adjacent centre divergences.
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no contraction, no fast-math).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Scalar type of the state.  The default build is FP64.  Built with
 * -DORC_COMPLEX_STEP the same code runs on complex numbers: evaluated at
 * U + i h V with a tiny h, every output's imaginary part divided by h is its
 * directional derivative along V, exact to rounding (complex-step
 * differentiation; no difference of nearby values is formed).  The tests use
 * it to pin the GPU adjoint.  Geometry and material constants stay FP64. */
#ifdef ORC_COMPLEX_STEP
#include <complex.h>
typedef double _Complex real;
#define RMAG(x) fabs(creal(x))
#else
typedef double real;
#define RMAG(x) fabs(x)
#endif

/* ---------------------------------------------------------------- types -- */

typedef struct { double cp, cv, pi_inf, mu, prandtl, omega, g_r; } orc_mat;
typedef struct { real *p, *ur, *ut, *uf, *T; } orc_fields;

/* Tangential wall velocities used for ghost values (2g - interior).  NULL
 * entries (or a NULL struct) mean g = 0.  Shapes:
 *   ur_t1, ur_t2 : [nr+1][np]    u_r on the theta = theta1 / theta2 walls
 *   ur_p1, ur_p2 : [nr+1][nt]    u_r on the phi walls
 *   ut_r1, ut_r2 : [nt+1][np]    u_theta on the r walls
 *   ut_p1, ut_p2 : [nr][nt+1]    u_theta on the phi walls
 *   uf_r1, uf_r2 : [nt][npf]     u_phi on the r walls
 *   uf_t1, uf_t2 : [nr][npf]     u_phi on the theta walls                     */
typedef struct {
  const real *ur_t1, *ur_t2, *ur_p1, *ur_p2;
  const real *ut_r1, *ut_r2, *ut_p1, *ut_p2;
  const real *uf_r1, *uf_r2, *uf_t1, *uf_t2;
} orc_wall;

typedef struct {
  int nr, nt, np, npf, periodic, pole_lo, pole_hi;
  double r1, r2, t1, t2, p1, p2, dr, dt, dp;
  double *rc, *rf; /* centre radii [nr], face radii [nr+1]                */
  double *sc, *cc; /* sin, cos at theta centres [nt]                       */
  double *sf, *cf; /* sin, cos at theta faces [nt+1] (0 exactly at a pole) */
} orc_grid;

enum { FP = 0, FR = 1, FT = 2, FF = 3, FTT = 4 };
enum { MR = 1, MT = 2, MF = 4, MM = 8, MALL = 15 };

#define IC(g, i, j, k) (((long)(i) * (g)->nt + (j)) * (g)->np + (k))
#define IR(g, f, j, k) (((long)(f) * (g)->nt + (j)) * (g)->np + (k))
#define IT(g, i, f, k) (((long)(i) * ((g)->nt + 1) + (f)) * (g)->np + (k))
#define IF(g, i, j, f) (((long)(i) * (g)->nt + (j)) * (g)->npf + (f))

static long fsize(const orc_grid *g, int fid) {
  switch (fid) {
  case FR: return (long)(g->nr + 1) * g->nt * g->np;
  case FT: return (long)g->nr * (g->nt + 1) * g->np;
  case FF: return (long)g->nr * g->nt * g->npf;
  default: return (long)g->nr * g->nt * g->np;
  }
}

/* ----------------------------------------------------------------- grid -- */

orc_grid *orc_grid_new(int nr, int nt, int np, double r1, double r2, double t1,
                       double t2, double p1, double p2, int periodic) {
  if (nr < 3 || nt < 3 || np < 3) return NULL;
  if (!(r1 > 0.0 && r2 > r1)) return NULL;
  if (!(t1 >= 0.0 && t2 > t1 && t2 <= M_PI + 1e-12)) return NULL;
  if (!(p2 > p1)) return NULL;
  if (periodic && fabs((p2 - p1) - 2.0 * M_PI) > 1e-12) return NULL;
  orc_grid *g = (orc_grid *)calloc(1, sizeof(orc_grid));
  g->nr = nr; g->nt = nt; g->np = np; g->periodic = periodic ? 1 : 0;
  g->npf = periodic ? np : np + 1;
  g->pole_lo = (t1 == 0.0);
  g->pole_hi = (fabs(t2 - M_PI) <= 1e-12);
  g->r1 = r1; g->r2 = r2; g->t1 = t1; g->t2 = t2; g->p1 = p1; g->p2 = p2;
  g->dr = (r2 - r1) / nr; g->dt = (t2 - t1) / nt; g->dp = (p2 - p1) / np;
  g->rc = malloc(sizeof(double) * nr); g->rf = malloc(sizeof(double) * (nr + 1));
  g->sc = malloc(sizeof(double) * nt); g->cc = malloc(sizeof(double) * nt);
  g->sf = malloc(sizeof(double) * (nt + 1)); g->cf = malloc(sizeof(double) * (nt + 1));
  for (int i = 0; i < nr; i++) g->rc[i] = r1 + (i + 0.5) * g->dr;
  for (int f = 0; f <= nr; f++) g->rf[f] = r1 + f * g->dr;
  for (int j = 0; j < nt; j++) {
    double th = t1 + (j + 0.5) * g->dt;
    g->sc[j] = sin(th); g->cc[j] = cos(th);
  }
  for (int f = 0; f <= nt; f++) {
    double th = t1 + f * g->dt;
    g->sf[f] = sin(th); g->cf[f] = cos(th);
  }
  if (g->pole_lo) { g->sf[0] = 0.0; g->cf[0] = 1.0; }
  if (g->pole_hi) { g->sf[nt] = 0.0; g->cf[nt] = -1.0; }
  return g;
}

void orc_grid_free(orc_grid *g) {
  if (!g) return;
  free(g->rc); free(g->rf); free(g->sc); free(g->cc); free(g->sf); free(g->cf);
  free(g);
}

/* ------------------------------------------------- operand + ghost rules -- */

/* An operand is either five arrays (with optional wall data for ghosts) or a
 * single unit entry (used to probe the line matrices; homogeneous ghosts). */
typedef struct {
  const real *a[5];
  const orc_wall *w;
  int ufid;  /* >= 0: unit operand */
  long uidx;
} opnd;

static inline real rd(const opnd *v, int fid, long idx) {
  if (v->ufid >= 0) return (fid == v->ufid && idx == v->uidx) ? 1.0 : 0.0;
  return v->a[fid][idx];
}

#define WV(w, name, idx) (((w) && (w)->name) ? (w)->name[(idx)] : 0.0)

static inline int kwrap(const orc_grid *g, int k) {
  int n = g->np;
  k %= n;
  return k < 0 ? k + n : k;
}
static inline int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* p, T at centres: zero-Neumann (copy) ghosts at every non-periodic boundary. */
static real cval(const orc_grid *g, const opnd *v, int fid, int i, int j, int k) {
  i = clampi(i, 0, g->nr - 1);
  j = clampi(j, 0, g->nt - 1);
  k = g->periodic ? kwrap(g, k) : clampi(k, 0, g->np - 1);
  return rd(v, fid, IC(g, i, j, k));
}

/* u_r at r-face f (0..nr, never a ghost in r).  Tangential to theta and phi
 * boundaries: wall ghost 2g - u; pole ghost +u (symmetry). */
static real urv(const orc_grid *g, const opnd *v, int f, int j, int k) {
  if (k < 0 || k >= g->np) {
    if (g->periodic) k = kwrap(g, k);
    else {
      int kin = k < 0 ? 0 : g->np - 1;
      long gi = (long)f * g->nt + clampi(j, 0, g->nt - 1);
      real gw = k < 0 ? WV(v->w, ur_p1, gi) : WV(v->w, ur_p2, gi);
      return 2.0 * gw - urv(g, v, f, j, kin);
    }
  }
  if (j < 0) {
    real in = rd(v, FR, IR(g, f, 0, k));
    return g->pole_lo ? in : 2.0 * WV(v->w, ur_t1, (long)f * g->np + k) - in;
  }
  if (j >= g->nt) {
    real in = rd(v, FR, IR(g, f, g->nt - 1, k));
    return g->pole_hi ? in : 2.0 * WV(v->w, ur_t2, (long)f * g->np + k) - in;
  }
  return rd(v, FR, IR(g, f, j, k));
}

/* u_theta at theta-face f (0..nt).  Tangential to r and phi boundaries. */
static real utv(const orc_grid *g, const opnd *v, int i, int f, int k) {
  if (k < 0 || k >= g->np) {
    if (g->periodic) k = kwrap(g, k);
    else {
      int kin = k < 0 ? 0 : g->np - 1;
      long gi = (long)clampi(i, 0, g->nr - 1) * (g->nt + 1) + f;
      real gw = k < 0 ? WV(v->w, ut_p1, gi) : WV(v->w, ut_p2, gi);
      return 2.0 * gw - utv(g, v, i, f, kin);
    }
  }
  if (i < 0) return 2.0 * WV(v->w, ut_r1, (long)f * g->np + k) - rd(v, FT, IT(g, 0, f, k));
  if (i >= g->nr)
    return 2.0 * WV(v->w, ut_r2, (long)f * g->np + k) - rd(v, FT, IT(g, g->nr - 1, f, k));
  return rd(v, FT, IT(g, i, f, k));
}

/* u_phi at phi-face f (0..npf-1; wraps when periodic).  Tangential to r and
 * theta boundaries; at a pole the ghost is -u. */
static real ufv(const orc_grid *g, const opnd *v, int i, int j, int f) {
  if (g->periodic) f = kwrap(g, f);
  if (j < 0 || j >= g->nt) {
    int jin = j < 0 ? 0 : g->nt - 1;
    real in = ufv(g, v, i, jin, f);
    if ((j < 0 && g->pole_lo) || (j >= g->nt && g->pole_hi)) return -in;
    long gi = (long)clampi(i, 0, g->nr - 1) * g->npf + f;
    real gw = j < 0 ? WV(v->w, uf_t1, gi) : WV(v->w, uf_t2, gi);
    return 2.0 * gw - in;
  }
  if (i < 0) return 2.0 * WV(v->w, uf_r1, (long)j * g->npf + f) - rd(v, FF, IF(g, 0, j, f));
  if (i >= g->nr)
    return 2.0 * WV(v->w, uf_r2, (long)j * g->npf + f) - rd(v, FF, IF(g, g->nr - 1, j, f));
  return rd(v, FF, IF(g, i, j, f));
}

/* velocity components averaged to the centre of cell (i,j,k) (may be a ghost
 * cell in the directions tangential to the component) */
static real urc(const orc_grid *g, const opnd *v, int i, int j, int k) {
  return 0.5 * (urv(g, v, i, j, k) + urv(g, v, i + 1, j, k));
}
static real utc(const orc_grid *g, const opnd *v, int i, int j, int k) {
  return 0.5 * (utv(g, v, i, j, k) + utv(g, v, i, j + 1, k));
}
static real ufc(const orc_grid *g, const opnd *v, int i, int j, int k) {
  return 0.5 * (ufv(g, v, i, j, k) + ufv(g, v, i, j, k + 1));
}

/* ------------------------------------------------ coefficients (from u) -- */

static real rho_c(const orc_grid *g, const orc_mat *m, const opnd *u, int i, int j, int k) {
  real P = cval(g, u, FP, i, j, k) + m->pi_inf;
  real T = cval(g, u, FTT, i, j, k);
  return P / ((m->cp - m->cv) * T); /* c_v (gamma-1) = c_p - c_v */
}

/* Velocity gradient G = grad u (physical spherical components) at a centre. */
typedef struct {
  real urc, utc, ufc, P, T, chi;
  real Grr, Gtt, Gff, Srt, Srf, Stf, tr;
} ccoef;

static void ccoef_at(const orc_grid *g, const orc_mat *m, const opnd *u, int i, int j, int k,
                     ccoef *c) {
  real r = g->rc[i], s = g->sc[j], ct = g->cc[j] / g->sc[j];
  real gam = m->cp / m->cv;
  real r0 = urv(g, u, i, j, k), r1 = urv(g, u, i + 1, j, k);
  real t0 = utv(g, u, i, j, k), t1 = utv(g, u, i, j + 1, k);
  real f0 = ufv(g, u, i, j, k), f1 = ufv(g, u, i, j, k + 1);
  c->urc = 0.5 * (r0 + r1);
  c->utc = 0.5 * (t0 + t1);
  c->ufc = 0.5 * (f0 + f1);
  c->P = cval(g, u, FP, i, j, k) + m->pi_inf;
  c->T = cval(g, u, FTT, i, j, k);
  c->chi = (gam - 1.0) * c->T / c->P;
  c->Grr = (r1 - r0) / g->dr;
  c->Gtt = (t1 - t0) / (r * g->dt) + c->urc / r;
  c->Gff = (f1 - f0) / (r * s * g->dp) + c->urc / r + c->utc * ct / r;
  c->Srt = (utc(g, u, i + 1, j, k) - utc(g, u, i - 1, j, k)) / (2.0 * g->dr) +
           (urc(g, u, i, j + 1, k) - urc(g, u, i, j - 1, k)) / (2.0 * r * g->dt) - c->utc / r;
  c->Srf = (ufc(g, u, i + 1, j, k) - ufc(g, u, i - 1, j, k)) / (2.0 * g->dr) +
           (urc(g, u, i, j, k + 1) - urc(g, u, i, j, k - 1)) / (2.0 * r * s * g->dp) - c->ufc / r;
  c->Stf = (ufc(g, u, i, j + 1, k) - ufc(g, u, i, j - 1, k)) / (2.0 * r * g->dt) +
           (utc(g, u, i, j, k + 1) - utc(g, u, i, j, k - 1)) / (2.0 * r * s * g->dp) -
           c->ufc * ct / r;
  c->tr = c->Grr + c->Gtt + c->Gff;
}

/* The operand's G(v) and div(v) at a centre, keeping only the parts whose
 * direction tag is in mask (paper Appendix B, operators A2, C2: the v_r terms
 * belong to r, the theta-derivative and v_theta terms to theta, ...). */
typedef struct { real Grr, Gtt, Gff, Srt, Srf, Stf, div; } cgrad;

static void cgrad_at(const orc_grid *g, const opnd *v, int i, int j, int k, int mask, cgrad *q) {
  real r = g->rc[i], s = g->sc[j], ct = g->cc[j] / g->sc[j];
  real r0 = urv(g, v, i, j, k), r1 = urv(g, v, i + 1, j, k);
  real t0 = utv(g, v, i, j, k), t1 = utv(g, v, i, j + 1, k);
  real f0 = ufv(g, v, i, j, k), f1 = ufv(g, v, i, j, k + 1);
  real vrc = 0.5 * (r0 + r1), vtc = 0.5 * (t0 + t1), vfc = 0.5 * (f0 + f1);
  memset(q, 0, sizeof(*q));
  if (mask & MR) {
    q->Grr = (r1 - r0) / g->dr;
    q->Gtt += vrc / r;
    q->Gff += vrc / r;
    q->div += (g->rf[i + 1] * g->rf[i + 1] * r1 - g->rf[i] * g->rf[i] * r0) / (r * r * g->dr);
  }
  if (mask & MT) {
    q->Gtt += (t1 - t0) / (r * g->dt);
    q->Gff += vtc * ct / r;
    q->Srt += -vtc / r;
    q->div += (g->sf[j + 1] * t1 - g->sf[j] * t0) / (r * s * g->dt);
  }
  if (mask & MF) {
    q->Gff += (f1 - f0) / (r * s * g->dp);
    q->Srf += -vfc / r;
    q->Stf += -vfc * ct / r;
    q->div += (f1 - f0) / (r * s * g->dp);
  }
  if (mask & MM) {
    q->Srt += (utc(g, v, i + 1, j, k) - utc(g, v, i - 1, j, k)) / (2.0 * g->dr) +
              (urc(g, v, i, j + 1, k) - urc(g, v, i, j - 1, k)) / (2.0 * r * g->dt);
    q->Srf += (ufc(g, v, i + 1, j, k) - ufc(g, v, i - 1, j, k)) / (2.0 * g->dr) +
              (urc(g, v, i, j, k + 1) - urc(g, v, i, j, k - 1)) / (2.0 * r * s * g->dp);
    q->Stf += (ufc(g, v, i, j + 1, k) - ufc(g, v, i, j - 1, k)) / (2.0 * r * g->dt) +
              (utc(g, v, i, j, k + 1) - utc(g, v, i, j, k - 1)) / (2.0 * r * s * g->dp);
  }
}

/* viscous dissipation grad(u) : sigma(v), bilinear, discrete */
static real phi_h(const orc_mat *m, const ccoef *c, const cgrad *q) {
  return m->mu * (2.0 * (c->Grr * q->Grr + c->Gtt * q->Gtt + c->Gff * q->Gff) + c->Srt * q->Srt +
                  c->Srf * q->Srf + c->Stf * q->Stf - (2.0 / 3.0) * c->tr * q->div);
}

/* u . grad f for a centre scalar, central differences over two cells */
static real cadv(const orc_grid *g, const opnd *v, int fid, const ccoef *c, int i, int j,
                   int k, int mask) {
  real r = g->rc[i], s = g->sc[j], a = 0.0;
  if (mask & MR)
    a += c->urc * (cval(g, v, fid, i + 1, j, k) - cval(g, v, fid, i - 1, j, k)) / (2.0 * g->dr);
  if (mask & MT)
    a += c->utc / r * (cval(g, v, fid, i, j + 1, k) - cval(g, v, fid, i, j - 1, k)) / (2.0 * g->dt);
  if (mask & MF)
    a += c->ufc / (r * s) * (cval(g, v, fid, i, j, k + 1) - cval(g, v, fid, i, j, k - 1)) /
         (2.0 * g->dp);
  return a;
}

/* conservative scalar Laplacian of a centre field (zero-flux through walls) */
static real clap(const orc_grid *g, const opnd *v, int fid, int i, int j, int k, int mask) {
  real r = g->rc[i], s = g->sc[j], f0 = cval(g, v, fid, i, j, k), L = 0.0;
  if (mask & MR)
    L += (g->rf[i + 1] * g->rf[i + 1] * (cval(g, v, fid, i + 1, j, k) - f0) -
          g->rf[i] * g->rf[i] * (f0 - cval(g, v, fid, i - 1, j, k))) /
         (r * r * g->dr * g->dr);
  if (mask & MT)
    L += (g->sf[j + 1] * (cval(g, v, fid, i, j + 1, k) - f0) -
          g->sf[j] * (f0 - cval(g, v, fid, i, j - 1, k))) /
         (r * r * s * g->dt * g->dt);
  if (mask & MF)
    L += (cval(g, v, fid, i, j, k + 1) - 2.0 * f0 + cval(g, v, fid, i, j, k - 1)) /
         (r * r * s * s * g->dp * g->dp);
  return L;
}

/* divergence of v at centre (i,j,k), split by direction */
static void cdiv(const orc_grid *g, const opnd *v, int i, int j, int k, real *dr_, real *dt_,
                 real *dp_) {
  real r = g->rc[i], s = g->sc[j];
  *dr_ = (g->rf[i + 1] * g->rf[i + 1] * urv(g, v, i + 1, j, k) -
          g->rf[i] * g->rf[i] * urv(g, v, i, j, k)) / (r * r * g->dr);
  *dt_ = (g->sf[j + 1] * utv(g, v, i, j + 1, k) - g->sf[j] * utv(g, v, i, j, k)) /
         (r * s * g->dt);
  *dp_ = (ufv(g, v, i, j, k + 1) - ufv(g, v, i, j, k)) / (r * s * g->dp);
}


/* ------------------------------------------------------- viscous vector -- */

/* The viscous term of F_h, -(1/rho) div sigma = -(mu/rho) (Lap u + grad div u / 3)
 * (eq. (nonconservmom), constant mu), is discretised as
 *     -(mu/rho) V(u),   V(u) = (4/3) grad_h(div_h u) - curl_h(curl_h u),
 * the vector-Laplacian identity Lap u = grad div u - curl curl u on the MAC
 * complex: div_h at cell centres (cdiv), the vorticity curl_h u at cell edges
 * as the circulation round a dual face over its area, and curl_h of an edge
 * field at a face as its circulation round the face over the face area (the
 * same face areas as div_h).  Then div_h(curl_h(.)) = 0 exactly, so the
 * viscous update of a discretely solenoidal velocity stays solenoidal; the
 * component form (scalar Laplacians plus curvature terms) does not do this in
 * spherical coordinates.  The implicit operators D_d keep the paper's
 * per-direction second derivatives (B2^{d,.} of Appendix B); the explicit
 * remainder D_M takes V minus their sum, a discretisation of the paper's
 * curvature and mixed terms (B2^{M,.}).  Ghost cells take their own radius
 * and colatitude. */
static double rc_any(const orc_grid *g, int i) { return g->r1 + (i + 0.5) * g->dr; }
static double sc_any(const orc_grid *g, int j) { return sin(g->t1 + (j + 0.5) * g->dt); }

static real div_at(const orc_grid *g, const opnd *v, int i, int j, int k) {
  real a, b, c;
  cdiv(g, v, i, j, k, &a, &b, &c);
  return a + b + c;
}
/* omega_phi at the edge (r face fr, theta face ft, phi centre k) */
static real om_phi(const orc_grid *g, const opnd *v, int fr, int ft, int k) {
  return (rc_any(g, fr) * utv(g, v, fr, ft, k) - rc_any(g, fr - 1) * utv(g, v, fr - 1, ft, k)) /
             (g->rf[fr] * g->dr) -
         (urv(g, v, fr, ft, k) - urv(g, v, fr, ft - 1, k)) / (g->rf[fr] * g->dt);
}
/* omega_theta at the edge (r face fr, theta centre j, phi face fk) */
static real om_theta(const orc_grid *g, const opnd *v, int fr, int j, int fk) {
  return (urv(g, v, fr, j, fk) - urv(g, v, fr, j, fk - 1)) / (g->rf[fr] * g->sc[j] * g->dp) -
         (rc_any(g, fr) * ufv(g, v, fr, j, fk) - rc_any(g, fr - 1) * ufv(g, v, fr - 1, j, fk)) /
             (g->rf[fr] * g->dr);
}
/* omega_r at the edge (r centre i, theta face ft off a pole, phi face fk) */
static real om_r(const orc_grid *g, const opnd *v, int i, int ft, int fk) {
  return (sc_any(g, ft) * ufv(g, v, i, ft, fk) - sc_any(g, ft - 1) * ufv(g, v, i, ft - 1, fk)) /
             (g->rc[i] * g->sf[ft] * g->dt) -
         (utv(g, v, i, ft, fk) - utv(g, v, i, ft, fk - 1)) / (g->rc[i] * g->sf[ft] * g->dp);
}
/* V at the r face (f, j, k) */
static real visc_r(const orc_grid *g, const opnd *v, int f, int j, int k) {
  real cc = ((g->sf[j + 1] * om_phi(g, v, f, j + 1, k) - g->sf[j] * om_phi(g, v, f, j, k)) / g->dt -
             (om_theta(g, v, f, j, k + 1) - om_theta(g, v, f, j, k)) / g->dp) /
            (g->rf[f] * g->sc[j]);
  return (4.0 / 3.0) * (div_at(g, v, f, j, k) - div_at(g, v, f - 1, j, k)) / g->dr - cc;
}
/* V at the theta face (i, f, k) */
static real visc_t(const orc_grid *g, const opnd *v, int i, int f, int k) {
  real cc = (om_r(g, v, i, f, k + 1) - om_r(g, v, i, f, k)) / (g->rc[i] * g->sf[f] * g->dp) -
            (g->rf[i + 1] * om_phi(g, v, i + 1, f, k) - g->rf[i] * om_phi(g, v, i, f, k)) /
                (g->rc[i] * g->dr);
  return (4.0 / 3.0) * (div_at(g, v, i, f, k) - div_at(g, v, i, f - 1, k)) / (g->rc[i] * g->dt) - cc;
}
/* V at the phi face (i, j, f), j not next to a pole */
static real visc_f(const orc_grid *g, const opnd *v, int i, int j, int f) {
  int k0 = g->periodic ? kwrap(g, f - 1) : f - 1, k1 = g->periodic ? kwrap(g, f) : f;
  real cc = (g->rf[i + 1] * om_theta(g, v, i + 1, j, f) - g->rf[i] * om_theta(g, v, i, j, f)) /
                (g->rc[i] * g->dr) -
            (om_r(g, v, i, j + 1, f) - om_r(g, v, i, j, f)) / (g->rc[i] * g->dt);
  return (4.0 / 3.0) * (div_at(g, v, i, j, k1) - div_at(g, v, i, j, k0)) /
             (g->rc[i] * g->sc[j] * g->dp) -
         cc;
}
/* The per-direction viscous parts of the implicit operators (Appendix B,
 * B2^{r,r} + B2^{theta,r} + B2^{phi,r} and their theta and phi counterparts:
 * the three second differences of the face's own component plus the
 * grad-div part along the face's own direction), summed over all three
 * directions, in the units of V. */
static real visc_dir_r(const orc_grid *g, const opnd *v, int f, int j, int k) {
  real rF = g->rf[f], s = g->sc[j], x0 = urv(g, v, f, j, k), a0, b0, c0, a1, b1, c1;
  cdiv(g, v, f - 1, j, k, &a0, &b0, &c0);
  cdiv(g, v, f, j, k, &a1, &b1, &c1);
  return (g->rc[f] * g->rc[f] * (urv(g, v, f + 1, j, k) - x0) -
          g->rc[f - 1] * g->rc[f - 1] * (x0 - urv(g, v, f - 1, j, k))) / (rF * rF * g->dr * g->dr) +
         (a1 - a0) / (3.0 * g->dr) +
         (g->sf[j + 1] * (urv(g, v, f, j + 1, k) - x0) - g->sf[j] * (x0 - urv(g, v, f, j - 1, k))) /
             (rF * rF * s * g->dt * g->dt) +
         (urv(g, v, f, j, k + 1) - 2.0 * x0 + urv(g, v, f, j, k - 1)) / (rF * rF * s * s * g->dp * g->dp);
}
static real visc_dir_t(const orc_grid *g, const opnd *v, int i, int f, int k) {
  real r = g->rc[i], s = g->sf[f], x0 = utv(g, v, i, f, k), a0, b0, c0, a1, b1, c1;
  cdiv(g, v, i, f - 1, k, &a0, &b0, &c0);
  cdiv(g, v, i, f, k, &a1, &b1, &c1);
  return (g->sc[f] * (utv(g, v, i, f + 1, k) - x0) - g->sc[f - 1] * (x0 - utv(g, v, i, f - 1, k))) /
             (r * r * s * g->dt * g->dt) +
         (b1 - b0) / (3.0 * r * g->dt) +
         (g->rf[i + 1] * g->rf[i + 1] * (utv(g, v, i + 1, f, k) - x0) -
          g->rf[i] * g->rf[i] * (x0 - utv(g, v, i - 1, f, k))) / (r * r * g->dr * g->dr) +
         (utv(g, v, i, f, k + 1) - 2.0 * x0 + utv(g, v, i, f, k - 1)) / (r * r * s * s * g->dp * g->dp);
}
static real visc_dir_f(const orc_grid *g, const opnd *v, int i, int j, int f) {
  real r = g->rc[i], s = g->sc[j], x0 = ufv(g, v, i, j, f), a0, b0, c0, a1, b1, c1;
  int k0 = g->periodic ? kwrap(g, f - 1) : f - 1, k1 = g->periodic ? kwrap(g, f) : f;
  cdiv(g, v, i, j, k0, &a0, &b0, &c0);
  cdiv(g, v, i, j, k1, &a1, &b1, &c1);
  return (ufv(g, v, i, j, f + 1) - 2.0 * x0 + ufv(g, v, i, j, f - 1)) / (r * r * s * s * g->dp * g->dp) +
         (c1 - c0) / (3.0 * r * s * g->dp) +
         (g->rf[i + 1] * g->rf[i + 1] * (ufv(g, v, i + 1, j, f) - x0) -
          g->rf[i] * g->rf[i] * (x0 - ufv(g, v, i - 1, j, f))) / (r * r * g->dr * g->dr) +
         (g->sf[j + 1] * (ufv(g, v, i, j + 1, f) - x0) - g->sf[j] * (x0 - ufv(g, v, i, j - 1, f))) /
             (r * r * s * g->dt * g->dt);
}
/* a phi-face row next to a pole: the edge vorticity omega_r on the polar axis
 * is one value for the whole ring of phi faces, so these rows keep the
 * component form of the vector Laplacian with the pole ghost rules */
static int next_to_pole(const orc_grid *g, int j) {
  return (j == 0 && g->pole_lo) || (j == g->nt - 1 && g->pole_hi);
}

/* ------------------------------------------------------------- row forms -- */

/* pressure equation (nonconservener) at a centre */
static real row_p(const orc_grid *g, const orc_mat *m, const ccoef *c, const opnd *v, int i,
                    int j, int k, int mask) {
  real gam = m->cp / m->cv, kap = m->mu * m->cp / m->prandtl;
  cgrad q;
  cgrad_at(g, v, i, j, k, mask, &q);
  return cadv(g, v, FP, c, i, j, k, mask) + gam * c->P * q.div - (gam - 1.0) * phi_h(m, c, &q) -
         (gam - 1.0) * kap * clap(g, v, FTT, i, j, k, mask);
}

/* temperature equation (nonconservmass) at a centre */
static real row_T(const orc_grid *g, const orc_mat *m, const ccoef *c, const opnd *v, int i,
                    int j, int k, int mask) {
  real gam = m->cp / m->cv, kap = m->mu * m->cp / m->prandtl;
  cgrad q;
  cgrad_at(g, v, i, j, k, mask, &q);
  return cadv(g, v, FTT, c, i, j, k, mask) + (gam - 1.0) * c->T * q.div - c->chi * phi_h(m, c, &q) -
         c->chi * kap * clap(g, v, FTT, i, j, k, mask);
}

/* coefficients at a face: density (mean of the two cells), the normal
 * velocity on the face and the two transverse components interpolated to it */
typedef struct { real rho, un, ua, ub; } fcoef;

static void fcoef_r(const orc_grid *g, const orc_mat *m, const opnd *u, int f, int j, int k,
                    fcoef *c) {
  c->rho = 0.5 * (rho_c(g, m, u, f - 1, j, k) + rho_c(g, m, u, f, j, k));
  c->un = urv(g, u, f, j, k);
  c->ua = 0.25 * (utv(g, u, f - 1, j, k) + utv(g, u, f - 1, j + 1, k) + utv(g, u, f, j, k) +
                  utv(g, u, f, j + 1, k));
  c->ub = 0.25 * (ufv(g, u, f - 1, j, k) + ufv(g, u, f - 1, j, k + 1) + ufv(g, u, f, j, k) +
                  ufv(g, u, f, j, k + 1));
}
static void fcoef_t(const orc_grid *g, const orc_mat *m, const opnd *u, int i, int f, int k,
                    fcoef *c) {
  c->rho = 0.5 * (rho_c(g, m, u, i, f - 1, k) + rho_c(g, m, u, i, f, k));
  c->un = utv(g, u, i, f, k);
  c->ua = 0.25 * (urv(g, u, i, f - 1, k) + urv(g, u, i, f, k) + urv(g, u, i + 1, f - 1, k) +
                  urv(g, u, i + 1, f, k));
  c->ub = 0.25 * (ufv(g, u, i, f - 1, k) + ufv(g, u, i, f - 1, k + 1) + ufv(g, u, i, f, k) +
                  ufv(g, u, i, f, k + 1));
}
static void fcoef_f(const orc_grid *g, const orc_mat *m, const opnd *u, int i, int j, int f,
                    fcoef *c) {
  int k0 = g->periodic ? kwrap(g, f - 1) : f - 1, k1 = g->periodic ? kwrap(g, f) : f;
  c->rho = 0.5 * (rho_c(g, m, u, i, j, k0) + rho_c(g, m, u, i, j, k1));
  c->un = ufv(g, u, i, j, f);
  c->ua = 0.25 * (urv(g, u, i, j, k0) + urv(g, u, i, j, k1) + urv(g, u, i + 1, j, k0) +
                  urv(g, u, i + 1, j, k1));
  c->ub = 0.25 * (utv(g, u, i, j, k0) + utv(g, u, i, j, k1) + utv(g, u, i, j + 1, k0) +
                  utv(g, u, i, j + 1, k1));
}

/* radial momentum (nonconservmom, r component) at interior r-face (f,j,k) */
static real row_ur(const orc_grid *g, const orc_mat *m, const fcoef *c, const opnd *v, int f,
                     int j, int k, int mask) {
  real rF = g->rf[f], s = g->sc[j], nu = m->mu / c->rho, N = 0.0, vis = 0.0, gd = 0.0;
  real x0 = urv(g, v, f, j, k);
  if (mask & MR) {
    N += (cval(g, v, FP, f, j, k) - cval(g, v, FP, f - 1, j, k)) / (c->rho * g->dr);
    N += c->un * (urv(g, v, f + 1, j, k) - urv(g, v, f - 1, j, k)) / (2.0 * g->dr);
    vis += (g->rc[f] * g->rc[f] * (urv(g, v, f + 1, j, k) - x0) -
            g->rc[f - 1] * g->rc[f - 1] * (x0 - urv(g, v, f - 1, j, k))) /
           (rF * rF * g->dr * g->dr);
    real a0, b0, c0, a1, b1, c1;
    cdiv(g, v, f - 1, j, k, &a0, &b0, &c0);
    cdiv(g, v, f, j, k, &a1, &b1, &c1);
    gd += (a1 - a0) / g->dr;
  }
  if (mask & MT) {
    N += c->ua / rF * (urv(g, v, f, j + 1, k) - urv(g, v, f, j - 1, k)) / (2.0 * g->dt);
    vis += (g->sf[j + 1] * (urv(g, v, f, j + 1, k) - x0) - g->sf[j] * (x0 - urv(g, v, f, j - 1, k))) /
           (rF * rF * s * g->dt * g->dt);
  }
  if (mask & MF) {
    N += c->ub / (rF * s) * (urv(g, v, f, j, k + 1) - urv(g, v, f, j, k - 1)) / (2.0 * g->dp);
    vis += (urv(g, v, f, j, k + 1) - 2.0 * x0 + urv(g, v, f, j, k - 1)) / (rF * rF * s * s * g->dp * g->dp);
  }
  if (mask & MM) {
    real va = 0.25 * (utv(g, v, f - 1, j, k) + utv(g, v, f - 1, j + 1, k) + utv(g, v, f, j, k) +
                        utv(g, v, f, j + 1, k));
    real vb = 0.25 * (ufv(g, v, f - 1, j, k) + ufv(g, v, f - 1, j, k + 1) + ufv(g, v, f, j, k) +
                        ufv(g, v, f, j, k + 1));
    N += -(c->ua * va + c->ub * vb) / rF;
    vis += visc_r(g, v, f, j, k) - visc_dir_r(g, v, f, j, k);
    N += -2.0 * m->omega * s * vb;
  }
  return N - nu * vis - nu / 3.0 * gd;
}

/* colatitudinal momentum at interior theta-face (i,f,k) */
static real row_ut(const orc_grid *g, const orc_mat *m, const fcoef *c, const opnd *v, int i,
                     int f, int k, int mask) {
  real r = g->rc[i], s = g->sf[f], ctF = g->cf[f] / g->sf[f];
  real nu = m->mu / c->rho, N = 0.0, vis = 0.0, gd = 0.0;
  int j0 = f - 1, j1 = f;
  real x0 = utv(g, v, i, f, k);
  if (mask & MT) {
    N += (cval(g, v, FP, i, j1, k) - cval(g, v, FP, i, j0, k)) / (c->rho * r * g->dt);
    N += c->un / r * (utv(g, v, i, f + 1, k) - utv(g, v, i, f - 1, k)) / (2.0 * g->dt);
    vis += (g->sc[j1] * (utv(g, v, i, f + 1, k) - x0) - g->sc[j0] * (x0 - utv(g, v, i, f - 1, k))) /
           (r * r * s * g->dt * g->dt);
    real a0, b0, c0, a1, b1, c1;
    cdiv(g, v, i, j0, k, &a0, &b0, &c0);
    cdiv(g, v, i, j1, k, &a1, &b1, &c1);
    gd += (b1 - b0) / (r * g->dt);
  }
  if (mask & MR) {
    N += c->ua * (utv(g, v, i + 1, f, k) - utv(g, v, i - 1, f, k)) / (2.0 * g->dr);
    vis += (g->rf[i + 1] * g->rf[i + 1] * (utv(g, v, i + 1, f, k) - x0) -
            g->rf[i] * g->rf[i] * (x0 - utv(g, v, i - 1, f, k))) /
           (r * r * g->dr * g->dr);
  }
  if (mask & MF) {
    N += c->ub / (r * s) * (utv(g, v, i, f, k + 1) - utv(g, v, i, f, k - 1)) / (2.0 * g->dp);
    vis += (utv(g, v, i, f, k + 1) - 2.0 * x0 + utv(g, v, i, f, k - 1)) / (r * r * s * s * g->dp * g->dp);
  }
  if (mask & MM) {
    real va = 0.25 * (urv(g, v, i, j0, k) + urv(g, v, i, j1, k) + urv(g, v, i + 1, j0, k) +
                        urv(g, v, i + 1, j1, k));
    real vb = 0.25 * (ufv(g, v, i, j0, k) + ufv(g, v, i, j0, k + 1) + ufv(g, v, i, j1, k) +
                        ufv(g, v, i, j1, k + 1));
    N += (c->un * va - c->ub * vb * ctF) / r;
    vis += visc_t(g, v, i, f, k) - visc_dir_t(g, v, i, f, k);
    N += -2.0 * m->omega * g->cf[f] * vb;
  }
  return N - nu * vis - nu / 3.0 * gd;
}

/* azimuthal momentum at interior phi-face (i,j,f) */
static real row_uf(const orc_grid *g, const orc_mat *m, const fcoef *c, const opnd *v, int i,
                     int j, int f, int mask) {
  real r = g->rc[i], s = g->sc[j], ct = g->cc[j] / g->sc[j];
  real nu = m->mu / c->rho, N = 0.0, vis = 0.0, gd = 0.0;
  int k0 = g->periodic ? kwrap(g, f - 1) : f - 1, k1 = g->periodic ? kwrap(g, f) : f;
  real x0 = ufv(g, v, i, j, f);
  if (mask & MF) {
    N += (cval(g, v, FP, i, j, k1) - cval(g, v, FP, i, j, k0)) / (c->rho * r * s * g->dp);
    N += c->un / (r * s) * (ufv(g, v, i, j, f + 1) - ufv(g, v, i, j, f - 1)) / (2.0 * g->dp);
    vis += (ufv(g, v, i, j, f + 1) - 2.0 * x0 + ufv(g, v, i, j, f - 1)) / (r * r * s * s * g->dp * g->dp);
    real a0, b0, c0, a1, b1, c1;
    cdiv(g, v, i, j, k0, &a0, &b0, &c0);
    cdiv(g, v, i, j, k1, &a1, &b1, &c1);
    gd += (c1 - c0) / (r * s * g->dp);
  }
  if (mask & MR) {
    N += c->ua * (ufv(g, v, i + 1, j, f) - ufv(g, v, i - 1, j, f)) / (2.0 * g->dr);
    vis += (g->rf[i + 1] * g->rf[i + 1] * (ufv(g, v, i + 1, j, f) - x0) -
            g->rf[i] * g->rf[i] * (x0 - ufv(g, v, i - 1, j, f))) /
           (r * r * g->dr * g->dr);
  }
  if (mask & MT) {
    N += c->ub / r * (ufv(g, v, i, j + 1, f) - ufv(g, v, i, j - 1, f)) / (2.0 * g->dt);
    vis += (g->sf[j + 1] * (ufv(g, v, i, j + 1, f) - x0) - g->sf[j] * (x0 - ufv(g, v, i, j - 1, f))) /
           (r * r * s * g->dt * g->dt);
  }
  if (mask & MM) {
    real va = 0.25 * (urv(g, v, i, j, k0) + urv(g, v, i, j, k1) + urv(g, v, i + 1, j, k0) +
                        urv(g, v, i + 1, j, k1));
    real vb = 0.25 * (utv(g, v, i, j, k0) + utv(g, v, i, j, k1) + utv(g, v, i, j + 1, k0) +
                        utv(g, v, i, j + 1, k1));
    N += c->un * (va + vb * ct) / r;
    real dphr = 0.5 *
                  ((urv(g, v, i, j, k1) - urv(g, v, i, j, k0)) +
                   (urv(g, v, i + 1, j, k1) - urv(g, v, i + 1, j, k0))) / g->dp;
    real dpht = 0.5 *
                  ((utv(g, v, i, j, k1) - utv(g, v, i, j, k0)) +
                   (utv(g, v, i, j + 1, k1) - utv(g, v, i, j + 1, k0))) / g->dp;
    if (next_to_pole(g, j)) { /* component form: curvature terms and the mixed grad-div */
      vis += -x0 / (r * r * s * s) + 2.0 / (r * r * s) * dphr + 2.0 * ct / (r * r * s) * dpht;
      real a0, b0, c0, a1, b1, c1;
      cdiv(g, v, i, j, k0, &a0, &b0, &c0);
      cdiv(g, v, i, j, k1, &a1, &b1, &c1);
      gd += (a1 - a0) / (r * s * g->dp) + (b1 - b0) / (r * s * g->dp);
    } else {
      vis += visc_f(g, v, i, j, f) - visc_dir_f(g, v, i, j, f);
    }
    N += 2.0 * m->omega * (g->cc[j] * vb + s * va);
  }
  return N - nu * vis - nu / 3.0 * gd;
}

/* first/last interior face index along a velocity component's own direction */
static int uf_lo(const orc_grid *g) { return g->periodic ? 0 : 1; }
static int uf_hi(const orc_grid *g) { return g->periodic ? g->np - 1 : g->np - 1; }

/* ------------------------------------------------------- operator apply -- */

static opnd mk_opnd(const orc_fields *x, const orc_wall *w) {
  opnd o;
  o.a[FP] = x->p; o.a[FR] = x->ur; o.a[FT] = x->ut; o.a[FF] = x->uf; o.a[FTT] = x->T;
  o.w = w; o.ufid = -1; o.uidx = -1;
  return o;
}

static void zero_fields(const orc_grid *g, orc_fields *x) {
  memset(x->p, 0, sizeof(real) * fsize(g, FP));
  memset(x->ur, 0, sizeof(real) * fsize(g, FR));
  memset(x->ut, 0, sizeof(real) * fsize(g, FT));
  memset(x->uf, 0, sizeof(real) * fsize(g, FF));
  memset(x->T, 0, sizeof(real) * fsize(g, FTT));
}

/* out = N(u; v) restricted to the terms in mask, at every unknown; boundary
 * normal faces (Dirichlet, not unknowns) get 0. */
int orc_apply(const orc_grid *g, const orc_mat *m, const orc_fields *uf_, const orc_wall *wu,
              const orc_fields *vf_, const orc_wall *wv, int mask, orc_fields *out) {
  opnd u = mk_opnd(uf_, wu), v = mk_opnd(vf_, wv);
  zero_fields(g, out);
#pragma omp parallel for collapse(2) schedule(static)
  for (int i = 0; i < g->nr; i++)
    for (int j = 0; j < g->nt; j++)
      for (int k = 0; k < g->np; k++) {
        ccoef c;
        ccoef_at(g, m, &u, i, j, k, &c);
        out->p[IC(g, i, j, k)] = row_p(g, m, &c, &v, i, j, k, mask);
        out->T[IC(g, i, j, k)] = row_T(g, m, &c, &v, i, j, k, mask);
      }
#pragma omp parallel for collapse(2) schedule(static)
  for (int f = 1; f < g->nr; f++)
    for (int j = 0; j < g->nt; j++)
      for (int k = 0; k < g->np; k++) {
        fcoef c;
        fcoef_r(g, m, &u, f, j, k, &c);
        out->ur[IR(g, f, j, k)] = row_ur(g, m, &c, &v, f, j, k, mask);
      }
#pragma omp parallel for collapse(2) schedule(static)
  for (int i = 0; i < g->nr; i++)
    for (int f = 1; f < g->nt; f++)
      for (int k = 0; k < g->np; k++) {
        fcoef c;
        fcoef_t(g, m, &u, i, f, k, &c);
        out->ut[IT(g, i, f, k)] = row_ut(g, m, &c, &v, i, f, k, mask);
      }
#pragma omp parallel for collapse(2) schedule(static)
  for (int i = 0; i < g->nr; i++)
    for (int j = 0; j < g->nt; j++)
      for (int f = uf_lo(g); f <= uf_hi(g); f++) {
        fcoef c;
        fcoef_f(g, m, &u, i, j, f, &c);
        out->uf[IF(g, i, j, f)] = row_uf(g, m, &c, &v, i, j, f, mask);
      }
  return 0;
}

/* ------------------------------------------------------------- residual -- */

/* R = -(Uk - Un) - tau*(N(Ubar;Ubar) + G - S) at every unknown (0 on boundary
 * normal faces), Ubar = (Uk + Un)/2 everywhere.  wall: ghost data for Ubar.
 * src may be NULL. */
int orc_residual(const orc_grid *g, const orc_mat *m, const orc_fields *Un, const orc_fields *Uk,
                 const orc_wall *wall, const orc_fields *src, double tau, orc_fields *R,
                 orc_fields *Ub) {
  real *un[5] = {Un->p, Un->ur, Un->ut, Un->uf, Un->T};
  real *uk[5] = {Uk->p, Uk->ur, Uk->ut, Uk->uf, Uk->T};
  real *ub[5] = {Ub->p, Ub->ur, Ub->ut, Ub->uf, Ub->T};
  real *rr[5] = {R->p, R->ur, R->ut, R->uf, R->T};
  for (int q = 0; q < 5; q++) {
    long n = fsize(g, q);
    for (long x = 0; x < n; x++) ub[q][x] = 0.5 * (uk[q][x] + un[q][x]);
  }
  orc_fields F;
  F.p = malloc(sizeof(real) * fsize(g, FP)); F.ur = malloc(sizeof(real) * fsize(g, FR));
  F.ut = malloc(sizeof(real) * fsize(g, FT)); F.uf = malloc(sizeof(real) * fsize(g, FF));
  F.T = malloc(sizeof(real) * fsize(g, FTT));
  orc_apply(g, m, Ub, wall, Ub, wall, MALL, &F);
  real *ff[5] = {F.p, F.ur, F.ut, F.uf, F.T};
  const real *ss[5] = {0, 0, 0, 0, 0};
  if (src) { ss[0] = src->p; ss[1] = src->ur; ss[2] = src->ut; ss[3] = src->uf; ss[4] = src->T; }
  for (int q = 0; q < 5; q++) {
    long n = fsize(g, q);
    for (long x = 0; x < n; x++) rr[q][x] = 0.0;
  }
  /* unknowns only */
  for (int i = 0; i < g->nr; i++)
    for (int j = 0; j < g->nt; j++)
      for (int k = 0; k < g->np; k++) {
        long x = IC(g, i, j, k);
        for (int q = 0; q < 5; q += 4) {
          real fx = ff[q][x] - (ss[q] ? ss[q][x] : 0.0);
          rr[q][x] = -(uk[q][x] - un[q][x]) - tau * fx;
        }
      }
  for (int f = 1; f < g->nr; f++)
    for (int j = 0; j < g->nt; j++)
      for (int k = 0; k < g->np; k++) {
        long x = IR(g, f, j, k);
        real fx = ff[FR][x] + m->g_r - (ss[FR] ? ss[FR][x] : 0.0);
        rr[FR][x] = -(uk[FR][x] - un[FR][x]) - tau * fx;
      }
  for (int i = 0; i < g->nr; i++)
    for (int f = 1; f < g->nt; f++)
      for (int k = 0; k < g->np; k++) {
        long x = IT(g, i, f, k);
        real fx = ff[FT][x] - (ss[FT] ? ss[FT][x] : 0.0);
        rr[FT][x] = -(uk[FT][x] - un[FT][x]) - tau * fx;
      }
  for (int i = 0; i < g->nr; i++)
    for (int j = 0; j < g->nt; j++)
      for (int f = uf_lo(g); f <= uf_hi(g); f++) {
        long x = IF(g, i, j, f);
        real fx = ff[FF][x] - (ss[FF] ? ss[FF][x] : 0.0);
        rr[FF][x] = -(uk[FF][x] - un[FF][x]) - tau * fx;
      }
  free(F.p); free(F.ur); free(F.ut); free(F.uf); free(F.T);
  return 0;
}

/* ------------------------------------------------------- small dense LU -- */

/* Solve A X = B, A bs x bs, B bs x nc (row-major), Gaussian elimination with
 * partial pivoting.  Result overwrites B.  Returns -1 on a zero pivot. */
static int small_solve(int bs, real *A, int nc, real *B) {
  for (int c = 0; c < bs; c++) {
    int piv = c;
    for (int r = c + 1; r < bs; r++)
      if (RMAG(A[r * bs + c]) > RMAG(A[piv * bs + c])) piv = r;
    if (A[piv * bs + c] == 0.0) return -1;
    if (piv != c) {
      for (int q = 0; q < bs; q++) { real t = A[c * bs + q]; A[c * bs + q] = A[piv * bs + q]; A[piv * bs + q] = t; }
      for (int q = 0; q < nc; q++) { real t = B[c * nc + q]; B[c * nc + q] = B[piv * nc + q]; B[piv * nc + q] = t; }
    }
    for (int r = c + 1; r < bs; r++) {
      real l = A[r * bs + c] / A[c * bs + c];
      for (int q = c; q < bs; q++) A[r * bs + q] -= l * A[c * bs + q];
      for (int q = 0; q < nc; q++) B[r * nc + q] -= l * B[c * nc + q];
    }
  }
  for (int c = bs - 1; c >= 0; c--)
    for (int q = 0; q < nc; q++) {
      real s = B[c * nc + q];
      for (int t = c + 1; t < bs; t++) s -= A[c * bs + t] * B[t * nc + q];
      B[c * nc + q] = s / A[c * bs + c];
    }
  return 0;
}

/* Block Thomas for rows 0..n-1: L[i] x[i-1] + D[i] x[i] + U[i] x[i+1] = b[i]
 * (L[0], U[n-1] ignored), bs x bs blocks, nc right-hand-side columns.
 * b (n x bs x nc) is overwritten by the solution.  work: n*bs*bs doubles. */
static int block_thomas(int n, int bs, const real *L, const real *D, const real *U,
                        int nc, real *b, real *C) {
  real A[9], T[9 * 8], tmp[3 * 8];
  int bb = bs * bs, bn = bs * nc, w = bs + nc;
  for (int i = 0; i < n; i++) {
    memcpy(A, D + (long)i * bb, sizeof(real) * bb);
    real *bi = b + (long)i * bn;
    if (i > 0) {
      const real *Li = L + (long)i * bb, *Cp = C + (long)(i - 1) * bb, *yp = b + (long)(i - 1) * bn;
      for (int r = 0; r < bs; r++)
        for (int c = 0; c < bs; c++) {
          real s = 0.0;
          for (int t = 0; t < bs; t++) s += Li[r * bs + t] * Cp[t * bs + c];
          A[r * bs + c] -= s;
        }
      for (int r = 0; r < bs; r++)
        for (int c = 0; c < nc; c++) {
          real s = 0.0;
          for (int t = 0; t < bs; t++) s += Li[r * bs + t] * yp[t * nc + c];
          tmp[r * nc + c] = bi[r * nc + c] - s;
        }
    } else {
      memcpy(tmp, bi, sizeof(real) * bn);
    }
    for (int r = 0; r < bs; r++) {
      for (int c = 0; c < bs; c++) T[r * w + c] = (i < n - 1) ? U[(long)i * bb + r * bs + c] : 0.0;
      for (int c = 0; c < nc; c++) T[r * w + bs + c] = tmp[r * nc + c];
    }
    if (small_solve(bs, A, w, T)) return -1;
    for (int r = 0; r < bs; r++) {
      for (int c = 0; c < bs; c++) C[(long)i * bb + r * bs + c] = T[r * w + c];
      for (int c = 0; c < nc; c++) bi[r * nc + c] = T[r * w + bs + c];
    }
  }
  for (int i = n - 2; i >= 0; i--) {
    real *xi = b + (long)i * bn, *xn = b + (long)(i + 1) * bn;
    const real *Ci = C + (long)i * bb;
    for (int r = 0; r < bs; r++)
      for (int c = 0; c < nc; c++) {
        real s = 0.0;
        for (int t = 0; t < bs; t++) s += Ci[r * bs + t] * xn[t * nc + c];
        xi[r * nc + c] -= s;
      }
  }
  return 0;
}

/* Cyclic block tridiagonal: row 0 couples x[n-1] through L[0], row n-1 couples
 * x[0] through U[n-1].  Bordered elimination of the last block: for rows
 * 0..n-2 solve A'[y | Z] = [b | E] (E: L[0] in row 0, U[n-2] in row n-2),
 * then x[n-1] from row n-1, then x = y - Z x[n-1].  b (n x bs) overwritten. */
static int block_cyclic(int n, int bs, const real *L, const real *D, const real *U,
                        real *b) {
  int bb = bs * bs, nc = 1 + bs, m = n - 1;
  real *L2 = calloc((size_t)m * bb, sizeof(real)), *U2 = calloc((size_t)m * bb, sizeof(real));
  real *B2 = calloc((size_t)m * bs * nc, sizeof(real)), *C = calloc((size_t)m * bb, sizeof(real));
  memcpy(L2, L, sizeof(real) * m * bb);
  memcpy(U2, U, sizeof(real) * m * bb);
  memset(L2, 0, sizeof(real) * bb);                      /* row 0 L -> border */
  memset(U2 + (long)(m - 1) * bb, 0, sizeof(real) * bb); /* row n-2 U -> border */
  for (int i = 0; i < m; i++)
    for (int r = 0; r < bs; r++) B2[(long)i * bs * nc + r * nc] = b[(long)i * bs + r];
  for (int r = 0; r < bs; r++)
    for (int c = 0; c < bs; c++) {
      B2[r * nc + 1 + c] += L[r * bs + c];
      B2[(long)(m - 1) * bs * nc + r * nc + 1 + c] += U[(long)(m - 1) * bb + r * bs + c];
    }
  int rc = block_thomas(m, bs, L2, D, U2, nc, B2, C);
  if (!rc) {
    real A[9], rhs[3];
    const real *Ln = L + (long)(n - 1) * bb, *Dn = D + (long)(n - 1) * bb, *Un = U + (long)(n - 1) * bb;
    const real *Yl = B2 + (long)(m - 1) * bs * nc, *Y0 = B2;
    for (int r = 0; r < bs; r++) {
      real s = b[(long)(n - 1) * bs + r];
      for (int t = 0; t < bs; t++) s -= Ln[r * bs + t] * Yl[t * nc] + Un[r * bs + t] * Y0[t * nc];
      rhs[r] = s;
      for (int c = 0; c < bs; c++) {
        real a = Dn[r * bs + c];
        for (int t = 0; t < bs; t++) a -= Ln[r * bs + t] * Yl[t * nc + 1 + c] + Un[r * bs + t] * Y0[t * nc + 1 + c];
        A[r * bs + c] = a;
      }
    }
    rc = small_solve(bs, A, 1, rhs);
    if (!rc) {
      for (int r = 0; r < bs; r++) b[(long)(n - 1) * bs + r] = rhs[r];
      for (int i = 0; i < m; i++)
        for (int r = 0; r < bs; r++) {
          real s = B2[(long)i * bs * nc + r * nc];
          for (int c = 0; c < bs; c++) s -= B2[(long)i * bs * nc + r * nc + 1 + c] * rhs[c];
          b[(long)i * bs + r] = s;
        }
    }
  }
  free(L2); free(U2); free(B2); free(C);
  return rc;
}

/* ------------------------------------------------------- line geometry -- */

/* A line is described by its direction d (0 r, 1 theta, 2 phi), its length n
 * and, for each position along it, the flat index of each unknown.  Block
 * lines carry (p, T, normal velocity on the face after the cell); scalar
 * lines carry one transverse velocity component. */
typedef struct {
  int d, n, cyclic, last_is_bnd; /* last block's face is a boundary face */
  int tcomp;                     /* scalar lines: field id; block: -1 */
  int a, b;                      /* the two transverse line coordinates */
} line_t;

static int dir_len(const orc_grid *g, int d) { return d == 0 ? g->nr : (d == 1 ? g->nt : g->np); }

/* flat index of (field, position s along line) */
static long line_idx(const orc_grid *g, const line_t *L, int fid, int s) {
  int n = L->n;
  if (L->d == 2 && g->periodic) s = ((s % n) + n) % n;
  switch (L->d) {
  case 0: /* (a,b) = (j,k) or face coords */
    if (fid == FP || fid == FTT) return IC(g, s, L->a, L->b);
    if (fid == FR) return IR(g, s, L->a, L->b);
    if (fid == FT) return IT(g, s, L->a, L->b);
    return IF(g, s, L->a, L->b);
  case 1: /* (a,b) = (i,k) */
    if (fid == FP || fid == FTT) return IC(g, L->a, s, L->b);
    if (fid == FR) return IR(g, L->a, s, L->b);
    if (fid == FT) return IT(g, L->a, s, L->b);
    return IF(g, L->a, s, L->b);
  default: /* (a,b) = (i,j) */
    if (fid == FP || fid == FTT) return IC(g, L->a, L->b, s);
    if (fid == FR) return IR(g, L->a, L->b, s);
    if (fid == FT) return IT(g, L->a, L->b, s);
    return IF(g, L->a, L->b, s);
  }
}

static const int NORMAL_FID[3] = {FR, FT, FF};

/* the (field, flat index) of unknown q (0 p, 1 T, 2 w) of block s; returns 0
 * if that unknown is a boundary face (not an unknown) */
static int block_unknown(const orc_grid *g, const line_t *L, int s, int q, int *fid, long *idx) {
  if (q == 0) { *fid = FP; *idx = line_idx(g, L, FP, s); return 1; }
  if (q == 1) { *fid = FTT; *idx = line_idx(g, L, FTT, s); return 1; }
  if (!L->cyclic && s == L->n - 1) return 0;
  *fid = NORMAL_FID[L->d];
  *idx = line_idx(g, L, *fid, s + 1);
  return 1;
}

static int dmask(int d) { return d == 0 ? MR : (d == 1 ? MT : MF); }

/* Evaluate the row of block s, component q (0 p-row, 1 T-row, 2 w-row) of
 * N_d(u; v). */
static real block_row(const orc_grid *g, const orc_mat *m, const opnd *u, const opnd *v,
                        const line_t *L, int s, int q, const ccoef *cc, const fcoef *fc) {
  int mask = dmask(L->d);
  int i, j, k;
  if (L->d == 0) { i = s; j = L->a; k = L->b; }
  else if (L->d == 1) { i = L->a; j = s; k = L->b; }
  else { i = L->a; j = L->b; k = s; }
  if (q == 0) return row_p(g, m, cc, v, i, j, k, mask);
  if (q == 1) return row_T(g, m, cc, v, i, j, k, mask);
  if (L->d == 0) return row_ur(g, m, fc, v, i + 1, j, k, mask);
  if (L->d == 1) return row_ut(g, m, fc, v, i, j + 1, k, mask);
  return row_uf(g, m, fc, v, i, j, g->periodic ? kwrap(g, k + 1) : k + 1, mask);
}

static void block_fcoef(const orc_grid *g, const orc_mat *m, const opnd *u, const line_t *L,
                        int s, fcoef *fc) {
  if (L->d == 0) fcoef_r(g, m, u, s + 1, L->a, L->b, fc);
  else if (L->d == 1) fcoef_t(g, m, u, L->a, s + 1, L->b, fc);
  else fcoef_f(g, m, u, L->a, L->b, g->periodic ? kwrap(g, s + 1) : s + 1, fc);
}

/* Assemble (I + tau/2 N_d(Ubar; .)) on a block line by probing with unit
 * operands.  Lb, Db, Ub: n x 9 each. */
static void assemble_block(const orc_grid *g, const orc_mat *m, const opnd *u, const line_t *L,
                           double tau, real *Lb, real *Db, real *Ub) {
  int n = L->n;
  memset(Lb, 0, sizeof(real) * 9 * n);
  memset(Db, 0, sizeof(real) * 9 * n);
  memset(Ub, 0, sizeof(real) * 9 * n);
  for (int s = 0; s < n; s++) {
    ccoef cc;
    fcoef fc;
    int i = L->d == 0 ? s : L->a, j = L->d == 0 ? L->a : (L->d == 1 ? s : L->b),
        k = L->d == 2 ? s : L->b;
    ccoef_at(g, m, u, i, j, k, &cc);
    int w_is_unknown = L->cyclic || s < n - 1;
    if (w_is_unknown) block_fcoef(g, m, u, L, s, &fc);
    for (int off = -1; off <= 1; off++) {
      int s2 = s + off;
      if (!L->cyclic && (s2 < 0 || s2 >= n)) continue;
      int s2w = L->cyclic ? ((s2 % n) + n) % n : s2;
      real *blk = off < 0 ? Lb : (off == 0 ? Db : Ub);
      for (int q2 = 0; q2 < 3; q2++) {
        opnd e;
        memset(&e, 0, sizeof(e));
        e.w = NULL;
        if (!block_unknown(g, L, s2w, q2, &e.ufid, &e.uidx)) continue;
        for (int q = 0; q < 3; q++) {
          if (q == 2 && !w_is_unknown) continue;
          real val = block_row(g, m, u, &e, L, s, q, &cc, &fc);
          blk[(long)s * 9 + q * 3 + q2] += 0.5 * tau * val;
        }
      }
    }
    for (int q = 0; q < 3; q++) Db[(long)s * 9 + q * 4] += 1.0;
    if (!w_is_unknown) { /* identity row for the boundary face */
      for (int q2 = 0; q2 < 3; q2++) {
        Lb[(long)s * 9 + 6 + q2] = 0.0;
        Db[(long)s * 9 + 6 + q2] = (q2 == 2) ? 1.0 : 0.0;
        Ub[(long)s * 9 + 6 + q2] = 0.0;
      }
    }
  }
}

/* scalar line: the component tcomp at position s */
static real scalar_row(const orc_grid *g, const orc_mat *m, const opnd *v, const line_t *L,
                         int s, const fcoef *fc) {
  int mask = dmask(L->d);
  int i, j, k; /* position of the face in (i,j,k) face-index space */
  if (L->d == 0) { i = s; j = L->a; k = L->b; }
  else if (L->d == 1) { i = L->a; j = s; k = L->b; }
  else { i = L->a; j = L->b; k = s; }
  if (L->tcomp == FR) return row_ur(g, m, fc, v, i, j, k, mask);
  if (L->tcomp == FT) return row_ut(g, m, fc, v, i, j, k, mask);
  return row_uf(g, m, fc, v, i, j, k, mask);
}

static void scalar_fcoef(const orc_grid *g, const orc_mat *m, const opnd *u, const line_t *L, int s,
                         fcoef *fc) {
  int i, j, k;
  if (L->d == 0) { i = s; j = L->a; k = L->b; }
  else if (L->d == 1) { i = L->a; j = s; k = L->b; }
  else { i = L->a; j = L->b; k = s; }
  if (L->tcomp == FR) fcoef_r(g, m, u, i, j, k, fc);
  else if (L->tcomp == FT) fcoef_t(g, m, u, i, j, k, fc);
  else fcoef_f(g, m, u, i, j, k, fc);
}

static void assemble_scalar(const orc_grid *g, const orc_mat *m, const opnd *u, const line_t *L,
                            double tau, real *a, real *bd, real *c) {
  int n = L->n;
  for (int s = 0; s < n; s++) {
    fcoef fc;
    scalar_fcoef(g, m, u, L, s, &fc);
    real co[3] = {0, 0, 0};
    for (int off = -1; off <= 1; off++) {
      int s2 = s + off;
      if (!L->cyclic && (s2 < 0 || s2 >= n)) continue;
      opnd e;
      memset(&e, 0, sizeof(e));
      e.ufid = L->tcomp;
      e.uidx = line_idx(g, L, L->tcomp, s2);
      co[off + 1] = scalar_row(g, m, &e, L, s, &fc);
    }
    a[s] = 0.5 * tau * co[0];
    bd[s] = 1.0 + 0.5 * tau * co[1];
    c[s] = 0.5 * tau * co[2];
  }
}

/* enumerate the lines of direction d: block lines first, then the two scalar
 * families.  Returns the number of lines; fills L if non-NULL. */
static long enum_lines(const orc_grid *g, int d, line_t *out) {
  long cnt = 0;
  int cyc = (d == 2 && g->periodic);
  int nr = g->nr, nt = g->nt, np = g->np;
#define PUSH(tc, A, B)                                                              \
  do {                                                                              \
    if (out) {                                                                      \
      out[cnt].d = d; out[cnt].n = dir_len(g, d); out[cnt].cyclic = cyc;            \
      out[cnt].last_is_bnd = !cyc; out[cnt].tcomp = (tc); out[cnt].a = (A); out[cnt].b = (B); \
    }                                                                               \
    cnt++;                                                                          \
  } while (0)
  int kf_lo = g->periodic ? 0 : 1, kf_hi = g->periodic ? np - 1 : np - 1;
  if (d == 0) {
    for (int j = 0; j < nt; j++) for (int k = 0; k < np; k++) PUSH(-1, j, k);
    for (int f = 1; f < nt; f++) for (int k = 0; k < np; k++) PUSH(FT, f, k);
    for (int j = 0; j < nt; j++) for (int f = kf_lo; f <= kf_hi; f++) PUSH(FF, j, f);
  } else if (d == 1) {
    for (int i = 0; i < nr; i++) for (int k = 0; k < np; k++) PUSH(-1, i, k);
    for (int f = 1; f < nr; f++) for (int k = 0; k < np; k++) PUSH(FR, f, k);
    for (int i = 0; i < nr; i++) for (int f = kf_lo; f <= kf_hi; f++) PUSH(FF, i, f);
  } else {
    for (int i = 0; i < nr; i++) for (int j = 0; j < nt; j++) PUSH(-1, i, j);
    for (int f = 1; f < nr; f++) for (int j = 0; j < nt; j++) PUSH(FR, f, j);
    for (int i = 0; i < nr; i++) for (int f = 1; f < nt; f++) PUSH(FT, i, f);
  }
#undef PUSH
  return cnt;
}

/* ------------------------------------------------------------ line solve -- */

static const real *fld(const orc_fields *x, int fid) {
  return fid == FP ? x->p : fid == FR ? x->ur : fid == FT ? x->ut : fid == FF ? x->uf : x->T;
}
static real *fldw(orc_fields *x, int fid) {
  return fid == FP ? x->p : fid == FR ? x->ur : fid == FT ? x->ut : fid == FF ? x->uf : x->T;
}

/* Solve (I + tau/2 D_d(Ubar)) x = rhs on every line of direction d (0 r, 1
 * theta, 2 phi) with homogeneous increment boundary conditions.  Returns 0,
 * or -1 if some block pivot vanished. */
int orc_line_solve(const orc_grid *g, const orc_mat *m, const orc_fields *Ub, const orc_wall *wall,
                   double tau, int d, const orc_fields *rhs, orc_fields *x) {
  long nl = enum_lines(g, d, NULL);
  line_t *lines = malloc(sizeof(line_t) * nl);
  enum_lines(g, d, lines);
  opnd u = mk_opnd(Ub, wall);
  zero_fields(g, x);
  int n = dir_len(g, d), err = 0;
#pragma omp parallel reduction(| : err)
  {
    real *Lb = malloc(sizeof(real) * 9 * n), *Db = malloc(sizeof(real) * 9 * n);
    real *Ubk = malloc(sizeof(real) * 9 * n), *bv = malloc(sizeof(real) * 3 * n);
    real *C = malloc(sizeof(real) * 9 * n);
#pragma omp for schedule(static)
    for (long l = 0; l < nl; l++) {
      const line_t *L = &lines[l];
      if (L->tcomp < 0) {
        assemble_block(g, m, &u, L, tau, Lb, Db, Ubk);
        for (int s = 0; s < n; s++)
          for (int q = 0; q < 3; q++) {
            int fid; long idx;
            bv[s * 3 + q] = block_unknown(g, L, s, q, &fid, &idx) ? fld(rhs, fid)[idx] : 0.0;
          }
        int rc = L->cyclic ? block_cyclic(n, 3, Lb, Db, Ubk, bv) : block_thomas(n, 3, Lb, Db, Ubk, 1, bv, C);
        if (rc) err |= 1;
        for (int s = 0; s < n; s++)
          for (int q = 0; q < 3; q++) {
            int fid; long idx;
            if (block_unknown(g, L, s, q, &fid, &idx)) fldw(x, fid)[idx] = bv[s * 3 + q];
          }
      } else {
        real *a = Lb, *bd = Db, *c = Ubk;
        assemble_scalar(g, m, &u, L, tau, a, bd, c);
        for (int s = 0; s < n; s++) bv[s] = fld(rhs, L->tcomp)[line_idx(g, L, L->tcomp, s)];
        int rc = L->cyclic ? block_cyclic(n, 1, a, bd, c, bv) : block_thomas(n, 1, a, bd, c, 1, bv, C);
        if (rc) err |= 1;
        for (int s = 0; s < n; s++) fldw(x, L->tcomp)[line_idx(g, L, L->tcomp, s)] = bv[s];
      }
    }
    free(Lb); free(Db); free(Ubk); free(bv); free(C);
  }
  free(lines);
  return err ? -1 : 0;
}

/* y = (I + tau/2 D_d(Ubar)) x using the assembled line matrices (for checking
 * the assembly against orc_apply). */
int orc_line_matvec(const orc_grid *g, const orc_mat *m, const orc_fields *Ub, const orc_wall *wall,
                    double tau, int d, const orc_fields *x, orc_fields *y) {
  long nl = enum_lines(g, d, NULL);
  line_t *lines = malloc(sizeof(line_t) * nl);
  enum_lines(g, d, lines);
  opnd u = mk_opnd(Ub, wall);
  zero_fields(g, y);
  int n = dir_len(g, d);
#pragma omp parallel
  {
    real *Lb = malloc(sizeof(real) * 9 * n), *Db = malloc(sizeof(real) * 9 * n);
    real *Ubk = malloc(sizeof(real) * 9 * n), *xv = malloc(sizeof(real) * 3 * n);
#pragma omp for schedule(static)
    for (long l = 0; l < nl; l++) {
      const line_t *L = &lines[l];
      int bs = L->tcomp < 0 ? 3 : 1;
      if (bs == 3) {
        assemble_block(g, m, &u, L, tau, Lb, Db, Ubk);
        for (int s = 0; s < n; s++)
          for (int q = 0; q < 3; q++) {
            int fid; long idx;
            xv[s * 3 + q] = block_unknown(g, L, s, q, &fid, &idx) ? fld(x, fid)[idx] : 0.0;
          }
      } else {
        assemble_scalar(g, m, &u, L, tau, Lb, Db, Ubk);
        for (int s = 0; s < n; s++) xv[s] = fld(x, L->tcomp)[line_idx(g, L, L->tcomp, s)];
      }
      for (int s = 0; s < n; s++) {
        for (int q = 0; q < bs; q++) {
          real acc = 0.0;
          for (int off = -1; off <= 1; off++) {
            int s2 = s + off;
            if (!L->cyclic && (s2 < 0 || s2 >= n)) continue;
            s2 = ((s2 % n) + n) % n;
            const real *blk = off < 0 ? Lb : (off == 0 ? Db : Ubk);
            for (int q2 = 0; q2 < bs; q2++) acc += blk[(long)s * bs * bs + q * bs + q2] * xv[s2 * bs + q2];
          }
          if (bs == 3) {
            int fid; long idx;
            if (block_unknown(g, L, s, q, &fid, &idx)) fldw(y, fid)[idx] = acc;
          } else {
            fldw(y, L->tcomp)[line_idx(g, L, L->tcomp, s)] = acc;
          }
        }
      }
    }
    free(Lb); free(Db); free(Ubk); free(xv);
  }
  free(lines);
  return 0;
}

/* Export the blocks of one line (for dense-LU tests).  kind: -1 block line,
 * else the scalar family's field id; (a, b) the line's transverse coords.
 * L/D/U: n*bs*bs; idx: n*bs flat indices (-1 for a boundary face), fid: n*bs. */
int orc_line_blocks(const orc_grid *g, const orc_mat *m, const orc_fields *Ub, const orc_wall *wall,
                    double tau, int d, int kind, int a, int b, real *Lo, real *Do, real *Uo,
                    long *idx, int *fid) {
  line_t L;
  L.d = d; L.n = dir_len(g, d); L.cyclic = (d == 2 && g->periodic); L.last_is_bnd = !L.cyclic;
  L.tcomp = kind; L.a = a; L.b = b;
  opnd u = mk_opnd(Ub, wall);
  if (kind < 0) {
    assemble_block(g, m, &u, &L, tau, Lo, Do, Uo);
    for (int s = 0; s < L.n; s++)
      for (int q = 0; q < 3; q++) {
        int f; long x;
        if (block_unknown(g, &L, s, q, &f, &x)) { idx[s * 3 + q] = x; fid[s * 3 + q] = f; }
        else { idx[s * 3 + q] = -1; fid[s * 3 + q] = NORMAL_FID[d]; }
      }
  } else {
    assemble_scalar(g, m, &u, &L, tau, Lo, Do, Uo);
    for (int s = 0; s < L.n; s++) { idx[s] = line_idx(g, &L, kind, s); fid[s] = kind; }
  }
  return L.cyclic;
}

/* ----------------------------------------------------------- split step -- */

static void alloc_fields(const orc_grid *g, orc_fields *x) {
  x->p = calloc(fsize(g, FP), sizeof(real)); x->ur = calloc(fsize(g, FR), sizeof(real));
  x->ut = calloc(fsize(g, FT), sizeof(real)); x->uf = calloc(fsize(g, FF), sizeof(real));
  x->T = calloc(fsize(g, FTT), sizeof(real));
}
static void free_fields(orc_fields *x) { free(x->p); free(x->ur); free(x->ut); free(x->uf); free(x->T); }

/* copy only the boundary-normal faces of src into dst */
static void copy_bnd_faces(const orc_grid *g, const orc_fields *src, orc_fields *dst) {
  for (int j = 0; j < g->nt; j++)
    for (int k = 0; k < g->np; k++) {
      dst->ur[IR(g, 0, j, k)] = src->ur[IR(g, 0, j, k)];
      dst->ur[IR(g, g->nr, j, k)] = src->ur[IR(g, g->nr, j, k)];
    }
  for (int i = 0; i < g->nr; i++)
    for (int k = 0; k < g->np; k++) {
      dst->ut[IT(g, i, 0, k)] = src->ut[IT(g, i, 0, k)];
      dst->ut[IT(g, i, g->nt, k)] = src->ut[IT(g, i, g->nt, k)];
    }
  if (!g->periodic)
    for (int i = 0; i < g->nr; i++)
      for (int j = 0; j < g->nt; j++) {
        dst->uf[IF(g, i, j, 0)] = src->uf[IF(g, i, j, 0)];
        dst->uf[IF(g, i, j, g->np)] = src->uf[IF(g, i, j, g->np)];
      }
}

/* wall data: lengths of the twelve arrays and a linear combination of two
 * sets (a NULL set or entry counts as zero) */
static long wall_len(const orc_grid *g, int q) {
  switch (q) {
  case 0: case 1: return (long)(g->nr + 1) * g->np;   /* ur_t1, ur_t2 */
  case 2: case 3: return (long)(g->nr + 1) * g->nt;   /* ur_p1, ur_p2 */
  case 4: case 5: return (long)(g->nt + 1) * g->np;   /* ut_r1, ut_r2 */
  case 6: case 7: return (long)g->nr * (g->nt + 1);   /* ut_p1, ut_p2 */
  case 8: case 9: return (long)g->nt * g->npf;        /* uf_r1, uf_r2 */
  default: return (long)g->nr * g->npf;               /* uf_t1, uf_t2 */
  }
}
static const real *wall_get(const orc_wall *w, int q) {
  if (!w) return NULL;
  const real *const a[12] = {w->ur_t1, w->ur_t2, w->ur_p1, w->ur_p2, w->ut_r1, w->ut_r2,
                             w->ut_p1, w->ut_p2, w->uf_r1, w->uf_r2, w->uf_t1, w->uf_t2};
  return a[q];
}
static void wall_set(orc_wall *w, int q, const real *x) {
  const real **a[12] = {&w->ur_t1, &w->ur_t2, &w->ur_p1, &w->ur_p2, &w->ut_r1, &w->ut_r2,
                        &w->ut_p1, &w->ut_p2, &w->uf_r1, &w->uf_r2, &w->uf_t1, &w->uf_t2};
  *a[q] = x;
}
/* out = ca a + cb b entry by entry; mem[12] receives the arrays to free */
static void wall_mix(const orc_grid *g, double ca, const orc_wall *a, double cb, const orc_wall *b,
                     orc_wall *out, real **mem) {
  memset(out, 0, sizeof(*out));
  for (int q = 0; q < 12; q++) {
    const real *x = wall_get(a, q), *y = wall_get(b, q);
    long n = wall_len(g, q);
    mem[q] = calloc(n, sizeof(real));
    for (long e = 0; e < n; e++) mem[q][e] = ca * (x ? x[e] : 0.0) + cb * (y ? y[e] : 0.0);
    wall_set(out, q, mem[q]);
  }
}
/* the walls of direction d (normal to it) take part in the d sweep: their
 * tangential data are the wall indices 4,5,8,9 (r), 0,1,10,11 (theta),
 * 2,3,6,7 (phi) */
static int wall_of_dir(int q, int d) {
  static const int dir[12] = {1, 1, 2, 2, 0, 0, 2, 2, 0, 0, 1, 1};
  return dir[q] == d;
}

/* One split time step: U^{n+1} from U^n with K iterations (section 2.2).
 *
 * Boundary data (velocity Dirichlet data, paper section 3.1: they vary in time
 * for a manufactured solution):
 *   wall0, wall1: tangential wall velocities at t^n and t^{n+1} (NULL: zero);
 *   bnd: fields whose boundary-normal faces hold the Dirichlet data at
 *   t^{n+1} (NULL: those of Un, unchanged); Un's hold those at t^n;
 *   src: the source taken at the midpoint time (may be NULL).
 * U^{n+1,0} = U^n, boundary faces and wall data included (eq.
 * (chapter3mainsd): the iteration starts from U^n).  Every iterate's
 * increment solves (spl1)-(spl3) carry the change of the boundary data from
 * iterate k to the new time level as inhomogeneous Dirichlet data of the
 * increments xi - U^{n+1,k}, eta - U^{n+1,k}, U^{n+1,k+1} - U^{n+1,k}: in the
 * d sweep the data on the walls normal to d are lifted out of the increment
 * (X = X_0 + X_b, X_b zero but on those walls), i.e. the right-hand side
 * loses tau/2 D_d(Ubar) X_b and X_0 solves the homogeneous line systems.
 * After the first iteration every iterate holds the new data, so the later
 * increments are homogeneous.  Ubar's ghost values take the mean wall data of
 * U^{n+1,k} and U^n.  Returns 0, or -1 on a vanishing pivot. */
int orc_split_step(const orc_grid *g, const orc_mat *m, const orc_fields *Un, orc_fields *Unp1,
                   double tau, int K, const orc_wall *wall0, const orc_wall *wall1,
                   const orc_fields *src, const orc_fields *bnd) {
  orc_fields Uk, R, Ub, X1, X2, X3, Xb, C;
  alloc_fields(g, &Uk); alloc_fields(g, &R); alloc_fields(g, &Ub);
  alloc_fields(g, &X1); alloc_fields(g, &X2); alloc_fields(g, &X3);
  alloc_fields(g, &Xb); alloc_fields(g, &C);
  const real *un[5] = {Un->p, Un->ur, Un->ut, Un->uf, Un->T};
  real *uk[5] = {Uk.p, Uk.ur, Uk.ut, Uk.uf, Uk.T};
  for (int q = 0; q < 5; q++) memcpy(uk[q], un[q], sizeof(real) * fsize(g, q));
  orc_fields Bn1; /* Dirichlet data of the new time level on boundary faces */
  alloc_fields(g, &Bn1);
  copy_bnd_faces(g, bnd ? bnd : Un, &Bn1);
  real *wmem[3][12];
  orc_wall wmid0, wmid1, dw0;   /* mean wall data of the iterates 0 and >= 1; change at 0 */
  wall_mix(g, 1.0, wall0, 0.0, NULL, &wmid0, wmem[0]);
  wall_mix(g, 0.5, wall0, 0.5, wall1, &wmid1, wmem[1]);
  wall_mix(g, 1.0, wall1, -1.0, wall0, &dw0, wmem[2]);
  int rc = 0;
  for (int it = 0; it < K && !rc; it++) {
    const orc_wall *wm = it == 0 ? &wmid0 : &wmid1;
    orc_residual(g, m, Un, &Uk, wm, src, tau, &R, &Ub);
    const orc_fields *rhs = &R;
    orc_fields *outs[3] = {&X1, &X2, &X3};
    for (int d = 0; d < 3 && !rc; d++) {
      if (it == 0) {
        /* X_b: the change of the data on the walls normal to d */
        zero_fields(g, &Xb);
        if (d == 0)
          for (int j = 0; j < g->nt; j++)
            for (int k = 0; k < g->np; k++)
              for (int f = 0; f <= g->nr; f += g->nr)
                Xb.ur[IR(g, f, j, k)] = Bn1.ur[IR(g, f, j, k)] - Uk.ur[IR(g, f, j, k)];
        if (d == 1)
          for (int i = 0; i < g->nr; i++)
            for (int k = 0; k < g->np; k++)
              for (int f = 0; f <= g->nt; f += g->nt)
                Xb.ut[IT(g, i, f, k)] = Bn1.ut[IT(g, i, f, k)] - Uk.ut[IT(g, i, f, k)];
        if (d == 2 && !g->periodic)
          for (int i = 0; i < g->nr; i++)
            for (int j = 0; j < g->nt; j++)
              for (int f = 0; f <= g->np; f += g->np)
                Xb.uf[IF(g, i, j, f)] = Bn1.uf[IF(g, i, j, f)] - Uk.uf[IF(g, i, j, f)];
        orc_wall dwd;
        memset(&dwd, 0, sizeof(dwd));
        for (int q = 0; q < 12; q++)
          if (wall_of_dir(q, d)) wall_set(&dwd, q, wall_get(&dw0, q));
        orc_apply(g, m, &Ub, wm, &Xb, &dwd, d == 0 ? MR : (d == 1 ? MT : MF), &C);
        real *cc[5] = {C.p, C.ur, C.ut, C.uf, C.T};
        const real *rr[5] = {rhs->p, rhs->ur, rhs->ut, rhs->uf, rhs->T};
        for (int q = 0; q < 5; q++) {
          long n = fsize(g, q);
          for (long x = 0; x < n; x++) cc[q][x] = rr[q][x] - 0.5 * tau * cc[q][x];
        }
        rc |= orc_line_solve(g, m, &Ub, wm, tau, d, &C, outs[d]);
      } else {
        rc |= orc_line_solve(g, m, &Ub, wm, tau, d, rhs, outs[d]);
      }
      rhs = outs[d];
    }
    real *x3[5] = {X3.p, X3.ur, X3.ut, X3.uf, X3.T};
    for (int q = 0; q < 5; q++) {
      long n = fsize(g, q);
      for (long x = 0; x < n; x++) uk[q][x] += x3[q][x];
    }
    copy_bnd_faces(g, &Bn1, &Uk); /* every later iterate holds the new data */
  }
  real *out[5] = {Unp1->p, Unp1->ur, Unp1->ut, Unp1->uf, Unp1->T};
  for (int q = 0; q < 5; q++) memcpy(out[q], uk[q], sizeof(real) * fsize(g, q));
  free_fields(&Uk); free_fields(&R); free_fields(&Ub);
  free_fields(&X1); free_fields(&X2); free_fields(&X3);
  free_fields(&Xb); free_fields(&C); free_fields(&Bn1);
  for (int a = 0; a < 3; a++)
    for (int q = 0; q < 12; q++) free(wmem[a][q]);
  return rc ? -1 : 0;
}

/* ------------------------------------ perturbation-pressure form (f4) -- */

/* Paper section 3.1 (remark after Table 3): with a large background pressure
 * p0 the errors of the pressure derivatives scale with p0, and the pressure
 * has to be rescaled a priori.  Here the state carries p' = p - pbar(r)
 * instead of p, for a reference column (pbar_i, Tbar_i) at the cell centres
 * that is discretely hydrostatic under the radial momentum row at rest:
 *   (pbar_f - pbar_{f-1}) / dr + g_r (rhobar_{f-1} + rhobar_f) / 2 = 0,
 *   rhobar_i = (pbar_i + pi_inf) / (R Tbar_i),   R = c_p - c_v.
 * The step is the same scheme with that balance subtracted analytically:
 *   - every coefficient (density, P, chi) sees the full p' + pbar;
 *   - the radial row's pressure gradient plus gravity,
 *       (p_f - p_{f-1}) / (rho_f dr) + g_r,
 *     reads (p'_f - p'_{f-1}) / (rho_f dr) + g_r (rho_f - rhobar_f) / rho_f,
 *     with rho_i - rhobar_i = (p'_i Tbar_i - (pbar_i + pi_inf)(T_i - Tbar_i))
 *     / (R T_i Tbar_i) formed without a difference of large numbers;
 *   - the advection of p gains the reference gradient, u_r (pbar_{i+1} -
 *     pbar_{i-1}) / (2 dr), with the copy ghosts of p at the r walls;
 *   - theta and phi differences of p are those of p' (pbar depends on r only).
 * In exact arithmetic this is orc_split_step on p = p' + pbar.  Plain walls,
 * no source term. */
static real drho_ref(const orc_grid *g, const orc_mat *m, const double *pbar, const double *Tbar,
                     const orc_fields *U, int i, int j, int k) {
  long x = IC(g, i, j, k);
  real T = U->T[x];
  return (U->p[x] * Tbar[i] - (pbar[i] + m->pi_inf) * (T - Tbar[i])) / ((m->cp - m->cv) * T * Tbar[i]);
}

/* R for the perturbation state: Un, Uk and Ub carry p'; Uf receives the full
 * midpoint (p' + pbar) that the line solves take as coefficients. */
static void residual_pert(const orc_grid *g, const orc_mat *m, const double *pbar, const double *Tbar,
                          const orc_fields *Un, const orc_fields *Uk, double tau, orc_fields *R,
                          orc_fields *Ub, orc_fields *Uf) {
  const real *un[5] = {Un->p, Un->ur, Un->ut, Un->uf, Un->T};
  const real *uk[5] = {Uk->p, Uk->ur, Uk->ut, Uk->uf, Uk->T};
  real *ub[5] = {Ub->p, Ub->ur, Ub->ut, Ub->uf, Ub->T};
  real *uf[5] = {Uf->p, Uf->ur, Uf->ut, Uf->uf, Uf->T};
  for (int q = 0; q < 5; q++) {
    long n = fsize(g, q);
    for (long x = 0; x < n; x++) ub[q][x] = 0.5 * (uk[q][x] + un[q][x]);
    memcpy(uf[q], ub[q], sizeof(real) * n);
  }
  for (int i = 0; i < g->nr; i++)
    for (int j = 0; j < g->nt; j++)
      for (int k = 0; k < g->np; k++) Uf->p[IC(g, i, j, k)] += pbar[i];
  orc_fields F;
  alloc_fields(g, &F);
  orc_apply(g, m, Uf, NULL, Ub, NULL, MALL, &F); /* coefficients of the full state, operand p' */
  opnd u = mk_opnd(Uf, NULL);
  real *rr[5] = {R->p, R->ur, R->ut, R->uf, R->T};
  for (int q = 0; q < 5; q++) memset(rr[q], 0, sizeof(real) * fsize(g, q));
  for (int i = 0; i < g->nr; i++) {
    double dpb = (pbar[i + 1 < g->nr ? i + 1 : g->nr - 1] - pbar[i > 0 ? i - 1 : 0]) / (2.0 * g->dr);
    for (int j = 0; j < g->nt; j++)
      for (int k = 0; k < g->np; k++) {
        long x = IC(g, i, j, k);
        real Fp = F.p[x] + urc(g, &u, i, j, k) * dpb;
        R->p[x] = -(uk[FP][x] - un[FP][x]) - tau * Fp;
        R->T[x] = -(uk[FTT][x] - un[FTT][x]) - tau * F.T[x];
      }
  }
  for (int f = 1; f < g->nr; f++)
    for (int j = 0; j < g->nt; j++)
      for (int k = 0; k < g->np; k++) {
        long x = IR(g, f, j, k);
        real rho_f = 0.5 * (rho_c(g, m, &u, f - 1, j, k) + rho_c(g, m, &u, f, j, k));
        real drho_f = 0.5 * (drho_ref(g, m, pbar, Tbar, Ub, f - 1, j, k) + drho_ref(g, m, pbar, Tbar, Ub, f, j, k));
        real Fx = F.ur[x] + m->g_r * drho_f / rho_f;
        R->ur[x] = -(uk[FR][x] - un[FR][x]) - tau * Fx;
      }
  for (int i = 0; i < g->nr; i++)
    for (int f = 1; f < g->nt; f++)
      for (int k = 0; k < g->np; k++) {
        long x = IT(g, i, f, k);
        R->ut[x] = -(uk[FT][x] - un[FT][x]) - tau * F.ut[x];
      }
  for (int i = 0; i < g->nr; i++)
    for (int j = 0; j < g->nt; j++)
      for (int f = uf_lo(g); f <= uf_hi(g); f++) {
        long x = IF(g, i, j, f);
        R->uf[x] = -(uk[FF][x] - un[FF][x]) - tau * F.uf[x];
      }
  free_fields(&F);
}

int orc_split_step_pert(const orc_grid *g, const orc_mat *m, const double *pbar, const double *Tbar,
                        const orc_fields *Un, orc_fields *Unp1, double tau, int K) {
  orc_fields Uk, R, Ub, Uf, X1, X2, X3;
  alloc_fields(g, &Uk); alloc_fields(g, &R); alloc_fields(g, &Ub); alloc_fields(g, &Uf);
  alloc_fields(g, &X1); alloc_fields(g, &X2); alloc_fields(g, &X3);
  const real *un[5] = {Un->p, Un->ur, Un->ut, Un->uf, Un->T};
  real *uk[5] = {Uk.p, Uk.ur, Uk.ut, Uk.uf, Uk.T};
  for (int q = 0; q < 5; q++) memcpy(uk[q], un[q], sizeof(real) * fsize(g, q));
  int rc = 0;
  for (int it = 0; it < K && !rc; it++) {
    residual_pert(g, m, pbar, Tbar, Un, &Uk, tau, &R, &Ub, &Uf);
    rc |= orc_line_solve(g, m, &Uf, NULL, tau, 0, &R, &X1);
    rc |= orc_line_solve(g, m, &Uf, NULL, tau, 1, &X1, &X2);
    rc |= orc_line_solve(g, m, &Uf, NULL, tau, 2, &X2, &X3);
    real *x3[5] = {X3.p, X3.ur, X3.ut, X3.uf, X3.T};
    for (int q = 0; q < 5; q++) {
      long n = fsize(g, q);
      for (long x = 0; x < n; x++) uk[q][x] += x3[q][x];
    }
  }
  real *out[5] = {Unp1->p, Unp1->ur, Unp1->ut, Unp1->uf, Unp1->T};
  for (int q = 0; q < 5; q++) memcpy(out[q], uk[q], sizeof(real) * fsize(g, q));
  free_fields(&Uk); free_fields(&R); free_fields(&Ub); free_fields(&Uf);
  free_fields(&X1); free_fields(&X2); free_fields(&X3);
  return rc ? -1 : 0;
}

#ifndef ORC_COMPLEX_STEP
/* Courant numbers of a state for the step tau (for a time-step controller:
 * the paper's section 3.2 discussion of Thermal 1 calls for small or adaptive
 * time steps once the bubble accelerates).  At every cell centre, with the
 * centre-averaged velocity and the local spacings h_r = dr,
 * h_t = r dtheta, h_f = r sin(theta) dphi:
 *   advective  tau (|u_r| / h_r + |u_theta| / h_t + |u_phi| / h_f)
 *   acoustic   tau c max(1/h_r, 1/h_t, 1/h_f),  c = sqrt(gamma R T)
 *              (the sound speed of the stiffened gas, c^2 = gamma (p + pi_inf) / rho);
 * out[0], out[1] = their maxima over the cells. */
void orc_courant(const orc_grid *g, const orc_mat *m, const orc_fields *U, double tau, double *out) {
  opnd u = mk_opnd(U, NULL);
  double gam = m->cp / m->cv, Rg = m->cp - m->cv, ca = 0.0, cs = 0.0;
  for (int i = 0; i < g->nr; i++)
    for (int j = 0; j < g->nt; j++)
      for (int k = 0; k < g->np; k++) {
        double hr = g->dr, ht = g->rc[i] * g->dt, hf = g->rc[i] * g->sc[j] * g->dp;
        double a = tau * (fabs(urc(g, &u, i, j, k)) / hr + fabs(utc(g, &u, i, j, k)) / ht +
                          fabs(ufc(g, &u, i, j, k)) / hf);
        double ih = 1.0 / hr;
        if (1.0 / ht > ih) ih = 1.0 / ht;
        if (1.0 / hf > ih) ih = 1.0 / hf;
        double c = tau * sqrt(gam * Rg * U->T[IC(g, i, j, k)]) * ih;
        if (a > ca) ca = a;
        if (c > cs) cs = c;
      }
  out[0] = ca;
  out[1] = cs;
}
#endif

/* residual values at a list of sample points only (for full-size checks of a
 * GPU residual without a full oracle pass).  fids/idx: npts entries; Ub must
 * already hold the midpoint state (ghost data wall).  out: R at each point. */
int orc_residual_at(const orc_grid *g, const orc_mat *m, const orc_fields *Un, const orc_fields *Uk,
                    const orc_fields *Ub, const orc_wall *wall, double tau, long npts,
                    const int *fids, const long *idx, real *out) {
  opnd u = mk_opnd(Ub, wall);
  const real *un[5] = {Un->p, Un->ur, Un->ut, Un->uf, Un->T};
  const real *uk[5] = {Uk->p, Uk->ur, Uk->ut, Uk->uf, Uk->T};
#pragma omp parallel for schedule(static)
  for (long s = 0; s < npts; s++) {
    int fid = fids[s];
    long x = idx[s];
    real F = 0.0;
    int unknown = 1;
    if (fid == FP || fid == FTT) {
      int k = (int)(x % g->np), j = (int)((x / g->np) % g->nt), i = (int)(x / ((long)g->np * g->nt));
      ccoef c;
      ccoef_at(g, m, &u, i, j, k, &c);
      F = fid == FP ? row_p(g, m, &c, &u, i, j, k, MALL) : row_T(g, m, &c, &u, i, j, k, MALL);
    } else if (fid == FR) {
      int k = (int)(x % g->np), j = (int)((x / g->np) % g->nt), f = (int)(x / ((long)g->np * g->nt));
      if (f == 0 || f == g->nr) unknown = 0;
      else { fcoef c; fcoef_r(g, m, &u, f, j, k, &c); F = row_ur(g, m, &c, &u, f, j, k, MALL) + m->g_r; }
    } else if (fid == FT) {
      int k = (int)(x % g->np), f = (int)((x / g->np) % (g->nt + 1)), i = (int)(x / ((long)g->np * (g->nt + 1)));
      if (f == 0 || f == g->nt) unknown = 0;
      else { fcoef c; fcoef_t(g, m, &u, i, f, k, &c); F = row_ut(g, m, &c, &u, i, f, k, MALL); }
    } else {
      int f = (int)(x % g->npf), j = (int)((x / g->npf) % g->nt), i = (int)(x / ((long)g->npf * g->nt));
      if (!g->periodic && (f == 0 || f == g->np)) unknown = 0;
      else { fcoef c; fcoef_f(g, m, &u, i, j, f, &c); F = row_uf(g, m, &c, &u, i, j, f, MALL); }
    }
    out[s] = unknown ? (-(uk[fid][x] - un[fid][x]) - tau * F) : 0.0;
  }
  return 0;
}

/* Solve a selection of lines only: x receives the solution on those lines
 * (other entries untouched).  kinds/as/bs: nl entries (kind -1 block line,
 * else the scalar family's field id). */
int orc_line_solve_some(const orc_grid *g, const orc_mat *m, const orc_fields *Ub,
                        const orc_wall *wall, double tau, int d, long nl, const int *kinds,
                        const int *as, const int *bs_, const orc_fields *rhs, orc_fields *x) {
  opnd u = mk_opnd(Ub, wall);
  int n = dir_len(g, d), err = 0;
#pragma omp parallel reduction(| : err)
  {
    real *Lb = malloc(sizeof(real) * 9 * n), *Db = malloc(sizeof(real) * 9 * n);
    real *Ubk = malloc(sizeof(real) * 9 * n), *bv = malloc(sizeof(real) * 3 * n);
    real *C = malloc(sizeof(real) * 9 * n);
#pragma omp for schedule(static)
    for (long l = 0; l < nl; l++) {
      line_t L;
      L.d = d; L.n = n; L.cyclic = (d == 2 && g->periodic); L.last_is_bnd = !L.cyclic;
      L.tcomp = kinds[l]; L.a = as[l]; L.b = bs_[l];
      if (L.tcomp < 0) {
        assemble_block(g, m, &u, &L, tau, Lb, Db, Ubk);
        for (int s = 0; s < n; s++)
          for (int q = 0; q < 3; q++) {
            int fid; long idx;
            bv[s * 3 + q] = block_unknown(g, &L, s, q, &fid, &idx) ? fld(rhs, fid)[idx] : 0.0;
          }
        int rc = L.cyclic ? block_cyclic(n, 3, Lb, Db, Ubk, bv) : block_thomas(n, 3, Lb, Db, Ubk, 1, bv, C);
        if (rc) err |= 1;
        for (int s = 0; s < n; s++)
          for (int q = 0; q < 3; q++) {
            int fid; long idx;
            if (block_unknown(g, &L, s, q, &fid, &idx)) fldw(x, fid)[idx] = bv[s * 3 + q];
          }
      } else {
        assemble_scalar(g, m, &u, &L, tau, Lb, Db, Ubk);
        for (int s = 0; s < n; s++) bv[s] = fld(rhs, L.tcomp)[line_idx(g, &L, L.tcomp, s)];
        int rc = L.cyclic ? block_cyclic(n, 1, Lb, Db, Ubk, bv) : block_thomas(n, 1, Lb, Db, Ubk, 1, bv, C);
        if (rc) err |= 1;
        for (int s = 0; s < n; s++) fldw(x, L.tcomp)[line_idx(g, &L, L.tcomp, s)] = bv[s];
      }
    }
    free(Lb); free(Db); free(Ubk); free(bv); free(C);
  }
  return err ? -1 : 0;
}

/* Solve one (cyclic or not) block-tridiagonal system given its blocks
 * (for dense-LU tests of the line solvers).  b (n x bs) is overwritten. */
int orc_block_solve(int n, int bs, int cyclic, const real *L, const real *D, const real *U,
                    real *b) {
  if (cyclic) return block_cyclic(n, bs, L, D, U, b);
  real *C = malloc(sizeof(real) * (size_t)n * bs * bs);
  int rc = block_thomas(n, bs, L, D, U, 1, b, C);
  free(C);
  return rc;
}

/* Threads of the OpenMP loops in the calls that follow (for timing the oracle
 * on a given number of host cores; no effect on the results, which depend on
 * no reduction order). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
