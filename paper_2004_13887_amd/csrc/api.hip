// api.hip -- host implementation of the C-ABI declared in include/dsw.h:
// descriptor validation, metric tables, workspace and the orchestration of
// one split time step (paper section 2.2: K iterations of residual + three
// sweeps on one HIP stream; eqs. (spl1)-(spl3)).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dsw.h"
#include "dsw_common.hpp"
#include "dsw_internal.hpp"
#include "rows.hpp"

using namespace dsw;

struct dsw_grid {
  dsw_grid_desc desc;
  dsw_material mat;
  Geo geo;
  Mat m;
  Cfg cfg{64, {256, 256}, 4, {-1, -1}}; // launch shapes
  double *tables = nullptr; // rc | rf | sc | cc | sf | cf
  Fields ub{}, ub2{}, r{}, x1{}, x2{}; // ub, ub2: midpoint states of consecutive iterations
  double *fields_mem = nullptr;
  Scratch sc{};
  double *scratch_mem = nullptr;
  double *adj_mem = nullptr; // adjoint workspace, allocated on first use
  double *fwall_mem = nullptr; // forced step: mean and change of the wall data, on first use
  double *ref_mem = nullptr;   // perturbation form: reference pressure | temperature [2 nr]
  unsigned long long *cour_mem = nullptr; // Courant maxima, on first use
  int adj_states = 0;         // five-field states it holds
  // the adjoint's second stream (non-blocking, default priority), its
  // fork/join events and the sweep scratch of the work it runs
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  Scratch sc2{};
  int *status = nullptr;
  long count[5];
  int device = 0;
  // optional event timing of split_step
  int timing = 0;
  std::vector<hipEvent_t> ev_free;
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> recs;
};

static hipEvent_t take_event(dsw_grid *G) {
  if (!G->ev_free.empty()) {
    hipEvent_t e = G->ev_free.back();
    G->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// run one enqueue, bracketed by events when timing is on
template <class Fn> static void timed(dsw_grid *G, int kind, hipStream_t st, Fn fn) {
  if (!G->timing) { fn(); return; }
  hipEvent_t a = take_event(G), b = take_event(G);
  if (!a || !b) { fn(); return; }
  (void)hipEventRecord(a, st);
  fn();
  (void)hipEventRecord(b, st);
  G->recs.push_back({kind, a, b});
}

static thread_local std::string g_err = "no error";

static int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(DSW_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

extern "C" const char *dsw_last_error(void) { return g_err.c_str(); }

// ------------------------------------------- allocation-free workspace --

// Workspace of dsw_split_step_noalloc: one file-scope device array of
// DSW_NOALLOC_BYTES.  Every GPU the library runs on holds its own copy from
// the library's first use on that GPU until the process ends.  In host code
// the array's name is not a device address: each device's address comes from
// hipGetSymbolAddress, taken once per device and kept in g_noalloc.
static __device__ __align__(256) double scratch[DSW_NOALLOC_BYTES / sizeof(double)];

static constexpr int NOALLOC_MAX_DEVICES = 64;
static double *g_noalloc[NOALLOC_MAX_DEVICES];
static std::mutex g_noalloc_mu;

// device address of the array on device dev, which must be current; taken on
// the first call for that device
static int noalloc_base(int dev, double **out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(DSW_EINVAL, "device index beyond the allocation-free workspace table");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DSW_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_noalloc[dev] = static_cast<double *>(p);
  }
  *out = g_noalloc[dev];
  return DSW_OK;
}

static void counts(const dsw_grid_desc &d, long c[5]) {
  const long nr = d.n_r, nt = d.n_theta, np = d.n_phi, npf = d.periodic_phi ? np : np + 1;
  c[0] = nr * nt * np;
  c[1] = (nr + 1) * nt * np;
  c[2] = nr * (nt + 1) * np;
  c[3] = nr * nt * npf;
  c[4] = nr * nt * np;
}

static Fields carve(double *base, const long c[5], long *off) {
  Fields f;
  f.p = base + *off; *off += c[0];
  f.ur = base + *off; *off += c[1];
  f.ut = base + *off; *off += c[2];
  f.uf = base + *off; *off += c[3];
  f.T = base + *off; *off += c[4];
  return f;
}

static int validate(const dsw_grid_desc *d, const dsw_material *m) {
  if (!d || !m) return fail(DSW_EINVAL, "null descriptor");
  if (d->n_r < 3 || d->n_theta < 3 || d->n_phi < 3)
    return fail(DSW_EINVAL, "every cell count must be >= 3");
  if (!(d->r1 > 0.0 && d->r2 > d->r1)) return fail(DSW_EINVAL, "need 0 < r1 < r2");
  if (!(d->theta1 >= 0.0 && d->theta2 > d->theta1 && d->theta2 <= M_PI + 1e-12))
    return fail(DSW_EINVAL, "need 0 <= theta1 < theta2 <= pi");
  if (!(d->phi2 > d->phi1)) return fail(DSW_EINVAL, "need phi1 < phi2");
  if (d->periodic_phi && std::fabs((d->phi2 - d->phi1) - 2.0 * M_PI) > 1e-12)
    return fail(DSW_EINVAL, "periodic phi requires phi2 - phi1 = 2 pi");
  if (!(m->cp > m->cv && m->cv > 0.0)) return fail(DSW_EINVAL, "need c_p > c_v > 0");
  if (!(m->mu >= 0.0 && m->prandtl > 0.0)) return fail(DSW_EINVAL, "need mu >= 0, Pr > 0");
  const double cells = (double)d->n_r * d->n_theta * d->n_phi;
  if (cells > 2.0e9) return fail(DSW_EINVAL, "grid too large for 32-bit line counts");
  return DSW_OK;
}

extern "C" int dsw_init_grid(const dsw_grid_desc *desc, const dsw_material *mat, dsw_grid **out) {
  if (!out) return fail(DSW_EINVAL, "null output handle");
  *out = nullptr;
  const int vrc = validate(desc, mat);
  if (vrc) return vrc;
  dsw_grid *G = new dsw_grid();
  G->desc = *desc;
  G->mat = *mat;
  HIPCHK(hipGetDevice(&G->device));
  {
    double *base = nullptr;  // the allocation-free workspace of this device
    const int src = noalloc_base(G->device, &base);
    if (src) {
      delete G;
      return src;
    }
  }
  const int nr = desc->n_r, nt = desc->n_theta, np = desc->n_phi;
  // metric tables (host, then device)
  const size_t nt1 = (size_t)nt + 1, nr1 = (size_t)nr + 1;
  std::vector<double> h(2 * (nr + nr1) + 4 * (nt + nt1) + (nt + 2));
  double *rc = h.data(), *rf = rc + nr, *sc = rf + nr1, *cc = sc + nt, *sf = cc + nt, *cf = sf + nt1;
  double *irc = cf + nt1, *irf = irc + nr, *isc = irf + nr1, *ctc = isc + nt, *isf = ctc + nt,
         *ctf = isf + nt1, *scx = ctf + nt1;
  const double dr = (desc->r2 - desc->r1) / nr, dt = (desc->theta2 - desc->theta1) / nt,
               dp = (desc->phi2 - desc->phi1) / np;
  for (int i = 0; i < nr; i++) rc[i] = desc->r1 + (i + 0.5) * dr;
  for (int f = 0; f <= nr; f++) rf[f] = desc->r1 + f * dr;
  for (int j = 0; j < nt; j++) {
    const double th = desc->theta1 + (j + 0.5) * dt;
    sc[j] = std::sin(th);
    cc[j] = std::cos(th);
  }
  for (int f = 0; f <= nt; f++) {
    const double th = desc->theta1 + f * dt;
    sf[f] = std::sin(th);
    cf[f] = std::cos(th);
  }
  for (int j = -1; j <= nt; j++) scx[j + 1] = std::sin(desc->theta1 + (j + 0.5) * dt);
  const int pole_lo = desc->theta1 == 0.0, pole_hi = std::fabs(desc->theta2 - M_PI) <= 1e-12;
  if (pole_lo) { sf[0] = 0.0; cf[0] = 1.0; }
  if (pole_hi) { sf[nt] = 0.0; cf[nt] = -1.0; }
  for (int i = 0; i < nr; i++) irc[i] = 1.0 / rc[i];
  for (int f = 0; f <= nr; f++) irf[f] = 1.0 / rf[f];
  for (int j = 0; j < nt; j++) { isc[j] = 1.0 / sc[j]; ctc[j] = cc[j] / sc[j]; }
  for (int f = 0; f <= nt; f++) {
    isf[f] = sf[f] != 0.0 ? 1.0 / sf[f] : 0.0;
    ctf[f] = sf[f] != 0.0 ? cf[f] / sf[f] : 0.0;
  }
  if (hipMalloc(&G->tables, h.size() * sizeof(double)) != hipSuccess) {
    delete G;
    return fail(DSW_ENOMEM, "metric tables");
  }
  HIPCHK(hipMemcpy(G->tables, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  Geo &g = G->geo;
  g.nr = nr; g.nt = nt; g.np = np; g.npf = desc->periodic_phi ? np : np + 1;
  g.periodic = desc->periodic_phi ? 1 : 0;
  g.pole_lo = pole_lo; g.pole_hi = pole_hi;
  g.dr = dr; g.dt = dt; g.dp = dp;
  g.idr = 1.0 / dr; g.idt = 1.0 / dt; g.idp = 1.0 / dp;
  double *t = G->tables;
  const long o_rf = nr, o_sc = o_rf + nr1, o_cc = o_sc + nt, o_sf = o_cc + nt, o_cf = o_sf + nt1,
             o_irc = o_cf + nt1, o_irf = o_irc + nr, o_isc = o_irf + nr1, o_ctc = o_isc + nt,
             o_isf = o_ctc + nt, o_ctf = o_isf + nt1, o_scx = o_ctf + nt1;
  g.rc = t; g.rf = t + o_rf; g.sc = t + o_sc; g.cc = t + o_cc; g.sf = t + o_sf; g.cf = t + o_cf;
  g.irc = t + o_irc; g.irf = t + o_irf; g.isc = t + o_isc; g.ctc = t + o_ctc; g.isf = t + o_isf;
  g.ctf = t + o_ctf;
  g.scx = t + o_scx;
  Mat &m = G->m;
  m.gam = mat->cp / mat->cv;
  m.Rg = mat->cp - mat->cv;
  m.pinf = mat->pi_inf;
  m.mu = mat->mu;
  m.kap = mat->mu * mat->cp / mat->prandtl;
  m.omega = mat->omega;
  m.g_r = mat->g_r;
  // workspace: Ubar, R, X1, X2 and the sweep scratch
  counts(*desc, G->count);
  const long per = G->count[0] + G->count[1] + G->count[2] + G->count[3] + G->count[4];
  if (hipMalloc(&G->fields_mem, 5 * per * sizeof(double)) != hipSuccess) {
    dsw_free_grid(G);
    return fail(DSW_ENOMEM, "workspace fields");
  }
  long off = 0;
  G->ub = carve(G->fields_mem, G->count, &off);
  G->ub2 = carve(G->fields_mem, G->count, &off);
  G->r = carve(G->fields_mem, G->count, &off);
  G->x1 = carve(G->fields_mem, G->count, &off);
  G->x2 = carve(G->fields_mem, G->count, &off);
  long sb, ss;
  sweep_scratch_size(g, &sb, &ss);
  if (hipMalloc(&G->scratch_mem, (sb + ss) * sizeof(double)) != hipSuccess) {
    dsw_free_grid(G);
    return fail(DSW_ENOMEM, "sweep scratch");
  }
  G->sc.blk = G->scratch_mem;
  G->sc.sca = G->scratch_mem + sb;
  G->sc.blk_len = sb;
  G->sc.sca_len = ss;
  if (hipMalloc(&G->status, ST_WORDS * sizeof(int)) != hipSuccess) {
    dsw_free_grid(G);
    return fail(DSW_ENOMEM, "status word");
  }
  HIPCHK(hipMemset(G->status, 0, ST_WORDS * sizeof(int)));
  HIPCHK(hipMemset(G->fields_mem, 0, 5 * per * sizeof(double)));
  *out = G;
  return DSW_OK;
}

extern "C" int dsw_free_grid(dsw_grid *G) {
  if (!G) return DSW_OK;
  (void)hipDeviceSynchronize();
  for (auto &r : G->recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (auto e : G->ev_free) (void)hipEventDestroy(e);
  if (G->tables) (void)hipFree(G->tables);
  if (G->fields_mem) (void)hipFree(G->fields_mem);
  if (G->scratch_mem) (void)hipFree(G->scratch_mem);
  if (G->adj_mem) (void)hipFree(G->adj_mem);
  if (G->fwall_mem) (void)hipFree(G->fwall_mem);
  if (G->ref_mem) (void)hipFree(G->ref_mem);
  if (G->cour_mem) (void)hipFree(G->cour_mem);
  if (G->side) (void)hipStreamDestroy(G->side);
  if (G->fork_ev) (void)hipEventDestroy(G->fork_ev);
  if (G->join_ev) (void)hipEventDestroy(G->join_ev);
  if (G->status) (void)hipFree(G->status);
  delete G;
  return DSW_OK;
}

extern "C" int dsw_layout(const dsw_grid *G, dsw_layout_info *info) {
  if (!G || !info) return fail(DSW_EINVAL, "null argument");
  const dsw_grid_desc &d = G->desc;
  const long nr = d.n_r, nt = d.n_theta, np = d.n_phi, npf = d.periodic_phi ? np : np + 1;
  const int64_t sh[5][3] = {{nr, nt, np}, {nr + 1, nt, np}, {nr, nt + 1, np}, {nr, nt, npf}, {nr, nt, np}};
  info->bytes_per_state = 0;
  for (int q = 0; q < 5; q++) {
    for (int a = 0; a < 3; a++) info->shape[q][a] = sh[q][a];
    info->count[q] = G->count[q];
    info->bytes_per_state += G->count[q] * (int64_t)sizeof(double);
  }
  return DSW_OK;
}

static int check_fields(const dsw_fields *f, const char *name) {
  if (!f || !f->p || !f->ur || !f->ut || !f->uf || !f->T)
    return fail(DSW_EINVAL, std::string("null field pointer in ") + name);
  return DSW_OK;
}

static Fields F(const dsw_fields *f) {
  Fields x;
  x.p = f->p; x.ur = f->ur; x.ut = f->ut; x.uf = f->uf; x.T = f->T;
  return x;
}

static int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DSW_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return DSW_OK;
}

extern "C" int dsw_residual(dsw_grid *G, const dsw_fields *Un, const dsw_fields *Uk, double tau,
                            dsw_fields *R, dsw_fields *Ubar, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  int rc;
  if ((rc = check_fields(Un, "Un")) || (rc = check_fields(Uk, "Uk")) || (rc = check_fields(R, "R")) ||
      (rc = check_fields(Ubar, "Ubar")))
    return rc;
  if (!(tau > 0.0)) return fail(DSW_EINVAL, "tau must be > 0");
  launch_residual(G->geo, G->m, F(Un), F(Uk), tau, F(R), F(Ubar), G->status, (hipStream_t)stream);
  return check_launch("residual kernel");
}

// ------------------------------------------------------------- passes --

static SrcOne src1(const Fields &f) {
  SrcOne u;
  u.a[F_P] = f.p; u.a[F_UR] = f.ur; u.a[F_UT] = f.ut; u.a[F_UF] = f.uf; u.a[F_T] = f.T;
  return u;
}

static Diff diff(const Fields &n, const Fields &k) {
  Diff d;
  const double *nn[5] = {n.p, n.ur, n.ut, n.uf, n.T}, *kk[5] = {k.p, k.ur, k.ut, k.uf, k.T};
  for (int q = 0; q < 5; q++) { d.n[q] = nn[q]; d.k[q] = kk[q]; }
  d.same = (n.p == k.p) ? 1 : 0;
  return d;
}

static PassArgs base_args(const dsw_grid *G) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.g = G->geo;
  a.m = G->m;
  a.scb = G->sc.blk;
  a.scs = G->sc.sca;
  a.status = G->status;
  return a;
}

// one pass of a plan: kernel kind, timing kind, arguments
struct Pass {
  int kind, tk;
  PassArgs a;
};

// the kind of an r (d = 0) or theta (d = 1) pass under a configuration
static int rt_kind(const Geo &g, const Cfg &c, int d) {
  const int pm = c.rt_pm[d] < 0 ? rt_default_pm(g, d) : c.rt_pm[d];  // -1: by line length
  if (pm > 0 && rt_part_supported(g, d, (unsigned)c.sweep_bs[d], pm)) return d == 0 ? PK_SW0P : PK_SW1P;
  const bool tw = families(g, d).nb < TWIST_LINES;
  return d == 0 ? (tw ? PK_SW0T : PK_SW0) : (tw ? PK_SW1T : PK_SW1);
}

static Pass sweep_pass(const dsw_grid *G, int d, const Fields &ubar, double tau, const Fields &rhs,
                       const Out &o) {
  Pass p;
  if (d == 2) p.kind = phi_kind(G->geo, G->cfg);
  else p.kind = rt_kind(G->geo, G->cfg, d);
  p.tk = 1 + d;
  p.a = base_args(G);
  p.a.u = src1(ubar);
  p.a.tau = 0.5 * tau;
  p.a.rhs = rhs;
  p.a.o = o;
  return p;
}

// A two-ended r or theta pass as the passes that run it: where the
// partitioned scalar-line solver takes the grid, the block lines two-ended
// and then the scalar lines partitioned (which need no scratch), else the
// pass itself.  Every plain sweep goes through here, so a grid's step, its
// taped step, its line solves and an ensemble's batched launches all solve
// the scalar lines the same way.  pad: every r and theta sweep gives two
// passes, the second one PK_NONE where it has no scalar pass (an ensemble's
// launch plan takes pass q of every member together).
template <class Emit>
static void emit_sweep(const dsw_grid *G, const Pass &p, Emit emit, bool pad = false) {
  const int d = p.kind == PK_SW0T ? 0 : (p.kind == PK_SW1T ? 1 : -1);
  Pass q = p;
  if (d < 0 || !rt_scalar_supported(G->geo, d, (unsigned)G->cfg.sweep_bs[d])) {
    emit(p);
    if (pad && p.tk >= 1 && p.tk <= 2) {
      q.kind = PK_NONE;
      emit(q);
    }
    return;
  }
  q.kind = d == 0 ? PK_SW0B : PK_SW1B;
  emit(q);
  q.kind = d == 0 ? PK_SW0S : PK_SW1S;
  emit(q);
}

// The workspace of one split step: the midpoint states of consecutive
// iterations, the residual, the outputs of the r and theta sweeps, and the
// sweep scratch.
struct Work {
  Fields ub, ub2, r, x1, x2;
  Scratch sc;
};

static Work own_work(const dsw_grid *G) { return Work{G->ub, G->ub2, G->r, G->x1, G->x2, G->sc}; }

// the passes of one split step, in stream order (paper section 2.2: K
// iterations of eqs. (spl1)-(spl3) after the residual), on workspace W;
// emit(const Pass &) receives each pass in turn
template <class Emit>
static void plan_step(const dsw_grid *G, const Work &W, const Fields &un, const Fields &uk, double tau,
                      int K, Emit emit) {
  const Fields none{};
  {
    // Dirichlet data of U^{n+1} and of both midpoint buffers = those of U^n
    Pass p{PK_BND, 4, base_args(G)};
    p.a.src = un; p.a.d0 = uk; p.a.d1 = W.ub; p.a.d2 = W.ub2;
    emit(p);
  }
  const Fields ubuf[2] = {W.ub, W.ub2};
  auto sweep = [&](int d, const Fields &ubar, const Fields &rhs, const Out &o) {
    Pass p = sweep_pass(G, d, ubar, tau, rhs, o);
    p.a.scb = W.sc.blk;
    p.a.scs = W.sc.sca;
    emit_sweep(G, p, emit, true);
  };
  for (int it = 0; it < K; it++) {
    // midpoint state of this iteration: U^n itself at the first one, else the
    // one written by the previous iteration's phi sweep
    const Fields ubar = it == 0 ? un : ubuf[(it - 1) % 2];
    Pass r{G->geo.periodic ? PK_RES_INP : PK_RES_IN, 0, base_args(G)};
    r.a.u = src1(ubar);
    r.a.d = diff(un, it == 0 ? un : uk);
    r.a.tau = tau;
    r.a.R = W.r;
    emit(r);  // interior workgroups
    r.kind = PK_RES;
    emit(r);  // the rest
    Out o1{}, o2{}, o3{};
    o1.x = W.x1; o1.mode = 0;
    o2.x = W.x2; o2.mode = 0;
    o3.x = uk; o3.base = it == 0 ? un : uk; o3.un = un;
    o3.ub = it < K - 1 ? ubuf[it % 2] : none;
    o3.mode = 1;
    sweep(0, ubar, W.r, o1);
    sweep(1, ubar, W.x1, o2);
    sweep(2, ubar, W.x2, o3);
  }
}

static unsigned kind_threads(int kind, const Geo &g, const Cfg &c) {
  switch (kind) {
  case PK_RES:
  case PK_RES_IN:
  case PK_RES_INP: return (unsigned)c.res_bs;
  case PK_SW0:
  case PK_SW0T:
  case PK_SW0B:
  case PK_SW0S:
  case PK_SW0P: return (unsigned)c.sweep_bs[0];
  case PK_SW1:
  case PK_SW1T:
  case PK_SW1B:
  case PK_SW1S:
  case PK_SW1P: return (unsigned)c.sweep_bs[1];
  case PK_SW2_PART:
  case PK_SW2_CP:
  case PK_SW2_CN: return phi_part_threads(g, c.phi_pm);
  default: return 128u; // boundary copy, thread-per-line phi
  }
}

static unsigned cdiv(unsigned long a, unsigned b) { return (unsigned)((a + b - 1) / b); }

static unsigned kind_blocks(int kind, const Geo &g, const Cfg &c, unsigned threads) {
  switch (kind) {
  case PK_BND: return cdiv(bnd_points(g), threads);
  case PK_RES: return residual_general_blocks(g, (int)threads);
  case PK_RES_IN:
  case PK_RES_INP: return residual_interior_blocks(g, (int)threads);
  case PK_SW0: return cdiv(sweep_lines(g, 0), threads);
  case PK_SW1: return cdiv(sweep_lines(g, 1), threads);
  case PK_SW0T: return sweep2_blocks(g, 0, threads);
  case PK_SW1T: return sweep2_blocks(g, 1, threads);
  case PK_SW0B: return sweep2_block_blocks(g, 0, threads);
  case PK_SW1B: return sweep2_block_blocks(g, 1, threads);
  case PK_SW0S: return rt_scalar_blocks(g, 0, threads);
  case PK_SW1S: return rt_scalar_blocks(g, 1, threads);
  case PK_SW0P: return rt_part_blocks(g, 0, threads, 4);
  case PK_SW1P: return rt_part_blocks(g, 1, threads, 4);
  case PK_SW2_LINE: return cdiv(sweep_lines(g, 2), threads);
  default: return (unsigned)g.nr * (unsigned)g.nt; // PK_SW2_PART
  }
}

static size_t kind_lds(int kind, const Geo &g, const Cfg &c) {
  if (kind == PK_SW0P || kind == PK_SW1P) return rt_part_lds(kind_threads(kind, g, c));
  if (kind == PK_SW0S || kind == PK_SW1S) return rt_scalar_lds(kind_threads(kind, g, c));
  return (kind == PK_SW2_PART || kind == PK_SW2_CP || kind == PK_SW2_CN) ? phi_part_lds(g, c.phi_pm) : 0;
}

static void launch_kind(int kind, const Cfg &c, const PassArgs &a, const Batch &b, unsigned blocks,
                        unsigned threads, size_t lds, hipStream_t st) {
  switch (kind) {
  case PK_BND: launch_bnd_pass(a, b, blocks, threads, st); break;
  case PK_RES: launch_residual_pass(a, b, blocks, threads, st); break;
  case PK_RES_IN: launch_residual_in_pass(false, a, b, blocks, threads, st); break;
  case PK_RES_INP: launch_residual_in_pass(true, a, b, blocks, threads, st); break;
  case PK_SW0: launch_sweep_pass(0, a, b, blocks, threads, st); break;
  case PK_SW1: launch_sweep_pass(1, a, b, blocks, threads, st); break;
  case PK_SW0T:
  case PK_SW0B: launch_sweep2_pass(0, a, b, blocks, threads, st); break;
  case PK_SW1T:
  case PK_SW1B: launch_sweep2_pass(1, a, b, blocks, threads, st); break;
  case PK_SW0S: launch_rt_scalar_pass(0, a, b, blocks, threads, st); break;
  case PK_SW1S: launch_rt_scalar_pass(1, a, b, blocks, threads, st); break;
  case PK_SW0P: launch_rt_pass(0, 4, a, b, blocks, threads, st); break;
  case PK_SW1P: launch_rt_pass(1, 4, a, b, blocks, threads, st); break;
  case PK_SW2_LINE: launch_sweep_pass(2, a, b, blocks, threads, st); break;
  case PK_SW2_CP: launch_phi_pass_c(c.phi_pm, true, a, b, blocks, threads, lds, st); break;
  case PK_SW2_CN: launch_phi_pass_c(c.phi_pm, false, a, b, blocks, threads, lds, st); break;
  default: launch_phi_pass(c.phi_pm, a, b, blocks, threads, lds, st); break;
  }
}

// one pass on one grid, arguments by value
static void launch_single(const dsw_grid *G, const Pass &p, hipStream_t st) {
  if (p.kind == PK_NONE) return;
  const unsigned th = kind_threads(p.kind, G->geo, G->cfg);
  const unsigned nb = kind_blocks(p.kind, G->geo, G->cfg, th);
  if (nb == 0) return;  // e.g. no interior workgroups on a tiny grid
  const Batch none{nullptr, nullptr, 0};
  launch_kind(p.kind, G->cfg, p.a, none, nb, th, kind_lds(p.kind, G->geo, G->cfg), st);
}

static int line_solve(int d, dsw_grid *G, const dsw_fields *Ubar, double tau, const dsw_fields *rhs,
                      dsw_fields *x, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  int rc;
  if ((rc = check_fields(Ubar, "Ubar")) || (rc = check_fields(rhs, "rhs")) || (rc = check_fields(x, "x")))
    return rc;
  if (!(tau > 0.0)) return fail(DSW_EINVAL, "tau must be > 0");
  if (rhs->p == x->p || rhs->ur == x->ur || rhs->ut == x->ut || rhs->uf == x->uf || rhs->T == x->T)
    return fail(DSW_EINVAL, "rhs and x must not alias");
  Out o{};
  o.x = F(x);
  o.mode = 0;
  emit_sweep(G, sweep_pass(G, d, F(Ubar), tau, F(rhs), o),
             [&](const Pass &q) { launch_single(G, q, (hipStream_t)stream); });
  return check_launch("sweep kernel");
}

extern "C" int dsw_line_solve_r(dsw_grid *G, const dsw_fields *Ubar, double tau, const dsw_fields *rhs,
                                dsw_fields *x, void *stream) {
  return line_solve(0, G, Ubar, tau, rhs, x, stream);
}
extern "C" int dsw_line_solve_theta(dsw_grid *G, const dsw_fields *Ubar, double tau,
                                    const dsw_fields *rhs, dsw_fields *x, void *stream) {
  return line_solve(1, G, Ubar, tau, rhs, x, stream);
}
extern "C" int dsw_line_solve_phi(dsw_grid *G, const dsw_fields *Ubar, double tau, const dsw_fields *rhs,
                                  dsw_fields *x, void *stream) {
  return line_solve(2, G, Ubar, tau, rhs, x, stream);
}

static int check_step_args(const dsw_fields *Un, const dsw_fields *Unp1, double tau, int32_t K) {
  int rc;
  if ((rc = check_fields(Un, "Un")) || (rc = check_fields(Unp1, "Unp1"))) return rc;
  if (!(tau > 0.0)) return fail(DSW_EINVAL, "tau must be > 0");
  if (K < 1) return fail(DSW_EINVAL, "K must be >= 1");
  if (Un->p == Unp1->p || Un->ur == Unp1->ur || Un->ut == Unp1->ut || Un->uf == Unp1->uf ||
      Un->T == Unp1->T)
    return fail(DSW_EINVAL, "Unp1 must not alias Un");
  return DSW_OK;
}

extern "C" int dsw_split_step(dsw_grid *G, const dsw_fields *Un, dsw_fields *Unp1, double tau,
                              int32_t K, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  const int rc = check_step_args(Un, Unp1, tau, K);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  std::vector<Pass> plan;
  plan_step(G, own_work(G), F(Un), F(Unp1), tau, K, [&](const Pass &p) { plan.push_back(p); });
  // the launches of one pass (the residual's interior and boundary
  // launches, a sweep's block and scalar lines) are timed together
  for (size_t q = 0; q < plan.size();) {
    if (plan[q].kind == PK_NONE) {
      q++;
      continue;
    }
    size_t e = q + 1;
    while (e < plan.size() && plan[e].tk == plan[q].tk && plan[e].kind != plan[q].kind &&
           (plan[q].kind == PK_RES_IN || plan[q].kind == PK_RES_INP || plan[q].kind == PK_SW0B ||
            plan[q].kind == PK_SW1B))
      e++;
    timed(G, plan[q].tk, st, [&] {
      for (size_t r = q; r < e; r++) launch_single(G, plan[r], st);
    });
    q = e;
  }
  return check_launch("split step kernels");
}

extern "C" int dsw_set_reference(dsw_grid *G, const double *p_ref, const double *T_ref) {
  if (!G || !p_ref || !T_ref) return fail(DSW_EINVAL, "null argument");
  const int nr = G->geo.nr;
  for (int i = 0; i < nr; i++) {
    if (!std::isfinite(p_ref[i]) || !(T_ref[i] > 0.0) || !std::isfinite(T_ref[i]) ||
        !(p_ref[i] + G->m.pinf > 0.0))
      return fail(DSW_EINVAL, "reference column: p_ref + pi_inf and T_ref must be positive and finite (row " +
                                  std::to_string(i) + ")");
  }
  if (!G->ref_mem && hipMalloc(&G->ref_mem, 2 * (size_t)nr * sizeof(double)) != hipSuccess) {
    G->ref_mem = nullptr;
    return fail(DSW_ENOMEM, "reference column");
  }
  HIPCHK(hipMemcpy(G->ref_mem, p_ref, nr * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(G->ref_mem + nr, T_ref, nr * sizeof(double), hipMemcpyHostToDevice));
  return DSW_OK;
}

extern "C" int dsw_split_step_pert(dsw_grid *G, const dsw_fields *Un, dsw_fields *Unp1, double tau,
                                   int32_t K, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  const int rc = check_step_args(Un, Unp1, tau, K);
  if (rc) return rc;
  if (!G->ref_mem) return fail(DSW_EINVAL, "perturbation step: no reference column (dsw_set_reference)");
  const Geo &g = G->geo;
  std::vector<Pass> plan;
  plan_step(G, own_work(G), F(Un), F(Unp1), tau, K, [&](const Pass &p) { plan.push_back(p); });
  for (const Pass &p : plan)  // the kernel kinds with a perturbation-form variant
    if (p.kind == PK_SW0 || p.kind == PK_SW1 || p.kind == PK_SW2_LINE)
      return fail(DSW_EINVAL, "perturbation step: the grid's lines need the thread-per-line solver, "
                              "which has no perturbation form");
  hipStream_t st = (hipStream_t)stream;
  for (const Pass &p : plan) {
    if (p.kind == PK_RES_IN || p.kind == PK_RES_INP) continue;  // inside the PK_RES launch below
    if (p.kind == PK_SW0S || p.kind == PK_SW1S || p.kind == PK_NONE) continue;  // inside the two-ended launch below
    PassArgs a = p.a;
    a.pref = G->ref_mem;
    a.tref = G->ref_mem + g.nr;
    timed(G, p.tk, st, [&] {
      const unsigned th = kind_threads(p.kind, g, G->cfg);
      switch (p.kind) {
      case PK_BND: launch_single(G, p, st); break;
      case PK_RES: launch_residual_pert(a, kind_blocks(PK_RES, g, G->cfg, th), th, st); break;
      case PK_SW0P: launch_rt_pert(0, a, th, st); break;
      case PK_SW1P: launch_rt_pert(1, a, th, st); break;
      case PK_SW0T:
      case PK_SW0B: launch_sweep2_pert(0, a, sweep2_blocks(g, 0, th), th, st); break;
      case PK_SW1T:
      case PK_SW1B: launch_sweep2_pert(1, a, sweep2_blocks(g, 1, th), th, st); break;
      default:  // PK_SW2_PART
        launch_phi_pert(G->cfg.phi_pm, a, kind_blocks(p.kind, g, G->cfg, th), th, kind_lds(p.kind, g, G->cfg), st);
      }
    });
  }
  return check_launch("perturbation split step kernels");
}

extern "C" int dsw_courant(dsw_grid *G, const dsw_fields *U, double tau, double out[2], void *stream) {
  if (!G || !out) return fail(DSW_EINVAL, "null argument");
  int rc;
  if ((rc = check_fields(U, "U"))) return rc;
  if (!(tau > 0.0)) return fail(DSW_EINVAL, "tau must be > 0");
  if (!G->cour_mem && hipMalloc(&G->cour_mem, 2 * sizeof(unsigned long long)) != hipSuccess) {
    G->cour_mem = nullptr;
    return fail(DSW_ENOMEM, "Courant maxima");
  }
  hipStream_t st = (hipStream_t)stream;
  launch_courant(G->geo, G->m, F(U), tau, G->cour_mem, st);
  unsigned long long h[2];
  HIPCHK(hipMemcpyAsync(h, G->cour_mem, sizeof(h), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(out, h, sizeof(h));
  return check_launch("Courant kernel");
}

// the workspace of one split step carved from the allocation-free array
static int noalloc_work(const dsw_grid *G, double *base, Work *W) {
  const long per = G->count[0] + G->count[1] + G->count[2] + G->count[3] + G->count[4];
  long sb, ss;
  sweep_scratch_size(G->geo, &sb, &ss);
  const long need = 5 * per + sb + ss;
  if ((unsigned long long)need * sizeof(double) > (unsigned long long)DSW_NOALLOC_BYTES)
    return fail(DSW_EINVAL, "allocation-free split step: the grid needs " +
                                std::to_string((unsigned long long)need * sizeof(double)) +
                                " bytes of workspace, more than DSW_NOALLOC_BYTES = " +
                                std::to_string((unsigned long long)DSW_NOALLOC_BYTES));
  long off = 0;
  W->ub = carve(base, G->count, &off);
  W->ub2 = carve(base, G->count, &off);
  W->r = carve(base, G->count, &off);
  W->x1 = carve(base, G->count, &off);
  W->x2 = carve(base, G->count, &off);
  W->sc.blk = base + off;
  W->sc.sca = base + off + sb;
  W->sc.blk_len = sb;
  W->sc.sca_len = ss;
  return DSW_OK;
}

extern "C" int dsw_split_step_noalloc(dsw_grid *G, const dsw_fields *Un, dsw_fields *Unp1, double tau,
                                      int32_t K, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  int rc = check_step_args(Un, Unp1, tau, K);
  if (rc) return rc;
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != G->device) return fail(DSW_EINVAL, "allocation-free split step: the handle's device is not current");
  double *base = nullptr;
  if ((rc = noalloc_base(dev, &base))) return rc;
  Work W;
  if ((rc = noalloc_work(G, base, &W))) return rc;
  // every buffer of W is written before it is read within the step, so no
  // part of the array needs clearing; passes launch as they are planned
  hipStream_t st = (hipStream_t)stream;
  plan_step(G, W, F(Un), F(Unp1), tau, K, [&](const Pass &p) { launch_single(G, p, st); });
  return check_launch("allocation-free split step kernels");
}

// lengths of the twelve wall arrays, in the order of dsw_wall
static void wall_lens(const Geo &g, long len[12]) {
  const long a = (long)(g.nr + 1) * g.np, b = (long)(g.nr + 1) * g.nt, c = (long)(g.nt + 1) * g.np,
             d = (long)g.nr * (g.nt + 1), e = (long)g.nt * g.npf, f = (long)g.nr * g.npf;
  const long l[12] = {a, a, b, b, c, c, d, d, e, e, f, f};
  for (int q = 0; q < 12; q++) len[q] = l[q];
}

static const double *wall_ptr(const dsw_wall *w, int q) {
  if (!w) return nullptr;
  const double *const a[12] = {w->ur_t1, w->ur_t2, w->ur_p1, w->ur_p2, w->ut_r1, w->ut_r2,
                               w->ut_p1, w->ut_p2, w->uf_r1, w->uf_r2, w->uf_t1, w->uf_t2};
  return a[q];
}

static Wall wall_of(double *const p[12]) {
  Wall o;
  o.ur_t1 = p[0]; o.ur_t2 = p[1]; o.ur_p1 = p[2]; o.ur_p2 = p[3];
  o.ut_r1 = p[4]; o.ut_r2 = p[5]; o.ut_p1 = p[6]; o.ut_p2 = p[7];
  o.uf_r1 = p[8]; o.uf_r2 = p[9]; o.uf_t1 = p[10]; o.uf_t2 = p[11];
  return o;
}

extern "C" int dsw_split_step_forced(dsw_grid *G, const dsw_fields *Un, dsw_fields *Unp1, double tau,
                                     int32_t K, const dsw_fields *src, const dsw_wall *wall0,
                                     const dsw_wall *wall1, const dsw_fields *bnd, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  int rc = check_step_args(Un, Unp1, tau, K);
  if (rc) return rc;
  if (bnd && (!bnd->ur || !bnd->ut || !bnd->uf)) return fail(DSW_EINVAL, "bnd needs ur, ut and uf");
  const Geo &g = G->geo;
  int pm = G->cfg.phi_pm;
  if (!(pm > 0 && phi_part_supported(g, pm))) pm = phi_part_supported(g, 4) ? 4 : (phi_part_supported(g, 2) ? 2 : 0);
  if (!pm) return fail(DSW_EINVAL, "forced step: the phi lines do not fit the partitioned solver");
  if (families(g, 0).nb >= TWIST_LINES || families(g, 1).nb >= TWIST_LINES)
    return fail(DSW_EINVAL, "forced step: too many r or theta lines");
  hipStream_t st = (hipStream_t)stream;
  const Fields un = F(Un), uk = F(Unp1), none{};
  // wall data: w0 at t^n (the first iteration's), the mean of w0 and w1 (the
  // later iterations'), and their change (the first iteration's lifted data)
  long len[12], off[13];
  wall_lens(g, len);
  off[0] = 0;
  for (int q = 0; q < 12; q++) off[q + 1] = off[q] + len[q];
  if (!G->fwall_mem && hipMalloc(&G->fwall_mem, 2 * off[12] * sizeof(double)) != hipSuccess)
    return fail(DSW_ENOMEM, "forced step: wall workspace");
  WallMix wm;
  for (int q = 0; q < 12; q++) {
    wm.a[q] = wall_ptr(wall0, q);
    wm.b[q] = wall_ptr(wall1, q);
    wm.mid[q] = G->fwall_mem + off[q];
    wm.dw[q] = G->fwall_mem + off[12] + off[q];
  }
  for (int q = 0; q < 13; q++) wm.off[q] = off[q];
  launch_wall_mix(wm, st);
  Wall w0{};
  {
    double *p0[12];
    for (int q = 0; q < 12; q++) p0[q] = const_cast<double *>(wall_ptr(wall0, q));
    w0 = wall_of(p0);
  }
  const Wall wmid = wall_of(wm.mid), dw = wall_of(wm.dw);
  // U^{n+1,0} = U^n in Unp1, boundary faces included
  const double *unf[5] = {un.p, un.ur, un.ut, un.uf, un.T};
  double *u1[5] = {uk.p, uk.ur, uk.ut, uk.uf, uk.T};
  for (int q = 0; q < 5; q++)
    HIPCHK(hipMemcpyAsync(u1[q], unf[q], sizeof(double) * (size_t)G->count[q], hipMemcpyDeviceToDevice, st));
  const Fields ubuf[2] = {G->ub, G->ub2};
  const unsigned rbs = (unsigned)G->cfg.res_bs;
  for (int it = 0; it < K; it++) {
    // the first iteration's midpoint is U^n itself (old data, wall w0)
    const Fields ubar = it == 0 ? un : ubuf[(it - 1) % 2];
    const Wall w = it == 0 ? w0 : wmid;
    PassArgs r = base_args(G);
    r.u = src1(ubar);
    r.d = diff(un, it == 0 ? un : uk);
    r.tau = tau;
    r.R = G->r;
    r.wall = w;
    if (src) r.fsrc = F(src);
    launch_residual_forced(r, residual_general_blocks(g, (int)rbs), rbs, st);
    Out o1{}, o2{}, o3{};
    o1.x = G->x1; o1.mode = 0;
    o2.x = G->x2; o2.mode = 0;
    o3.x = uk; o3.base = uk; o3.un = un;
    o3.ub = it < K - 1 ? ubuf[it % 2] : none;
    o3.mode = 1;
    const Fields rhs_of[3] = {G->r, G->x1, G->x2};
    for (int d = 0; d < 3; d++) {
      Pass p = sweep_pass(G, d, ubar, tau, rhs_of[d], d == 0 ? o1 : (d == 1 ? o2 : o3));
      p.a.wall = w;
      if (it == 0) {  // the change of the boundary data, lifted out of the increment
        PassArgs l = p.a;
        l.src = un;
        l.d0 = bnd ? F(bnd) : none;
        launch_lift(d, l, dw, st);
      }
      if (d < 2) {
        const unsigned bs = (unsigned)G->cfg.sweep_bs[d];
        if (rt_kind(g, G->cfg, d) == (d == 0 ? PK_SW0P : PK_SW1P)) launch_rt_forced(d, 4, p.a, bs, st);
        else launch_sweep2_forced(d, p.a, sweep2_blocks(g, d, bs), bs, st);
      } else {
        launch_phi_forced(pm, p.a, (unsigned)g.nr * (unsigned)g.nt, phi_part_threads(g, pm), phi_part_lds(g, pm), st);
      }
    }
    if (it == 0) {
      // from here on U^{n+1,k} holds the new Dirichlet data and the midpoint
      // buffers their mean with U^n's
      PassArgs a = base_args(G);
      a.src = un;
      a.rhs = bnd ? F(bnd) : none;
      a.d0 = uk; a.d1 = G->ub; a.d2 = G->ub2;
      launch_bnd_forced(a, cdiv(bnd_points(g), 128), 128, st);
    }
  }
  return check_launch("forced split step kernels");
}

static int check_cfg(const dsw_config *c) {
  if (!c) return fail(DSW_EINVAL, "null config");
  auto bs_ok = [](int v) { return v == 64 || v == 128 || v == 256; };
  if (!bs_ok(c->residual_block) || !bs_ok(c->sweep_block_r) || !bs_ok(c->sweep_block_theta))
    return fail(DSW_EINVAL, "block sizes must be 64, 128 or 256");
  if (c->phi_rows_per_thread != 0 && c->phi_rows_per_thread != 2 && c->phi_rows_per_thread != 4)
    return fail(DSW_EINVAL, "phi_rows_per_thread must be 0, 2 or 4");
  auto rt_ok = [](int v) { return v == -1 || v == 0 || v == 4; };
  if (!rt_ok(c->rows_per_thread_r) || !rt_ok(c->rows_per_thread_theta))
    return fail(DSW_EINVAL, "rows_per_thread_r and rows_per_thread_theta must be -1, 0 or 4");
  return DSW_OK;
}

static Cfg to_cfg(const dsw_config *c) {
  return Cfg{c->residual_block, {c->sweep_block_r, c->sweep_block_theta}, c->phi_rows_per_thread,
             {c->rows_per_thread_r, c->rows_per_thread_theta}};
}

static dsw_config from_cfg(const Cfg &c) {
  dsw_config o;
  o.residual_block = c.res_bs;
  o.sweep_block_r = c.sweep_bs[0];
  o.sweep_block_theta = c.sweep_bs[1];
  o.phi_rows_per_thread = c.phi_pm;
  o.rows_per_thread_r = c.rt_pm[0];
  o.rows_per_thread_theta = c.rt_pm[1];
  return o;
}

extern "C" int dsw_set_config(dsw_grid *G, const dsw_config *cfg) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  const int rc = check_cfg(cfg);
  if (rc) return rc;
  G->cfg = to_cfg(cfg);
  return DSW_OK;
}

extern "C" int dsw_get_config(const dsw_grid *G, dsw_config *cfg) {
  if (!G || !cfg) return fail(DSW_EINVAL, "null argument");
  *cfg = from_cfg(G->cfg);
  return DSW_OK;
}

extern "C" int dsw_set_timing(dsw_grid *G, int32_t enable) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  G->timing = enable ? 1 : 0;
  return DSW_OK;
}

extern "C" int dsw_read_timing(dsw_grid *G, void *stream, double ms[DSW_TIMING_KINDS],
                               int64_t launches[DSW_TIMING_KINDS]) {
  if (!G || !ms || !launches) return fail(DSW_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  for (int q = 0; q < DSW_TIMING_KINDS; q++) { ms[q] = 0.0; launches[q] = 0; }
  // read every pair first; the events return to the free list only once all
  // reads succeeded, and the record is left as it was otherwise (a read can
  // fail when the step ran on another stream that is still busy)
  double acc[DSW_TIMING_KINDS] = {0.0};
  int64_t cnt[DSW_TIMING_KINDS] = {0};
  for (auto &r : G->recs) {
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    acc[r.kind] += t;
    cnt[r.kind] += 1;
  }
  for (auto &r : G->recs) {
    G->ev_free.push_back(r.a);
    G->ev_free.push_back(r.b);
  }
  G->recs.clear();
  for (int q = 0; q < DSW_TIMING_KINDS; q++) { ms[q] = acc[q]; launches[q] = cnt[q]; }
  return DSW_OK;
}

extern "C" int dsw_get_status(dsw_grid *G, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  int h[ST_WORDS];
  HIPCHK(hipMemcpy(h, G->status, sizeof(h), hipMemcpyDeviceToHost));
  HIPCHK(hipMemset(G->status, 0, sizeof(h)));
  if (h[ST_NONPHYS]) return fail(DSW_ENONPHYS, "non-positive temperature or pressure met");  // the cause of what follows
  // a non-finite residual comes first: the line solves that follow it see
  // non-finite pivots as well
  if (h[ST_DIVERGED]) return fail(DSW_EDIVERGED, "non-finite residual (diverged iteration or a NaN/Inf in the state)");
  if (h[ST_SINGULAR]) return fail(DSW_ESINGULAR, "zero pivot in a line solve");
  return DSW_OK;
}

// --------------------------------------------------------------- adjoint --

// transposed line solve of direction d on one grid: phi lines by the
// partitioned solver when the configuration and the line allow it
static void launch_T(const dsw_grid *G, int d, const Pass &p, hipStream_t st) {
  if (d == 2 && (p.kind == PK_SW2_PART || p.kind == PK_SW2_CP || p.kind == PK_SW2_CN)) {
    // two rows per chunk where the line allows it: twice the chunks in
    // flight for the same line (measured faster than four on the transposed
    // systems, whose row windows hold more registers)
    const int pm = phi_part_supported(G->geo, 2) ? 2 : G->cfg.phi_pm;
    launch_phi_T(pm, p.a, (unsigned)G->geo.nr * (unsigned)G->geo.nt, phi_part_threads(G->geo, pm),
                 phi_part_lds(G->geo, pm), st);
  } else if (d == 0 && p.kind == PK_SW0P) {
    // the transposed theta lines keep the two-ended solver: their row window
    // costs the partitioned kernel its second wave per SIMD (theta 0.59 ms
    // against 0.37 ms on the 256 x 128 x 64 sector; r 0.20 against 0.33 ms)
    launch_rt_T(d, p.a, (unsigned)G->cfg.sweep_bs[d], st);
  } else if (d < 2 && families(G->geo, d).nb < TWIST_LINES) {
    const unsigned bs = (unsigned)G->cfg.sweep_bs[d];
    launch_sweep2_T(d, p.a, sweep2_blocks(G->geo, d, bs), bs, st);
  } else {
    launch_sweep_T(d, p.a, cdiv(sweep_lines(G->geo, d), 128), 128, st);
  }
}

static int line_solve_T(int d, dsw_grid *G, const dsw_fields *Ubar, double tau, const dsw_fields *rhs,
                        dsw_fields *x, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  int rc;
  if ((rc = check_fields(Ubar, "Ubar")) || (rc = check_fields(rhs, "rhs")) || (rc = check_fields(x, "x")))
    return rc;
  if (!(tau > 0.0)) return fail(DSW_EINVAL, "tau must be > 0");
  if (rhs->p == x->p || rhs->ur == x->ur || rhs->ut == x->ut || rhs->uf == x->uf || rhs->T == x->T)
    return fail(DSW_EINVAL, "rhs and x must not alias");
  Out o{};
  o.x = F(x);
  o.mode = 0;
  launch_T(G, d, sweep_pass(G, d, F(Ubar), tau, F(rhs), o), (hipStream_t)stream);
  return check_launch("transposed sweep kernel");
}

extern "C" int dsw_line_solve_T_r(dsw_grid *G, const dsw_fields *Ubar, double tau,
                                  const dsw_fields *rhs, dsw_fields *x, void *stream) {
  return line_solve_T(0, G, Ubar, tau, rhs, x, stream);
}
extern "C" int dsw_line_solve_T_theta(dsw_grid *G, const dsw_fields *Ubar, double tau,
                                      const dsw_fields *rhs, dsw_fields *x, void *stream) {
  return line_solve_T(1, G, Ubar, tau, rhs, x, stream);
}
extern "C" int dsw_line_solve_T_phi(dsw_grid *G, const dsw_fields *Ubar, double tau,
                                    const dsw_fields *rhs, dsw_fields *x, void *stream) {
  return line_solve_T(2, G, Ubar, tau, rhs, x, stream);
}

static int line_vjp(int d, dsw_grid *G, const dsw_fields *Ubar, double tau, const dsw_fields *X,
                    const dsw_fields *mu, dsw_fields *acc, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  int rc;
  if ((rc = check_fields(Ubar, "Ubar")) || (rc = check_fields(X, "X")) || (rc = check_fields(mu, "mu")) ||
      (rc = check_fields(acc, "acc")))
    return rc;
  if (!(tau > 0.0)) return fail(DSW_EINVAL, "tau must be > 0");
  launch_line_vjp(d, G->geo, G->m, F(Ubar), tau, F(X), F(mu), F(acc), (hipStream_t)stream);
  return check_launch("line vjp kernel");
}

extern "C" int dsw_line_vjp_r(dsw_grid *G, const dsw_fields *Ubar, double tau, const dsw_fields *X,
                              const dsw_fields *mu, dsw_fields *acc, void *stream) {
  return line_vjp(0, G, Ubar, tau, X, mu, acc, stream);
}
extern "C" int dsw_line_vjp_theta(dsw_grid *G, const dsw_fields *Ubar, double tau, const dsw_fields *X,
                                  const dsw_fields *mu, dsw_fields *acc, void *stream) {
  return line_vjp(1, G, Ubar, tau, X, mu, acc, stream);
}
extern "C" int dsw_line_vjp_phi(dsw_grid *G, const dsw_fields *Ubar, double tau, const dsw_fields *X,
                                const dsw_fields *mu, dsw_fields *acc, void *stream) {
  return line_vjp(2, G, Ubar, tau, X, mu, acc, stream);
}

extern "C" int dsw_residual_vjp(dsw_grid *G, const dsw_fields *Ubar, double tau, const dsw_fields *mu,
                                dsw_fields *acc, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  int rc;
  if ((rc = check_fields(Ubar, "Ubar")) || (rc = check_fields(mu, "mu")) || (rc = check_fields(acc, "acc")))
    return rc;
  if (!(tau > 0.0)) return fail(DSW_EINVAL, "tau must be > 0");
  launch_residual_vjp(G->geo, G->m, F(Ubar), tau, F(mu), F(acc), (hipStream_t)stream);
  return check_launch("residual vjp kernel");
}

// adjoint workspace: nstates five-field states (their use is the caller's),
// then the sweep scratch of the second stream
static int adj_workspace(dsw_grid *G, int nstates, std::vector<Fields> &ws) {
  const long per = G->count[0] + G->count[1] + G->count[2] + G->count[3] + G->count[4];
  const long extra = G->sc.blk_len + G->sc.sca_len;
  if (!G->adj_mem || G->adj_states < nstates) {
    if (G->adj_mem) {
      HIPCHK(hipDeviceSynchronize());
      (void)hipFree(G->adj_mem);
      G->adj_mem = nullptr;
      G->adj_states = 0;
    }
    if (hipMalloc(&G->adj_mem, ((size_t)nstates * per + extra) * sizeof(double)) != hipSuccess) {
      G->adj_mem = nullptr;
      return fail(DSW_ENOMEM, "adjoint workspace");
    }
    G->adj_states = nstates;
  }
  // non-blocking: no implicit ordering against a caller's null stream
  if (!G->side && hipStreamCreateWithFlags(&G->side, hipStreamNonBlocking) != hipSuccess) {
    G->side = nullptr;
    return fail(DSW_EHIP, "adjoint stream");
  }
  if (!G->fork_ev && hipEventCreateWithFlags(&G->fork_ev, hipEventDisableTiming) != hipSuccess) {
    G->fork_ev = nullptr;
    return fail(DSW_EHIP, "adjoint events");
  }
  if (!G->join_ev && hipEventCreateWithFlags(&G->join_ev, hipEventDisableTiming) != hipSuccess) {
    G->join_ev = nullptr;
    return fail(DSW_EHIP, "adjoint events");
  }
  long off = 0;
  ws.clear();
  for (int q = 0; q < nstates; q++) ws.push_back(carve(G->adj_mem, G->count, &off));
  // the states of the largest workspace allocated so far come first
  double *s2 = G->adj_mem + (size_t)G->adj_states * per;
  G->sc2.blk = s2;
  G->sc2.sca = s2 + G->sc.blk_len;
  G->sc2.blk_len = G->sc.blk_len;
  G->sc2.sca_len = G->sc.sca_len;
  return DSW_OK;
}

// The states one iteration of the reverse reads: the midpoint (U^n itself
// at k = 0) and the three line-solve outputs, per iteration k.
struct Tape {
  std::vector<Fields> ub, x1, x2, x3;
};

// a tape held in workspace states q0 .. q0 + 4K - 1, in carve_tape's order
static Tape tape_from(const std::vector<Fields> &ws, int q0, int K, const Fields &un) {
  Tape t;
  for (int k = 0; k < K; k++) {
    t.ub.push_back(k == 0 ? un : ws[q0 + 4 * k]);
    t.x1.push_back(ws[q0 + 4 * k + 1]);
    t.x2.push_back(ws[q0 + 4 * k + 2]);
    t.x3.push_back(ws[q0 + 4 * k + 3]);
  }
  return t;
}

// 4K states carved from one buffer: Ubar (the slot of k = 0 unused), X1, X2, X3
static Tape carve_tape(double *base, const long *cnt, int K, const Fields &un) {
  Tape t;
  long off = 0;
  for (int k = 0; k < K; k++) {
    const Fields ub = carve(base, cnt, &off);
    t.ub.push_back(k == 0 ? un : ub);
    t.x1.push_back(carve(base, cnt, &off));
    t.x2.push_back(carve(base, cnt, &off));
    t.x3.push_back(carve(base, cnt, &off));
  }
  return t;
}

// The forward step from U^n into U (the running iterate, U^{n+1} at the
// end), keeping every iteration's midpoint and line-solve outputs in the
// tape.  The midpoint of the first iteration is U^n itself; the phi sweep
// updates U in place and writes the next midpoint and its own solution X3.
// Boundary-normal faces of U and of the midpoints are those of U^n (the
// sweeps leave them alone); those of X3 are never read.
// adj_record_bnd: those faces; adj_record_iter: iteration k.
static void adj_record_bnd(const dsw_grid *G, const Fields &un, int K, const Tape &t, const Fields &U,
                           hipStream_t st) {
  const Fields none{};
  std::vector<Fields> dst{U};
  for (int k = 1; k < K; k++) dst.push_back(t.ub[k]);
  for (size_t q = 0; q < dst.size(); q += 3) {
    Pass p{PK_BND, 4, base_args(G)};
    p.a.src = un;
    p.a.d0 = dst[q];
    p.a.d1 = q + 1 < dst.size() ? dst[q + 1] : none;
    p.a.d2 = q + 2 < dst.size() ? dst[q + 2] : none;
    launch_single(G, p, st);
  }
}

// scr: the sweep scratch of the line solves (the grid's, or the second
// stream's).  keep_last false: the last iterate U^{n+1} is not needed (a
// recompute for the reverse), so the last phi pass writes X3 alone.
static void adj_record_iter(const dsw_grid *G, const Fields &un, double tau, int K, int k, const Tape &t,
                            const Fields &U, const Scratch &scr, hipStream_t st, bool keep_last = true) {
  const Fields none{};
  const Fields ubk = t.ub[k];
  Pass r{G->geo.periodic ? PK_RES_INP : PK_RES_IN, 0, base_args(G)};
  r.a.u = src1(ubk);
  r.a.d = diff(un, k == 0 ? un : U);
  r.a.tau = tau;
  r.a.R = G->r;
  launch_single(G, r, st);
  r.kind = PK_RES;
  launch_single(G, r, st);
  Out o1{}, o2{}, o3{};
  o1.x = t.x1[k]; o2.x = t.x2[k];
  if (k == K - 1 && !keep_last) {
    o3.mode = 0;
    o3.x = t.x3[k];
  } else {
    o3.mode = 1;
    o3.x = U;
    o3.base = k == 0 ? un : U;
    o3.un = un;
    o3.ub = k < K - 1 ? t.ub[k + 1] : none;
    o3.raw = t.x3[k];
  }
  auto sw = [&](int d, const Fields &rhs, const Out &o) {
    Pass p = sweep_pass(G, d, ubk, tau, rhs, o);
    p.a.scb = scr.blk;
    p.a.scs = scr.sca;
    return p;
  };
  const auto run = [&](const Pass &q) { launch_single(G, q, st); };
  emit_sweep(G, sw(0, G->r, o1), run);
  emit_sweep(G, sw(1, t.x1[k], o2), run);
  emit_sweep(G, sw(2, t.x2[k], o3), run);
}

static void adj_record(const dsw_grid *G, const Fields &un, double tau, int K, const Tape &t,
                       const Fields &U, const Scratch &scr, hipStream_t st, bool keep_last = true) {
  adj_record_bnd(G, un, K, t, U, st);
  for (int k = 0; k < K; k++) adj_record_iter(G, un, tau, K, k, t, U, scr, st, keep_last);
}

// The reverse sweep (reverse of every statement of adj_record, last
// iteration first).  sc: two cotangents of the iterate, mu3, mu2, mu1 and
// the cotangent of Ubar.  Iteration k of it: the three transposed solves
// (adj_reverse_solves: they read only the midpoint of iteration k and the
// incoming cotangent L), then the reverse of the local rows and the mix
// (adj_reverse_local: these read X1, X2, X3 of iteration k as well).
struct Rev {
  Fields La, Lb, M3, M2, M1, UBB;
  Fields L, Lnext;
};

// Ordering between the caller's stream and the handle's second stream.  If
// a join fails, the second stream is synchronised before the error returns,
// so that no work of a failed call is left running beside the caller's.
static int side_fork(dsw_grid *G, hipStream_t st) {
  HIPCHK(hipEventRecord(G->fork_ev, st));
  HIPCHK(hipStreamWaitEvent(G->side, G->fork_ev, 0));
  return DSW_OK;
}
static int side_record(dsw_grid *G) {
  const hipError_t e = hipEventRecord(G->join_ev, G->side);
  if (e == hipSuccess) return DSW_OK;
  (void)hipStreamSynchronize(G->side);
  return fail(DSW_EHIP, std::string("second stream: ") + hipGetErrorString(e));
}
static int side_join(dsw_grid *G, hipStream_t st) {
  const hipError_t e = hipStreamWaitEvent(st, G->join_ev, 0);
  if (e == hipSuccess) return DSW_OK;
  (void)hipStreamSynchronize(G->side);
  return fail(DSW_EHIP, std::string("second stream: ") + hipGetErrorString(e));
}

// The mix of the last iteration (the first one reversed) writes lam_n; the
// cotangent of Ubar accumulates from zero, and every mix leaves it zero:
// zero_ubb clears it first (a call's first reverse).
static Rev adj_reverse_init(const dsw_grid *G, const Fields &un, const Fields &lam_np1, const Fields *sc,
                            bool zero_ubb, hipStream_t st) {
  const Fields none{};
  Rev v{sc[0], sc[1], sc[2], sc[3], sc[4], sc[5], lam_np1, sc[0]};
  if (zero_ubb) launch_axpy3(G->count, 0.0, un, 0.0, none, 0.0, none, v.UBB, st);
  return v;
}

// scr: the sweep scratch the solves use (the grid's, or the second stream's)
static void adj_reverse_solves(const dsw_grid *G, double tau, int k, const Tape &t, const Rev &v,
                               const Scratch &scr, hipStream_t st) {
  const Fields ubk = t.ub[k];
  Out o{};
  o.mode = 0;
  auto pass = [&](int d, const Fields &rhs) {
    Pass p = sweep_pass(G, d, ubk, tau, rhs, o);
    p.a.scb = scr.blk;
    p.a.scs = scr.sca;
    return p;
  };
  o.x = v.M3;
  launch_T(G, 2, pass(2, v.L), st);
  o.x = v.M2;
  launch_T(G, 1, pass(1, v.M3), st);
  o.x = v.M1;
  launch_T(G, 0, pass(0, v.M2), st);
}

static void adj_reverse_local(const dsw_grid *G, double tau, int K, int k, const Tape &t, Rev &v,
                              const Fields &lam_n, hipStream_t st) {
  const Fields xs[3] = {t.x1[k], t.x2[k], t.x3[k]}, mus[3] = {v.M1, v.M2, v.M3};
  launch_adj_local(G->geo, G->m, t.ub[k], tau, xs, mus, v.UBB, st);
  // also clears UBB; at k = 0 it adds the cotangent of U^{n+1,0} = U^n
  // to lam_n as well
  launch_adj_mix(G->geo, G->count, v.L, v.M1, v.UBB, v.Lnext, lam_n, k == 0, k == K - 1, st);
  v.L = v.Lnext;
  v.Lnext = (v.Lnext.p == v.La.p) ? v.Lb : v.La;
}

static void adj_reverse(const dsw_grid *G, const Fields &un, double tau, int K, const Tape &t,
                        const Fields &lam_np1, const Fields &lam_n, const Fields *sc, bool zero_ubb,
                        hipStream_t st) {
  Rev v = adj_reverse_init(G, un, lam_np1, sc, zero_ubb, st);
  for (int k = K - 1; k >= 0; k--) {
    adj_reverse_solves(G, tau, k, t, v, G->sc, st);
    adj_reverse_local(G, tau, K, k, t, v, lam_n, st);
  }
}

static int check_adjoint_args(const dsw_grid *G, const dsw_fields *Un, double tau, int32_t K,
                              const dsw_fields *lam_np1, const dsw_fields *lam_n) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  int rc;
  if ((rc = check_fields(Un, "Un")) || (rc = check_fields(lam_np1, "lam_np1")) ||
      (rc = check_fields(lam_n, "lam_n")))
    return rc;
  if (!(tau > 0.0)) return fail(DSW_EINVAL, "tau must be > 0");
  if (K < 1) return fail(DSW_EINVAL, "K must be >= 1");
  if (lam_n->p == lam_np1->p || lam_n->p == Un->p) return fail(DSW_EINVAL, "lam_n must not alias the inputs");
  return DSW_OK;
}

// One adjoint step with its recompute from un (into the iterate U and the
// tape t).  The last iteration's transposed solves read only its midpoint
// and lam_in: they run on the second stream (with a sweep scratch of their
// own) while the recompute finishes that iteration, whose X1, X2, X3 the
// rest of the reverse needs.  The two sides write disjoint buffers.
// then: called once the recompute has been enqueued and the solves joined,
// before the rest of the reverse (the trajectory queues its next recompute
// on the second stream there).
template <class Then>
static int adj_step_overlapped(dsw_grid *G, const Fields &un, double tau, int K, const Tape &t,
                               const Fields &U, const Fields &lam_in, const Fields &lam_out,
                               const Fields *sc, hipStream_t st, Then then) {
  int rc;
  adj_record_bnd(G, un, K, t, U, st);
  for (int k = 0; k < K - 1; k++) adj_record_iter(G, un, tau, K, k, t, U, G->sc, st);
  if ((rc = side_fork(G, st))) return rc;
  Rev v = adj_reverse_init(G, un, lam_in, sc, true, G->side);
  adj_reverse_solves(G, tau, K - 1, t, v, G->sc2, G->side);
  if ((rc = side_record(G))) return rc;
  adj_record_iter(G, un, tau, K, K - 1, t, U, G->sc, st, false);
  if ((rc = side_join(G, st))) return rc;
  if ((rc = then())) return rc;
  adj_reverse_local(G, tau, K, K - 1, t, v, lam_out, st);
  for (int k = K - 2; k >= 0; k--) {
    adj_reverse_solves(G, tau, k, t, v, G->sc, st);
    adj_reverse_local(G, tau, K, k, t, v, lam_out, st);
  }
  return DSW_OK;
}

extern "C" int dsw_adjoint_step(dsw_grid *G, const dsw_fields *Un, double tau, int32_t K,
                                const dsw_fields *lam_np1, dsw_fields *lam_n, void *stream) {
  int rc;
  if ((rc = check_adjoint_args(G, Un, tau, K, lam_np1, lam_n))) return rc;
  // workspace: the tape (4K states), the running iterate, the reverse's six
  std::vector<Fields> ws;
  if ((rc = adj_workspace(G, 4 * K + 7, ws))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Fields un = F(Un);
  const Tape t = tape_from(ws, 0, K, un);
  // forward recompute from the checkpoint into the workspace's iterate
  if ((rc = adj_step_overlapped(G, un, tau, K, t, ws[4 * K], F(lam_np1), F(lam_n), &ws[4 * K + 1], st,
                                [] { return (int)DSW_OK; })))
    return rc;
  return check_launch("adjoint step kernels");
}

extern "C" int dsw_tape_bytes(const dsw_grid *G, int32_t K, int64_t *bytes) {
  if (!G || !bytes) return fail(DSW_EINVAL, "null argument");
  if (K < 1) return fail(DSW_EINVAL, "K must be >= 1");
  const long per = G->count[0] + G->count[1] + G->count[2] + G->count[3] + G->count[4];
  *bytes = (int64_t)4 * K * per * (int64_t)sizeof(double);
  return DSW_OK;
}

extern "C" int dsw_split_step_taped(dsw_grid *G, const dsw_fields *Un, dsw_fields *Unp1, double tau,
                                    int32_t K, void *tape, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  const int rc = check_step_args(Un, Unp1, tau, K);
  if (rc) return rc;
  if (!tape || ((uintptr_t)tape % sizeof(double)) != 0) return fail(DSW_EINVAL, "tape must be a non-null 8-byte aligned pointer");
  hipStream_t st = (hipStream_t)stream;
  const Fields un = F(Un);
  const Tape t = carve_tape((double *)tape, G->count, K, un);
  adj_record(G, un, tau, K, t, F(Unp1), G->sc, st);
  return check_launch("taped split step kernels");
}

extern "C" int dsw_adjoint_step_taped(dsw_grid *G, const dsw_fields *Un, double tau, int32_t K,
                                      const void *tape, const dsw_fields *lam_np1, dsw_fields *lam_n,
                                      void *stream) {
  int rc;
  if ((rc = check_adjoint_args(G, Un, tau, K, lam_np1, lam_n))) return rc;
  if (!tape || ((uintptr_t)tape % sizeof(double)) != 0) return fail(DSW_EINVAL, "tape must be a non-null 8-byte aligned pointer");
  std::vector<Fields> ws;
  if ((rc = adj_workspace(G, 6, ws))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Fields un = F(Un);
  const Tape t = carve_tape((double *)const_cast<void *>(tape), G->count, K, un);
  adj_reverse(G, un, tau, K, t, F(lam_np1), F(lam_n), &ws[0], true, st);
  return check_launch("taped adjoint step kernels");
}

// The adjoint of nsteps consecutive split steps from their checkpoints.
// Step n - 1 is recomputed into one of two tapes on the second stream (with
// its own sweep scratch) while the reverse of step n runs from the other
// tape on the caller's stream.  A tape is overwritten only after the
// reverse that read it: the second stream waits for everything enqueued on
// the caller's stream before each recompute.  The last step (the first one
// reversed) runs as one overlapped adjoint step, whose recompute nothing
// overlaps otherwise.
extern "C" int dsw_adjoint_trajectory(dsw_grid *G, const dsw_fields *ckpts, int32_t nsteps, double tau,
                                      int32_t K, const dsw_fields *lam_end, dsw_fields *lam_0,
                                      void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  if (!ckpts || nsteps < 1) return fail(DSW_EINVAL, "need nsteps >= 1 checkpoints");
  int rc;
  if ((rc = check_adjoint_args(G, &ckpts[0], tau, K, lam_end, lam_0))) return rc;
  for (int n = 0; n < nsteps; n++) {
    if ((rc = check_fields(&ckpts[n], "checkpoint"))) return rc;
    if (ckpts[n].p == lam_0->p) return fail(DSW_EINVAL, "lam_0 must not alias a checkpoint");
  }
  // workspace: two tapes, the running iterate, the reverse's six states,
  // two cotangents of the step states
  std::vector<Fields> ws;
  if ((rc = adj_workspace(G, 8 * K + 9, ws))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Fields U = ws[8 * K];
  const Fields *sc = &ws[8 * K + 1];
  const Fields P[2] = {ws[8 * K + 7], ws[8 * K + 8]};
  auto tape = [&](int n) { return tape_from(ws, (n & 1) ? 4 * K : 0, K, F(&ckpts[n])); };
  // the next recompute, on the second stream, once everything enqueued on
  // the caller's stream so far is done
  auto next_record = [&](int n) {
    int r;
    if ((r = side_fork(G, st))) return r;
    adj_record(G, F(&ckpts[n]), tau, K, tape(n), U, G->sc2, G->side, false);
    return side_record(G);
  };
  const int last = nsteps - 1;
  Fields lin = last == 0 ? F(lam_0) : P[last & 1];
  if ((rc = adj_step_overlapped(G, F(&ckpts[last]), tau, K, tape(last), U, F(lam_end), lin, sc, st,
                                [&] { return last >= 1 ? next_record(last - 1) : (int)DSW_OK; })))
    return rc;
  if (last >= 1 && (rc = side_join(G, st))) return rc;
  for (int n = last - 1; n >= 0; n--) {
    if (n >= 1 && (rc = next_record(n - 1))) return rc;
    const Fields lout = n == 0 ? F(lam_0) : P[n & 1];
    // the cotangent of Ubar is zero here: every reverse iteration's mix clears it
    adj_reverse(G, F(&ckpts[n]), tau, K, tape(n), lin, lout, sc, false, st);
    lin = lout;
    if (n >= 1 && (rc = side_join(G, st))) return rc;
  }
  return check_launch("adjoint trajectory kernels");
}

// ------------------------------------------------------------- ensembles --

struct dsw_ensemble {
  std::vector<dsw_grid *> mem;
  Cfg cfg{64, {256, 256}, 4, {-1, -1}};
  hipStream_t cap = nullptr, cap2 = nullptr;  // capture streams of the two lanes
  hipEvent_t fork = nullptr, stagger = nullptr, join = nullptr;
  // one launch of a batched plan
  struct Group {
    int kind, tk;
    unsigned blocks, threads;
    size_t lds;
    size_t tab_off, woff_off; // byte offsets into the plan's device buffer
    int n;
  };
  struct Plan {
    std::vector<Group> groups;
    char *dev = nullptr;
  };
  struct Entry {
    std::vector<uint64_t> key;
    Plan plan[2];  // the two lanes' plans (plan[1] empty with one member)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
  };
  std::vector<Entry> cache;
  uint64_t tick = 0;
};

static void free_plan(dsw_ensemble::Plan &p) {
  if (p.dev) (void)hipFree(p.dev);
  p.dev = nullptr;
  p.groups.clear();
}

static void drop_entry(dsw_ensemble::Entry &e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.graph) (void)hipGraphDestroy(e.graph);
  e.exec = nullptr;
  e.graph = nullptr;
  free_plan(e.plan[0]);
  free_plan(e.plan[1]);
}

extern "C" int dsw_ensemble_create(const dsw_grid_desc *descs, const dsw_material *mats, int32_t n,
                                   dsw_ensemble **out) {
  if (!out) return fail(DSW_EINVAL, "null output handle");
  *out = nullptr;
  if (!descs || !mats || n < 1) return fail(DSW_EINVAL, "need n >= 1 descriptors and materials");
  dsw_ensemble *E = new dsw_ensemble();
  for (int m = 0; m < n; m++) {
    dsw_grid *G = nullptr;
    const int rc = dsw_init_grid(&descs[m], &mats[m], &G);
    if (rc) {
      const std::string msg = "member " + std::to_string(m) + ": " + g_err;
      dsw_ensemble_free(E);
      return fail(rc, msg);
    }
    G->cfg = E->cfg;  // a member's own steps take the ensemble's launch shapes
    E->mem.push_back(G);
  }
  if (hipStreamCreateWithFlags(&E->cap, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&E->cap2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&E->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&E->stagger, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&E->join, hipEventDisableTiming) != hipSuccess) {
    dsw_ensemble_free(E);
    return fail(DSW_EHIP, "capture streams");
  }
  *out = E;
  return DSW_OK;
}

extern "C" int dsw_ensemble_free(dsw_ensemble *E) {
  if (!E) return DSW_OK;
  (void)hipDeviceSynchronize();
  for (auto &e : E->cache) drop_entry(e);
  if (E->cap) (void)hipStreamDestroy(E->cap);
  if (E->cap2) (void)hipStreamDestroy(E->cap2);
  if (E->fork) (void)hipEventDestroy(E->fork);
  if (E->stagger) (void)hipEventDestroy(E->stagger);
  if (E->join) (void)hipEventDestroy(E->join);
  for (dsw_grid *G : E->mem) dsw_free_grid(G);
  delete E;
  return DSW_OK;
}

extern "C" int dsw_ensemble_member(dsw_ensemble *E, int32_t m, dsw_grid **grid) {
  if (!E || !grid) return fail(DSW_EINVAL, "null argument");
  if (m < 0 || m >= (int)E->mem.size()) return fail(DSW_EINVAL, "member index out of range");
  *grid = E->mem[m];
  return DSW_OK;
}

static int check_ens_args(dsw_ensemble *E, const dsw_fields *Un, dsw_fields *Unp1, const double *tau,
                          int32_t K) {
  if (!E || !Un || !Unp1 || !tau) return fail(DSW_EINVAL, "null argument");
  for (size_t m = 0; m < E->mem.size(); m++) {
    const int rc = check_step_args(&Un[m], &Unp1[m], tau[m], K);
    if (rc) return fail(rc, "member " + std::to_string(m) + ": " + g_err);
  }
  for (size_t m = 0; m < E->mem.size(); m++) // outputs of different members must be distinct
    for (size_t q = 0; q < E->mem.size(); q++)
      if (q != m && (Unp1[m].p == Unp1[q].p || Unp1[m].p == Un[q].p))
        return fail(DSW_EINVAL, "member " + std::to_string(m) + ": Unp1 aliases another member's state");
  return DSW_OK;
}

// Batched plan of one ensemble step over the members ids (all members when
// empty): pass q of every member's plan goes into one launch (two for the
// phi pass when members differ in solver kind).
static int build_plan(dsw_ensemble *E, const Cfg &cfg, const dsw_fields *Un, dsw_fields *Unp1,
                      const double *tau, int K, dsw_ensemble::Plan &plan,
                      std::vector<int> ids = std::vector<int>()) {
  if (ids.empty())
    for (int m = 0; m < (int)E->mem.size(); m++) ids.push_back(m);
  const int n = (int)ids.size();
  std::vector<dsw_grid *> mem(n);
  std::vector<std::vector<Pass>> per(n);
  for (int m = 0; m < n; m++) {
    dsw_grid *G = mem[m] = E->mem[ids[m]];
    const Cfg keep = G->cfg;
    G->cfg = cfg;
    plan_step(G, own_work(G), F(&Un[ids[m]]), F(&Unp1[ids[m]]), tau[ids[m]], K,
              [&](const Pass &p) { per[m].push_back(p); });
    G->cfg = keep;
  }
  // plan_step gives every grid the same sequence of passes (PK_NONE where a
  // grid's sweep has one pass fewer): pass q of every member runs together
  const size_t npass = per[0].size();
  for (int m = 1; m < n; m++)
    if (per[m].size() != npass) return fail(DSW_EINVAL, "ensemble members' steps do not align");
  std::vector<char> host;
  auto append = [&](const void *src, size_t bytes) {
    size_t off = (host.size() + 255) & ~size_t(255);
    host.resize(off + bytes);
    std::memcpy(host.data() + off, src, bytes);
    return off;
  };
  for (size_t q = 0; q < npass; q++) {
    std::vector<int> kinds;  // distinct kinds of pass q over the members, in order
    for (int m = 0; m < n; m++)
      if (per[m][q].kind != PK_NONE && std::find(kinds.begin(), kinds.end(), per[m][q].kind) == kinds.end())
        kinds.push_back(per[m][q].kind);
    for (const int kind : kinds) {
      // one launch per (kind, workgroup width): members whose phi lines need
      // narrower workgroups do not pay for the widest one
      std::vector<unsigned> widths;
      for (int m = 0; m < n; m++) {
        if (per[m][q].kind != kind) continue;
        const unsigned w0 = kind_threads(kind, mem[m]->geo, cfg);
        if (std::find(widths.begin(), widths.end(), w0) == widths.end()) widths.push_back(w0);
      }
      for (const unsigned width : widths) {
      std::vector<int> who;
      for (int m = 0; m < n; m++)
        if (per[m][q].kind == kind && kind_threads(kind, mem[m]->geo, cfg) == width) who.push_back(m);
      unsigned th = 0;
      size_t lds = 0;
      for (int m : who) {
        th = std::max(th, kind_threads(kind, mem[m]->geo, cfg));
        lds = std::max(lds, kind_lds(kind, mem[m]->geo, cfg));
      }
      std::vector<PassArgs> tab;
      std::vector<unsigned> woff(1, 0u);
      unsigned long total = 0;
      for (int m : who) {
        tab.push_back(per[m][q].a);
        total += kind_blocks(kind, mem[m]->geo, cfg, th);
        if (total > 0x7fffffffUL) return fail(DSW_EINVAL, "ensemble too large for one launch");
        woff.push_back((unsigned)total);
      }
      dsw_ensemble::Group gr;
      gr.kind = kind;
      gr.tk = per[0][q].tk;
      if (total == 0) continue;  // nothing to launch (e.g. no interior workgroups)
      gr.blocks = (unsigned)total;
      gr.threads = th;
      gr.lds = lds;
      gr.n = (int)who.size();
      gr.tab_off = append(tab.data(), tab.size() * sizeof(PassArgs));
      gr.woff_off = append(woff.data(), woff.size() * sizeof(unsigned));
      plan.groups.push_back(gr);
      }
    }
  }
  if (hipMalloc(&plan.dev, host.size()) != hipSuccess) {
    plan.dev = nullptr;
    return fail(DSW_ENOMEM, "ensemble launch tables");
  }
  HIPCHK(hipMemcpy(plan.dev, host.data(), host.size(), hipMemcpyHostToDevice));
  return DSW_OK;
}

// enqueue groups [g0, g1) of a batched plan (g1 < 0: to the end); ev
// (optional) receives one event pair per group
static void enqueue_plan(const dsw_ensemble::Plan &plan, const Cfg &cfg, hipStream_t st,
                         std::vector<std::pair<hipEvent_t, hipEvent_t>> *ev, size_t g0 = 0, long g1 = -1) {
  PassArgs dummy;
  std::memset(&dummy, 0, sizeof(dummy));
  const size_t end = g1 < 0 ? plan.groups.size() : (size_t)g1;
  for (size_t q = g0; q < end; q++) {
    const auto &gr = plan.groups[q];
    const Batch b{(CPassArgs *)(plan.dev + gr.tab_off), (const unsigned *)(plan.dev + gr.woff_off),
                  gr.n};
    if (ev) (void)hipEventRecord((*ev)[q].first, st);
    launch_kind(gr.kind, cfg, dummy, b, gr.blocks, gr.threads, gr.lds, st);
    if (ev) (void)hipEventRecord((*ev)[q].second, st);
  }
}

static std::vector<uint64_t> plan_key(const dsw_ensemble *E, const Cfg &cfg, const dsw_fields *Un,
                                      const dsw_fields *Unp1, const double *tau, int K) {
  std::vector<uint64_t> k;
  k.push_back((uint64_t)K);
  k.push_back((uint64_t)cfg.res_bs | ((uint64_t)cfg.sweep_bs[0] << 16) |
              ((uint64_t)cfg.sweep_bs[1] << 32) | ((uint64_t)cfg.phi_pm << 48) |
              ((uint64_t)(cfg.rt_pm[0] + 1) << 52) | ((uint64_t)(cfg.rt_pm[1] + 1) << 56));
  for (size_t m = 0; m < E->mem.size(); m++) {
    const double *pu[10] = {Un[m].p, Un[m].ur, Un[m].ut, Un[m].uf, Un[m].T,
                            Unp1[m].p, Unp1[m].ur, Unp1[m].ut, Unp1[m].uf, Unp1[m].T};
    for (int q = 0; q < 10; q++) k.push_back((uint64_t)(uintptr_t)pu[q]);
    uint64_t tb;
    std::memcpy(&tb, &tau[m], sizeof(tb));
    k.push_back(tb);
  }
  return k;
}

extern "C" int dsw_ensemble_step(dsw_ensemble *E, const dsw_fields *Un, dsw_fields *Unp1,
                                 const double *tau, int32_t K, void *stream) {
  int rc = check_ens_args(E, Un, Unp1, tau, K);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const std::vector<uint64_t> key = plan_key(E, E->cfg, Un, Unp1, tau, K);
  dsw_ensemble::Entry *hit = nullptr;
  for (auto &e : E->cache)
    if (e.exec && e.key == key) hit = &e;
  if (!hit) {
    if (E->cache.size() >= 8) { // drop the least recently used graph
      size_t old = 0;
      for (size_t q = 1; q < E->cache.size(); q++)
        if (E->cache[q].used < E->cache[old].used) old = q;
      HIPCHK(hipDeviceSynchronize());
      drop_entry(E->cache[old]);
      E->cache.erase(E->cache.begin() + old);
    }
    dsw_ensemble::Entry e;
    e.key = key;
    // Two lanes of members, balanced by cells: the graph runs each lane's
    // batched launches in order, the second lane starting when the first
    // one's first residual launch has ended, so that one lane's residual
    // (bound by load latency) runs beside the other's sweeps (bound by HBM).
    // Members share no buffers: the lanes need no other ordering.
    const int n = (int)E->mem.size();
    std::vector<int> lane[2];
    {
      std::vector<int> order(n);
      for (int m = 0; m < n; m++) order[m] = m;
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return E->mem[x]->count[0] > E->mem[y]->count[0];
      });
      long load[2] = {0, 0};
      for (int m : order) {
        const int l = load[1] < load[0] ? 1 : 0;
        lane[l].push_back(m);
        load[l] += E->mem[m]->count[0];
      }
      for (auto &v : lane) std::sort(v.begin(), v.end());
    }
    if ((rc = build_plan(E, E->cfg, Un, Unp1, tau, K, e.plan[0], lane[0]))) return rc;
    if (!lane[1].empty() && (rc = build_plan(E, E->cfg, Un, Unp1, tau, K, e.plan[1], lane[1]))) {
      drop_entry(e);
      return rc;
    }
    HIPCHK(hipStreamBeginCapture(E->cap, hipStreamCaptureModeThreadLocal));
    if (lane[1].empty()) {
      enqueue_plan(e.plan[0], E->cfg, E->cap, nullptr);
    } else {
      size_t s0 = 0;  // lane 0's groups up to its first r sweep
      while (s0 < e.plan[0].groups.size() && e.plan[0].groups[s0].tk != 1) s0++;
      (void)hipEventRecord(E->fork, E->cap);
      (void)hipStreamWaitEvent(E->cap2, E->fork, 0);
      enqueue_plan(e.plan[0], E->cfg, E->cap, nullptr, 0, (long)s0);
      (void)hipEventRecord(E->stagger, E->cap);
      (void)hipStreamWaitEvent(E->cap2, E->stagger, 0);
      enqueue_plan(e.plan[1], E->cfg, E->cap2, nullptr);
      (void)hipEventRecord(E->join, E->cap2);
      enqueue_plan(e.plan[0], E->cfg, E->cap, nullptr, s0);
      (void)hipStreamWaitEvent(E->cap, E->join, 0);
    }
    const hipError_t ce = hipStreamEndCapture(E->cap, &e.graph);
    if (ce != hipSuccess) {
      drop_entry(e);
      return fail(DSW_EHIP, std::string("graph capture: ") + hipGetErrorString(ce));
    }
    const hipError_t ie = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      drop_entry(e);
      return fail(DSW_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
    }
    E->cache.push_back(e);
    hit = &E->cache.back();
  }
  hit->used = ++E->tick;
  HIPCHK(hipGraphLaunch(hit->exec, st));
  return DSW_OK;
}

extern "C" int dsw_ensemble_set_config(dsw_ensemble *E, const dsw_config *cfg) {
  if (!E) return fail(DSW_EINVAL, "null handle");
  const int rc = check_cfg(cfg);
  if (rc) return rc;
  E->cfg = to_cfg(cfg);
  for (dsw_grid *G : E->mem) G->cfg = E->cfg;
  return DSW_OK;
}

extern "C" int dsw_ensemble_get_config(const dsw_ensemble *E, dsw_config *cfg) {
  if (!E || !cfg) return fail(DSW_EINVAL, "null argument");
  *cfg = from_cfg(E->cfg);
  return DSW_OK;
}

extern "C" int dsw_ensemble_tune(dsw_ensemble *E, const dsw_fields *Un, dsw_fields *Unp1,
                                 const double *tau, int32_t K, int32_t reps, void *stream,
                                 dsw_config *best) {
  int rc = check_ens_args(E, Un, Unp1, tau, K);
  if (rc) return rc;
  if (reps < 1) return fail(DSW_EINVAL, "reps must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  // A tuned result is kept per set of member shapes (and K) for the process:
  // a second ensemble of the same shapes takes it without timing.
  static std::mutex cache_mu;
  static std::vector<std::pair<std::vector<long>, Cfg>> cache;
  std::vector<long> key{(long)K};
  for (const dsw_grid *G : E->mem)
    for (long v : {(long)G->geo.nr, (long)G->geo.nt, (long)G->geo.np, (long)G->geo.periodic}) key.push_back(v);
  {
    std::lock_guard<std::mutex> lk(cache_mu);
    for (const auto &e : cache)
      if (e.first == key) {
        E->cfg = e.second;
        for (dsw_grid *G : E->mem) G->cfg = e.second;
        if (best) *best = from_cfg(e.second);
        return DSW_OK;
      }
  }
  // candidate (v, p) sets every workgroup width to its v-th value, the phi
  // solver to its v-th kind and the r and theta solvers to p (-1: each
  // member by its line length, 4 partitioned, 0 two-ended); passes are timed
  // separately, so each pass keeps its own best value
  const int bsz[3] = {64, 128, 256}, pms[3] = {4, 2, 0}, rts[3] = {-1, 4, 0};
  double tbest[4] = {1e300, 1e300, 1e300, 1e300};
  Cfg out = E->cfg;
  for (int vp = 0; vp < 9; vp++) {
    const int v = vp % 3, pr = rts[vp / 3];
    if (pr == 0 && v == 0) continue;  // the two-ended solver: 128 and 256 only
    const Cfg c{bsz[v], {bsz[v], bsz[v]}, pms[v], {pr, pr}};
    dsw_ensemble::Plan plan;
    if ((rc = build_plan(E, c, Un, Unp1, tau, K, plan))) return rc;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev(plan.groups.size());
    for (auto &e : ev) {
      HIPCHK(hipEventCreate(&e.first));
      HIPCHK(hipEventCreate(&e.second));
    }
    double t[4] = {0, 0, 0, 0};
    enqueue_plan(plan, c, st, nullptr); // warm-up
    for (int r = 0; r < reps; r++) {
      enqueue_plan(plan, c, st, &ev);
      HIPCHK(hipStreamSynchronize(st));
      for (size_t q = 0; q < plan.groups.size(); q++) {
        const int tk = plan.groups[q].tk;
        if (tk < 0 || tk > 3) continue;
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, ev[q].first, ev[q].second));
        t[tk] += ms;
      }
    }
    for (auto &e : ev) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    free_plan(plan);
    if (t[0] < tbest[0]) { tbest[0] = t[0]; out.res_bs = c.res_bs; }
    if (t[1] < tbest[1]) { tbest[1] = t[1]; out.sweep_bs[0] = c.sweep_bs[0]; out.rt_pm[0] = c.rt_pm[0]; }
    if (t[2] < tbest[2]) { tbest[2] = t[2]; out.sweep_bs[1] = c.sweep_bs[1]; out.rt_pm[1] = c.rt_pm[1]; }
    if (vp < 3 && t[3] < tbest[3]) { tbest[3] = t[3]; out.phi_pm = c.phi_pm; }
  }
  rc = check_launch("ensemble tuning kernels");
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(cache_mu);
    cache.emplace_back(key, out);
  }
  E->cfg = out;
  for (dsw_grid *G : E->mem) G->cfg = out;
  if (best) *best = from_cfg(out);
  return DSW_OK;
}

extern "C" int dsw_ensemble_get_status(dsw_ensemble *E, void *stream) {
  if (!E) return fail(DSW_EINVAL, "null handle");
  int first = DSW_OK;
  std::string msg;
  for (size_t m = 0; m < E->mem.size(); m++) {
    const int rc = dsw_get_status(E->mem[m], stream);
    if (rc && first == DSW_OK) { first = rc; msg = "member " + std::to_string(m) + ": " + g_err; }
  }
  if (first) return fail(first, msg);
  return DSW_OK;
}
