// api.hip -- host implementation of the C-ABI declared in include/dsw.h:
// descriptor validation, metric tables, workspace and the orchestration of
// one split time step (paper section 2.2: K iterations of residual + three
// sweeps on one HIP stream; eqs. (spl1)-(spl3)).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dsw.h"
#include "dsw_common.hpp"
#include "dsw_internal.hpp"

using namespace dsw;

struct dsw_grid {
  dsw_grid_desc desc;
  dsw_material mat;
  Geo geo;
  Mat m;
  double *tables = nullptr; // rc | rf | sc | cc | sf | cf
  Fields ub{}, ub2{}, r{}, x1{}, x2{}; // ub, ub2: midpoint states of consecutive iterations
  double *fields_mem = nullptr;
  Scratch sc{};
  double *scratch_mem = nullptr;
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
  const int nr = desc->n_r, nt = desc->n_theta, np = desc->n_phi;
  // metric tables (host, then device)
  const size_t nt1 = (size_t)nt + 1, nr1 = (size_t)nr + 1;
  std::vector<double> h(2 * (nr + nr1) + 4 * (nt + nt1));
  double *rc = h.data(), *rf = rc + nr, *sc = rf + nr1, *cc = sc + nt, *sf = cc + nt, *cf = sf + nt1;
  double *irc = cf + nt1, *irf = irc + nr, *isc = irf + nr1, *ctc = isc + nt, *isf = ctc + nt,
         *ctf = isf + nt1;
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
             o_isf = o_ctc + nt, o_ctf = o_isf + nt1;
  g.rc = t; g.rf = t + o_rf; g.sc = t + o_sc; g.cc = t + o_cc; g.sf = t + o_sf; g.cf = t + o_cf;
  g.irc = t + o_irc; g.irf = t + o_irf; g.isc = t + o_isc; g.ctc = t + o_ctc; g.isf = t + o_isf;
  g.ctf = t + o_ctf;
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
  launch_sweep(d, G->geo, G->m, F(Ubar), tau, F(rhs), o, G->sc, G->status, (hipStream_t)stream);
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

extern "C" int dsw_split_step(dsw_grid *G, const dsw_fields *Un, dsw_fields *Unp1, double tau,
                              int32_t K, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  int rc;
  if ((rc = check_fields(Un, "Un")) || (rc = check_fields(Unp1, "Unp1"))) return rc;
  if (!(tau > 0.0)) return fail(DSW_EINVAL, "tau must be > 0");
  if (K < 1) return fail(DSW_EINVAL, "K must be >= 1");
  if (Un->p == Unp1->p || Un->ur == Unp1->ur || Un->ut == Unp1->ut || Un->uf == Unp1->uf ||
      Un->T == Unp1->T)
    return fail(DSW_EINVAL, "Unp1 must not alias Un");
  hipStream_t st = (hipStream_t)stream;
  const Fields un = F(Un), uk = F(Unp1);
  const Fields none{};
  // Dirichlet data of U^{n+1} and of both midpoint buffers = those of U^n
  timed(G, 4, st, [&] { launch_bnd_copy(G->geo, un, uk, G->ub, G->ub2, st); });
  const Fields ubuf[2] = {G->ub, G->ub2};
  for (int it = 0; it < K; it++) {
    // midpoint state of this iteration: U^n itself at the first one, else the
    // one written by the previous iteration's phi sweep
    const Fields ubar = it == 0 ? un : ubuf[(it - 1) % 2];
    timed(G, 0, st, [&] {
      launch_residual_given_mid(G->geo, G->m, un, it == 0 ? un : uk, ubar, tau, G->r, G->status, st);
    });
    Out o1{}, o2{}, o3{};
    o1.x = G->x1; o1.mode = 0;
    o2.x = G->x2; o2.mode = 0;
    o3.x = uk; o3.base = it == 0 ? un : uk; o3.un = un;
    o3.ub = it < K - 1 ? ubuf[it % 2] : none;
    o3.mode = 1;
    timed(G, 1, st, [&] { launch_sweep(0, G->geo, G->m, ubar, tau, G->r, o1, G->sc, G->status, st); });
    timed(G, 2, st, [&] { launch_sweep(1, G->geo, G->m, ubar, tau, G->x1, o2, G->sc, G->status, st); });
    timed(G, 3, st, [&] { launch_sweep(2, G->geo, G->m, ubar, tau, G->x2, o3, G->sc, G->status, st); });
  }
  return check_launch("split step kernels");
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
  for (auto &r : G->recs) {
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.kind] += t;
    launches[r.kind] += 1;
    G->ev_free.push_back(r.a);
    G->ev_free.push_back(r.b);
  }
  G->recs.clear();
  return DSW_OK;
}

extern "C" int dsw_get_status(dsw_grid *G, void *stream) {
  if (!G) return fail(DSW_EINVAL, "null handle");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  int h[ST_WORDS];
  HIPCHK(hipMemcpy(h, G->status, sizeof(h), hipMemcpyDeviceToHost));
  HIPCHK(hipMemset(G->status, 0, sizeof(h)));
  if (h[ST_NONPHYS]) return fail(DSW_ENONPHYS, "non-positive temperature or pressure met");
  if (h[ST_SINGULAR]) return fail(DSW_ESINGULAR, "zero pivot in a line solve");
  return DSW_OK;
}
