// C ABI of the GRFFE DG-FD hot path: domain set-up, state transfer and the
// orchestration of one IMEX-SSP3(4,3,3) step with the hybrid DG-FD control.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "grffe_internal.h"

namespace grffe {
void launch_fd_to_dg_policy(const KArgs& a, int N, bool curved, int policy, const uint8_t* forced, hipStream_t s);
void launch_bg_derive_q(const KArgs& a, int N, double* bg_fd, double* bg_face, const double* Q, hipStream_t s);
}  // namespace grffe

using namespace grffe;

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess) return fail(GRFFE_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

static hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

static int check_dom(grffe_domain* d) {
  if (!d) return fail(GRFFE_EINVAL, "domain is NULL");
  return GRFFE_OK;
}

extern "C" const char* grffe_last_error(void) { return g_err.c_str(); }

extern "C" void grffe_default_params(grffe_params* p) {
  std::memset(p, 0, sizeof(*p));
  p->eta = 1e6;
  p->kappa_psi = 1.0;
  p->kappa_phi = 1.0;
  p->cfl = 0.25;
  p->stab_c = 0.0;
  p->tci_M = 0;
  p->tci_mode = 2;
  p->tci_alpha = 4.0;
  p->tci_alpha_fd = 5.0;
  p->filter_a = 36.0;
  p->filter_b = 50.0;
  p->filter_on = 1;
  p->fd_order = 4;
  p->weno_eps = 1e-40;
  p->ff_clamp = 0;
  p->ff_margin = 1e-12;
  p->hybrid = GRFFE_HYBRID_ADAPTIVE;
  p->precision = 0;
}

namespace grffe {

KArgs make_args(grffe_domain* d) {
  KArgs a{};
  a.E = d->E;
  a.nx = d->nx;
  a.ny = d->ny;
  a.nz = d->nz;
  for (int k = 0; k < 3; ++k) a.h[k] = d->h[k];
  a.nbr = d->nbr;
  a.live = d->live;
  a.bg_dg = d->bg_dg;
  a.bg_fd = d->bg_fd;
  a.bg_face = d->bg_face;
  a.ops = d->ops;
  a.dg = d->dg;
  a.fd = d->fd;
  a.rep0 = d->rep0;
  a.rep = d->rep;
  a.troubled = d->troubled;
  a.ratio = d->ratio;
  a.w_fd = d->w_fd;
  a.trace = d->trace;
  a.slab = d->slab;
  a.fhat = d->fhat;
  a.dt = d->dt_cfl;
  a.eta = d->par.eta;
  a.kpsi = d->par.kappa_psi;
  a.kphi = d->par.kappa_phi;
  const int M = d->par.tci_M > 0 ? d->par.tci_M : default_tci_M(d->N);
  a.tci_thr = std::pow((double)(d->N + 1 - M), -d->par.tci_alpha);
  a.tci_thr_fd = std::pow((double)(d->N + 1 - M), -d->par.tci_alpha_fd);
  a.tci_mode = d->par.tci_mode;
  a.filter_on = d->par.filter_on;
  a.fd_order = d->par.fd_order;
  a.ff_clamp = d->par.ff_clamp;
  a.hybrid = d->par.hybrid;
  a.weno_eps = d->par.weno_eps;
  a.ff_margin = d->par.ff_margin;
  a.parts = GRFFE_PART_ALL;
  return a;
}

}  // namespace grffe

static int dalloc(grffe_domain* d, void** p, size_t bytes) {
  if (bytes == 0) {
    *p = nullptr;
    return GRFFE_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return fail(GRFFE_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  d->allocs.push_back(*p);
  return GRFFE_OK;
}

static void free_all(grffe_domain* d) {
  for (void* p : d->allocs) (void)hipFree(p);
  d->allocs.clear();
}

extern "C" int grffe_destroy(grffe_domain* d) {
  if (!d) return GRFFE_OK;
  for (hipEvent_t e : d->ev) (void)hipEventDestroy(e);
  d->ev.clear();
  free_all(d);
  delete d;
  return GRFFE_OK;
}

// Half the extent of SSP-RK3's stability interval on the negative real axis:
// the root of 1 + x + x^2/2 + x^3/6 = -1, found by Newton's method.
static double ssp_rk3_stability_c() {
  double x = -2.5;
  for (int it = 0; it < 50; ++it) {
    const double f = 2.0 + x + 0.5 * x * x + x * x * x / 6.0;
    const double df = 1.0 + x + 0.5 * x * x;
    const double dx = f / df;
    x -= dx;
    if (std::fabs(dx) < 1e-16 * std::fabs(x)) break;
  }
  return -x / 2.0;
}

static int validate(const grffe_grid* g, const grffe_params* p) {
  if (!g || !p) return fail(GRFFE_EINVAL, "grid and params must not be NULL");
  if (g->degree < 3 || g->degree > MAX_DEG) return fail(GRFFE_EINVAL, "degree must be in [3, 7]");
  for (int k = 0; k < 3; ++k) {
    if (g->n_elem[k] < 1) return fail(GRFFE_EINVAL, "n_elem must be positive");
    if (!(g->upper[k] > g->lower[k])) return fail(GRFFE_EINVAL, "upper must exceed lower");
  }
  for (int k = 0; k < 6; ++k)
    if (g->bc[k] != GRFFE_BC_PERIODIC && g->bc[k] != GRFFE_BC_NO_INCOMING_POYNTING)
      return fail(GRFFE_EINVAL, "unknown boundary kind");
  for (int d = 0; d < 3; ++d)
    if ((g->bc[2 * d] == GRFFE_BC_PERIODIC) != (g->bc[2 * d + 1] == GRFFE_BC_PERIODIC))
      return fail(GRFFE_EINVAL, "periodic faces must come in pairs");
  if (p->precision != 0) return fail(GRFFE_EUNSUPPORTED, "only FP64 is built");
  if (p->hybrid < 0 || p->hybrid > 2) return fail(GRFFE_EINVAL, "hybrid must be 0, 1 or 2");
  if (p->fd_order != 2 && p->fd_order != 4) return fail(GRFFE_EINVAL, "fd_order must be 2 or 4");
  if (p->tci_mode != 1 && p->tci_mode != 2) return fail(GRFFE_EINVAL, "tci_mode must be 1 or 2");
  if (!(p->cfl > 0.0)) return fail(GRFFE_EINVAL, "cfl must be positive");
  if (p->eta < 0.0 || p->kappa_psi < 0.0 || p->kappa_phi < 0.0) return fail(GRFFE_EINVAL, "negative rates");
  const int M = p->tci_M > 0 ? p->tci_M : default_tci_M(g->degree);
  if (M < 1 || M > g->degree) return fail(GRFFE_EINVAL, "tci_M out of range");
  return GRFFE_OK;
}

extern "C" int grffe_init_domain(const grffe_grid* g, const grffe_params* p, const double* bg, void* stream,
                                 grffe_domain** out) {
  if (!out) return fail(GRFFE_EINVAL, "out must not be NULL");
  *out = nullptr;
  int rc = validate(g, p);
  if (rc) return rc;
  grffe_domain* d = new grffe_domain();
  d->N = g->degree;
  d->n = d->N + 1;
  d->m = 2 * d->N + 1;
  d->nn = d->n * d->n * d->n;
  d->mm = d->m * d->m * d->m;
  d->nx = g->n_elem[0];
  d->ny = g->n_elem[1];
  d->nz = g->n_elem[2];
  d->E = d->nx * d->ny * d->nz;
  for (int k = 0; k < 3; ++k) {
    d->lower[k] = g->lower[k];
    d->upper[k] = g->upper[k];
    d->h[k] = (g->upper[k] - g->lower[k]) / g->n_elem[k];
  }
  for (int k = 0; k < 6; ++k) d->bc[k] = g->bc[k];
  d->par = *p;
  d->curved = bg != nullptr;
  const int E = d->E;
  // neighbour table (host)
  d->live_h.assign(E, 1);
  if (g->excised)
    for (int e = 0; e < E; ++e) d->live_h[e] = g->excised[e] ? 0 : 1;
  d->nbr_h.assign((size_t)E * 6, -1);
  const int ne[3] = {d->nx, d->ny, d->nz};
  for (int e = 0; e < E; ++e) {
    const int c[3] = {e % d->nx, (e / d->nx) % d->ny, e / (d->nx * d->ny)};
    for (int dd = 0; dd < 3; ++dd)
      for (int s = 0; s < 2; ++s) {
        int cc[3] = {c[0], c[1], c[2]};
        cc[dd] += s ? 1 : -1;
        if (cc[dd] < 0 || cc[dd] >= ne[dd]) {
          if (d->bc[2 * dd + s] != GRFFE_BC_PERIODIC) continue;
          cc[dd] = (cc[dd] + ne[dd]) % ne[dd];
        }
        const int o = cc[0] + d->nx * (cc[1] + d->ny * cc[2]);
        if (!d->live_h[o]) continue;
        d->nbr_h[(size_t)e * 6 + 2 * dd + s] = o;
      }
  }
  hipStream_t st = S(stream);
  const int M = p->tci_M > 0 ? p->tci_M : default_tci_M(d->N);
  d->ops_h = build_ops(d->N, p->filter_a, p->filter_b, M, p->tci_mode);
  DevOps ho{};
  const int n = d->n, m = d->m;
  for (int k = 0; k < n; ++k) ho.w[k] = d->ops_h.w[k];
  for (int k = 0; k < n * n; ++k) {
    ho.D[k] = d->ops_h.D[k];
    ho.F[k] = d->ops_h.F[k];
    ho.L[k] = d->ops_h.L[k];
  }
  for (int k = 0; k < m * n; ++k) {
    ho.P[k] = d->ops_h.P[k];
    ho.R[k] = d->ops_h.R[k];
  }
  const size_t nn = d->nn, mm = d->mm, nf = (size_t)(m + 1) * m * m;
  const size_t regdg = (size_t)NV * E * nn * sizeof(double);
  const size_t regfd = (size_t)NV * E * mm * sizeof(double);
  void* ptr;
#define ALLOC(field, bytes)                        \
  do {                                             \
    if ((rc = dalloc(d, &ptr, (bytes)))) {         \
      grffe_destroy(d);                            \
      return rc;                                   \
    }                                              \
    d->field = reinterpret_cast<decltype(d->field)>(ptr); \
  } while (0)
  ALLOC(nbr, sizeof(int32_t) * E * 6);
  ALLOC(live, E);
  ALLOC(ops, sizeof(DevOps));
  ALLOC(dg.Un, regdg);
  ALLOC(dg.X0, regdg);
  ALLOC(dg.X1, regdg);
  ALLOC(dg.A, regdg);
  ALLOC(fd.Un, regfd);
  ALLOC(fd.X0, regfd);
  ALLOC(fd.X1, regfd);
  ALLOC(fd.A, regfd);
  ALLOC(rep, sizeof(int32_t) * E);
  ALLOC(rep0, sizeof(int32_t) * E);
  ALLOC(troubled, E);
  ALLOC(ratio, sizeof(double) * E);
  ALLOC(w_fd, sizeof(double) * NW * E * mm);
  ALLOC(trace, sizeof(double) * NW * E * 6 * n * n);
  ALLOC(slab, sizeof(double) * NW * E * 6 * 3 * m * m);
  ALLOC(fhat, sizeof(double) * 3 * NV * E * mm);
  double* qdev = nullptr;
  if (d->curved) {
    ALLOC(bg_dg, sizeof(double) * NBG * E * nn);
    ALLOC(bg_fd, sizeof(double) * NBG * E * mm);
    ALLOC(bg_face, sizeof(double) * 3 * NBGF * E * nf);
    if ((rc = dalloc(d, &ptr, sizeof(double) * (m + 1) * n))) {
      grffe_destroy(d);
      return rc;
    }
    qdev = reinterpret_cast<double*>(ptr);
  }
#undef ALLOC
  HIPCHK(hipMemcpyAsync(d->nbr, d->nbr_h.data(), sizeof(int32_t) * E * 6, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d->live, d->live_h.data(), E, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d->ops, &ho, sizeof(DevOps), hipMemcpyHostToDevice, st));
  for (void* r : {(void*)d->dg.Un, (void*)d->dg.X0, (void*)d->dg.X1, (void*)d->dg.A})
    HIPCHK(hipMemsetAsync(r, 0, regdg, st));
  for (void* r : {(void*)d->fd.Un, (void*)d->fd.X0, (void*)d->fd.X1, (void*)d->fd.A})
    HIPCHK(hipMemsetAsync(r, 0, regfd, st));
  HIPCHK(hipMemsetAsync(d->rep, 0, sizeof(int32_t) * E, st));
  HIPCHK(hipMemsetAsync(d->rep0, 0, sizeof(int32_t) * E, st));
  HIPCHK(hipMemsetAsync(d->troubled, 0, E, st));
  HIPCHK(hipMemsetAsync(d->ratio, 0, sizeof(double) * E, st));
  // time step: lambda_max from the background (1 in flat space)
  double lam = 1.0;
  if (d->curved) {
    HIPCHK(hipMemcpyAsync(d->bg_dg, bg, sizeof(double) * NBG * E * nn, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(qdev, d->ops_h.Q.data(), sizeof(double) * (m + 1) * n, hipMemcpyHostToDevice, st));
    KArgs a = make_args(d);
    launch_bg_derive_q(a, d->N, d->bg_fd, d->bg_face, qdev, st);
    HIPCHK(hipGetLastError());
    double* lmax = nullptr;
    HIPCHK(hipMalloc((void**)&lmax, sizeof(double) * E));
    launch_lambda_max(a, d->N, lmax, st);
    std::vector<double> hl(E);
    hipError_t e1 = hipMemcpyAsync(hl.data(), lmax, sizeof(double) * E, hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipStreamSynchronize(st);
    (void)hipFree(lmax);
    if (e1 != hipSuccess || e2 != hipSuccess) {
      grffe_destroy(d);
      return fail(GRFFE_EHIP, "lambda_max reduction failed");
    }
    lam = 0.0;
    for (int e = 0; e < E; ++e) lam = std::fmax(lam, hl[e]);
  }
  d->lambda_max = lam;
  double gap = 1e300;
  for (int k = 0; k < d->N; ++k) gap = std::fmin(gap, d->ops_h.x[k + 1] - d->ops_h.x[k]);
  const double hmin = std::fmin(d->h[0], std::fmin(d->h[1], d->h[2]));
  const double c = p->stab_c > 0.0 ? p->stab_c : ssp_rk3_stability_c();
  d->dt_cfl = p->cfl * gap * hmin / 2.0 / lam * c / 3.0;
  HIPCHK(hipGetLastError());
  *out = d;
  return GRFFE_OK;
}

extern "C" int grffe_set_state(grffe_domain* d, const double* dg, const double* fd, const int32_t* rep, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (!dg || !fd || !rep) return fail(GRFFE_EINVAL, "state pointers must not be NULL");
  hipStream_t st = S(stream);
  HIPCHK(hipMemcpyAsync(d->dg.Un, dg, sizeof(double) * NV * d->E * d->nn, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(d->fd.Un, fd, sizeof(double) * NV * d->E * d->mm, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(d->rep, rep, sizeof(int32_t) * d->E, hipMemcpyDeviceToDevice, st));
  return GRFFE_OK;
}

extern "C" int grffe_get_state(grffe_domain* d, double* dg, double* fd, int32_t* rep, void* stream) {
  if (int rc = check_dom(d)) return rc;
  hipStream_t st = S(stream);
  if (dg) HIPCHK(hipMemcpyAsync(dg, d->dg.Un, sizeof(double) * NV * d->E * d->nn, hipMemcpyDeviceToDevice, st));
  if (fd) HIPCHK(hipMemcpyAsync(fd, d->fd.Un, sizeof(double) * NV * d->E * d->mm, hipMemcpyDeviceToDevice, st));
  if (rep) HIPCHK(hipMemcpyAsync(rep, d->rep, sizeof(int32_t) * d->E, hipMemcpyDeviceToDevice, st));
  return GRFFE_OK;
}

extern "C" int grffe_init_from_fd(grffe_domain* d, const double* u_fd, const uint8_t* forced, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (!u_fd) return fail(GRFFE_EINVAL, "u_fd must not be NULL");
  hipStream_t st = S(stream);
  HIPCHK(hipMemcpyAsync(d->fd.Un, u_fd, sizeof(double) * NV * d->E * d->mm, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemsetAsync(d->dg.Un, 0, sizeof(double) * NV * d->E * d->nn, st));
  std::vector<int32_t> ones(d->E);
  for (int e = 0; e < d->E; ++e) ones[e] = d->live_h[e] ? 1 : 0;
  HIPCHK(hipMemcpyAsync(d->rep, ones.data(), sizeof(int32_t) * d->E, hipMemcpyHostToDevice, st));
  KArgs a = make_args(d);
  const int policy = d->par.hybrid == GRFFE_HYBRID_ADAPTIVE ? 0 : (d->par.hybrid == GRFFE_HYBRID_DG_ONLY ? 1 : 2);
  launch_fd_to_dg_policy(a, d->N, d->curved, policy, forced, st);
  HIPCHK(hipGetLastError());
  // the pageable host copy above must finish before `ones` leaves scope
  HIPCHK(hipStreamSynchronize(st));
  return GRFFE_OK;
}

namespace grffe {
LaunchEvents& armed_launch_events() {
  static thread_local LaunchEvents le;
  return le;
}
}  // namespace grffe

// Arms an event pair for the one kernel launched in its scope when its family is
// the timed one; the launch attaches the events to the kernel's own dispatch.
struct TimedLaunch {
  grffe_domain* d;
  bool on;
  hipStream_t st;
  TimedLaunch(grffe_domain* dd, int family, hipStream_t s) : d(dd), on(dd->timed_family == family), st(s) {
    if (!on) return;
    if (d->ev_used + 2 > d->ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        on = false;
        return;
      }
      d->ev.push_back(a);
      d->ev.push_back(b);
    }
    armed_launch_events().start = d->ev[d->ev_used];
    armed_launch_events().stop = d->ev[d->ev_used + 1];
  }
  ~TimedLaunch() {
    if (!on) return;
    armed_launch_events().start = nullptr;
    armed_launch_events().stop = nullptr;
    d->ev_used += 2;
    d->ev_stream = st;
  }
};

// One substep (or a pure right-hand side evaluation when mode == MODE_RHS).
static void run_substep(grffe_domain* d, KArgs& a, int mode, hipStream_t st) {
  const int N = d->N;
  const bool cv = d->curved;
  { TimedLaunch t(d, 4, st); launch_fd_stage(a, N, cv, mode, mode != MODE_RHS, st); }
  { TimedLaunch t(d, 5, st); launch_fd_trace(a, N, st); }
  { TimedLaunch t(d, 1, st); launch_dg_substep(a, N, cv, mode, st); }
  { TimedLaunch t(d, 6, st); launch_dg_slab(a, N, cv, mode, st); }
  if (mode != MODE_RHS && a.hybrid == GRFFE_HYBRID_ADAPTIVE) {
    { TimedLaunch t(d, 7, st); launch_project_troubled(a, N, cv, mode, st); }
  }
  { TimedLaunch t(d, 2, st); launch_fd_flux(a, N, cv, st); }
  { TimedLaunch t(d, 3, st); launch_fd_update(a, N, cv, mode, st); }
}

extern "C" int grffe_timing_enable(grffe_domain* d, int family) {
  if (int rc = check_dom(d)) return rc;
  if (family < 0 || family > 8) return fail(GRFFE_EINVAL, "unknown kernel family");
  d->timed_family = family;
  d->ev_used = 0;
  return GRFFE_OK;
}

extern "C" int grffe_timing_read(grffe_domain* d, double* total_ms, int64_t* launches) {
  if (int rc = check_dom(d)) return rc;
  double tot = 0.0;
  if (d->ev_used) {
    HIPCHK(hipStreamSynchronize(d->ev_stream));
    for (size_t k = 0; k < d->ev_used; k += 2) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, d->ev[k], d->ev[k + 1]));
      tot += ms;
    }
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (int64_t)(d->ev_used / 2);
  d->ev_used = 0;
  return GRFFE_OK;
}

extern "C" int grffe_rhs(grffe_domain* d, const double* dg, const double* fd, const int32_t* rep, double* ddg,
                         double* dfd, int parts, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (!dg || !fd || !rep || !ddg || !dfd) return fail(GRFFE_EINVAL, "rhs pointers must not be NULL");
  if (parts < 1 || parts > 3) return fail(GRFFE_EINVAL, "parts must be 1, 2 or 3");
  hipStream_t st = S(stream);
  KArgs a = make_args(d);
  a.dg.Un = const_cast<double*>(dg);
  a.fd.Un = const_cast<double*>(fd);
  a.rep0 = const_cast<int32_t*>(rep);
  a.out_dg = ddg;
  a.out_fd = dfd;
  a.parts = parts;
  HIPCHK(hipMemsetAsync(d->troubled, 0, d->E, st));
  run_substep(d, a, MODE_RHS, st);
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}

extern "C" int grffe_step(grffe_domain* d, int n_steps, double dt, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (n_steps < 0) return fail(GRFFE_EINVAL, "n_steps must be >= 0");
  hipStream_t st = S(stream);
  KArgs a = make_args(d);
  if (dt > 0.0) a.dt = dt;
  for (int it = 0; it < n_steps; ++it) {
    run_substep(d, a, MODE_SUB1, st);
    run_substep(d, a, MODE_SUB2, st);
    run_substep(d, a, MODE_SUB3, st);
    if (a.hybrid == GRFFE_HYBRID_ADAPTIVE) {
      TimedLaunch t(d, 8, st);
      launch_fd_to_dg(a, d->N, d->curved, 0, st);
    }
  }
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}

extern "C" int grffe_tci(grffe_domain* d, const double* dg, const double* fd, const int32_t* rep, uint8_t* troubled,
                         double* ratio, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (!dg || !fd || !rep || !troubled) return fail(GRFFE_EINVAL, "tci pointers must not be NULL");
  KArgs a = make_args(d);
  launch_tci(a, d->N, d->curved, dg, fd, rep, troubled, ratio, S(stream));
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}

extern "C" int grffe_project_dg_to_fd(grffe_domain* d, const double* u_dg, double* u_fd, const int32_t* elems,
                                      int32_t n, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (n < 0) return fail(GRFFE_EINVAL, "n must be >= 0");
  if (n == 0) return GRFFE_OK;
  if (!u_dg || !u_fd || !elems) return fail(GRFFE_EINVAL, "transfer pointers must not be NULL");
  KArgs a = make_args(d);
  launch_transfer(a, d->N, 1, u_dg, u_fd, n, S(stream));
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}

extern "C" int grffe_reconstruct_fd_to_dg(grffe_domain* d, const double* u_fd, double* u_dg, const int32_t* elems,
                                          int32_t n, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (n < 0) return fail(GRFFE_EINVAL, "n must be >= 0");
  if (n == 0) return GRFFE_OK;
  if (!u_dg || !u_fd || !elems) return fail(GRFFE_EINVAL, "transfer pointers must not be NULL");
  KArgs a = make_args(d);
  launch_transfer(a, d->N, 0, u_fd, u_dg, n, S(stream));
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}

extern "C" int grffe_get_dt(grffe_domain* d, double* dt) {
  if (int rc = check_dom(d)) return rc;
  if (!dt) return fail(GRFFE_EINVAL, "dt must not be NULL");
  *dt = d->dt_cfl;
  return GRFFE_OK;
}

extern "C" int grffe_get_counts(grffe_domain* d, int32_t* n_dg, int32_t* n_fd) {
  if (int rc = check_dom(d)) return rc;
  std::vector<int32_t> r(d->E);
  HIPCHK(hipMemcpy(r.data(), d->rep, sizeof(int32_t) * d->E, hipMemcpyDeviceToHost));
  int a = 0, b = 0;
  for (int e = 0; e < d->E; ++e) {
    if (!d->live_h[e]) continue;
    if (r[e] == 1) ++b;
    else ++a;
  }
  if (n_dg) *n_dg = a;
  if (n_fd) *n_fd = b;
  return GRFFE_OK;
}

extern "C" int grffe_operator(int degree, int which, double* out, int capacity) {
  if (degree < 3 || degree > MAX_DEG) return fail(GRFFE_EINVAL, "degree must be in [3, 7]");
  grffe_params p;
  grffe_default_params(&p);
  Ops1D o = build_ops(degree, p.filter_a, p.filter_b, default_tci_M(degree), 2);
  const std::vector<double>* v = nullptr;
  switch (which) {
    case 0: v = &o.x; break;
    case 1: v = &o.w; break;
    case 2: v = &o.D; break;
    case 3: v = &o.F; break;
    case 4: v = &o.L; break;
    case 5: v = &o.P; break;
    case 6: v = &o.R; break;
    case 7: v = &o.Q; break;
    default: return fail(GRFFE_EINVAL, "unknown operator");
  }
  const int cnt = (int)v->size();
  if (out) {
    if (capacity < cnt) return fail(GRFFE_EINVAL, "capacity too small");
    std::memcpy(out, v->data(), sizeof(double) * cnt);
  }
  return cnt;
}

