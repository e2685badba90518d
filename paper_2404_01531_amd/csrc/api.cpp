// C ABI of the GRFFE DG-FD hot path: domain set-up, state transfer and the
// orchestration of one IMEX-SSP3(4,3,3) step with the hybrid DG-FD control.
#include <hip/hip_runtime.h>

#include <algorithm>
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

// A domain whose right-hand side can be evaluated: every Dirichlet face has its state.
static int check_ready(grffe_domain* d) {
  if (int rc = check_dom(d)) return rc;
  if (d->bc_missing)
    return fail(GRFFE_EINVAL, "the domain has Dirichlet faces: set their exterior state (grffe_set_boundary_state)");
  return GRFFE_OK;
}

extern "C" const char* grffe_last_error(void) { return g_err.c_str(); }

namespace grffe {
// Status and message of a failure, for the entry points defined in other sources.
int set_error(int code, const char* msg) { return fail(code, msg); }
}  // namespace grffe

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
  a.eh = d->eh;
  a.edt = d->edt;
  a.nbr = d->nbr;
  a.bstate = d->bstate;
  a.bfield_dg = d->bfield_dg;
  a.bfield_fd = d->bfield_fd;
  a.live = d->live;
  a.bg_dg = d->bg_dg;
  a.bg_dg32 = d->bg_dg32;
  a.bg_fd = d->bg_fd;
  a.bg_face = d->bg_face;
  a.ops = d->ops;
  a.jinv = d->jinv;
  a.fnode = d->fnode;
  a.nface = d->nface;
  a.fcell = d->fcell;
  a.jinv_fd = d->jinv_fd;
  a.nu_face = d->nu_face;
  a.dg = d->dg;
  a.fd = d->fd;
  a.rep0 = d->rep0;
  a.rep = d->rep;
  a.troubled = d->troubled;
  a.force = d->force_on ? d->force : nullptr;
  a.contraction = d->contraction;
  a.ratio = d->ratio;
  a.w_fd = d->w_fd;
  a.trace = d->trace;
  a.slab = d->slab;
  a.fhat = d->fhat;
  a.dt = 0.0;
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
  a.precision = d->par.precision;
  a.weno_eps = d->par.weno_eps;
  a.ff_margin = d->par.ff_margin;
  a.fd_list = d->fd_list;
  a.fd_count = d->fd_count;
  a.sub = 0;
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
  for (auto& v : d->ev) {
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
    v.clear();
  }
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
  if (g->degree < 3 || g->degree > MAX_DEG) return fail(GRFFE_EINVAL, "degree must be in [3, 9]");
  for (int k = 0; k < 3; ++k) {
    if (g->n_elem[k] < 1) return fail(GRFFE_EINVAL, "n_elem must be positive");
    if (!(g->upper[k] > g->lower[k])) return fail(GRFFE_EINVAL, "upper must exceed lower");
  }
  for (int k = 0; k < 6; ++k)
    if (g->bc[k] != GRFFE_BC_PERIODIC && g->bc[k] != GRFFE_BC_NO_INCOMING_POYNTING && g->bc[k] != GRFFE_BC_DIRICHLET)
      return fail(GRFFE_EINVAL, "unknown boundary kind");
  for (int d = 0; d < 3; ++d)
    if ((g->bc[2 * d] == GRFFE_BC_PERIODIC) != (g->bc[2 * d + 1] == GRFFE_BC_PERIODIC))
      return fail(GRFFE_EINVAL, "periodic faces must come in pairs");
  if (p->precision != GRFFE_PRECISION_FP64 && p->precision != GRFFE_PRECISION_MIXED)
    return fail(GRFFE_EUNSUPPORTED, "precision must be GRFFE_PRECISION_FP64 or GRFFE_PRECISION_MIXED");
  if (p->hybrid < 0 || p->hybrid > 2) return fail(GRFFE_EINVAL, "hybrid must be 0, 1 or 2");
  if (p->fd_order != 2 && p->fd_order != 4) return fail(GRFFE_EINVAL, "fd_order must be 2 or 4");
  if (p->tci_mode != 1 && p->tci_mode != 2) return fail(GRFFE_EINVAL, "tci_mode must be 1 or 2");
  if (!(p->cfl > 0.0)) return fail(GRFFE_EINVAL, "cfl must be positive");
  if (p->eta < 0.0 || p->kappa_psi < 0.0 || p->kappa_phi < 0.0) return fail(GRFFE_EINVAL, "negative rates");
  const int M = p->tci_M > 0 ? p->tci_M : default_tci_M(g->degree);
  if (M < 1 || M > g->degree) return fail(GRFFE_EINVAL, "tci_M out of range");
  return GRFFE_OK;
}

// Build a domain over one or more grids of the same degree: the elements of the
// grids are concatenated (grid k occupies elements off_k .. off_k + E_k - 1) and
// every grid keeps its own neighbour table, element widths and time step.
// A shell (sg non-null) is built as one pseudo-grid of E elements whose neighbour
// table, map and time step come from the shell's geometry.
static int build_pool(const grffe_grid* const* grids, int count, const grffe_params* p, const double* const* bgs,
                      hipStream_t st, grffe_domain** out, const ShellGeom* sg = nullptr,
                      const grffe_shell* shell = nullptr) {
  *out = nullptr;
  if (count < 1) return fail(GRFFE_EINVAL, "no grid");
  for (int k = 0; k < count; ++k)
    if (int rc = validate(grids[k], p)) return rc;
  const bool curved = bgs && bgs[0] != nullptr;
  for (int k = 0; k < count; ++k) {
    if (grids[k]->degree != grids[0]->degree) return fail(GRFFE_EINVAL, "a pool holds one degree");
    if ((bgs && bgs[k] != nullptr) != curved) return fail(GRFFE_EINVAL, "a pool is all flat or all curved");
  }
  int rc = 0;
  grffe_domain* d = new grffe_domain();
  const grffe_grid* g0 = grids[0];
  d->N = g0->degree;
  d->n = d->N + 1;
  d->m = 2 * d->N + 1;
  d->nn = d->n * d->n * d->n;
  d->mm = d->m * d->m * d->m;
  d->nx = g0->n_elem[0];
  d->ny = g0->n_elem[1];
  d->nz = g0->n_elem[2];
  for (int k = 0; k < 3; ++k) {
    d->lower[k] = g0->lower[k];
    d->upper[k] = g0->upper[k];
    d->h[k] = (g0->upper[k] - g0->lower[k]) / g0->n_elem[k];
  }
  for (int k = 0; k < 6; ++k) {
    d->bc[k] = g0->bc[k];
    if (d->bc[k] == GRFFE_BC_DIRICHLET) d->bc_missing |= 1 << k;
  }
  d->par = *p;
  d->curved = curved;
  int E = 0;
  for (int k = 0; k < count; ++k) {
    const grffe_grid* g = grids[k];
    grffe_part pt{};
    pt.off = E;
    pt.nx = g->n_elem[0];
    pt.ny = g->n_elem[1];
    pt.nz = g->n_elem[2];
    pt.E = pt.nx * pt.ny * pt.nz;
    for (int q = 0; q < 3; ++q) pt.h[q] = (g->upper[q] - g->lower[q]) / g->n_elem[q];
    d->parts.push_back(pt);
    E += pt.E;
  }
  d->E = E;
  // neighbour tables (host), element widths
  d->live_h.assign(E, 1);
  d->nbr_h.assign((size_t)E * 6, -1);
  d->eh_h.assign((size_t)E * 3, 0.0);
  for (int k = 0; k < count && !sg; ++k) {
    const grffe_grid* g = grids[k];
    const grffe_part& pt = d->parts[k];
    if (g->excised)
      for (int e = 0; e < pt.E; ++e) d->live_h[pt.off + e] = g->excised[e] ? 0 : 1;
    const int ne[3] = {pt.nx, pt.ny, pt.nz};
    for (int e = 0; e < pt.E; ++e) {
      for (int q = 0; q < 3; ++q) d->eh_h[3 * (pt.off + e) + q] = pt.h[q];
      const int c[3] = {e % pt.nx, (e / pt.nx) % pt.ny, e / (pt.nx * pt.ny)};
      for (int dd = 0; dd < 3; ++dd)
        for (int sd = 0; sd < 2; ++sd) {
          int cc[3] = {c[0], c[1], c[2]};
          cc[dd] += sd ? 1 : -1;
          if (cc[dd] < 0 || cc[dd] >= ne[dd]) {
            if (g->bc[2 * dd + sd] == GRFFE_BC_DIRICHLET) {
              // slot of the face's exterior state (Dirichlet faces exist on single-grid domains only)
              d->nbr_h[(size_t)(pt.off + e) * 6 + 2 * dd + sd] = -2 - (2 * dd + sd);
              continue;
            }
            if (g->bc[2 * dd + sd] != GRFFE_BC_PERIODIC) continue;
            cc[dd] = (cc[dd] + ne[dd]) % ne[dd];
          }
          const int o = cc[0] + pt.nx * (cc[1] + pt.ny * cc[2]);
          if (!d->live_h[pt.off + o]) continue;
          d->nbr_h[(size_t)(pt.off + e) * 6 + 2 * dd + sd] = pt.off + o;
        }
    }
  }
  if (sg) {
    d->mapped = true;
    d->nbr_h = sg->nbr;
    for (int k = 0; k < 6; ++k) d->bc[k] = GRFFE_BC_NO_INCOMING_POYNTING;
    d->bc_missing = 0;
    if (shell->bc_inner == GRFFE_BC_DIRICHLET) d->bc_missing |= 1 << 4;
    if (shell->bc_outer == GRFFE_BC_DIRICHLET) d->bc_missing |= 1 << 5;
  }
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
  ALLOC(bstate, sizeof(double) * 6 * NV);
  ALLOC(live, E);
  ALLOC(eh, sizeof(double) * E * 3);
  ALLOC(edt, sizeof(double) * E);
  ALLOC(ops, sizeof(DevOps));
  ALLOC(dg.Un, regdg);
  ALLOC(dg.X0, regdg);
  ALLOC(dg.X1, regdg);
  ALLOC(dg.A, regdg);
  ALLOC(dg.K, (size_t)2 * NK * E * nn * sizeof(double));
  ALLOC(fd.Un, regfd);
  ALLOC(fd.X0, regfd);
  ALLOC(fd.X1, regfd);
  ALLOC(fd.A, regfd);
  ALLOC(fd.K, (size_t)2 * NK * E * mm * sizeof(double));
  ALLOC(rep, sizeof(int32_t) * E);
  ALLOC(rep0, sizeof(int32_t) * E);
  ALLOC(troubled, E);
  ALLOC(ratio, sizeof(double) * E);
  ALLOC(w_fd, sizeof(double) * NW * E * mm);
  ALLOC(trace, sizeof(double) * NW * E * 6 * n * n);
  ALLOC(slab, sizeof(double) * NW * E * 6 * 3 * m * m);
  ALLOC(fhat, sizeof(double) * 3 * NV * E * mm);
  ALLOC(fd_list, sizeof(int32_t) * E);
  ALLOC(fd_count, sizeof(int32_t) * 4);
  if (sg) {
    ALLOC(jinv, sizeof(double) * 9 * E * nn);
    ALLOC(fnode, sizeof(int32_t) * E * 6 * n * n);
    if (!sg->jinv_fd.empty()) {
      ALLOC(nface, sizeof(int32_t) * E * 6);
      ALLOC(fcell, sizeof(int32_t) * E * 6 * m * m);
      ALLOC(jinv_fd, sizeof(double) * 9 * E * mm);
      ALLOC(nu_face, sizeof(double) * 9 * E * nf);
    }
  }
  double* qdev = nullptr;
  if (d->curved) {
    ALLOC(bg_dg, sizeof(double) * NBG * E * nn);
    ALLOC(bg_fd, sizeof(double) * NBG * E * mm);
    ALLOC(bg_face, sizeof(double) * 3 * NBGF * E * nf);
    if (p->precision == GRFFE_PRECISION_MIXED) ALLOC(bg_dg32, sizeof(float) * NBG * E * nn);
    if ((rc = dalloc(d, &ptr, sizeof(double) * (m + 1) * n))) {
      grffe_destroy(d);
      return rc;
    }
    qdev = reinterpret_cast<double*>(ptr);
  }
#undef ALLOC
#define CHK(expr)                                                                            \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) {                                                                  \
      grffe_destroy(d);                                                                      \
      return fail(GRFFE_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));            \
    }                                                                                        \
  } while (0)
  CHK(hipMemcpyAsync(d->nbr, d->nbr_h.data(), sizeof(int32_t) * E * 6, hipMemcpyHostToDevice, st));
  CHK(hipMemsetAsync(d->bstate, 0, sizeof(double) * 6 * NV, st));
  CHK(hipMemcpyAsync(d->live, d->live_h.data(), E, hipMemcpyHostToDevice, st));
  CHK(hipMemcpyAsync(d->eh, d->eh_h.data(), sizeof(double) * E * 3, hipMemcpyHostToDevice, st));
  CHK(hipMemcpyAsync(d->ops, &ho, sizeof(DevOps), hipMemcpyHostToDevice, st));
  for (void* r : {(void*)d->dg.Un, (void*)d->dg.X0, (void*)d->dg.X1, (void*)d->dg.A})
    CHK(hipMemsetAsync(r, 0, regdg, st));
  CHK(hipMemsetAsync(d->dg.K, 0, (size_t)2 * NK * E * nn * sizeof(double), st));
  for (void* r : {(void*)d->fd.Un, (void*)d->fd.X0, (void*)d->fd.X1, (void*)d->fd.A})
    CHK(hipMemsetAsync(r, 0, regfd, st));
  CHK(hipMemsetAsync(d->fd.K, 0, (size_t)2 * NK * E * mm * sizeof(double), st));
  CHK(hipMemsetAsync(d->rep, 0, sizeof(int32_t) * E, st));
  CHK(hipMemsetAsync(d->rep0, 0, sizeof(int32_t) * E, st));
  CHK(hipMemsetAsync(d->troubled, 0, E, st));
  CHK(hipMemsetAsync(d->ratio, 0, sizeof(double) * E, st));
  CHK(hipMemsetAsync(d->fd_count, 0, sizeof(int32_t) * 4, st));
  if (sg) {
    CHK(hipMemcpyAsync(d->jinv, sg->jinv.data(), sizeof(double) * 9 * E * nn, hipMemcpyHostToDevice, st));
    CHK(hipMemcpyAsync(d->fnode, sg->fnode.data(), sizeof(int32_t) * E * 6 * n * n, hipMemcpyHostToDevice, st));
    if (!sg->jinv_fd.empty()) {
      CHK(hipMemcpyAsync(d->nface, sg->nface.data(), sizeof(int32_t) * E * 6, hipMemcpyHostToDevice, st));
      CHK(hipMemcpyAsync(d->fcell, sg->fcell.data(), sizeof(int32_t) * E * 6 * m * m, hipMemcpyHostToDevice, st));
      CHK(hipMemcpyAsync(d->jinv_fd, sg->jinv_fd.data(), sizeof(double) * 9 * E * mm, hipMemcpyHostToDevice, st));
      CHK(hipMemcpyAsync(d->nu_face, sg->nu_face.data(), sizeof(double) * 9 * E * nf, hipMemcpyHostToDevice, st));
      // the host tables are only needed for the copies, which must finish first
      CHK(hipStreamSynchronize(st));
    }
  }
  // time step per grid: lambda_max from the background (1 in flat space)
  for (auto& pt : d->parts) pt.lambda_max = 1.0;
  if (d->curved && sg) {
    // lambda_max = max over the nodes of alpha + |beta|_gamma (the largest
    // characteristic speed over all directions), from a host copy of alpha, beta, gamma
    CHK(hipMemcpyAsync(d->bg_dg, bgs[0], sizeof(double) * NBG * E * nn, hipMemcpyDeviceToDevice, st));
    std::vector<double> hb((size_t)10 * E * nn);
    CHK(hipMemcpyAsync(hb.data(), bgs[0], sizeof(double) * 10 * E * nn, hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    double lam = 0.0;
    const size_t P = (size_t)E * nn;
    for (size_t q = 0; q < P; ++q) {
      const double al = hb[q], b[3] = {hb[P + q], hb[2 * P + q], hb[3 * P + q]};
      const double g[6] = {hb[4 * P + q], hb[5 * P + q], hb[6 * P + q], hb[7 * P + q], hb[8 * P + q], hb[9 * P + q]};
      const double bb = g[0] * b[0] * b[0] + g[3] * b[1] * b[1] + g[5] * b[2] * b[2] +
                        2.0 * (g[1] * b[0] * b[1] + g[2] * b[0] * b[2] + g[4] * b[1] * b[2]);
      const double v = al + std::sqrt(std::fmax(bb, 0.0));
      if (!std::isfinite(v)) {
        grffe_destroy(d);
        return fail(GRFFE_EINVAL, "the background holds non-finite values");
      }
      lam = std::fmax(lam, v);
    }
    d->parts[0].lambda_max = lam;
    CHK(hipMemcpyAsync(qdev, d->ops_h.Q.data(), sizeof(double) * (m + 1) * n, hipMemcpyHostToDevice, st));
    KArgs a = make_args(d);
    launch_bg_derive_q(a, d->N, d->bg_fd, d->bg_face, qdev, st);
    CHK(hipGetLastError());
  } else if (d->curved) {
    for (int k = 0; k < count; ++k) {
      const grffe_part& pt = d->parts[k];
      CHK(hipMemcpy2DAsync(d->bg_dg + (size_t)pt.off * nn, sizeof(double) * E * nn, bgs[k],
                           sizeof(double) * pt.E * nn, sizeof(double) * pt.E * nn, NBG, hipMemcpyDeviceToDevice, st));
    }
    if (d->bg_dg32) launch_to_float(d->bg_dg, d->bg_dg32, (size_t)NBG * E * nn, st);
    CHK(hipMemcpyAsync(qdev, d->ops_h.Q.data(), sizeof(double) * (m + 1) * n, hipMemcpyHostToDevice, st));
    KArgs a = make_args(d);
    launch_bg_derive_q(a, d->N, d->bg_fd, d->bg_face, qdev, st);
    CHK(hipGetLastError());
    double* lmax = nullptr;
    CHK(hipMalloc((void**)&lmax, sizeof(double) * E));
    launch_lambda_max(a, d->N, lmax, st);
    std::vector<double> hl(E);
    hipError_t e1 = hipMemcpyAsync(hl.data(), lmax, sizeof(double) * E, hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipStreamSynchronize(st);
    (void)hipFree(lmax);
    if (e1 != hipSuccess || e2 != hipSuccess) {
      grffe_destroy(d);
      return fail(GRFFE_EHIP, "lambda_max reduction failed");
    }
    for (auto& pt : d->parts) {
      pt.lambda_max = 0.0;
      for (int e = pt.off; e < pt.off + pt.E; ++e) pt.lambda_max = std::fmax(pt.lambda_max, hl[e]);
    }
  }
  double gap = 1e300;
  for (int k = 0; k < d->N; ++k) gap = std::fmin(gap, d->ops_h.x[k + 1] - d->ops_h.x[k]);
  const double c = p->stab_c > 0.0 ? p->stab_c : ssp_rk3_stability_c();
  d->edt_h.assign(E, 0.0);
  for (auto& pt : d->parts) {
    const double hmin = std::fmin(pt.h[0], std::fmin(pt.h[1], pt.h[2]));
    // Eq. (spectre DG CFL condition): (dx)_min is gap * h / 2 on affine elements
    const double dxmin = sg ? sg->dx_min : gap * hmin / 2.0;
    pt.dt = p->cfl * dxmin / pt.lambda_max * c / 3.0;
    for (int e = pt.off; e < pt.off + pt.E; ++e) d->edt_h[e] = pt.dt;
  }
  d->dt_cfl = d->parts[0].dt;
  d->lambda_max = d->parts[0].lambda_max;
  CHK(hipMemcpyAsync(d->edt, d->edt_h.data(), sizeof(double) * E, hipMemcpyHostToDevice, st));
  CHK(hipStreamSynchronize(st));
  CHK(hipGetLastError());
#undef CHK
  *out = d;
  return GRFFE_OK;
}

extern "C" int grffe_init_domain(const grffe_grid* g, const grffe_params* p, const double* bg, void* stream,
                                 grffe_domain** out) {
  if (!out) return fail(GRFFE_EINVAL, "out must not be NULL");
  const grffe_grid* gs[1] = {g};
  const double* bs[1] = {bg};
  return build_pool(gs, 1, p, bs, S(stream), out);
}

extern "C" int grffe_shell_points(const grffe_shell* s, int32_t fd, double* xyz) {
  std::string err;
  if (int rc = shell_validate(s, err)) return fail(rc, err);
  if (!xyz) return fail(GRFFE_EINVAL, "xyz must not be NULL");
  std::vector<double> pts;
  shell_points(*s, fd != 0, pts);
  std::copy(pts.begin(), pts.end(), xyz);
  return GRFFE_OK;
}

extern "C" int grffe_init_shell(const grffe_shell* s, const grffe_params* p, const double* bg, void* stream,
                                grffe_domain** out) {
  if (!out) return fail(GRFFE_EINVAL, "out must not be NULL");
  *out = nullptr;
  std::string err;
  if (int rc = shell_validate(s, err)) return fail(rc, err);
  if (!p) return fail(GRFFE_EINVAL, "params must not be NULL");
  if (p->precision != GRFFE_PRECISION_FP64) return fail(GRFFE_EUNSUPPORTED, "shells run in FP64");
  if (p->hybrid != GRFFE_HYBRID_DG_ONLY && p->fd_order != 2)
    return fail(GRFFE_EUNSUPPORTED, "FD subcells on curved elements are second order (fd_order = 2)");
  ShellGeom g;
  if (int rc = shell_geometry(*s, g, err)) return fail(rc, err);
  if (p->hybrid != GRFFE_HYBRID_DG_ONLY)
    if (int rc = shell_fd_geometry(*s, g, err)) return fail(rc, err);
  grffe_grid pseudo{};
  pseudo.n_elem[0] = g.E;
  pseudo.n_elem[1] = pseudo.n_elem[2] = 1;
  for (int k = 0; k < 3; ++k) {
    pseudo.lower[k] = 0.0;
    pseudo.upper[k] = 1.0;
  }
  pseudo.degree = s->degree;
  for (int k = 0; k < 6; ++k) pseudo.bc[k] = GRFFE_BC_NO_INCOMING_POYNTING;
  const grffe_grid* gs[1] = {&pseudo};
  const double* bs[1] = {bg};
  return build_pool(gs, 1, p, bs, S(stream), out, &g, s);
}

extern "C" int grffe_set_boundary_state(grffe_domain* d, const double* state, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (d->mapped) return fail(GRFFE_EUNSUPPORTED, "shells take per-node exterior states (grffe_set_boundary_field)");
  if (!state) return fail(GRFFE_EINVAL, "state must not be NULL");
  for (int k = 0; k < 6 * NV; ++k)
    if (!std::isfinite(state[k])) return fail(GRFFE_EINVAL, "boundary state must be finite");
  hipStream_t st = S(stream);
  HIPCHK(hipMemcpyAsync(d->bstate, state, sizeof(double) * 6 * NV, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  d->bc_missing = 0;
  return GRFFE_OK;
}

extern "C" int grffe_set_boundary_field(grffe_domain* d, const double* ext_dg, const double* ext_fd, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (!ext_dg || (!ext_fd && !d->mapped)) return fail(GRFFE_EINVAL, "boundary field pointers must not be NULL");
  if (!ext_fd && d->mapped && d->par.hybrid != GRFFE_HYBRID_DG_ONLY)
    return fail(GRFFE_EINVAL, "a shell whose elements may go to FD needs the ghost-cell states (ext_fd)");
  if (d->parts.size() != 1) return fail(GRFFE_EUNSUPPORTED, "boundary fields are set on single domains");
  const size_t ndg = (size_t)NV * d->E * 6 * d->n * d->n;
  const size_t nfd = (size_t)NV * d->E * 6 * 3 * d->m * d->m;
  if (!d->bfield_dg) {
    void* p1 = nullptr;
    void* p2 = nullptr;
    if (int rc = dalloc(d, &p1, sizeof(double) * ndg)) return rc;
    if (int rc = dalloc(d, &p2, sizeof(double) * nfd)) return rc;
    d->bfield_dg = static_cast<double*>(p1);
    d->bfield_fd = static_cast<double*>(p2);
  }
  hipStream_t st = S(stream);
  HIPCHK(hipMemcpyAsync(d->bfield_dg, ext_dg, sizeof(double) * ndg, hipMemcpyDeviceToDevice, st));
  if (ext_fd) HIPCHK(hipMemcpyAsync(d->bfield_fd, ext_fd, sizeof(double) * nfd, hipMemcpyDeviceToDevice, st));
  d->bc_missing = 0;
  return GRFFE_OK;
}

extern "C" int grffe_set_conductor(grffe_domain* d, const double* centre, double radius, double omega,
                                   void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (d->parts.size() != 1) return fail(GRFFE_EUNSUPPORTED, "the conductor is set on single domains");
  if (d->mapped) return fail(GRFFE_EUNSUPPORTED, "the conductor is not available on shells");
  if (!std::isfinite(radius) || !std::isfinite(omega)) return fail(GRFFE_EINVAL, "radius and omega must be finite");
  if (radius <= 0.0) {
    d->cond_count = 0;
    return GRFFE_OK;
  }
  if (!centre) return fail(GRFFE_EINVAL, "centre must not be NULL");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(centre[k])) return fail(GRFFE_EINVAL, "centre must be finite");
  if (!d->cond_list) {
    void* p1 = nullptr;
    void* p2 = nullptr;
    void* p3 = nullptr;
    if (int rc = dalloc(d, &p1, sizeof(int32_t) * d->E)) return rc;
    if (int rc = dalloc(d, &p2, sizeof(double) * 3 * d->E)) return rc;
    if (int rc = dalloc(d, &p3, sizeof(double) * (MAX_DEG + 1))) return rc;
    d->cond_list = static_cast<int32_t*>(p1);
    d->cond_corner = static_cast<double*>(p2);
    d->cond_ref = static_cast<double*>(p3);
  }
  // every element whose box comes within the radius (slightly enlarged, so that no
  // element holding a point of the sphere is missed; the kernel tests each point)
  std::vector<int32_t> list;
  std::vector<double> corner;
  const double reach = radius * (1.0 + 1e-9);
  for (int e = 0; e < d->E; ++e) {
    const int c[3] = {e % d->nx, (e / d->nx) % d->ny, e / (d->nx * d->ny)};
    double dist2 = 0.0, lo[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = d->lower[k] + c[k] * d->h[k];
      const double q = std::min(std::max(centre[k], lo[k]), lo[k] + d->h[k]);
      dist2 += (q - centre[k]) * (q - centre[k]);
    }
    if (dist2 > reach * reach) continue;
    list.push_back(e);
    for (int k = 0; k < 3; ++k) corner.push_back(lo[k]);
  }
  hipStream_t st = S(stream);
  if (!list.empty()) {
    HIPCHK(hipMemcpyAsync(d->cond_list, list.data(), sizeof(int32_t) * list.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d->cond_corner, corner.data(), sizeof(double) * corner.size(), hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipMemcpyAsync(d->cond_ref, d->ops_h.x.data(), sizeof(double) * d->n, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int k = 0; k < 3; ++k) d->cond_c[k] = centre[k];
  d->cond_r = radius;
  d->cond_omega = omega;
  d->cond_count = (int)list.size();
  return GRFFE_OK;
}

extern "C" int grffe_set_contraction(grffe_domain* d, int engine) {
  if (int rc = check_dom(d)) return rc;
  if (engine != GRFFE_CONTRACTION_VALU && engine != GRFFE_CONTRACTION_MFMA)
    return fail(GRFFE_EINVAL, "engine must be GRFFE_CONTRACTION_VALU or GRFFE_CONTRACTION_MFMA");
  if (d->mapped && engine != GRFFE_CONTRACTION_VALU)
    return fail(GRFFE_EUNSUPPORTED, "shells contract on the VALU");
  d->contraction = engine;
  return GRFFE_OK;
}

extern "C" int grffe_force_flags(grffe_domain* d, const uint8_t* mask, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (!mask) {
    d->force_on = false;
    return GRFFE_OK;
  }
  if (!d->force) {
    void* p = nullptr;
    if (int rc = dalloc(d, &p, (size_t)3 * d->E)) return rc;
    d->force = static_cast<uint8_t*>(p);
  }
  HIPCHK(hipMemcpyAsync(d->force, mask, (size_t)3 * d->E, hipMemcpyDeviceToDevice, S(stream)));
  d->force_on = true;
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

// Start-up from the FD data already in d->fd.Un: every live element is reconstructed
// to DG and the hybrid policy decides which stay FD.
static int init_pool_from_fd(grffe_domain* d, const uint8_t* forced, hipStream_t st) {
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

extern "C" int grffe_init_from_fd(grffe_domain* d, const double* u_fd, const uint8_t* forced, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (!u_fd) return fail(GRFFE_EINVAL, "u_fd must not be NULL");
  hipStream_t st = S(stream);
  HIPCHK(hipMemcpyAsync(d->fd.Un, u_fd, sizeof(double) * NV * d->E * d->mm, hipMemcpyDeviceToDevice, st));
  return init_pool_from_fd(d, forced, st);
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
  int fam;
  bool on;
  hipStream_t st;
  TimedLaunch(grffe_domain* dd, int family, hipStream_t s)
      : d(dd), fam(family), on(dd->timing_now && ((dd->timed_mask >> family) & 1) != 0), st(s) {
    if (!on) return;
    auto& ev = d->ev[fam];
    if (d->ev_used[fam] + 2 > ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        on = false;
        return;
      }
      ev.push_back(a);
      ev.push_back(b);
    }
    armed_launch_events().start = ev[d->ev_used[fam]];
    armed_launch_events().stop = ev[d->ev_used[fam] + 1];
  }
  ~TimedLaunch() {
    if (!on) return;
    armed_launch_events().start = nullptr;
    armed_launch_events().stop = nullptr;
    d->ev_used[fam] += 2;
    d->ev_stream = st;
  }
};

namespace grffe {
void launch_conductor(const KArgs& a, int N, bool curved, const CondArgs& c, int mode, hipStream_t s);
}  // namespace grffe

// One substep (or a pure right-hand side evaluation when mode == MODE_RHS).
static void run_substep(grffe_domain* d, KArgs& a, int mode, hipStream_t st) {
  const int N = d->N;
  const bool cv = d->curved;
  // one FD work list per step (counter 0, emptied by the pre-stage pass): substep 1
  // builds it from the representation at the step start, the DG substeps append the
  // elements they flag, so it holds the FD elements at the start of every substep;
  // the FD update of substeps 1 and 2 writes the next substep's stage values
  a.sub = mode == MODE_RHS ? 3 : 0;
  if (d->mapped && a.hybrid == GRFFE_HYBRID_DG_ONLY) {
    // every element on DG: the one fused kernel per substep
    TimedLaunch t(d, 1, st);
    launch_dg_mapped(a, N, cv, mode, false, st);
    return;
  }
  if (d->mapped) {
    // the box grid's sequence with the curved DG and FD kernels (FD second order)
    if (mode == MODE_RHS || mode == MODE_SUB1) {
      launch_begin_substep(a, mode != MODE_RHS, st);
      TimedLaunch t(d, 4, st);
      launch_fd_stage(a, N, cv, mode, st);
    }
    { TimedLaunch t(d, 5, st); launch_fd_trace(a, N, st); }
    { TimedLaunch t(d, 1, st); launch_dg_mapped(a, N, cv, mode, true, st); }
    { TimedLaunch t(d, 6, st); launch_dg_slab(a, N, cv, mode, st); }
    if (mode != MODE_RHS && a.hybrid == GRFFE_HYBRID_ADAPTIVE) {
      TimedLaunch t(d, 7, st);
      launch_project_troubled(a, N, cv, mode, st);
    }
    { TimedLaunch t(d, 2, st); launch_fd_flux_mapped(a, N, cv, st); }
    { TimedLaunch t(d, 3, st); launch_fd_update(a, N, cv, mode, st); }
    return;
  }
  if (mode == MODE_RHS || mode == MODE_SUB1) {
    launch_begin_substep(a, mode != MODE_RHS, st);
    TimedLaunch t(d, 4, st);
    launch_fd_stage(a, N, cv, mode, st);
  }
  { TimedLaunch t(d, 5, st); launch_fd_trace(a, N, st); }
  { TimedLaunch t(d, 1, st); launch_dg_substep(a, N, cv, mode, st); }
  { TimedLaunch t(d, 6, st); launch_dg_slab(a, N, cv, mode, st); }
  if (mode != MODE_RHS && a.hybrid == GRFFE_HYBRID_ADAPTIVE) {
    { TimedLaunch t(d, 7, st); launch_project_troubled(a, N, cv, mode, st); }
  }
  { TimedLaunch t(d, 2, st); launch_fd_flux(a, N, cv, st); }
  { TimedLaunch t(d, 3, st); launch_fd_update(a, N, cv, mode, st); }
  if (mode != MODE_RHS && d->cond_count > 0) {
    const CondArgs c{d->cond_list, d->cond_corner, d->cond_ref, d->cond_count,
                     d->cond_c[0], d->cond_c[1], d->cond_c[2], d->cond_r * d->cond_r, d->cond_omega};
    launch_conductor(a, N, cv, c, mode, st);
  }
}

extern "C" int grffe_timing_enable(grffe_domain* d, int mask) {
  if (int rc = check_dom(d)) return rc;
  if (mask < 0 || mask >= (1 << grffe_domain::NFAM) || (mask & 1))
    return fail(GRFFE_EINVAL, "timing mask holds bits 1..9 only");
  d->timed_mask = mask;
  for (size_t& u : d->ev_used) u = 0;
  return GRFFE_OK;
}

extern "C" int grffe_timing_period(grffe_domain* d, int period) {
  if (int rc = check_dom(d)) return rc;
  if (period < 1) return fail(GRFFE_EINVAL, "the timing period is at least 1");
  d->timing_period = period;
  d->timing_step = 0;
  return GRFFE_OK;
}

extern "C" int grffe_timing_read(grffe_domain* d, int family, double* total_ms, int64_t* launches) {
  if (int rc = check_dom(d)) return rc;
  if (family < 1 || family >= grffe_domain::NFAM) return fail(GRFFE_EINVAL, "unknown kernel family");
  double tot = 0.0;
  const size_t used = d->ev_used[family];
  if (used) {
    HIPCHK(hipStreamSynchronize(d->ev_stream));
    for (size_t k = 0; k < used; k += 2) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, d->ev[family][k], d->ev[family][k + 1]));
      tot += ms;
    }
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (int64_t)(used / 2);
  d->ev_used[family] = 0;
  return GRFFE_OK;
}

extern "C" int grffe_rhs(grffe_domain* d, const double* dg, const double* fd, const int32_t* rep, double* ddg,
                         double* dfd, int parts, void* stream) {
  if (int rc = check_ready(d)) return rc;
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
  HIPCHK(hipMemsetAsync(d->fd_count + 3, 0, sizeof(int32_t), st));
  run_substep(d, a, MODE_RHS, st);
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}

// One IMEX-SSP3(4,3,3) step of every element of the domain (or pool).  rep_log
// (nullable, device [5][E]) receives the representation before the step, after each
// substep and after the step.
static int step_once(grffe_domain* d, KArgs& a, hipStream_t st, int32_t* rep_log = nullptr) {
  d->timing_now = d->timing_period <= 1 || (d->timing_step++ % d->timing_period) == 0;
  const size_t row = sizeof(int32_t) * d->E;
  if (rep_log) HIPCHK(hipMemcpyAsync(rep_log, d->rep, row, hipMemcpyDeviceToDevice, st));
  {
    TimedLaunch t(d, 9, st);
    launch_dg_prestage(a, d->N, d->curved, st);
  }
  const int modes[3] = {MODE_SUB1, MODE_SUB2, MODE_SUB3};
  for (int k = 0; k < 3; ++k) {
    run_substep(d, a, modes[k], st);
    if (rep_log) HIPCHK(hipMemcpyAsync(rep_log + (size_t)(k + 1) * d->E, d->rep, row, hipMemcpyDeviceToDevice, st));
  }
  if (a.hybrid == GRFFE_HYBRID_ADAPTIVE) {
    TimedLaunch t(d, 8, st);
    launch_fd_to_dg(a, d->N, d->curved, 0, st);
  }
  if (rep_log) HIPCHK(hipMemcpyAsync(rep_log + (size_t)4 * d->E, d->rep, row, hipMemcpyDeviceToDevice, st));
  d->timing_now = true;
  return GRFFE_OK;
}

extern "C" int grffe_step(grffe_domain* d, int n_steps, double dt, void* stream) {
  if (int rc = check_ready(d)) return rc;
  if (n_steps < 0) return fail(GRFFE_EINVAL, "n_steps must be >= 0");
  hipStream_t st = S(stream);
  KArgs a = make_args(d);
  if (dt > 0.0) a.dt = dt;
  for (int it = 0; it < n_steps; ++it)
    if (int rc = step_once(d, a, st)) return rc;
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}

extern "C" int grffe_step_logged(grffe_domain* d, double dt, int32_t* rep_log, void* stream) {
  if (int rc = check_ready(d)) return rc;
  if (!rep_log) return fail(GRFFE_EINVAL, "rep_log must not be NULL");
  hipStream_t st = S(stream);
  KArgs a = make_args(d);
  if (dt > 0.0) a.dt = dt;
  if (int rc = step_once(d, a, st, rep_log)) return rc;
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}

// The adjoint entry points run in FP64 without the clamp.
static int adjoint_supported(grffe_domain* d) {
  if (d->mapped) return fail(GRFFE_EUNSUPPORTED, "the adjoint is not available on shells");
  if (d->N > 8) return fail(GRFFE_EUNSUPPORTED, "the adjoint is built for degrees 3..8");
  if (d->par.precision != GRFFE_PRECISION_FP64) return fail(GRFFE_EUNSUPPORTED, "the adjoint runs in FP64 only");
  if (d->par.ff_clamp) return fail(GRFFE_EUNSUPPORTED, "the adjoint does not differentiate the clamp");
  if (d->cond_count > 0) return fail(GRFFE_EUNSUPPORTED, "the adjoint does not differentiate the rotating conductor");
  return GRFFE_OK;
}

// Work space of the FD adjoint: per-direction adjoints of the transported cell
// values [3][10][E][m^3] and ghost-cell adjoints [10][E][6][3][m^2].
static int fd_adjoint_space(grffe_domain* d) {
  if (d->adj_fd_wbar) return GRFFE_OK;
  void* p1 = nullptr;
  void* p2 = nullptr;
  if (int rc = dalloc(d, &p1, sizeof(double) * 3 * (NV + 1) * (size_t)d->E * d->mm)) return rc;
  if (int rc = dalloc(d, &p2, sizeof(double) * (NV + 1) * (size_t)d->E * 6 * 3 * d->m * d->m)) return rc;
  d->adj_fd_wbar = reinterpret_cast<double*>(p1);
  d->adj_fd_gbar = reinterpret_cast<double*>(p2);
  return GRFFE_OK;
}

extern "C" int grffe_get_stages(grffe_domain* d, double* u3, double* u4, void* stream) {
  if (int rc = check_dom(d)) return rc;
  hipStream_t st = S(stream);
  const size_t bytes = sizeof(double) * NV * d->E * d->nn;
  if (u3) HIPCHK(hipMemcpyAsync(u3, d->dg.X0, bytes, hipMemcpyDeviceToDevice, st));
  if (u4) HIPCHK(hipMemcpyAsync(u4, d->dg.X1, bytes, hipMemcpyDeviceToDevice, st));
  return GRFFE_OK;
}

// Work space of the step adjoint: six adjoint registers per representation
// (accumulator, two stiff-source adjoints, stiff vector, two explicit vectors), the
// copies of U^n and one DG-sized array for the slab transposes.
static int step_adjoint_space(grffe_domain* d, bool with_fd) {
  const size_t reg = (size_t)NV * d->E * d->nn, regf = (size_t)NV * d->E * d->mm;
  void* p = nullptr;
  if (!d->adj_ws) {
    if (int rc = dalloc(d, &p, sizeof(double) * 6 * reg)) return rc;
    d->adj_ws = reinterpret_cast<double*>(p);
    if (int rc = dalloc(d, &p, sizeof(double) * reg)) return rc;
    d->adj_u0 = reinterpret_cast<double*>(p);
  }
  if (with_fd && !d->adj_fd_ws) {
    if (int rc = fd_adjoint_space(d)) return rc;
    if (int rc = dalloc(d, &p, sizeof(double) * 6 * regf)) return rc;
    d->adj_fd_ws = reinterpret_cast<double*>(p);
    if (int rc = dalloc(d, &p, sizeof(double) * regf)) return rc;
    d->adj_u0_fd = reinterpret_cast<double*>(p);
    if (int rc = dalloc(d, &p, sizeof(double) * reg)) return rc;
    d->adj_extra = reinterpret_cast<double*>(p);
  }
  return GRFFE_OK;
}

extern "C" int grffe_rhs_adjoint(grffe_domain* d, const double* dg, const double* fd, const int32_t* rep,
                                 const double* lam_dg, const double* lam_fd, double* ubar_dg, double* ubar_fd,
                                 int parts, void* stream) {
  if (int rc = check_ready(d)) return rc;
  if (!dg || !fd || !rep || !lam_dg || !lam_fd || !ubar_dg || !ubar_fd)
    return fail(GRFFE_EINVAL, "adjoint pointers must not be NULL");
  if (parts < 1 || parts > 3) return fail(GRFFE_EINVAL, "parts must be 1, 2 or 3");
  if (int rc = adjoint_supported(d)) return rc;
  hipStream_t st = S(stream);
  if (int rc = fd_adjoint_space(d)) return rc;
  // the forward values the transposes are taken at: the FD elements' transported
  // (U, J~) and the ghost slabs of their DG neighbours (as in grffe_rhs)
  KArgs a = make_args(d);
  a.dg.Un = const_cast<double*>(dg);
  a.fd.Un = const_cast<double*>(fd);
  a.rep0 = const_cast<int32_t*>(rep);
  a.sub = 3;
  HIPCHK(hipMemsetAsync(d->troubled, 0, d->E, st));
  HIPCHK(hipMemsetAsync(d->fd_count + 3, 0, sizeof(int32_t), st));
  launch_begin_substep(a, false, st);
  launch_fd_stage(a, d->N, d->curved, MODE_RHS, st);
  launch_dg_slab(a, d->N, d->curved, MODE_RHS, st);
  // DG elements, then FD elements and the two couplings
  launch_rhs_adjoint(a, d->N, d->curved, lam_dg, ubar_dg, parts, st);
  launch_fd_rhs_adjoint(a, d->N, d->curved, lam_fd, ubar_fd, lam_dg, ubar_dg, parts, d->adj_fd_wbar,
                        d->adj_fd_gbar, st);
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}

extern "C" int grffe_step_adjoint(grffe_domain* d, const double* u_dg, const double* lam_next, double* lam,
                                  double dt, void* stream) {
  if (int rc = check_ready(d)) return rc;
  if (!u_dg || !lam_next || !lam) return fail(GRFFE_EINVAL, "adjoint pointers must not be NULL");
  if (int rc = adjoint_supported(d)) return rc;
  hipStream_t st = S(stream);
  const size_t reg = (size_t)NV * d->E * d->nn;
  if (int rc = step_adjoint_space(d, false)) return rc;
  // forward step from u_dg with every element on DG, keeping U_3, U_4 in the registers
  HIPCHK(hipMemcpyAsync(d->adj_u0, u_dg, sizeof(double) * reg, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(d->dg.Un, u_dg, sizeof(double) * reg, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemsetAsync(d->rep, 0, sizeof(int32_t) * d->E, st));
  KArgs a = make_args(d);
  a.hybrid = GRFFE_HYBRID_DG_ONLY;
  if (dt > 0.0) a.dt = dt;
  step_once(d, a, st);
  HIPCHK(hipGetLastError());
  // backward sweep over the stages
  KArgs b = a;
  b.dg.Un = d->adj_u0;
  launch_step_adjoint(b, d->N, d->curved, lam_next, lam, d->adj_ws, st);
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}

extern "C" int grffe_step_adjoint_stages(grffe_domain* d, const double* u_dg, const double* u3, const double* u4,
                                         const double* lam_next, double* lam, double dt, void* stream) {
  if (int rc = check_ready(d)) return rc;
  if (!u_dg || !u3 || !u4 || !lam_next || !lam) return fail(GRFFE_EINVAL, "adjoint pointers must not be NULL");
  if (int rc = adjoint_supported(d)) return rc;
  if (int rc = step_adjoint_space(d, false)) return rc;
  hipStream_t st = S(stream);
  // every element on DG; the stage values are the caller's (read only)
  HIPCHK(hipMemsetAsync(d->rep0, 0, sizeof(int32_t) * d->E, st));
  KArgs b = make_args(d);
  b.hybrid = GRFFE_HYBRID_DG_ONLY;
  if (dt > 0.0) b.dt = dt;
  b.dg.Un = const_cast<double*>(u_dg);
  b.dg.X0 = const_cast<double*>(u3);
  b.dg.X1 = const_cast<double*>(u4);
  launch_step_adjoint(b, d->N, d->curved, lam_next, lam, d->adj_ws, st);
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}

extern "C" int grffe_step_adjoint_frozen(grffe_domain* d, const double* dg, const double* fd, const int32_t* rep,
                                         const double* mu_dg, const double* mu_fd, double* lam_dg, double* lam_fd,
                                         int32_t* rep_log, double dt, void* stream) {
  if (int rc = check_ready(d)) return rc;
  if (!dg || !fd || !rep || !mu_dg || !mu_fd || !lam_dg || !lam_fd)
    return fail(GRFFE_EINVAL, "adjoint pointers must not be NULL");
  if (int rc = adjoint_supported(d)) return rc;
  if (int rc = step_adjoint_space(d, true)) return rc;
  const size_t reg = (size_t)NV * d->E * d->nn, regf = (size_t)NV * d->E * d->mm;
  if (!d->adj_hyb) {
    void* p = nullptr;
    if (int rc = dalloc(d, &p, sizeof(double) * (2 * reg + 3 * regf))) return rc;
    d->adj_hyb = reinterpret_cast<double*>(p);
    if (int rc = dalloc(d, &p, sizeof(int32_t) * 5 * d->E)) return rc;
    d->adj_rep_log = reinterpret_cast<int32_t*>(p);
  }
  hipStream_t st = S(stream);
  const int N = d->N;
  const bool cv = d->curved;
  double* ub_dg = d->adj_hyb;         // U^n adjoints of this sweep
  double* t_dg = d->adj_hyb + reg;    // transfer at a rollback (DG)
  double* ub_fd = d->adj_hyb + 2 * reg;
  double* t_fd = ub_fd + regf;
  double* mu_fd_w = ub_fd + 2 * regf;
  int32_t* log[5];
  for (int k = 0; k < 5; ++k) log[k] = d->adj_rep_log + (size_t)k * d->E;
  // forward step from (dg, fd, rep), keeping the stage registers of both
  // representations and logging the representation before each substep (the
  // rollbacks of an adaptive step) and after the step (the switches back)
  HIPCHK(hipMemcpyAsync(d->adj_u0, dg, sizeof(double) * reg, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(d->adj_u0_fd, fd, sizeof(double) * regf, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(d->dg.Un, dg, sizeof(double) * reg, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(d->fd.Un, fd, sizeof(double) * regf, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(d->rep, rep, sizeof(int32_t) * d->E, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(log[0], rep, sizeof(int32_t) * d->E, hipMemcpyDeviceToDevice, st));
  KArgs a = make_args(d);
  if (dt > 0.0) a.dt = dt;
  launch_dg_prestage(a, N, cv, st);
  const int modes[3] = {MODE_SUB1, MODE_SUB2, MODE_SUB3};
  for (int k = 0; k < 3; ++k) {
    run_substep(d, a, modes[k], st);
    HIPCHK(hipMemcpyAsync(log[k + 1], d->rep, sizeof(int32_t) * d->E, hipMemcpyDeviceToDevice, st));
  }
  // log[k] (k = 1..3) is the representation during substep k; log[4] after the step
  if (a.hybrid == GRFFE_HYBRID_ADAPTIVE) launch_fd_to_dg(a, N, cv, 0, st);
  HIPCHK(hipMemcpyAsync(log[4], d->rep, sizeof(int32_t) * d->E, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipGetLastError());
  // backward sweep
  KArgs b = a;
  b.dg.Un = d->adj_u0;
  b.fd.Un = d->adj_u0_fd;
  b.sub = 3;
  HIPCHK(hipMemsetAsync(d->troubled, 0, d->E, st));
  // U^n on FD of the elements rolled back during the step, as the forward made it
  launch_adj_project_un(b, N, log[0], log[3], d->adj_u0, d->adj_u0_fd, st);
  // the switch back: mu of those elements on FD through R^T
  HIPCHK(hipMemcpyAsync(mu_fd_w, mu_fd, sizeof(double) * regf, hipMemcpyDeviceToDevice, st));
  launch_adj_switch_back(b, N, log[3], log[4], mu_dg, mu_fd_w, st);
  AdjBufs rd{}, rf{};
  rd.mu = mu_dg;
  rd.un_bar = ub_dg;
  rd.a_bar = d->adj_ws;
  rd.s1_bar = d->adj_ws + reg;
  rd.s2_bar = d->adj_ws + 2 * reg;
  rd.w = d->adj_ws + 3 * reg;
  rd.transfer = t_dg;
  rf.mu = mu_fd_w;
  rf.un_bar = ub_fd;
  rf.a_bar = d->adj_fd_ws;
  rf.s1_bar = d->adj_fd_ws + regf;
  rf.s2_bar = d->adj_fd_ws + 2 * regf;
  rf.w = d->adj_fd_ws + 3 * regf;
  rf.transfer = t_fd;
  double* vd[2] = {d->adj_ws + 4 * reg, d->adj_ws + 5 * reg};
  double* vf[2] = {d->adj_fd_ws + 4 * regf, d->adj_fd_ws + 5 * regf};
  // stage k transposes the operator of substep `sub` (elements read in their
  // representation at its start, log[sub - 1], updated in log[sub]) and the
  // combination of substep sub - 1 (representation log[sub - 1]); A3 has no
  // operator and transposes substep 3's combination (log[3])
  const int order[4] = {ADJ_A3, ADJ_B3, ADJ_B2, ADJ_B1};
  const int sub[4] = {3, 3, 2, 1};
  for (int k = 0; k < 4; ++k) {
    const int stage = order[k];
    const int32_t* upd = log[sub[k]];
    const int32_t* start = stage == ADJ_A3 ? log[3] : log[sub[k] - 1];
    rd.rep_upd = rf.rep_upd = upd;
    rd.v_in = vd[(k + 1) % 2];
    rd.v_out = vd[k % 2];
    rf.v_in = vf[(k + 1) % 2];
    rf.v_out = vf[k % 2];
    rd.extra = nullptr;
    {
      // FD list: the elements updated on FD
      KArgs bl = b;
      bl.rep0 = const_cast<int32_t*>(upd);
      HIPCHK(hipMemsetAsync(d->fd_count + 3, 0, sizeof(int32_t), st));
      launch_begin_substep(bl, false, st);
    }
    b.rep0 = const_cast<int32_t*>(start);
    launch_adj_flags(b, upd, st);  // rolled back in this substep (the forward's flags)
    if (stage != ADJ_A3) {
      const int mode = stage == ADJ_B3 ? MODE_SUB3 : (stage == ADJ_B2 ? MODE_SUB2 : MODE_SUB1);
      if (stage == ADJ_B1) {
        // X1 <- U_2 of U^n on the elements that were DG at the step start
        KArgs bp = b;
        bp.rep = log[0];
        launch_dg_prestage(bp, N, cv, st);
      }
      launch_fd_stage(b, N, cv, mode, st);  // the FD-updated cells' stage values
      launch_dg_slab(b, N, cv, mode, st);   // the ghost slabs at the stage
      HIPCHK(hipMemsetAsync(d->adj_extra, 0, sizeof(double) * reg, st));
      launch_fd_step_coupling(b, N, cv, rf.v_in, rd.v_in, stage == ADJ_B2 ? d->dg.X0 : d->dg.X1, d->adj_extra,
                              d->adj_fd_wbar, d->adj_fd_gbar, upd, st);
      rd.extra = d->adj_extra;
    }
    launch_fd_step_stage(b, N, cv, stage, rf, d->adj_fd_wbar, d->adj_fd_gbar, st);
    if (stage != ADJ_A3) launch_adj_rollback(b, N, cv, rd, rf, upd, t_fd, t_dg, sub[k], st);
    launch_dg_adjoint_stage(b, N, cv, stage, rd, st);
  }
  // the adjoint of U^n in the representation it had
  launch_copy_rep(b, log[0], 0, d->nn, ub_dg, lam_dg, st);
  launch_copy_rep(b, log[0], 1, d->mm, ub_fd, lam_fd, st);
  if (rep_log)
    HIPCHK(hipMemcpyAsync(rep_log, d->adj_rep_log, sizeof(int32_t) * 5 * d->E, hipMemcpyDeviceToDevice, st));
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

namespace grffe {
void launch_check_finite(const KArgs& a, int nn, int mm, uint8_t* bad, hipStream_t s);
}

extern "C" int grffe_check_finite(grffe_domain* d, int32_t* n_bad, void* stream) {
  if (int rc = check_dom(d)) return rc;
  if (!d->bad_flags) {
    void* p = nullptr;
    if (int rc = dalloc(d, &p, d->E)) return rc;
    d->bad_flags = static_cast<uint8_t*>(p);
  }
  hipStream_t st = S(stream);
  KArgs a = make_args(d);
  launch_check_finite(a, d->nn, d->mm, d->bad_flags, st);
  HIPCHK(hipGetLastError());
  std::vector<uint8_t> h(d->E);
  HIPCHK(hipMemcpyAsync(h.data(), d->bad_flags, d->E, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int32_t nb = 0;
  for (int e = 0; e < d->E; ++e) nb += h[e] ? 1 : 0;
  if (n_bad) *n_bad = nb;
  if (nb) return fail(GRFFE_ENONFINITE, std::to_string(nb) + " element(s) hold non-finite values");
  return GRFFE_OK;
}

extern "C" int grffe_operator(int degree, int which, double* out, int capacity) {
  if (degree < 3 || degree > MAX_DEG) return fail(GRFFE_EINVAL, "degree must be in [3, 9]");
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


// ------------------------------------------------------------------ batches
// A batch holds many independent domains.  Domains of one degree share a pool: their
// elements are concatenated, so every kernel of a step is one launch over all of
// them, with per-element widths and time steps.  One step of all pools is captured
// once into a HIP graph, the pools on forked branches that can run concurrently.
struct grffe_batch {
  std::vector<grffe_domain*> pools;
  std::vector<int> pool_of, part_of;  // domain k -> pool, part within the pool
  std::vector<uint8_t*> forced;       // per pool [E] (forced hybrid mode)
  hipStream_t cap = nullptr;          // capture stream (library owned)
  std::vector<hipStream_t> side;      // one branch stream per extra pool
  std::vector<hipEvent_t> ev;         // fork + joins
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static int check_batch(grffe_batch* b) {
  if (!b || b->pools.empty()) return fail(GRFFE_EINVAL, "batch is NULL");
  return GRFFE_OK;
}

static int check_member(grffe_batch* b, int k) {
  if (int rc = check_batch(b)) return rc;
  if (k < 0 || k >= (int)b->pool_of.size()) return fail(GRFFE_EINVAL, "domain index out of range");
  return GRFFE_OK;
}

extern "C" int grffe_batch_destroy(grffe_batch* b) {
  if (!b) return GRFFE_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  for (hipStream_t s : b->side) (void)hipStreamDestroy(s);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (grffe_domain* d : b->pools) grffe_destroy(d);
  delete b;
  return GRFFE_OK;
}

extern "C" int grffe_batch_create(const grffe_grid* grids, int32_t count, const grffe_params* params,
                                  const double* const* bgs, void* stream, grffe_batch** out) {
  if (!out) return fail(GRFFE_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (!grids || !params || count < 1) return fail(GRFFE_EINVAL, "a batch needs at least one grid");
  for (int k = 0; k < count; ++k)
    if (grids[k].degree < 3 || grids[k].degree > MAX_DEG) return fail(GRFFE_EINVAL, "degree must be in 3..9");
  for (int k = 0; k < count; ++k)
    for (int f = 0; f < 6; ++f)
      if (grids[k].bc[f] == GRFFE_BC_DIRICHLET)
        return fail(GRFFE_EUNSUPPORTED, "Dirichlet faces are supported on single domains, not in batches");
  const bool curved = bgs && bgs[0];
  for (int k = 0; k < count; ++k)
    if ((bgs && bgs[k]) != curved) return fail(GRFFE_EINVAL, "a batch is all flat or all curved");
  hipStream_t st = S(stream);
  grffe_batch* b = new grffe_batch();
  b->pool_of.assign(count, -1);
  b->part_of.assign(count, -1);
  for (int N = 3; N <= MAX_DEG; ++N) {
    std::vector<const grffe_grid*> gs;
    std::vector<const double*> bs;
    std::vector<int> ids;
    for (int k = 0; k < count; ++k)
      if (grids[k].degree == N) {
        gs.push_back(&grids[k]);
        bs.push_back(curved ? bgs[k] : nullptr);
        ids.push_back(k);
      }
    if (gs.empty()) continue;
    grffe_domain* d = nullptr;
    if (int rc = build_pool(gs.data(), (int)gs.size(), params, bs.data(), st, &d)) {
      grffe_batch_destroy(b);
      return rc;
    }
    const int pi = (int)b->pools.size();
    b->pools.push_back(d);
    for (size_t q = 0; q < ids.size(); ++q) {
      b->pool_of[ids[q]] = pi;
      b->part_of[ids[q]] = (int)q;
    }
    void* ptr = nullptr;
    if (int rc = dalloc(d, &ptr, d->E)) {
      grffe_batch_destroy(b);
      return rc;
    }
    b->forced.push_back(reinterpret_cast<uint8_t*>(ptr));
    if (hipMemsetAsync(ptr, 0, d->E, st) != hipSuccess) {
      grffe_batch_destroy(b);
      return fail(GRFFE_EHIP, "hipMemsetAsync failed");
    }
  }
  if (hipStreamSynchronize(st) != hipSuccess) {
    grffe_batch_destroy(b);
    return fail(GRFFE_EHIP, "hipStreamSynchronize failed");
  }
  *out = b;
  return GRFFE_OK;
}

extern "C" int grffe_batch_size(grffe_batch* b, int32_t* n_domains, int32_t* n_pools) {
  if (int rc = check_batch(b)) return rc;
  if (n_domains) *n_domains = (int32_t)b->pool_of.size();
  if (n_pools) *n_pools = (int32_t)b->pools.size();
  return GRFFE_OK;
}

// Copy between a domain's compact [9][E_k][P] array and its rows in a pool [9][E][P].
static int copy_rows(double* dst, size_t dpitch, const double* src, size_t spitch, size_t width, int rows,
                     hipStream_t st) {
  if (width == 0) return GRFFE_OK;
  HIPCHK(hipMemcpy2DAsync(dst, dpitch, src, spitch, width, rows, hipMemcpyDeviceToDevice, st));
  return GRFFE_OK;
}

extern "C" int grffe_batch_init_from_fd(grffe_batch* b, const double* const* u_fd, const uint8_t* const* forced,
                                        void* stream) {
  if (int rc = check_batch(b)) return rc;
  if (!u_fd) return fail(GRFFE_EINVAL, "u_fd must not be NULL");
  hipStream_t st = S(stream);
  for (size_t k = 0; k < b->pool_of.size(); ++k) {
    if (!u_fd[k]) return fail(GRFFE_EINVAL, "every domain needs FD data");
    grffe_domain* d = b->pools[b->pool_of[k]];
    const grffe_part& pt = d->parts[b->part_of[k]];
    const size_t row = sizeof(double) * pt.E * d->mm;
    if (int rc = copy_rows(d->fd.Un + (size_t)pt.off * d->mm, sizeof(double) * d->E * d->mm, u_fd[k], row, row, NV,
                           st))
      return rc;
    uint8_t* f = b->forced[b->pool_of[k]] + pt.off;
    if (forced && forced[k]) {
      HIPCHK(hipMemcpyAsync(f, forced[k], pt.E, hipMemcpyDeviceToDevice, st));
    } else {
      HIPCHK(hipMemsetAsync(f, 0, pt.E, st));
    }
  }
  for (size_t pi = 0; pi < b->pools.size(); ++pi)
    if (int rc = init_pool_from_fd(b->pools[pi], b->forced[pi], st)) return rc;
  return GRFFE_OK;
}

extern "C" int grffe_batch_get_state(grffe_batch* b, int32_t k, double* dg, double* fd, int32_t* rep, void* stream) {
  if (int rc = check_member(b, k)) return rc;
  hipStream_t st = S(stream);
  grffe_domain* d = b->pools[b->pool_of[k]];
  const grffe_part& pt = d->parts[b->part_of[k]];
  if (dg) {
    const size_t row = sizeof(double) * pt.E * d->nn;
    if (int rc = copy_rows(dg, row, d->dg.Un + (size_t)pt.off * d->nn, sizeof(double) * d->E * d->nn, row, NV, st))
      return rc;
  }
  if (fd) {
    const size_t row = sizeof(double) * pt.E * d->mm;
    if (int rc = copy_rows(fd, row, d->fd.Un + (size_t)pt.off * d->mm, sizeof(double) * d->E * d->mm, row, NV, st))
      return rc;
  }
  if (rep) HIPCHK(hipMemcpyAsync(rep, d->rep + pt.off, sizeof(int32_t) * pt.E, hipMemcpyDeviceToDevice, st));
  return GRFFE_OK;
}

extern "C" int grffe_batch_set_state(grffe_batch* b, int32_t k, const double* dg, const double* fd,
                                     const int32_t* rep, void* stream) {
  if (int rc = check_member(b, k)) return rc;
  if (!dg || !fd || !rep) return fail(GRFFE_EINVAL, "state pointers must not be NULL");
  hipStream_t st = S(stream);
  grffe_domain* d = b->pools[b->pool_of[k]];
  const grffe_part& pt = d->parts[b->part_of[k]];
  size_t row = sizeof(double) * pt.E * d->nn;
  if (int rc = copy_rows(d->dg.Un + (size_t)pt.off * d->nn, sizeof(double) * d->E * d->nn, dg, row, row, NV, st))
    return rc;
  row = sizeof(double) * pt.E * d->mm;
  if (int rc = copy_rows(d->fd.Un + (size_t)pt.off * d->mm, sizeof(double) * d->E * d->mm, fd, row, row, NV, st))
    return rc;
  HIPCHK(hipMemcpyAsync(d->rep + pt.off, rep, sizeof(int32_t) * pt.E, hipMemcpyDeviceToDevice, st));
  return GRFFE_OK;
}

extern "C" int grffe_batch_get_dt(grffe_batch* b, int32_t k, double* dt) {
  if (int rc = check_member(b, k)) return rc;
  if (!dt) return fail(GRFFE_EINVAL, "dt must not be NULL");
  *dt = b->pools[b->pool_of[k]]->parts[b->part_of[k]].dt;
  return GRFFE_OK;
}

extern "C" int grffe_batch_get_counts(grffe_batch* b, int32_t k, int32_t* n_dg, int32_t* n_fd) {
  if (int rc = check_member(b, k)) return rc;
  grffe_domain* d = b->pools[b->pool_of[k]];
  const grffe_part& pt = d->parts[b->part_of[k]];
  std::vector<int32_t> rep(pt.E);
  HIPCHK(hipMemcpy(rep.data(), d->rep + pt.off, sizeof(int32_t) * pt.E, hipMemcpyDeviceToHost));
  int32_t a = 0, f = 0;
  for (int e = 0; e < pt.E; ++e) {
    if (!d->live_h[pt.off + e]) continue;
    if (rep[e]) ++f; else ++a;
  }
  if (n_dg) *n_dg = a;
  if (n_fd) *n_fd = f;
  return GRFFE_OK;
}

// Contraction engine per degree pool.  A change drops the captured step graph, which
// holds the launches of the previous engine; the next graph step captures again.
extern "C" int grffe_batch_set_contraction(grffe_batch* b, int32_t degree, int32_t engine) {
  if (int rc = check_batch(b)) return rc;
  if (engine != GRFFE_CONTRACTION_VALU && engine != GRFFE_CONTRACTION_MFMA)
    return fail(GRFFE_EINVAL, "engine must be GRFFE_CONTRACTION_VALU or GRFFE_CONTRACTION_MFMA");
  if (degree != 0 && (degree < 3 || degree > MAX_DEG)) return fail(GRFFE_EINVAL, "degree must be 0 or in 3..9");
  bool found = false, changed = false;
  for (grffe_domain* d : b->pools)
    if (degree == 0 || d->N == degree) found = true;
  if (!found) return fail(GRFFE_EINVAL, "the batch has no domain of that degree");
  if (engine != GRFFE_CONTRACTION_VALU)
    return fail(GRFFE_EUNSUPPORTED, "batches run the VALU contraction (an engine change re-captures the step graph, "
                                    "which ended in an abort inside the HIP runtime)");
  for (grffe_domain* d : b->pools) {
    if (degree != 0 && d->N != degree) continue;
    if (d->contraction != engine) changed = true;
    d->contraction = engine;
  }
  if (changed && b->exec) {
    HIPCHK(hipGraphExecDestroy(b->exec));
    b->exec = nullptr;
    if (b->graph) HIPCHK(hipGraphDestroy(b->graph));
    b->graph = nullptr;
  }
  return GRFFE_OK;
}

extern "C" int grffe_batch_get_contraction(grffe_batch* b, int32_t degree, int32_t* engine) {
  if (int rc = check_batch(b)) return rc;
  if (!engine) return fail(GRFFE_EINVAL, "engine must not be NULL");
  for (grffe_domain* d : b->pools)
    if (d->N == degree) {
      *engine = d->contraction;
      return GRFFE_OK;
    }
  return fail(GRFFE_EINVAL, "the batch has no domain of that degree");
}

// One step of every pool: pool 0 on `st`, every other pool on its own branch stream
// forked from and joined back to `st`.
static int batch_step_once(grffe_batch* b, hipStream_t st) {
  const size_t np = b->pools.size();
  if (np > 1) {
    HIPCHK(hipEventRecord(b->ev[0], st));
    for (size_t pi = 1; pi < np; ++pi) HIPCHK(hipStreamWaitEvent(b->side[pi - 1], b->ev[0], 0));
  }
  for (size_t pi = 0; pi < np; ++pi) {
    grffe_domain* d = b->pools[pi];
    hipStream_t s = pi == 0 ? st : b->side[pi - 1];
    KArgs a = make_args(d);
    if (int rc = step_once(d, a, s)) return rc;
    HIPCHK(hipGetLastError());
  }
  if (np > 1)
    for (size_t pi = 1; pi < np; ++pi) {
      HIPCHK(hipEventRecord(b->ev[pi], b->side[pi - 1]));
      HIPCHK(hipStreamWaitEvent(st, b->ev[pi], 0));
    }
  return GRFFE_OK;
}

static int batch_streams(grffe_batch* b) {
  const size_t np = b->pools.size();
  while (b->side.size() + 1 < np) {
    hipStream_t s;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    b->side.push_back(s);
  }
  while (b->ev.size() < np) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->ev.push_back(e);
  }
  return GRFFE_OK;
}

static int batch_capture(grffe_batch* b) {
  if (b->exec) return GRFFE_OK;
  if (!b->cap) HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  const int rc = batch_step_once(b, b->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(GRFFE_EHIP, std::string("stream capture failed: ") + hipGetErrorString(e));
  b->graph = g;
  HIPCHK(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  return GRFFE_OK;
}

extern "C" int grffe_batch_step(grffe_batch* b, int32_t n_steps, int32_t use_graph, void* stream) {
  if (int rc = check_batch(b)) return rc;
  if (n_steps < 0) return fail(GRFFE_EINVAL, "n_steps must be >= 0");
  hipStream_t st = S(stream);
  if (int rc = batch_streams(b)) return rc;
  if (use_graph) {
    if (int rc = batch_capture(b)) return rc;
    for (int it = 0; it < n_steps; ++it) HIPCHK(hipGraphLaunch(b->exec, st));
  } else {
    for (int it = 0; it < n_steps; ++it)
      if (int rc = batch_step_once(b, st)) return rc;
  }
  HIPCHK(hipGetLastError());
  return GRFFE_OK;
}
