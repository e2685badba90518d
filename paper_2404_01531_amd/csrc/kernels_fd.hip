// FD subcell kernels and the DG <-> FD transfers.
//
// Sec. III C 2, Eq. (fd time derivative): conservative finite differences on
// (2N+1)^3 uniform subcells.  Dimension by dimension, the point values of U and
// of J~ are reconstructed to the subcell faces with WENO5-Z (exponent q = 2),
// the Rusanov flux F* is formed with the metric at the face, and the
// fourth-order corrector of Eq. (higher order flux correction), built from the
// cell-centred fluxes,
//   Fhat_{i+1/2} = F*_{i+1/2} - (F_i - 2 F*_{i+1/2} + F_{i+1}) / 6,
// gives dU_i/dt = -sum_d (2N+1)/h_d (Fhat_{i+1/2} - Fhat_{i-1/2}) + S(U_i).
// Three ghost layers per face come from the neighbour's subcells, from the
// P-projection of a DG neighbour (slab buffer), or from the no-incoming-Poynting
// state of the outermost own cell (Sec. III D).
#include "common.h"
#include "fd_common.h"

namespace grffe {

// ---------------------------------------------------------------- substep start
// Opens a step (or a right-hand side evaluation): with `copy` the representation
// at the start (rep0) is taken from rep and the flags are cleared; every live FD
// element is appended to the work list fd_list (count fd_count[sub], emptied
// before: by the pre-stage pass for a step).  The DG substep kernel appends the
// elements it flags, so the FD flux and update launches see both, and the FD
// update of a flagged element marks it FD for the next substep: the list then
// holds the FD elements at the start of every substep of the step.  List order
// does not affect any result.
__global__ __launch_bounds__(256) void k_begin_substep(KArgs a, int copy) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= a.E) return;
  int r;
  if (copy) {
    r = a.rep[e];
    a.rep0[e] = r;
    a.troubled[e] = 0;
  } else {
    r = a.rep0[e];
  }
  if (a.live[e] && r == 1) a.fd_list[atomicAdd(a.fd_count + a.sub, 1)] = e;
}

// ---------------------------------------------------------------- FD stage values + J~
// Work items: (listed FD element, block of 256 cells).
template <int N, bool CURVED, int MODE>
__global__ __launch_bounds__(256) void k_fd_stage(KArgs a) {
  using Dm = Dims<N>;
  constexpr int mm = Dm::mm;
  constexpr int BPE = (mm + 255) / 256;
  const int items = a.fd_count[a.sub] * BPE;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int e = a.fd_list[item / BPE];
    const int p = (item % BPE) * 256 + threadIdx.x;
    if (p >= mm) continue;
    Metric M;
    load_metric<CURVED>(a.bg_fd, a.E, mm, e, p, M);
    double X[NV], J[3];
    if (MODE == MODE_SUB1) {
      // the implicit pre-stages of the step: U_2 is this substep's input, the
      // stiff-source terms of substeps 2 and 3 are kept for the updates
      double Un[NV], S1[NV], S2[NV];
      load9(a.fd.Un, a.E, mm, e, p, Un);
      const double dt = dt_of(a, e);
      derived_stages(Un, M, a, dt, X, S1, S2);
      store_stiff_terms(a.fd, a.E, mm, e, p, dt, S1, S2);
    } else {
      stage_input<MODE>(a.fd, a.E, mm, e, p, M, a, X);
    }
    current_total(X, M, a.eta, J);
    const size_t st = (size_t)a.E * mm;
    double* w = a.w_fd + (size_t)e * mm + p;
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v * st] = X[v];
#pragma unroll
    for (int c = 0; c < 3; ++c) w[(9 + c) * st] = J[c];
  }
}

// ---------------------------------------------------------------- R-traces of FD elements
// One workgroup per (FD element, transported component): the six face traces of
// R (x) R (x) R applied to that component.
template <int N>
__global__ __launch_bounds__(256) void k_fd_trace(KArgs a) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, mm = Dm::mm;
  __shared__ double sW[mm];
  __shared__ double s1[6 * m * m];
  __shared__ double s2[6 * n * m];
  __shared__ double sR[n * m];
  const int t = threadIdx.x;
  for (int q = t; q < n * m; q += 256) sR[q] = a.ops->R[q];
  // work items: (listed FD element, transported component); the list holds the
  // elements on FD at the substep start only at this point
  const int items = a.fd_count[a.sub] * NW;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
  const int e = a.fd_list[item / NW];
  const int c = item % NW;
  int need = 0;
  for (int f = 0; f < 6; ++f) {
    const int o = a.nbr[e * 6 + f];
    if (o >= 0 && a.rep0[o] == 0) need |= 1 << f;
  }
  if (!need) continue;
  __syncthreads();
  for (int q = t; q < mm; q += 256) sW[q] = a.w_fd[((size_t)c * a.E + e) * mm + q];
  __syncthreads();
  const int str[3] = {1, m, m * m};
  // 1) normal direction of every face: R row 0 (lower face) or N (upper face)
  for (int q = t; q < 6 * m * m; q += 256) {
    const int f = q / (m * m), r = q % (m * m);
    if (!(need & (1 << f))) continue;
    const int d = f >> 1, row = (f & 1) ? N : 0;
    const int t1ax = (d == 0) ? 1 : 0, t2ax = (d == 2) ? 1 : 2;
    const int c1 = r % m, c2 = r / m;
    double acc = 0.0;
    for (int z = 0; z < m; ++z) acc += sR[row * m + z] * sW[z * str[d] + c1 * str[t1ax] + c2 * str[t2ax]];
    s1[q] = acc;  // [f][c2][c1]
  }
  __syncthreads();
  // 2) first tangential axis
  for (int q = t; q < 6 * n * m; q += 256) {
    const int f = q / (n * m), r = q % (n * m);
    if (!(need & (1 << f))) continue;
    const int a1 = r % n, c2 = r / n;
    double acc = 0.0;
    for (int z = 0; z < m; ++z) acc += sR[a1 * m + z] * s1[(f * m + c2) * m + z];
    s2[q] = acc;  // [f][c2][a1]
  }
  __syncthreads();
  // 3) second tangential axis, written as [f][a2][a1]
  for (int q = t; q < 6 * n * n; q += 256) {
    const int f = q / (n * n), r = q % (n * n);
    if (!(need & (1 << f))) continue;
    const int a1 = r % n, a2 = r / n;
    double acc = 0.0;
    for (int z = 0; z < m; ++z) acc += sR[a2 * m + z] * s2[(f * m + z) * n + a1];
    a.trace[((size_t)c * a.E * 6 + (size_t)e * 6 + f) * (n * n) + r] = acc;
  }
  }
}

// ---------------------------------------------------------------- DG -> FD of flagged elements
// P (x) P (x) P of the live registers of every element flagged in this substep,
// followed by the FD stage values (U and J~) of its subcells.
template <int N, bool CURVED, int MODE>
__global__ __launch_bounds__(256) void k_project_troubled(KArgs a) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, nn = Dm::nn, mm = Dm::mm;
  const int e = blockIdx.x;
  if (!a.live[e] || !a.troubled[e]) return;
  __shared__ double s0[nn];
  __shared__ double s1[m * n * n];
  __shared__ double s2[m * m * n];
  __shared__ double sP[m * n];
  const int t = threadIdx.x;
  for (int q = t; q < m * n; q += 256) sP[q] = a.ops->P[q];
  const double* src[3];
  double* dst[3];
  int nreg = 0;
  src[nreg] = a.dg.Un;
  dst[nreg++] = a.fd.Un;
  if (MODE == MODE_SUB2) {
    src[nreg] = a.dg.X0;
    dst[nreg++] = a.fd.X0;
  }
  if (MODE == MODE_SUB3) {
    src[nreg] = a.dg.X1;
    dst[nreg++] = a.fd.X1;
  }
  if (MODE == MODE_SUB2 || MODE == MODE_SUB3) {
    src[nreg] = a.dg.A;
    dst[nreg++] = a.fd.A;
  }
  for (int r = 0; r < nreg; ++r)
    for (int v = 0; v < NV; ++v) {
      __syncthreads();
      for (int q = t; q < nn; q += 256) s0[q] = src[r][((size_t)v * a.E + e) * nn + q];
      __syncthreads();
      for (int q = t; q < m * n * n; q += 256) {  // x: [z][y][cx]
        const int cx = q % m, yz = q / m;
        double acc = 0.0;
        for (int z = 0; z < n; ++z) acc += sP[cx * n + z] * s0[yz * n + z];
        s1[q] = acc;
      }
      __syncthreads();
      for (int q = t; q < m * m * n; q += 256) {  // y: [z][cy][cx]
        const int cx = q % m, cy = (q / m) % m, z0 = q / (m * m);
        double acc = 0.0;
        for (int z = 0; z < n; ++z) acc += sP[cy * n + z] * s1[(z0 * n + z) * m + cx];
        s2[q] = acc;
      }
      __syncthreads();
      double* out = dst[r] + ((size_t)v * a.E + e) * mm;
      for (int q = t; q < mm; q += 256) {  // z: [cz][cy][cx]
        const int cxy = q % (m * m), cz = q / (m * m);
        double acc = 0.0;
        for (int z = 0; z < n; ++z) acc += sP[cz * n + z] * s2[z * m * m + cxy];
        out[q] = acc;
      }
    }
  // the block's own global writes are visible to it after the barrier
  __syncthreads();
  for (int p = t; p < mm; p += 256) {
    Metric M;
    load_metric<CURVED>(a.bg_fd, a.E, mm, e, p, M);
    double X[NV], J[3];
    {
      // pre-stages re-derived from the projected U^n
      double Un[NV], U2[NV], S1[NV], S2[NV];
      load9(a.fd.Un, a.E, mm, e, p, Un);
      const double dt = dt_of(a, e);
      derived_stages(Un, M, a, dt, U2, S1, S2);
      store_stiff_terms(a.fd, a.E, mm, e, p, dt, S1, S2);
      if (MODE == MODE_SUB1)
        for (int v = 0; v < NV; ++v) X[v] = U2[v];
    }
    if (MODE != MODE_SUB1) stage_input<MODE>(a.fd, a.E, mm, e, p, M, a, X);
    current_total(X, M, a.eta, J);
    const size_t st = (size_t)a.E * mm;
    double* w = a.w_fd + (size_t)e * mm + p;
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v * st] = X[v];
#pragma unroll
    for (int c = 0; c < 3; ++c) w[(9 + c) * st] = J[c];
  }
}


// One workgroup per (FD element, direction d, row t2 of pencils along d): the
// m pencils of the row, with three ghost cells at each end, are staged in LDS
// once; then every (component, face, pencil) is reconstructed, the cell-centred
// fluxes of the corrector are formed once per cell, and finally every (face,
// pencil) forms the Rusanov flux and the fourth-order corrected flux.  Only
// J~^d enters F^d, so ten components (U and J~^d) are reconstructed.  LDS tiles are
// [component][cell or face][pencil] with the pencil index fastest: the row length
// m = 2N+1 is odd, so both the pencil-contiguous and the cell-contiguous thread
// mappings touch 16 distinct bank pairs per 16 lanes (no bank conflicts).
// Workgroups per CU the flux kernel is compiled for: the curved FP64 instantiations
// of degree <= 5 fit three in LDS, and are held to the registers of three (168 per
// lane; without the bound they take ~175, which allows two).
template <int N, bool CURVED>
constexpr int flux_min_blocks() {
  return (CURVED && N <= 5) ? 3 : 1;
}

template <int N, bool CURVED, typename R>
__global__ __launch_bounds__(flux_tpb<N>(), (flux_min_blocks<N, CURVED>())) void k_fd_flux(KArgs a) {
  using Dm = Dims<N>;
  constexpr int m = Dm::m, mm = Dm::mm;
  constexpr int nf = (m + 1) * m * m;
  constexpr int L = m;      // pencils per workgroup
  constexpr int C = m + 6;  // cells per pencil including ghosts
  constexpr int F = m + 1;  // faces per pencil
  constexpr int NR = NV + 1;  // reconstructed components: U and J~^d
  constexpr int TPB = flux_tpb<N>();
  constexpr int FP = m + 2;  // state slots per pencil: one per target cell -1 .. m
  static_assert(L % 2 == 1, "odd pencil count keeps the LDS tiles free of bank conflicts");
  __shared__ double sW[NR * C * L];    // [k][extended cell][pencil]
  // reconstructed states by target cell c (slot c + 1): the left state of face c + 1
  // in sLf (face f at slot f), the right state of face c in sRf (face f at slot
  // f + 1); the unused slots (left m + 1, right 0) take the two edge targets' other
  // state, so that the reconstruction loop stores without conditions
  __shared__ double sLf[NR * FP * L];  // [k][slot][pencil]
  __shared__ double sRf[NR * FP * L];
  __shared__ double sM[CURVED ? NBGF * L * (m + 2) : 1];
  const int t = threadIdx.x;
  // work items: (listed FD element, direction, row of pencils).  Workgroups are
  // dealt to the eight XCDs in turn (block b to XCD b mod 8), each with its own
  // L2: every XCD takes a contiguous run of items, so that the 3m items of one
  // element, which read the same cells, share one L2.
  const int items = a.fd_count[a.sub] * 3 * m;
  constexpr int NX = 8;
  const bool split = gridDim.x % NX == 0;
  const int xcd = split ? (int)blockIdx.x % NX : 0;
  const int per = split ? (items + NX - 1) / NX : items;
  const int step = split ? (int)gridDim.x / NX : (int)gridDim.x;
  for (int l = split ? (int)blockIdx.x / NX : (int)blockIdx.x; l < per; l += step) {
  const int item = xcd * per + l;
  if (item >= items) break;  // the same for every thread of the block
  const int e = a.fd_list[item / (3 * m)];
  const int d = (item / m) % 3;
  const int t2 = item % m;
  const RowNbrs nb = row_neighbours(a, e, d);
  // phase 1: stage cells -3 .. m+2 of every pencil (and the metric of cells -1 .. m)
  // curved: the phases with fewer work items than threads start at different waves,
  // so that the wavefronts (one per SIMD) carry similar loads: staging on waves 2, 3,
  // 0, the last reconstruction round on waves 3, 0, 1, the face fluxes on waves 1, 2,
  // 3 (-4% on the curved kernel; neutral on the flat one, which keeps the plain order)
  constexpr bool ROT = CURVED && TPB == 256;
  const int t_stage = ROT ? (t + 128) & 255 : t, t_weno = ROT ? (t + 64) & 255 : t;
  const int t_face = ROT ? (t + 192) & 255 : t;
  for (int q = t_stage; q < L * C; q += TPB) {
    int c, t1;
    if (d == 0) {
      c = q % C;
      t1 = q / C;
    } else {
      t1 = q % L;
      c = q / L;
    }
    const CellSrc cs = cell_source<N>(a, nb, e, d, c - 3, t1, t2);
    double W[NR];
    Metric Mc;
    if (cs.ptr) {
#pragma unroll
      for (int k = 0; k < NV; ++k) W[k] = cs.ptr[k * cs.stride];
      W[NV] = cs.ptr[(NV + d) * cs.stride];
      if (CURVED && c >= 2 && c <= m + 3) load_metric<CURVED>(a.bg_fd, a.E, mm, cs.elem, cs.cell, Mc);
    } else {
      double Ui[NV], Ub[NV], J[3];
      load_metric<CURVED>(a.bg_fd, a.E, mm, e, cs.cell, Mc);
      load9(a.w_fd, a.E, mm, e, cs.cell, Ui);
      // ghost layer lg (0 next to the face) of the pencil's cell (t1, t2)
      const int sg = (c >= m + 3) ? 1 : 0, lg = sg ? c - 3 - m : 2 - c;
      exterior_state(a, cs.bnd, d, sg, Ui, Mc, a.bfield_fd,
                     ((((size_t)e * 6 + 2 * d + sg) * 3 + lg) * m + t2) * m + t1,
                     (size_t)a.E * 6 * 3 * m * m, Ub);
      current_total(Ub, Mc, a.eta, J);
#pragma unroll
      for (int k = 0; k < NV; ++k) W[k] = Ub[k];
      W[NV] = (d == 0) ? J[0] : (d == 1 ? J[1] : J[2]);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) sW[(k * C + c) * L + t1] = W[k];
    if (CURVED && c >= 2 && c <= m + 3) {
      const int cm = c - 2;
      double* o = sM + cm * L + t1;  // [field][cell -1 .. m][pencil]
      o[0] = Mc.alpha;
      o[1 * L * (m + 2)] = Mc.beta[0];
      o[2 * L * (m + 2)] = Mc.beta[1];
      o[3 * L * (m + 2)] = Mc.beta[2];
#pragma unroll
      for (int k = 0; k < 6; ++k) o[(4 + k) * L * (m + 2)] = Mc.g[k];
    }
  }
  __syncthreads();
  // phase 2: WENO5-Z of every component at every face of every pencil, and the
  // cell-centred fluxes of cells -1 .. m used by the corrector
  const double eps = a.weno_eps;
  // target cells c = -1 .. m: left state of face c+1 and right state of face c.  The
  // work index q = (k FP + c + 1) L + t1 is also the states' slot index, and the
  // target's cells c-2 .. c+2 start at extended index c+1 of component k's tile:
  // only the component is divided out
  for (int q = t_weno; q < NR * L * FP; q += TPB) {
    const int k = q / (L * FP);
    const double* v = sW + q + k * (C - FP) * L;  // cells c-2 .. c+2
    double vl[5];
#pragma unroll
    for (int z = 0; z < 5; ++z) vl[z] = v[z * L];
    double lft, rgt;
    weno5z_cell(vl, eps, lft, rgt);
    sLf[q] = lft;
    sRf[q] = rgt;
  }
  __syncthreads();
  // phase 3a: cell-centred fluxes of cells -1 .. m of every pencil (the corrector's
  // F_i), each computed once; they replace the staged cells in LDS
  static_assert(L * (m + 2) <= TPB && L * F <= TPB, "one cell / one face per thread in phase 3");
  constexpr int CF = m + 2;  // cells -1 .. m
  R Fcell[NV];
  const bool corr = a.fd_order == 4;
  if (corr && t < L * CF) {
    const int t1 = t % L, c = t / L;
    R W[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) W[k] = (R)sW[(k * C + c + 2) * L + t1];
    Metric Mc;
    if (CURVED) {
      double fm[10];
      const double* o = sM + c * L + t1;
#pragma unroll
      for (int k = 0; k < 10; ++k) fm[k] = o[k * L * (m + 2)];
      metric_from10(fm, Mc);
    } else {
      metric_flat(Mc);
    }
    MetricT<R> Mcr;
    metric_cast(Mc, Mcr);
    flux_any_jd(d, W, W[NV], Mcr, Fcell);
  }
  __syncthreads();
  double* sFc = sW;  // [9][cell -1 .. m][pencil]
  if (corr && t < L * CF) {
    const int t1 = t % L, c = t / L;
#pragma unroll
    for (int v = 0; v < NV; ++v) sFc[(v * CF + c) * L + t1] = (double)Fcell[v];
  }
  __syncthreads();
  // phase 3b: fluxes at every face of every pencil
  double Fh[NV];
  const int q3 = t_face;
  int f3 = 0, t13 = 0;
  if (q3 < L * F) {
    if (d == 0) {
      f3 = q3 % F;
      t13 = q3 / F;
    } else {
      t13 = q3 % L;
      f3 = q3 / L;
    }
    int tix;
    if (d == 0) tix = f3 + (m + 1) * (t13 + m * t2);
    else if (d == 1) tix = t13 + m * (f3 + (m + 1) * t2);
    else tix = t13 + m * (t2 + m * f3);
    // face fluxes, Rusanov and the corrector in R (FP64, or FP32 in the
    // mixed-precision mode; the reconstruction above is always FP64)
    R WL[NR], WR[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      WL[k] = (R)sLf[(k * FP + f3) * L + t13];
      WR[k] = (R)sRf[(k * FP + f3 + 1) * L + t13];
    }
    Metric Mf;
    load_metric<CURVED>(a.bg_face + (size_t)d * NBGF * a.E * nf, a.E, nf, e, tix, Mf);
    MetricT<R> Mfr;
    metric_cast(Mf, Mfr);
    R Fr[NV], Ft[NV];
    flux_any_jd(d, WL, WL[NV], Mfr, Fr);
    flux_any_jd(d, WR, WR[NV], Mfr, Ft);
    const R lam = CURVED ? (R)char_speed(d, Mf) : R(1);
#pragma unroll
    for (int v = 0; v < NV; ++v) Fr[v] = R(0.5) * (Fr[v] + Ft[v]) - R(0.5) * lam * (WR[v] - WL[v]);
    if (corr) {
      // F* - (F_{f-1} - 2 F* + F_f) / 6 with the cell fluxes of cells f-1 and f
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double* fc = sFc + (v * CF + f3) * L + t13;
        const R G = ((R)fc[0] - R(2) * Fr[v] + (R)fc[L]) * R(1.0 / 6.0);
        Fr[v] = Fr[v] - G;
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) Fh[v] = (double)Fr[v];
  }
  __syncthreads();
  double* sFh = sLf;  // the reconstructed states are no longer needed
  if (q3 < L * F) {
#pragma unroll
    for (int v = 0; v < NV; ++v) sFh[(v * F + f3) * L + t13] = Fh[v];
  }
  __syncthreads();
  // phase 4: flux difference of every cell of the row, -(2N+1)/h_d (Fhat_{i+1/2} - Fhat_{i-1/2})
  const double sc = (double)m / h_of(a, e, d);
  const int str[3] = {1, m, m * m};
  const int t1ax = (d == 0) ? 1 : 0, t2ax = (d == 2) ? 1 : 2;
  for (int q = t; q < L * m; q += TPB) {
    int c, t1;
    if (d == 0) {
      c = q % m;
      t1 = q / m;
    } else {
      t1 = q % L;
      c = q / L;
    }
    const int cell = c * str[d] + t1 * str[t1ax] + t2 * str[t2ax];
    double* out = a.fhat + ((size_t)d * NV * a.E + e) * mm + cell;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double* fh = sFh + (v * F + c) * L + t1;
      out[(size_t)v * a.E * mm] = -sc * (fh[L] - fh[0]);
    }
  }
  __syncthreads();  // the next item restages sW
  }
}

template <int N, bool CURVED, int MODE>
__global__ __launch_bounds__(256) void k_fd_update(KArgs a) {
  using Dm = Dims<N>;
  constexpr int mm = Dm::mm;
  constexpr int BPE = (mm + 255) / 256;
  // work items: (listed FD element, block of 256 cells); the list holds the
  // substep's FD elements and the elements flagged in it
  const int items = a.fd_count[a.sub] * BPE;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
  const int e = a.fd_list[item / BPE];
  const int p = (item % BPE) * 256 + threadIdx.x;
  if (p >= mm) continue;
  Metric M;
  load_metric<CURVED>(a.bg_fd, a.E, mm, e, p, M);
  double X[NV];
  load9(a.w_fd, a.E, mm, e, p, X);
  double Jd[3], Je[3], dU[NV];
  current(X, M, a.eta, Jd, Je);
  {
    MetricDeriv Dv;
    load_deriv<CURVED>(a.bg_fd, a.E, mm, e, p, Dv);
    source_explicit<CURVED>(X, M, Dv, Jd, dU);
  }
  for (int d = 0; d < 3; ++d) {
    const double* fd_ = a.fhat + ((size_t)d * NV * a.E + e) * mm + p;
#pragma unroll
    for (int v = 0; v < NV; ++v) dU[v] += fd_[(size_t)v * a.E * mm];
  }
  if (MODE == MODE_RHS) {
    double St[NV], out[NV];
    source_stiff(X, M, a.eta, a.kpsi, a.kphi, St);
    for (int v = 0; v < NV; ++v) out[v] = ((a.parts & 1) ? dU[v] : 0.0) + ((a.parts & 2) ? St[v] : 0.0);
    store9(a.out_fd, a.E, mm, e, p, out);
    continue;
  }
  double Y[NV], Anew[NV];
  stage_update<MODE, true>(a.fd, a.E, mm, e, p, M, a, X, dU, Y, Anew);
  if (MODE != MODE_SUB3) implicit_solve(Y, M, a.eta, a.kpsi, a.kphi, dt_of(a, e) * IMEX_A);
  if (a.ff_clamp) constraint_clamp(Y, M, a.ff_margin);
  if (MODE == MODE_SUB1) {
    store9(a.fd.X0, a.E, mm, e, p, Y);
    store9(a.fd.A, a.E, mm, e, p, Anew);
  } else if (MODE == MODE_SUB2) {
    store9(a.fd.X1, a.E, mm, e, p, Y);
    store9(a.fd.A, a.E, mm, e, p, Anew);
  } else {
    store9(a.fd.Un, a.E, mm, e, p, Y);
  }
  if (MODE == MODE_SUB1 || MODE == MODE_SUB2) {
    // the next substep's transported values (U, J~) of the cell: every element on FD
    // at its start is in this substep's list (elements flagged in it get theirs from
    // the projection)
    double J[3];
    current_total(Y, M, a.eta, J);
    const size_t st = (size_t)a.E * mm;
    double* w = a.w_fd + (size_t)e * mm + p;
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v * st] = Y[v];
#pragma unroll
    for (int c = 0; c < 3; ++c) w[(9 + c) * st] = J[c];
  }
  if (p == 0 && a.troubled[e]) {
    // redone on FD: FD from here on (representation at the next substep's start)
    a.rep[e] = 1;
    a.rep0[e] = 1;
    a.troubled[e] = 0;
  }
  }
}

// ---------------------------------------------------------------- indicator helpers
// u = |B~| at the DG nodes of R (x) R (x) R applied to the FD B~ of element e (from `fd`),
// or taken directly from `dg`; returns the indicator ratio (block-wide).  Each of the
// 256 threads holds PER = ceil((N+1)^3 / 256) nodes (up to four at N = 9).
template <int N, bool CURVED>
__device__ inline double block_ratio(const KArgs& a, int e, const double* Bn /* [3][nn] in LDS */,
                                     double* su, double* sred, const double* sL) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, nn = Dm::nn, TPB = 256;
  constexpr int PER = (nn + TPB - 1) / TPB;
  const int t = threadIdx.x;
  double num = 0.0, den = 0.0;
  double u[PER], uh[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int p = t + r * TPB;
    u[r] = 0.0;
    if (p < nn) {
      Metric M;
      load_metric_dg<CURVED>(a, nn, e, p, M);
      double B[3] = {Bn[p], Bn[nn + p], Bn[2 * nn + p]};
      u[r] = sqrt(dot3(M, B, B));
    }
    uh[r] = u[r];
  }
  const int str[3] = {1, n, n * n};
  for (int d = 0; d < 3; ++d) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r)
      if (t + r * TPB < nn) su[t + r * TPB] = uh[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int p = t + r * TPB;
      if (p >= nn) continue;
      const int id = (p / str[d]) % n;
      const int p0 = p - id * str[d];
      double acc = 0.0;
      for (int q = 0; q < n; ++q) acc += sL[id * n + q] * su[p0 + q * str[d]];
      uh[r] = acc;
    }
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    if (t + r * TPB >= nn) continue;
    const double hp = (a.tci_mode == 1) ? uh[r] : (u[r] - uh[r]);
    num += hp * hp;
    den += u[r] * u[r];
  }
  block_sum2<TPB>(num, den, sred);
  return den > 0.0 ? sqrt(num / den) : 0.0;
}

// R (x) R (x) R of one component (m^3 values in s_in) into s_out (n^3), using two scratch arrays.
template <int N>
__device__ inline void recon3(const double* sR, const double* s_in, double* s1, double* s2, double* s_out) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m;
  const int t = threadIdx.x;
  for (int q = t; q < n * m * m; q += 256) {  // x: [cz][cy][a]
    const int ax = q % n, yz = q / n;
    double acc = 0.0;
    for (int z = 0; z < m; ++z) acc += sR[ax * m + z] * s_in[yz * m + z];
    s1[q] = acc;
  }
  __syncthreads();
  for (int q = t; q < n * n * m; q += 256) {  // y: [cz][b][a]
    const int ax = q % n, by = (q / n) % n, cz = q / (n * n);
    double acc = 0.0;
    for (int z = 0; z < m; ++z) acc += sR[by * m + z] * s1[(cz * m + z) * n + ax];
    s2[q] = acc;
  }
  __syncthreads();
  for (int q = t; q < n * n * n; q += 256) {  // z: [c][b][a]
    const int ab = q % (n * n), cz = q / (n * n);
    double acc = 0.0;
    for (int z = 0; z < m; ++z) acc += sR[cz * m + z] * s2[z * n * n + ab];
    s_out[q] = acc;
  }
  __syncthreads();
}

// End of step (and start-up): FD elements whose reconstruction passes the indicator with
// alpha_fd go back to DG.  policy: 0 indicator decides, 1 all go DG, 2 forced mask decides.
// With `listed` the elements are those of the step's FD work list (every element on FD
// at the end of the step: FD at the step start or flagged in one of its substeps), on a
// persistent grid; otherwise one workgroup per element of the domain (start-up).
template <int N, bool CURVED>
__device__ inline void fd_to_dg_one(const KArgs& a, int e, int policy, const uint8_t* forced) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, nn = Dm::nn, mm = Dm::mm;
  __syncthreads();  // the previous element's tiles are no longer read
  __shared__ double sin_[mm];
  __shared__ double s1[n * m * m];
  __shared__ double s2[n * n * m];
  __shared__ double sB[3 * nn];
  __shared__ double su[nn];
  __shared__ double sR[n * m];
  __shared__ double sL[n * n];
  __shared__ double sred[8];
  const int t = threadIdx.x;
  for (int q = t; q < n * m; q += 256) sR[q] = a.ops->R[q];
  for (int q = t; q < n * n; q += 256) sL[q] = a.ops->L[q];
  bool go;
  if (policy == 1) {
    go = true;
  } else if (policy == 2) {
    go = !(forced && forced[e]);
  } else {
    for (int c = 0; c < 3; ++c) {
      __syncthreads();
      for (int q = t; q < mm; q += 256) sin_[q] = a.fd.Un[((size_t)(3 + c) * a.E + e) * mm + q];
      __syncthreads();
      recon3<N>(sR, sin_, s1, s2, sB + c * nn);
    }
    const double ratio = block_ratio<N, CURVED>(a, e, sB, su, sred, sL);
    if (t == 0) a.ratio[e] = ratio;
    go = !(ratio > a.tci_thr_fd);
  }
  if (!go) return;
  for (int v = 0; v < NV; ++v) {
    __syncthreads();
    for (int q = t; q < mm; q += 256) sin_[q] = a.fd.Un[((size_t)v * a.E + e) * mm + q];
    __syncthreads();
    recon3<N>(sR, sin_, s1, s2, su);
    for (int q = t; q < nn; q += 256) a.dg.Un[((size_t)v * a.E + e) * nn + q] = su[q];
  }
  if (t == 0) a.rep[e] = 0;
}

template <int N, bool CURVED>
__global__ __launch_bounds__(256) void k_fd_to_dg(KArgs a, int policy, const uint8_t* forced, int listed) {
  const int items = listed ? a.fd_count[a.sub] : a.E;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int e = listed ? a.fd_list[item] : item;
    if (!a.live[e] || a.rep[e] != 1) continue;  // the same for every thread of the block
    fd_to_dg_one<N, CURVED>(a, e, policy, forced);
  }
}

// Stand-alone indicator: DG elements on dg (alpha), FD elements on R(fd) (alpha_fd).
template <int N, bool CURVED>
__global__ __launch_bounds__(256) void k_tci(KArgs a, const double* dg, const double* fd, const int32_t* rep,
                                             uint8_t* troubled, double* ratio) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, nn = Dm::nn, mm = Dm::mm;
  const int e = blockIdx.x;
  if (!a.live[e]) {
    if (threadIdx.x == 0) {
      troubled[e] = 0;
      if (ratio) ratio[e] = 0.0;
    }
    return;
  }
  __shared__ double sin_[mm];
  __shared__ double s1[n * m * m];
  __shared__ double s2[n * n * m];
  __shared__ double sB[3 * nn];
  __shared__ double su[nn];
  __shared__ double sR[n * m];
  __shared__ double sL[n * n];
  __shared__ double sred[8];
  const int t = threadIdx.x;
  for (int q = t; q < n * m; q += 256) sR[q] = a.ops->R[q];
  for (int q = t; q < n * n; q += 256) sL[q] = a.ops->L[q];
  const bool isfd = rep[e] == 1;
  for (int c = 0; c < 3; ++c) {
    __syncthreads();
    if (isfd) {
      for (int q = t; q < mm; q += 256) sin_[q] = fd[((size_t)(3 + c) * a.E + e) * mm + q];
      __syncthreads();
      recon3<N>(sR, sin_, s1, s2, sB + c * nn);
    } else {
      for (int q = t; q < nn; q += 256) sB[c * nn + q] = dg[((size_t)(3 + c) * a.E + e) * nn + q];
    }
  }
  __syncthreads();
  const double r = block_ratio<N, CURVED>(a, e, sB, su, sred, sL);
  if (t == 0) {
    troubled[e] = r > (isfd ? a.tci_thr_fd : a.tci_thr) ? 1 : 0;
    if (ratio) ratio[e] = r;
  }
}

// Compact-layout transfers: to_fd = 1: P (x) P (x) P of [9][count][n^3] into [9][count][m^3];
// to_fd = 0: R (x) R (x) R the other way.
template <int N>
__global__ __launch_bounds__(256) void k_transfer(KArgs a, int to_fd, const double* in, double* out, int count) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, nn = Dm::nn, mm = Dm::mm;
  const int e = blockIdx.x;
  const int v = blockIdx.y;
  __shared__ double sin_[mm];
  __shared__ double s1[n * m * m + nn];  // P: first stage; R: first stage, then the result
  __shared__ double s2[m * m * n];       // P and R: second stage
  __shared__ double sO[n * m];
  const int t = threadIdx.x;
  if (to_fd) {
    for (int q = t; q < m * n; q += 256) sO[q] = a.ops->P[q];
    for (int q = t; q < nn; q += 256) sin_[q] = in[((size_t)v * count + e) * nn + q];
    __syncthreads();
    for (int q = t; q < m * n * n; q += 256) {
      const int cx = q % m, yz = q / m;
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += sO[cx * n + z] * sin_[yz * n + z];
      s1[q] = acc;
    }
    __syncthreads();
    for (int q = t; q < m * m * n; q += 256) {
      const int cx = q % m, cy = (q / m) % m, z0 = q / (m * m);
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += sO[cy * n + z] * s1[(z0 * n + z) * m + cx];
      s2[q] = acc;
    }
    __syncthreads();
    for (int q = t; q < mm; q += 256) {
      const int cxy = q % (m * m), cz = q / (m * m);
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += sO[cz * n + z] * s2[z * m * m + cxy];
      out[((size_t)v * count + e) * mm + q] = acc;
    }
  } else {
    for (int q = t; q < n * m; q += 256) sO[q] = a.ops->R[q];
    for (int q = t; q < mm; q += 256) sin_[q] = in[((size_t)v * count + e) * mm + q];
    __syncthreads();
    recon3<N>(sO, sin_, s1, s2, s1 + n * m * m);
    for (int q = t; q < nn; q += 256) out[((size_t)v * count + e) * nn + q] = s1[n * m * m + q];
  }
}

// Background at FD cells ([26][E][m^3], P along every axis) and at FD faces
// ([3][10][E][(m+1) m^2], face evaluation along d, P along the others).
template <int N>
__global__ __launch_bounds__(256) void k_bg_derive(KArgs a, double* bg_fd, double* bg_face, const double* Q) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, nn = Dm::nn, mm = Dm::mm;
  constexpr int nf = (m + 1) * m * m;
  const int e = blockIdx.x;
  const int fld = blockIdx.y;  // 0..25
  __shared__ double s0[nn];
  __shared__ double s1[(m + 1) * n * n];
  __shared__ double s2[(m + 1) * (m + 1) * n];
  __shared__ double sP[m * n];
  __shared__ double sQ[(m + 1) * n];
  const int t = threadIdx.x;
  for (int q = t; q < m * n; q += 256) sP[q] = a.ops->P[q];
  for (int q = t; q < (m + 1) * n; q += 256) sQ[q] = Q[q];
  for (int q = t; q < nn; q += 256) s0[q] = a.bg_dg[((size_t)fld * a.E + e) * nn + q];
  __syncthreads();
  const int ndir = (fld < NBGF) ? 4 : 1;  // cells, then faces along x, y, z
  for (int dir = 0; dir < ndir; ++dir) {
    // along each axis: Q if the axis is the face direction, else P
    const int lx = (dir == 1) ? m + 1 : m, ly = (dir == 2) ? m + 1 : m, lz = (dir == 3) ? m + 1 : m;
    const double* Ox = (dir == 1) ? sQ : sP;
    const double* Oy = (dir == 2) ? sQ : sP;
    const double* Oz = (dir == 3) ? sQ : sP;
    for (int q = t; q < lx * n * n; q += 256) {
      const int cx = q % lx, yz = q / lx;
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += Ox[cx * n + z] * s0[yz * n + z];
      s1[q] = acc;  // [z][y][cx]
    }
    __syncthreads();
    for (int q = t; q < lx * ly * n; q += 256) {
      const int cx = q % lx, cy = (q / lx) % ly, z0 = q / (lx * ly);
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += Oy[cy * n + z] * s1[(z0 * n + z) * lx + cx];
      s2[q] = acc;  // [z][cy][cx]
    }
    __syncthreads();
    const int tot = lx * ly * lz;
    for (int q = t; q < tot; q += 256) {
      const int cxy = q % (lx * ly), cz = q / (lx * ly);
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += Oz[cz * n + z] * s2[z * lx * ly + cxy];
      if (dir == 0) {
        bg_fd[((size_t)fld * a.E + e) * mm + q] = acc;
      } else {
        // q = cx + lx (cy + ly cz) is exactly the face ordering of direction dir-1
        bg_face[(((size_t)(dir - 1) * NBGF + fld) * a.E + e) * nf + q] = acc;
      }
    }
    __syncthreads();
  }
}

// Per-block maximum of the coordinate light speed over the live DG nodes.
template <int N>
__global__ __launch_bounds__(256) void k_lambda_max(KArgs a, double* out) {
  using Dm = Dims<N>;
  constexpr int nn = Dm::nn;
  const int e = blockIdx.x;
  __shared__ double sm[4];
  double v = 0.0;
  if (a.live[e]) {
    for (int p = threadIdx.x; p < nn; p += 256) {
      Metric M;
      load_metric<true>(a.bg_dg, a.E, nn, e, p, M);
      for (int d = 0; d < 3; ++d) v = fmax(v, char_speed(d, M));
    }
  }
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[e] = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
}


// ------------------------------------------------------------------ launchers
// Persistent grids of the list-driven kernels: enough workgroups to fill the chip,
// never more than the largest possible number of work items.
static dim3 list_grid(size_t max_items, int cap) {
  return dim3((unsigned)(max_items < (size_t)cap ? (max_items > 0 ? max_items : 1) : cap));
}

template <int N, bool CURVED>
static void fd_stage_t(const KArgs& a, int mode, hipStream_t s) {
  const dim3 grid = list_grid((size_t)a.E * ((Dims<N>::mm + 255) / 256), 2048), block(256);
  switch (mode) {
    case MODE_RHS: launch_kernel(k_fd_stage<N, CURVED, MODE_RHS>, grid, block, s, a); break;
    case MODE_SUB1: launch_kernel(k_fd_stage<N, CURVED, MODE_SUB1>, grid, block, s, a); break;
    case MODE_SUB2: launch_kernel(k_fd_stage<N, CURVED, MODE_SUB2>, grid, block, s, a); break;
    default: launch_kernel(k_fd_stage<N, CURVED, MODE_SUB3>, grid, block, s, a); break;
  }
}

void launch_fd_stage(const KArgs& a, int N, bool curved, int mode, hipStream_t s) {
  if (curved) GRFFE_SWITCH_N((fd_stage_t<NN, true>(a, mode, s)))
  else GRFFE_SWITCH_N((fd_stage_t<NN, false>(a, mode, s)))
}

void launch_fd_trace(const KArgs& a, int N, hipStream_t s) {
  GRFFE_SWITCH_N(launch_kernel(k_fd_trace<NN>, list_grid((size_t)a.E * NW, 4096), dim3(256), s, a))
}

template <int N, bool CURVED>
static void project_t(const KArgs& a, int mode, hipStream_t s) {
  switch (mode) {
    case MODE_SUB1: launch_kernel(k_project_troubled<N, CURVED, MODE_SUB1>, dim3(a.E), dim3(256), s, a); break;
    case MODE_SUB2: launch_kernel(k_project_troubled<N, CURVED, MODE_SUB2>, dim3(a.E), dim3(256), s, a); break;
    default: launch_kernel(k_project_troubled<N, CURVED, MODE_SUB3>, dim3(a.E), dim3(256), s, a); break;
  }
}

void launch_project_troubled(const KArgs& a, int N, bool curved, int mode, hipStream_t s) {
  if (curved) GRFFE_SWITCH_N((project_t<NN, true>(a, mode, s)))
  else GRFFE_SWITCH_N((project_t<NN, false>(a, mode, s)))
}

template <int N, bool CURVED>
static void fd_flux_t(const KArgs& a, hipStream_t s) {
  constexpr int m = Dims<N>::m;
  const dim3 grid = list_grid((size_t)a.E * 3 * m, 2048), block(flux_tpb<N>());
  if (a.precision == GRFFE_PRECISION_MIXED) launch_kernel(k_fd_flux<N, CURVED, float>, grid, block, s, a);
  else launch_kernel(k_fd_flux<N, CURVED, double>, grid, block, s, a);
}

void launch_fd_flux(const KArgs& a, int N, bool curved, hipStream_t s) {
  if (curved) GRFFE_SWITCH_N((fd_flux_t<NN, true>(a, s)))
  else GRFFE_SWITCH_N((fd_flux_t<NN, false>(a, s)))
}

template <int N, bool CURVED>
static void fd_update_t(const KArgs& a, int mode, hipStream_t s) {
  const dim3 grid = list_grid((size_t)a.E * ((Dims<N>::mm + 255) / 256), 2048), block(256);
  switch (mode) {
    case MODE_RHS: launch_kernel(k_fd_update<N, CURVED, MODE_RHS>, grid, block, s, a); break;
    case MODE_SUB1: launch_kernel(k_fd_update<N, CURVED, MODE_SUB1>, grid, block, s, a); break;
    case MODE_SUB2: launch_kernel(k_fd_update<N, CURVED, MODE_SUB2>, grid, block, s, a); break;
    default: launch_kernel(k_fd_update<N, CURVED, MODE_SUB3>, grid, block, s, a); break;
  }
}

void launch_fd_update(const KArgs& a, int N, bool curved, int mode, hipStream_t s) {
  if (curved) GRFFE_SWITCH_N((fd_update_t<NN, true>(a, mode, s)))
  else GRFFE_SWITCH_N((fd_update_t<NN, false>(a, mode, s)))
}

void launch_fd_to_dg_policy(const KArgs& a, int N, bool curved, int policy, const uint8_t* forced, hipStream_t s) {
  if (curved) GRFFE_SWITCH_N(launch_kernel(k_fd_to_dg<NN, true>, dim3(a.E), dim3(256), s, a, policy, forced, 0))
  else GRFFE_SWITCH_N(launch_kernel(k_fd_to_dg<NN, false>, dim3(a.E), dim3(256), s, a, policy, forced, 0))
}

void launch_fd_to_dg(const KArgs& a, int N, bool curved, int init, hipStream_t s) {
  if (init) {
    launch_fd_to_dg_policy(a, N, curved, init, nullptr, s);
    return;
  }
  // end of a step: the step's FD work list holds every element on FD
  const dim3 grid = list_grid((size_t)a.E, 2048);
  if (curved) GRFFE_SWITCH_N(launch_kernel(k_fd_to_dg<NN, true>, grid, dim3(256), s, a, 0, nullptr, 1))
  else GRFFE_SWITCH_N(launch_kernel(k_fd_to_dg<NN, false>, grid, dim3(256), s, a, 0, nullptr, 1))
}

void launch_begin_substep(const KArgs& a, bool copy, hipStream_t s) {
  launch_kernel(k_begin_substep, dim3((a.E + 255) / 256), dim3(256), s, a, copy ? 1 : 0);
}

void launch_tci(const KArgs& a, int N, bool curved, const double* dg, const double* fd, const int32_t* rep,
                uint8_t* troubled, double* ratio, hipStream_t s) {
  if (curved)
    GRFFE_SWITCH_N(launch_kernel(k_tci<NN, true>, dim3(a.E), dim3(256), s, a, dg, fd, rep, troubled, ratio))
  else
    GRFFE_SWITCH_N(launch_kernel(k_tci<NN, false>, dim3(a.E), dim3(256), s, a, dg, fd, rep, troubled, ratio))
}

void launch_transfer(const KArgs& a, int N, int to_fd, const double* in, double* out, int count, hipStream_t s) {
  GRFFE_SWITCH_N(launch_kernel(k_transfer<NN>, dim3(count, NV), dim3(256), s, a, to_fd, in, out, count))
}

void launch_bg_derive_q(const KArgs& a, int N, double* bg_fd, double* bg_face, const double* Q, hipStream_t s) {
  GRFFE_SWITCH_N(launch_kernel(k_bg_derive<NN>, dim3(a.E, NBG), dim3(256), s, a, bg_fd, bg_face, Q))
}

void launch_lambda_max(const KArgs& a, int N, double* out, hipStream_t s) {
  GRFFE_SWITCH_N(launch_kernel(k_lambda_max<NN>, dim3(a.E), dim3(256), s, a, out))
}

}  // namespace grffe
