// DG kernels: the fused per-element DG substep and the DG -> FD ghost slabs.
//
// One workgroup per element, one thread per GLL node (Sec. III A).  The
// strong-form DG-SEM operator with a lumped GLL mass matrix is
//   dU/dt = -sum_d (2/h_d) [ D_d F^d + W^-1 (e_N (F*_+ - F_N) - e_0 (F*_- - F_0)) ] + S,
// the face flux F* is Rusanov with speed max(lambda_int, lambda_ext),
// lambda = alpha sqrt(gamma^dd) + |beta^d|.  The whole substep -- stage input,
// fluxes, derivative and lift, sources, IMEX stage update, exponential filter
// (Eq. exponential filter) on the explicit update, pointwise implicit solve,
// optional algebraic clamp and the troubled-cell indicator (Eq. persson tci) --
// runs in one launch; the candidate is written only when it is admissible, so a
// troubled element keeps its substep-start registers for the FD redo.
#include "common.h"

namespace grffe {

// Exterior data of the element's six faces, staged in LDS at the start of the
// substep so that their loads are in flight together with the element's own: for a
// DG neighbour its stage input at the nodes of its face towards this element (the
// nine state components), for an FD neighbour its R-trace on that face (state and
// J~).  Layout sX[f][c][t1 + n t2], with (t1, t2) the face node's two tangential
// indices in increasing axis order; sO[f], sR[f] hold the neighbour across face f
// and its representation (set by the caller, visible to every thread).
template <int N, int MODE, int TPB>
__device__ inline void stage_faces(const KArgs& a, const int* sO, const int* sR, double* sX) {
  constexpr int n = N + 1, nf = n * n, nn = n * n * n;
  constexpr int ITEMS = 6 * NW * nf, PER = (ITEMS + TPB - 1) / TPB;
  const double* src = (MODE == MODE_RHS) ? a.dg.Un : (MODE == MODE_SUB2 ? a.dg.X0 : a.dg.X1);
  const int t = threadIdx.x;
  double v[PER];
  // all loads first, then the LDS writes: one memory latency for the whole stage
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int q = t + r * TPB;
    v[r] = 0.0;
    if (q >= ITEMS) continue;
    const int f = q / (NW * nf), c = (q / nf) % NW, tt = q % nf;
    const int o = sO[f], ro = sR[f];
    if (o < 0) continue;
    const int d = f >> 1, s = f & 1;
    if (ro == 0) {
      if (c >= NV) continue;
      const int t1 = tt % n, t2 = tt / n, lay = s ? 0 : N;  // the neighbour's layer facing us
      const int pn = (d == 0) ? lay + n * (t1 + n * t2) : (d == 1 ? t1 + n * (lay + n * t2) : t1 + n * (t2 + n * lay));
      v[r] = src[((size_t)c * a.E + o) * nn + pn];
    } else {
      const int fo = 2 * d + (1 - s);
      v[r] = a.trace[(((size_t)c * a.E + o) * 6 + fo) * nf + tt];
    }
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int q = t + r * TPB;
    if (q < ITEMS) sX[q] = v[r];
  }
}

// External (neighbour or boundary) state (Ux, Jx) at the face node tt of face 2 d + s, from
// the staged face data (neighbour o, representation ro).  The face node is one point
// of a continuous background: the element's own nodal metric Mi there is the
// neighbour's as well.
template <int N>
__device__ inline void external_state(const KArgs& a, int e, int d, int s, int o, int ro, int tt, const double* sX,
                                      const double* Ui, const Metric& Mi, double* Ux, double* Jx) {
  constexpr int nf = (N + 1) * (N + 1);
  if (o < 0) {
    exterior_state(a, o, d, s, Ui, Mi, a.bfield_dg, ((size_t)e * 6 + 2 * d + s) * nf + tt, (size_t)a.E * 6 * nf, Ux);
    current_total(Ux, Mi, a.eta, Jx);
    return;
  }
  const double* x = sX + (size_t)(2 * d + s) * NW * nf + tt;
#pragma unroll
  for (int c = 0; c < NV; ++c) Ux[c] = x[c * nf];
  if (ro == 0) {
    current_total(Ux, Mi, a.eta, Jx);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) Jx[c] = x[(NV + c) * nf];
  }
}

// The derivative contraction of one direction on the matrix cores: for every column
// (component v, line of the element along d) out[v][node(line, i)] = sum_q D[i][q]
// F[v][node(line, q)], as 16 x 16 x 4 FP64 MFMA tiles (rows i and the contraction
// index q padded to 16 and to a multiple of 4, 16 columns per tile, the tiles dealt
// to the workgroup's wavefronts).  Operand layouts of v_mfma_f64_16x16x4: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; result register r holds row 4 r + l / 16,
// column l % 16.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <int N, int TPB, int D>
__device__ inline void mfma_derivative(const double* sFd, const double* sDd, double* sOut) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, COLS = NV * nf, TILES = (COLS + 15) / 16;
  constexpr int KS = (n + 3) / 4, WAVES = TPB / 64;
  constexpr int STR = D == 0 ? 1 : (D == 1 ? n : nf);
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lo = l & 15, kq = l >> 4;
  double av[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int q = 4 * ks + kq;
    av[ks] = (lo < n && q < n) ? sDd[lo * n + q] : 0.0;
  }
  for (int tile = w; tile < TILES; tile += WAVES) {
    const int c = 16 * tile + lo;
    const bool cv = c < COLS;
    const int v = cv ? c / nf : 0, line = cv ? c % nf : 0;
    const int t1 = line % n, t2 = line / n;
    const int base = v * nn + (D == 0 ? n * (t1 + n * t2) : (D == 1 ? t1 + nf * t2 : t1 + n * t2));
    mfma_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int q = 4 * ks + kq;
      const double b = (cv && q < n) ? sFd[base + q * STR] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * r + kq;
      if (cv && i < n) sOut[base + i * STR] = acc[r];
    }
  }
}

// Workgroups per CU the substep kernel is compiled for: two resident wavefronts per
// SIMD when curved (about 256 VGPRs per lane hold the metric next to the state),
// three when flat.
template <int N, bool CURVED>
constexpr int dg_min_blocks() {
  constexpr int waves = Dims<N>::tpb / 64;
  constexpr int want = (CURVED ? 2 : 3) * 4 / waves;
  return want > 1 ? want : 1;
}

template <int N, bool CURVED, int MODE, typename R, bool MF = false>
__global__ __launch_bounds__(Dims<N>::tpb, (dg_min_blocks<N, CURVED>())) void k_dg_substep(KArgs a) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, nn = Dm::nn, TPB = Dm::tpb;
  static_assert(!MF || sizeof(R) == sizeof(double), "the MFMA contraction is the FP64 one");
  __shared__ double sF[NV * nn];
  __shared__ double sOut[MF ? NV * nn : 1];  // the MFMA contraction's results
  __shared__ double sred[2 * (TPB / 64)];
  __shared__ double sop[2 * n * n];  // filter, indicator operator
  __shared__ R sD[n * n];            // derivative matrix in the flux arithmetic type
  __shared__ double sX[6 * NW * n * n];  // exterior face data
  __shared__ int sO[6], sR[6];
  // XCD-aware order: workgroups are dealt to the eight XCDs in turn, each with its
  // own L2; XCD x takes the contiguous run of elements [x per, (x + 1) per), so the
  // face data an element reads from its neighbours is mostly in the same L2 (the
  // grid is 8 per blocks; those past the last element exit)
  const int per = (a.E + 7) / 8;
  const int e = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (e >= a.E || !a.live[e] || a.rep0[e] != 0) return;
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int p = act ? t : 0;
  const int i = p % n, j = (p / n) % n, k = p / (n * n);
  if (t < 6) {
    const int o = a.nbr[e * 6 + t];
    sO[t] = o;
    sR[t] = o >= 0 ? a.rep0[o] : -1;
  }
  for (int q = t; q < n * n; q += TPB) {
    sD[q] = (R)a.ops->D[q];
    sop[q] = a.ops->F[q];
    sop[n * n + q] = a.ops->L[q];
  }
  Metric M;
  load_metric_dg_r<CURVED, R>(a, nn, e, p, M);
  double X[NV], Jd[3], Je[3], dU[NV];
  stage_input<MODE, true>(a.dg, a.E, nn, e, p, M, a, X);
  __syncthreads();
  stage_faces<N, MODE, TPB>(a, sO, sR, sX);
  current(X, M, a.eta, Jd, Je);
  {
    MetricDeriv Dv;
    load_deriv_dg_r<CURVED, R>(a, nn, e, p, Dv);
    source_explicit<CURVED>(X, M, Dv, Jd, dU);
  }
  // fluxes, derivative and lift in R (FP64, or FP32 in the mixed-precision mode),
  // accumulated in R and added to the FP64 sources
  MetricT<R> Mr;
  metric_cast(M, Mr);
  R Xr[NV], Jr[3], dUr[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    Xr[v] = (R)X[v];
    dUr[v] = 0;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) Jr[c] = (R)(Jd[c] + Je[c]);
  R* sFr = reinterpret_cast<R*>(sF);
  const int idx[3] = {i, j, k};
  const int strideN[3] = {1, n, n * n};
  #pragma unroll
  for (int d = 0; d < 3; ++d) {
    R F[NV];
    flux_any(d, Xr, Jr, Mr, F);
    __syncthreads();
    if (act)
      for (int v = 0; v < NV; ++v) sFr[v * nn + p] = F[v];
    __syncthreads();
    const double sc = 2.0 / h_of(a, e, d);
    const int id = idx[d];
    const int p0 = p - id * strideN[d];
    if (MF) {
      if (d == 0) mfma_derivative<N, TPB, 0>(sF, reinterpret_cast<const double*>(sD), sOut);
      else if (d == 1) mfma_derivative<N, TPB, 1>(sF, reinterpret_cast<const double*>(sD), sOut);
      else mfma_derivative<N, TPB, 2>(sF, reinterpret_cast<const double*>(sD), sOut);
      __syncthreads();
#pragma unroll
      for (int v = 0; v < NV; ++v) dUr[v] -= (R)sc * (R)sOut[v * nn + p];
    } else {
      const R* Drow = sD + id * n;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        R acc = 0;
#pragma unroll
        for (int q = 0; q < n; ++q) acc += Drow[q] * sFr[v * nn + p0 + q * strideN[d]];
        dUr[v] -= (R)sc * acc;
      }
    }
    if (act && (id == 0 || id == N)) {
      const int s = (id == N) ? 1 : 0;
      const int f = 2 * d + s;
      const int tt = (d == 0) ? j + n * k : (d == 1 ? i + n * k : i + n * j);
      double Wx[NV], Jx[3];
      external_state<N>(a, e, d, s, sO[f], sR[f], tt, sX, X, M, Wx, Jx);
      R Wr[NV], Jxr[3], Fx[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Wr[v] = (R)Wx[v];
#pragma unroll
      for (int c = 0; c < 3; ++c) Jxr[c] = (R)Jx[c];
      flux_any(d, Wr, Jxr, Mr, Fx);
      // Rusanov speed: the larger of the two sides', which share the metric
      const R lam = CURVED ? (R)char_speed(d, M) : R(1);
      if (s == 0) {
        const R wl = (R)(sc / a.ops->w[0]);
        for (int v = 0; v < NV; ++v) {
          const R Fs = R(0.5) * (Fx[v] + F[v]) - R(0.5) * lam * (Xr[v] - Wr[v]);
          dUr[v] += wl * (Fs - F[v]);
        }
      } else {
        const R wr = (R)(sc / a.ops->w[N]);
        for (int v = 0; v < NV; ++v) {
          const R Fs = R(0.5) * (F[v] + Fx[v]) - R(0.5) * lam * (Wr[v] - Xr[v]);
          dUr[v] -= wr * (Fs - F[v]);
        }
      }
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) dU[v] += (double)dUr[v];
  if (MODE == MODE_RHS) {
    if (!act) return;
    double St[NV];
    source_stiff(X, M, a.eta, a.kpsi, a.kphi, St);
    double out[NV];
    for (int v = 0; v < NV; ++v) out[v] = ((a.parts & 1) ? dU[v] : 0.0) + ((a.parts & 2) ? St[v] : 0.0);
    store9(a.out_dg, a.E, nn, e, p, out);
    return;
  }
  // IMEX stage update, filter on the explicit update, implicit solve
  double Y[NV], Anew[NV];
  stage_update<MODE, true>(a.dg, a.E, nn, e, p, M, a, X, dU, Y, Anew);
  if (a.filter_on) {
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      __syncthreads();
      if (act)
        for (int v = 0; v < NV; ++v) sF[v * nn + p] = Y[v];
      __syncthreads();
      const int id = idx[d];
      const int p0 = p - id * strideN[d];
      const double* Frow = sop + id * n;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < n; ++q) acc += Frow[q] * sF[v * nn + p0 + q * strideN[d]];
        Y[v] = acc;
      }
    }
  }
  if (MODE != MODE_SUB3) implicit_solve(Y, M, a.eta, a.kpsi, a.kphi, dt_of(a, e) * IMEX_A);
  if (a.ff_clamp) constraint_clamp(Y, M, a.ff_margin);
  // troubled-cell indicator on u = |B~|
  bool bad = false;
  if (a.hybrid == GRFFE_HYBRID_ADAPTIVE) {
    const double u = act ? sqrt(dot3(M, Y + 3, Y + 3)) : 0.0;
    double uh = u;
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      __syncthreads();
      if (act) sF[p] = uh;
      __syncthreads();
      const int id = idx[d];
      const int p0 = p - id * strideN[d];
      const double* Lrow = sop + n * n + id * n;
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < n; ++q) acc += Lrow[q] * sF[p0 + q * strideN[d]];
      uh = acc;
    }
    double num = act ? (a.tci_mode == 1 ? uh * uh : (u - uh) * (u - uh)) : 0.0;
    double den = act ? u * u : 0.0;
    block_sum2<TPB>(num, den, sred);
    const double ratio = den > 0.0 ? sqrt(num / den) : 0.0;
    bad = ratio > a.tci_thr || (a.force != nullptr && a.force[(size_t)(MODE - 1) * a.E + e] != 0);
    if (t == 0) {
      a.ratio[e] = ratio;
      if (bad) {
        a.troubled[e] = 1;
        a.fd_list[atomicAdd(a.fd_count + a.sub, 1)] = e;  // redone on FD in this substep
      }
    }
  }
  if (bad || !act) return;
  if (MODE == MODE_SUB1) {
    store9(a.dg.X0, a.E, nn, e, p, Y);
    store9(a.dg.A, a.E, nn, e, p, Anew);
  } else if (MODE == MODE_SUB2) {
    store9(a.dg.X1, a.E, nn, e, p, Y);
    store9(a.dg.A, a.E, nn, e, p, Anew);
  } else {
    store9(a.dg.Un, a.E, nn, e, p, Y);
  }
}

// Pre-stage pass at the start of a step, pointwise on every DG node: the implicit
// stages U_1 = solve(U^n), U_2 = solve(U^n - a dt S(U_1)) of IMEX-SSP3(4,3,3) depend
// on U^n alone, so they are computed once per step: U_2 (the input of substep 1)
// goes to X1, and the stiff-source terms that substeps 2 and 3 add,
// dt (b S(U_1) + e S(U_2)) and dt S(U_2) / 6, go to K (their five non-zero
// components).  Neighbours read U_2 from X1 for their face states.
template <int N, bool CURVED>
__global__ __launch_bounds__(256) void k_dg_prestage(KArgs a) {
  constexpr int nn = Dims<N>::nn;
  const int gid = blockIdx.x * 256 + threadIdx.x;
  // the step's FD work list starts empty (substep 1 builds it, substeps 2 and 3
  // extend it with the elements they flag)
  if (gid == 0) a.fd_count[0] = 0;
  const int e = gid / nn, p = gid % nn;
  if (e >= a.E || !a.live[e] || a.rep[e] != 0) return;
  Metric M;
  load_metric_dg<CURVED>(a, nn, e, p, M);
  double Un[NV], U2[NV], S1[NV], S2[NV];
  load9(a.dg.Un, a.E, nn, e, p, Un);
  const double dt = dt_of(a, e);
  derived_stages(Un, M, a, dt, U2, S1, S2);
  store9(a.dg.X1, a.E, nn, e, p, U2);
  store_stiff_terms(a.dg, a.E, nn, e, p, dt, S1, S2);
}

// P-projection (3 subcell layers next to each face) of the DG stage input of
// elements whose neighbour across that face is on FD or has just been flagged.
// Work items: (listed element o, face f of o), the list holding the elements on FD
// at the substep start and those flagged in it: the DG neighbour e across f projects
// its face towards o.  Every (e, face) pair is one item, so no two items write the
// same slab.  The twelve transported components (U, J~) are projected together in
// three separable stages.
template <int N, bool CURVED, int MODE>
__global__ __launch_bounds__(Dims<N>::tpb) void k_dg_slab(KArgs a) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, nn = Dm::nn, TPB = Dm::tpb;
  // the components are projected in chunks of CH so that the tiles fit in LDS at high degree
  constexpr int CH = (NW * (nn + 3 * n * n + 3 * m * n) * 8 <= 150 * 1024) ? NW : NW / 2;
  __shared__ double sW[NW * nn];
  __shared__ double sA[CH * 3 * n * n];
  __shared__ double sB[CH * 3 * m * n];
  __shared__ double sP[m * n];
  const int t = threadIdx.x;
  for (int q = t; q < m * n; q += TPB) sP[q] = a.ops->P[q];
  const int str[3] = {1, n, n * n};
  const int items = a.fd_count[a.sub] * 6;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int o = a.fd_list[item / 6], fo = item % 6;
    const int e = a.nbr[o * 6 + fo];
    if (e < 0 || !a.live[e] || a.rep0[e] != 0) continue;  // the same for every thread of the block
    // e's face towards o (the opposite face on the box grid; a table on shells)
    const int f = a.nface ? a.nface[o * 6 + fo] : 2 * (fo >> 1) + 1 - (fo & 1);
    __syncthreads();  // the previous item's tiles are no longer read
    if (t < nn) {
      Metric M;
      load_metric_dg<CURVED>(a, nn, e, t, M);
      double X[NV];
      stage_input<MODE, true>(a.dg, a.E, nn, e, t, M, a, X);
      double J[3];
      current_total(X, M, a.eta, J);
      for (int v = 0; v < NV; ++v) sW[v * nn + t] = X[v];
      for (int c = 0; c < 3; ++c) sW[(9 + c) * nn + t] = J[c];
    }
    __syncthreads();
    const int d = f >> 1, s = f & 1;
    // axes: normal d, tangential t1 < t2
    const int t1ax = (d == 0) ? 1 : 0, t2ax = (d == 2) ? 1 : 2;
    for (int c0 = 0; c0 < NW; c0 += CH) {
      // 1) normal direction: layers l = 0..2, cell index m-1-l (upper face) or l (lower face)
      for (int q = t; q < CH * 3 * n * n; q += TPB) {
        const int c = q / (3 * n * n), r0 = q % (3 * n * n);
        const int l = r0 / (n * n), r = r0 % (n * n);
        const int a1 = r % n, a2 = r / n;
        const int cell = s ? (m - 1 - l) : l;
        const double* W = sW + (c0 + c) * nn;
        double acc = 0.0;
        for (int z = 0; z < n; ++z) acc += sP[cell * n + z] * W[z * str[d] + a1 * str[t1ax] + a2 * str[t2ax]];
        sA[q] = acc;  // [c][l][a2][a1]
      }
      __syncthreads();
      // 2) first tangential axis: a1 (n) -> c1 (m)
      for (int q = t; q < CH * 3 * m * n; q += TPB) {
        const int c1 = q % m, rest = q / m;  // rest = (c*3 + l)*n + a2
        double acc = 0.0;
        for (int z = 0; z < n; ++z) acc += sP[c1 * n + z] * sA[rest * n + z];
        sB[q] = acc;  // [c][l][a2][c1]
      }
      __syncthreads();
      // 3) second tangential axis: a2 (n) -> c2 (m), written as [c][l][c2][c1]
      for (int q = t; q < CH * 3 * m * m; q += TPB) {
        const int c1 = q % m, c2 = (q / m) % m, cl = q / (m * m);  // cl = c*3 + l
        const int c = c0 + cl / 3, l = cl % 3;
        double acc = 0.0;
        for (int z = 0; z < n; ++z) acc += sP[c2 * n + z] * sB[(cl * n + z) * m + c1];
        a.slab[((size_t)c * a.E * 6 + (size_t)e * 6 + f) * (3 * m * m) + (l * m + c2) * m + c1] = acc;
      }
      __syncthreads();
    }
  }
}

template <int N, bool CURVED, typename R, bool MF>
static void launch_dg_substep_r(const KArgs& a, int mode, hipStream_t s) {
  dim3 grid(8 * ((a.E + 7) / 8)), block(Dims<N>::tpb);
  switch (mode) {
    case MODE_RHS: launch_kernel(k_dg_substep<N, CURVED, MODE_RHS, R, MF>, grid, block, s, a); break;
    case MODE_SUB1: launch_kernel(k_dg_substep<N, CURVED, MODE_SUB1, R, MF>, grid, block, s, a); break;
    case MODE_SUB2: launch_kernel(k_dg_substep<N, CURVED, MODE_SUB2, R, MF>, grid, block, s, a); break;
    default: launch_kernel(k_dg_substep<N, CURVED, MODE_SUB3, R, MF>, grid, block, s, a); break;
  }
}

template <int N, bool CURVED>
static void launch_dg_substep_t(const KArgs& a, int mode, hipStream_t s) {
  if (a.precision == GRFFE_PRECISION_MIXED) launch_dg_substep_r<N, CURVED, float, false>(a, mode, s);
  // (at N = 9 the MFMA result tile does not fit in LDS beside the others: VALU there)
  else if (a.contraction == GRFFE_CONTRACTION_MFMA) launch_dg_substep_r<N, CURVED, double, (N <= 8)>(a, mode, s);
  else launch_dg_substep_r<N, CURVED, double, false>(a, mode, s);
}

template <int N, bool CURVED>
static void launch_dg_slab_t(const KArgs& a, int mode, hipStream_t s) {
  // persistent grid over the (listed element, face) items: enough workgroups to fill
  // the chip, never more than the largest possible number of items
  const size_t max_items = (size_t)a.E * 6;
  dim3 grid((unsigned)(max_items < 2048 ? max_items : 2048)), block(Dims<N>::tpb);
  switch (mode) {
    case MODE_RHS: launch_kernel(k_dg_slab<N, CURVED, MODE_RHS>, grid, block, s, a); break;
    case MODE_SUB1: launch_kernel(k_dg_slab<N, CURVED, MODE_SUB1>, grid, block, s, a); break;
    case MODE_SUB2: launch_kernel(k_dg_slab<N, CURVED, MODE_SUB2>, grid, block, s, a); break;
    default: launch_kernel(k_dg_slab<N, CURVED, MODE_SUB3>, grid, block, s, a); break;
  }
}

// Element-wise rounding of an FP64 array to FP32 (the mixed-precision background copy).
__global__ __launch_bounds__(256) void k_to_float(const double* in, float* out, size_t count) {
  for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < count; q += (size_t)gridDim.x * 256)
    out[q] = (float)in[q];
}

void launch_to_float(const double* in, float* out, size_t count, hipStream_t s) {
  const size_t blocks = (count + 255) / 256;
  launch_kernel(k_to_float, dim3((unsigned)(blocks < 8192 ? (blocks > 0 ? blocks : 1) : 8192)), dim3(256), s, in, out,
                count);
}

// Elements holding a non-finite value in their own representation (DG registers
// U^n for DG elements, FD registers U^n for FD elements): bad[e] = 1, else 0.
__global__ __launch_bounds__(256) void k_check_finite(KArgs a, int nn, int mm, uint8_t* bad) {
  const int e = blockIdx.x;
  __shared__ int flag;
  if (threadIdx.x == 0) flag = 0;
  __syncthreads();
  if (a.live[e]) {
    const bool fd = a.rep[e] == 1;
    const double* u = fd ? a.fd.Un : a.dg.Un;
    const int P = fd ? mm : nn;
    int mine = 0;
    for (int q = threadIdx.x; q < NV * P; q += 256) {
      const int v = q / P, p = q % P;
      if (!isfinite(u[((size_t)v * a.E + e) * P + p])) mine = 1;
    }
    if (mine) flag = 1;  // every writer stores the same value
  }
  __syncthreads();
  if (threadIdx.x == 0) bad[e] = (uint8_t)flag;
}

void launch_check_finite(const KArgs& a, int nn, int mm, uint8_t* bad, hipStream_t s) {
  launch_kernel(k_check_finite, dim3(a.E), dim3(256), s, a, nn, mm, bad);
}

#define GRFFE_DISPATCH_N(FN, ...)                 \
  switch (N) {                                    \
    case 3: FN<3, CURVED_T>(__VA_ARGS__); break;  \
    case 4: FN<4, CURVED_T>(__VA_ARGS__); break;  \
    case 5: FN<5, CURVED_T>(__VA_ARGS__); break;  \
    case 6: FN<6, CURVED_T>(__VA_ARGS__); break;  \
    case 7: FN<7, CURVED_T>(__VA_ARGS__); break;  \
    case 8: FN<8, CURVED_T>(__VA_ARGS__); break;  \
    default: FN<9, CURVED_T>(__VA_ARGS__); break; \
  }

void launch_dg_substep(const KArgs& a, int N, bool curved, int mode, hipStream_t s) {
  if (curved) {
#define CURVED_T true
    GRFFE_DISPATCH_N(launch_dg_substep_t, a, mode, s)
#undef CURVED_T
  } else {
#define CURVED_T false
    GRFFE_DISPATCH_N(launch_dg_substep_t, a, mode, s)
#undef CURVED_T
  }
}

template <int N, bool CURVED>
static void launch_dg_prestage_t(const KArgs& a, hipStream_t s) {
  const int blocks = (int)(((size_t)a.E * Dims<N>::nn + 255) / 256);
  launch_kernel(k_dg_prestage<N, CURVED>, dim3(blocks), dim3(256), s, a);
}

void launch_dg_prestage(const KArgs& a, int N, bool curved, hipStream_t s) {
  if (curved) {
#define CURVED_T true
    GRFFE_DISPATCH_N(launch_dg_prestage_t, a, s)
#undef CURVED_T
  } else {
#define CURVED_T false
    GRFFE_DISPATCH_N(launch_dg_prestage_t, a, s)
#undef CURVED_T
  }
}

void launch_dg_slab(const KArgs& a, int N, bool curved, int mode, hipStream_t s) {
  if (curved) {
#define CURVED_T true
    GRFFE_DISPATCH_N(launch_dg_slab_t, a, mode, s)
#undef CURVED_T
  } else {
#define CURVED_T false
    GRFFE_DISPATCH_N(launch_dg_slab_t, a, mode, s)
#undef CURVED_T
  }
}

}  // namespace grffe
