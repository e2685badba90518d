// Adjoint of the hybrid control inside a step (Sec. III C 1) with its decisions
// frozen from the forward pass: an element flagged in substep k redid that substep
// on FD from its DG registers projected by P (U^n, the substep's input, the
// accumulator; the FD pre-stages re-derived from P U^n), and an FD element that
// passes the indicator at the end of the step became R U^{n+1} on DG.  The
// transposes: Rᵀ of the end switch, and at the rollback the FD adjoints of the
// projected registers taken back through Pᵀ into the DG registers' adjoints, after
// the adjoints of the re-derived FD pre-stages have been folded into that of U^n.
// P (m x n) and R (n x m) act per axis; their transposes here are applied in three
// separable stages as in the forward transfers.
#include "adjoint.h"

namespace grffe {

// out (n^3) = (P^T x P^T x P^T) in (m^3): out[a + n (b + n c)] =
// sum P[cx][a] P[cy][b] P[cz][c] in[cx + m (cy + m cz)].  All threads call it.
template <int N>
__device__ inline void pt3(const double* sP, const double* in, double* s1, double* s2, double* out_lds) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m;
  const int t = threadIdx.x;
  __syncthreads();
  for (int q = t; q < m * m * n; q += 256) {  // [cz][cy][a]
    const int a = q % n, r = q / n;
    double acc = 0.0;
    for (int z = 0; z < m; ++z) acc += sP[z * n + a] * in[r * m + z];
    s1[q] = acc;
  }
  __syncthreads();
  for (int q = t; q < m * n * n; q += 256) {  // [cz][b][a]
    const int a = q % n, b = (q / n) % n, cz = q / (n * n);
    double acc = 0.0;
    for (int z = 0; z < m; ++z) acc += sP[z * n + b] * s1[(cz * m + z) * n + a];
    s2[q] = acc;
  }
  __syncthreads();
  for (int q = t; q < n * n * n; q += 256) {  // [c][b][a]
    const int ab = q % (n * n), c = q / (n * n);
    double acc = 0.0;
    for (int z = 0; z < m; ++z) acc += sP[z * n + c] * s2[z * n * n + ab];
    out_lds[q] = acc;
  }
  __syncthreads();
}

// Transition at the rollback in substep k of the elements flagged there (a.rep0 DG
// at the substep start, rep_upd FD): for k = 2, 3 the FD pre-stage adjoints (s1, s2
// of the FD registers) folded into U^n's, then U^n, the accumulator and the substep
// input (the transfer vector written by the FD stage kernel) taken through P^T to
// DG (written: the DG chain of the element resumes here); for k = 1 (the FD chain
// has already run through its pre-stages) U^n only.  The DG stiff-term adjoints
// start at zero.
template <int N, bool CURVED>
__global__ __launch_bounds__(256) void k_adj_rollback(KArgs a, AdjBufs rd, AdjBufs rf, const int32_t* rep_upd,
                                                      const double* t_fd, double* t_dg, int k) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, nn = Dm::nn, mm = Dm::mm;
  const int e = blockIdx.x;
  if (!a.live[e] || a.rep0[e] != 0 || rep_upd[e] != 1) return;
  __shared__ double sP[m * n];
  __shared__ double sin_[mm];
  __shared__ double s1[m * m * n];
  __shared__ double s2[m * n * n];
  __shared__ double so[nn];
  const int t = threadIdx.x;
  for (int q = t; q < m * n; q += 256) sP[q] = a.ops->P[q];
  const double dt = dt_of(a, e);
  if (k >= 2) {
    // U^n's adjoint gains the FD pre-stages' (S1, S2 of the re-derived U_1, U_2)
    for (int p = t; p < mm; p += 256) {
      Metric M;
      load_metric<CURVED>(a.bg_fd, a.E, mm, e, p, M);
      double Un[NV], U1[NV], U2[NV], S1[NV], s2b[NV], ubU2[NV];
      load9(a.fd.Un, a.E, mm, e, p, Un);
      pre_stages(Un, M, a, dt, U1, U2, S1);
      load9(rf.s2_bar, a.E, mm, e, p, s2b);
#pragma unroll
      for (int v = 0; v < NV; ++v) ubU2[v] = 0.0;
      stiff_vjp(U2, M, a, s2b, ubU2);
      if (k == 3) {
        // the FD chain ended before substep 2's combination: no S1 adjoint on FD
        const double zero[NV] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        store9(rf.s1_bar, a.E, mm, e, p, zero);
      }
      adj_b1_tail(a, rf, a.E, mm, e, p, M, dt, U2, U1, ubU2);
    }
  }
  // registers through P^T: U^n (always), accumulator and substep input (k >= 2)
  const int nreg = k >= 2 ? 3 : 1;
  for (int r = 0; r < nreg; ++r) {
    const double* src = r == 0 ? rf.un_bar : (r == 1 ? rf.a_bar : t_fd);
    double* dst = r == 0 ? rd.un_bar : (r == 1 ? rd.a_bar : t_dg);
    for (int v = 0; v < NV; ++v) {
      __syncthreads();
      for (int q = t; q < mm; q += 256) sin_[q] = src[((size_t)v * a.E + e) * mm + q];
      pt3<N>(sP, sin_, s1, s2, so);
      for (int q = t; q < nn; q += 256) dst[((size_t)v * a.E + e) * nn + q] = so[q];
    }
  }
  // the DG stiff-term adjoints of the element start here (its DG pre-stages fed
  // only the substeps before k)
  for (int q = t; q < NV * nn; q += 256) {
    const int v = q / nn, p = q % nn;
    rd.s1_bar[((size_t)v * a.E + e) * nn + p] = 0.0;
    rd.s2_bar[((size_t)v * a.E + e) * nn + p] = 0.0;
  }
}

// troubled[e] = 1 for the elements rolled back in the substep (on DG at its start,
// a.rep0, and updated on FD), so that the ghost slabs are made as in the forward.
__global__ __launch_bounds__(256) void k_adj_flags(KArgs a, const int32_t* rep_upd) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= a.E) return;
  a.troubled[e] = (a.live[e] && a.rep0[e] == 0 && rep_upd[e] == 1) ? 1 : 0;
}

// The end switch transposed: an element that was FD in substep 3 and is DG after
// the step (rep3 FD, repF DG) has mu_fd = (R^T x R^T x R^T) mu_dg.
template <int N>
__global__ __launch_bounds__(256) void k_adj_switch_back(KArgs a, const int32_t* rep3, const int32_t* repF,
                                                         const double* mu_dg, double* mu_fd) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, nn = Dm::nn, mm = Dm::mm;
  const int e = blockIdx.x;
  if (!a.live[e] || rep3[e] != 1 || repF[e] != 0) return;
  __shared__ double sR[n * m];
  __shared__ double sin_[nn];
  __shared__ double s1[n * n * m];
  __shared__ double s2[n * m * m];
  const int t = threadIdx.x;
  for (int q = t; q < n * m; q += 256) sR[q] = a.ops->R[q];
  for (int v = 0; v < NV; ++v) {
    __syncthreads();
    for (int q = t; q < nn; q += 256) sin_[q] = mu_dg[((size_t)v * a.E + e) * nn + q];
    __syncthreads();
    for (int q = t; q < n * n * m; q += 256) {  // [c][b][cx]
      const int cx = q % m, r = q / m;
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += sR[z * m + cx] * sin_[r * n + z];
      s1[q] = acc;
    }
    __syncthreads();
    for (int q = t; q < n * m * m; q += 256) {  // [c][cy][cx]
      const int cx = q % m, cy = (q / m) % m, c = q / (m * m);
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += sR[z * m + cy] * s1[(c * n + z) * m + cx];
      s2[q] = acc;
    }
    __syncthreads();
    for (int q = t; q < mm; q += 256) {  // [cz][cy][cx]
      const int cxy = q % (m * m), cz = q / (m * m);
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += sR[z * m + cz] * s2[z * m * m + cxy];
      mu_fd[((size_t)v * a.E + e) * mm + q] = acc;
    }
  }
}

// U^n on FD of the elements flagged during the step (rep0 DG, rep3 FD): P U^n, as the
// forward projection made it (the FD pre-stages of those elements are taken there).
template <int N>
__global__ __launch_bounds__(256) void k_adj_project_un(KArgs a, const int32_t* rep0, const int32_t* rep3,
                                                        const double* un_dg, double* un_fd) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, nn = Dm::nn, mm = Dm::mm;
  const int e = blockIdx.x;
  if (!a.live[e] || rep0[e] != 0 || rep3[e] != 1) return;
  __shared__ double sP[m * n];
  __shared__ double s0[nn];
  __shared__ double s1[m * n * n];
  __shared__ double s2[m * m * n];
  const int t = threadIdx.x;
  for (int q = t; q < m * n; q += 256) sP[q] = a.ops->P[q];
  for (int v = 0; v < NV; ++v) {
    __syncthreads();
    for (int q = t; q < nn; q += 256) s0[q] = un_dg[((size_t)v * a.E + e) * nn + q];
    __syncthreads();
    for (int q = t; q < m * n * n; q += 256) {  // [z][y][cx]
      const int cx = q % m, yz = q / m;
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += sP[cx * n + z] * s0[yz * n + z];
      s1[q] = acc;
    }
    __syncthreads();
    for (int q = t; q < m * m * n; q += 256) {  // [z][cy][cx]
      const int cx = q % m, cy = (q / m) % m, z0 = q / (m * m);
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += sP[cy * n + z] * s1[(z0 * n + z) * m + cx];
      s2[q] = acc;
    }
    __syncthreads();
    for (int q = t; q < mm; q += 256) {  // [cz][cy][cx]
      const int cxy = q % (m * m), cz = q / (m * m);
      double acc = 0.0;
      for (int z = 0; z < n; ++z) acc += sP[cz * n + z] * s2[z * m * m + cxy];
      un_fd[((size_t)v * a.E + e) * mm + q] = acc;
    }
  }
}

// dst = src on the live elements whose representation in rep is `want`: one
// (component, element) row of P values per workgroup pass, rows of other elements
// skipped whole (32-bit row arithmetic; the rows are contiguous in the [9][E][P]
// layout).
__global__ __launch_bounds__(256) void k_copy_rep(const KArgs a, const int32_t* rep, int want, int P,
                                                  const double* src, double* dst) {
  const int rows = NV * a.E;
  for (int r = blockIdx.x; r < rows; r += gridDim.x) {
    const int e = r % a.E;
    if (!a.live[e] || rep[e] != want) continue;  // the same for every thread of the block
    const size_t base = (size_t)r * P;
    for (int p = threadIdx.x; p < P; p += 256) dst[base + p] = src[base + p];
  }
}

void launch_adj_rollback(const KArgs& a, int N, bool curved, const AdjBufs& rd, const AdjBufs& rf,
                         const int32_t* rep_upd, const double* t_fd, double* t_dg, int k, hipStream_t s) {
  if (curved)
    GRFFE_SWITCH_N(launch_kernel(k_adj_rollback<NN, true>, dim3(a.E), dim3(256), s, a, rd, rf, rep_upd, t_fd, t_dg, k))
  else
    GRFFE_SWITCH_N(launch_kernel(k_adj_rollback<NN, false>, dim3(a.E), dim3(256), s, a, rd, rf, rep_upd, t_fd, t_dg, k))
}

void launch_adj_flags(const KArgs& a, const int32_t* rep_upd, hipStream_t s) {
  launch_kernel(k_adj_flags, dim3((a.E + 255) / 256), dim3(256), s, a, rep_upd);
}

void launch_adj_switch_back(const KArgs& a, int N, const int32_t* rep3, const int32_t* repF, const double* mu_dg,
                            double* mu_fd, hipStream_t s) {
  GRFFE_SWITCH_N(launch_kernel(k_adj_switch_back<NN>, dim3(a.E), dim3(256), s, a, rep3, repF, mu_dg, mu_fd))
}

void launch_adj_project_un(const KArgs& a, int N, const int32_t* rep0, const int32_t* rep3, const double* un_dg,
                           double* un_fd, hipStream_t s) {
  GRFFE_SWITCH_N(launch_kernel(k_adj_project_un<NN>, dim3(a.E), dim3(256), s, a, rep0, rep3, un_dg, un_fd))
}

void launch_copy_rep(const KArgs& a, const int32_t* rep, int want, int P, const double* src, double* dst,
                     hipStream_t s) {
  const int rows = NV * a.E;
  launch_kernel(k_copy_rep, dim3(rows < 4096 ? rows : 4096), dim3(256), s, a, rep, want, P, src, dst);
}

}  // namespace grffe
