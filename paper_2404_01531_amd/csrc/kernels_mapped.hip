// DG substep on curved element maps (the spherical shell of cubed-sphere wedges,
// Sec. IV B; Sec. III A with a non-affine map x(xi) per element).
//
// One workgroup per element, one thread per GLL node, every element on DG.  The
// strong-form operator takes the logical derivative of each Cartesian flux
// component and contracts it with the inverse Jacobian at the node,
//   dU/dt = S - sum_{i,j} (d xi^i / d x^j) D_i F^j - sum_faces lift,
// (the placement of the inverse Jacobian of the paper's FD time derivative, Eq.
// (fd time derivative)); a node of the face xi^i = +-1 adds
//   -(1 / w_end) (G*(m) - m_j F^j(U_int)),
// with m = +-grad xi^i (row i of the inverse Jacobian) and the Rusanov flux along m,
// G*(m) = m_j (F^j_int + F^j_ext) / 2 - lambda(m) (U_ext - U_int) / 2,
// lambda(m) = alpha sqrt(gamma^{jk} m_j m_k) + |beta^j m_j|.  The exterior state of
// a face node is the neighbour's node at the same point (the host matched them:
// faces between wedges meet in other orientations).  The rest of the substep --
// stage input, sources, IMEX stage update, exponential filter on the explicit
// update, pointwise implicit solve and the optional clamp -- is the box grid's.
#include "common.h"

namespace grffe {

// gamma^{jk} m_j m_k
__device__ inline double gi_norm2(const Metric& M, const double* m) {
  return M.gi[0] * m[0] * m[0] + M.gi[3] * m[1] * m[1] + M.gi[5] * m[2] * m[2] +
         2.0 * (M.gi[1] * m[0] * m[1] + M.gi[2] * m[0] * m[2] + M.gi[4] * m[1] * m[2]);
}

// m_j F^j(U) with the current J
__device__ inline void normal_flux(const double* U, const double* J, const Metric& M, const double* m, double* G) {
  double F[NV];
  flux_dir<0>(U, J[0], M, F);
#pragma unroll
  for (int v = 0; v < NV; ++v) G[v] = m[0] * F[v];
  flux_dir<1>(U, J[1], M, F);
#pragma unroll
  for (int v = 0; v < NV; ++v) G[v] += m[1] * F[v];
  flux_dir<2>(U, J[2], M, F);
#pragma unroll
  for (int v = 0; v < NV; ++v) G[v] += m[2] * F[v];
}

// No-incoming-Poynting state (Sec. III D) along the outward covector m: E~, B~, q~
// copied, psi~ = phi~ = 0, E~ = 0 where m_i [ijk] E~_j B~_k < 0.
__device__ inline void boundary_state_normal(const double* m, const double* Ui, const Metric& M, double* Ub) {
  double El[3], Bl[3];
  lower3(M, Ui, El);
  lower3(M, Ui + 3, Bl);
  const double S = m[0] * (El[1] * Bl[2] - El[2] * Bl[1]) + m[1] * (El[2] * Bl[0] - El[0] * Bl[2]) +
                   m[2] * (El[0] * Bl[1] - El[1] * Bl[0]);
  const bool inward = S < 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Ub[i] = inward ? 0.0 : Ui[i];
    Ub[3 + i] = Ui[3 + i];
  }
  Ub[6] = 0.0;
  Ub[7] = 0.0;
  Ub[8] = Ui[8];
}

// Derivative along reference direction D of the nine staged components at node p
// (its index along D is id): acc[v] = sum_q D[id][q] sF[v][line(p) at q].
template <int N, int D>
__device__ inline void ref_derivative(const double* sF, const double* sD, int p, int id, double* acc) {
  constexpr int n = N + 1, nn = n * n * n, str = D == 0 ? 1 : (D == 1 ? n : n * n);
  const int p0 = p - id * str;
  const double* Drow = sD + id * n;
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll 1
  for (int q = 0; q < n; ++q) {
    const double dq = Drow[q];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += dq * sF[v * nn + p0 + q * str];
  }
}

// Volume term of the Cartesian flux component JD: dU -= sum_i (d xi^i / d x^JD) D_i F^JD.
// Every thread of the block calls it (it stages F^JD in LDS).
template <int N, int JD>
__device__ inline void volume_part(const double* X, const double* J, const Metric& M, const double* ji, double* sF,
                                   const double* sD, bool act, int p, int i, int j, int k, double* dU) {
  constexpr int nn = (N + 1) * (N + 1) * (N + 1);
  double F[NV], acc[NV];
  flux_dir<JD>(X, J[JD], M, F);
  __syncthreads();
  if (act)
    for (int v = 0; v < NV; ++v) sF[v * nn + p] = F[v];
  __syncthreads();
  ref_derivative<N, 0>(sF, sD, p, i, acc);
#pragma unroll
  for (int v = 0; v < NV; ++v) dU[v] -= ji[JD] * acc[v];
  ref_derivative<N, 1>(sF, sD, p, j, acc);
#pragma unroll
  for (int v = 0; v < NV; ++v) dU[v] -= ji[3 + JD] * acc[v];
  ref_derivative<N, 2>(sF, sD, p, k, acc);
#pragma unroll
  for (int v = 0; v < NV; ++v) dU[v] -= ji[6 + JD] * acc[v];
}

// Lift of the face of reference direction D on which the node lies (index id along
// D, face node tt), if any.
template <int N, int D>
__device__ inline void face_part(const KArgs& a, int e, int id, int tt, const int* sO, const double* sX,
                                 const double* X, const double* J, const Metric& M, const double* ji, double* dU) {
  constexpr int nf = (N + 1) * (N + 1);
  if (id != 0 && id != N) return;
  const int s = (id == N) ? 1 : 0;
  const int f = 2 * D + s;
  const int o = sO[f];
  if (o == NBR_OUTFLOW) return;  // the exterior state is the interior one
  const double sg = s ? 1.0 : -1.0;
  const double m[3] = {sg * ji[3 * D], sg * ji[3 * D + 1], sg * ji[3 * D + 2]};
  double Ux[NV];
  if (o >= 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) Ux[c] = sX[(f * NV + c) * nf + tt];
  } else if (o < -1) {
    const size_t fs = (size_t)a.E * 6 * nf;
    const double* b = a.bfield_dg + ((size_t)e * 6 + f) * nf + tt;
#pragma unroll
    for (int c = 0; c < NV; ++c) Ux[c] = b[c * fs];
  } else {
    boundary_state_normal(m, X, M, Ux);
  }
  double Jx[3], Gi[NV], Gx[NV];
  current_total(Ux, M, a.eta, Jx);
  normal_flux(X, J, M, m, Gi);
  normal_flux(Ux, Jx, M, m, Gx);
  const double lam = M.alpha * sqrt(gi_norm2(M, m)) + fabs(M.beta[0] * m[0] + M.beta[1] * m[1] + M.beta[2] * m[2]);
  const double wl = 1.0 / a.ops->w[s ? N : 0];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double G = 0.5 * (Gi[v] + Gx[v]) - 0.5 * lam * (Ux[v] - X[v]);
    dU[v] -= wl * (G - Gi[v]);
  }
}

// The three Cartesian flux components staged together (sF3 [j][v][node]): each
// reference derivative reads the three at the same line point, three independent
// accumulator chains per component.
template <int N, int D>
__device__ inline void ref_derivative3(const double* sF3, const double* sD, int p, int id, const double* ji,
                                       double* dU) {
  constexpr int n = N + 1, nn = n * n * n, str = D == 0 ? 1 : (D == 1 ? n : n * n);
  const int p0 = p - id * str;
  const double* Drow = sD + id * n;
  const double c0 = ji[3 * D], c1 = ji[3 * D + 1], c2 = ji[3 * D + 2];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < n; ++q) {
      const double dq = Drow[q];
      const int o = v * nn + p0 + q * str;
      s0 += dq * sF3[o];
      s1 += dq * sF3[NV * nn + o];
      s2 += dq * sF3[2 * NV * nn + o];
    }
    dU[v] -= c0 * s0 + c1 * s1 + c2 * s2;
  }
}

// Workgroups per CU: two at N <= 5 in the substeps (256 VGPRs, two waves per SIMD,
// 12 B of spills per lane, against one wave and 120 AGPRs unbounded: 1023 -> 620 us
// per launch on the 32 x 384 P5 shell); the right-hand side entry point would spill
// ~500 B there and keeps one.
template <int N, bool CURVED, int MODE>
__global__ __launch_bounds__(Dims<N>::tpb, ((N <= 5 && MODE != MODE_RHS) ? 2 : 1)) void k_dg_mapped(KArgs a) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, nn = Dm::nn, nf = n * n, TPB = Dm::tpb;
  constexpr int ITEMS = 6 * NV * nf, PER = (ITEMS + TPB - 1) / TPB;
  // at N <= 5 the three flux components are staged together and differentiated in
  // one fully unrolled loop (three independent accumulator chains per component);
  // above, one component at a time (the merged form spills at P7)
  constexpr bool MERGE = N <= 5;
  __shared__ double sF[MERGE ? 3 * NV * nn : NV * nn];
  __shared__ double sFil[n * n];  // filter
  __shared__ double sD[n * n];    // derivative matrix
  __shared__ double sX[ITEMS];    // neighbours' face nodes [f][c][t]
  __shared__ int sO[6];
  // XCD-aware order (as on the box grid): XCD x takes elements [x per, (x + 1) per)
  const int per = (a.E + 7) / 8;
  const int e = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (e >= a.E || !a.live[e]) return;
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int p = act ? t : 0;
  const int i = p % n, j = (p / n) % n, k = p / (n * n);
  if (t < 6) sO[t] = a.nbr[e * 6 + t];
  for (int q = t; q < n * n; q += TPB) {
    sD[q] = a.ops->D[q];
    sFil[q] = a.ops->F[q];
  }
  Metric M;
  load_metric<CURVED>(a.bg_dg, a.E, nn, e, p, M);
  double ji[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) ji[q] = a.jinv[((size_t)q * a.E + e) * nn + p];
  double X[NV];
  stage_input<MODE, true>(a.dg, a.E, nn, e, p, M, a, X);
  __syncthreads();
  {
    // the neighbours' stage input at their nodes facing this element's face nodes:
    // all loads first, then the LDS writes
    const double* src = (MODE == MODE_RHS) ? a.dg.Un : (MODE == MODE_SUB2 ? a.dg.X0 : a.dg.X1);
    double v[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int q = t + r * TPB;
      v[r] = 0.0;
      if (q >= ITEMS) continue;
      const int f = q / (NV * nf), c = (q / nf) % NV, tt = q % nf;
      const int o = sO[f];
      if (o < 0) continue;
      const int pn = a.fnode[((size_t)e * 6 + f) * nf + tt];
      v[r] = src[((size_t)c * a.E + o) * nn + pn];
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int q = t + r * TPB;
      if (q < ITEMS) sX[q] = v[r];
    }
  }
  double Jd[3], Je[3], dU[NV];
  current(X, M, a.eta, Jd, Je);
  {
    MetricDeriv Dv;
    load_deriv<CURVED>(a.bg_dg, a.E, nn, e, p, Dv);
    source_explicit<CURVED>(X, M, Dv, Jd, dU);
  }
  double J[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) J[c] = Jd[c] + Je[c];
  // volume term: every Cartesian flux component differentiated along every
  // reference direction, contracted with the inverse Jacobian at the node
  if (MERGE) {
    double F[NV];
    flux_dir<0>(X, J[0], M, F);
    if (act)
      for (int v = 0; v < NV; ++v) sF[v * nn + p] = F[v];
    flux_dir<1>(X, J[1], M, F);
    if (act)
      for (int v = 0; v < NV; ++v) sF[(NV + v) * nn + p] = F[v];
    flux_dir<2>(X, J[2], M, F);
    if (act)
      for (int v = 0; v < NV; ++v) sF[(2 * NV + v) * nn + p] = F[v];
    __syncthreads();
    ref_derivative3<N, 0>(sF, sD, p, i, ji, dU);
    ref_derivative3<N, 1>(sF, sD, p, j, ji, dU);
    ref_derivative3<N, 2>(sF, sD, p, k, ji, dU);
  } else {
    volume_part<N, 0>(X, J, M, ji, sF, sD, act, p, i, j, k, dU);
    volume_part<N, 1>(X, J, M, ji, sF, sD, act, p, i, j, k, dU);
    volume_part<N, 2>(X, J, M, ji, sF, sD, act, p, i, j, k, dU);
  }
  // face terms
  if (act) {
    face_part<N, 0>(a, e, i, j + n * k, sO, sX, X, J, M, ji, dU);
    face_part<N, 1>(a, e, j, i + n * k, sO, sX, X, J, M, ji, dU);
    face_part<N, 2>(a, e, k, i + n * j, sO, sX, X, J, M, ji, dU);
  }
  const int idx[3] = {i, j, k};
  const int strideN[3] = {1, n, n * n};
  if (MODE == MODE_RHS) {
    if (!act) return;
    double St[NV];
    source_stiff(X, M, a.eta, a.kpsi, a.kphi, St);
    double out[NV];
    for (int v = 0; v < NV; ++v) out[v] = ((a.parts & 1) ? dU[v] : 0.0) + ((a.parts & 2) ? St[v] : 0.0);
    store9(a.out_dg, a.E, nn, e, p, out);
    return;
  }
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
      const double* Frow = sFil + id * n;
      const int str = strideN[d];
#pragma unroll
      for (int v = 0; v < NV; ++v) Y[v] = 0.0;
#pragma unroll 1
      for (int q = 0; q < n; ++q) {
        const double fq = Frow[q];
#pragma unroll
        for (int v = 0; v < NV; ++v) Y[v] += fq * sF[v * nn + p0 + q * str];
      }
    }
  }
  if (!act) return;
  if (MODE != MODE_SUB3) implicit_solve(Y, M, a.eta, a.kpsi, a.kphi, dt_of(a, e) * IMEX_A);
  if (a.ff_clamp) constraint_clamp(Y, M, a.ff_margin);
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

template <int N, bool CURVED>
static void launch_dg_mapped_t(const KArgs& a, int mode, hipStream_t s) {
  dim3 grid(8 * ((a.E + 7) / 8)), block(Dims<N>::tpb);
  switch (mode) {
    case MODE_RHS: launch_kernel(k_dg_mapped<N, CURVED, MODE_RHS>, grid, block, s, a); break;
    case MODE_SUB1: launch_kernel(k_dg_mapped<N, CURVED, MODE_SUB1>, grid, block, s, a); break;
    case MODE_SUB2: launch_kernel(k_dg_mapped<N, CURVED, MODE_SUB2>, grid, block, s, a); break;
    default: launch_kernel(k_dg_mapped<N, CURVED, MODE_SUB3>, grid, block, s, a); break;
  }
}

void launch_dg_mapped(const KArgs& a, int N, bool curved, int mode, hipStream_t s) {
  if (curved) {
    GRFFE_SWITCH_N((launch_dg_mapped_t<NN, true>(a, mode, s)))
  } else {
    GRFFE_SWITCH_N((launch_dg_mapped_t<NN, false>(a, mode, s)))
  }
}

}  // namespace grffe
