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
#include "fd_common.h"

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
// sR[f] is the neighbour's representation: an FD neighbour's J~ is its R-trace's
// (read here from the trace buffer at the matched node of its face sFo[f]), not that
// of the traced state.
template <int N, int D, bool HYB>
__device__ inline void face_part(const KArgs& a, int e, int id, int tt, const int* sO, const int* sR,
                                 const int* sFo, const double* sX, const double* X, const double* J,
                                 const Metric& M, const double* ji, double* dU) {
  constexpr int NC = NV;
  constexpr int nf = (N + 1) * (N + 1);
  if (id != 0 && id != N) return;
  const int s = (id == N) ? 1 : 0;
  const int f = 2 * D + s;
  const int o = sO[f];
  if (o == NBR_OUTFLOW) return;  // the exterior state is the interior one
  const double sg = s ? 1.0 : -1.0;
  const double m[3] = {sg * ji[3 * D], sg * ji[3 * D + 1], sg * ji[3 * D + 2]};
  double Ux[NV], Jx[3];
  bool have_j = false;
  if (o >= 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) Ux[c] = sX[(f * NC + c) * nf + tt];
    if (HYB && sR[f] == 1) {
      constexpr int n = N + 1;
      const int pn = a.fnode[((size_t)e * 6 + f) * nf + tt];
      const int fo = sFo[f], dd = fo >> 1;
      const int ci[3] = {pn % n, (pn / n) % n, pn / (n * n)};
      const int u = ci[dd == 0 ? 1 : 0] + n * ci[dd == 2 ? 1 : 2];
#pragma unroll
      for (int c = 0; c < 3; ++c) Jx[c] = a.trace[(((size_t)(NV + c) * a.E + o) * 6 + fo) * nf + u];
      have_j = true;
    }
  } else if (o < -1) {
    const size_t fs = (size_t)a.E * 6 * nf;
    const double* b = a.bfield_dg + ((size_t)e * 6 + f) * nf + tt;
#pragma unroll
    for (int c = 0; c < NV; ++c) Ux[c] = b[c * fs];
  } else {
    boundary_state_normal(m, X, M, Ux);
  }
  double Gi[NV], Gx[NV];
  if (!have_j) current_total(Ux, M, a.eta, Jx);
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
//
// HYB: elements may be on FD (hybrid modes).  Only the DG elements run; an FD
// neighbour's face state is its R-trace (U and J~, written by the trace kernel),
// read at the face node matched to ours (U staged with the DG neighbours' states, J~
// read where the face term needs it); with the adaptive mode the troubled-cell
// indicator (Eq. persson tci) runs on the substep's result, and a troubled element
// is appended to the substep's FD list and keeps its substep-start registers for the
// FD redo, as on the box grid.
template <int N, bool CURVED, int MODE, bool HYB>
__global__ __launch_bounds__(Dims<N>::tpb, ((N <= 5 && MODE != MODE_RHS) ? 2 : 1)) void k_dg_mapped(KArgs a) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, nn = Dm::nn, nf = n * n, TPB = Dm::tpb;
  constexpr int NC = NV;
  constexpr int ITEMS = 6 * NC * nf, PER = (ITEMS + TPB - 1) / TPB;
  // at N <= 5 the three flux components are staged together and differentiated in
  // one fully unrolled loop (three independent accumulator chains per component);
  // above, one component at a time (the merged form spills at P7)
  constexpr bool MERGE = N <= 5;
  __shared__ double sF[MERGE ? 3 * NV * nn : NV * nn];
  __shared__ double sFil[n * n];  // filter
  __shared__ double sD[n * n];    // derivative matrix
  __shared__ double sX[ITEMS];    // neighbours' face nodes [f][c][t]
  __shared__ double sL[HYB ? n * n : 1];  // indicator operator
  __shared__ double sred[2 * (TPB / 64)];
  __shared__ int sO[6], sR[6], sFo[6];
  // XCD-aware order (as on the box grid): XCD x takes elements [x per, (x + 1) per)
  const int per = (a.E + 7) / 8;
  const int e = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (e >= a.E || !a.live[e] || (HYB && a.rep0[e] != 0)) return;
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int p = act ? t : 0;
  const int i = p % n, j = (p / n) % n, k = p / (n * n);
  if (t < 6) {
    const int o = a.nbr[e * 6 + t];
    sO[t] = o;
    sR[t] = (HYB && o >= 0) ? a.rep0[o] : 0;
    sFo[t] = (HYB && o >= 0) ? a.nface[e * 6 + t] : 0;
  }
  for (int q = t; q < n * n; q += TPB) {
    sD[q] = a.ops->D[q];
    sFil[q] = a.ops->F[q];
    if (HYB) sL[q] = a.ops->L[q];
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
      const int f = q / (NC * nf), c = (q / nf) % NC, tt = q % nf;
      const int o = sO[f];
      if (o < 0) continue;
      const int pn = a.fnode[((size_t)e * 6 + f) * nf + tt];
      if (HYB && sR[f] == 1) {
        // the FD neighbour's R-trace on its face towards us, at the matched node
        const int fo = sFo[f], dd = fo >> 1;
        const int ci[3] = {pn % n, (pn / n) % n, pn / (n * n)};
        const int u1 = ci[dd == 0 ? 1 : 0], u2 = ci[dd == 2 ? 1 : 2];
        v[r] = a.trace[(((size_t)c * a.E + o) * 6 + fo) * nf + u1 + n * u2];
      } else {
        v[r] = src[((size_t)c * a.E + o) * nn + pn];
      }
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
    face_part<N, 0, HYB>(a, e, i, j + n * k, sO, sR, sFo, sX, X, J, M, ji, dU);
    face_part<N, 1, HYB>(a, e, j, i + n * k, sO, sR, sFo, sX, X, J, M, ji, dU);
    face_part<N, 2, HYB>(a, e, k, i + n * j, sO, sR, sFo, sX, X, J, M, ji, dU);
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
  if (!HYB && !act) return;
  if (act) {
    if (MODE != MODE_SUB3) implicit_solve(Y, M, a.eta, a.kpsi, a.kphi, dt_of(a, e) * IMEX_A);
    if (a.ff_clamp) constraint_clamp(Y, M, a.ff_margin);
  }
  if (HYB && a.hybrid == GRFFE_HYBRID_ADAPTIVE) {
    // troubled-cell indicator on u = |B~| (every thread of the block takes part)
    const double u = act ? sqrt(dot3(M, Y + 3, Y + 3)) : 0.0;
    double uh = u;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      __syncthreads();
      if (act) sF[p] = uh;
      __syncthreads();
      const int id = idx[d];
      const int p0 = p - id * strideN[d];
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < n; ++q) acc += sL[id * n + q] * sF[p0 + q * strideN[d]];
      uh = acc;
    }
    double num = act ? (a.tci_mode == 1 ? uh * uh : (u - uh) * (u - uh)) : 0.0;
    double den = act ? u * u : 0.0;
    block_sum2<TPB>(num, den, sred);
    const double ratio = den > 0.0 ? sqrt(num / den) : 0.0;
    const bool bad = ratio > a.tci_thr || (a.force != nullptr && a.force[(size_t)(MODE - 1) * a.E + e] != 0);
    if (t == 0) {
      a.ratio[e] = ratio;
      if (bad) {
        a.troubled[e] = 1;
        a.fd_list[atomicAdd(a.fd_count + a.sub, 1)] = e;  // redone on FD in this substep
      }
    }
    if (bad) return;
  }
  if (!act) return;
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

// ---------------------------------------------------------------- FD subcells on curved elements
// Sec. III C 2, Eq. (fd time derivative), second order (F-hat = F*: the corrector is
// Cartesian only).  Work items: (listed FD element, reference direction d, plane of
// pencils t2), as on the box grid.  Per item: the m pencils along xi^d with three
// ghost cells per side are staged in LDS (all twelve transported components: every
// Cartesian flux needs its component of J~); ghost cells are the neighbour's cells
// next to the shared face in its own orientation (face cell from the host's match
// table), its P-slab if it is on DG, or on a sphere the outermost own cell (outflow),
// its no-incoming-Poynting state along the outward covector, or the given exterior
// state of the ghost cell (Dirichlet).  WENO5-Z gives both states at every face; the
// Rusanov flux of each Cartesian component j, with the dissipation along the face's
// unit covector nu, is
//   F-hat^j = (F^j(U_L) + F^j(U_R)) / 2 - lambda(nu) (U_R - U_L) nu_j / 2;
// each cell then takes -(m / 2) sum_j (d xi^d / d x^j) (F-hat^j_{+} - F-hat^j_{-})
// with the inverse Jacobian at its centre, written as direction d's share of the
// flux divergence for the update kernel.
template <int N, bool CURVED>
__global__ __launch_bounds__(flux_tpb<N>()) void k_fd_flux_mapped(KArgs a) {
  using Dm = Dims<N>;
  constexpr int m = Dm::m, mm = Dm::mm, mf = m * m;
  constexpr int nfc = (m + 1) * m * m;
  constexpr int L = m, C = m + 6, F = m + 1;
  constexpr int TPB = flux_tpb<N>();
  constexpr int NA = (NW * C > 3 * NV * F) ? NW * C * L : 3 * NV * F * L;
  __shared__ double sA[NA];          // staged cells [k][cell][pencil], then F-hat [j][v][face][pencil]
  // reconstructed states by target cell c = -1 .. m (slot c + 1): the left state of
  // face c + 1 in sLf (face f at slot f), the right state of face c in sRf (face f at
  // slot f + 1); the unused slots take the edge targets' other state
  constexpr int FP = m + 2;
  __shared__ double sLf[NW * FP * L];  // [k][slot][pencil]
  __shared__ double sRf[NW * FP * L];
  __shared__ int sNb[8];
  const int t = threadIdx.x;
  const int items = a.fd_count[a.sub] * 3 * m;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int e = a.fd_list[item / (3 * m)];
    const int d = (item / m) % 3;
    const int t2 = item % m;
    const int str[3] = {1, m, mf};
    const int t1ax = (d == 0) ? 1 : 0, t2ax = (d == 2) ? 1 : 2;
    __syncthreads();  // the previous item's tiles are no longer read
    if (t < 2) {
      const int f = 2 * d + t, o = a.nbr[e * 6 + f];
      sNb[t] = o;
      sNb[2 + t] = o >= 0 ? a.rep0[o] : -1;
      sNb[4 + t] = o >= 0 ? a.nface[e * 6 + f] : -1;
    }
    __syncthreads();
    // phase 1: cells -3 .. m+2 of every pencil
    for (int q = t; q < L * C; q += TPB) {
      int c, t1;
      if (d == 0) {
        c = q % C;
        t1 = q / C;
      } else {
        t1 = q % L;
        c = q / L;
      }
      const int cc = c - 3;
      double W[NW];
      if (cc >= 0 && cc < m) {
        const int idx = cc * str[d] + t1 * str[t1ax] + t2 * str[t2ax];
#pragma unroll
        for (int k = 0; k < NW; ++k) W[k] = a.w_fd[((size_t)k * a.E + e) * mm + idx];
      } else {
        const int s = cc >= m ? 1 : 0, f = 2 * d + s, l = s ? cc - m : -1 - cc;
        const int o = sNb[s];
        if (o >= 0) {
          const int tp = a.fcell[((size_t)e * 6 + f) * mf + t1 + m * t2];
          const int fo = sNb[4 + s];
          if (sNb[2 + s] == 1) {
            const int dd = fo >> 1, so = fo & 1;
            int ci[3];
            ci[dd] = so ? m - 1 - l : l;
            ci[dd == 0 ? 1 : 0] = tp % m;
            ci[dd == 2 ? 1 : 2] = tp / m;
            const int idx = ci[0] + m * ci[1] + mf * ci[2];
#pragma unroll
            for (int k = 0; k < NW; ++k) W[k] = a.w_fd[((size_t)k * a.E + o) * mm + idx];
          } else {
#pragma unroll
            for (int k = 0; k < NW; ++k)
              W[k] = a.slab[((size_t)k * a.E * 6 + (size_t)o * 6 + fo) * (3 * mf) + l * mf + tp];
          }
        } else {
          // a sphere: from the outermost own cell of the pencil
          const int ib = (s ? m - 1 : 0) * str[d] + t1 * str[t1ax] + t2 * str[t2ax];
#pragma unroll
          for (int k = 0; k < NW; ++k) W[k] = a.w_fd[((size_t)k * a.E + e) * mm + ib];
          if (o != NBR_OUTFLOW) {
            Metric Mc;
            load_metric<CURVED>(a.bg_fd, a.E, mm, e, ib, Mc);
            double Ub[NV], J[3];
            if (o == -1) {
              const double sg = s ? 1.0 : -1.0;
              double mv[3];
#pragma unroll
              for (int j = 0; j < 3; ++j) mv[j] = sg * a.jinv_fd[((size_t)(3 * d + j) * a.E + e) * mm + ib];
              boundary_state_normal(mv, W, Mc, Ub);
            } else {
              const size_t fs = (size_t)a.E * 6 * 3 * mf;
              const double* b = a.bfield_fd + (((size_t)e * 6 + f) * 3 + l) * mf + t1 + m * t2;
#pragma unroll
              for (int k = 0; k < NV; ++k) Ub[k] = b[k * fs];
            }
            current_total(Ub, Mc, a.eta, J);
#pragma unroll
            for (int k = 0; k < NV; ++k) W[k] = Ub[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) W[NV + k] = J[k];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < NW; ++k) sA[(k * C + c) * L + t1] = W[k];
    }
    __syncthreads();
    // phase 2: WENO5-Z of every component; target cells c = -1 .. m give the left
    // state of face c+1 and the right state of face c
    const double eps = a.weno_eps;
    // (the work index q = (k FP + c + 1) L + t1 is also the states' slot index, and
    // the target's cells c-2 .. c+2 start at extended index c+1 of component k's tile)
    for (int q = t; q < NW * L * FP; q += TPB) {
      const int k = q / (L * FP);
      const double* v = sA + q + k * (C - FP) * L;
      double vl[5];
#pragma unroll
      for (int z = 0; z < 5; ++z) vl[z] = v[z * L];
      double lft, rgt;
      weno5z_cell(vl, eps, lft, rgt);
      sLf[q] = lft;
      sRf[q] = rgt;
    }
    __syncthreads();
    // phase 3: F-hat^j at every face of every pencil, into sA
    for (int q = t; q < L * F; q += TPB) {
      int f3, t13;
      if (d == 0) {
        f3 = q % F;
        t13 = q / F;
      } else {
        t13 = q % L;
        f3 = q / L;
      }
      int tix;
      if (d == 0) tix = f3 + (m + 1) * (t13 + m * t2);
      else if (d == 1) tix = t13 + m * (f3 + (m + 1) * t2);
      else tix = t13 + m * (t2 + m * f3);
      double WL[NW], WR[NW];
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        WL[k] = sLf[(k * FP + f3) * L + t13];
        WR[k] = sRf[(k * FP + f3 + 1) * L + t13];
      }
      Metric Mf;
      load_metric<CURVED>(a.bg_face + (size_t)d * NBGF * a.E * nfc, a.E, nfc, e, tix, Mf);
      double nu[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) nu[j] = a.nu_face[((size_t)(3 * d + j) * a.E + e) * nfc + tix];
      const double lam =
          Mf.alpha * sqrt(gi_norm2(Mf, nu)) + fabs(Mf.beta[0] * nu[0] + Mf.beta[1] * nu[1] + Mf.beta[2] * nu[2]);
      double FL[NV], FR[NV];
      flux_dir<0>(WL, WL[NV], Mf, FL);
      flux_dir<0>(WR, WR[NV], Mf, FR);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        sA[((0 * NV + v) * F + f3) * L + t13] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam * nu[0] * (WR[v] - WL[v]);
      flux_dir<1>(WL, WL[NV + 1], Mf, FL);
      flux_dir<1>(WR, WR[NV + 1], Mf, FR);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        sA[((1 * NV + v) * F + f3) * L + t13] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam * nu[1] * (WR[v] - WL[v]);
      flux_dir<2>(WL, WL[NV + 2], Mf, FL);
      flux_dir<2>(WR, WR[NV + 2], Mf, FR);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        sA[((2 * NV + v) * F + f3) * L + t13] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam * nu[2] * (WR[v] - WL[v]);
    }
    __syncthreads();
    // phase 4: -(m/2) sum_j (d xi^d / d x^j) (F-hat^j_{c+1/2} - F-hat^j_{c-1/2}) per cell
    const double sc = 0.5 * (double)m;
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
      double ji[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) ji[j] = a.jinv_fd[((size_t)(3 * d + j) * a.E + e) * mm + cell];
      double* out = a.fhat + ((size_t)d * NV * a.E + e) * mm + cell;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double* fh = sA + ((j * NV + v) * F + c) * L + t1;
          acc += ji[j] * (fh[L] - fh[0]);
        }
        out[(size_t)v * a.E * mm] = -sc * acc;
      }
    }
  }
}

template <int N, bool CURVED>
static void launch_fd_flux_mapped_t(const KArgs& a, hipStream_t s) {
  constexpr int m = Dims<N>::m;
  const size_t cap = (size_t)a.E * 3 * m;
  const dim3 grid((unsigned)(cap < 2048 ? (cap > 0 ? cap : 1) : 2048)), block(flux_tpb<N>());
  launch_kernel(k_fd_flux_mapped<N, CURVED>, grid, block, s, a);
}

void launch_fd_flux_mapped(const KArgs& a, int N, bool curved, hipStream_t s) {
  if (curved) {
    GRFFE_SWITCH_N((launch_fd_flux_mapped_t<NN, true>(a, s)))
  } else {
    GRFFE_SWITCH_N((launch_fd_flux_mapped_t<NN, false>(a, s)))
  }
}

template <int N, bool CURVED, bool HYB>
static void launch_dg_mapped_t(const KArgs& a, int mode, hipStream_t s) {
  dim3 grid(8 * ((a.E + 7) / 8)), block(Dims<N>::tpb);
  switch (mode) {
    case MODE_RHS: launch_kernel(k_dg_mapped<N, CURVED, MODE_RHS, HYB>, grid, block, s, a); break;
    case MODE_SUB1: launch_kernel(k_dg_mapped<N, CURVED, MODE_SUB1, HYB>, grid, block, s, a); break;
    case MODE_SUB2: launch_kernel(k_dg_mapped<N, CURVED, MODE_SUB2, HYB>, grid, block, s, a); break;
    default: launch_kernel(k_dg_mapped<N, CURVED, MODE_SUB3, HYB>, grid, block, s, a); break;
  }
}

void launch_dg_mapped(const KArgs& a, int N, bool curved, int mode, bool hybrid, hipStream_t s) {
  if (curved && hybrid) {
    GRFFE_SWITCH_N((launch_dg_mapped_t<NN, true, true>(a, mode, s)))
  } else if (curved) {
    GRFFE_SWITCH_N((launch_dg_mapped_t<NN, true, false>(a, mode, s)))
  } else if (hybrid) {
    GRFFE_SWITCH_N((launch_dg_mapped_t<NN, false, true>(a, mode, s)))
  } else {
    GRFFE_SWITCH_N((launch_dg_mapped_t<NN, false, false>(a, mode, s)))
  }
}

}  // namespace grffe
