// Adjoint (vector-Jacobian products) of the DG right-hand side and of the
// IMEX-SSP3(4,3,3) step.  The representation is frozen (the indicator is not
// differentiated); the step adjoint holds every element on DG, the right-hand side
// adjoint takes any mix of DG and FD elements (this file covers the DG elements;
// the FD elements and the two couplings are in the FD adjoint).
//
// The explicit DG operator at a node p of element e is (Sec. III A, strong form)
//   L(X)_p = -sum_d s_d [ sum_q D[i_d(p)][q] F^d(X_q) ] + lift terms + S_ex(X_p),
// with s_d = 2/h_d and the Rusanov face terms of the lower (s = 0) and upper
// (s = 1) faces.  Its transpose applied to V gathers, at every node r:
//   - the transposed derivative g_d(r) = -s_d sum_p D[i_d(p)][i_d(r)] V(p) along
//     the three lines through r, multiplied by (dF^d/dX)^T at r;
//   - the node's own face terms and the terms of the neighbouring DG element's
//     faces whose exterior state is X_r (no scatter: every element gathers from its
//     neighbours' V at the mirror nodes; an FD neighbour sees X only through the
//     projected ghost slab, whose transpose is applied separately);
//   - (dS_ex/dX)^T V(r), and at physical boundaries the derivative through the
//     no-incoming-Poynting state.
// All products with pointwise Jacobians are formed as the gradient of one scalar
// functional of X_r, evaluated with forward-mode dual numbers (one pass per
// component), so they are exact up to rounding.
//
// The step adjoint runs the step's stages backwards (substep 3, 2, 1, then the two
// implicit pre-stages); the implicit solve U = Y + h S_stiff(U) has the adjoint
//   Y_bar = (I - h dS_stiff/dU)^-T U_bar
// (a 9x9 solve per node), the filter the transposed tensor-product filter.
#include "adjoint.h"

namespace grffe {

// Element-wise transposed filter of the nine fields held in sZ (LDS, [9][nn]) at
// node p: returns (F^T x F^T x F^T) Z at p.  All threads of the block must call it.
template <int N>
__device__ inline void filter_transpose(const double* sF, double* sZ, int p, bool act, double* Z) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, nn = Dm::nn;
  const int idx[3] = {p % n, (p / n) % n, p / (n * n)};
  const int str[3] = {1, n, n * n};
  for (int d = 0; d < 3; ++d) {
    __syncthreads();
    if (act)
      for (int v = 0; v < NV; ++v) sZ[v * nn + p] = Z[v];
    __syncthreads();
    const int id = idx[d];
    const int p0 = p - id * str[d];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < n; ++q) acc += sF[q * n + id] * sZ[v * nn + p0 + q * str[d]];
      Z[v] = acc;
    }
  }
}

// ub = (dL_ex/dX)^T V + (dS_stiff/dX)^T W at node p of element e, where L_ex is the
// explicit DG operator evaluated on the stage field X (own value X, metric M).
// V is read from b.v_in for this element and its neighbours, W is given.
// use_v / use_w switch the two parts off.  All threads of the block must call it.
// own_v = false keeps only the neighbours' terms (the element's own operator
// result was discarded: rolled back to FD in this substep).
template <int N, bool CURVED>
__device__ void operator_vjp(const KArgs& a, const AdjBufs& b, int e, int p, bool act, const double* X,
                             const Metric& M, const double* Wst, bool use_v, bool use_w, double* sV, const double* sD,
                             double* ub, bool own_v = true) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, nn = Dm::nn;
  const int idx[3] = {p % n, (p / n) % n, p / (n * n)};
  const int str[3] = {1, n, n * n};
  const int32_t* upd = b.rep_upd ? b.rep_upd : a.rep0;
  double Vp[NV];
  __syncthreads();
  if (use_v && own_v) {
    if (act) load9(b.v_in, a.E, nn, e, p, Vp);
  } else {
    for (int v = 0; v < NV; ++v) Vp[v] = 0.0;
  }
  if (use_v && act)
    for (int v = 0; v < NV; ++v) sV[v * nn + p] = Vp[v];
  __syncthreads();
  for (int v = 0; v < NV; ++v) ub[v] = 0.0;
  double G[3][NV];
  // boundary faces of this node: coefficient of V.F^d(B(X)) and of V.B(X)
  double bA[3] = {0.0, 0.0, 0.0}, bI[3] = {0.0, 0.0, 0.0};
  int bside[3] = {0, 0, 0};
  if (use_v) {
    for (int d = 0; d < 3; ++d) {
      const double sc = 2.0 / h_of(a, e, d);
      const int id = idx[d];
      const int p0 = p - id * str[d];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < n; ++q) acc += sD[q * n + id] * sV[v * nn + p0 + q * str[d]];
        G[d][v] = -sc * acc;
      }
      if (!act || (id != 0 && id != N)) continue;
      const int s = (id == N) ? 1 : 0;
      const double wl = sc / a.ops->w[0], wr = sc / a.ops->w[N];
      // the node's own face term (interior dependence)
      const int o = a.nbr[e * 6 + 2 * d + s];
      int pn = 0;
      if (o >= 0) {
        int ii = idx[0], jj = idx[1], kk = idx[2];
        if (d == 0) ii = s ? 0 : N;
        else if (d == 1) jj = s ? 0 : N;
        else kk = s ? 0 : N;
        pn = ii + n * (jj + n * kk);
      }
      // both sides of a face node use the element's own nodal metric (one point of
      // a continuous background), so the Rusanov speed is that of X's node
      const double lam = CURVED ? char_speed(d, M) : 1.0;
      if (s == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          G[d][v] += -0.5 * wl * Vp[v];
          ub[v] += -0.5 * wl * lam * Vp[v];
        }
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          G[d][v] += 0.5 * wr * Vp[v];
          ub[v] += -0.5 * wr * lam * Vp[v];
        }
      }
      if (o < 0) {
        // exterior state = no-incoming-Poynting state of X itself (a Dirichlet face's
        // exterior state is constant)
        if (o == -1) {
          bside[d] = s ? 1 : -1;
          bA[d] = s ? -0.5 * wr : 0.5 * wl;
          bI[d] = s ? 0.5 * wr * lam : 0.5 * wl * lam;
        }
      } else if (upd[o] == 0) {
        // the neighbour updated on DG: its face term on its opposite face uses X as
        // exterior state
        const double sco = 2.0 / h_of(a, o, d);
        double Vo[NV];
        load9(b.v_in, a.E, nn, o, pn, Vo);
        if (s == 1) {  // neighbour's lower face
          const double wlo = sco / a.ops->w[0];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            G[d][v] += 0.5 * wlo * Vo[v];
            ub[v] += 0.5 * wlo * lam * Vo[v];
          }
        } else {  // neighbour's upper face
          const double wro = sco / a.ops->w[N];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            G[d][v] += -0.5 * wro * Vo[v];
            ub[v] += 0.5 * wro * lam * Vo[v];
          }
        }
      }
    }
  }
  if (!act) return;
  // gradient of  sum_d G_d.F^d(X) + V.S_ex(X) + W.S_stiff(X) + boundary terms: the
  // parts linear in X transposed by hand, the current's part by dual numbers
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  if (use_v) {
    MetricDeriv Dv;
    load_deriv<CURVED>(a.bg_dg, a.E, nn, e, p, Dv);
    flux_lin_vjp<0>(M, G[0], acc);
    flux_lin_vjp<1>(M, G[1], acc);
    flux_lin_vjp<2>(M, G[2], acc);
    source_lin_vjp<CURVED>(M, Dv, Vp, acc);
  }
  if (use_w) {
    acc[6] += -M.alpha * a.kpsi * Wst[6];
    acc[7] += -M.alpha * a.kphi * Wst[7];
  }
  {
    // J~^d enters F^d_q with weight G_d[8]; S_ex,E = -J_drift; S_stiff,E = -J_driver
    double wa[3], wb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      wa[i] = use_v ? G[i][8] - Vp[i] : 0.0;
      wb[i] = (use_v ? G[i][8] : 0.0) - (use_w ? Wst[i] : 0.0);
    }
    current_vjp(X, M, a.eta, wa, wb, acc);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!bside[d]) continue;
    // exterior state Y = B(X) (the no-incoming-Poynting state, linear in X on the
    // branch the forward evaluation took): d/dX = P^T d/dY with P the branch's mask
    double Y[NV], gY[NV], bv[NV];
    boundary_state(d, (double)bside[d], X, M, Y);
    double El[3], Bl[3];
    lower3(M, X, El);
    lower3(M, X + 3, Bl);
    const int j1 = (d + 1) % 3, k1 = (d + 2) % 3;
    const bool inward = (double)bside[d] * (El[j1] * Bl[k1] - El[k1] * Bl[j1]) < 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      bv[v] = bA[d] * Vp[v];
      gY[v] = bI[d] * Vp[v];
    }
    if (d == 0) flux_lin_vjp<0>(M, bv, gY);
    else if (d == 1) flux_lin_vjp<1>(M, bv, gY);
    else flux_lin_vjp<2>(M, bv, gY);
    double cj[3] = {0.0, 0.0, 0.0};
    cj[d] = bv[8];
    current_vjp(Y, M, a.eta, cj, cj, gY);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const bool keep = (v < 3) ? !inward : (v != 6 && v != 7);
      if (keep) acc[v] += gY[v];
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) ub[v] += acc[v];
}

template <int N, bool CURVED, int STAGE>
__global__ __launch_bounds__(Dims<N>::tpb) void k_dg_adjoint(KArgs a, AdjBufs b) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, nn = Dm::nn, TPB = Dm::tpb;
  __shared__ double sV[NV * nn];
  __shared__ double sD[n * n];
  __shared__ double sF[n * n];
  const int e = blockIdx.x;
  if (!a.live[e] || a.rep0[e] != 0) return;
  // rolled back in this stage's substep: its own operator result was discarded
  const bool own_op = (b.rep_upd ? b.rep_upd[e] : 0) == 0;
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int p = act ? t : 0;
  for (int q = t; q < n * n; q += TPB) {
    sD[q] = a.ops->D[q];
    sF[q] = a.ops->F[q];
  }
  Metric M;
  load_metric<CURVED>(a.bg_dg, a.E, nn, e, p, M);
  const double dt = dt_of(a, e);
  const double h = dt * IMEX_A;
  double Un[NV];
  load9(a.dg.Un, a.E, nn, e, p, Un);
  if (STAGE == ADJ_RHS) {
    double lam[NV], ub[NV];
    load9(b.mu, a.E, nn, e, p, lam);
    operator_vjp<N, CURVED>(a, b, e, p, act, Un, M, lam, (b.parts & 1) != 0, (b.parts & 2) != 0, sV, sD, ub);
    if (!act) return;
    double o[NV];
    load9(b.un_bar, a.E, nn, e, p, o);
    for (int v = 0; v < NV; ++v) o[v] += ub[v];
    store9(b.un_bar, a.E, nn, e, p, o);
    return;
  }
  if (STAGE == ADJ_A3) {
    // U^{n+1} = Phi(Y3),  Y3 = U^n + A' + dt S2/6 + (2/3) dt (L(U4) + S(U4))
    double Z[NV];
    load9(b.mu, a.E, nn, e, p, Z);
    if (a.filter_on) filter_transpose<N>(sF, sV, p, act, Z);
    if (!act) return;
    adj_a3_tail(b, a.E, nn, e, p, dt, Z);
    return;
  }
  // stage value the transposed operator is taken at
  double X[NV], U1[NV], S1[NV];
  if (STAGE == ADJ_B3) load9(a.dg.X1, a.E, nn, e, p, X);       // U_4
  else if (STAGE == ADJ_B2) load9(a.dg.X0, a.E, nn, e, p, X);  // U_3
  else pre_stages(Un, M, a, dt, U1, X, S1);                    // U_2
  double W[NV], ub[NV];
  load9(b.w, a.E, nn, e, p, W);
  operator_vjp<N, CURVED>(a, b, e, p, act, X, M, W, true, own_op, sV, sD, ub, own_op);
  if (!own_op && STAGE != ADJ_B1 && act) {
    // the substep input's adjoint from the FD redo, through P^T
    double T[NV];
    load9(b.transfer, a.E, nn, e, p, T);
#pragma unroll
    for (int v = 0; v < NV; ++v) ub[v] += T[v];
  }
  if (b.extra && act) {
    // the transposed ghost slabs read by FD neighbours at this stage
#pragma unroll
    for (int v = 0; v < NV; ++v) ub[v] += b.extra[((size_t)v * a.E + e) * nn + p];
  }
  if (STAGE == ADJ_B3 || STAGE == ADJ_B2) {
    // X = solve(Phi(Y)): Y_bar = Phi^T (I - h S'(X))^-T X_bar
    double Z[NV];
    if (act) solve_vjp(X, M, a, h, ub, Z);
    if (a.filter_on) filter_transpose<N>(sF, sV, p, act, Z);
    if (!act) return;
    adj_b_tail<STAGE>(b, a.E, nn, e, p, dt, Z);
    return;
  }
  if (!act) return;
  adj_b1_tail(a, b, a.E, nn, e, p, M, dt, X, U1, ub);
}

template <int N, bool CURVED>
static void launch_adj_t(const KArgs& a, const AdjBufs& b, int stage, hipStream_t s) {
  dim3 grid(a.E), block(Dims<N>::tpb);
  switch (stage) {
    case ADJ_A3: launch_kernel(k_dg_adjoint<N, CURVED, ADJ_A3>, grid, block, s, a, b); break;
    case ADJ_B3: launch_kernel(k_dg_adjoint<N, CURVED, ADJ_B3>, grid, block, s, a, b); break;
    case ADJ_B2: launch_kernel(k_dg_adjoint<N, CURVED, ADJ_B2>, grid, block, s, a, b); break;
    case ADJ_B1: launch_kernel(k_dg_adjoint<N, CURVED, ADJ_B1>, grid, block, s, a, b); break;
    default: launch_kernel(k_dg_adjoint<N, CURVED, ADJ_RHS>, grid, block, s, a, b); break;
  }
}

template <bool CURVED>
static void launch_adj_c(const KArgs& a, const AdjBufs& b, int N, int stage, hipStream_t s) {
  switch (N) {
    case 3: launch_adj_t<3, CURVED>(a, b, stage, s); break;
    case 4: launch_adj_t<4, CURVED>(a, b, stage, s); break;
    case 5: launch_adj_t<5, CURVED>(a, b, stage, s); break;
    case 6: launch_adj_t<6, CURVED>(a, b, stage, s); break;
    case 7: launch_adj_t<7, CURVED>(a, b, stage, s); break;
    default: launch_adj_t<8, CURVED>(a, b, stage, s); break;  // the adjoint entry points refuse N > 8
  }
}

void launch_dg_adjoint_stage(const KArgs& a, int N, bool curved, int stage, const AdjBufs& b, hipStream_t s) {
  if (curved) launch_adj_c<true>(a, b, N, stage, s);
  else launch_adj_c<false>(a, b, N, stage, s);
}

void launch_rhs_adjoint(const KArgs& a, int N, bool curved, const double* lam, double* ubar, int parts,
                        hipStream_t s) {
  AdjBufs b{};
  b.mu = lam;
  b.un_bar = ubar;
  b.v_in = const_cast<double*>(lam);
  b.parts = parts;
  if (curved) launch_adj_c<true>(a, b, N, ADJ_RHS, s);
  else launch_adj_c<false>(a, b, N, ADJ_RHS, s);
}

// ws: six [9][E][n^3] arrays (accumulator adjoints, stiff vector, two explicit vectors).
void launch_step_adjoint(const KArgs& a, int N, bool curved, const double* mu, double* lam, double* ws,
                         hipStream_t s) {
  const size_t n3 = (size_t)(N + 1) * (N + 1) * (N + 1);
  const size_t reg = (size_t)NV * a.E * n3;
  AdjBufs b{};
  b.mu = mu;
  b.un_bar = lam;
  b.a_bar = ws;
  b.s1_bar = ws + reg;
  b.s2_bar = ws + 2 * reg;
  b.w = ws + 3 * reg;
  double* va = ws + 4 * reg;
  double* vb = ws + 5 * reg;
  const int order[4] = {ADJ_A3, ADJ_B3, ADJ_B2, ADJ_B1};
  for (int k = 0; k < 4; ++k) {
    b.v_in = (k % 2 == 0) ? vb : va;
    b.v_out = (k % 2 == 0) ? va : vb;
    if (curved) launch_adj_c<true>(a, b, N, order[k], s);
    else launch_adj_c<false>(a, b, N, order[k], s);
  }
}

}  // namespace grffe
