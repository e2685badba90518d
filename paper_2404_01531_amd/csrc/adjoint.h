// Pointwise transposes shared by the DG and FD adjoint kernels: the state-linear
// parts of the flux and the sources transposed by hand, the current's gradient by
// forward-mode dual numbers, and the adjoint of the pointwise implicit solve.
#pragma once
#include "common.h"
#include "dual.h"

namespace grffe {

// Levi-Civita symbol [i d k] for i, d, k in {0, 1, 2}.
__device__ constexpr int levi(int i, int d, int k) { return (i - d) * (d - k) * (k - i) / 2; }

// out += d(G . F^d_lin)/dX, the transpose of the part of the flux F^d that is linear
// in the state at a fixed metric (every component but the current J~^d of the q~
// flux):  F_E = -beta^d E + alpha (gamma^{id} psi - [i d k] B_k / sqrt(gamma)),
// F_B = -beta^d B + alpha (gamma^{id} phi + [i d k] E_k / sqrt(gamma)),
// F_psi = -beta^d psi + alpha E^d, F_phi = -beta^d phi + alpha B^d, F_q = -beta^d q.
template <int D>
__device__ inline void flux_lin_vjp(const Metric& M, const double* G, double* out) {
  double c[3] = {0.0, 0.0, 0.0}, cp[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int lv = levi(i, D, k);
      if (lv) {
        c[k] += lv * G[3 + i];
        cp[k] += lv * G[i];
      }
    }
  double gc[3], gcp[3];
  lower3(M, c, gc);
  lower3(M, cp, gcp);
  const double al = M.alpha, bd = M.beta[D], isg = M.isqrtg;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    out[j] += -bd * G[j] + al * isg * gc[j] + (j == D ? al * G[6] : 0.0);
    out[3 + j] += -bd * G[3 + j] - al * isg * gcp[j] + (j == D ? al * G[7] : 0.0);
  }
  double s6 = 0.0, s7 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s6 += G[i] * M.gi[sym(i, D)];
    s7 += G[3 + i] * M.gi[sym(i, D)];
  }
  out[6] += al * s6 - bd * G[6];
  out[7] += al * s7 - bd * G[7];
  out[8] += -bd * G[8];
}

// out += gradient of  wa . J_drift(X) + wb . J_driver(X)  (the densitized current's two
// parts), by forward-mode dual numbers; psi~ and phi~ do not enter the current.
__device__ inline void current_vjp(const double* X, const Metric& M, double eta, const double* wa, const double* wb,
                                   double* out) {
  MetricT<Dual> Md;
  metric_cast(M, Md);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k == 6 || k == 7) continue;
    Dual Xd[NV], Jd[3], Je[3];
#pragma unroll
    for (int v = 0; v < NV; ++v) Xd[v] = Dual(X[v], v == k ? 1.0 : 0.0);
    current(Xd, Md, eta, Jd, Je);
    Dual tot(0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i) tot += wa[i] * Jd[i] + wb[i] * Je[i];
    out[k] += tot.d;
  }
}

// out += (dS_ex/dX)^T V for the parts of the explicit source that are linear in X
// (the drift current's part is taken by current_vjp).
template <bool CURVED>
__device__ inline void source_lin_vjp(const Metric& M, const MetricDeriv& Dv, const double* V, double* out) {
  if (!CURVED) {
    out[8] += V[6];  // S_psi = q
    return;
  }
  const double al = M.alpha;
  double ga[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    ga[i] = M.gi[sym(i, 0)] * Dv.da[0] + M.gi[sym(i, 1)] * Dv.da[1] + M.gi[sym(i, 2)] * Dv.da[2];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    double se = 0.0, sb = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      se += V[i] * Dv.db[3 * j + i];
      sb += V[3 + i] * Dv.db[3 * j + i];
    }
    out[j] += -se + V[6] * Dv.da[j];
    out[3 + j] += -sb + V[7] * Dv.da[j];
  }
  double pe = 0.0, pb = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    pe += V[i] * (ga[i] - al * Dv.Gam[i]);
    pb += V[3 + i] * (ga[i] - al * Dv.Gam[i]);
  }
  out[6] += pe - al * Dv.K * V[6];
  out[7] += pb - al * Dv.K * V[7];
  out[8] += al * V[6];
}

// out += (dS_stiff/dU)^T w at U:  S_E = -J_driver, S_psi = -alpha kappa_psi psi,
// S_phi = -alpha kappa_phi phi.
__device__ inline void stiff_vjp(const double* U, const Metric& M, const KArgs& a, const double* w, double* out) {
  const double wa[3] = {0.0, 0.0, 0.0}, wb[3] = {-w[0], -w[1], -w[2]};
  current_vjp(U, M, a.eta, wa, wb, out);
  out[6] += -M.alpha * a.kpsi * w[6];
  out[7] += -M.alpha * a.kphi * w[7];
}

// y = (I - h dS_stiff/dU)^-T ub at the solution U of the implicit solve with step h.
// Only the driver current couples components: with JE = dJe/dE, JB = dJe/dB,
//   (I + h JE^T) y_E = ub_E,  y_B = ub_B - h JB^T y_E,
//   y_psi = ub_psi / (1 + h alpha kappa_psi),  y_phi likewise,  y_q = ub_q.
__device__ inline void solve_vjp(const double* U, const Metric& M, const KArgs& a, double h, const double* ub,
                                 double* y) {
  double JE[3][3], JB[3][3];  // [i][k] = dJe_i / dE_k (dB_k)
  MetricT<Dual> Md;
  metric_cast(M, Md);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    Dual Xd[NV], Jd[3], Je[3];
#pragma unroll
    for (int v = 0; v < NV; ++v) Xd[v] = Dual(U[v], v == k ? 1.0 : 0.0);
    current(Xd, Md, a.eta, Jd, Je);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (k < 3) JE[i][k] = Je[i].d;
      else JB[i][k - 3] = Je[i].d;
    }
  }
  // A = I + h JE^T, A[r][c] = delta + h JE[c][r]; solve A y_E = ub_E (Cramer's rule)
  double A[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) A[r][c] = (r == c ? 1.0 : 0.0) + h * JE[c][r];
  const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
  const double idet = 1.0 / det;
  const double b0 = ub[0], b1 = ub[1], b2 = ub[2];
  // inverse via the adjugate
  y[0] = idet * (c00 * b0 + (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * b1 + (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * b2);
  y[1] = idet * (c01 * b0 + (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * b1 + (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * b2);
  y[2] = idet * (c02 * b0 + (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * b1 + (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * b2);
#pragma unroll
  for (int k = 0; k < 3; ++k) y[3 + k] = ub[3 + k] - h * (JB[0][k] * y[0] + JB[1][k] * y[1] + JB[2][k] * y[2]);
  y[6] = ub[6] / (1.0 + h * M.alpha * a.kpsi);
  y[7] = ub[7] / (1.0 + h * M.alpha * a.kphi);
  y[8] = ub[8];
}

// U_1, U_2 of the implicit pre-stages from U^n (as in the forward step).
__device__ inline void pre_stages(const double* Un, const Metric& M, const KArgs& a, double dt, double* U1,
                                  double* U2, double* S1) {
  const double h = dt * IMEX_A;
#pragma unroll
  for (int v = 0; v < NV; ++v) U1[v] = Un[v];
  implicit_solve(U1, M, a.eta, a.kpsi, a.kphi, h);
  source_stiff(U1, M, a.eta, a.kpsi, a.kphi, S1);
#pragma unroll
  for (int v = 0; v < NV; ++v) U2[v] = Un[v] - dt * IMEX_A * S1[v];
  implicit_solve(U2, M, a.eta, a.kpsi, a.kphi, h);
}

// The step's stage algebra transposed, point by point (the same on DG nodes and FD
// cells; on DG, Z has been taken through the transposed filter first).
// Last substep: U^{n+1} = Phi(Y3), Y3 = U^n + A' + dt S2/6 + (2/3) dt (L(U_4) + S(U_4)),
// Z the adjoint of Y3.
__device__ inline void adj_a3_tail(const AdjBufs& b, int E, int P, int e, int p, double dt, const double* Z) {
  double V[NV], S2b[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    V[v] = (2.0 / 3.0) * dt * Z[v];
    S2b[v] = dt / 6.0 * Z[v];
  }
  store9(b.un_bar, E, P, e, p, Z);
  store9(b.a_bar, E, P, e, p, Z);
  store9(b.s2_bar, E, P, e, p, S2b);
  store9(b.v_out, E, P, e, p, V);
  store9(b.w, E, P, e, p, V);
}

// Substeps 2 (B3: Y2 -> U_4) and 1 (B2: Y1 -> U_3), Z the adjoint of the substep's
// input combination Y.
template <int STAGE>
__device__ inline void adj_b_tail(const AdjBufs& b, int E, int P, int e, int p, double dt, const double* Z) {
  double unb[NV], Ab[NV];
  load9(b.un_bar, E, P, e, p, unb);
  load9(b.a_bar, E, P, e, p, Ab);
#pragma unroll
  for (int v = 0; v < NV; ++v) unb[v] += Z[v];
  store9(b.un_bar, E, P, e, p, unb);
  double V[NV], Wn[NV];
  if (STAGE == ADJ_B3) {
    // Y2 = U^n + (A + dt L(U3))/4 + dt (b S1 + e S2 + c3 S(U3)),  A' = (A + dt L(U3))/6 + dt S(U3)/6
    const double c3 = 0.5 - IMEX_B - IMEX_E - IMEX_A;
    double S1b[NV], S2b[NV];
    load9(b.s2_bar, E, P, e, p, S2b);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double inc = 0.25 * Z[v] + Ab[v] / 6.0;
      Wn[v] = c3 * dt * Z[v] + dt / 6.0 * Ab[v];
      V[v] = dt * inc;
      Ab[v] = inc;
      S1b[v] = IMEX_B * dt * Z[v];
      S2b[v] += IMEX_E * dt * Z[v];
    }
    store9(b.a_bar, E, P, e, p, Ab);
    store9(b.s1_bar, E, P, e, p, S1b);
    store9(b.s2_bar, E, P, e, p, S2b);
  } else {
    // Y1 = U^n + dt L(U2) + dt (1 - a) S(U2),  A = dt L(U2);  S2 = S(U2)
    double S2b[NV];
    load9(b.s2_bar, E, P, e, p, S2b);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      V[v] = dt * (Z[v] + Ab[v]);
      Wn[v] = (1.0 - IMEX_A) * dt * Z[v] + S2b[v];
    }
  }
  store9(b.v_out, E, P, e, p, V);
  store9(b.w, E, P, e, p, Wn);
}

// The implicit pre-stages: U_2 = solve(U^n - a dt S1), S1 = S(U_1), U_1 = solve(U^n);
// ub is the adjoint of U_2 (operator and stiff parts of the first substep).
__device__ inline void adj_b1_tail(const KArgs& a, const AdjBufs& b, int E, int P, int e, int p, const Metric& M,
                                   double dt, const double* U2, const double* U1, const double* ub) {
  const double h = dt * IMEX_A;
  double Y[NV], S1b[NV], U1b[NV], Yn[NV], unb[NV];
  solve_vjp(U2, M, a, h, ub, Y);
  load9(b.s1_bar, E, P, e, p, S1b);
  load9(b.un_bar, E, P, e, p, unb);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    unb[v] += Y[v];
    S1b[v] -= IMEX_A * dt * Y[v];
    U1b[v] = 0.0;
  }
  stiff_vjp(U1, M, a, S1b, U1b);
  solve_vjp(U1, M, a, h, U1b, Yn);
#pragma unroll
  for (int v = 0; v < NV; ++v) unb[v] += Yn[v];
  store9(b.un_bar, E, P, e, p, unb);
}

}  // namespace grffe
