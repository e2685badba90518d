// Device helpers shared by the kernel translation units.
#pragma once
#include <hip/hip_ext.h>

#include "grffe_internal.h"
#include "physics.h"

namespace grffe {

// Launch a kernel; if timing events are armed, they are attached to the kernel's own
// dispatch (hipExtLaunchKernelGGL), so they bracket exactly that kernel.
template <typename... P, typename... A>
inline void launch_kernel(void (*kernel)(P...), dim3 grid, dim3 block, hipStream_t s, A... args) {
  LaunchEvents& le = armed_launch_events();
  if (le.start) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, le.start, le.stop, 0, args...);
    le.start = nullptr;
    le.stop = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
  }
}

template <int N>
struct Dims {
  static constexpr int n = N + 1;
  static constexpr int m = 2 * N + 1;
  static constexpr int nn = n * n * n;
  static constexpr int mm = m * m * m;
  static constexpr int tpb = ((nn + 63) / 64) * 64;  // threads of a per-element DG block
};

// Block-wide sum of two doubles (all threads of the block must call it).
template <int TPB>
__device__ inline void block_sum2(double& a, double& b, double* sred) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  constexpr int NWAVE = TPB / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sred[2 * wave] = a;
    sred[2 * wave + 1] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int w = 0; w < NWAVE; ++w) {
    a += sred[2 * w];
    b += sred[2 * w + 1];
  }
  __syncthreads();
}

// Metric (10 leading fields) of point `p` of element `e` from a [F][E][P] array (FP64, or
// its FP32 copy; the metric is formed in FP64 either way).
template <bool CURVED, typename TB>
__device__ inline void load_metric(const TB* bg, int E, int P, int e, int p, Metric& M) {
  if (!CURVED) {
    metric_flat(M);
    return;
  }
  double f[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) f[k] = (double)bg[((size_t)k * E + e) * P + p];
  metric_from10(f, M);
}

template <bool CURVED, typename TB>
__device__ inline void load_deriv(const TB* bg, int E, int P, int e, int p, MetricDeriv& Dv) {
  if (!CURVED) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) Dv.da[k] = (double)bg[((size_t)(10 + k) * E + e) * P + p];
#pragma unroll
  for (int k = 0; k < 9; ++k) Dv.db[k] = (double)bg[((size_t)(13 + k) * E + e) * P + p];
  Dv.K = (double)bg[((size_t)22 * E + e) * P + p];
#pragma unroll
  for (int k = 0; k < 3; ++k) Dv.Gam[k] = (double)bg[((size_t)(23 + k) * E + e) * P + p];
}

// The background at DG node p of element e for the kernels that work on DG nodes:
// from the FP32 copy when the domain keeps one (mixed precision on a curved
// background: every DG-node kernel then sees the same rounded metric, so that the
// stiff current, which multiplies the metric's rounding of E.B by eta, is consistent
// between them), else from the FP64 array.
template <bool CURVED>
__device__ inline void load_metric_dg(const KArgs& a, int nn, int e, int p, Metric& M) {
  if (CURVED && a.bg_dg32) load_metric<CURVED>(a.bg_dg32, a.E, nn, e, p, M);
  else load_metric<CURVED>(a.bg_dg, a.E, nn, e, p, M);
}

template <bool CURVED>
__device__ inline void load_deriv_dg(const KArgs& a, int nn, int e, int p, MetricDeriv& Dv) {
  if (CURVED && a.bg_dg32) load_deriv<CURVED>(a.bg_dg32, a.E, nn, e, p, Dv);
  else load_deriv<CURVED>(a.bg_dg, a.E, nn, e, p, Dv);
}

// The same for a kernel compiled for one arithmetic R of the flux evaluation: the
// FP64 instantiations (which run only in the FP64 mode, where no FP32 copy exists)
// read the FP64 array without the run-time choice.
template <bool CURVED, typename R>
__device__ inline void load_metric_dg_r(const KArgs& a, int nn, int e, int p, Metric& M) {
  if (sizeof(R) == sizeof(double)) load_metric<CURVED>(a.bg_dg, a.E, nn, e, p, M);
  else load_metric_dg<CURVED>(a, nn, e, p, M);
}

template <bool CURVED, typename R>
__device__ inline void load_deriv_dg_r(const KArgs& a, int nn, int e, int p, MetricDeriv& Dv) {
  if (sizeof(R) == sizeof(double)) load_deriv<CURVED>(a.bg_dg, a.E, nn, e, p, Dv);
  else load_deriv_dg<CURVED>(a, nn, e, p, Dv);
}

__device__ inline void load9(const double* base, int E, int P, int e, int p, double* U) {
#pragma unroll
  for (int v = 0; v < NV; ++v) U[v] = base[((size_t)v * E + e) * P + p];
}

__device__ inline void store9(double* base, int E, int P, int e, int p, const double* U) {
#pragma unroll
  for (int v = 0; v < NV; ++v) base[((size_t)v * E + e) * P + p] = U[v];
}

// Exterior state of a boundary face (neighbour entry o < 0 of the face of direction d
// and side s): a Dirichlet face (o = -2 - slot) holds a stored state, the point's
// own entry of a per-point field (component 0 at field[fidx], components fstride
// apart) when one is set, else the face's uniform row bstate[slot]; any other
// boundary face (o = -1: an outer face of the no-incoming-Poynting kind, or a face
// towards an excised element) takes the no-incoming-Poynting state of the interior
// value Ui.
__device__ inline void exterior_state(const KArgs& a, int o, int d, int s, const double* Ui, const Metric& M,
                                      const double* field, size_t fidx, size_t fstride, double* Ub) {
  // branch-free, so that Ub stays in registers: both states are formed and the
  // Dirichlet one selected (slot 0, always allocated, is read and unused elsewhere)
  boundary_state(d, s ? 1.0 : -1.0, Ui, M, Ub);
  const bool dir = o < -1;
  const bool per_point = dir && field != nullptr;
  const double* st = per_point ? field + fidx : a.bstate + (size_t)(dir ? -2 - o : 0) * NV;
  const size_t str = per_point ? fstride : 1;
#pragma unroll
  for (int c = 0; c < NV; ++c) Ub[c] = dir ? st[c * str] : Ub[c];
}

__device__ inline double dt_of(const KArgs& a, int e) { return a.dt > 0.0 ? a.dt : a.edt[e]; }
__device__ inline double h_of(const KArgs& a, int e, int d) { return a.eh[3 * e + d]; }

// U_1, U_2 and their stiff sources from U^n (the implicit pre-stages of IMEX-SSP3(4,3,3)).
__device__ inline void derived_stages(const double* Un, const Metric& M, const KArgs& a, double dt, double* U2,
                                      double* S1, double* S2) {
  double U1[NV];
  const double h = dt * IMEX_A;
#pragma unroll
  for (int v = 0; v < NV; ++v) U1[v] = Un[v];
  implicit_solve(U1, M, a.eta, a.kpsi, a.kphi, h);
  source_stiff(U1, M, a.eta, a.kpsi, a.kphi, S1);
#pragma unroll
  for (int v = 0; v < NV; ++v) U2[v] = Un[v] - dt * IMEX_A * S1[v];
  implicit_solve(U2, M, a.eta, a.kpsi, a.kphi, h);
  source_stiff(U2, M, a.eta, a.kpsi, a.kphi, S2);
}

// Stage value that is the input of substep MODE, at point p of element e of a register set.
// PRE: the register set holds the pre-stage pass's U_2 (in X1) and stiff terms (in K).
template <int MODE, bool PRE = false>
__device__ inline void stage_input(const Regs& r, int E, int P, int e, int p, const Metric& M, const KArgs& a,
                                   double* X) {
  if (MODE == MODE_RHS) {
    load9(r.Un, E, P, e, p, X);
  } else if (MODE == MODE_SUB1) {
    if (PRE) {
      load9(r.X1, E, P, e, p, X);
    } else {
      double Un[NV], S1[NV], S2[NV];
      load9(r.Un, E, P, e, p, Un);
      derived_stages(Un, M, a, dt_of(a, e), X, S1, S2);
    }
  } else if (MODE == MODE_SUB2) {
    load9(r.X0, E, P, e, p, X);
  } else {
    load9(r.X1, E, P, e, p, X);
  }
}

// Store the stiff-source terms of substeps 2 and 3 (the five non-zero components of
// dt (b S_1 + e S_2) and of dt S_2 / 6) computed from the pre-stages.
__device__ inline void store_stiff_terms(const Regs& r, int E, int P, int e, int p, double dt, const double* S1,
                                         const double* S2) {
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int v = stiff_comp(k);
    r.K[((size_t)k * E + e) * P + p] = dt * (IMEX_B * S1[v] + IMEX_E * S2[v]);
    r.K[((size_t)(NK + k) * E + e) * P + p] = dt * S2[v] / 6.0;
  }
}

// Stiff-source term of substep 2 (half = 0: dt (b S_1 + e S_2)) or substep 3
// (half = 1: dt S_2 / 6) as a nine-component vector, from the pre-stage pass.
__device__ inline void load_stiff_terms(const Regs& r, int E, int P, int e, int p, int half, double* T) {
#pragma unroll
  for (int v = 0; v < NV; ++v) T[v] = 0.0;
#pragma unroll
  for (int k = 0; k < NK; ++k) T[stiff_comp(k)] = r.K[((size_t)(half * NK + k) * E + e) * P + p];
}

// Explicit update Y of substep MODE (before the filter and the implicit solve) and the new
// accumulator.  L is the explicit operator at the stage input X.
template <int MODE, bool PRE = false>
__device__ inline void stage_update(const Regs& r, int E, int P, int e, int p, const Metric& M, const KArgs& a,
                                    const double* X, const double* L, double* Y, double* Anew) {
  double Un[NV];
  load9(r.Un, E, P, e, p, Un);
  const double dt = dt_of(a, e);
  if (MODE == MODE_SUB1) {
    // the substep input X is U_2 itself
    double S2[NV];
    source_stiff(X, M, a.eta, a.kpsi, a.kphi, S2);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Y[v] = Un[v] + dt * L[v] + dt * (1.0 - IMEX_A) * S2[v];
      Anew[v] = dt * L[v];
    }
  } else if (MODE == MODE_SUB2) {
    double A[NV], S3[NV], T[NV];
    load9(r.A, E, P, e, p, A);
    if (PRE) {
      load_stiff_terms(r, E, P, e, p, 0, T);
    } else {
      double S1[NV], S2[NV], U2[NV];
      derived_stages(Un, M, a, dt, U2, S1, S2);
#pragma unroll
      for (int v = 0; v < NV; ++v) T[v] = dt * (IMEX_B * S1[v] + IMEX_E * S2[v]);
    }
    source_stiff(X, M, a.eta, a.kpsi, a.kphi, S3);
    const double c3 = 0.5 - IMEX_B - IMEX_E - IMEX_A;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double inc = A[v] + dt * L[v];
      Y[v] = Un[v] + 0.25 * inc + T[v] + dt * c3 * S3[v];
      Anew[v] = inc / 6.0 + dt * S3[v] / 6.0;
    }
  } else {
    double A[NV], S4[NV], T[NV];
    load9(r.A, E, P, e, p, A);
    if (PRE) {
      load_stiff_terms(r, E, P, e, p, 1, T);
    } else {
      double S1[NV], S2[NV], U2[NV];
      derived_stages(Un, M, a, dt, U2, S1, S2);
#pragma unroll
      for (int v = 0; v < NV; ++v) T[v] = dt * S2[v] / 6.0;
    }
    source_stiff(X, M, a.eta, a.kpsi, a.kphi, S4);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Y[v] = Un[v] + A[v] + T[v] + (2.0 / 3.0) * dt * (L[v] + S4[v]);
      Anew[v] = 0.0;
    }
  }
}

// Dispatch of a launch over the supported degrees: CALL sees the degree as the
// compile-time constant NN.
#define GRFFE_SWITCH_N(CALL)      \
  switch (N) {                    \
    case 3: { constexpr int NN = 3; CALL; } break; \
    case 4: { constexpr int NN = 4; CALL; } break; \
    case 5: { constexpr int NN = 5; CALL; } break; \
    case 6: { constexpr int NN = 6; CALL; } break; \
    case 7: { constexpr int NN = 7; CALL; } break; \
    case 8: { constexpr int NN = 8; CALL; } break; \
    default: { constexpr int NN = 9; CALL; } break; \
  }


}  // namespace grffe
