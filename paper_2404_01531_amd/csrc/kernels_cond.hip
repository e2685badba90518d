// Rotating perfect conductor (Sec. IV C, pulsar magnetospheres).
//
// After the update of every substep, at each DG node or FD cell centre of the
// substep's result that lies inside the conductor's sphere |x - c| <= R, the
// electric field is replaced by the value the ideal condition E + v x B = 0 gives
// for the conductor's rigid rotation, and psi~ and q~ are set to zero; B~ and phi~
// keep their evolved values.  Flat space with the grid at rest: v = Omega z^ x
// (x - c).  On a 3+1 background (the frame that rotates with the star, whose shift
// is beta = Omega_frame z^ x x): the conductor's coordinate velocity is
// Omega z^ x (x - c) (Omega relative to the grid, 0 when the grid rotates with it),
// its velocity relative to the normal observers v = (Omega z^ x (x - c) + beta) /
// alpha, and E_i = -[ijk] v^j B~^k, E~^i = sqrt(gamma) gamma^{ij} E_j.  The indicator
// of the DG substep has already looked at the candidate by then, but it reads only
// |B~|, which the overwrite leaves alone.  The FD elements of substeps 1 and 2 also
// get their next-substep transported values (U and J~) rewritten at those cells.
#include "common.h"

namespace grffe {

template <int N, bool CURVED>
__global__ __launch_bounds__(256) void k_conductor(KArgs a, CondArgs c, int mode) {
  constexpr int n = N + 1, m = 2 * N + 1;
  constexpr int nn = n * n * n, mm = m * m * m;
  constexpr int BPE = (mm + 255) / 256;
  const int items = c.count * BPE;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int k = item / BPE;
    const int e = c.list[k];
    if (!a.live[e]) continue;
    const bool fd = a.rep[e] == 1;
    const int P = fd ? mm : nn;
    const int w = fd ? m : n;
    const int p = (item % BPE) * 256 + threadIdx.x;
    if (p >= P) continue;
    const int ix[3] = {p % w, (p / w) % w, p / (w * w)};
    double r[3];
    const double cc[3] = {c.cx, c.cy, c.cz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double xi = fd ? -1.0 + (2.0 * ix[d] + 1.0) / m : c.ref[ix[d]];
      r[d] = (c.corner[3 * k + d] + 0.5 * h_of(a, e, d) * (xi + 1.0)) - cc[d];
    }
    if (r[0] * r[0] + r[1] * r[1] + r[2] * r[2] > c.r2) continue;
    const Regs& R = fd ? a.fd : a.dg;
    double* out = mode == MODE_SUB1 ? R.X0 : (mode == MODE_SUB2 ? R.X1 : R.Un);
    double U[NV];
    load9(out, a.E, P, e, p, U);
    Metric M;
    if (CURVED) load_metric<true>(fd ? a.bg_fd : a.bg_dg, a.E, P, e, p, M);
    else metric_flat(M);
    double vx = -c.omega * r[1], vy = c.omega * r[0], vz = 0.0;
    if (CURVED) {
      vx = (vx + M.beta[0]) / M.alpha;
      vy = (vy + M.beta[1]) / M.alpha;
      vz = (vz + M.beta[2]) / M.alpha;
      // E_i = -[ijk] v^j B~^k, raised and densitized
      const double El[3] = {-(vy * U[5] - vz * U[4]), -(vz * U[3] - vx * U[5]), -(vx * U[4] - vy * U[3])};
#pragma unroll
      for (int i = 0; i < 3; ++i)
        U[i] = M.sqrtg * (M.gi[sym(i, 0)] * El[0] + M.gi[sym(i, 1)] * El[1] + M.gi[sym(i, 2)] * El[2]);
    } else {
      U[0] = -(vy * U[5]);
      U[1] = vx * U[5];
      U[2] = -(vx * U[4] - vy * U[3]);
    }
    U[6] = 0.0;
    U[8] = 0.0;
    store9(out, a.E, P, e, p, U);
    if (fd && mode != MODE_SUB3) {
      double J[3];
      current_total(U, M, a.eta, J);
      const size_t st = (size_t)a.E * mm;
      double* wf = a.w_fd + (size_t)e * mm + p;
#pragma unroll
      for (int v = 0; v < NV; ++v) wf[v * st] = U[v];
#pragma unroll
      for (int q = 0; q < 3; ++q) wf[(NV + q) * st] = J[q];
    }
  }
}

void launch_conductor(const KArgs& a, int N, bool curved, const CondArgs& c, int mode, hipStream_t s) {
  if (c.count <= 0) return;
  GRFFE_SWITCH_N({
    constexpr int m = 2 * NN + 1;
    const int items = c.count * ((m * m * m + 255) / 256);
    if (curved) launch_kernel(k_conductor<NN, true>, dim3(items), dim3(256), s, a, c, mode);
    else launch_kernel(k_conductor<NN, false>, dim3(items), dim3(256), s, a, c, mode);
  })
}

}  // namespace grffe
