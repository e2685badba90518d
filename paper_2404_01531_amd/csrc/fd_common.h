// FD subcell helpers shared by the FD kernels and their adjoint.
#pragma once
#include "common.h"

namespace grffe {

// Where the (U, J~) of cell c (-3 <= c <= m+2 along d) of element e lives.
struct CellSrc {
  const double* ptr;  // component 0; null for the computed boundary state
  size_t stride;      // between components
  int elem, cell;     // element / cell index used for the cell metric
  int bnd;            // the face's neighbour entry (< 0) when ptr is null
};

// The neighbours of element e across its two faces normal to d (lower, upper) and
// their representations: read once per work item, whose element and direction are
// the same for every thread, so that the ghost cells' sources need no dependent
// per-thread loads.
struct RowNbrs {
  int o0, o1;  // neighbour entries (< 0: a physical face)
  int r0, r1;  // their representations (-1 for a physical face)
};

__device__ inline RowNbrs row_neighbours(const KArgs& a, int e, int d) {
  RowNbrs nb;
  nb.o0 = a.nbr[e * 6 + 2 * d];
  nb.o1 = a.nbr[e * 6 + 2 * d + 1];
  nb.r0 = nb.o0 >= 0 ? a.rep0[nb.o0] : -1;
  nb.r1 = nb.o1 >= 0 ? a.rep0[nb.o1] : -1;
  return nb;
}

template <int N>
__device__ inline CellSrc cell_source(const KArgs& a, const RowNbrs& nb, int e, int d, int c, int t1, int t2) {
  using Dm = Dims<N>;
  constexpr int m = Dm::m, mm = Dm::mm;
  const int str[3] = {1, m, m * m};
  const int t1ax = (d == 0) ? 1 : 0, t2ax = (d == 2) ? 1 : 2;
  CellSrc cs;
  if (c >= 0 && c < m) {
    cs.cell = c * str[d] + t1 * str[t1ax] + t2 * str[t2ax];
    cs.elem = e;
    cs.ptr = a.w_fd + (size_t)e * mm + cs.cell;
    cs.stride = (size_t)a.E * mm;
    return cs;
  }
  const int s = (c >= m) ? 1 : 0;
  const int o = s ? nb.o1 : nb.o0;
  if (o < 0) {
    const int cb = s ? m - 1 : 0;
    cs.cell = cb * str[d] + t1 * str[t1ax] + t2 * str[t2ax];
    cs.elem = e;
    cs.ptr = nullptr;
    cs.stride = 0;
    cs.bnd = o;
    return cs;
  }
  const int cn = s ? c - m : c + m;  // cell index inside the neighbour
  cs.cell = cn * str[d] + t1 * str[t1ax] + t2 * str[t2ax];
  cs.elem = o;
  if ((s ? nb.r1 : nb.r0) == 1) {
    cs.ptr = a.w_fd + (size_t)o * mm + cs.cell;
    cs.stride = (size_t)a.E * mm;
  } else {
    // DG neighbour: its slab on the face facing us, layer = distance from the face
    const int fo = 2 * d + (1 - s);
    const int l = s ? (c - m) : (-1 - c);
    cs.ptr = a.slab + ((size_t)o * 6 + fo) * (3 * m * m) + l * m * m + t1 + m * t2;
    cs.stride = (size_t)a.E * 6 * 3 * m * m;
  }
  return cs;
}

// ---------------------------------------------------------------- WENO5-Z on point values
// Candidates are the quadratic Lagrange interpolants of the point values at the
// face; optimal weights (1, 10, 5)/16; Z weights alpha_k = d_k (1 + (tau5 /
// (beta_k + eps))^2) with tau5 = |beta_0 - beta_2| (exponent q = 2).  With
// b_k = beta_k + eps the normalised combination sum alpha_k q_k / sum alpha_k is
// evaluated after multiplying numerator and denominator by b_0^2 b_1^2 b_2^2,
// which leaves a single quotient.

// n / d for the WENO normalisation, whose denominator is positive and in the normal
// range (at least eps^6): the hardware reciprocal estimate refined by two
// Newton-Raphson steps r <- r (2 - d r), then one multiplication (within about one
// unit in the last place of the correctly rounded quotient).
__device__ inline double div_weno(double n, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return n * r;
}

// Both WENO5-Z reconstructions whose target cell is c, from the five point
// values v[0..4] = cells c-2 .. c+2: `left` is the state on the left of face
// c+1/2, `right` the state on the right of face c-1/2.  The two share the
// smoothness indicators of the target cell (the mirrored reconstruction sees
// beta_0 and beta_2 swapped) and tau5 = |beta_0 - beta_2|.  Z weights with
// exponent 2, optimal weights (1, 10, 5)/16, candidates are quadratic Lagrange
// interpolants of point values; the normalisation is done with one quotient
// (div_weno) per state after multiplying by b_0^2 b_1^2 b_2^2, b_k = beta_k + eps.
__device__ inline void weno5z_cell(const double* v, double eps, double& left, double& right) {
  // b_k here is 4 (beta_k + eps), and the candidates below carry their 1/8: both
  // are power-of-two scalings, exact in floating point (the first cancels in the
  // normalised combination), which save the separate scaling multiplications of
  // the indicators and of the two states
  const double d0 = v[0] - 2.0 * v[1] + v[2], e0 = v[0] - 4.0 * v[1] + 3.0 * v[2];
  const double d1 = v[1] - 2.0 * v[2] + v[3], e1 = v[1] - v[3];
  const double d2 = v[2] - 2.0 * v[3] + v[4], e2 = 3.0 * v[2] - 4.0 * v[3] + v[4];
  const double eps4 = 4.0 * eps;
  const double b0 = (13.0 / 3.0) * d0 * d0 + e0 * e0 + eps4;
  const double b1 = (13.0 / 3.0) * d1 * d1 + e1 * e1 + eps4;
  const double b2 = (13.0 / 3.0) * d2 * d2 + e2 * e2 + eps4;
  const double tau = fabs(b0 - b2);
  const double t2 = tau * tau;
  const double s0 = b0 * b0, s1 = b1 * b1, s2 = b2 * b2;
  const double p01 = s0 * s1, p02 = s0 * s2, p12 = s1 * s2;
  const double a0 = (s0 + t2), a1 = (s1 + t2), a2 = (s2 + t2);
  // the common factor 1/16 of the weights cancels in the normalisation and is left out
  const double a1p = 10.0 * a1 * p02;
  {
    const double w0 = a0 * p12;
    const double w2 = 5.0 * a2 * p01;
    const double q0 = 0.375 * v[0] - 1.25 * v[1] + 1.875 * v[2];
    const double q1 = -0.125 * v[1] + 0.75 * v[2] + 0.375 * v[3];
    const double q2 = 0.375 * v[2] + 0.75 * v[3] - 0.125 * v[4];
    left = div_weno(w0 * q0 + a1p * q1 + w2 * q2, w0 + a1p + w2);
  }
  {
    const double w0 = a2 * p01;
    const double w2 = 5.0 * a0 * p12;
    const double q0 = 0.375 * v[4] - 1.25 * v[3] + 1.875 * v[2];
    const double q1 = -0.125 * v[3] + 0.75 * v[2] + 0.375 * v[1];
    const double q2 = 0.375 * v[2] + 0.75 * v[1] - 0.125 * v[0];
    right = div_weno(w0 * q0 + a1p * q1 + w2 * q2, w0 + a1p + w2);
  }
}

// Threads of an FD flux workgroup: at least one per (cell -1 .. m, pencil) of a row,
// the flux phase's work items.
template <int N>
constexpr int flux_tpb() {
  return (2 * N + 1) * (2 * N + 3) <= 256 ? 256 : 512;
}

}  // namespace grffe
