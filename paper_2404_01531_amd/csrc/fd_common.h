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

}  // namespace grffe
