// Adjoint of the FD subcell right-hand side (Sec. III C 2) and of the DG-FD
// coupling (ghost data and traces between the two grids, Sec. III C 1 and 2) for
// any mix of DG and FD elements.
//
// Along each pencil of direction d the right-hand side of cell c is
//   L_c = -(m/h) (Fhat_{c+1/2} - Fhat_{c-1/2}) + S(U_c),
//   Fhat = (4/3) F* - (F_{c-1} + F_c) / 6    (fourth-order corrector; Fhat = F* for FD2),
//   F* = (F(W_L) + F(W_R)) / 2 - lambda (U_R - U_L) / 2,
// with W_L, W_R the WENO5-Z reconstructions of the ten transported components
// (U and J~^d) and F_c the flux of the cell values.  Every flux is linear in the
// transported components, so the transposes are the hand-written linear ones;
// the reconstruction is differentiated in reverse mode (weno5z_cell_vjp).  The
// adjoint of the transported J~^d is carried back to U through the current's
// gradient at the cell.  Each element computes its own faces, so the face fluxes
// of cells next to a face carry adjoints into the neighbour's cells (ghost
// cells): they are written per face and layer and gathered by the element that
// owns the cells, so no atomics are needed and the result is deterministic.
//
// Coupling.  An FD element's ghost cells next to a DG neighbour are the
// P-projection of the neighbour's (U, J~) (the ghost slab), so their adjoints go
// back through P^T to the DG nodes and through the current's gradient to U there.
// A DG element's exterior state next to an FD neighbour is the R-trace of the FD
// element's (U, J~), and the DG face flux is linear in it (the Rusanov speed is
// the DG node's), so the adjoint of the trace is formed at the DG face nodes and
// taken back through R^T to the FD cells.
#include "adjoint.h"
#include "fd_common.h"

namespace grffe {

// Reverse-mode derivative of weno5z_cell (same formulas, same order): given the
// adjoints gL of `left` and gR of `right`, vb[z] = gL dleft/dv_z + gR dright/dv_z.
// tau5^2 = (beta_0 - beta_2)^2 is smooth, so no branch is differentiated.
__device__ inline void weno5z_cell_vjp(const double* v, double eps, double gL, double gR, double* vb) {
  const double c13 = 13.0 / 12.0;
  const double d0 = v[0] - 2.0 * v[1] + v[2], e0 = v[0] - 4.0 * v[1] + 3.0 * v[2];
  const double d1 = v[1] - 2.0 * v[2] + v[3], e1 = v[1] - v[3];
  const double d2 = v[2] - 2.0 * v[3] + v[4], e2 = 3.0 * v[2] - 4.0 * v[3] + v[4];
  const double b0 = c13 * d0 * d0 + 0.25 * e0 * e0 + eps;
  const double b1 = c13 * d1 * d1 + 0.25 * e1 * e1 + eps;
  const double b2 = c13 * d2 * d2 + 0.25 * e2 * e2 + eps;
  const double td = b0 - b2;
  const double t2 = td * td;
  const double s0 = b0 * b0, s1 = b1 * b1, s2 = b2 * b2;
  const double p01 = s0 * s1, p02 = s0 * s2, p12 = s1 * s2;
  const double a0 = s0 + t2, a1 = s1 + t2, a2 = s2 + t2;
  const double wl0 = (1.0 / 16.0) * a0 * p12, wl1 = (10.0 / 16.0) * a1 * p02, wl2 = (5.0 / 16.0) * a2 * p01;
  const double ql0 = (3.0 * v[0] - 10.0 * v[1] + 15.0 * v[2]) * 0.125;
  const double ql1 = (-v[1] + 6.0 * v[2] + 3.0 * v[3]) * 0.125;
  const double ql2 = (3.0 * v[2] + 6.0 * v[3] - v[4]) * 0.125;
  const double DL = wl0 + wl1 + wl2;
  const double left = (wl0 * ql0 + wl1 * ql1 + wl2 * ql2) / DL;
  const double wr0 = (1.0 / 16.0) * a2 * p01, wr1 = (10.0 / 16.0) * a1 * p02, wr2 = (5.0 / 16.0) * a0 * p12;
  const double qr0 = (3.0 * v[4] - 10.0 * v[3] + 15.0 * v[2]) * 0.125;
  const double qr1 = (-v[3] + 6.0 * v[2] + 3.0 * v[1]) * 0.125;
  const double qr2 = (3.0 * v[2] + 6.0 * v[1] - v[0]) * 0.125;
  const double DR = wr0 + wr1 + wr2;
  const double right = (wr0 * qr0 + wr1 * qr1 + wr2 * qr2) / DR;
  // normalised sums: d(N/D)/dw_k = (q_k - N/D)/D, d(N/D)/dq_k = w_k/D
  const double iL = gL / DL, iR = gR / DR;
  const double bql0 = iL * wl0, bql1 = iL * wl1, bql2 = iL * wl2;
  const double bqr0 = iR * wr0, bqr1 = iR * wr1, bqr2 = iR * wr2;
  // weights: a0 p12 enters wl0 (1/16) and wr2 (5/16); a1 p02 enters wl1, wr1 (10/16);
  // a2 p01 enters wl2 (5/16) and wr0 (1/16)
  const double k0 = (1.0 / 16.0) * iL * (ql0 - left) + (5.0 / 16.0) * iR * (qr2 - right);
  const double k1 = (10.0 / 16.0) * (iL * (ql1 - left) + iR * (qr1 - right));
  const double k2 = (5.0 / 16.0) * iL * (ql2 - left) + (1.0 / 16.0) * iR * (qr0 - right);
  const double bp12 = k0 * a0, bp02 = k1 * a1, bp01 = k2 * a2;
  const double ba0 = k0 * p12, ba1 = k1 * p02, ba2 = k2 * p01;
  const double bt2 = ba0 + ba1 + ba2;
  const double bs0 = ba0 + bp01 * s1 + bp02 * s2;
  const double bs1 = ba1 + bp01 * s0 + bp12 * s2;
  const double bs2 = ba2 + bp02 * s0 + bp12 * s1;
  const double bb0 = 2.0 * b0 * bs0 + 2.0 * td * bt2;
  const double bb1 = 2.0 * b1 * bs1;
  const double bb2 = 2.0 * b2 * bs2 - 2.0 * td * bt2;
  const double bd0 = 2.0 * c13 * d0 * bb0, be0 = 0.5 * e0 * bb0;
  const double bd1 = 2.0 * c13 * d1 * bb1, be1 = 0.5 * e1 * bb1;
  const double bd2 = 2.0 * c13 * d2 * bb2, be2 = 0.5 * e2 * bb2;
  vb[0] = bd0 + be0 + 0.125 * (3.0 * bql0 - bqr2);
  vb[1] = -2.0 * bd0 - 4.0 * be0 + bd1 + be1 + 0.125 * (-10.0 * bql0 - bql1 + 3.0 * bqr1 + 6.0 * bqr2);
  vb[2] = bd0 + 3.0 * be0 - 2.0 * bd1 + bd2 + 3.0 * be2 +
          0.125 * (15.0 * bql0 + 6.0 * bql1 + 3.0 * bql2 + 15.0 * bqr0 + 6.0 * bqr1 + 3.0 * bqr2);
  vb[3] = bd1 - be1 - 2.0 * bd2 - 4.0 * be2 + 0.125 * (3.0 * bql1 + 6.0 * bql2 - 10.0 * bqr0 - bqr1);
  vb[4] = bd2 + be2 + 0.125 * (-bql2 + 3.0 * bqr0);
}

// out += d(G . F^d_lin)/dW for a run-time direction.
__device__ inline void flux_lin_vjp_d(int d, const Metric& M, const double* G, double* out) {
  if (d == 0) flux_lin_vjp<0>(M, G, out);
  else if (d == 1) flux_lin_vjp<1>(M, G, out);
  else flux_lin_vjp<2>(M, G, out);
}

struct FdAdj {
  const double* lam;     // [9][E][m^3] adjoint input (lambda) of the FD elements
  double* ubar;          // [9][E][m^3] output (accumulated)
  const double* lam_dg;  // [9][E][n^3] adjoint input of the DG elements
  double* ubar_dg;       // [9][E][n^3] output of the DG elements (accumulated)
  const double* x_dg;    // [9][E][n^3] the DG values the ghost slabs were projected from
  double* wbar;          // [3][10][E][m^3] per-direction adjoints of the transported cell values
  double* gbar;          // [10][E][6][3][m^2] adjoints of ghost cells, per face and layer
  // nullable: the representation that updated each element in the substep, when
  // it differs from a.rep0 (what neighbours read) for elements rolled back in it
  const int32_t* rep_upd;
  int parts;
};

// One workgroup per (listed FD element, direction, row of pencils), as the forward
// flux kernel: adjoints of the transported components (U, J~^d) of the row's cells
// and of its ghost cells.
template <int N, bool CURVED>
__global__ __launch_bounds__(256) void k_fd_adj_flux(KArgs a, FdAdj b) {
  using Dm = Dims<N>;
  constexpr int m = Dm::m, mm = Dm::mm;
  constexpr int nf = (m + 1) * m * m;
  constexpr int L = m, C = m + 6, F = m + 1, CF = m + 2, NR = NV + 1;
  constexpr int TPB = 256;
  __shared__ double sW[NR * C * L];   // staged cells [k][ext cell][pencil]
  __shared__ double sWb[NR * C * L];  // their adjoints
  __shared__ double sLb[NR * F * L];  // adjoints of the left states [k][face][pencil]
  __shared__ double sRb[NR * F * L];  // adjoints of the right states
  __shared__ double sG[NV * F * L];   // adjoints of the face fluxes
  __shared__ double sM[CURVED ? NBGF * CF * L : 1];
  const int t = threadIdx.x;
  const int items = a.fd_count[a.sub] * 3 * m;
  // XCD-aware order, as in the forward flux kernel: each of the eight XCDs (which
  // receive workgroups in turn) takes a contiguous run of items, so the rows of
  // one element share one L2
  constexpr int NX = 8;
  const bool split = gridDim.x % NX == 0;
  const int xcd = split ? (int)blockIdx.x % NX : 0;
  const int per = split ? (items + NX - 1) / NX : items;
  const int step = split ? (int)gridDim.x / NX : (int)gridDim.x;
  for (int l = split ? (int)blockIdx.x / NX : (int)blockIdx.x; l < per; l += step) {
    const int item = xcd * per + l;
    if (item >= items) break;  // the same for every thread of the block
    const int e = a.fd_list[item / (3 * m)];
    const int d = (item / m) % 3;
    const int t2 = item % m;
    const RowNbrs nb = row_neighbours(a, e, d);
    const int str[3] = {1, m, m * m};
    const int t1ax = (d == 0) ? 1 : 0, t2ax = (d == 2) ? 1 : 2;
    // stage the cells -3 .. m+2 (as the forward kernel) and clear their adjoints
    for (int q = t; q < L * C; q += TPB) {
      int c, t1;
      if (d == 0) {
        c = q % C;
        t1 = q / C;
      } else {
        t1 = q % L;
        c = q / L;
      }
      const CellSrc cs = cell_source<N>(a, nb, e, d, c - 3, t1, t2);
      double W[NR];
      Metric Mc;
      if (cs.ptr) {
#pragma unroll
        for (int k = 0; k < NV; ++k) W[k] = cs.ptr[k * cs.stride];
        W[NV] = cs.ptr[(NV + d) * cs.stride];
        if (CURVED && c >= 2 && c <= m + 3) load_metric<CURVED>(a.bg_fd, a.E, mm, cs.elem, cs.cell, Mc);
      } else {
        double Ui[NV], Ub[NV], J[3];
        load_metric<CURVED>(a.bg_fd, a.E, mm, e, cs.cell, Mc);
        load9(a.w_fd, a.E, mm, e, cs.cell, Ui);
        // ghost layer lg (0 next to the face) of the pencil's cell (t1, t2)
        const int sg = (c >= m + 3) ? 1 : 0, lg = sg ? c - 3 - m : 2 - c;
        exterior_state(a, cs.bnd, d, sg, Ui, Mc, a.bfield_fd,
                       ((((size_t)e * 6 + 2 * d + sg) * 3 + lg) * m + t2) * m + t1,
                       (size_t)a.E * 6 * 3 * m * m, Ub);
        current_total(Ub, Mc, a.eta, J);
#pragma unroll
        for (int k = 0; k < NV; ++k) W[k] = Ub[k];
        W[NV] = (d == 0) ? J[0] : (d == 1 ? J[1] : J[2]);
      }
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        sW[(k * C + c) * L + t1] = W[k];
        sWb[(k * C + c) * L + t1] = 0.0;
      }
      if (CURVED && c >= 2 && c <= m + 3) {
        double* o = sM + (c - 2) * L + t1;
        o[0] = Mc.alpha;
        o[1 * CF * L] = Mc.beta[0];
        o[2 * CF * L] = Mc.beta[1];
        o[3 * CF * L] = Mc.beta[2];
#pragma unroll
        for (int k = 0; k < 6; ++k) o[(4 + k) * CF * L] = Mc.g[k];
      }
    }
    // adjoints of the face fluxes: L_c = -(m/h)(Fhat_{c+1/2} - Fhat_{c-1/2}) gives
    // Fhat_f the adjoint (m/h)(lambda_f - lambda_{f-1}) (cells of this element only)
    const double sc = (double)m / h_of(a, e, d);
    for (int q = t; q < F * L; q += TPB) {
      const int t1 = q % L, f = q / L;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const size_t base = ((size_t)v * a.E + e) * mm + t1 * str[t1ax] + t2 * str[t2ax];
        const double lr = (f < m) ? b.lam[base + (size_t)f * str[d]] : 0.0;
        const double ll = (f > 0) ? b.lam[base + (size_t)(f - 1) * str[d]] : 0.0;
        sG[(v * F + f) * L + t1] = sc * (lr - ll);
      }
    }
    __syncthreads();
    const bool corr = a.fd_order == 4;
    const double cs_ = corr ? 4.0 / 3.0 : 1.0;
    // adjoints of the reconstructed states at every face (Rusanov, linear fluxes)
    for (int q = t; q < F * L; q += TPB) {
      const int t1 = q % L, f = q / L;
      int tix;
      if (d == 0) tix = f + (m + 1) * (t1 + m * t2);
      else if (d == 1) tix = t1 + m * (f + (m + 1) * t2);
      else tix = t1 + m * (t2 + m * f);
      Metric Mf;
      load_metric<CURVED>(a.bg_face + (size_t)d * NBGF * a.E * nf, a.E, nf, e, tix, Mf);
      const double lam = CURVED ? char_speed(d, Mf) : 1.0;
      double Gh[NV], bl[NR], br[NR];
#pragma unroll
      for (int v = 0; v < NV; ++v) Gh[v] = 0.5 * cs_ * sG[(v * F + f) * L + t1];
#pragma unroll
      for (int k = 0; k < NR; ++k) bl[k] = 0.0;
      flux_lin_vjp_d(d, Mf, Gh, bl);
#pragma unroll
      for (int k = 0; k < NR; ++k) br[k] = bl[k];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        bl[v] += lam * Gh[v];
        br[v] -= lam * Gh[v];
      }
      bl[NV] += Gh[8];  // the q~ flux carries J~^d
      br[NV] += Gh[8];
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        sLb[(k * F + f) * L + t1] = bl[k];
        sRb[(k * F + f) * L + t1] = br[k];
      }
    }
    // adjoints of the corrector's cell fluxes F_c = F(w_c), cells -1 .. m
    if (corr) {
      for (int q = t; q < CF * L; q += TPB) {
        const int t1 = q % L, c = q / L - 1;
        Metric Mc;
        if (CURVED) {
          double fm[10];
          const double* o = sM + (c + 1) * L + t1;
#pragma unroll
          for (int k = 0; k < 10; ++k) fm[k] = o[k * CF * L];
          metric_from10(fm, Mc);
        } else {
          metric_flat(Mc);
        }
        double Gc[NV], wb[NR];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double gf0 = (c >= 0) ? sG[(v * F + c) * L + t1] : 0.0;
          const double gf1 = (c + 1 <= m) ? sG[(v * F + c + 1) * L + t1] : 0.0;
          Gc[v] = -(gf0 + gf1) / 6.0;
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) wb[k] = 0.0;
        flux_lin_vjp_d(d, Mc, Gc, wb);
        wb[NV] += Gc[8];
#pragma unroll
        for (int k = 0; k < NR; ++k) sWb[(k * C + c + 3) * L + t1] = wb[k];
      }
    }
    __syncthreads();
    // reconstruction: target cell c gives the left state of face c+1 and the right
    // state of face c from cells c-2 .. c+2; the five contributions of a target go to
    // five different cells, added one offset at a time (no two targets collide)
    const double eps = a.weno_eps;
    constexpr int NT = NR * CF * L;
    for (int base = 0; base < NT; base += TPB) {
      const int q = base + t;
      const bool ok = q < NT;
      int t1 = 0, c = 0, k = 0;
      double vb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      if (ok) {
        t1 = q % L;
        c = (q / L) % CF - 1;
        k = q / (CF * L);
        double vl[5];
#pragma unroll
        for (int z = 0; z < 5; ++z) vl[z] = sW[(k * C + c + 1 + z) * L + t1];
        const double gL = (c < m) ? sLb[(k * F + c + 1) * L + t1] : 0.0;
        const double gR = (c >= 0) ? sRb[(k * F + c) * L + t1] : 0.0;
        weno5z_cell_vjp(vl, eps, gL, gR, vb);
      }
#pragma unroll
      for (int z = 0; z < 5; ++z) {
        __syncthreads();
        if (ok) sWb[(k * C + c + 1 + z) * L + t1] += vb[z];
      }
    }
    __syncthreads();
    // own cells -> per-direction adjoints; ghost cells -> per face and layer
    for (int q = t; q < C * L; q += TPB) {
      int x, t1;
      if (d == 0) {
        x = q % C;
        t1 = q / C;
      } else {
        t1 = q % L;
        x = q / L;
      }
      const int c = x - 3;
      if (c >= 0 && c < m) {
        const int cell = c * str[d] + t1 * str[t1ax] + t2 * str[t2ax];
#pragma unroll
        for (int k = 0; k < NR; ++k)
          b.wbar[(((size_t)d * NR + k) * a.E + e) * mm + cell] = sWb[(k * C + x) * L + t1];
      } else {
        const int s = (c >= m) ? 1 : 0;
        const int l = s ? (c - m) : (-1 - c);
        const int f = 2 * d + s;
        // the ghosts of a Dirichlet face are constants: their adjoints are dropped
        const bool fixed = a.nbr[e * 6 + f] < -1;
#pragma unroll
        for (int k = 0; k < NR; ++k)
          b.gbar[((((size_t)k * a.E + e) * 6 + f) * 3 + l) * (m * m) + t1 + m * t2] =
              fixed ? 0.0 : sWb[(k * C + x) * L + t1];
      }
    }
    __syncthreads();  // the next item restages the tiles
  }
}

// At FD cell p of element e:  ub = (dL_ex/dX)^T V + (dS_stiff/dX)^T W, with X the
// cell's value (the stage value staged in w_fd).  The explicit part gathers the
// three directions' transported-component adjoints, the ghost adjoints the FD
// neighbours wrote for this cell (or, at a physical boundary, this element's own
// ghosts through the no-incoming-Poynting state; those of a Dirichlet face are
// zero, as its ghosts do not depend on the state; a DG neighbour reads this cell
// through its R-trace, whose transpose is already in wbar), the current's gradient
// and the sources; use_v / use_w switch the two parts off.
template <int N, bool CURVED>
__device__ inline void fd_cell_vjp(const KArgs& a, const FdAdj& b, int e, int p, const double* X, const Metric& M,
                                   const double* V, bool use_v, const double* W, bool use_w, double* ub) {
  using Dm = Dims<N>;
  constexpr int m = Dm::m, mm = Dm::mm;
  constexpr int NR = NV + 1;
  const int ci[3] = {p % m, (p / m) % m, p / (m * m)};
  const int32_t* upd = b.rep_upd ? b.rep_upd : a.rep0;
#pragma unroll
  for (int v = 0; v < NV; ++v) ub[v] = 0.0;
  double wJ[3] = {0.0, 0.0, 0.0};
  if (use_v) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
      for (int v = 0; v < NV; ++v) ub[v] += b.wbar[(((size_t)d * NR + v) * a.E + e) * mm + p];
      wJ[d] += b.wbar[(((size_t)d * NR + NV) * a.E + e) * mm + p];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int t1ax = (d == 0) ? 1 : 0, t2ax = (d == 2) ? 1 : 2;
      const int tt = ci[t1ax] + m * ci[t2ax];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int l = s ? (m - 1 - ci[d]) : ci[d];
        if (l > 2) continue;
        const int f = 2 * d + s;
        const int o = a.nbr[e * 6 + f];
        // a neighbour updated on DG read this cell through the R-trace; a neighbour
        // updated on FD read it as a ghost only if this element was on FD at the
        // substep start (else it read this element's ghost slab)
        if (o >= 0 && (upd[o] == 0 || a.rep0[e] != 1)) continue;
        if (o >= 0) {
          // the FD neighbour's ghost layer l on its face towards us is this cell
          const int fo = f ^ 1;
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            const double g = b.gbar[((((size_t)k * a.E + o) * 6 + fo) * 3 + l) * (m * m) + tt];
            if (k < NV) ub[k] += g;
            else wJ[d] += g;
          }
        } else if (l == 0) {
          // own ghosts: the no-incoming-Poynting state of this cell in all three layers
          double G10[NR];
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            G10[k] = 0.0;
#pragma unroll
            for (int ll = 0; ll < 3; ++ll)
              G10[k] += b.gbar[((((size_t)k * a.E + e) * 6 + f) * 3 + ll) * (m * m) + tt];
          }
          double Y[NV], gY[NV];
          const double side = s ? 1.0 : -1.0;
          boundary_state(d, side, X, M, Y);
          double El[3], Bl[3];
          lower3(M, X, El);
          lower3(M, X + 3, Bl);
          const int j1 = (d + 1) % 3, k1 = (d + 2) % 3;
          const bool inward = side * (El[j1] * Bl[k1] - El[k1] * Bl[j1]) < 0.0;
#pragma unroll
          for (int v = 0; v < NV; ++v) gY[v] = G10[v];
          double cj[3] = {0.0, 0.0, 0.0};
          cj[d] = G10[NV];
          current_vjp(Y, M, a.eta, cj, cj, gY);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const bool keep = (v < 3) ? !inward : (v != 6 && v != 7);
            if (keep) ub[v] += gY[v];
          }
        }
      }
    }
  }
  // the transported current J~^d of the cell, the explicit and the stiff sources
  double wa[3], wb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    wa[i] = wJ[i] - (use_v ? V[i] : 0.0);
    wb[i] = wJ[i] - (use_w ? W[i] : 0.0);
  }
  current_vjp(X, M, a.eta, wa, wb, ub);
  if (use_v) {
    MetricDeriv Dv;
    load_deriv<CURVED>(a.bg_fd, a.E, mm, e, p, Dv);
    source_lin_vjp<CURVED>(M, Dv, V, ub);
  }
  if (use_w) {
    ub[6] += -M.alpha * a.kpsi * W[6];
    ub[7] += -M.alpha * a.kphi * W[7];
  }
}

// Right-hand side adjoint of the FD cells: ubar += (dL/dU)^T lambda.
template <int N, bool CURVED>
__global__ __launch_bounds__(256) void k_fd_adj_gather(KArgs a, FdAdj b) {
  constexpr int mm = Dims<N>::mm;
  constexpr int BPE = (mm + 255) / 256;
  const int items = a.fd_count[a.sub] * BPE;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int e = a.fd_list[item / BPE];
    const int p = (item % BPE) * 256 + threadIdx.x;
    if (p >= mm) continue;
    Metric M;
    load_metric<CURVED>(a.bg_fd, a.E, mm, e, p, M);
    double X[NV], lam[NV], ub[NV];
    load9(a.w_fd, a.E, mm, e, p, X);
    load9(b.lam, a.E, mm, e, p, lam);
    fd_cell_vjp<N, CURVED>(a, b, e, p, X, M, lam, (b.parts & 1) != 0, lam, (b.parts & 2) != 0, ub);
#pragma unroll
    for (int v = 0; v < NV; ++v) b.ubar[((size_t)v * a.E + e) * mm + p] += ub[v];
  }
}

// One stage of the step adjoint on the FD cells (the DG nodes' kernel without the
// filter): the explicit operator is transposed at the stage value staged in w_fd,
// applied to the stage's vector V = r.v_in and the stiff vector r.w, then the
// implicit solve and the stage combination are transposed.
template <int N, bool CURVED, int STAGE>
__global__ __launch_bounds__(256) void k_fd_adj_stage(KArgs a, FdAdj b, AdjBufs r) {
  constexpr int mm = Dims<N>::mm;
  constexpr int BPE = (mm + 255) / 256;
  const int items = a.fd_count[a.sub] * BPE;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int e = a.fd_list[item / BPE];
    const int p = (item % BPE) * 256 + threadIdx.x;
    if (p >= mm) continue;
    const double dt = dt_of(a, e);
    if (STAGE == ADJ_A3) {
      double Z[NV];
      load9(r.mu, a.E, mm, e, p, Z);
      adj_a3_tail(r, a.E, mm, e, p, dt, Z);
      continue;
    }
    Metric M;
    load_metric<CURVED>(a.bg_fd, a.E, mm, e, p, M);
    double X[NV], V[NV], W[NV], ub[NV];
    load9(a.w_fd, a.E, mm, e, p, X);
    load9(r.v_in, a.E, mm, e, p, V);
    load9(r.w, a.E, mm, e, p, W);
    fd_cell_vjp<N, CURVED>(a, b, e, p, X, M, V, true, W, true, ub);
    if ((STAGE == ADJ_B3 || STAGE == ADJ_B2) && a.rep0[e] == 0) {
      // rolled back in this substep: the input came from DG through P
      store9(r.transfer, a.E, mm, e, p, ub);
      continue;
    }
    if (STAGE == ADJ_B3 || STAGE == ADJ_B2) {
      double Z[NV];
      solve_vjp(X, M, a, dt * IMEX_A, ub, Z);
      adj_b_tail<STAGE>(r, a.E, mm, e, p, dt, Z);
    } else {
      double Un[NV], U1[NV], U2[NV], S1[NV];
      load9(a.fd.Un, a.E, mm, e, p, Un);
      pre_stages(Un, M, a, dt, U1, U2, S1);
      adj_b1_tail(a, r, a.E, mm, e, p, M, dt, X, U1, ub);
    }
  }
}

// Adjoint of the R-traces the DG neighbours of an FD element read: one work item per
// (listed FD element, direction d), its two faces normal to d handled together.  At
// the DG face node the exterior state enters the lower-face lift as
// +(2/h)/w_0 (F(Ux)/2 + lambda Ux/2) and the upper-face lift as
// -(2/h)/w_N (F(Ux)/2 - lambda Ux/2); the adjoint of (Ux, J~x^d) is taken through
// R (x) R (x) R restricted to the face (row 0 or N along the normal) transposed, and
// the two faces' results are added to the element's adjoints wbar of direction d
// (after the flux adjoint) in one pass over its cells.  Work items of different
// directions write different parts of wbar, so none of them collide.
template <int N, bool CURVED>
__global__ __launch_bounds__(256) void k_fd_adj_trace(KArgs a, FdAdj b) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, nn = Dm::nn, mm = Dm::mm;
  constexpr int NR = NV + 1;
  __shared__ double sR[n * m];
  __shared__ double sT[NR * n * n];     // trace adjoint [k][a2][a1]
  __shared__ double s1[NR * n * m];     // [k][a2][c1]
  __shared__ double s2[2 * NR * m * m];  // per face side: [s][k][c2][c1]
  const int t = threadIdx.x;
  for (int q = t; q < n * m; q += 256) sR[q] = a.ops->R[q];
  const int32_t* upd = b.rep_upd ? b.rep_upd : a.rep0;
  const int items = a.fd_count[a.sub] * 3;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int e = a.fd_list[item / 3];
    const int d = item % 3;
    if (a.rep0[e] != 1) continue;  // rolled back in this substep: no trace was read
    const int t1ax = (d == 0) ? 1 : 0, t2ax = (d == 2) ? 1 : 2;
    const int strn[3] = {1, n, n * n};
    bool used[2];
    for (int s = 0; s < 2; ++s) {
      const int f = 2 * d + s;
      const int g = a.nbr[e * 6 + f];
      used[s] = g >= 0 && upd[g] == 0;
      if (!used[s]) continue;
      const int sg = 1 - s;  // the DG element's side of the shared face
      __syncthreads();
      for (int q = t; q < n * n; q += 256) {
        const int a1 = q % n, a2 = q / n;
        const int pn = (sg ? N : 0) * strn[d] + a1 * strn[t1ax] + a2 * strn[t2ax];
        Metric M;
        load_metric<CURVED>(a.bg_dg, a.E, nn, g, pn, M);
        double V[NV];
        load9(b.lam_dg, a.E, nn, g, pn, V);
        const double sc = 2.0 / h_of(a, g, d);
        const double lam = CURVED ? char_speed(d, M) : 1.0;
        const double wgt = sg ? sc / a.ops->w[N] : sc / a.ops->w[0];
        const double cG = sg ? -0.5 * wgt : 0.5 * wgt, cU = 0.5 * wgt * lam;
        double Gb[NV], Tb[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          Gb[v] = cG * V[v];
          Tb[v] = cU * V[v];
        }
        flux_lin_vjp_d(d, M, Gb, Tb);
#pragma unroll
        for (int v = 0; v < NV; ++v) sT[v * n * n + q] = Tb[v];
        sT[NV * n * n + q] = Gb[8];  // the q~ flux carries J~^d
      }
      __syncthreads();
      // first tangential axis: a1 (n) -> c1 (m)
      for (int q = t; q < NR * n * m; q += 256) {
        const int c1 = q % m, rest = q / m;  // rest = k n + a2
        double acc = 0.0;
#pragma unroll
        for (int z = 0; z < n; ++z) acc += sR[z * m + c1] * sT[rest * n + z];
        s1[q] = acc;
      }
      __syncthreads();
      // second tangential axis: a2 (n) -> c2 (m)
      double* s2s = s2 + s * NR * m * m;
      for (int q = t; q < NR * m * m; q += 256) {
        const int c1 = q % m, c2 = (q / m) % m, k = q / (m * m);
        double acc = 0.0;
#pragma unroll
        for (int z = 0; z < n; ++z) acc += sR[z * m + c2] * s1[(k * n + z) * m + c1];
        s2s[q] = acc;
      }
    }
    if (!used[0] && !used[1]) continue;  // the same for every thread of the block
    __syncthreads();
    // normal axis: row 0 of R for the lower face, row N for the upper one, spread
    // over the line, both faces in one pass
    for (int q = t; q < mm; q += 256) {
      const int ci[3] = {q % m, (q / m) % m, q / (m * m)};
      const double r0 = used[0] ? sR[ci[d]] : 0.0;
      const double r1 = used[1] ? sR[N * m + ci[d]] : 0.0;
      const int tt = ci[t1ax] + m * ci[t2ax];
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        double add = 0.0;
        if (used[0]) add += r0 * s2[k * m * m + tt];
        if (used[1]) add += r1 * s2[(NR + k) * m * m + tt];
        b.wbar[(((size_t)d * NR + k) * a.E + e) * mm + q] += add;
      }
    }
    __syncthreads();  // the next item rewrites s2
  }
}

// Adjoint of the ghost slabs a DG element hands to its FD neighbours: for each face
// with an FD neighbour, the neighbour's ghost adjoints (three layers, U and J~^d)
// taken back through P (x) P (x) P transposed to the element's nodes, then through
// the current's gradient to U.  One workgroup per DG element.
template <int N, bool CURVED>
__global__ __launch_bounds__(Dims<N>::tpb) void k_dg_adj_slab(KArgs a, FdAdj b) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, m = Dm::m, nn = Dm::nn, TPB = Dm::tpb;
  constexpr int NR = NV + 1;
  const int g = blockIdx.x;
  if (!a.live[g] || a.rep0[g] != 0) return;
  const int32_t* upd = b.rep_upd ? b.rep_upd : a.rep0;
  int need = 0;
  for (int f = 0; f < 6; ++f) {
    const int o = a.nbr[g * 6 + f];
    if (o >= 0 && upd[o] == 1) need |= 1 << f;
  }
  if (!need) return;
  // the ten components pass the three stages together (four barriers per face)
  __shared__ double sP[m * n];
  __shared__ double sG[NR * 3 * m * m];  // [k][l][c2][c1]
  __shared__ double sB[NR * 3 * n * m];  // [k][l][a2][c1]
  __shared__ double sA[NR * 3 * n * n];  // [k][l][a2][a1]
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int p = act ? t : 0;
  for (int q = t; q < m * n; q += TPB) sP[q] = a.ops->P[q];
  const int idx[3] = {p % n, (p / n) % n, p / (n * n)};
  double Wb[NV], Jb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int v = 0; v < NV; ++v) Wb[v] = 0.0;
  for (int f = 0; f < 6; ++f) {
    if (!(need & (1 << f))) continue;
    const int e = a.nbr[g * 6 + f];
    const int d = f >> 1, s = f & 1, fe = f ^ 1;
    const int t1ax = (d == 0) ? 1 : 0, t2ax = (d == 2) ? 1 : 2;
    __syncthreads();
    for (int q = t; q < NR * 3 * m * m; q += TPB) {
      const int k = q / (3 * m * m), r = q % (3 * m * m);
      sG[q] = b.gbar[(((size_t)k * a.E + e) * 6 + fe) * (3 * m * m) + r];
    }
    __syncthreads();
    // second tangential axis back: c2 (m) -> a2 (n)
    for (int q = t; q < NR * 3 * n * m; q += TPB) {
      const int c1 = q % m, a2 = (q / m) % n, kl = q / (n * m);  // kl = k 3 + l
      double acc = 0.0;
      for (int z = 0; z < m; ++z) acc += sP[z * n + a2] * sG[(kl * m + z) * m + c1];
      sB[q] = acc;
    }
    __syncthreads();
    // first tangential axis back: c1 (m) -> a1 (n)
    for (int q = t; q < NR * 3 * n * n; q += TPB) {
      const int a1 = q % n, rest = q / n;  // rest = (k 3 + l) n + a2
      double acc = 0.0;
      for (int z = 0; z < m; ++z) acc += sP[z * n + a1] * sB[rest * m + z];
      sA[q] = acc;
    }
    __syncthreads();
    // normal axis back: layers l (cells l or m-1-l) -> node index along d
    if (act) {
      const int zi = idx[d], a1 = idx[t1ax], a2 = idx[t2ax];
      double w3[3];
#pragma unroll
      for (int l = 0; l < 3; ++l) w3[l] = sP[(s ? (m - 1 - l) : l) * n + zi];
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) acc += w3[l] * sA[((k * 3 + l) * n + a2) * n + a1];
        if (k < NV) Wb[k] += acc;
        else Jb[d] += acc;
      }
    }
  }
  if (!act) return;
  Metric M;
  load_metric<CURVED>(a.bg_dg, a.E, nn, g, p, M);
  double X[NV];
  load9(b.x_dg, a.E, nn, g, p, X);
  current_vjp(X, M, a.eta, Jb, Jb, Wb);
#pragma unroll
  for (int v = 0; v < NV; ++v) b.ubar_dg[((size_t)v * a.E + g) * nn + p] += Wb[v];
}

template <int N, bool CURVED>
static void fd_coupling_t(const KArgs& a, const FdAdj& b, hipStream_t s) {
  constexpr int m = Dims<N>::m;
  const size_t flux_items = (size_t)a.E * 3 * m;
  launch_kernel(k_fd_adj_flux<N, CURVED>, dim3((unsigned)(flux_items < 2048 ? flux_items : 2048)), dim3(256), s, a,
                b);
  const size_t trace_items = (size_t)a.E * 3;
  launch_kernel(k_fd_adj_trace<N, CURVED>, dim3((unsigned)(trace_items < 2048 ? trace_items : 2048)), dim3(256), s,
                a, b);
  launch_kernel(k_dg_adj_slab<N, CURVED>, dim3(a.E), dim3(Dims<N>::tpb), s, a, b);
}

template <int N, bool CURVED>
static void fd_rhs_adjoint_t(const KArgs& a, const FdAdj& b, hipStream_t s) {
  constexpr int mm = Dims<N>::mm;
  const size_t cell_items = (size_t)a.E * ((mm + 255) / 256);
  if (b.parts & 1) fd_coupling_t<N, CURVED>(a, b, s);
  launch_kernel(k_fd_adj_gather<N, CURVED>, dim3((unsigned)(cell_items < 2048 ? cell_items : 2048)), dim3(256), s,
                a, b);
}

template <int N, bool CURVED>
static void fd_stage_adjoint_t(const KArgs& a, const FdAdj& b, const AdjBufs& r, int stage, hipStream_t s) {
  constexpr int mm = Dims<N>::mm;
  const size_t cell_items = (size_t)a.E * ((mm + 255) / 256);
  const dim3 grid((unsigned)(cell_items < 2048 ? cell_items : 2048)), block(256);
  switch (stage) {
    case ADJ_A3: launch_kernel(k_fd_adj_stage<N, CURVED, ADJ_A3>, grid, block, s, a, b, r); break;
    case ADJ_B3: launch_kernel(k_fd_adj_stage<N, CURVED, ADJ_B3>, grid, block, s, a, b, r); break;
    case ADJ_B2: launch_kernel(k_fd_adj_stage<N, CURVED, ADJ_B2>, grid, block, s, a, b, r); break;
    default: launch_kernel(k_fd_adj_stage<N, CURVED, ADJ_B1>, grid, block, s, a, b, r); break;
  }
}

// Degrees 3..8 (the adjoint entry points refuse N > 8).
#define GRFFE_FD_ADJ_DISPATCH(CALL)                 \
  if (curved) {                                     \
    switch (N) {                                    \
      case 3: CALL(3, true); break;                 \
      case 4: CALL(4, true); break;                 \
      case 5: CALL(5, true); break;                 \
      case 6: CALL(6, true); break;                 \
      case 7: CALL(7, true); break;                 \
      default: CALL(8, true); break;                \
    }                                               \
  } else {                                          \
    switch (N) {                                    \
      case 3: CALL(3, false); break;                \
      case 4: CALL(4, false); break;                \
      case 5: CALL(5, false); break;                \
      case 6: CALL(6, false); break;                \
      case 7: CALL(7, false); break;                \
      default: CALL(8, false); break;               \
    }                                               \
  }

void launch_fd_rhs_adjoint(const KArgs& a, int N, bool curved, const double* lam, double* ubar,
                           const double* lam_dg, double* ubar_dg, int parts, double* wbar, double* gbar,
                           hipStream_t s) {
  FdAdj b{};
  b.lam = lam;
  b.ubar = ubar;
  b.lam_dg = lam_dg;
  b.ubar_dg = ubar_dg;
  b.x_dg = a.dg.Un;
  b.wbar = wbar;
  b.gbar = gbar;
  b.parts = parts;
#define CALL(NN, CV) fd_rhs_adjoint_t<NN, CV>(a, b, s)
  GRFFE_FD_ADJ_DISPATCH(CALL)
#undef CALL
}

void launch_fd_step_coupling(const KArgs& a, int N, bool curved, const double* v_fd, const double* v_dg,
                             const double* x_dg, double* extra_dg, double* wbar, double* gbar,
                             const int32_t* rep_upd, hipStream_t s) {
  FdAdj b{};
  b.rep_upd = rep_upd;
  b.lam = v_fd;
  b.lam_dg = v_dg;
  b.ubar_dg = extra_dg;
  b.x_dg = x_dg;
  b.wbar = wbar;
  b.gbar = gbar;
  b.parts = 3;
#define CALL(NN, CV) fd_coupling_t<NN, CV>(a, b, s)
  GRFFE_FD_ADJ_DISPATCH(CALL)
#undef CALL
}

void launch_fd_step_stage(const KArgs& a, int N, bool curved, int stage, const AdjBufs& r, double* wbar,
                          double* gbar, hipStream_t s) {
  FdAdj b{};
  b.rep_upd = r.rep_upd;
  b.wbar = wbar;
  b.gbar = gbar;
  b.parts = 3;
#define CALL(NN, CV) fd_stage_adjoint_t<NN, CV>(a, b, r, stage, s)
  GRFFE_FD_ADJ_DISPATCH(CALL)
#undef CALL
}

}  // namespace grffe
