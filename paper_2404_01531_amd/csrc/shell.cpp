// Host geometry of the spherical shell of cubed-sphere wedges (Sec. IV B, the
// black-hole grid) with curved element maps (Sec. III A, x(xi) per element).
//
// Wedge w about s e_k (k = w / 2, s = +1 for even w, -1 for odd w) has coordinates
// (A, B, Z) in [-1, 1]^3: the equiangular map X = tan(pi A / 4), Y = tan(pi B / 4)
// along the angular directions and the logarithmic map r = r_in (r_out/r_in)^((Z+1)/2)
// along the radial one; its local point r (X, Y, 1) / sqrt(1 + X^2 + Y^2) is turned
// onto the axes (s e_{k+1}, e_{k+2}, s e_k).  Each wedge is cut into n_radial x
// n_angular x n_angular elements of equal extent in (A, B, Z).  Everything here runs
// once at set-up: the inverse Jacobian at the DG nodes (closed-form chain rule), the
// neighbour across every face (faces are matched by their centres, face nodes by
// position, so the orientations between wedges need no table) and the smallest
// distance between neighbouring nodes along a reference line (the time step).
#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "grffe_internal.h"

namespace grffe {

namespace {

struct ElemIdx {
  int w, ir, ib, ia;
};

ElemIdx split(const grffe_shell& s, int e) {
  const int na = s.n_angular, nr = s.n_radial;
  return ElemIdx{e / (na * na * nr), (e / (na * na)) % nr, (e / na) % na, e % na};
}

// Position and, if J is given, d x^a / d xi^i (J[3 a + i]) of the reference point
// (x1, x2, x3) of element e.
void map_point(const grffe_shell& s, int e, double x1, double x2, double x3, double* P, double* J) {
  const ElemIdx q = split(s, e);
  const double na = s.n_angular, nr = s.n_radial;
  const double A = -1.0 + (q.ia + 0.5 * (x1 + 1.0)) * 2.0 / na;
  const double B = -1.0 + (q.ib + 0.5 * (x2 + 1.0)) * 2.0 / na;
  const double Z = -1.0 + (q.ir + 0.5 * (x3 + 1.0)) * 2.0 / nr;
  const double X = std::tan(0.25 * M_PI * A), Y = std::tan(0.25 * M_PI * B);
  const double lg = std::log(s.r_out / s.r_in);
  const double r = s.r_in * std::exp(0.5 * (Z + 1.0) * lg);
  const double rho = std::sqrt(1.0 + X * X + Y * Y);
  // local frame: L = (r / rho) (X, Y, 1)
  const double L[3] = {r * X / rho, r * Y / rho, r / rho};
  // dL/dX = r [e_1 / rho - X (X, Y, 1) / rho^3], dL/dY likewise, dL/dr = (X, Y, 1) / rho
  double dL[3][3];  // dL[l][i] = d L_l / d xi^i
  const double r3 = r / (rho * rho * rho);
  const double dX = 0.25 * M_PI * (1.0 + X * X) / na, dY = 0.25 * M_PI * (1.0 + Y * Y) / na;
  const double dr = 0.5 * r * lg / nr;
  const double v[3] = {X, Y, 1.0};
  for (int l = 0; l < 3; ++l) {
    dL[l][0] = ((l == 0 ? r / rho : 0.0) - r3 * X * v[l]) * dX;
    dL[l][1] = ((l == 1 ? r / rho : 0.0) - r3 * Y * v[l]) * dY;
    dL[l][2] = v[l] / rho * dr;
  }
  // rotation onto the wedge's axis: local l -> physical axis ax[l] with sign sg[l]
  const int k = q.w / 2;
  const double sw = (q.w % 2 == 0) ? 1.0 : -1.0;
  const int ax[3] = {(k + 1) % 3, (k + 2) % 3, k};
  const double sg[3] = {sw, 1.0, sw};
  for (int l = 0; l < 3; ++l) {
    P[ax[l]] = sg[l] * L[l];
    if (J)
      for (int i = 0; i < 3; ++i) J[3 * ax[l] + i] = sg[l] * dL[l][i];
  }
}

// inv[3 i + a] = d xi^i / d x^a from J[3 a + i] = d x^a / d xi^i, by cofactors;
// returns det J.
double invert(const double* J, double* inv) {
  const double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
  const double c10 = J[2] * J[7] - J[1] * J[8], c11 = J[0] * J[8] - J[2] * J[6], c12 = J[1] * J[6] - J[0] * J[7];
  const double c20 = J[1] * J[5] - J[2] * J[4], c21 = J[2] * J[3] - J[0] * J[5], c22 = J[0] * J[4] - J[1] * J[3];
  const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
  const double cof[9] = {c00, c01, c02, c10, c11, c12, c20, c21, c22};
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) inv[3 * i + a] = cof[3 * a + i] / det;
  return det;
}

// Flat node index of face node t = t1 + n t2 of face f = 2 d + s.
int face_node(int n, int f, int t) {
  const int d = f >> 1, lay = (f & 1) ? n - 1 : 0, t1 = t % n, t2 = t / n;
  return d == 0 ? lay + n * (t1 + n * t2) : (d == 1 ? t1 + n * (lay + n * t2) : t1 + n * (t2 + n * lay));
}

}  // namespace

int shell_validate(const grffe_shell* s, std::string& err) {
  if (!s) return err = "shell must not be NULL", GRFFE_EINVAL;
  if (s->degree < 3 || s->degree > MAX_DEG) return err = "degree must be in [3, 9]", GRFFE_EINVAL;
  if (s->n_radial < 1 || s->n_angular < 1) return err = "element counts must be positive", GRFFE_EINVAL;
  if (!(s->r_in > 0.0) || !(s->r_out > s->r_in) || !std::isfinite(s->r_out))
    return err = "radii must satisfy 0 < r_in < r_out", GRFFE_EINVAL;
  for (int b : {s->bc_inner, s->bc_outer})
    if (b != GRFFE_BC_OUTFLOW && b != GRFFE_BC_DIRICHLET && b != GRFFE_BC_NO_INCOMING_POYNTING)
      return err = "a sphere takes GRFFE_BC_OUTFLOW, _DIRICHLET or _NO_INCOMING_POYNTING", GRFFE_EINVAL;
  const double E = 6.0 * s->n_radial * (double)s->n_angular * s->n_angular;
  if (E > 1.0e7) return err = "too many elements", GRFFE_EINVAL;
  return GRFFE_OK;
}

void shell_points(const grffe_shell& s, bool fd, std::vector<double>& xyz) {
  const int N = s.degree, k = fd ? 2 * N + 1 : N + 1;
  std::vector<double> ref(k), w;
  if (fd) {
    for (int c = 0; c < k; ++c) ref[c] = -1.0 + (2.0 * c + 1.0) / k;
  } else {
    gll_nodes_weights(N, ref, w);
  }
  const int E = 6 * s.n_radial * s.n_angular * s.n_angular;
  const size_t P = (size_t)k * k * k;
  xyz.assign(3 * (size_t)E * P, 0.0);
  for (int e = 0; e < E; ++e)
    for (int c = 0; c < k; ++c)
      for (int b = 0; b < k; ++b)
        for (int a = 0; a < k; ++a) {
          double X[3];
          map_point(s, e, ref[a], ref[b], ref[c], X, nullptr);
          const size_t p = a + (size_t)k * (b + (size_t)k * c);
          for (int q = 0; q < 3; ++q) xyz[((size_t)q * E + e) * P + p] = X[q];
        }
}

int shell_geometry(const grffe_shell& s, ShellGeom& g, std::string& err) {
  const int N = s.degree, n = N + 1, nn = n * n * n, nf = n * n;
  const int E = 6 * s.n_radial * s.n_angular * s.n_angular;
  g.E = E;
  std::vector<double> x, w;
  gll_nodes_weights(N, x, w);
  std::vector<double> pos(3 * (size_t)E * nn);
  g.jinv.assign(9 * (size_t)E * nn, 0.0);
  for (int e = 0; e < E; ++e)
    for (int p = 0; p < nn; ++p) {
      double P[3], J[9];
      map_point(s, e, x[p % n], x[(p / n) % n], x[p / (n * n)], P, J);
      for (int q = 0; q < 3; ++q) pos[((size_t)e * nn + p) * 3 + q] = P[q];
      double inv[9];
      if (!(invert(J, inv) > 0.0)) return err = "degenerate element map", GRFFE_EINVAL;
      for (int q = 0; q < 9; ++q) g.jinv[((size_t)q * E + e) * nn + p] = inv[q];
    }
  // smallest distance between neighbouring nodes along a reference line
  g.dx_min = 1e300;
  for (int e = 0; e < E; ++e)
    for (int p = 0; p < nn; ++p)
      for (int d = 0; d < 3; ++d) {
        const int id = d == 0 ? p % n : (d == 1 ? (p / n) % n : p / (n * n));
        if (id == N) continue;
        const int q = p + (d == 0 ? 1 : (d == 1 ? n : n * n));
        double s2 = 0.0;
        for (int c = 0; c < 3; ++c) {
          const double dx = pos[((size_t)e * nn + q) * 3 + c] - pos[((size_t)e * nn + p) * 3 + c];
          s2 += dx * dx;
        }
        g.dx_min = std::min(g.dx_min, std::sqrt(s2));
      }
  // face centres, hashed on a grid much finer than any element and much coarser
  // than rounding; a match is searched in the 27 cells around a centre
  const double tol = 1e-9 * s.r_out;
  const double cell = 1e-6 * s.r_out;
  std::vector<double> cen(3 * (size_t)E * 6);
  auto key = [&](long long a, long long b, long long c) {
    return (unsigned long long)(a * 73856093LL) ^ (unsigned long long)(b * 19349663LL) ^
           (unsigned long long)(c * 83492791LL);
  };
  std::unordered_multimap<unsigned long long, int> table;
  for (int e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      double c[3] = {0.0, 0.0, 0.0};
      for (int t = 0; t < nf; ++t)
        for (int q = 0; q < 3; ++q) c[q] += pos[((size_t)e * nn + face_node(n, f, t)) * 3 + q];
      for (int q = 0; q < 3; ++q) cen[((size_t)e * 6 + f) * 3 + q] = c[q] / nf;
      const double* cc = &cen[((size_t)e * 6 + f) * 3];
      table.emplace(key(std::llround(cc[0] / cell), std::llround(cc[1] / cell), std::llround(cc[2] / cell)), e * 6 + f);
    }
  g.nbr.assign((size_t)E * 6, 0);
  g.fnode.assign((size_t)E * 6 * nf, -1);
  for (int e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      const double* cc = &cen[((size_t)e * 6 + f) * 3];
      const long long k0 = std::llround(cc[0] / cell), k1 = std::llround(cc[1] / cell), k2 = std::llround(cc[2] / cell);
      int match = -1, found = 0;
      for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
          for (int c = -1; c <= 1; ++c) {
            auto range = table.equal_range(key(k0 + a, k1 + b, k2 + c));
            for (auto it = range.first; it != range.second; ++it) {
              const int of = it->second;
              if (of == e * 6 + f) continue;
              const double* oc = &cen[(size_t)of * 3];
              const double d2 = (oc[0] - cc[0]) * (oc[0] - cc[0]) + (oc[1] - cc[1]) * (oc[1] - cc[1]) +
                                (oc[2] - cc[2]) * (oc[2] - cc[2]);
              if (d2 <= tol * tol && of != match) {
                match = of;
                ++found;
              }
            }
          }
      const int ir = split(s, e).ir;
      if (found == 0) {
        const bool inner = f == 4 && ir == 0, outer = f == 5 && ir == s.n_radial - 1;
        if (!inner && !outer) return err = "a face inside the shell has no neighbour", GRFFE_EINVAL;
        const int bc = inner ? s.bc_inner : s.bc_outer;
        g.nbr[(size_t)e * 6 + f] =
            bc == GRFFE_BC_OUTFLOW ? NBR_OUTFLOW : (bc == GRFFE_BC_DIRICHLET ? -2 - f : -1);
        continue;
      }
      if (found != 1) return err = "a face matches more than one neighbour face", GRFFE_EINVAL;
      const int o = match / 6, fo = match % 6;
      g.nbr[(size_t)e * 6 + f] = o;
      std::vector<char> used(nf, 0);
      for (int t = 0; t < nf; ++t) {
        const double* pe = &pos[((size_t)e * nn + face_node(n, f, t)) * 3];
        int hit = -1;
        for (int u = 0; u < nf; ++u) {
          const double* po = &pos[((size_t)o * nn + face_node(n, fo, u)) * 3];
          const double d2 = (po[0] - pe[0]) * (po[0] - pe[0]) + (po[1] - pe[1]) * (po[1] - pe[1]) +
                            (po[2] - pe[2]) * (po[2] - pe[2]);
          if (d2 <= tol * tol) {
            hit = u;
            break;
          }
        }
        if (hit < 0 || used[hit]) return err = "face nodes of neighbours do not coincide", GRFFE_EINVAL;
        used[hit] = 1;
        g.fnode[((size_t)e * 6 + f) * nf + t] = face_node(n, fo, hit);
      }
    }
  return GRFFE_OK;
}

// FD subcells: the inverse Jacobian at the cell centres, the unit covectors at the
// faces, and for every face between elements the neighbour's face and, per face
// cell, its face cell at the same point.  The orientation between two matched faces
// is one of the eight symmetries of the square; it is read off the DG face-node
// match (three corners), applied to the face cells, and every face-cell pair is
// checked by position.  Needs shell_geometry's tables.
int shell_fd_geometry(const grffe_shell& s, ShellGeom& g, std::string& err) {
  const int N = s.degree, n = N + 1, nf = n * n, m = 2 * N + 1, mm = m * m * m, mf = m * m;
  const int E = g.E;
  std::vector<double> cen(m), fac(m + 1);
  for (int c = 0; c < m; ++c) cen[c] = -1.0 + (2.0 * c + 1.0) / m;
  for (int c = 0; c <= m; ++c) fac[c] = -1.0 + 2.0 * c / m;
  g.jinv_fd.assign(9 * (size_t)E * mm, 0.0);
  const size_t nfc = (size_t)(m + 1) * mf;
  g.nu_face.assign(9 * (size_t)E * nfc, 0.0);
  for (int e = 0; e < E; ++e) {
    for (int p = 0; p < mm; ++p) {
      double P[3], J[9], inv[9];
      map_point(s, e, cen[p % m], cen[(p / m) % m], cen[p / mf], P, J);
      if (!(invert(J, inv) > 0.0)) return err = "degenerate element map", GRFFE_EINVAL;
      for (int q = 0; q < 9; ++q) g.jinv_fd[((size_t)q * E + e) * mm + p] = inv[q];
    }
    for (int d = 0; d < 3; ++d) {
      const int lx = d == 0 ? m + 1 : m, ly = d == 1 ? m + 1 : m;
      for (size_t q = 0; q < nfc; ++q) {
        const int cx = (int)(q % lx), cy = (int)((q / lx) % ly), cz = (int)(q / ((size_t)lx * ly));
        double P[3], J[9], inv[9];
        map_point(s, e, d == 0 ? fac[cx] : cen[cx], d == 1 ? fac[cy] : cen[cy], d == 2 ? fac[cz] : cen[cz], P, J);
        invert(J, inv);
        const double* r = inv + 3 * d;
        const double len = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        for (int j = 0; j < 3; ++j) g.nu_face[(((size_t)d * 3 + j) * E + e) * nfc + q] = r[j] / len;
      }
    }
  }
  // tangential coordinates (u1, u2) of a node or cell on face f (lower axis first)
  auto tang = [](int k, int f, int p, int& u1, int& u2) {
    const int d = f >> 1, c[3] = {p % k, (p / k) % k, p / (k * k)};
    const int lo = d == 0 ? 1 : 0, hi = d == 2 ? 1 : 2;
    u1 = c[lo];
    u2 = c[hi];
  };
  // point of face cell (c1, c2) on face f of element e
  auto face_cell_point = [&](int e, int f, int c1, int c2, double* P) {
    const int d = f >> 1;
    double r[3];
    const int lo = d == 0 ? 1 : 0, hi = d == 2 ? 1 : 2;
    r[d] = (f & 1) ? 1.0 : -1.0;
    r[lo] = cen[c1];
    r[hi] = cen[c2];
    map_point(s, e, r[0], r[1], r[2], P, nullptr);
  };
  const double tol = 1e-9 * s.r_out;
  g.nface.assign((size_t)E * 6, -1);
  g.fcell.assign((size_t)E * 6 * mf, -1);
  for (int e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      const int o = g.nbr[(size_t)e * 6 + f];
      if (o < 0) continue;
      const int32_t* fn = &g.fnode[((size_t)e * 6 + f) * nf];
      // the neighbour's face: the one on which its matched nodes lie
      int fo = -1;
      for (int cand = 0; cand < 6 && fo < 0; ++cand) {
        const int dd = cand >> 1, lay = (cand & 1) ? N : 0;
        bool all = true;
        for (int t = 0; t < nf && all; ++t) {
          const int pn = fn[t], c[3] = {pn % n, (pn / n) % n, pn / (n * n)};
          all = c[dd] == lay;
        }
        if (all && g.nbr[(size_t)o * 6 + cand] == e) fo = cand;
      }
      if (fo < 0) return err = "no neighbour face holds the matched nodes", GRFFE_EINVAL;
      g.nface[(size_t)e * 6 + f] = fo;
      int u00[2], u10[2], u01[2];
      tang(n, fo, fn[0], u00[0], u00[1]);
      tang(n, fo, fn[N], u10[0], u10[1]);
      tang(n, fo, fn[N * n], u01[0], u01[1]);
      const int a1[2] = {(u10[0] - u00[0]) / N, (u10[1] - u00[1]) / N};
      const int a2[2] = {(u01[0] - u00[0]) / N, (u01[1] - u00[1]) / N};
      const int b[2] = {u00[0] / N * (m - 1), u00[1] / N * (m - 1)};
      for (int c2 = 0; c2 < m; ++c2)
        for (int c1 = 0; c1 < m; ++c1) {
          const int v1 = b[0] + a1[0] * c1 + a2[0] * c2, v2 = b[1] + a1[1] * c1 + a2[1] * c2;
          if (v1 < 0 || v1 >= m || v2 < 0 || v2 >= m) return err = "face orientation out of range", GRFFE_EINVAL;
          double Pe[3], Po[3];
          face_cell_point(e, f, c1, c2, Pe);
          face_cell_point(o, fo, v1, v2, Po);
          const double d2 = (Pe[0] - Po[0]) * (Pe[0] - Po[0]) + (Pe[1] - Po[1]) * (Pe[1] - Po[1]) +
                            (Pe[2] - Po[2]) * (Pe[2] - Po[2]);
          if (!(d2 <= tol * tol)) return err = "face cells of neighbours do not coincide", GRFFE_EINVAL;
          g.fcell[((size_t)e * 6 + f) * mf + c1 + m * c2] = v1 + m * v2;
        }
    }
  (void)tang;
  return GRFFE_OK;
}

}  // namespace grffe
