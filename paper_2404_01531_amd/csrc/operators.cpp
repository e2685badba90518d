// Host construction of the 1D operators of the DG and FD grids.
//
// Sec. III A: nodal basis on Legendre-Gauss-Lobatto (GLL) points with a lumped
// mass matrix, modal Legendre representation (Eq. modal expansion), exponential
// filter (Eq. exponential filter).  Sec. III C: 2N+1 uniform subcells, DG -> FD
// by evaluating the nodal polynomial at subcell centres, FD -> DG by the
// least-squares inverse of that projection (the degree-N least-squares fit of
// the cell-centre values of one axis, evaluated at the GLL nodes).
#include "grffe_internal.h"

#include <cmath>
#include <stdexcept>
#include <vector>

namespace grffe {

static void legendre_and_derivs(int N, double x, double& p, double& dp, double& ddp) {
  // P_N(x), P_N'(x), P_N''(x) by the three-term recurrence and the Legendre ODE
  double p0 = 1.0, p1 = x;
  if (N == 0) {
    p = 1.0;
    dp = 0.0;
    ddp = 0.0;
    return;
  }
  for (int k = 1; k < N; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // (1 - x^2) P' = N (P_{N-1} - x P_N)
  const double one = 1.0 - x * x;
  dp = N * (p0 - x * p1) / one;
  // (1 - x^2) P'' - 2 x P' + N (N+1) P = 0
  ddp = (2.0 * x * dp - N * (N + 1.0) * p) / one;
}

static double legendre(int p, double x) {
  if (p == 0) return 1.0;
  double a = 1.0, b = x;
  for (int k = 1; k < p; ++k) {
    const double c = ((2.0 * k + 1.0) * x * b - k * a) / (k + 1.0);
    a = b;
    b = c;
  }
  return b;
}

void gll_nodes_weights(int N, std::vector<double>& x, std::vector<double>& w) {
  const int n = N + 1;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  x[0] = -1.0;
  x[N] = 1.0;
  for (int j = 1; j < N; ++j) {
    // interior nodes: roots of P_N', Newton from the Chebyshev-Gauss-Lobatto guess
    double t = -std::cos(M_PI * j / N);
    for (int it = 0; it < 100; ++it) {
      double p, dp, ddp;
      legendre_and_derivs(N, t, p, dp, ddp);
      const double dt = dp / ddp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[j] = t;
  }
  for (int j = 0; j < n / 2; ++j) {  // exact symmetry
    const double s = 0.5 * (x[N - j] - x[j]);
    x[j] = -s;
    x[N - j] = s;
  }
  if (n % 2) x[N / 2] = 0.0;
  for (int j = 0; j < n; ++j) {
    const double pn = legendre(N, x[j]);
    w[j] = 2.0 / (N * (N + 1.0) * pn * pn);
  }
}

static std::vector<double> bary_weights(const std::vector<double>& x) {
  const int n = (int)x.size();
  std::vector<double> b(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) b[j] /= (x[j] - x[k]);
  return b;
}

// row-major M[r*n + j] = l_j(pts[r]) (barycentric form of the Lagrange basis)
static std::vector<double> lagrange_eval(const std::vector<double>& x, const std::vector<double>& pts) {
  const int n = (int)x.size();
  const std::vector<double> b = bary_weights(x);
  std::vector<double> M(pts.size() * n, 0.0);
  for (size_t r = 0; r < pts.size(); ++r) {
    int hit = -1;
    for (int j = 0; j < n; ++j)
      if (pts[r] == x[j]) hit = j;
    if (hit >= 0) {
      M[r * n + hit] = 1.0;
      continue;
    }
    double den = 0.0;
    for (int j = 0; j < n; ++j) den += b[j] / (pts[r] - x[j]);
    for (int j = 0; j < n; ++j) M[r * n + j] = b[j] / (pts[r] - x[j]) / den;
  }
  return M;
}

static std::vector<double> invert(std::vector<double> A, int n) {
  // Gauss-Jordan with partial pivoting
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    for (int k = 0; k < n; ++k) {
      std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(I[c * n + k], I[piv * n + k]);
    }
    const double d = 1.0 / A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] *= d;
      I[c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[c * n + k];
        I[r * n + k] -= f * I[c * n + k];
      }
    }
  }
  return I;
}

static std::vector<double> modal_op(const std::vector<double>& x, const std::vector<double>& diag) {
  // V diag V^-1 with V[i][p] = L_p(x_i)
  const int n = (int)x.size();
  std::vector<double> V(n * n);
  for (int i = 0; i < n; ++i)
    for (int p = 0; p < n; ++p) V[i * n + p] = legendre(p, x[i]);
  const std::vector<double> Vi = invert(V, n);
  std::vector<double> out(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int p = 0; p < n; ++p) s += V[i * n + p] * diag[p] * Vi[p * n + j];
      out[i * n + j] = s;
    }
  return out;
}

int default_tci_M(int N) {
  int M = (N + 1) / 2;
  if (M > 3) M = 3;
  if (M < 2) M = 2;
  return M;
}

Ops1D build_ops(int N, double filter_a, double filter_b, int tci_M, int tci_mode) {
  Ops1D o;
  o.N = N;
  const int n = N + 1, m = 2 * N + 1;
  gll_nodes_weights(N, o.x, o.w);
  // derivative matrix D[i][j] = l_j'(x_i): barycentric differentiation formula
  const std::vector<double> b = bary_weights(o.x);
  o.D.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const double v = (b[j] / b[i]) / (o.x[i] - o.x[j]);
      o.D[i * n + j] = v;
      diag -= v;
    }
    o.D[i * n + i] = diag;
  }
  std::vector<double> sig(n), low(n);
  for (int p = 0; p < n; ++p) {
    sig[p] = std::exp(-filter_a * std::pow((double)p / N, 2.0 * filter_b));
    low[p] = (tci_mode == 1) ? (p >= tci_M ? 1.0 : 0.0) : (p < tci_M ? 1.0 : 0.0);
  }
  o.F = modal_op(o.x, sig);
  o.L = modal_op(o.x, low);
  std::vector<double> xc(m), xf(m + 1);
  for (int k = 0; k < m; ++k) xc[k] = -1.0 + (2.0 * k + 1.0) / m;
  for (int k = 0; k <= m; ++k) xf[k] = -1.0 + 2.0 * k / m;
  xf[0] = -1.0;
  xf[m] = 1.0;
  o.P = lagrange_eval(o.x, xc);   // m x n
  o.Q = lagrange_eval(o.x, xf);   // (m+1) x n
  // reconstruction: least-squares fit of degree N to the m cell values, evaluated at the nodes
  const int q = n;
  std::vector<double> A(m * q), AtA(q * q, 0.0);
  for (int k = 0; k < m; ++k)
    for (int p = 0; p < q; ++p) A[k * q + p] = legendre(p, xc[k]);
  for (int p = 0; p < q; ++p)
    for (int r = 0; r < q; ++r) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += A[k * q + p] * A[k * q + r];
      AtA[p * q + r] = s;
    }
  const std::vector<double> G = invert(AtA, q);
  o.R.assign(n * m, 0.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < m; ++k) {
      double s = 0.0;
      for (int p = 0; p < q; ++p) {
        double c = 0.0;  // (G A^T)[p][k]
        for (int r = 0; r < q; ++r) c += G[p * q + r] * A[k * q + r];
        s += legendre(p, o.x[j]) * c;
      }
      o.R[j * m + k] = s;
    }
  return o;
}

}  // namespace grffe
