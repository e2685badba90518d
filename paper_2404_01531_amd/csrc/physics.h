// Pointwise GRFFE physics on the device (FP64).
//
// Densitized evolved variables U = sqrt(gamma) (E^i, B^i, psi, phi, q),
// component order (Ex, Ey, Ez, Bx, By, Bz, psi, phi, q) (Sec. II A, the
// conservative form).  Spatial Levi-Civita tensor eps^{ijk} = [ijk]/sqrt(gamma)
// from the sign convention eps_abcd = sqrt(-g)[abcd], [0123] = +1.
//
//   current  (Eq. electric current density), densitized J~ = alpha sqrt(gamma) J:
//     J~ = alpha q~ [ijk] E~_j B~_k / (sqrt(gamma) B~^2)                 (drift)
//        + alpha eta [ (E~.B~/B~^2) B~ + max(E~^2 - B~^2, 0)/B~^2 E~ ]  (driver)
//   fluxes   (Eq. fluxes), sources (Eq. sources); the IMEX split (Sec. III B)
//   treats the driver current and the kappa damping as stiff.
#pragma once
#include <hip/hip_runtime.h>

namespace grffe {

// Metric at one point.  g and gi are symmetric, stored xx, xy, xz, yy, yz, zz.
template <typename T>
struct MetricT {
  T alpha, beta[3], g[6], gi[6], sqrtg, isqrtg;  // isqrtg = 1 / sqrt(gamma)
};
using Metric = MetricT<double>;

// The metric rounded to another arithmetic type (the FP32 flux evaluation of the
// mixed-precision mode).
template <typename T>
__device__ inline void metric_cast(const Metric& M, MetricT<T>& o) {
  o.alpha = (T)M.alpha;
  o.sqrtg = (T)M.sqrtg;
  o.isqrtg = (T)M.isqrtg;
  for (int k = 0; k < 3; ++k) o.beta[k] = (T)M.beta[k];
  for (int k = 0; k < 6; ++k) {
    o.g[k] = (T)M.g[k];
    o.gi[k] = (T)M.gi[k];
  }
}

__host__ __device__ inline int sym(int i, int j) {
  // index of (i, j) in the packed symmetric storage
  return (i == 0) ? j : (i == 1 ? (j == 0 ? 1 : 2 + j) : (j == 0 ? 2 : (j == 1 ? 4 : 5)));
}

__device__ inline void metric_flat(Metric& M) {
  M.alpha = 1.0;
  M.beta[0] = M.beta[1] = M.beta[2] = 0.0;
  for (int k = 0; k < 6; ++k) M.g[k] = M.gi[k] = 0.0;
  M.g[0] = M.g[3] = M.g[5] = 1.0;
  M.gi[0] = M.gi[3] = M.gi[5] = 1.0;
  M.sqrtg = 1.0;
  M.isqrtg = 1.0;
}

// From the 10 leading background fields (alpha, beta^i, gamma_ij packed).
__device__ inline void metric_from10(const double f[10], Metric& M) {
  M.alpha = f[0];
  M.beta[0] = f[1];
  M.beta[1] = f[2];
  M.beta[2] = f[3];
  for (int k = 0; k < 6; ++k) M.g[k] = f[4 + k];
  const double xx = f[4], xy = f[5], xz = f[6], yy = f[7], yz = f[8], zz = f[9];
  const double c_xx = yy * zz - yz * yz;
  const double c_xy = xz * yz - xy * zz;
  const double c_xz = xy * yz - xz * yy;
  const double c_yy = xx * zz - xz * xz;
  const double c_yz = xy * xz - xx * yz;
  const double c_zz = xx * yy - xy * xy;
  const double det = xx * c_xx + xy * c_xy + xz * c_xz;
  const double inv = 1.0 / det;
  M.gi[0] = c_xx * inv;
  M.gi[1] = c_xy * inv;
  M.gi[2] = c_xz * inv;
  M.gi[3] = c_yy * inv;
  M.gi[4] = c_yz * inv;
  M.gi[5] = c_zz * inv;
  M.sqrtg = sqrt(det);
  M.isqrtg = M.sqrtg * inv;
}

template <typename T>
__device__ inline void lower3(const MetricT<T>& M, const T* v, T* o) {
  o[0] = M.g[0] * v[0] + M.g[1] * v[1] + M.g[2] * v[2];
  o[1] = M.g[1] * v[0] + M.g[3] * v[1] + M.g[4] * v[2];
  o[2] = M.g[2] * v[0] + M.g[4] * v[1] + M.g[5] * v[2];
}

__device__ inline double dot3(const Metric& M, const double* u, const double* v) {
  double l[3];
  lower3(M, v, l);
  return u[0] * l[0] + u[1] * l[1] + u[2] * l[2];
}

// Densitized current split into drift (Jd) and driver (Je) parts.  T is the
// arithmetic type of the state (FP64, or a dual number for derivatives).
template <typename T>
__device__ inline void current(const T* U, const MetricT<T>& M, double eta, T* Jd, T* Je) {
  const T* E = U;
  const T* B = U + 3;
  T El[3], Bl[3];
  lower3(M, E, El);
  lower3(M, B, Bl);
  const T B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
  const T E2 = E[0] * El[0] + E[1] * El[1] + E[2] * El[2];
  const T EB = E[0] * Bl[0] + E[1] * Bl[1] + E[2] * Bl[2];
  // B^2 = 0: both parts vanish (1/B^2 is replaced by 0; no branch, so the
  // outputs stay in registers)
  const T iB2 = (B2 > 0.0) ? T(1.0) / B2 : T(0.0);
  const T cd = M.alpha * U[8] * iB2 * M.isqrtg;
  Jd[0] = cd * (El[1] * Bl[2] - El[2] * Bl[1]);
  Jd[1] = cd * (El[2] * Bl[0] - El[0] * Bl[2]);
  Jd[2] = cd * (El[0] * Bl[1] - El[1] * Bl[0]);
  const T ce = M.alpha * eta;
  const T par = EB * iB2;
  const T rec = fmax(E2 - B2, T(0.0)) * iB2;
  for (int i = 0; i < 3; ++i) Je[i] = ce * (par * B[i] + rec * E[i]);
}

template <typename T>
__device__ inline void current_total(const T* U, const MetricT<T>& M, double eta, T* J) {
  T Jd[3], Je[3];
  current(U, M, eta, Jd, Je);
  J[0] = Jd[0] + Je[0];
  J[1] = Jd[1] + Je[1];
  J[2] = Jd[2] + Je[2];
}

// F^d(U) with jd = J~^d, the component along d of the total densitized current
// (Eq. fluxes); only that component enters F^d.  T is the arithmetic type (FP64,
// or FP32 for the flux evaluation of the mixed-precision mode).
template <int D, typename T>
__device__ inline void flux_dir(const T* U, T jd, const MetricT<T>& M, T* F) {
  const T* E = U;
  const T* B = U + 3;
  T El[3], Bl[3];
  lower3(M, E, El);
  lower3(M, B, Bl);
  const T a = M.alpha, bd = M.beta[D], isg = M.isqrtg;
  const T psi = U[6], phi = U[7];
  // [i D k] X_k for i = 0..2
  T eB[3], eE[3];
  if (D == 0) {
    eB[0] = 0; eB[1] = -Bl[2]; eB[2] = Bl[1];
    eE[0] = 0; eE[1] = -El[2]; eE[2] = El[1];
  } else if (D == 1) {
    eB[0] = Bl[2]; eB[1] = 0; eB[2] = -Bl[0];
    eE[0] = El[2]; eE[1] = 0; eE[2] = -El[0];
  } else {
    eB[0] = -Bl[1]; eB[1] = Bl[0]; eB[2] = 0;
    eE[0] = -El[1]; eE[1] = El[0]; eE[2] = 0;
  }
  for (int i = 0; i < 3; ++i) {
    const T gid = M.gi[sym(i, D)];
    F[i] = -bd * E[i] + a * (gid * psi - eB[i] * isg);
    F[3 + i] = -bd * B[i] + a * (gid * phi + eE[i] * isg);
  }
  F[6] = -bd * psi + a * E[D];
  F[7] = -bd * phi + a * B[D];
  F[8] = jd - bd * U[8];
}

// F^d with the whole current vector J (its component d is used).
template <typename T>
__device__ inline void flux_any(int d, const T* U, const T* J, const MetricT<T>& M, T* F) {
  if (d == 0) flux_dir<0>(U, J[0], M, F);
  else if (d == 1) flux_dir<1>(U, J[1], M, F);
  else flux_dir<2>(U, J[2], M, F);
}

// F^d with the scalar jd = J~^d.
template <typename T>
__device__ inline void flux_any_jd(int d, const T* U, T jd, const MetricT<T>& M, T* F) {
  if (d == 0) flux_dir<0>(U, jd, M, F);
  else if (d == 1) flux_dir<1>(U, jd, M, F);
  else flux_dir<2>(U, jd, M, F);
}

// Background derivative fields at a point (curved only).
struct MetricDeriv {
  double da[3], db[9], K, Gam[3];  // db[3*j + i] = d_j beta^i
};

// Explicit (non-stiff) sources: everything but the driver current and kappa damping.
// The background (metric and its derivatives) is FP64; T is the state's type.
template <bool CURVED, typename T>
__device__ inline void source_explicit(const T* U, const MetricT<T>& M, const MetricDeriv& Dv, const T* Jd, T* S) {
  for (int i = 0; i < 3; ++i) S[i] = -Jd[i];
  S[3] = S[4] = S[5] = S[6] = S[7] = S[8] = T(0.0);
  if (CURVED) {
    const T a = M.alpha;
    T ga[3];
    for (int i = 0; i < 3; ++i)
      ga[i] = M.gi[sym(i, 0)] * Dv.da[0] + M.gi[sym(i, 1)] * Dv.da[1] + M.gi[sym(i, 2)] * Dv.da[2];
    for (int i = 0; i < 3; ++i) {
      T se = T(0.0), sb = T(0.0);
      for (int j = 0; j < 3; ++j) {
        se += U[j] * Dv.db[3 * j + i];
        sb += U[3 + j] * Dv.db[3 * j + i];
      }
      S[i] += -se + U[6] * (ga[i] - a * Dv.Gam[i]);
      S[3 + i] = -sb + U[7] * (ga[i] - a * Dv.Gam[i]);
    }
    S[6] = U[0] * Dv.da[0] + U[1] * Dv.da[1] + U[2] * Dv.da[2] + a * U[8] - a * U[6] * Dv.K;
    S[7] = U[3] * Dv.da[0] + U[4] * Dv.da[1] + U[5] * Dv.da[2] - a * U[7] * Dv.K;
  } else {
    S[6] = U[8];
  }
}

// Stiff sources: -J~_eta for E~, -alpha kappa for psi~, phi~.
template <typename T>
__device__ inline void source_stiff(const T* U, const MetricT<T>& M, double eta, double kpsi, double kphi, T* S) {
  T Jd[3], Je[3];
  current(U, M, eta, Jd, Je);
  S[0] = -Je[0];
  S[1] = -Je[1];
  S[2] = -Je[2];
  S[3] = S[4] = S[5] = T(0.0);
  S[6] = -M.alpha * kpsi * U[6];
  S[7] = -M.alpha * kphi * U[7];
  S[8] = T(0.0);
}

// Solve U = Y + h S_stiff(U) in place (Sec. III B).  B~ and q~ are unchanged;
// psi~, phi~ by the linear inversion; E~ split parallel/perpendicular to B~:
//   E = E*_perp / (1 + c s) + E*_par / (1 + c + c s),  c = alpha eta h,
// with s = 0 when that gives E^2 <= B^2, else the root s > 0 of
//   g(s) = |E*_perp|^2/(1+cs)^2 + |E*_par|^2/(1+c+cs)^2 - (1+s) B^2.
// g is decreasing and convex, so Newton's method started at s = 0 climbs
// monotonically to the root.
__device__ inline void implicit_solve(double* U, const Metric& M, double eta, double kpsi, double kphi, double h) {
  const double a = M.alpha;
  U[6] = U[6] / (1.0 + a * kpsi * h);
  U[7] = U[7] / (1.0 + a * kphi * h);
  const double* B = U + 3;
  double Bl[3];
  lower3(M, B, Bl);
  const double B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
  if (!(B2 > 0.0)) return;
  const double c = a * eta * h;
  const double EB = U[0] * Bl[0] + U[1] * Bl[1] + U[2] * Bl[2];
  const double k = EB / B2;
  double par[3], perp[3];
  for (int i = 0; i < 3; ++i) {
    par[i] = k * B[i];
    perp[i] = U[i] - par[i];
  }
  const double P2 = dot3(M, perp, perp);
  const double Q2 = dot3(M, par, par);
  const double ic = 1.0 / (1.0 + c);
  double cand[3];
  for (int i = 0; i < 3; ++i) cand[i] = perp[i] + par[i] * ic;
  double s = 0.0;
  if (dot3(M, cand, cand) > B2) {
    for (int it = 0; it < 200; ++it) {
      const double u = 1.0 / (1.0 + c * s);
      const double v = 1.0 / (1.0 + c + c * s);
      const double g = P2 * u * u + Q2 * v * v - (1.0 + s) * B2;
      if (!(g > 0.0)) break;
      const double dg = -2.0 * c * (P2 * u * u * u + Q2 * v * v * v) - B2;
      const double ds = -g / dg;
      const double sn = s + ds;
      if (!(sn > s)) break;
      s = sn;
      if (ds <= 1e-17 * s) break;
    }
  }
  const double fp = 1.0 / (1.0 + c * s);
  const double fq = 1.0 / (1.0 + c + c * s);
  for (int i = 0; i < 3; ++i) U[i] = perp[i] * fp + par[i] * fq;
}

// Algebraic force-free fix (Sec. II B): drop E parallel to B, then E^2 <= (1 - margin) B^2.
__device__ inline void constraint_clamp(double* U, const Metric& M, double margin) {
  const double* B = U + 3;
  double Bl[3];
  lower3(M, B, Bl);
  const double B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
  if (!(B2 > 0.0)) return;
  const double k = (U[0] * Bl[0] + U[1] * Bl[1] + U[2] * Bl[2]) / B2;
  for (int i = 0; i < 3; ++i) U[i] -= k * B[i];
  const double E2 = dot3(M, U, U);
  const double lim = (1.0 - margin) * B2;
  if (E2 > lim) {
    const double sc = sqrt(lim / E2);
    U[0] *= sc;
    U[1] *= sc;
    U[2] *= sc;
  }
}

// No-incoming-Poynting external state (Sec. III D); side = sign of the outward normal along x^d.
template <typename T>
__device__ inline void boundary_state(int d, double side, const T* Ui, const MetricT<T>& M, T* Ub) {
  T El[3], Bl[3];
  lower3(M, Ui, El);
  lower3(M, Ui + 3, Bl);
  const int j = (d + 1) % 3, k = (d + 2) % 3;
  const T Sd = El[j] * Bl[k] - El[k] * Bl[j];  // [d j k] E_j B_k
  const bool inward = side * Sd < 0.0;
  for (int i = 0; i < 3; ++i) {
    Ub[i] = inward ? T(0.0) : Ui[i];
    Ub[3 + i] = Ui[3 + i];
  }
  Ub[6] = T(0.0);
  Ub[7] = T(0.0);
  Ub[8] = Ui[8];
}

__device__ inline double char_speed(int d, const Metric& M) {
  // blended with 0/1 weights (exact for finite metric values), not indexed or
  // selected: with a run-time direction either form is turned into an indexed load,
  // which puts the whole Metric in private memory
  const double w0 = d == 0 ? 1.0 : 0.0, w1 = d == 1 ? 1.0 : 0.0, w2 = d == 2 ? 1.0 : 0.0;
  const double gdd = w0 * M.gi[0] + w1 * M.gi[3] + w2 * M.gi[5];
  const double bd = w0 * M.beta[0] + w1 * M.beta[1] + w2 * M.beta[2];
  return M.alpha * sqrt(gdd) + fabs(bd);
}

}  // namespace grffe
