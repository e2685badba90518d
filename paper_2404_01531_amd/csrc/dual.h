// Forward-mode dual numbers (value, one directional derivative) for the pointwise
// Jacobians of the adjoint: instantiating the pointwise physics with Dual and
// seeding U_k with derivative 1 gives column k of dF/dU exactly (no truncation).
// Comparisons act on the value, so a branch taken in the forward evaluation is
// also the branch differentiated.
#pragma once
#include <hip/hip_runtime.h>

namespace grffe {

// keep the FP64 overloads visible next to the Dual ones declared below
using ::fmax;
using ::sqrt;

struct Dual {
  double v, d;
  __device__ Dual() = default;
  __device__ constexpr Dual(double x) : v(x), d(0.0) {}
  __device__ constexpr Dual(double x, double y) : v(x), d(y) {}
  explicit __device__ operator double() const { return v; }
  __device__ Dual& operator+=(const Dual& b) {
    v += b.v;
    d += b.d;
    return *this;
  }
  __device__ Dual& operator-=(const Dual& b) {
    v -= b.v;
    d -= b.d;
    return *this;
  }
  __device__ Dual& operator*=(const Dual& b) {
    d = d * b.v + v * b.d;
    v *= b.v;
    return *this;
  }
};

__device__ inline Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
__device__ inline Dual operator+(const Dual& a, const Dual& b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ inline Dual operator-(const Dual& a, const Dual& b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ inline Dual operator*(const Dual& a, const Dual& b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ inline Dual operator/(const Dual& a, const Dual& b) {
  const double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ inline Dual operator+(const Dual& a, double b) { return Dual(a.v + b, a.d); }
__device__ inline Dual operator+(double a, const Dual& b) { return Dual(a + b.v, b.d); }
__device__ inline Dual operator-(const Dual& a, double b) { return Dual(a.v - b, a.d); }
__device__ inline Dual operator-(double a, const Dual& b) { return Dual(a - b.v, -b.d); }
__device__ inline Dual operator*(const Dual& a, double b) { return Dual(a.v * b, a.d * b); }
__device__ inline Dual operator*(double a, const Dual& b) { return Dual(a * b.v, a * b.d); }
__device__ inline Dual operator/(const Dual& a, double b) { return Dual(a.v / b, a.d / b); }
__device__ inline Dual operator/(double a, const Dual& b) {
  const double q = a / b.v;
  return Dual(q, -q * b.d / b.v);
}
__device__ inline bool operator<(const Dual& a, double b) { return a.v < b; }
__device__ inline bool operator>(const Dual& a, double b) { return a.v > b; }
__device__ inline bool operator<(const Dual& a, const Dual& b) { return a.v < b.v; }
__device__ inline bool operator>(const Dual& a, const Dual& b) { return a.v > b.v; }
// max(a, b): the derivative of the larger argument (of a at a tie)
__device__ inline Dual fmax(const Dual& a, const Dual& b) { return (b.v > a.v) ? b : a; }
__device__ inline Dual sqrt(const Dual& a) {
  const double r = ::sqrt(a.v);
  return Dual(r, r > 0.0 ? 0.5 * a.d / r : 0.0);
}

}  // namespace grffe
