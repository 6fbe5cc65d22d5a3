// Forward-mode dual number (value, one tangent) for device code. The reverse
// pass evaluates the bond function on it to obtain exact Jacobian columns.
#pragma once
#include <hip/hip_runtime.h>

namespace rodmx {

struct DD {
  double v, d;
  __device__ DD() : v(0.0), d(0.0) {}
  __device__ DD(double a) : v(a), d(0.0) {}
  __device__ DD(double a, double b) : v(a), d(b) {}
  __device__ explicit operator double() const { return v; }
  __device__ explicit operator float() const { return (float)v; }
};

__device__ __forceinline__ DD operator+(DD a, DD b) { return DD(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ DD operator+(DD a, double b) { return DD(a.v + b, a.d); }
__device__ __forceinline__ DD operator+(double a, DD b) { return DD(a + b.v, b.d); }
__device__ __forceinline__ DD operator-(DD a, DD b) { return DD(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ DD operator-(DD a, double b) { return DD(a.v - b, a.d); }
__device__ __forceinline__ DD operator-(double a, DD b) { return DD(a - b.v, -b.d); }
__device__ __forceinline__ DD operator-(DD a) { return DD(-a.v, -a.d); }
__device__ __forceinline__ DD operator*(DD a, DD b) { return DD(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ DD operator*(DD a, double b) { return DD(a.v * b, a.d * b); }
__device__ __forceinline__ DD operator*(double a, DD b) { return DD(a * b.v, a * b.d); }
__device__ __forceinline__ DD operator/(DD a, DD b) {
  return DD(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
__device__ __forceinline__ DD operator/(DD a, double b) { return DD(a.v / b, a.d / b); }
__device__ __forceinline__ DD operator/(double a, DD b) { return DD(a / b.v, -a * b.d / (b.v * b.v)); }
__device__ __forceinline__ DD& operator+=(DD& a, DD b) { a = a + b; return a; }
__device__ __forceinline__ DD& operator-=(DD& a, DD b) { a = a - b; return a; }
__device__ __forceinline__ bool operator<(DD a, DD b) { return a.v < b.v; }
__device__ __forceinline__ bool operator>(DD a, DD b) { return a.v > b.v; }
__device__ __forceinline__ bool operator<(DD a, double b) { return a.v < b; }
__device__ __forceinline__ bool operator>(DD a, double b) { return a.v > b; }

__device__ __forceinline__ DD sqrt(DD a) {
  const double s = ::sqrt(a.v);
  return DD(s, s > 0.0 ? a.d / (2.0 * s) : 0.0);
}
__device__ __forceinline__ DD rsqrt_norm(DD a) { return 1.0 / sqrt(a); }
__device__ __forceinline__ DD atan2(DD y, DD x) {
  const double den = x.v * x.v + y.v * y.v;
  return DD(::atan2(y.v, x.v), den > 0.0 ? (x.v * y.d - y.v * x.d) / den : 0.0);
}

template <class R> __device__ __forceinline__ R atan2_(R y, R x);
template <class R> __device__ __forceinline__ R sqrt_(R a);
template <> __device__ __forceinline__ DD atan2_(DD y, DD x) { return atan2(y, x); }
template <> __device__ __forceinline__ DD sqrt_(DD a) { return sqrt(a); }

}  // namespace rodmx
