// Device vector and quaternion helpers for the rod kernels (gfx950).
// Quaternions are (w, x, y, z) with the Hamilton product; q v q* is the active
// rotation of v by q.
#pragma once
#include <hip/hip_runtime.h>

namespace rodmx {

template <class R> struct V3 { R x, y, z; };
template <class R> struct Q4 { R w, x, y, z; };

template <class R> __device__ __forceinline__ V3<R> mk3(R x, R y, R z) { return V3<R>{x, y, z}; }
template <class R> __device__ __forceinline__ V3<R> operator+(V3<R> a, V3<R> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator-(V3<R> a, V3<R> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator-(V3<R> a) { return {-a.x, -a.y, -a.z}; }
template <class R> __device__ __forceinline__ V3<R> operator*(R s, V3<R> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class R> __device__ __forceinline__ R dot(V3<R> a, V3<R> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class R> __device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class To, class From> __device__ __forceinline__ V3<To> cvt(V3<From> a) {
  return {(To)a.x, (To)a.y, (To)a.z};
}
template <class To, class From> __device__ __forceinline__ Q4<To> cvtq(Q4<From> a) {
  return {(To)a.w, (To)a.x, (To)a.y, (To)a.z};
}

template <class R> __device__ __forceinline__ Q4<R> qmul(Q4<R> a, Q4<R> b) {
  return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
          a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
          a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
template <class R> __device__ __forceinline__ Q4<R> qconj(Q4<R> a) { return {a.w, -a.x, -a.y, -a.z}; }
template <class R> __device__ __forceinline__ R qdot(Q4<R> a, Q4<R> b) {
  return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z;
}
template <class R> __device__ __forceinline__ Q4<R> qscale(R s, Q4<R> a) { return {s * a.w, s * a.x, s * a.y, s * a.z}; }
template <class R> __device__ __forceinline__ Q4<R> qadd(Q4<R> a, Q4<R> b) {
  return {a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z};
}

// 1/sqrt(a) for a positive normal double: the hardware estimate (v_rsq_f64,
// about 23 correct bits) refined by two Newton steps y <- y (3/2 - (a/2) y^2),
// each of which doubles the correct bits; the result is within a few ulp. The
// quotient of a correctly rounded square root costs about three times as many
// instructions (scaled square root, then a full division).
__device__ __forceinline__ double rsqrt_nr(double a) {
  double y = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
  y = y * __builtin_fma(-h, y * y, 1.5);
  y = y * __builtin_fma(-h, y * y, 1.5);
  return y;
}
__device__ __forceinline__ double rsqrt_norm(double a) { return rsqrt_nr(a); }
__device__ __forceinline__ float rsqrt_norm(float a) { return 1.0f / sqrtf(a); }

// a / |a|; in FP64 with the refined reciprocal square root (the integrator
// renormalises four times per step, on the step's critical path).
template <class R> __device__ __forceinline__ Q4<R> qnormalize(Q4<R> a) {
  return qscale(rsqrt_norm(qdot(a, a)), a);
}

// q v q* for a unit quaternion: v + 2 w (u x v) + 2 u x (u x v), u = vector part.
template <class R> __device__ __forceinline__ V3<R> qrot(Q4<R> q, V3<R> v) {
  V3<R> u{q.x, q.y, q.z};
  V3<R> t = R(2) * cross(u, v);
  return v + q.w * t + cross(u, t);
}
// q* v q (rotation by the inverse).
template <class R> __device__ __forceinline__ V3<R> qrot_inv(Q4<R> q, V3<R> v) {
  return qrot(qconj(q), v);
}

// SoA plane access.
template <class R> __device__ __forceinline__ V3<R> ld3(const R* __restrict__ a, long n, long i) {
  return {a[i], a[n + i], a[2 * n + i]};
}
template <class R> __device__ __forceinline__ void st3(R* __restrict__ a, long n, long i, V3<R> v) {
  a[i] = v.x; a[n + i] = v.y; a[2 * n + i] = v.z;
}
template <class R> __device__ __forceinline__ Q4<R> ld4(const R* __restrict__ a, long n, long i) {
  return {a[i], a[n + i], a[2 * n + i], a[3 * n + i]};
}
template <class R> __device__ __forceinline__ void st4(R* __restrict__ a, long n, long i, Q4<R> q) {
  a[i] = q.w; a[n + i] = q.x; a[2 * n + i] = q.y; a[3 * n + i] = q.z;
}

}  // namespace rodmx
