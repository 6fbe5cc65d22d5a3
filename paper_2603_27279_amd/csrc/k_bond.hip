// Bond kernel: forces and torques of the co-rotational bond between consecutive
// particles of a rod (main text eq:bpm-fr, eq:bpm-fst, eq:bpm-tst, eq:bpm-tb,
// eq:bpm-tt, eq:bpm-vector; SI "Symmetric rotational decomposition").
//
// One thread per bond (k, k+1); results are written per bond and gathered by
// the particle kernel from bonds k-1 and k, so no two threads ever add into the
// same particle (no atomics).
//
// Precision. The quantities that cancel are formed in FP64 (the "head"): the
// central frame q_C, the bond vector seen from it, its length change r - r0,
// its direction change delta = r_f^[C] - r_i^, the half rotation u0 = q_C* q2
// and the alignment quaternion m. Everything derived from those small, well
// conditioned values runs in the body type R (FP32 on the mixed path, FP64
// otherwise); results are stored in FP64.
#include "rod_internal.h"
#include "rod_math.h"

namespace rodmx {

template <class R> __device__ __forceinline__ R atan2_(R y, R x);
template <> __device__ __forceinline__ float atan2_(float y, float x) { return atan2f(y, x); }
template <> __device__ __forceinline__ double atan2_(double y, double x) { return atan2(y, x); }
template <class R> __device__ __forceinline__ R sqrt_(R a);
template <> __device__ __forceinline__ float sqrt_(float a) { return sqrtf(a); }
template <> __device__ __forceinline__ double sqrt_(double a) { return sqrt(a); }

template <class R>
__device__ __forceinline__ void bond_one(V3<double> x1, V3<double> x2, Q4<double> q1,
                                         Q4<double> q2, V3<double> rref, double r0,
                                         const double* __restrict__ K4, V3<double>& Fo,
                                         V3<double>& Tso, V3<double>& Tbto, double* e) {
  // ---- FP64 head
  const V3<double> rf = x2 - x1;
  if (qdot(q1, q2) < 0.0) q2 = qscale(-1.0, q2);        // short arc
  const Q4<double> qc = qnormalize(qadd(q1, q2));        // central frame (spherical midpoint)
  const V3<double> rho = qrot_inv(qc, rf);               // r_f seen from C
  const double r = sqrt(dot(rho, rho));
  const double dr = r - r0;
  const V3<double> rhat = (1.0 / r) * rho;
  const V3<double> rih = (1.0 / r0) * rref;
  const V3<double> del = rhat - rih;                     // small for a near-reference bond
  const Q4<double> u0 = qmul(qconj(qc), q2);              // half rotation C -> 2
  Q4<double> m;                                          // z of C onto r_f-hat (shortest arc)
  if (1.0 + rhat.z > 1e-12) m = qnormalize(Q4<double>{1.0 + rhat.z, -rhat.y, rhat.x, 0.0});
  else m = Q4<double>{0.0, 1.0, 0.0, 0.0};
  const double r0inv = 1.0 / r0;
  const double Kr = K4[0] * r0inv, Ks = K4[1] * r0inv * r0inv * r0inv;
  const double Kt = K4[2] * r0inv, Kb = K4[3] * r0inv;

  // ---- body in R
  const V3<R> rh = cvt<R>(rhat);
  const V3<R> ri = cvt<R>(rih);
  const V3<R> c = cross(ri, cvt<R>(del));                // = r_i^ x r_f^ (r_i^ x r_i^ = 0)
  const R sigma = sqrt_(dot(c, c));
  const R cg = dot(ri, rh);
  const R gamma = atan2_(sigma, cg);                     // shear angle
  const R g = sigma > R(0) ? gamma / sigma : R(1) / cg;  // gamma / |c|, with its limit at 0
  const R rR = (R)r;
  V3<R> f = (R)(Kr * dr) * rh + (R(Ks) * rR * g) * cross(c, rh);    // f_r + f_s in C
  const V3<R> ts = (R(0.5) * R(Ks) * rR * rR * g) * c;              // tau_s in C

  // u = m* u0 m: same scalar part, vector part rotated by m*.
  const Q4<R> mR = cvtq<R>(m);
  const V3<R> uv = qrot_inv(mR, V3<R>{(R)u0.x, (R)u0.y, (R)u0.z});
  const Q4<R> u{(R)u0.w, uv.x, uv.y, uv.z};
  // Bend before twist: u = t2 b2 with t2 the twist about z; t1 = t2*.
  const R tn = sqrt_(u.w * u.w + u.z * u.z);
  const Q4<R> t2{u.w / tn, R(0), R(0), u.z / tn};
  const R psi = R(4) * atan2_(u.z, u.w);                 // psi2 - psi1
  // b = b2 b1* with b2 = t2* u and b1 = t2 u*, i.e. b = t2* u u t2*.
  Q4<R> b = qmul(qmul(qconj(t2), qmul(u, u)), qconj(t2));
  if (b.w < R(0)) b = qscale(R(-1), b);
  const V3<R> bv{b.x, b.y, b.z};
  const R bn = sqrt_(dot(bv, bv));
  const R theta = R(2) * atan2_(bn, b.w);
  const R fac = bn > R(0) ? theta / bn : R(2) / b.w;
  const V3<R> tbt{R(Kb) * fac * bv.x, R(Kb) * fac * bv.y, R(Kb) * fac * bv.z + R(Kt) * psi};

  // Back to the global frame.
  const Q4<R> qcR = cvtq<R>(qc);
  Fo = cvt<double>(qrot(qcR, f));
  Tso = cvt<double>(qrot(qcR, ts));
  Tbto = cvt<double>(qrot(qcR, qrot(mR, tbt)));
  if (e) {
    e[0] = 0.5 * Kr * dr * dr;
    e[1] = 0.5 * Ks * r * r * (double)gamma * (double)gamma;
    e[2] = 0.5 * Kt * (double)psi * (double)psi;
    e[3] = 0.5 * Kb * (double)theta * (double)theta;
  }
}

template <class R>
__global__ __launch_bounds__(256) void k_bond(Dev d, int want_energy) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long N = d.n;
  if (k >= N || !(d.bflags[k] & 1)) return;
  V3<double> F, Ts, Tbt;
  double e[4];
  bond_one<R>(ld3(d.x, N, k), ld3(d.x, N, k + 1), ld4(d.q, N, k), ld4(d.q, N, k + 1),
              V3<double>{d.bref[k], d.bref[N + k], d.bref[2 * N + k]}, d.bref[3 * N + k],
              d.rodK + 4 * d.rod[k], F, Ts, Tbt, want_energy ? e : nullptr);
  st3(d.bF, N, k, F);
  st3(d.bTs, N, k, Ts);
  st3(d.bTbt, N, k, Tbt);
  if (want_energy)
    for (int t = 0; t < 4; ++t) d.bE[t * N + k] = e[t];
}

hipError_t launch_bond(const Dev& d, int precision, int want_energy, hipStream_t s) {
  const int bs = particle_block(d.n);
  dim3 grid((unsigned)((d.n + bs - 1) / bs));
  if (precision == 1)
    hipLaunchKernelGGL(k_bond<float>, grid, dim3(bs), 0, s, d, want_energy);
  else
    hipLaunchKernelGGL(k_bond<double>, grid, dim3(bs), 0, s, d, want_energy);
  return hipGetLastError();
}

}  // namespace rodmx
