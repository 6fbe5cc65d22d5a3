// One co-rotational bond (main text eq:bpm-fr, eq:bpm-fst, eq:bpm-tst,
// eq:bpm-tb, eq:bpm-tt, eq:bpm-vector; SI "Symmetric rotational decomposition"),
// generic over the head type H (quantities that cancel) and the body type R.
// The forward kernels use <double, double> (FP64 path) and <double, float>
// (mixed path); the reverse pass differentiates <Dual, Dual>, the very same code.
#pragma once
#include "rod_math.h"

namespace rodmx {

template <class R> __device__ __forceinline__ R atan2_(R y, R x);
template <> __device__ __forceinline__ float atan2_(float y, float x) { return atan2f(y, x); }
template <> __device__ __forceinline__ double atan2_(double y, double x) { return atan2(y, x); }
template <class R> __device__ __forceinline__ R sqrt_(R a);
template <> __device__ __forceinline__ float sqrt_(float a) { return sqrtf(a); }
template <> __device__ __forceinline__ double sqrt_(double a) { return sqrt(a); }

// Bond damping of one evaluation (Methods "Damping"): the damping factors,
// the measures of the previous time level (shear angle, twist, bend vector in
// C'; valid only with `rates`, none before the first evaluation), this level's
// measures (written), the relative velocity v2 - v1 and 1 / dt. Held by value
// (no pointers into it), so that it stays in registers.
struct BondDamp {
  double gr, gs, gt, gb;
  bool rates;
  double hprev[5];
  double hnow[5];
  V3<double> dv;
  double idt;
};

template <class H, class R, bool DAMP = false>
__device__ __forceinline__ void bond_one(V3<H> x1, V3<H> x2, Q4<H> q1, Q4<H> q2, V3<double> rref,
                                         double r0, const double* __restrict__ K4, V3<H>& Fo,
                                         V3<H>& Tso, V3<H>& Tbto, double* e,
                                         BondDamp* dm = nullptr) {
  // ---- FP64 head
  const V3<H> rf = x2 - x1;
  if (qdot(q1, q2) < 0.0) q2 = qscale(H(-1.0), q2);     // short arc
  const Q4<H> qc = qnormalize(qadd(q1, q2));             // central frame (spherical midpoint)
  const V3<H> rho = qrot_inv(qc, rf);                    // r_f seen from C
  const H r = sqrt(dot(rho, rho));
  const H dr = r - r0;
  const V3<H> rhat = (H(1.0) / r) * rho;
  const V3<H> rih{H(rref.x / r0), H(rref.y / r0), H(rref.z / r0)};
  const V3<H> del = rhat - rih;                          // small for a near-reference bond
  const Q4<H> u0 = qmul(qconj(qc), q2);                  // half rotation C -> 2
  Q4<H> m;                                               // z of C onto r_f-hat (shortest arc)
  if (H(1.0) + rhat.z > 1e-12) m = qnormalize(Q4<H>{H(1.0) + rhat.z, -rhat.y, rhat.x, H(0.0)});
  else m = Q4<H>{H(0.0), H(1.0), H(0.0), H(0.0)};
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
  V3<R> f;
  V3<R> ts;
  if constexpr (!DAMP) {
    f = (R)(H(Kr) * dr) * rh + (R(Ks) * rR * g) * cross(c, rh);  // f_r + f_s in C
    ts = (R(0.5) * R(Ks) * rR * rR * g) * c;                     // tau_s in C
  } else {
    // radial: + g_r (v2 - v1) . r_f-hat, the relative velocity seen from C;
    // shear: K_s gamma becomes K_s gamma + g_s gamma-dot (no term where s-hat is
    // undefined, sigma = 0)
    const H frad = H(Kr) * dr + H(dm->gr) * dot(qrot_inv(qc, V3<H>{dm->dv.x, dm->dv.y, dm->dv.z}), rhat);
    R ks = R(Ks) * g;
    if (dm->rates && sigma > R(0))
      ks = ks + R(dm->gs) * (R)(((double)gamma - dm->hprev[0]) * dm->idt) / sigma;
    f = (R)frad * rh + (rR * ks) * cross(c, rh);
    ts = (R(0.5) * rR * rR * ks) * c;
  }

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
  V3<R> tbt{R(Kb) * fac * bv.x, R(Kb) * fac * bv.y, R(Kb) * fac * bv.z + R(Kt) * psi};
  if constexpr (DAMP) {
    // twist and bend: + g_t psi-dot (the change taken modulo 2 pi) and
    // + g_b theta-dot per component in C'
    const double th[3] = {(double)(fac * bv.x), (double)(fac * bv.y), (double)(fac * bv.z)};
    if (dm->rates) {
      const double twopi = 6.28318530717958647692;
      double dpsi = (double)psi - dm->hprev[1];
      dpsi -= twopi * rint(dpsi / twopi);
      tbt = tbt + V3<R>{(R)(dm->gb * (th[0] - dm->hprev[2]) * dm->idt),
                        (R)(dm->gb * (th[1] - dm->hprev[3]) * dm->idt),
                        (R)(dm->gb * (th[2] - dm->hprev[4]) * dm->idt + dm->gt * dpsi * dm->idt)};
    }
    dm->hnow[0] = (double)gamma;
    dm->hnow[1] = (double)psi;
    dm->hnow[2] = th[0]; dm->hnow[3] = th[1]; dm->hnow[4] = th[2];
  }

  // Back to the global frame.
  const Q4<R> qcR = cvtq<R>(qc);
  Fo = cvt<H>(qrot(qcR, f));
  Tso = cvt<H>(qrot(qcR, ts));
  Tbto = cvt<H>(qrot(qcR, qrot(mR, tbt)));
  if (e) {
    const double rd = (double)r, drd = (double)dr;
    e[0] = 0.5 * Kr * drd * drd;
    e[1] = 0.5 * Ks * rd * rd * (double)gamma * (double)gamma;
    e[2] = 0.5 * Kt * (double)psi * (double)psi;
    e[3] = 0.5 * Kb * (double)theta * (double)theta;
  }
}

}  // namespace rodmx
