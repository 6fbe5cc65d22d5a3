// Bond forces and torques of the co-rotational bond between consecutive
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
#pragma once
#include "rod_internal.h"
#include "bond_core.h"

namespace rodmx {

// Bond (k, k+1) if particle k has one; energies only when asked.
template <class R>
__device__ __forceinline__ void bond_thread(const Dev& d, long k, int want_energy) {
  const long N = d.n;
  if (k >= d.i_hi || !(d.bflags[k] & 1)) return;
  V3<double> F, Ts, Tbt;
  double e[4];
  bond_one<double, R>(ld3(d.x, N, k), ld3(d.x, N, k + 1), ld4(d.q, N, k), ld4(d.q, N, k + 1),
                      V3<double>{d.bref[k], d.bref[N + k], d.bref[2 * N + k]}, d.bref[3 * N + k],
                      d.rodK + 4 * d.rod[k], F, Ts, Tbt, want_energy ? e : nullptr);
  st3(d.bF, N, k, F);
  st3(d.bTs, N, k, Ts);
  st3(d.bTbt, N, k, Tbt);
  if (want_energy)
    for (int t = 0; t < 4; ++t) d.bE[t * N + k] = e[t];
}

}  // namespace rodmx
