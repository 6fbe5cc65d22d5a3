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
// With bond damping (d.bdamp set) the rates are taken against the measures
// of the previous level, hist[(L - 1) & 1] (from level hist_from on), and this
// level's go to hist[L & 1] when the evaluation records them, L being the
// level under evaluation.
// ALL: every particle below i_hi is evaluated with its successor, whether or
// not the two are bonded, so that no load waits for the bond flag (the
// standalone bond kernel); the particle kernels read a bond's outputs only
// where the flag is set, and what the last particle of a rod stores (its
// partner is the next rod's first, or itself at the end of the system) is never
// read. Without ALL the flag is tested first: the fused force kernel keeps the
// registers of its dipole work items that way.
template <class R, bool ALL = false>
__device__ __forceinline__ void bond_thread(const Dev& d, long k, int want_energy) {
  const long N = d.n;
  if (k >= d.i_hi) return;
  if (!ALL && !(d.bflags[k] & 1)) return;
  const long k2 = ALL && k + 1 >= N ? k : k + 1;
  V3<double> F, Ts, Tbt;
  double e[4];
  if (d.bdamp) {
    const long long L = d.step[d.lc];
    const int rod = d.rod[k];
    BondDamp dm;
    dm.gr = d.bdamp[4 * rod]; dm.gs = d.bdamp[4 * rod + 1];
    dm.gt = d.bdamp[4 * rod + 2]; dm.gb = d.bdamp[4 * rod + 3];
    const double* hprev = d.hist + (long)((L - 1) & 1) * 5 * N;
    for (int c = 0; c < 5; ++c) dm.hprev[c] = hprev[c * N + k];
    dm.rates = L >= d.hist_from;
    dm.dv = ld3(d.v, N, k2) - ld3(d.v, N, k);
    dm.idt = 1.0 / d.dt;
    bond_one<double, R, true>(ld3(d.x, N, k), ld3(d.x, N, k2), ld4(d.q, N, k), ld4(d.q, N, k2),
                              V3<double>{d.bref[k], d.bref[N + k], d.bref[2 * N + k]},
                              d.bref[3 * N + k], d.rodK + 4 * rod, F, Ts, Tbt,
                              want_energy ? e : nullptr, &dm);
    if (d.hist_write) {
      double* hnow = d.hist + (long)(L & 1) * 5 * N;
      for (int c = 0; c < 5; ++c) hnow[c * N + k] = dm.hnow[c];
    }
  } else {
    bond_one<double, R>(ld3(d.x, N, k), ld3(d.x, N, k2), ld4(d.q, N, k), ld4(d.q, N, k2),
                        V3<double>{d.bref[k], d.bref[N + k], d.bref[2 * N + k]},
                        d.bref[3 * N + k], d.rodK + 4 * d.rod[k], F, Ts, Tbt,
                        want_energy ? e : nullptr);
  }
  st3(d.bF, N, k, F);
  st3(d.bTs, N, k, Ts);
  st3(d.bTbt, N, k, Tbt);
  if (want_energy)
    for (int t = 0; t < 4; ++t) d.bE[t * N + k] = e[t];
}

}  // namespace rodmx
