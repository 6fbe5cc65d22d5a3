// Exact, order-free sums of contact terms (used by the contact kernels and the
// reverse pass of the contact force).
#pragma once
#include "rod_internal.h"
#include "rod_math.h"

namespace rodmx {

// Every pair term t of a contact sum is multiplied by the power of two 2^s of its
// quantity (force, torque, energy: Dev::fix_scale, chosen on the host so that a
// bound B on one pair's term becomes 2^80, i.e. a quantum of B 2^-80), rounded
// once to an integer, and added as a 128-bit two's-complement integer. Integer
// addition is exact, so a sum does not depend on the order in which the search
// meets its pairs, and each term is rounded by at most B 2^-81: every term down
// to 2^-40 B keeps FP64's 1e-12 relative bar, whatever the contact stiffness or
// the unit system. A term of 2^108 quanta or more (2^28 B), or a non-finite one,
// raises the range flag (ROD_E_OVERFLOW at rod_sync) and is dropped; below
// that, 2^18 terms still fit in 127 bits.
struct Fix128 { unsigned long long lo; long long hi; };
struct Fix3 { Fix128 x, y, z; };

constexpr double FIX_TERM_MAX = 0x1p108;

__device__ __forceinline__ Fix128 fix_neg(Fix128 v) {
  v.lo = ~v.lo + 1ull;
  v.hi = ~v.hi + (v.lo == 0ull ? 1 : 0);
  return v;
}

// The integer nearest u (u = t 2^s, already scaled).
__device__ __forceinline__ Fix128 fix_of(double u, unsigned* range_flag) {
  const double a = fabs(u);
  if (!(a < FIX_TERM_MAX)) {
    atomicOr(range_flag, 1u);
    return Fix128{0ull, 0};
  }
  const double h = floor(a * 0x1p-64);  // exact: a power-of-two scaling
  const double rem = a - h * 0x1p64;    // exact: the bits of a below 2^64
  Fix128 v{__double2ull_rn(rem), (long long)h};
  return u < 0.0 ? fix_neg(v) : v;
}

__device__ __forceinline__ void fix_add(Fix128& acc, Fix128 t) {
  acc.lo += t.lo;
  acc.hi += t.hi + (acc.lo < t.lo ? 1 : 0);
}

__device__ __forceinline__ void fix_add(Fix128& acc, double t, double scale, unsigned* flag) {
  fix_add(acc, fix_of(t * scale, flag));
}

__device__ __forceinline__ void fix_add(Fix3& acc, V3<double> t, double scale, unsigned* flag) {
  fix_add(acc.x, t.x, scale, flag);
  fix_add(acc.y, t.y, scale, flag);
  fix_add(acc.z, t.z, scale, flag);
}

// The sum as a double (rounded once more), in the quantity's units.
__device__ __forceinline__ double fix_value(Fix128 v, double inv_scale) {
  const bool neg = v.hi < 0;
  if (neg) v = fix_neg(v);
  const double r = ((double)v.hi * 0x1p64 + (double)v.lo) * inv_scale;
  return neg ? -r : r;
}
__device__ __forceinline__ V3<double> fix_value(const Fix3& v, double inv_scale) {
  return V3<double>{fix_value(v.x, inv_scale), fix_value(v.y, inv_scale),
                    fix_value(v.z, inv_scale)};
}

// Sum over the 32 lanes of each half wave (integer adds: exact, any order).
__device__ __forceinline__ Fix128 half_sum(Fix128 v) {
  for (int o = 16; o > 0; o >>= 1) {
    const Fix128 w{(unsigned long long)__shfl_xor((long long)v.lo, o, 32),
                   __shfl_xor(v.hi, o, 32)};
    fix_add(v, w);
  }
  return v;
}
__device__ __forceinline__ Fix3 half_sum(Fix3 v) {
  return Fix3{half_sum(v.x), half_sum(v.y), half_sum(v.z)};
}

}  // namespace rodmx
