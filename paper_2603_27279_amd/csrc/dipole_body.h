// All-pairs dipole-dipole sums (Methods, "Magnetic interactions").
//
// For every particle i and every other particle j of the same member, with
// r = x_i - x_j, a = m_i.r, b = m_j.r, c = m_i.m_j and s = 1 / r^5:
//   F_i += 3 s [ (c - 5 a b / r^2) r + b m_i + a m_j ]        (= -dU_ij/dx_i)
//   B_i += 3 s b r - m_j / r^3                                (field of j at x_i)
// and both are scaled by mu0/4pi at the end. The factor 3 is applied once per
// particle, so the pair sums are kept as F/3 and as the two parts of B; the
// torque m_i x B_i is formed by the particle kernel. The m_i term of F is
// accumulated as the scalar sum of s b.
//
// Layout. A work item is a block of 64 consecutive i of one member (one i per
// lane) against a j range of the same member. The four waves of a workgroup
// split every staged j tile of TJ sources four ways and are reduced through LDS at
// the end. Tiles are read from LDS as wavefront-uniform broadcasts. Position
// differences are taken in FP64 and rounded once; on the mixed path the pair
// arithmetic and the per-tile sums are FP32 and each tile is flushed into FP64
// accumulators. When a member's j range is split over several work items,
// each writes its own FP64 partial slot, and the particle kernel adds the
// slots in slot order (deterministic, no atomics, no cross-workgroup fences).
#pragma once
#include "rod_internal.h"
#include "rod_math.h"

namespace rodmx {

template <class R> __device__ __forceinline__ R rsq(R a);
template <> __device__ __forceinline__ float rsq(float a) { return __builtin_amdgcn_rsqf(a); }
template <> __device__ __forceinline__ double rsq(double a) { return rsqrt_nr(a); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// A value the compiler must treat as held per lane (a vector register). Used
// for the constant -5, which would otherwise be a literal operand, and for the
// tile index, so that LDS addresses are formed in vector registers once per
// unrolled step instead of being copied from scalar registers per read.
__device__ __forceinline__ int lane_value(int v) {
  int r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
  return r;
}
__device__ __forceinline__ float lane_value(float v) {
  float r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
  return r;
}

__device__ __forceinline__ float minus5(float) { return lane_value(-5.0f); }
__device__ __forceinline__ double minus5(double) { return -5.0; }

constexpr int TJ = 512;   // j tile staged per workgroup (a quarter per wave)

// Pair sums: f = sum s[(c - 5ab/r^2) r + a m_j], fm = sum s b,
// bs = sum s b r, bm = sum m_j / r^3.
template <class R>
struct Acc { R fx, fy, fz, fm, bsx, bsy, bsz, bmx, bmy, bmz; };
constexpr int NACC = 10;

// Add the contribution of source j (moment mj) at offset (dx, dy, dz) to target i.
template <class R>
__device__ __forceinline__ void pair_acc(R dx, R dy, R dz, R mjx, R mjy, R mjz, R mix, R miy,
                                         R miz, R rinv, R m5, Acc<R>& A) {
  const R rinv2 = rinv * rinv;
  const R rinv3 = rinv2 * rinv;
  const R s = rinv3 * rinv2;
  const R a = fma_(miz, dz, fma_(miy, dy, mix * dx));
  const R b = fma_(mjz, dz, fma_(mjy, dy, mjx * dx));
  const R c = fma_(miz, mjz, fma_(miy, mjy, mix * mjx));
  const R sb = s * b, sa = s * a;
  const R al = fma_((sb * a) * rinv2, m5, s * c);
  A.fx = fma_(sa, mjx, fma_(al, dx, A.fx));
  A.fy = fma_(sa, mjy, fma_(al, dy, A.fy));
  A.fz = fma_(sa, mjz, fma_(al, dz, A.fz));
  A.fm += sb;
  A.bsx = fma_(sb, dx, A.bsx);
  A.bsy = fma_(sb, dy, A.bsy);
  A.bsz = fma_(sb, dz, A.bsz);
  A.bmx = fma_(rinv3, mjx, A.bmx);
  A.bmy = fma_(rinv3, mjy, A.bmy);
  A.bmz = fma_(rinv3, mjz, A.bmz);
}

template <class R>
__device__ __forceinline__ void acc_add(Acc<R>& A, const Acc<R>& B) {
  A.fx += B.fx; A.fy += B.fy; A.fz += B.fz; A.fm += B.fm;
  A.bsx += B.bsx; A.bsy += B.bsy; A.bsz += B.bsz;
  A.bmx += B.bmx; A.bmy += B.bmy; A.bmz += B.bmz;
}

// Slot values of one target from its pair sums (FP64): force and field, stored
// in the work item's slot. The mixed path stores them in FP32: they are sums of
// FP32 pair terms, and the particle kernel adds the slots in FP64; this halves
// the bytes and registers of that sum, whose loads then travel in one batch.
template <class R> __device__ __forceinline__ R* slot_base(const Dev& d, int slot);
template <> __device__ __forceinline__ float* slot_base(const Dev& d, int slot) {
  return d.dslotf + (long)slot * 6 * d.n;
}
template <> __device__ __forceinline__ double* slot_base(const Dev& d, int slot) {
  return d.dpart + (long)slot * 6 * d.n;
}
template <class T>
__device__ __forceinline__ void write_slot(T* p, long N, long i, double C, const double* F,
                                           double mix, double miy, double miz) {
  const double C3 = 3.0 * C;
  p[i] = (T)(C3 * (F[0] + F[3] * mix));
  p[N + i] = (T)(C3 * (F[1] + F[3] * miy));
  p[2 * N + i] = (T)(C3 * (F[2] + F[3] * miz));
  p[3 * N + i] = (T)(C * (3.0 * F[4] - F[7]));
  p[4 * N + i] = (T)(C * (3.0 * F[5] - F[8]));
  p[5 * N + i] = (T)(C * (3.0 * F[6] - F[9]));
}

// One staged source: position (FP64) and moment, contiguous so that a single
// vector-register address with immediate offsets reaches every field.
template <class R>
struct alignas(8) Src { double x, y, z; R mx, my, mz; };

template <class R, bool SELF>
__device__ __forceinline__ void tile_pairs(int jb, int je, int jbase, int i, double xi, double yi,
                                           double zi, R mix, R miy, R miz, const Src<R>* tile,
                                           Acc<R>& A) {
  const R m5 = minus5(R(0));
  const Src<R>* p = tile + lane_value(jb);  // per-lane address: one increment per step
  // even and odd sources go to separate sums, so consecutive pairs do not wait
  // on each other's accumulation
  Acc<R> B{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int n = je - jb;
  for (int k = 0; k + 1 < n; k += 2) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const Src<R> e = p[k + u];
      const R dx = (R)(xi - e.x), dy = (R)(yi - e.y), dz = (R)(zi - e.z);
      const R r2 = fma_(dz, dz, fma_(dy, dy, dx * dx));
      R rinv = rsq(r2);
      if (SELF) rinv = (jbase + jb + k + u == i) ? R(0) : rinv;  // the pair (i, i) adds nothing
      pair_acc(dx, dy, dz, e.mx, e.my, e.mz, mix, miy, miz, rinv, m5, u ? B : A);
    }
  }
  if (n & 1) {
    const Src<R> e = p[n - 1];
    const R dx = (R)(xi - e.x), dy = (R)(yi - e.y), dz = (R)(zi - e.z);
    const R r2 = fma_(dz, dz, fma_(dy, dy, dx * dx));
    R rinv = rsq(r2);
    if (SELF) rinv = (jbase + je - 1 == i) ? R(0) : rinv;
    pair_acc(dx, dy, dz, e.mx, e.my, e.mz, mix, miy, miz, rinv, m5, A);
  }
  acc_add(A, B);
}

// Far sub-tiles (mixed path). A sub-tile is far from the wave when every
// target lies more than three half-diagonals h from the centre o of a box
// holding the sub-tile's sources (the union of the boxes of the 64-particle
// chunks it touches, written where positions were set). Then a difference is
// formed as (x_i - o) - (x_j - o), each offset taken in FP64 and rounded to
// FP32 once. Since |x_j - o| <= h and |r| > 2h, the error stays below 3 ulp of
// |r|, the size of the FP32 pair arithmetic's own error, and a pair costs three
// FP32 subtractions instead of three FP64 subtractions and conversions.
// Returns false (nothing done) when some target is near; the sub-tile then
// takes the exact path.
__device__ __forceinline__ bool far_tile_pairs(const Dev& d, int jg0, int jg1, int jb, int je,
                                               bool act, double xi, double yi, double zi,
                                               float mix, float miy, float miz,
                                               const Src<float>* tile, float4* rel,
                                               Acc<float>& A) {
  const int lane = threadIdx.x & 63;
  const double* boxes = d.dperm ? d.sbox : d.cbox;  // chunks of positions
  double lx = 1e300, ly = 1e300, lz = 1e300, hx = -1e300, hy = -1e300, hz = -1e300;
  for (int c = jg0 >> 6; c <= (jg1 - 1) >> 6; ++c) {  // every chunk the sub-tile touches
    const double* b = boxes + 6 * c;
    lx = fmin(lx, b[0]); ly = fmin(ly, b[1]); lz = fmin(lz, b[2]);
    hx = fmax(hx, b[3]); hy = fmax(hy, b[4]); hz = fmax(hz, b[5]);
  }
  const double ox = 0.5 * (lx + hx), oy = 0.5 * (ly + hy), oz = 0.5 * (lz + hz);
  const double ex = 0.5 * (hx - lx), ey = 0.5 * (hy - ly), ez = 0.5 * (hz - lz);
  const double h2 = ex * ex + ey * ey + ez * ez;
  const double tx = xi - ox, ty = yi - oy, tz = zi - oz;
  if (!__all(!act || tx * tx + ty * ty + tz * tz > 9.0 * h2)) return false;
  const int n = je - jb;
  for (int k = lane; k < n; k += 64) {
    const Src<float>& e = tile[jb + k];
    rel[k] = make_float4((float)(e.x - ox), (float)(e.y - oy), (float)(e.z - oz), 0.0f);
  }
  const float xr = (float)tx, yr = (float)ty, zr = (float)tz;
  const float m5 = minus5(0.0f);
  const float4* pr = rel + lane_value(0);
  const Src<float>* p = tile + lane_value(jb);
  Acc<float> B{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // odd sources (see tile_pairs)
  for (int k = 0; k + 1 < n; k += 2) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const float4 r = pr[k + u];
      const float dx = xr - r.x, dy = yr - r.y, dz = zr - r.z;
      const float r2 = fma_(dz, dz, fma_(dy, dy, dx * dx));
      pair_acc(dx, dy, dz, p[k + u].mx, p[k + u].my, p[k + u].mz, mix, miy, miz, rsq(r2), m5,
               u ? B : A);
    }
  }
  if (n & 1) {
    const float4 r = pr[n - 1];
    const float dx = xr - r.x, dy = yr - r.y, dz = zr - r.z;
    const float r2 = fma_(dz, dz, fma_(dy, dy, dx * dx));
    pair_acc(dx, dy, dz, p[n - 1].mx, p[n - 1].my, p[n - 1].mz, mix, miy, miz, rsq(r2), m5, A);
  }
  acc_add(A, B);
  return true;
}

// LDS of one split work item: the staged tile and the per-wave relative source
// positions of far sub-tiles, reused for the final reduction.
template <class R>
union DipSmem {
  struct {
    Src<R> tile[TJ];
    float4 rel[4][TJ / 4];
  } st;
  double red[4][NACC][64];
};

// One work item of the split layout (256 threads). Its ranges are positions:
// particles themselves, or places in the spatial order (d.dperm).
template <class R>
__device__ __forceinline__ void dipole_item(const Dev& d, const DipWork& wk, DipSmem<R>& sm) {
  Src<R>* tile = sm.st.tile;
  const long N = d.n;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int ip = wk.i0 + lane;  // target position
  const bool act = ip < wk.i1;
  const int i = act && d.dperm ? d.dperm[ip] : ip;  // target particle
  const R* mu;
  if constexpr (sizeof(R) == 4) mu = (const R*)d.muf;
  else mu = (const R*)d.mu;
  double xi = 0, yi = 0, zi = 0;
  R mix = 0, miy = 0, miz = 0;
  if (act) {
    xi = d.x[i]; yi = d.x[N + i]; zi = d.x[2 * N + i];
    mix = mu[i]; miy = mu[N + i]; miz = mu[2 * N + i];
  }
  double F[NACC] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int t0 = wk.j0; t0 < wk.j1; t0 += TJ) {
    const int jn = min(TJ, wk.j1 - t0);
    for (int t = threadIdx.x; t < jn; t += blockDim.x) {
      const int j = d.dperm ? d.dperm[t0 + t] : t0 + t;
      tile[t] = Src<R>{d.x[j], d.x[N + j], d.x[2 * N + j], mu[j], mu[N + j], mu[2 * N + j]};
    }
    __syncthreads();
    const int q = (jn + 3) >> 2;  // the four waves take equal quarters of the staged tile
    const int jb = min(wave * q, jn), je = min(jb + q, jn);
    if (jb < je) {
      Acc<R> A{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      bool far = false;
      if constexpr (sizeof(R) == 4)
        if (d.far_ok)
          far = far_tile_pairs(d, t0 + jb, t0 + je, jb, je, act, xi, yi, zi, mix, miy, miz, tile,
                               sm.st.rel[wave], A);
      const bool self = (t0 + jb < wk.i1) && (t0 + je > wk.i0);  // sub-tile may contain i
      if (far) {
      } else if (self) {  // (the pair of a position with itself adds nothing)
        tile_pairs<R, true>(jb, je, t0, ip, xi, yi, zi, mix, miy, miz, tile, A);
      } else {
        tile_pairs<R, false>(jb, je, t0, ip, xi, yi, zi, mix, miy, miz, tile, A);
      }
      F[0] += A.fx; F[1] += A.fy; F[2] += A.fz; F[3] += A.fm;
      F[4] += A.bsx; F[5] += A.bsy; F[6] += A.bsz;
      F[7] += A.bmx; F[8] += A.bmy; F[9] += A.bmz;
    }
    __syncthreads();
  }
  // Sum the four waves in wave order and write this work item's slot.
  // (the last tile pass ended with a barrier, so the tile may be overwritten)
  for (int k = 0; k < NACC; ++k) sm.red[wave][k][lane] = F[k];
  __syncthreads();
  if (wave == 0 && act) {
    for (int k = 0; k < NACC; ++k)
      F[k] = ((sm.red[0][k][lane] + sm.red[1][k][lane]) + sm.red[2][k][lane]) + sm.red[3][k][lane];
    write_slot(slot_base<R>(d, wk.slot), N, i, d.C, F, mix, miy, miz);
  }
}

// Small-member layout: a work item of up to DIP_SMALL_I consecutive targets of one
// member, one wave per target; the 64 lanes of the wave stride over the
// member's sources, four sources in flight per lane, and their sums are
// combined across lanes by a fixed xor tree. No LDS and no barriers, so these
// items share launches with any other workgroup.
template <class R>
__device__ __forceinline__ void dipole_small_item(const Dev& d, const DipWork& wk) {
  const long N = d.n;
  const int lane = threadIdx.x & 63;
  const int i = wk.i0 + (int)(threadIdx.x >> 6);
  if (i >= wk.i1) return;  // the whole wave
  const R* mu;
  if constexpr (sizeof(R) == 4) mu = (const R*)d.muf;
  else mu = (const R*)d.mu;
  const double xi = d.x[i], yi = d.x[N + i], zi = d.x[2 * N + i];
  const R mix = mu[i], miy = mu[N + i], miz = mu[2 * N + i];
  Acc<R> A{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const R m5 = minus5(R(0));
  for (int jb = wk.j0 + lane; jb < wk.j1; jb += 4 * 64) {
    double sx[4], sy[4], sz[4];
    R smx[4], smy[4], smz[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {  // loads first; out-of-range entries read source j0
      const int j = jb + 64 * u < wk.j1 ? jb + 64 * u : wk.j0;
      sx[u] = d.x[j]; sy[u] = d.x[N + j]; sz[u] = d.x[2 * N + j];
      smx[u] = mu[j]; smy[u] = mu[N + j]; smz[u] = mu[2 * N + j];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = jb + 64 * u;
      if (j >= wk.j1) break;
      const R dx = (R)(xi - sx[u]), dy = (R)(yi - sy[u]), dz = (R)(zi - sz[u]);
      const R r2 = fma_(dz, dz, fma_(dy, dy, dx * dx));
      const R rinv = (j == i) ? R(0) : rsq(r2);
      pair_acc(dx, dy, dz, smx[u], smy[u], smz[u], mix, miy, miz, rinv, m5, A);
    }
  }
  double F[NACC] = {(double)A.fx,  (double)A.fy,  (double)A.fz,  (double)A.fm,  (double)A.bsx,
                    (double)A.bsy, (double)A.bsz, (double)A.bmx, (double)A.bmy, (double)A.bmz};
#pragma unroll
  for (int k = 0; k < NACC; ++k)
    for (int o = 32; o > 0; o >>= 1) F[k] += __shfl_xor(F[k], o);
  if (lane == 0)
    write_slot(slot_base<R>(d, wk.slot), N, i, d.C, F, (double)mix, (double)miy, (double)miz);
}

}  // namespace rodmx
