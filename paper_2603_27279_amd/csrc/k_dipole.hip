// All-pairs dipole-dipole kernel (Methods, "Magnetic interactions").
//
// For every particle i and every other particle j of the same member, with
// r = x_i - x_j, a = m_i.r, b = m_j.r, c = m_i.m_j and s = 3 / r^5:
//   F_i += s [ (c - 5 a b / r^2) r + b m_i + a m_j ]          (= -dU_ij/dx_i)
//   B_i += s b r - m_j / r^3                                  (field of j at x_i)
// and the caller scales both by mu0/4pi. The torque m_i x B_i is formed by the
// particle kernel. The m_i term is accumulated as the scalar sum of s b and
// multiplied by m_i once per tile.
//
// Layout. Work items pair a block of 256 consecutive i of one member (one i
// per lane) with a j range of the same member; each work item writes its sums
// to its own FP64 partial slot, and the particle kernel adds the slots in a
// fixed order (deterministic, no atomics). j tiles of 256 are staged in LDS and
// read as wavefront-uniform broadcasts. Position differences are taken in FP64
// and rounded once; on the mixed path the pair arithmetic and the per-tile
// sums are FP32 and every tile is flushed into FP64 accumulators.
#include "rod_internal.h"
#include "rod_math.h"

namespace rodmx {

template <class R> __device__ __forceinline__ R rsq(R a);
template <> __device__ __forceinline__ float rsq(float a) { return __builtin_amdgcn_rsqf(a); }
template <> __device__ __forceinline__ double rsq(double a) { return 1.0 / sqrt(a); }

constexpr int TJ = 256;

template <class R, bool SELF>
__device__ __forceinline__ void tile_pairs(int jn, int jbase, int i, double xi, double yi, double zi,
                                           R mix, R miy, R miz, const double* sx, const double* sy,
                                           const double* sz, const R* smx, const R* smy,
                                           const R* smz, R& fx, R& fy, R& fz, R& fm, R& bx,
                                           R& by, R& bz) {
#pragma unroll 4
  for (int jj = 0; jj < jn; ++jj) {
    const R dx = (R)(xi - sx[jj]), dy = (R)(yi - sy[jj]), dz = (R)(zi - sz[jj]);
    const R mjx = smx[jj], mjy = smy[jj], mjz = smz[jj];
    const R r2 = dx * dx + dy * dy + dz * dz;
    R rinv = rsq(r2);
    if (SELF) rinv = (jbase + jj == i) ? R(0) : rinv;
    const R rinv2 = rinv * rinv;
    const R rinv3 = rinv2 * rinv;
    const R s = R(3) * rinv3 * rinv2;
    const R a = mix * dx + miy * dy + miz * dz;
    const R b = mjx * dx + mjy * dy + mjz * dz;
    const R c = mix * mjx + miy * mjy + miz * mjz;
    const R sb = s * b;
    const R sa = s * a;
    const R al = s * c - R(5) * (sb * a) * rinv2;
    fx += al * dx + sa * mjx;
    fy += al * dy + sa * mjy;
    fz += al * dz + sa * mjz;
    fm += sb;
    bx += sb * dx - rinv3 * mjx;
    by += sb * dy - rinv3 * mjy;
    bz += sb * dz - rinv3 * mjz;
  }
}

template <class R>
__global__ __launch_bounds__(256) void k_dipole(Dev d, const DipWork* __restrict__ work) {
  __shared__ double sx[TJ], sy[TJ], sz[TJ];
  __shared__ R smx[TJ], smy[TJ], smz[TJ];
  const DipWork wk = work[blockIdx.x];
  const long N = d.n;
  const int i = wk.i0 + threadIdx.x;
  const bool act = i < wk.i1;
  const R* mu = nullptr;
  if constexpr (sizeof(R) == 4) mu = (const R*)d.muf;
  else mu = (const R*)d.mu;
  double xi = 0, yi = 0, zi = 0;
  R mix = 0, miy = 0, miz = 0;
  if (act) {
    xi = d.x[i]; yi = d.x[N + i]; zi = d.x[2 * N + i];
    mix = mu[i]; miy = mu[N + i]; miz = mu[2 * N + i];
  }
  double Fx = 0, Fy = 0, Fz = 0, Fm = 0, Bx = 0, By = 0, Bz = 0;
  for (int t0 = wk.j0; t0 < wk.j1; t0 += TJ) {
    const int jn = min(TJ, wk.j1 - t0);
    const int j = t0 + threadIdx.x;
    if ((int)threadIdx.x < jn) {
      sx[threadIdx.x] = d.x[j]; sy[threadIdx.x] = d.x[N + j]; sz[threadIdx.x] = d.x[2 * N + j];
      smx[threadIdx.x] = mu[j]; smy[threadIdx.x] = mu[N + j]; smz[threadIdx.x] = mu[2 * N + j];
    }
    __syncthreads();
    R fx = 0, fy = 0, fz = 0, fm = 0, bx = 0, by = 0, bz = 0;
    const bool self = (t0 < wk.i1) && (t0 + jn > wk.i0);  // tile may contain i itself
    if (self)
      tile_pairs<R, true>(jn, t0, i, xi, yi, zi, mix, miy, miz, sx, sy, sz, smx, smy, smz, fx, fy,
                          fz, fm, bx, by, bz);
    else
      tile_pairs<R, false>(jn, t0, i, xi, yi, zi, mix, miy, miz, sx, sy, sz, smx, smy, smz, fx,
                           fy, fz, fm, bx, by, bz);
    Fx += fx; Fy += fy; Fz += fz; Fm += fm; Bx += bx; By += by; Bz += bz;
    __syncthreads();
  }
  if (act) {
    double* p = d.dpart + (long)wk.slot * 6 * N;
    const double C = d.C;
    p[i] = C * (Fx + Fm * (double)mix);
    p[N + i] = C * (Fy + Fm * (double)miy);
    p[2 * N + i] = C * (Fz + Fm * (double)miz);
    p[3 * N + i] = C * Bx;
    p[4 * N + i] = C * By;
    p[5 * N + i] = C * Bz;
  }
}

hipError_t launch_dipole(const Dev& d, int precision, const DipWork* work, int nwork,
                         hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (precision == 1)
    hipLaunchKernelGGL(k_dipole<float>, dim3(nwork), dim3(256), 0, s, d, work);
  else
    hipLaunchKernelGGL(k_dipole<double>, dim3(nwork), dim3(256), 0, s, d, work);
  return hipGetLastError();
}

}  // namespace rodmx
