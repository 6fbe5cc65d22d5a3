// All-pairs dipole-dipole kernel (Methods, "Magnetic interactions").
//
// For every particle i and every other particle j of the same member, with
// r = x_i - x_j, a = m_i.r, b = m_j.r, c = m_i.m_j and s = 3 / r^5:
//   F_i += s [ (c - 5 a b / r^2) r + b m_i + a m_j ]          (= -dU_ij/dx_i)
//   B_i += s b r - m_j / r^3                                  (field of j at x_i)
// and both are scaled by mu0/4pi at the end. The torque m_i x B_i is formed by
// the particle kernel. The m_i term is accumulated as the scalar sum of s b.
//
// Layout. A work item is a block of 64 consecutive i of one member (one i per
// lane) against a j range of the same member. The four waves of a workgroup
// split every staged j tile of 256 four ways and are reduced through LDS at
// the end. Tiles are read from LDS as wavefront-uniform broadcasts. Position
// differences are taken in FP64 and rounded once; on the mixed path the pair
// arithmetic and the per-tile sums are FP32 and each tile is flushed into FP64
// accumulators. When a member's j range is split over several work items,
// each writes its own FP64 partial slot, and the particle kernel adds the
// slots in slot order (deterministic, no atomics, no cross-workgroup fences).
#include "rod_internal.h"
#include "rod_math.h"

namespace rodmx {

template <class R> __device__ __forceinline__ R rsq(R a);
template <> __device__ __forceinline__ float rsq(float a) { return __builtin_amdgcn_rsqf(a); }
template <> __device__ __forceinline__ double rsq(double a) { return 1.0 / sqrt(a); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

constexpr int TJ = 256;   // j tile staged per workgroup
constexpr int JW = 64;    // j entries of a tile handled by one wave

template <class R>
struct Acc { R fx, fy, fz, fm, bx, by, bz; };

template <class R, bool SELF>
__device__ __forceinline__ void tile_pairs(int jb, int je, int jbase, int i, double xi, double yi,
                                           double zi, R mix, R miy, R miz, const double* sx,
                                           const double* sy, const double* sz, const R* smx,
                                           const R* smy, const R* smz, Acc<R>& A) {
#pragma unroll 4
  for (int jj = jb; jj < je; ++jj) {
    const R dx = (R)(xi - sx[jj]), dy = (R)(yi - sy[jj]), dz = (R)(zi - sz[jj]);
    const R mjx = smx[jj], mjy = smy[jj], mjz = smz[jj];
    const R r2 = fma_(dz, dz, fma_(dy, dy, dx * dx));
    R rinv = rsq(r2);
    if (SELF) rinv = (jbase + jj == i) ? R(0) : rinv;   // the pair (i, i) contributes nothing
    const R rinv2 = rinv * rinv;
    const R rinv3 = rinv2 * rinv;
    const R s = (R(3) * rinv3) * rinv2;
    const R a = fma_(miz, dz, fma_(miy, dy, mix * dx));
    const R b = fma_(mjz, dz, fma_(mjy, dy, mjx * dx));
    const R c = fma_(miz, mjz, fma_(miy, mjy, mix * mjx));
    const R sb = s * b, sa = s * a;
    const R al = fma_((sb * a) * rinv2, R(-5), s * c);
    A.fx = fma_(sa, mjx, fma_(al, dx, A.fx));
    A.fy = fma_(sa, mjy, fma_(al, dy, A.fy));
    A.fz = fma_(sa, mjz, fma_(al, dz, A.fz));
    A.fm += sb;
    A.bx = fma_(-rinv3, mjx, fma_(sb, dx, A.bx));
    A.by = fma_(-rinv3, mjy, fma_(sb, dy, A.by));
    A.bz = fma_(-rinv3, mjz, fma_(sb, dz, A.bz));
  }
}

template <class R>
__global__ __launch_bounds__(256) void k_dipole(Dev d, const DipWork* __restrict__ work) {
  __shared__ double sx[TJ], sy[TJ], sz[TJ];
  __shared__ R smx[TJ], smy[TJ], smz[TJ];
  __shared__ double red[4][7][64];
  const DipWork wk = work[blockIdx.x];
  const long N = d.n;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int i = wk.i0 + lane;
  const bool act = i < wk.i1;
  const R* mu;
  if constexpr (sizeof(R) == 4) mu = (const R*)d.muf;
  else mu = (const R*)d.mu;
  double xi = 0, yi = 0, zi = 0;
  R mix = 0, miy = 0, miz = 0;
  if (act) {
    xi = d.x[i]; yi = d.x[N + i]; zi = d.x[2 * N + i];
    mix = mu[i]; miy = mu[N + i]; miz = mu[2 * N + i];
  }
  double F[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int t0 = wk.j0; t0 < wk.j1; t0 += TJ) {
    const int jn = min(TJ, wk.j1 - t0);
    if ((int)threadIdx.x < jn) {
      const int j = t0 + threadIdx.x;
      sx[threadIdx.x] = d.x[j]; sy[threadIdx.x] = d.x[N + j]; sz[threadIdx.x] = d.x[2 * N + j];
      smx[threadIdx.x] = mu[j]; smy[threadIdx.x] = mu[N + j]; smz[threadIdx.x] = mu[2 * N + j];
    }
    __syncthreads();
    const int jb = wave * JW, je = min(jb + JW, jn);
    if (jb < je) {
      Acc<R> A{0, 0, 0, 0, 0, 0, 0};
      const bool self = (t0 + jb < wk.i1) && (t0 + je > wk.i0);  // sub-tile may contain i
      if (self)
        tile_pairs<R, true>(jb, je, t0, i, xi, yi, zi, mix, miy, miz, sx, sy, sz, smx, smy, smz, A);
      else
        tile_pairs<R, false>(jb, je, t0, i, xi, yi, zi, mix, miy, miz, sx, sy, sz, smx, smy, smz, A);
      F[0] += A.fx; F[1] += A.fy; F[2] += A.fz; F[3] += A.fm;
      F[4] += A.bx; F[5] += A.by; F[6] += A.bz;
    }
    __syncthreads();
  }
  // Sum the four waves in wave order and write this work item's slot.
  for (int k = 0; k < 7; ++k) red[wave][k][lane] = F[k];
  __syncthreads();
  if (wave == 0 && act) {
    for (int k = 0; k < 7; ++k)
      F[k] = ((red[0][k][lane] + red[1][k][lane]) + red[2][k][lane]) + red[3][k][lane];
    const double C = d.C;
    double* p = d.dpart + (long)wk.slot * 6 * N;
    p[i] = C * (F[0] + F[3] * (double)mix);
    p[N + i] = C * (F[1] + F[3] * (double)miy);
    p[2 * N + i] = C * (F[2] + F[3] * (double)miz);
    p[3 * N + i] = C * F[4];
    p[4 * N + i] = C * F[5];
    p[5 * N + i] = C * F[6];
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
