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

// Add the contribution of source j (position xj, moment mj) to target i.
template <class R>
__device__ __forceinline__ void pair_acc(R dx, R dy, R dz, R mjx, R mjy, R mjz, R mix, R miy,
                                         R miz, R rinv, Acc<R>& A) {
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

template <class R, bool SELF>
__device__ __forceinline__ void tile_pairs(int jb, int je, int jbase, int i, double xi, double yi,
                                           double zi, R mix, R miy, R miz, const double* sx,
                                           const double* sy, const double* sz, const R* smx,
                                           const R* smy, const R* smz, Acc<R>& A) {
#pragma unroll 2
  for (int jj = jb; jj < je; ++jj) {
    const R dx = (R)(xi - sx[jj]), dy = (R)(yi - sy[jj]), dz = (R)(zi - sz[jj]);
    const R r2 = fma_(dz, dz, fma_(dy, dy, dx * dx));
    R rinv = rsq(r2);
    if (SELF) rinv = (jbase + jj == i) ? R(0) : rinv;   // the pair (i, i) contributes nothing
    pair_acc(dx, dy, dz, smx[jj], smy[jj], smz[jj], mix, miy, miz, rinv, A);
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

// Layout for small members: a workgroup of 1024 threads serves 16 consecutive
// i of one member; thread (il, jl) visits j = j0 + jl, j0 + jl + 64, ... of
// the member, so every member pair is spread over the whole workgroup. The
// 64 partial sums of each i are added by a fixed LDS tree. One slot.
template <class R>
__global__ __launch_bounds__(1024) void k_dipole_small(Dev d, const DipWork* __restrict__ work) {
  __shared__ double red[7][64][16];
  const DipWork wk = work[blockIdx.x];
  const long N = d.n;
  const int il = threadIdx.x & 15, jl = threadIdx.x >> 4;
  const int i = wk.i0 + il;
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
  Acc<R> A{0, 0, 0, 0, 0, 0, 0};
  for (int j = wk.j0 + jl; j < wk.j1; j += 64) {
    const R dx = (R)(xi - d.x[j]), dy = (R)(yi - d.x[N + j]), dz = (R)(zi - d.x[2 * N + j]);
    const R r2 = fma_(dz, dz, fma_(dy, dy, dx * dx));
    const R rinv = (j == i) ? R(0) : rsq(r2);
    pair_acc(dx, dy, dz, mu[j], mu[N + j], mu[2 * N + j], mix, miy, miz, rinv, A);
  }
  const double v[7] = {(double)A.fx, (double)A.fy, (double)A.fz, (double)A.fm,
                       (double)A.bx, (double)A.by, (double)A.bz};
  for (int k = 0; k < 7; ++k) red[k][jl][il] = v[k];
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if (jl < w)
      for (int k = 0; k < 7; ++k) red[k][jl][il] += red[k][jl + w][il];
    __syncthreads();
  }
  if (jl == 0 && act) {
    const double C = d.C;
    double* p = d.dpart + (long)wk.slot * 6 * N;
    const double fm = red[3][0][il];
    p[i] = C * (red[0][0][il] + fm * (double)mix);
    p[N + i] = C * (red[1][0][il] + fm * (double)miy);
    p[2 * N + i] = C * (red[2][0][il] + fm * (double)miz);
    p[3 * N + i] = C * red[4][0][il];
    p[4 * N + i] = C * red[5][0][il];
    p[5 * N + i] = C * red[6][0][il];
  }
}

hipError_t launch_dipole(const Dev& d, int precision, const DipWork* work, int nwork,
                         hipStream_t s, const hipEvent_t* ev) {
  if (nwork <= 0) return hipSuccess;
  if (d.dip_small) {
    if (precision == 1)
      launch_k(ev, k_dipole_small<float>, dim3(nwork), dim3(1024), s, d, work);
    else
      launch_k(ev, k_dipole_small<double>, dim3(nwork), dim3(1024), s, d, work);
  } else if (precision == 1) {
    launch_k(ev, k_dipole<float>, dim3(nwork), dim3(256), s, d, work);
  } else {
    launch_k(ev, k_dipole<double>, dim3(nwork), dim3(256), s, d, work);
  }
  return hipGetLastError();
}

}  // namespace rodmx
