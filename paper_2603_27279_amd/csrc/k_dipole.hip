// Dipole kernels (Methods, "Magnetic interactions"); the pair arithmetic and
// the split-layout work item are in dipole_body.h.
#include "dipole_body.h"

namespace rodmx {

template <class R>
__global__ __launch_bounds__(256) void k_dipole(Dev d, const DipWork* __restrict__ work) {
  __shared__ DipSmem<R> sm;
  dipole_item<R>(d, work[blockIdx.x], sm);
}

// Layout for small members: a workgroup of 1024 threads serves 16 consecutive
// i of one member; thread (il, jl) visits j = j0 + jl, j0 + jl + 64, ... of
// the member, so every member pair is spread over the whole workgroup. The
// 64 partial sums of each i are added by a fixed LDS tree. One slot.
template <class R>
__global__ __launch_bounds__(1024) void k_dipole_small(Dev d, const DipWork* __restrict__ work) {
  __shared__ double red[NACC][16][16];
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
  Acc<R> A{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const R m5 = minus5(R(0));
  for (int j = wk.j0 + jl; j < wk.j1; j += 64) {
    const R dx = (R)(xi - d.x[j]), dy = (R)(yi - d.x[N + j]), dz = (R)(zi - d.x[2 * N + j]);
    const R r2 = fma_(dz, dz, fma_(dy, dy, dx * dx));
    const R rinv = (j == i) ? R(0) : rsq(r2);
    pair_acc(dx, dy, dz, mu[j], mu[N + j], mu[2 * N + j], mix, miy, miz, rinv, m5, A);
  }
  const double v[NACC] = {(double)A.fx,  (double)A.fy,  (double)A.fz,  (double)A.fm,
                          (double)A.bsx, (double)A.bsy, (double)A.bsz, (double)A.bmx,
                          (double)A.bmy, (double)A.bmz};
  // the four jl of a wave first (lanes 16 and 32 apart), then a tree over waves
  for (int k = 0; k < NACC; ++k) {
    double t = v[k] + __shfl_xor(v[k], 16);
    t += __shfl_xor(t, 32);
    if ((jl & 3) == 0) red[k][jl >> 2][il] = t;
  }
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (jl < w)  // jl < 8 here: rows of the 16 per-wave sums
      for (int k = 0; k < NACC; ++k) red[k][jl][il] += red[k][jl + w][il];
    __syncthreads();
  }
  if (jl == 0 && act) {
    double F[NACC];
    for (int k = 0; k < NACC; ++k) F[k] = red[k][0][il];
    write_slot(d.dpart + (long)wk.slot * 6 * N, N, i, d.C, F, mix, miy, miz);
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
