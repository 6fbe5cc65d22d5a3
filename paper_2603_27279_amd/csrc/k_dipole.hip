// Dipole kernels (Methods, "Magnetic interactions"); the pair arithmetic and
// the work items of both layouts are in dipole_body.h, the list walk of the
// cutoff interaction in dipole_list.h.
#include "dipole_body.h"
#include "dipole_list.h"

namespace rodmx {

template <class R>
__global__ __launch_bounds__(256) void k_dipole(Dev d, const DipWork* __restrict__ work) {
  __shared__ DipSmem<R> sm;
  dipole_item<R>(d, work[blockIdx.x], sm);
}

template <class R>
__global__ __launch_bounds__(256) void k_dipole_small(Dev d, const DipWork* __restrict__ work) {
  dipole_small_item<R>(d, work[blockIdx.x]);
}

hipError_t launch_dipole(const Dev& d, int precision, const DipWork* work, int nwork,
                         hipStream_t s, const hipEvent_t* ev) {
  if (nwork <= 0) return hipSuccess;
  if (d.dip_small) {
    if (precision == 1)
      launch_k(ev, k_dipole_small<float>, dim3(nwork), dim3(256), s, d, work);
    else
      launch_k(ev, k_dipole_small<double>, dim3(nwork), dim3(256), s, d, work);
  } else if (precision == 1) {
    launch_k(ev, k_dipole<float>, dim3(nwork), dim3(256), s, d, work);
  } else {
    launch_k(ev, k_dipole<double>, dim3(nwork), dim3(256), s, d, work);
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_dipole_l(Dev d, int build) {
  dipole_listed(d, blockIdx.x, lists_stale(d, build));
}

hipError_t launch_dipole_cut(const Dev& d, int build, hipStream_t s, const hipEvent_t* ev) {
  const unsigned g = (unsigned)((d.i_hi - d.i_lo + 255) / 256);
  launch_k(ev, k_dipole_l, dim3(g), dim3(256), s, d, build);
  return hipGetLastError();
}

}  // namespace rodmx
