// Bond kernel (main text eq:bpm-fr to eq:bpm-vector); the arithmetic is in
// bond_body.h and bond_core.h.
#include "bond_body.h"

namespace rodmx {

template <class R>
__global__ __launch_bounds__(256) void k_bond(Dev d, int want_energy) {
  bond_thread<R, true>(d, d.i_lo + (long)blockIdx.x * blockDim.x + threadIdx.x, want_energy);
}

hipError_t launch_bond(const Dev& d, int precision, int want_energy, hipStream_t s,
                       const hipEvent_t* ev) {
  const int bs = particle_block(d.n);
  dim3 grid((unsigned)((d.i_hi - d.i_lo + bs - 1) / bs));
  if (precision == 1)
    launch_k(ev, k_bond<float>, grid, dim3(bs), s, d, want_energy);
  else
    launch_k(ev, k_bond<double>, grid, dim3(bs), s, d, want_energy);
  return hipGetLastError();
}

}  // namespace rodmx
