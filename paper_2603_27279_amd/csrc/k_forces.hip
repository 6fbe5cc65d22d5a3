// Force pass of one time step in a single launch: the dipole work items first
// (either layout), then the bond threads, then the contact search. The three
// parts read the same drifted state and write disjoint buffers, so their
// workgroups run side by side and the latency-bound bond and contact work hides
// under the dipole arithmetic.
#include "dipole_body.h"
#include "bond_body.h"
#include "contact_body.h"

namespace rodmx {

template <class R, bool LANES>
__global__ __launch_bounds__(256) void k_forces(Dev d, const DipWork* __restrict__ work, int ndip,
                                                int nbond, int build) {
  __shared__ DipSmem<R> sm;
  const int b = blockIdx.x;
  if (b < ndip) {
    if (d.dip_small) dipole_small_item<R>(d, work[b]);
    else dipole_item<R>(d, work[b], sm);
  } else if (b < ndip + nbond) {
    bond_thread<R>(d, d.i_lo + (long)(b - ndip) * 256 + threadIdx.x, 0);
  } else if (LANES) {
    contact_pass<OUT_FORCE>(d, b - ndip - nbond, nullptr, 0, nullptr);
  } else {
    contact_listed(d, b - ndip - nbond, lists_stale(d, build));
  }
}

hipError_t launch_forces(const Dev& d, int precision, const DipWork* work, int nwork, int build,
                         hipStream_t s, const hipEvent_t* ev) {
  const int ndip = d.dipole_on ? nwork : 0;
  const int nbond = (int)((d.i_hi - d.i_lo + 255) / 256);
  const unsigned ncont = d.contact_on ? contact_blocks(d) : 0;
  const dim3 g((unsigned)ndip + (unsigned)nbond + ncont), b(256);
  const bool lanes = d.n < CONTACT_LANES_MAX_N;
  if (precision == 1) {
    if (lanes) launch_k(ev, k_forces<float, true>, g, b, s, d, work, ndip, nbond, build);
    else launch_k(ev, k_forces<float, false>, g, b, s, d, work, ndip, nbond, build);
  } else {
    if (lanes) launch_k(ev, k_forces<double, true>, g, b, s, d, work, ndip, nbond, build);
    else launch_k(ev, k_forces<double, false>, g, b, s, d, work, ndip, nbond, build);
  }
  return hipGetLastError();
}

}  // namespace rodmx
