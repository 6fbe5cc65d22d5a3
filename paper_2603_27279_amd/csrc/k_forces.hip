// Force pass of one time step in a single launch: the dipole work items first
// (either layout), then the bond threads, then (LANES) the lane-parallel
// contact search. The parts read the same drifted state and write disjoint
// buffers, so their workgroups run side by side and the latency-bound bond and
// contact work hides under the dipole arithmetic. Large systems search contacts
// through candidate lists in a launch of their own: the list walk and rebuild
// need more registers than the dipole arithmetic, and in one kernel they would
// cost the dipole work items a wave per SIMD.
#include "dipole_body.h"
#include "bond_body.h"
#include "contact_body.h"

namespace rodmx {

// HM: the lane-parallel search is the Hertz-Mindlin one (a kernel of its own,
// k_forces_hm, so that the Hookean kernels keep their register budget).
template <class R, bool LANES, bool HM>
__device__ __forceinline__ void forces_body(const Dev& d, const DipWork* __restrict__ work,
                                            int ndip, int nbond) {
  __shared__ DipSmem<R> sm;
  const int b = blockIdx.x;
  if (b < ndip) {
    if (d.dip_small) dipole_small_item<R>(d, work[b]);
    else dipole_item<R>(d, work[b], sm);
  } else if (b < ndip + nbond) {
    bond_thread<R>(d, d.i_lo + (long)(b - ndip) * 256 + threadIdx.x, 0);
  } else if constexpr (LANES) {
    if constexpr (HM) contact_hm_lanes<OUT_FORCE>(d, b - ndip - nbond);
    else contact_pass<OUT_FORCE>(d, b - ndip - nbond, nullptr, 0, nullptr);
  }
}

template <class R, bool LANES>
__global__ __launch_bounds__(256) void k_forces(Dev d, const DipWork* __restrict__ work, int ndip,
                                                int nbond) {
  forces_body<R, LANES, false>(d, work, ndip, nbond);
}

template <class R>
__global__ __launch_bounds__(256) void k_forces_hm(Dev d, const DipWork* __restrict__ work,
                                                   int ndip, int nbond) {
  forces_body<R, true, true>(d, work, ndip, nbond);
}

static void forces_kernel(const Dev& d, int precision, const DipWork* work, int ndip,
                          hipStream_t s, const hipEvent_t* ev);

hipError_t launch_forces(const Dev& d, int precision, const DipWork* work, int nwork,
                         hipStream_t s, const hipEvent_t* ev) {
  const int ndip = d.dipole_on ? nwork : 0;
  if (ndip > 0 && d.dperm && precision == 1 && d.far_ok) {
    // the chunk boxes of the spatial order first; a timed launch brackets both
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    if ((e = launch_spatial_boxes(d, s)) != hipSuccess) return e;
    forces_kernel(d, precision, work, ndip, s, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return ev ? hipEventRecord(ev[1], s) : hipSuccess;
  }
  forces_kernel(d, precision, work, ndip, s, ev);
  return hipGetLastError();
}

static void forces_kernel(const Dev& d, int precision, const DipWork* work, int ndip,
                          hipStream_t s, const hipEvent_t* ev) {
  const int nbond = (int)((d.i_hi - d.i_lo + 255) / 256);
  const bool lanes = contact_in_forces(d);
  const unsigned ncont = d.contact_on && lanes ? contact_lane_blocks(d) : 0;
  const dim3 g((unsigned)ndip + (unsigned)nbond + ncont), b(256);
  const bool hm = lanes && d.contact_on && d.hm;
  if (precision == 1) {
    if (hm) launch_k(ev, k_forces_hm<float>, g, b, s, d, work, ndip, nbond);
    else if (lanes) launch_k(ev, k_forces<float, true>, g, b, s, d, work, ndip, nbond);
    else launch_k(ev, k_forces<float, false>, g, b, s, d, work, ndip, nbond);
  } else {
    if (hm) launch_k(ev, k_forces_hm<double>, g, b, s, d, work, ndip, nbond);
    else if (lanes) launch_k(ev, k_forces<double, true>, g, b, s, d, work, ndip, nbond);
    else launch_k(ev, k_forces<double, false>, g, b, s, d, work, ndip, nbond);
  }
}

hipError_t launch_force_pass(const Dev& d, int precision, const DipWork* work, int nwork,
                             int build, hipStream_t s) {
  // with a dipole cutoff the items (if any) are the reverse pass's; the
  // forward walks the lists
  hipError_t e = launch_forces(d, precision, work, d.dcut > 0.0 ? 0 : nwork, s);
  if (e == hipSuccess && d.contact_on && !contact_in_forces(d)) e = launch_contact(d, 0, build, s);
  if (e == hipSuccess && d.dipole_on && d.dcut > 0.0) e = launch_dipole_cut(d, build, s);
  return e;
}

}  // namespace rodmx
