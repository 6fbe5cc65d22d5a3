// Contact kernels (Methods, "Contact"); the search itself is in contact_body.h.
#include "contact_body.h"

namespace rodmx {

__global__ __launch_bounds__(256) void k_contact(Dev d) {
  contact_pass<OUT_FORCE>(d, blockIdx.x, nullptr, 0, nullptr);
}
__global__ __launch_bounds__(256) void k_contact_e(Dev d) {
  contact_pass<OUT_ENERGY>(d, blockIdx.x, nullptr, 0, nullptr);
}
__global__ __launch_bounds__(256) void k_contact_l(Dev d, int build) {
  contact_listed(d, blockIdx.x, lists_stale(d, build));
}
__global__ __launch_bounds__(256) void k_contact_te(Dev d) {
  contact_thread<OUT_ENERGY>(d, blockIdx.x);
}
// At least three waves per SIMD: the exact 128-bit sums would otherwise take the
// list walk to 182 VGPRs (two waves); capped at 168 it spills 15 and is faster
// (4.2M particles: 112 against 125 us per walk, list build 1.9 against 2.3 ms).
__global__ __launch_bounds__(256, 3) void k_contact_hm(Dev d, int build) {
  contact_hm_thread<OUT_FORCE>(d, blockIdx.x, d.use_lists && lists_stale(d, build));
}
__global__ __launch_bounds__(256) void k_contact_hm_e(Dev d) {
  contact_hm_thread<OUT_ENERGY>(d, blockIdx.x, false);
}
__global__ __launch_bounds__(256) void k_contact_hm_lanes(Dev d) {
  contact_hm_lanes<OUT_FORCE>(d, blockIdx.x);
}
__global__ __launch_bounds__(256) void k_contact_hm_lanes_e(Dev d) {
  contact_hm_lanes<OUT_ENERGY>(d, blockIdx.x);
}
__global__ __launch_bounds__(256) void k_contact_pairs(Dev d, int* pairs, int cap, int* count) {
  contact_pass<OUT_PAIRS>(d, blockIdx.x, pairs, cap, count);
}

// Empty the cell list built by a pre pass that had no particle pass after it.
__global__ __launch_bounds__(256) void k_clear_cells(Dev d) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const CellTab tab = cell_tab(d, d.step[d.lc]);
  if (i < d.n) tab.cnt[d.key[i]] = 0;
  if (i == 0) *tab.ovf_cnt = 0;
}

// Fill n ints with v (a kernel rather than a memset node).
__global__ __launch_bounds__(256) void k_fill_i32(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int* p, int n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_clear_cells(const Dev& d, hipStream_t s) {
  if (!d.contact_on) return hipSuccess;
  hipLaunchKernelGGL(k_clear_cells, dim3((unsigned)((d.n + 255) / 256)), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_contact(const Dev& d, int want_energy, int build, hipStream_t s,
                          const hipEvent_t* ev) {
  if (!d.contact_on) return hipSuccess;
  if (d.hm) {
    const dim3 g(contact_blocks(d));
    if (d.n < CONTACT_LANES_MAX_N) {
      if (want_energy) launch_k(ev, k_contact_hm_lanes_e, g, dim3(256), s, d);
      else launch_k(ev, k_contact_hm_lanes, g, dim3(256), s, d);
    } else {
      if (want_energy) launch_k(ev, k_contact_hm_e, g, dim3(256), s, d);
      else launch_k(ev, k_contact_hm, g, dim3(256), s, d, build);
    }
    return hipGetLastError();
  }
  if (d.n >= CONTACT_LANES_MAX_N) {
    if (want_energy) launch_k(ev, k_contact_te, dim3(contact_blocks(d)), dim3(256), s, d);
    else launch_k(ev, k_contact_l, dim3(contact_blocks(d)), dim3(256), s, d, build);
    return hipGetLastError();
  }
  if (want_energy)
    launch_k(ev, k_contact_e, dim3(contact_lane_blocks(d)), dim3(256), s, d);
  else
    launch_k(ev, k_contact, dim3(contact_lane_blocks(d)), dim3(256), s, d);
  return hipGetLastError();
}

hipError_t launch_contact_pairs(const Dev& d, int* pairs, int cap, int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_pairs, dim3(contact_lane_blocks(d)), dim3(256), 0, s, d, pairs, cap,
                     count);
  return hipGetLastError();
}

}  // namespace rodmx
