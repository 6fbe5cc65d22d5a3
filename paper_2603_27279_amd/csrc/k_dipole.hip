// Dipole kernels (Methods, "Magnetic interactions"); the pair arithmetic and
// the work items of both layouts are in dipole_body.h, the list walk of the
// cutoff interaction in dipole_list.h.
#include "dipole_body.h"
#include "dipole_list.h"
#include "particle_body.h"

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

// Boxes of the 64-position chunks of the spatial order, one wave per chunk
// (the far test of the mixed split layout reads them).
__global__ __launch_bounds__(256) void k_spatial_box(Dev d) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = p < d.n;
  V3<double> x{0.0, 0.0, 0.0};
  if (valid) x = ld3(d.x, d.n, d.dperm[p]);
  wave_box(d.sbox + 6 * (p >> 6), x, valid, p < d.n);
}

hipError_t launch_spatial_boxes(const Dev& d, hipStream_t s) {
  if (!d.dperm || !d.far_ok) return hipSuccess;
  hipLaunchKernelGGL(k_spatial_box, dim3((unsigned)((d.n + 255) / 256)), dim3(256), 0, s, d);
  return hipGetLastError();
}

static void dipole_items(const Dev& d, int precision, const DipWork* work, int nwork,
                         hipStream_t s, const hipEvent_t* ev) {
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
}

hipError_t launch_dipole(const Dev& d, int precision, const DipWork* work, int nwork,
                         hipStream_t s, const hipEvent_t* ev) {
  if (nwork <= 0) return hipSuccess;
  if (d.dperm && precision == 1 && d.far_ok) {
    // the chunk boxes of the spatial order first; a timed launch brackets both
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    if ((e = launch_spatial_boxes(d, s)) != hipSuccess) return e;
    dipole_items(d, precision, work, nwork, s, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return ev ? hipEventRecord(ev[1], s) : hipSuccess;
  }
  dipole_items(d, precision, work, nwork, s, ev);
  return hipGetLastError();
}

// ------------------------------------------------------- the cutoff sort
// Each launch does nothing unless the lists are rebuilt at this step (the
// decision is the same for every thread: the flag is written by the previous
// step's kernels).

// Each particle's bucket and counting slot.
__global__ __launch_bounds__(256) void k_dl_bin(Dev d, int build) {
  if (!lists_stale(d, build)) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const double* p = static_cast<const double*>(__builtin_assume_aligned(d.xm + 8 * i, 64));
  const unsigned b = dl_bucket(d, dl_coord(p[0], d.dl_org[0], d.dl_inv),
                               dl_coord(p[1], d.dl_org[1], d.dl_inv),
                               dl_coord(p[2], d.dl_org[2], d.dl_inv), d.mem[i]);
  d.dl_bkt[i] = (int)b;
  d.dl_slot[i] = atomicAdd(&d.dl_cnt[b], 1);
}

// Sum over the 256 threads of a workgroup, returned to every thread.
__device__ __forceinline__ int dl_block_sum(int v, int* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();  // sh may still be read from an earlier call
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return sh[0] + sh[1] + sh[2] + sh[3];
}

// Particles in each block of DL_SCAN buckets (eight buckets per thread).
__global__ __launch_bounds__(256) void k_dl_bsum(Dev d, int build) {
  if (!lists_stale(d, build)) return;
  __shared__ int sh[4];
  const int* c = d.dl_cnt + (long)blockIdx.x * DL_SCAN + 8 * threadIdx.x;
  int s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += c[k];
  s = dl_block_sum(s, sh);
  if (threadIdx.x == 0) d.dl_aux[blockIdx.x] = s;
}

// First sorted position of every bucket: the particles of the blocks before
// (each workgroup adds them itself), then an exclusive scan inside the block.
// The counts are cleared for the next rebuild.
__global__ __launch_bounds__(256) void k_dl_start(Dev d, int build) {
  if (!lists_stale(d, build)) return;
  __shared__ int sh[256];
  const int t = threadIdx.x;
  int off = 0;
  for (int k = t; k < (int)blockIdx.x; k += 256) off += d.dl_aux[k];
  off = dl_block_sum(off, sh);
  int* c = d.dl_cnt + (long)blockIdx.x * DL_SCAN + 8 * t;
  int v[8], s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) { v[k] = c[k]; s += v[k]; }
  __syncthreads();
  sh[t] = s;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {  // inclusive scan of the threads' sums
    const int u = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += u;
    __syncthreads();
  }
  int run = off + sh[t] - s;
  int* st = d.dl_start + (long)blockIdx.x * DL_SCAN + 8 * t;
#pragma unroll
  for (int k = 0; k < 8; ++k) { st[k] = run; run += v[k]; c[k] = 0; }
  if (blockIdx.x == gridDim.x - 1 && t == 255) d.dl_start[d.dl_nb] = run;
}

// Particles grouped by bucket, in the arbitrary order of the counting slots.
__global__ __launch_bounds__(256) void k_dl_scatter(Dev d, int build) {
  if (!lists_stale(d, build)) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  d.dl_tmp[d.dl_start[d.dl_bkt[i]] + d.dl_slot[i]] = (int)i;
}

// Each bucket's particles in ascending index: a particle's place is the number
// of its bucket's particles with a smaller index. Writes the sorted order, its
// inverse and each sorted position's record.
__global__ __launch_bounds__(256) void k_dl_rank(Dev d, int build) {
  if (!lists_stale(d, build)) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int b = d.dl_bkt[i];
  const int lo = d.dl_start[b], hi = d.dl_start[b + 1];
  int r = 0;
  for (int q = lo; q < hi; ++q) r += d.dl_tmp[q] < (int)i;
  const int t = lo + r;
  d.dl_sorted[t] = (int)i;
  d.dl_pos[i] = t;
  const double* p = static_cast<const double*>(__builtin_assume_aligned(d.xm + 8 * i, 64));
  DlRec e;
  e.x = p[0]; e.y = p[1]; e.z = p[2];
  e.i = (int)i;
  e.tag = dl_tag(d, dl_coord(p[0], d.dl_org[0], d.dl_inv), dl_coord(p[1], d.dl_org[1], d.dl_inv),
                 dl_coord(p[2], d.dl_org[2], d.dl_inv));
  d.dl_rec[t] = e;
}

hipError_t launch_dipole_sort(const Dev& d, int build, hipStream_t s) {
  const unsigned gp = (unsigned)((d.n + 255) / 256), gb = (unsigned)(d.dl_nb / DL_SCAN);
  hipLaunchKernelGGL(k_dl_bin, dim3(gp), dim3(256), 0, s, d, build);
  hipLaunchKernelGGL(k_dl_bsum, dim3(gb), dim3(256), 0, s, d, build);
  hipLaunchKernelGGL(k_dl_start, dim3(gb), dim3(256), 0, s, d, build);
  hipLaunchKernelGGL(k_dl_scatter, dim3(gp), dim3(256), 0, s, d, build);
  hipLaunchKernelGGL(k_dl_rank, dim3(gp), dim3(256), 0, s, d, build);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_dipole_lb(Dev d, int build) {
  if (!lists_stale(d, build)) return;
  __shared__ DlCells cells[DL_BUILD_GROUPS];
  dipole_list_build(d, blockIdx.x, cells);
}
__global__ __launch_bounds__(256) void k_dipole_l(Dev d) { dipole_list_walk(d, blockIdx.x); }

// Over the whole system: the sort and the list build (at a rebuild), then the
// walk; over one rod's range (per-rod loop) the build and the walk, the sort
// having run before.
hipError_t launch_dipole_cut(const Dev& d, int build, hipStream_t s, const hipEvent_t* ev) {
  const bool whole = d.i_lo == 0 && d.i_hi == d.n;
  hipError_t e;
  // the event pair (timing mode) brackets the whole sequence
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
  if (whole && (e = launch_dipole_sort(d, build, s)) != hipSuccess) return e;
  const long n = d.i_hi - d.i_lo, pb = 256 / DL_LANES, pw = 256 / DL_WALK_LANES;
  hipLaunchKernelGGL(k_dipole_lb, dim3((unsigned)((n + pb - 1) / pb)), dim3(256), 0, s, d, build);
  hipLaunchKernelGGL(k_dipole_l, dim3((unsigned)((n + pw - 1) / pw)), dim3(256), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev) return hipEventRecord(ev[1], s);
  return hipSuccess;
}

}  // namespace rodmx
