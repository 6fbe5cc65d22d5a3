// Contact kernel: Hookean normal repulsion k (r_c - r) between particles of the
// same member that are closer than r_c and not bonded within the exclusion
// depth (Methods, "Contact", with the normal-only Hookean law of the workloads).
//
// Candidates come from the hashed cell list built by the pre kernel (cell side
// r_c, 27 neighbouring cells, plus the short list of particles whose cell was
// full). The selection r^2 = (dx dx + dy dy) + dz dz < r_c^2 is evaluated with
// explicitly rounded FP64 operations (no contraction), so the pair set is
// exactly that of a brute-force search with the same expression. Each
// particle's contacts are kept sorted by j and summed in that order.
#include "rod_internal.h"
#include "rod_math.h"

namespace rodmx {

__device__ __forceinline__ int cell_coord_c(double x, double inv) {
  double c = floor(x * inv);
  c = fmin(fmax(c, -1.0e9), 1.0e9);
  return (int)c;
}
__device__ __forceinline__ unsigned cell_hash_c(int cx, int cy, int cz, int mem, unsigned mask) {
  unsigned h = (unsigned)cx * 73856093u ^ (unsigned)cy * 19349663u ^ (unsigned)cz * 83492791u ^
               (unsigned)mem * 2654435761u;
  return h & mask;
}

__device__ __forceinline__ double r2_exact(V3<double> a, V3<double> b) {
  double dx = __dsub_rn(a.x, b.x), dy = __dsub_rn(a.y, b.y), dz = __dsub_rn(a.z, b.z);
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

// Visit every candidate j of particle i (duplicates possible when cells share
// a hash bucket) and keep the accepted ones, sorted and unique, in `list`.
__device__ __forceinline__ int gather_contacts(const Dev& d, long i, int* list, bool& ovf) {
  const long N = d.n;
  const V3<double> xi = ld3(d.x, N, i);
  const int mem = d.mem[i], rod = d.rod[i];
  const double rc2 = d.rc * d.rc;
  const int cx = cell_coord_c(xi.x, d.inv_cell), cy = cell_coord_c(xi.y, d.inv_cell),
            cz = cell_coord_c(xi.z, d.inv_cell);
  int cnt = 0;
  auto consider = [&](int j) {
    if (j == (int)i || d.mem[j] != mem) return;
    if (d.rod[j] == rod && abs(j - (int)i) <= d.depth) return;
    if (!(r2_exact(xi, ld3(d.x, N, j)) < rc2)) return;
    int p = cnt;
    while (p > 0 && list[p - 1] > j) --p;
    if (p > 0 && list[p - 1] == j) return;  // already listed
    if (cnt == CONTACT_MAX) { ovf = true; return; }
    for (int s = cnt; s > p; --s) list[s] = list[s - 1];
    list[p] = j;
    ++cnt;
  };
  for (int oz = -1; oz <= 1; ++oz)
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        unsigned key = cell_hash_c(cx + ox, cy + oy, cz + oz, mem, d.cell_mask);
        int nb = min(d.cell_cnt[key], CELL_CAP);
        const int* slot = d.cell_slot + (long)key * CELL_CAP;
        for (int s = 0; s < nb; ++s) consider(slot[s]);
      }
  int no = min(*d.ovf_cnt, OVF_CAP);
  for (int o = 0; o < no; ++o) consider(d.ovf_list[o]);
  return cnt;
}

__global__ __launch_bounds__(256) void k_contact(Dev d, int want_energy) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long N = d.n;
  if (i >= N) return;
  int list[CONTACT_MAX];
  bool ovf = false;
  const int cnt = gather_contacts(d, i, list, ovf);
  if (ovf) atomicOr(&d.flags[FLAG_CONTACT_OVF], 1u);
  const V3<double> xi = ld3(d.x, N, i);
  V3<double> F{0.0, 0.0, 0.0};
  double E = 0.0;
  for (int k = 0; k < cnt; ++k) {
    const V3<double> dd = xi - ld3(d.x, N, list[k]);
    const double r = sqrt(r2_exact(xi, ld3(d.x, N, list[k])));
    const double ov = d.rc - r;
    F = F + ((d.kc * ov) / r) * dd;
    E += 0.25 * d.kc * ov * ov;  // each pair is seen from both ends
  }
  st3(d.cF, N, i, F);
  if (want_energy) d.cE[i] = E;
}

// Debug/inspection: append every pair (i < j) found by the cell list.
__global__ __launch_bounds__(256) void k_contact_pairs(Dev d, int* pairs, int cap, int* count) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  int list[CONTACT_MAX];
  bool ovf = false;
  const int cnt = gather_contacts(d, i, list, ovf);
  if (ovf) atomicOr(&d.flags[FLAG_CONTACT_OVF], 1u);
  for (int k = 0; k < cnt; ++k) {
    if (list[k] <= (int)i) continue;
    int p = atomicAdd(count, 1);
    if (p < cap) { pairs[2 * p] = (int)i; pairs[2 * p + 1] = list[k]; }
  }
}

// Empty the cell list built by a pre pass that had no particle pass after it.
__global__ __launch_bounds__(256) void k_clear_cells(Dev d) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.n) d.cell_cnt[d.key[i]] = 0;
  if (i == 0) *d.ovf_cnt = 0;
}

hipError_t launch_clear_cells(const Dev& d, hipStream_t s) {
  if (!d.contact_on) return hipSuccess;
  hipLaunchKernelGGL(k_clear_cells, dim3((unsigned)((d.n + 255) / 256)), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_contact(const Dev& d, int want_energy, hipStream_t s) {
  if (!d.contact_on) return hipSuccess;
  hipLaunchKernelGGL(k_contact, dim3((unsigned)((d.n + 255) / 256)), dim3(256), 0, s, d,
                     want_energy);
  return hipGetLastError();
}

hipError_t launch_contact_pairs(const Dev& d, int* pairs, int cap, int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_pairs, dim3((unsigned)((d.n + 255) / 256)), dim3(256), 0, s, d,
                     pairs, cap, count);
  return hipGetLastError();
}

}  // namespace rodmx
