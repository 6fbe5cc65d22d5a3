// Per-particle code shared by the integration kernels and the reverse pass.
#pragma once
#include "rod_internal.h"
#include "rod_math.h"

namespace rodmx {

// Cell-list key of a particle at x in member mem.
__device__ __forceinline__ unsigned cell_key(const Dev& d, V3<double> x, int mem) {
  return cell_hash(cell_coord(x.x, d.inv_cell), cell_coord(x.y, d.inv_cell),
                   cell_coord(x.z, d.inv_cell), mem, d.cell_mask);
}

// Store particle i in the slot it claimed in cell `key` of table t (the
// overflow list past CELL_CAP entries), and its key.
__device__ __forceinline__ void cell_place(const Dev& d, const CellTab& t, long i, V3<double> x,
                                           int rod, unsigned key, int slot) {
  if (slot < CELL_CAP) {
    CellSlot e;
    e.x = x.x; e.y = x.y; e.z = x.z;
    e.tag = (long long)(unsigned)i | ((long long)rod << 32);
    t.slot[(long)key * CELL_CAP + slot] = e;
  } else {
    int o = atomicAdd(t.ovf_cnt, 1);
    if (o < OVF_CAP) t.ovf[o] = (int)i;
    else atomicOr(&d.flags[FLAG_LIST_OVF], 1u);
  }
  d.key[i] = (int)key;
}

// The particle's entry in the cell list of level lvl.
__device__ __forceinline__ void cell_insert(const Dev& d, long i, V3<double> x, int mem, int rod,
                                            long long lvl) {
  const CellTab t = cell_tab(d, lvl);
  const unsigned key = cell_key(d, x, mem);
  cell_place(d, t, i, x, rod, key, atomicAdd(&t.cnt[key], 1));
}

// Dipole moment in the global frame, m = q m_body q*, and (insert) the
// particle's entry in the cell list of level lvl.
__device__ __forceinline__ void moment_and_cell(const Dev& d, long i, Q4<double> q, V3<double> x,
                                                V3<double> mb, int mem, int rod, long long lvl,
                                                bool insert = true) {
#pragma clang fp contract(on)  // round alike wherever it is inlined
  const long N = d.n;
  V3<double> m = qrot(q, mb);
  st3(d.mu, N, i, m);
  if (d.muf) st3(d.muf, N, i, V3<float>{(float)m.x, (float)m.y, (float)m.z});
  if (d.xm) {  // interleaved copy for the cutoff list walk: one line per partner
    double* p = d.xm + 8 * i;
    p[0] = x.x; p[1] = x.y; p[2] = x.z;
    p[3] = m.x; p[4] = m.y; p[5] = m.z; p[6] = 0.0; p[7] = 0.0;
  }
  if (d.contact_on && insert) cell_insert(d, i, x, mem, rod, lvl);
}

// Bounding box of the x of the wave's lanes into out[0..6) (low then high;
// `valid` marks lanes with a particle), written by lane 0 when `write`.
__device__ __forceinline__ void wave_box(double* out, V3<double> x, bool valid, bool write) {
  double lx = valid ? x.x : 1e300, ly = valid ? x.y : 1e300, lz = valid ? x.z : 1e300;
  double hx = valid ? x.x : -1e300, hy = valid ? x.y : -1e300, hz = valid ? x.z : -1e300;
  for (int o = 32; o > 0; o >>= 1) {
    lx = fmin(lx, __shfl_xor(lx, o)); hx = fmax(hx, __shfl_xor(hx, o));
    ly = fmin(ly, __shfl_xor(ly, o)); hy = fmax(hy, __shfl_xor(hy, o));
    lz = fmin(lz, __shfl_xor(lz, o)); hz = fmax(hz, __shfl_xor(hz, o));
  }
  if ((threadIdx.x & 63) == 0 && write) {
    out[0] = lx; out[1] = ly; out[2] = lz; out[3] = hx; out[4] = hy; out[5] = hz;
  }
}

// Bounding box of the wave's 64 particles (a 64-aligned chunk: the
// per-particle kernels start at particle 0 in blocks of 64 or 256) into
// d.cbox. Every lane of the wave calls it; `valid` marks lanes with a particle.
__device__ __forceinline__ void chunk_box(const Dev& d, long i, V3<double> x, bool valid) {
  if (!d.far_ok) return;
  wave_box(d.cbox + 6 * (i >> 6), x, valid, i < d.n);
}

}  // namespace rodmx
