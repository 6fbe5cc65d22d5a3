// Dipole-dipole interaction with a cutoff (Methods, "Magnetic interactions",
// truncated as the paper's pair style truncates it): particle i feels the
// particles j of its member with r^2 = (dx dx + dy dy) + dz dz < dcut^2 (exact
// FP64 selection, as in the contact search), through the same pair law as the
// all-pairs sum. Each particle keeps a Verlet list of the member's particles
// closer than dcut + skin, rebuilt with the contact lists (first step of a
// call, or when a particle has moved more than NBR_MOVE * skin).
//
// A rebuild first sorts the particles by cell (cells of side dcut + skin, so a
// particle's candidates lie in the 3 x 3 x 3 cells around its own). A cell's
// bucket is its member number above the low bits of its three coordinates,
// interleaved bit by bit (a Z-order curve), so that consecutive buckets are
// neighbouring cells. Counting sort: each particle's bucket and an atomic slot
// in it; exclusive sums of the counts in two passes; the particles grouped by
// bucket; within a bucket ranked by index (a fixed order). The list walk runs
// over the sorted positions, and the positions are dealt to the XCDs in
// contiguous ranges, so a workgroup's particles share their partners' lines
// with the workgroups running beside it on the same L2.
//
// Cells whose coordinates differ by a multiple of 2^bits along an axis share a
// bucket; every sorted record carries the high bits of its cell's coordinates
// (a tag), and a walk takes from a bucket only the records of the cell it
// visits. The list order and the summation are fixed by the sort: a run
// repeated gives the same bits.
#pragma once
#include "contact_body.h"

namespace rodmx {

// Cell coordinates of x relative to the key origin.
__device__ __forceinline__ int dl_coord(double x, double org, double inv) {
  return cell_coord(x - org, inv);
}

// The low bits of g deposited at the set bits of `mask`, lowest first.
__device__ __forceinline__ unsigned dl_spread(unsigned g, unsigned mask) {
  unsigned out = 0u;
  for (unsigned m = mask; m != 0u; m &= m - 1u, g >>= 1) out |= (g & 1u) ? (m & (0u - m)) : 0u;
  return out;
}

// High bits of a cell's coordinates (those above each axis's key bits), ten
// signed bits per axis; DL_TAG_FAR when one does not fit.
constexpr unsigned DL_TAG_FAR = 0xffffffffu;
__device__ __forceinline__ unsigned dl_tag(const Dev& d, int gx, int gy, int gz) {
  const int h[3] = {gx >> d.dl_bits[0], gy >> d.dl_bits[1], gz >> d.dl_bits[2]};
  unsigned t = 0u;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (h[a] < -512 || h[a] > 511) return DL_TAG_FAR;
    t |= ((unsigned)h[a] & 1023u) << (10 * a);
  }
  return t;
}

__device__ __forceinline__ unsigned dl_bucket(const Dev& d, int gx, int gy, int gz, int mem) {
  return ((unsigned)mem << d.dl_mshift) | dl_spread((unsigned)gx, d.dl_axis[0]) |
         dl_spread((unsigned)gy, d.dl_axis[1]) | dl_spread((unsigned)gz, d.dl_axis[2]);
}

// Workgroup b of G as dealt to the XCDs in turn, renumbered so that each XCD
// holds a contiguous range of the sorted positions.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned G) {
  const unsigned per = G >> 3, rem = G & 7u, x = b & 7u, k = b >> 3;
  return x < rem ? x * (per + 1u) + k : rem * (per + 1u) + (x - rem) * per + k;
}

// Lanes per particle in the list build and walk.
constexpr int DL_LANES = 8;

// The particle and sorted position served by lane group `g` of workgroup blk:
// over the whole system sorted position t (workgroups dealt to the XCDs in
// contiguous ranges), over one rod's range (the per-rod loop) the rod's
// particle i at its own position. False past the end.
__device__ __forceinline__ bool dl_target(const Dev& d, unsigned blk, long* i, long* t) {
  const long g = threadIdx.x / DL_LANES;
  const long per = blockDim.x / DL_LANES;
  if (d.i_lo == 0 && d.i_hi == d.n) {
    *t = (long)xcd_block(blk, gridDim.x) * per + g;
    if (*t >= d.n) return false;
    *i = d.dl_sorted[*t];
  } else {
    *i = d.i_lo + (long)blk * per + g;
    if (*i >= d.i_hi) return false;
    *t = d.dl_pos[*i];
  }
  return true;
}

// Per lane group of a list-build workgroup: the 27 cells' first sorted
// position, the number of candidates before each cell, and each cell's tag.
struct DlCells { int qb[27]; int pre[28]; unsigned tag[27]; };
constexpr int DL_BUILD_GROUPS = 256 / DL_LANES;

// List rebuild. The candidates are the records of the 27 cells around the
// particle's own, taken in a fixed order (cells by z, y, x offset, each cell's
// records in sorted order). The particle's eight lanes first fetch the 27
// cells' ranges together (four cells per lane) and keep their first positions
// and running counts in LDS; they then take the candidates eight at a time,
// four such chunks in flight, and write the accepted ones in candidate order
// (each lane's place from a ballot), so the list is what one thread taking the
// candidates in that order would write.
__device__ __forceinline__ void dipole_list_build(const Dev& d, unsigned blk, DlCells* cells) {
  constexpr int CH = 4;  // chunks of eight candidates in flight
  const long N = d.n;
  long i, t;
  const bool live = dl_target(d, blk, &i, &t);  // whole lane groups agree
  if (!live) return;
  const int s = threadIdx.x % DL_LANES;
  DlCells& cl = cells[threadIdx.x / DL_LANES];
  const int gshift = (int)(__lane_id() & ~(unsigned)(DL_LANES - 1));
  const unsigned gmask = (1u << DL_LANES) - 1u;
  const double* own = static_cast<const double*>(__builtin_assume_aligned(d.xm + 8 * i, 64));
  const V3<double> xi{own[0], own[1], own[2]};
  const double rs = d.dcut + d.skin, rs2 = rs * rs;
  const int mem = d.mem[i];
  const int gx = dl_coord(xi.x, d.dl_org[0], d.dl_inv), gy = dl_coord(xi.y, d.dl_org[1], d.dl_inv),
            gz = dl_coord(xi.z, d.dl_org[2], d.dl_inv);
  // cells s, s + 8, s + 16, s + 24 of this lane: ranges, then running counts
  int qb[4], len[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int c = s + DL_LANES * m;
    qb[m] = 0; len[m] = 0;
    if (c < 27) {
      const int cx = gx + c % 3 - 1, cy = gy + (c / 3) % 3 - 1, cz = gz + c / 9 - 1;
      const unsigned key = dl_bucket(d, cx, cy, cz, mem);
      qb[m] = d.dl_start[key];
      len[m] = d.dl_start[key + 1] - qb[m];
      cl.tag[c] = dl_tag(d, cx, cy, cz);
    }
  }
  int run = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    int v = len[m];  // inclusive scan over the group's eight lanes
#pragma unroll
    for (int o = 1; o < DL_LANES; o <<= 1) {
      const int u = __shfl_up(v, o, DL_LANES);
      if (s >= o) v += u;
    }
    const int c = s + DL_LANES * m;
    if (c < 27) { cl.qb[c] = qb[m]; cl.pre[c] = run + v - len[m]; }
    run += __shfl(v, DL_LANES - 1, DL_LANES);
  }
  if (s == 0) cl.pre[27] = run;
  __builtin_amdgcn_wave_barrier();  // the group's LDS entries are written by its own wave
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int total = run;
  int nc = 0, c = 0;
  for (int p0 = 0; p0 < total; p0 += CH * DL_LANES) {
    DlRec e[CH];
    int cc[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int p = p0 + u * DL_LANES + s;
      cc[u] = -1;
      if (p < total) {
        while (cl.pre[c + 1] <= p) ++c;
        cc[u] = c;
        e[u] = d.dl_rec[cl.qb[c] + (p - cl.pre[c])];
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      bool acc = false;
      if (cc[u] >= 0) {
        const int k = cc[u];
        const unsigned tag = cl.tag[k];
        const V3<double> xj{e[u].x, e[u].y, e[u].z};
        bool same = e[u].tag == tag && tag != DL_TAG_FAR;
        if (!same && (e[u].tag == DL_TAG_FAR || tag == DL_TAG_FAR))  // another cell of the bucket?
          same = dl_coord(xj.x, d.dl_org[0], d.dl_inv) == gx + k % 3 - 1 &&
                 dl_coord(xj.y, d.dl_org[1], d.dl_inv) == gy + (k / 3) % 3 - 1 &&
                 dl_coord(xj.z, d.dl_org[2], d.dl_inv) == gz + k / 9 - 1;
        acc = same && e[u].i != (int)i && r2_exact(xi, xj) < rs2;
      }
      const unsigned grp = (unsigned)(__ballot(acc) >> gshift) & gmask;
      const int at = nc + __popc(grp & ((1u << s) - 1u));
      if (acc && at < DNBR_CAP) d.dnbr[(long)at * N + t] = e[u].i;
      nc += __popc(grp);
    }
  }
  if (s == 0) {
    d.dnbr_cnt[t] = min(nc, DNBR_CAP);
    if (nc > DNBR_CAP) atomicOr(&d.flags[FLAG_DIP_OVF], 1u);
    st3(d.xb, N, i, xi);
  }
}

// Dipole force and field of one particle from its list, written to slot 0 of
// the FP64 partial sums (the only slot in this mode). W lanes per particle:
// lane s takes entries s, s + W, s + 2W, ... in order with U partners' gathers
// in flight; the W partial sums are added by a fixed xor tree.
constexpr int DL_WALK_LANES = 8;
constexpr int DL_WALK_FLIGHT = 2;
__device__ __forceinline__ void dipole_list_walk(const Dev& d, unsigned blk) {
  constexpr int W = DL_WALK_LANES, U = DL_WALK_FLIGHT;
  const long N = d.n;
  long i, t;
  {
    const long g = threadIdx.x / W, per = blockDim.x / W;
    if (d.i_lo == 0 && d.i_hi == N) {
      t = (long)xcd_block(blk, gridDim.x) * per + g;
      if (t >= N) return;
      i = d.dl_sorted[t];
    } else {
      i = d.i_lo + (long)blk * per + g;
      if (i >= d.i_hi) return;
      t = d.dl_pos[i];
    }
  }
  const int s = threadIdx.x % W;
  const double* own = static_cast<const double*>(__builtin_assume_aligned(d.xm + 8 * i, 64));
  const V3<double> xi{own[0], own[1], own[2]}, mi{own[3], own[4], own[5]};
  const double rd2 = d.dcut * d.dcut, C = d.C;
  V3<double> F{0.0, 0.0, 0.0}, B{0.0, 0.0, 0.0};
  // partner j's position and moment from the interleaved copy (one line,
  // three 16-byte loads)
  auto partner = [&](int j, V3<double>& xj, V3<double>& mj) {
    const double2* p = reinterpret_cast<const double2*>(d.xm + 8 * (long)j);
    const double2 a = p[0], b = p[1], c = p[2];
    xj = V3<double>{a.x, a.y, b.x};
    mj = V3<double>{b.y, c.x, c.y};
  };
  auto pair = [&](V3<double> xj, V3<double> mj) {
    const double r2 = r2_exact(xi, xj);
    if (!(r2 < rd2)) return;
    const V3<double> r = xi - xj;
    const double rinv = rsqrt_nr(r2);  // hardware estimate, two Newton steps
    const double rinv3 = rinv * rinv * rinv, rinv5 = rinv3 * rinv * rinv;
    const double a = dot(mi, r), b = dot(mj, r), cmm = dot(mi, mj);
    F = F + (3.0 * C * rinv5) * ((cmm * r + b * mi + a * mj) - (5.0 * a * b * rinv * rinv) * r);
    B = B + (3.0 * C * b * rinv5) * r - (C * rinv3) * mj;
  };
  const int nc = d.dnbr_cnt[t];
  int k = s;
  for (; k + (U - 1) * W < nc; k += U * W) {
    int j[U];
    V3<double> xj[U], mj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = d.dnbr[(long)(k + u * W) * N + t];
#pragma unroll
    for (int u = 0; u < U; ++u) partner(j[u], xj[u], mj[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) pair(xj[u], mj[u]);
  }
  for (; k < nc; k += W) {
    V3<double> xj, mj;
    partner(d.dnbr[(long)k * N + t], xj, mj);
    pair(xj, mj);
  }
  double v[6] = {F.x, F.y, F.z, B.x, B.y, B.z};
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1)
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] += __shfl_xor(v[c], o, 64);
  if (s == 0) {
    double* p = d.dpart;
#pragma unroll
    for (int c = 0; c < 6; ++c) p[c * N + i] = v[c];
  }
}

}  // namespace rodmx
