// Dipole-dipole interaction with a cutoff (Methods, "Magnetic interactions",
// truncated as the paper's pair style truncates it): particle i feels the
// particles j of its member with r^2 = (dx dx + dy dy) + dz dz < dcut^2 (exact
// FP64 selection, as in the contact search), through the same pair law as the
// all-pairs sum. Each particle keeps a Verlet list of the member's particles
// closer than dcut + skin, rebuilt with the contact lists (first step of a
// call, or when a particle has moved more than NBR_MOVE * skin), found by
// walking the hashed cells within dcell_k cells of its own.
//
// The sums run in list order, which follows the cell table's insertion order:
// results agree to rounding between runs and launch forms, not bit for bit.
#pragma once
#include "contact_body.h"

namespace rodmx {

// Squared distance from coordinate x to the cell interval [g h, (g + 1) h),
// widened by a relative 1e-9 so that rounding never drops a cell.
__device__ __forceinline__ double gap2(double x, int g, double h) {
  const double lo = (double)g * h, hi = lo + h, e = 1e-9 * h;
  const double t = fmax(fmax(lo - e - x, x - hi - e), 0.0);
  return t * t;
}

// Visit every particle listed in the cells within k cells of xi's cell that
// come closer to xi than sqrt(reach2), and in the overflow list: take(j,
// position of j). A slot counts only when visited from its own cell, so a hash
// bucket shared by two cells of the walk never yields a particle twice; other
// members' particles are left to the caller.
template <class Take>
__device__ __forceinline__ void for_cells_within(const Dev& d, const CellTab& tab, V3<double> xi,
                                                 int mem, int k, double reach2, Take&& take) {
  const long N = d.n;
  const double h = 1.0 / d.inv_cell;
  const int cx = cell_coord(xi.x, d.inv_cell), cy = cell_coord(xi.y, d.inv_cell),
            cz = cell_coord(xi.z, d.inv_cell);
  for (int gz = cz - k; gz <= cz + k; ++gz) {
    const double dz2 = gap2(xi.z, gz, h);
    if (dz2 > reach2) continue;
    for (int gy = cy - k; gy <= cy + k; ++gy) {
      const double dyz2 = dz2 + gap2(xi.y, gy, h);
      if (dyz2 > reach2) continue;
      for (int gx = cx - k; gx <= cx + k; ++gx) {
        if (dyz2 + gap2(xi.x, gx, h) > reach2) continue;
        const unsigned key = cell_hash(gx, gy, gz, mem, d.cell_mask);
        const int nb = min(tab.cnt[key], CELL_CAP);
        const CellSlot* sl = tab.slot + (long)key * CELL_CAP;
        for (int s = 0; s < nb; ++s) {
          const CellSlot e = sl[s];
          if (cell_coord(e.x, d.inv_cell) != gx || cell_coord(e.y, d.inv_cell) != gy ||
              cell_coord(e.z, d.inv_cell) != gz)
            continue;
          take((int)(e.tag & 0xffffffffll), V3<double>{e.x, e.y, e.z});
        }
      }
    }
  }
  const int no = min(*tab.ovf_cnt, OVF_CAP);
  for (int o = 0; o < no; ++o) {
    const int j = tab.ovf[o];
    take(j, ld3(d.x, N, j));
  }
}

// Dipole force and field of particle i from its neighbours within the cutoff,
// written to slot 0 of the FP64 partial sums (the only slot in this mode).
__device__ __forceinline__ void dipole_listed(const Dev& d, long blk, bool build) {
  const long N = d.n;
  const long i = d.i_lo + blk * blockDim.x + threadIdx.x;
  if (i >= d.i_hi) return;
  const V3<double> xi = ld3(d.x, N, i), mi = ld3(d.mu, N, i);
  const int mem = d.mem[i];
  const int mb = d.mrange[2 * mem], me = d.mrange[2 * mem + 1];
  const double rd2 = d.dcut * d.dcut, C = d.C;
  V3<double> F{0.0, 0.0, 0.0}, B{0.0, 0.0, 0.0};
  // partner j's position and moment from the interleaved copy (one line)
  auto partner = [&](int j, V3<double>& xj, V3<double>& mj) {
    const double* p = static_cast<const double*>(__builtin_assume_aligned(d.xm + 8 * (long)j, 64));
    xj = V3<double>{p[0], p[1], p[2]};
    mj = V3<double>{p[4], p[5], p[6]};
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
  if (build) {
    const double rs = d.dcut + d.skin, rs2 = rs * rs;
    int nc = 0;
    for_cells_within(d, cell_tab(d, d.step[d.lc]), xi, mem, d.dcell_k, rs2 * (1.0 + 1e-9),
                     [&](int j, V3<double> xj) {
      if (j == (int)i || j < mb || j >= me) return;
      if (r2_exact(xi, xj) < rs2) {
        if (nc < DNBR_CAP) d.dnbr[(long)nc * N + i] = j;
        ++nc;
      }
      V3<double> xk, mk;
      partner(j, xk, mk);
      pair(xk, mk);
    });
    d.dnbr_cnt[i] = min(nc, DNBR_CAP);
    if (nc > DNBR_CAP) atomicOr(&d.flags[FLAG_DIP_OVF], 1u);
    st3(d.xb, N, i, xi);
  } else {
    // four neighbours' gathers in flight at a time
    const int nc = d.dnbr_cnt[i];
    int k = 0;
    for (; k + 4 <= nc; k += 4) {
      int j[4];
      V3<double> xj[4], mj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) j[u] = d.dnbr[(long)(k + u) * N + i];
#pragma unroll
      for (int u = 0; u < 4; ++u) partner(j[u], xj[u], mj[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) pair(xj[u], mj[u]);
    }
    for (; k < nc; ++k) {
      V3<double> xj, mj;
      partner(d.dnbr[(long)k * N + i], xj, mj);
      pair(xj, mj);
    }
  }
  double* p = d.dpart;
  p[i] = F.x; p[N + i] = F.y; p[2 * N + i] = F.z;
  p[3 * N + i] = B.x; p[4 * N + i] = B.y; p[5 * N + i] = B.z;
}

}  // namespace rodmx
