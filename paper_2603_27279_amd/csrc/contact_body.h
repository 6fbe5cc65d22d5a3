// Contact search and force: Hookean normal repulsion k (r_c - r) between
// particles of the same member that are closer than r_c and not bonded within
// the exclusion depth (Methods, "Contact", with the normal-only Hookean law of
// the workloads).
//
// Candidates come from the hashed cell list of the current time level (cell
// side r_c) plus the short list of particles whose cell was full. The search is
// lane-parallel: half a wavefront serves one particle, lane c (0..26) scans
// neighbouring cell c, whose count and first slots (each slot holds the
// particle's position and tag) are fetched in one round trip. Lanes whose hash
// bucket repeats a lower lane's bucket stand down, so no pair is seen twice.
// The selection r^2 = (dx dx + dy dy) + dz dz < r_c^2 uses explicitly rounded
// FP64 operations (no contraction), so the pair set is exactly that of a
// brute-force search with the same expression. Pair terms are summed exactly
// as 128-bit integers (see Fix128): the result does not depend on the order in
// which particles were inserted into their cells.
#pragma once
#include "rod_internal.h"
#include "rod_math.h"
#include "fixsum.h"

namespace rodmx {


__device__ __forceinline__ double r2_exact(V3<double> a, V3<double> b) {
  double dx = __dsub_rn(a.x, b.x), dy = __dsub_rn(a.y, b.y), dz = __dsub_rn(a.z, b.z);
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

enum ContactOut { OUT_FORCE = 0, OUT_ENERGY = 1, OUT_PAIRS = 2 };

// Cell slots fetched together with the cell count in the lane-parallel search.
// With cells of side r_c and particles about r_c apart a cell rarely holds more.
constexpr int CELL_SPEC = 2;

// One pass of the search; what is produced depends on `OUT`.
template <int OUT>
__device__ __forceinline__ void contact_pass(const Dev& d, long blk, int* pairs, int cap,
                                             int* count) {
  const long N = d.n;
  const int lane = threadIdx.x & 31;
  const long i = d.i_lo + ((blk * blockDim.x + threadIdx.x) >> 5);
  const bool pv = i < d.i_hi;
  const long ii = pv ? i : d.i_lo;
  const V3<double> xi = ld3(d.x, N, ii);
  const int mem = d.mem[ii], rod = d.rod[ii];
  const int mb = d.mrange[2 * mem], me = d.mrange[2 * mem + 1];
  const double rc2 = d.rc * d.rc;
  const int cx = cell_coord(xi.x, d.inv_cell), cy = cell_coord(xi.y, d.inv_cell),
            cz = cell_coord(xi.z, d.inv_cell);
  const int c = lane < 27 ? lane : 0;
  const unsigned key = cell_hash(cx + c % 3 - 1, cy + (c / 3) % 3 - 1, cz + c / 9 - 1, mem,
                                   d.cell_mask);
  const CellTab tab = cell_tab(d, d.step[d.lc]);  // cell list of the level being evaluated
  bool scan = pv && lane < 27;
  for (int o = 0; o < 26; ++o) {  // stand down if a lower lane has the same bucket
    unsigned ko = __shfl(key, o, 32);
    if (o < lane && ko == key) scan = false;
  }
  Fix3 f{};
  Fix128 fe{};
  auto take = [&](int j, int rj, V3<double> xj) {
    if (j == (int)i || j < mb || j >= me) return;
    if (rj == rod && abs(j - (int)i) <= d.depth) return;
    const double r2 = r2_exact(xi, xj);
    if (!(r2 < rc2)) return;
    if (OUT == OUT_PAIRS) {
      if (j > (int)i) {
        int p = atomicAdd(count, 1);
        if (p < cap) { pairs[2 * p] = (int)i; pairs[2 * p + 1] = j; }
      }
      return;
    }
    const double r = sqrt(r2);
    const double ov = d.rc - r;
    const double s = (d.kc * ov) / r;
    fix_add(f, s * (xi - xj), d.fix_scale[0], d.flags + FLAG_CONTACT_RANGE);
    if (OUT == OUT_ENERGY)  // each pair seen from both ends
      fix_add(fe, 0.25 * d.kc * ov * ov, d.fix_scale[2], d.flags + FLAG_CONTACT_RANGE);
  };
  if (scan) {
    // The first CELL_SPEC slots travel with the count (stale entries past the
    // count are ignored); fuller cells take a second round trip.
    const CellSlot* sl = tab.slot + (long)key * CELL_CAP;
    const int nb = min(tab.cnt[key], CELL_CAP);
    CellSlot e[CELL_SPEC];
#pragma unroll
    for (int s = 0; s < CELL_SPEC; ++s) e[s] = sl[s];
#pragma unroll
    for (int s = 0; s < CELL_SPEC; ++s)
      if (s < nb) take((int)(e[s].tag & 0xffffffffll), (int)(e[s].tag >> 32),
                       V3<double>{e[s].x, e[s].y, e[s].z});
    for (int s = CELL_SPEC; s < nb; ++s) {
      const CellSlot f = sl[s];
      take((int)(f.tag & 0xffffffffll), (int)(f.tag >> 32), V3<double>{f.x, f.y, f.z});
    }
  }
  if (pv && lane == 27) {  // particles whose cell was full
    const int no = min(*tab.ovf_cnt, OVF_CAP);
    for (int o = 0; o < no; ++o) {
      const int j = tab.ovf[o];
      take(j, d.rod[j], ld3(d.x, N, j));
    }
  }
  if (OUT == OUT_PAIRS) return;
  f = half_sum(f);
  if (OUT == OUT_ENERGY) fe = half_sum(fe);
  if (pv && lane == 0) {
    st3(d.cF, N, i, fix_value(f, d.fix_inv[0]));
    if (OUT == OUT_ENERGY) d.cE[i] = fix_value(fe, d.fix_inv[2]);
  }
}

// Visit every particle listed in the 27 cells around xi (each bucket once) and
// in the overflow list: take(j, rod of j, position of j). The hash is linear in
// the cell's x index, so the three cells of a row along x are consecutive
// buckets after the row's base; the cells are taken three rows at a time, which
// keeps nine counts in flight instead of 27 (the register peak of the walk).
template <class Take>
__device__ __forceinline__ void for_cell_candidates(const Dev& d, const CellTab& tab, V3<double> xi,
                                                    int mem, Take&& take) {
  const long N = d.n;
  const unsigned mask = d.cell_mask;
  const int cx = cell_coord(xi.x, d.inv_cell), cy = cell_coord(xi.y, d.inv_cell),
            cz = cell_coord(xi.z, d.inv_cell);
  unsigned base[9];  // bucket of cell (cx - 1, cy + r % 3 - 1, cz + r / 3 - 1)
#pragma unroll
  for (int r = 0; r < 9; ++r) base[r] = cell_hash(cx - 1, cy + r % 3 - 1, cz + r / 3 - 1, mem, mask);
#pragma unroll
  for (int r0 = 0; r0 < 9; r0 += 3) {
    int nc[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) nc[u] = tab.cnt[(base[r0 + u / 3] + u % 3) & mask];
#pragma unroll
    for (int u = 0; u < 9; ++u) {
      const int c = 3 * r0 + u;  // cells in the order x fastest, then y, then z
      const unsigned key = (base[c / 3] + c % 3) & mask;
      int nb = min(nc[u], CELL_CAP);
#pragma unroll
      for (int o = 0; o < c; ++o)
        if (((base[o / 3] + o % 3) & mask) == key) nb = 0;  // bucket already visited
      const CellSlot* sl = tab.slot + (long)key * CELL_CAP;
      for (int s = 0; s < nb; ++s) {
        const CellSlot e = sl[s];
        take((int)(e.tag & 0xffffffffll), (int)(e.tag >> 32), V3<double>{e.x, e.y, e.z});
      }
    }
  }
  const int no = min(*tab.ovf_cnt, OVF_CAP);
  for (int o = 0; o < no; ++o) {
    const int j = tab.ovf[o];
    take(j, d.rod[j], ld3(d.x, N, j));
  }
}

// Variant for large systems: one thread per particle walks the 27 cells, each
// non-empty cell costing one round trip for the slots it actually holds. Same
// selection, same exact sums.
template <int OUT>
__device__ __forceinline__ void contact_thread(const Dev& d, long blk) {
  const long N = d.n;
  const long i = d.i_lo + blk * blockDim.x + threadIdx.x;
  if (i >= d.i_hi) return;
  const V3<double> xi = ld3(d.x, N, i);
  const int mem = d.mem[i], rod = d.rod[i];
  const int mb = d.mrange[2 * mem], me = d.mrange[2 * mem + 1];
  const double rc2 = d.rc * d.rc;
  Fix3 f{};
  Fix128 fe{};
  for_cell_candidates(d, cell_tab(d, d.step[d.lc]), xi, mem, [&](int j, int rj, V3<double> xj) {
    if (j == (int)i || j < mb || j >= me) return;
    if (rj == rod && abs(j - (int)i) <= d.depth) return;
    const double r2 = r2_exact(xi, xj);
    if (!(r2 < rc2)) return;
    const double r = sqrt(r2);
    const double ov = d.rc - r;
    const double s = (d.kc * ov) / r;
    fix_add(f, s * (xi - xj), d.fix_scale[0], d.flags + FLAG_CONTACT_RANGE);
    if (OUT == OUT_ENERGY)
      fix_add(fe, 0.25 * d.kc * ov * ov, d.fix_scale[2], d.flags + FLAG_CONTACT_RANGE);
  });
  st3(d.cF, N, i, fix_value(f, d.fix_inv[0]));
  if (OUT == OUT_ENERGY) d.cE[i] = fix_value(fe, d.fix_inv[2]);
}

// Contact force of a large system from per-particle candidate lists (Verlet
// lists with a skin). A list holds every non-excluded particle of the member
// closer than r_c + skin when it was built. It is rebuilt from the cells at the
// first step of every rod_step call and whenever some particle has moved more
// than NBR_MOVE * skin since the last build; the displacement check runs where
// particles move. Between builds every pair closer than r_c is still listed, so
// the exact selection r^2 < r_c^2 and the fixed-point sums give the cell
// search's result bit for bit, while a step reads a short contiguous list
// instead of 27 scattered cells. A particle with more than NBR_CAP candidates
// searches the cells every step.
__device__ __forceinline__ void contact_listed(const Dev& d, long blk, bool build) {
  const long N = d.n;
  const long i = d.i_lo + blk * blockDim.x + threadIdx.x;
  if (i >= d.i_hi) return;
  const V3<double> xi = ld3(d.x, N, i);
  const int cnt = build ? -1 : d.nbr_cnt[i];
  const double rc2 = d.rc * d.rc;
  Fix3 f{};
  auto force = [&](V3<double> xj) {
    const double r2 = r2_exact(xi, xj);
    if (!(r2 < rc2)) return;
    const double r = sqrt(r2);
    const double s = (d.kc * (d.rc - r)) / r;
    fix_add(f, s * (xi - xj), d.fix_scale[0], d.flags + FLAG_CONTACT_RANGE);
  };
  if (cnt >= 0) {  // the list: its entries passed the exclusions when it was built
    for (int k = 0; k < cnt; ++k) force(ld3(d.x, N, d.nbr[(long)k * N + i]));
  } else {
    // a rebuild, or a list that overflowed: search the cells (the member range
    // and rod id are read only here, so that a walk is one round trip)
    const int mem = d.mem[i], rod = d.rod[i];
    const int mb = d.mrange[2 * mem], me = d.mrange[2 * mem + 1];
    auto excluded = [&](int j, int rj) {
      return j == (int)i || j < mb || j >= me || (rj == rod && abs(j - (int)i) <= d.depth);
    };
    const CellTab tab = cell_tab(d, d.step[d.lc]);
    if (build) {
      const double rs = d.rc + d.skin, rs2 = rs * rs;
      int nc = 0;
      for_cell_candidates(d, tab, xi, mem, [&](int j, int rj, V3<double> xj) {
        if (excluded(j, rj)) return;
        if (r2_exact(xi, xj) < rs2) {
          if (nc < NBR_CAP) d.nbr[(long)nc * N + i] = j;
          ++nc;
        }
        force(xj);
      });
      d.nbr_cnt[i] = nc <= NBR_CAP ? nc : -1;
      st3(d.xb, N, i, xi);
    } else {
      for_cell_candidates(d, tab, xi, mem, [&](int j, int rj, V3<double> xj) {
        if (!excluded(j, rj)) force(xj);
      });
    }
  }
  st3(d.cF, N, i, fix_value(f, d.fix_inv[0]));
}

// ---------------------------------------------------------------- Hertz-Mindlin
// One Hertz-Mindlin contact of particle i with j (Methods, "Contact"; the
// constants of two equal elastic spheres of diameter r_c), seen from i, with
// n = (x_i - x_j) / r, overlap delta = r_c - r and a = sqrt(R* delta):
//   normal force max(0, 4/3 E* a delta - g_n v_n), v the velocity of i's
//     contact point relative to j's: (v_i - v_j) - r/2 (w_i + w_j) x n;
//   tangential displacement s: zero for a new contact (sp null), else the
//     previous s turned into the current tangent plane at its length, plus
//     v_t dt; force -8 G* a s - g_t v_t, limited to mu times the normal force
//     (s then holds the limited force);
//   force on i F_n n + F_t, torque on i (and on j) (-r/2 n) x F_t.
// Seen from j every vector changes sign exactly, so the pair's forces cancel.
struct HmOut {
  V3<double> F, T, s;
  double e;  // normal elastic energy 8/15 E* sqrt(R*) delta^(5/2)
};

__device__ __forceinline__ HmOut hm_pair(const Dev& d, V3<double> xi, V3<double> xj, double r2,
                                         V3<double> vi, V3<double> vj, V3<double> wi,
                                         V3<double> wj, const V3<double>* sp) {
  HmOut o;
  const V3<double> dx = xi - xj;
  const double r = sqrt(r2);
  const V3<double> n = (1.0 / r) * dx;
  const double delta = d.rc - r;
  const double a = sqrt(d.hm_Rs * delta);
  const double kn = 4.0 / 3.0 * d.hm_Es * a, kt = 8.0 * d.hm_Gs * a;
  const V3<double> vrel = (vi - vj) - (0.5 * r) * cross(wi + wj, n);
  const double vn = dot(vrel, n);
  const V3<double> vt = vrel - vn * n;
  const double Fn = fmax(0.0, kn * delta - d.hm_gn * vn);
  V3<double> sv{0.0, 0.0, 0.0};
  if (sp) {
    const V3<double> p = *sp;
    V3<double> st = p - dot(p, n) * n;
    const double lt = sqrt(dot(st, st)), lp = sqrt(dot(p, p));
    if (lt > 0.0) st = (lp / lt) * st;
    sv = st + d.dt * vt;
  }
  V3<double> Ft = (-kt) * sv - d.hm_gt * vt;
  const double ft = sqrt(dot(Ft, Ft)), fmx = d.hm_mu * Fn;
  if (ft > fmx) {
    Ft = (fmx / ft) * Ft;
    sv = (-1.0 / kt) * (Ft + d.hm_gt * vt);
  }
  o.F = Fn * n + Ft;
  o.T = cross((-0.5 * r) * n, Ft);
  o.s = sv;
  o.e = 8.0 / 15.0 * d.hm_Es * sqrt(d.hm_Rs) * delta * delta * sqrt(delta);
  return o;
}

// Hertz-Mindlin contact force and torque of particle i, one thread per
// particle: the candidates are those of the Hookean search (same exact
// selection and exclusions), from the 27 cells, or in large systems from the
// particle's candidate list (built from the cells when `build`, see
// contact_listed). Each contact is looked up among i's contacts of the
// previous level (plane (L - 1) & 1, from level hist_from on); when the
// evaluation records, i's contacts of this level go to plane L & 1 in the
// order found (lookups go by partner, so the order never shows). Force and
// torque are summed in fixed point, so cells and lists give the same bits.
template <int OUT>
__device__ __forceinline__ void contact_hm_thread(const Dev& d, long blk, bool build) {
  const long N = d.n;
  const long i = d.i_lo + blk * blockDim.x + threadIdx.x;
  if (i >= d.i_hi) return;
  const V3<double> xi = ld3(d.x, N, i), vi = ld3(d.v, N, i), wi = ld3(d.w, N, i);
  const double rc2 = d.rc * d.rc;
  const long long L = d.step[d.lc];
  const long pp = (long)((L - 1) & 1), pc = (long)(L & 1);
  const int np = L >= d.hist_from ? min(d.hc_cnt[pp * N + i], HM_CAP) : 0;
  const int* pj = d.hc_j + pp * HM_CAP * N;
  const double* ps = d.hc_s + pp * 3 * HM_CAP * N;
  int* cj = d.hc_j + pc * HM_CAP * N;
  double* cs = d.hc_s + pc * 3 * HM_CAP * N;
  Fix3 f{}, t{};
  Fix128 fe{};
  int cnt = 0;
  auto visit = [&](int j, V3<double> xj) {
    const double r2 = r2_exact(xi, xj);
    if (!(r2 < rc2)) return;
    V3<double> sprev;
    bool found = false;
    for (int k = 0; k < np; ++k)
      if (pj[(long)k * N + i] == j) {
        sprev = V3<double>{ps[(long)k * N + i], ps[(long)(HM_CAP + k) * N + i],
                           ps[(long)(2 * HM_CAP + k) * N + i]};
        found = true;
      }
    const HmOut o = hm_pair(d, xi, xj, r2, vi, ld3(d.v, N, j), wi, ld3(d.w, N, j),
                            found ? &sprev : nullptr);
    fix_add(f, o.F, d.fix_scale[0], d.flags + FLAG_CONTACT_RANGE);
    fix_add(t, o.T, d.fix_scale[1], d.flags + FLAG_CONTACT_RANGE);
    if (OUT == OUT_ENERGY)  // each pair seen from both ends
      fix_add(fe, 0.5 * o.e, d.fix_scale[2], d.flags + FLAG_CONTACT_RANGE);
    if (d.hist_write) {
      if (cnt < HM_CAP) {
        cj[(long)cnt * N + i] = j;
        cs[(long)cnt * N + i] = o.s.x;
        cs[(long)(HM_CAP + cnt) * N + i] = o.s.y;
        cs[(long)(2 * HM_CAP + cnt) * N + i] = o.s.z;
      }
      ++cnt;
    }
  };
  // one cell walk (which also rebuilds the candidate list when asked) or one
  // list walk, so that the contact arithmetic is generated twice, not more
  const bool lists = OUT != OUT_ENERGY && d.use_lists;
  const int listed = lists && !build ? d.nbr_cnt[i] : -1;
  if (listed >= 0) {
    for (int k = 0; k < listed; ++k) {
      const int j = d.nbr[(long)k * N + i];
      visit(j, ld3(d.x, N, j));
    }
  } else {
    // the cell search (member range and rod id read only here)
    const int mem = d.mem[i], rod = d.rod[i];
    const int mb = d.mrange[2 * mem], me = d.mrange[2 * mem + 1];
    auto excluded = [&](int j, int rj) {
      return j == (int)i || j < mb || j >= me || (rj == rod && abs(j - (int)i) <= d.depth);
    };
    const bool mk = lists && build;
    const double rs = d.rc + d.skin, rs2 = rs * rs;
    int nc = 0;
    for_cell_candidates(d, cell_tab(d, L), xi, mem, [&](int j, int rj, V3<double> xj) {
      if (excluded(j, rj)) return;
      if (mk && r2_exact(xi, xj) < rs2) {
        if (nc < NBR_CAP) d.nbr[(long)nc * N + i] = j;
        ++nc;
      }
      visit(j, xj);
    });
    if (mk) {
      d.nbr_cnt[i] = nc <= NBR_CAP ? nc : -1;
      st3(d.xb, N, i, xi);
    }
  }
  if (d.hist_write) {
    d.hc_cnt[pc * N + i] = min(cnt, HM_CAP);
    if (cnt > HM_CAP) atomicOr(&d.flags[FLAG_HM_OVF], 1u);
  }
  st3(d.cF, N, i, fix_value(f, d.fix_inv[0]));
  st3(d.cT, N, i, fix_value(t, d.fix_inv[1]));
  if (OUT == OUT_ENERGY) d.cE[i] = fix_value(fe, d.fix_inv[2]);
}

// The same, lane-parallel for systems below the list size: half a wavefront
// per particle, lane c (0..26) scanning neighbouring cell c and lane 27 the
// overflow list, as in contact_pass. A contact's slot in this level's plane is
// taken with an LDS counter per particle, so slots fill in whatever order the
// lanes find contacts; lookups go by partner and the sums are fixed point, so
// nothing depends on that order. Workgroups of 256 threads (8 particles).
template <int OUT>
__device__ __forceinline__ void contact_hm_lanes(const Dev& d, long blk) {
  __shared__ int slots[8];
  const long N = d.n;
  const int lane = threadIdx.x & 31, sub = threadIdx.x >> 5;
  const long i = d.i_lo + ((blk * blockDim.x + threadIdx.x) >> 5);
  const bool pv = i < d.i_hi;
  const long ii = pv ? i : d.i_lo;
  const V3<double> xi = ld3(d.x, N, ii), vi = ld3(d.v, N, ii), wi = ld3(d.w, N, ii);
  const int mem = d.mem[ii], rod = d.rod[ii];
  const int mb = d.mrange[2 * mem], me = d.mrange[2 * mem + 1];
  const double rc2 = d.rc * d.rc;
  const long long L = d.step[d.lc];
  const long pp = (long)((L - 1) & 1), pc = (long)(L & 1);
  const int np = pv && L >= d.hist_from ? min(d.hc_cnt[pp * N + ii], HM_CAP) : 0;
  const int* pj = d.hc_j + pp * HM_CAP * N;
  const double* ps = d.hc_s + pp * 3 * HM_CAP * N;
  int* cj = d.hc_j + pc * HM_CAP * N;
  double* cs = d.hc_s + pc * 3 * HM_CAP * N;
  const int cx = cell_coord(xi.x, d.inv_cell), cy = cell_coord(xi.y, d.inv_cell),
            cz = cell_coord(xi.z, d.inv_cell);
  const int c = lane < 27 ? lane : 0;
  const unsigned key = cell_hash(cx + c % 3 - 1, cy + (c / 3) % 3 - 1, cz + c / 9 - 1, mem,
                                 d.cell_mask);
  const CellTab tab = cell_tab(d, L);
  bool scan = pv && lane < 27;
  for (int o = 0; o < 26; ++o) {  // stand down if a lower lane has the same bucket
    unsigned ko = __shfl(key, o, 32);
    if (o < lane && ko == key) scan = false;
  }
  if (lane == 0) slots[sub] = 0;
  __syncthreads();
  Fix3 f{}, t{};
  Fix128 fe{};
  auto take = [&](int j, int rj, V3<double> xj) {
    if (j == (int)i || j < mb || j >= me) return;
    if (rj == rod && abs(j - (int)i) <= d.depth) return;
    const double r2 = r2_exact(xi, xj);
    if (!(r2 < rc2)) return;
    V3<double> sprev;
    bool found = false;
    for (int k = 0; k < np; ++k)
      if (pj[(long)k * N + i] == j) {
        sprev = V3<double>{ps[(long)k * N + i], ps[(long)(HM_CAP + k) * N + i],
                           ps[(long)(2 * HM_CAP + k) * N + i]};
        found = true;
      }
    const HmOut o = hm_pair(d, xi, xj, r2, vi, ld3(d.v, N, j), wi, ld3(d.w, N, j),
                            found ? &sprev : nullptr);
    fix_add(f, o.F, d.fix_scale[0], d.flags + FLAG_CONTACT_RANGE);
    fix_add(t, o.T, d.fix_scale[1], d.flags + FLAG_CONTACT_RANGE);
    if (OUT == OUT_ENERGY)
      fix_add(fe, 0.5 * o.e, d.fix_scale[2], d.flags + FLAG_CONTACT_RANGE);
    if (d.hist_write) {
      const int k = atomicAdd(&slots[sub], 1);
      if (k < HM_CAP) {
        cj[(long)k * N + i] = j;
        cs[(long)k * N + i] = o.s.x;
        cs[(long)(HM_CAP + k) * N + i] = o.s.y;
        cs[(long)(2 * HM_CAP + k) * N + i] = o.s.z;
      }
    }
  };
  if (scan) {
    const CellSlot* sl = tab.slot + (long)key * CELL_CAP;
    const int nb = min(tab.cnt[key], CELL_CAP);
    for (int q = 0; q < nb; ++q) {
      const CellSlot e = sl[q];
      take((int)(e.tag & 0xffffffffll), (int)(e.tag >> 32), V3<double>{e.x, e.y, e.z});
    }
  }
  if (pv && lane == 27) {  // particles whose cell was full
    const int no = min(*tab.ovf_cnt, OVF_CAP);
    for (int o = 0; o < no; ++o) {
      const int j = tab.ovf[o];
      take(j, d.rod[j], ld3(d.x, N, j));
    }
  }
  __syncthreads();
  f = half_sum(f);
  t = half_sum(t);
  if (OUT == OUT_ENERGY) fe = half_sum(fe);
  if (pv && lane == 0) {
    st3(d.cF, N, i, fix_value(f, d.fix_inv[0]));
    st3(d.cT, N, i, fix_value(t, d.fix_inv[1]));
    if (OUT == OUT_ENERGY) d.cE[i] = fix_value(fe, d.fix_inv[2]);
    if (d.hist_write) {
      const int cnt = slots[sub];
      d.hc_cnt[pc * N + i] = min(cnt, HM_CAP);
      if (cnt > HM_CAP) atomicOr(&d.flags[FLAG_HM_OVF], 1u);
    }
  }
}

// Whether the lists must be rebuilt this step: asked by the host, or some
// particle moved too far since the last build (flag of the level's parity).
__device__ __forceinline__ bool lists_stale(const Dev& d, int build) {
  return build || d.rebuild[d.step[d.lc] & 1] != 0u;
}


// Workgroups of 256 threads that a pass over [i_lo, i_hi) takes: lane-parallel
// (32 lanes per particle), and the variant chosen for this system size.
inline unsigned contact_lane_blocks(const Dev& d) {
  return (unsigned)((32 * (d.i_hi - d.i_lo) + 255) / 256);
}
inline unsigned contact_blocks(const Dev& d) {
  return d.n >= CONTACT_LANES_MAX_N ? (unsigned)((d.i_hi - d.i_lo + 255) / 256)
                                    : contact_lane_blocks(d);
}

}  // namespace rodmx
