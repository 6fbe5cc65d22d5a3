// Periodic dipole-dipole interaction by Ewald summation: the long-range solvers
// the paper's LAMMPS implementation offers beside its truncated pair style
// (Introduction; SI "Magnetic dipoles"). Each member is its own periodic system
// in the box L_x x L_y x L_z, with conducting boundaries at infinity. With
// C = mu0/4pi and splitting parameter a:
//   real space, pairs closer than rc by the minimum image (rc <= L/2):
//     F_i += C [(mi.mj) C(r) r + C(r) ((mj.r) mi + (mi.r) mj) - (mi.r)(mj.r) D(r) r]
//     B_i += C [C(r) (mj.r) r - B(r) mj],
//     B, C, D the erfc-screened forms of 1/r^3, 3/r^5, 15/r^7;
//   reciprocal space, k = 2 pi n / L over the half space of 0 < |n|^2 <= kmax^2
//   (k and -k give equal terms), with S(k) = sum_j (mj.k) exp(i k.x_j):
//     F_i += 2 (4 pi C / V) g(k) (mi.k) k Im[exp(i k.x_i) S*(k)]
//     B_i -= 2 (4 pi C / V) g(k) k Re[exp(i k.x_i) S*(k)],  g = exp(-k^2/4a^2)/k^2;
//   self: B_i += C 4 a^3 / (3 sqrt(pi)) m_i.
// The torque is m_i x B_i (in the particle kernels' gather) and the energy
// -1/2 sum m_i.B_i. FP64, except on the mixed path, which takes the real-space
// pair law and the reciprocal phases and per-thread sums in FP32 (as that
// path's other pair arithmetic), from FP64 phase arguments, with FP64 sums
// across lanes, chunks and rows; its real-space separations and cutoff test
// are FP32 from the positions' offsets to their cells' centres when every
// axis is at least seven cells wide and no cell is wider than rc (FP64
// otherwise).
//
// Data flow of one evaluation (all on one stream, no atomics in any sum; ten
// launches):
//   bin:     each particle's cell (side >= rc / 3, member-major numbering) and
//            its place in the cell (an atomic count);
//   scan:    first sorted position of every cell (one workgroup);
//   scatter: particles grouped by cell; rank: each cell's particles by index
//            (so the sums below run in a fixed order); pack: an interleaved
//            copy of wrapped position and moment in sorted order;
//   real:    8 (FP64: 16) lanes per sorted position walk the 7 x 7 x 7 neighbouring
//            cells that come within rc (every cell of an axis under seven
//            cells wide), their sums added by a fixed xor tree; writes F, B;
//   sk:      partial structure factors of 256-particle chunks, one thread per
//            segment of up to 8 k vectors along a row;
//   sreduce: S(k) of each member, its chunks added in a fixed order;
//   kspace:  eight waves per 64 sorted positions, each wave its own rows of
//            k vectors, their partial sums added in a fixed order; add to F, B.
#include <type_traits>

#include "rod.h"
#include "rod_internal.h"
#include "rod_math.h"

namespace rodmx {

constexpr int EW_BLOCK = 256;

// Coordinate wrapped into [0, L).
__device__ __forceinline__ double ew_wrap(double x, double L) {
  double u = x - L * floor(x / L);
  if (u >= L) u -= L;
  if (u < 0.0) u += L;
  return u;
}

// Cell index along one axis (a non-finite coordinate lands in cell 0).
__device__ __forceinline__ int ew_cell_of(double u, double L, int nc) {
  const double t = u * ((double)nc / L);
  return t >= 0.0 && t < (double)nc ? (int)t : (t >= (double)nc ? nc - 1 : 0);
}

__global__ __launch_bounds__(EW_BLOCK) void k_ew_bin(Dev d) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const long N = d.n;
  const int cx = ew_cell_of(ew_wrap(d.x[i], d.box[0]), d.box[0], d.ew_nc[0]);
  const int cy = ew_cell_of(ew_wrap(d.x[N + i], d.box[1]), d.box[1], d.ew_nc[1]);
  const int cz = ew_cell_of(ew_wrap(d.x[2 * N + i], d.box[2]), d.box[2], d.ew_nc[2]);
  const int cell = d.mem[i] * d.ew_ncell + (cz * d.ew_nc[1] + cy) * d.ew_nc[0] + cx;
  d.ew_cell[i] = cell;
  d.ew_slot[i] = atomicAdd(&d.ew_cnt[cell], 1);
}

// Exclusive prefix sums of cnt[0..total) into start[0..total]; one workgroup of
// 1024 threads, each scanning a contiguous segment.
__global__ __launch_bounds__(1024) void k_ew_scan(const int* cnt, int* start, int total) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (total + 1023) / 1024;
  const int b = min(t * per, total), e = min(b + per, total);
  int s = 0;
  for (int k = b; k < e; ++k) s += cnt[k];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t > 0 ? part[t - 1] : 0;
  for (int k = b; k < e; ++k) {
    start[k] = run;
    run += cnt[k];
  }
  if (t == 1023) start[total] = part[1023];
}

// Particles grouped by cell, in the arbitrary order of the counting slots.
__global__ __launch_bounds__(EW_BLOCK) void k_ew_scatter(Dev d) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  d.ew_tmp[d.ew_start[d.ew_cell[i]] + d.ew_slot[i]] = (int)i;
}

// Each cell's particles in ascending index: a particle's place in its cell is
// the number of the cell's particles with a smaller index (one thread per
// particle reads its cell's group, which its neighbours read too).
__global__ __launch_bounds__(EW_BLOCK) void k_ew_rank(Dev d) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int c = d.ew_cell[i];
  const int b = d.ew_start[c], e = d.ew_start[c + 1];
  int r = 0;
  for (int q = b; q < e; ++q) r += d.ew_tmp[q] < (int)i;
  d.ew_sorted[b + r] = (int)i;
}

// Wrapped positions and moments in sorted order, one 64-byte record each.
__global__ __launch_bounds__(EW_BLOCK) void k_ew_pack(Dev d) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.n) return;
  const long N = d.n;
  const long i = d.ew_sorted[p];
  double* o = d.ew_xm + 8 * p;
  o[0] = ew_wrap(d.x[i], d.box[0]);
  o[1] = ew_wrap(d.x[N + i], d.box[1]);
  o[2] = ew_wrap(d.x[2 * N + i], d.box[2]);
  o[3] = 0.0;
  o[4] = d.mu[i];
  o[5] = d.mu[N + i];
  o[6] = d.mu[2 * N + i];
  o[7] = 0.0;
  if (d.ew_xf) {  // the mixed path's record: offset from the cell's centre, FP32
    const int loc = d.ew_cell[i] % d.ew_ncell;
    const int nx = d.ew_nc[0], ny = d.ew_nc[1];
    const int cc[3] = {loc % nx, (loc / nx) % ny, loc / (nx * ny)};
    float* f = d.ew_xf + 8 * p;
    for (int a = 0; a < 3; ++a)
      f[a] = (float)(o[a] - ((double)cc[a] + 0.5) * (d.box[a] / d.ew_nc[a]));
    f[3] = 0.0f;
    for (int a = 0; a < 3; ++a) f[4 + a] = d.muf[a * N + i];
    f[7] = 0.0f;
  }
}

// Neighbouring cell offsets along an axis of nc cells of side >= rc / EW_REACH:
// -EW_REACH .. EW_REACH, or every cell of the axis once when it has fewer than
// 2 EW_REACH + 1 of them.
__device__ __forceinline__ void ew_offsets(int nc, int& lo, int& hi) {
  if (nc >= 2 * EW_REACH + 1) {
    lo = -EW_REACH;
    hi = EW_REACH;
  } else {
    lo = 0;
    hi = nc - 1;
  }
}

// Real-space force and field: EW_RL lanes per sorted position, lane l taking
// every EW_RL-th particle of each neighbouring cell; the lanes' sums are added
// by a fixed xor tree, so the result does not depend on scheduling. The image
// shift, the separation and the cutoff test are FP64, except on the mixed path
// with every axis wide (FP32 from cell offsets, below). The pair
// law runs in R: FP64 with 1/r from the refined reciprocal square root, r =
// r^2 / r (no FP64 square root or division per pair); on the mixed path FP32
// from the separation rounded once (the pair arithmetic of that path), each
// lane's sums in FP32 and their tree in FP64.
// lanes per sorted position: 8 on the mixed path (FP32 walk; 16 lanes took
// 0.75 ms per walk where 8 take 0.70), 16 on the FP64 path (2.82 against 2.95
// ms per evaluation)
template <class R> constexpr int ew_rl() { return sizeof(R) == 4 ? 8 : 16; }

// erfc(x), x >= 0, on the mixed path: the Chebyshev-fitted form of Numerical
// Recipes' erfcc, erfc(x) = t exp(-x^2 + P(t)) with t = 1 / (1 + x/2) and P of
// degree 9, whose fractional error stays below 1.2e-7 for every x >= 0. exp(-x^2)
// is the pair law's own factor ex, so only exp(P) (-1.3 < P <= 0) is taken
// here, as a base-2 exponential with the coefficients prescaled by log2(e).
constexpr double EW_LOG2E = 1.4426950408889634;
__device__ __forceinline__ float erfc_fit(float x, float ex) {
  constexpr float c0 = (float)(-1.26551223 * EW_LOG2E), c1 = (float)(1.00002368 * EW_LOG2E),
                  c2 = (float)(0.37409196 * EW_LOG2E), c3 = (float)(0.09678418 * EW_LOG2E),
                  c4 = (float)(-0.18628806 * EW_LOG2E), c5 = (float)(0.27886807 * EW_LOG2E),
                  c6 = (float)(-1.13520398 * EW_LOG2E), c7 = (float)(1.48851587 * EW_LOG2E),
                  c8 = (float)(-0.82215223 * EW_LOG2E), c9 = (float)(0.17087277 * EW_LOG2E);
  const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.5f, x, 1.0f));
  float q = __builtin_fmaf(c9, t, c8);
  q = __builtin_fmaf(q, t, c7);
  q = __builtin_fmaf(q, t, c6);
  q = __builtin_fmaf(q, t, c5);
  q = __builtin_fmaf(q, t, c4);
  q = __builtin_fmaf(q, t, c3);
  q = __builtin_fmaf(q, t, c2);
  q = __builtin_fmaf(q, t, c1);
  q = __builtin_fmaf(q, t, c0);
  return (t * ex) * __builtin_amdgcn_exp2f(q);
}

// The screened pair law: C (mm Cf r + Cf (dmj mi + dmi mj) - dmi dmj Df r) to
// F and C (Cf dmj r - Bf mj) to B, with Bf, Cf, Df the erfc-screened 1/r^3,
// 3/r^5, 15/r^7 (file header). The FP32 form takes exp(-(a r)^2) with the
// rounding of (a r)^2 put back to first order (its exact low part from an FMA),
// and erfc from the fit above.
template <class R>
__device__ __forceinline__ void ew_pair(V3<R> r, R r2, V3<R> mi, V3<R> mj, R a, R sp, R C,
                                        V3<R>& F, V3<R>& B) {
  R ri, ex, ec, ar2;
  if constexpr (sizeof(R) == 8) {
    ri = rsqrt_nr(r2);  // hardware estimate, two Newton steps
  } else {
    ri = __builtin_amdgcn_rsqf(r2);
  }
  const R rr = r2 * ri, ar = a * rr;
  ar2 = ar * ar;
  if constexpr (sizeof(R) == 8) {
    ex = exp(-ar2);
    ec = erfc(ar);
  } else {
    const float lo = __builtin_fmaf(ar, ar, -ar2);
    ex = expf(-ar2);
    ex = __builtin_fmaf(-lo, ex, ex);
    ec = erfc_fit(ar, ex);
  }
  const R ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2;
  const R Bf = (ec + sp * rr * ex) * ri3;
  const R Cf = (R(3) * ec + sp * rr * (R(3) + R(2) * ar2) * ex) * ri5;
  const R Df = (R(15) * ec + sp * rr * (R(15) + R(10) * ar2 + R(4) * ar2 * ar2) * ex) *
               (ri5 * ri2);
  const R dmi = dot(mi, r), dmj = dot(mj, r), mm = dot(mi, mj);
  F = F + C * ((mm * Cf) * r + Cf * (dmj * mi + dmi * mj) - (dmi * dmj * Df) * r);
  B = B + C * ((Cf * dmj) * r - Bf * mj);
}

template <class R>
__global__ __launch_bounds__(EW_BLOCK) void k_ew_real(Dev d) {
  constexpr int EW_RL = ew_rl<R>();
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long p = t / EW_RL;
  const int sub = (int)(t % EW_RL);
  const bool pv = p < d.n;
  const long N = d.n;
  const long pp = pv ? p : 0;
  const double* rec = d.ew_xm + 8 * pp;
  const V3<double> xi{rec[0], rec[1], rec[2]}, mi{rec[4], rec[5], rec[6]};
  const int i = d.ew_sorted[pp];
  const int cell = d.ew_cell[i];
  const int nx = d.ew_nc[0], ny = d.ew_nc[1], nz = d.ew_nc[2];
  const int mem = cell / d.ew_ncell;
  const int loc = cell - mem * d.ew_ncell;
  const int cx = loc % nx, cy = (loc / nx) % ny, cz = loc / (nx * ny);
  const double Lx = d.box[0], Ly = d.box[1], Lz = d.box[2];
  // minimum image by the reciprocal lengths: a shift that rounding could make
  // differ from that of a division only for |r_a| near L_a / 2, where the
  // distance is at least rc and the pair is left out either way
  const double iLx = 1.0 / Lx, iLy = 1.0 / Ly, iLz = 1.0 / Lz;
  const double a = d.ew_alpha, rc2 = d.ew_rc * d.ew_rc, C = d.C;
  const double sp = 2.0 * a * 0.56418958354775628695;  // 2 a / sqrt(pi)
  const R aR = (R)a, spR = (R)sp, CR = (R)C;
  const V3<R> miR = cvt<R>(mi);
  V3<R> FR{R(0), R(0), R(0)}, BR{R(0), R(0), R(0)};
  int lx, hx, ly, hy, lz, hz;
  ew_offsets(nx, lx, hx);
  ew_offsets(ny, ly, hy);
  ew_offsets(nz, lz, hz);
  // Along an axis of at least 2 EW_REACH + 1 cells each neighbouring cell is
  // visited once, at offset o from the particle's own: its particles' image
  // nearest the particle is shifted by a whole box length when cell + o leaves
  // the box (a pair closer than rc <= L/2 has no other image that close), and a
  // cell whose slab lies farther than rc from the particle is skipped. Narrower
  // axes take the minimum image of each pair and skip nothing.
  const bool wx = nx < 2 * EW_REACH + 1, wy = ny < 2 * EW_REACH + 1, wz = nz < 2 * EW_REACH + 1;
  const double hxs = Lx / nx, hys = Ly / ny, hzs = Lz / nz;
  const double reach2 = rc2 * (1.0 + 1e-9);  // widened so that rounding never drops a cell
  auto gap = [](double x, int u, double h, bool w) {
    const double g = w ? 0.0 : fmax(fmax((double)u * h - x, x - (double)(u + 1) * h), 0.0);
    return g * g;
  };
  // Mixed path, every axis wide: separations in FP32 from the offsets of the
  // positions to their cells' centres, r = (o_i - o_j) - (cell offset) h, the
  // cell part taken once per neighbouring cell (it holds the image shift).
  // Each term is at most |r| + h and rounded once, so r carries a few ulp of
  // |r| + h, the size of the FP32 pair arithmetic's own error; the cutoff test
  // is then FP32 too.
  // (cells no wider than rc, as they are unless the per-axis cell count is
  // capped in a box far larger than rc: the error then stays within a few ulp
  // of |r| + 2 rc)
  const double rc_ = d.ew_rc;
  const bool f32walk = sizeof(R) == 4 && !(wx || wy || wz) && hxs <= rc_ && hys <= rc_ &&
                       hzs <= rc_;
  if constexpr (sizeof(R) == 4) {
    if (f32walk) {
      const float4 fi = pv ? *reinterpret_cast<const float4*>(d.ew_xf + 8 * pp)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
      const float rc2f = (float)rc2;
      for (int oz = lz; oz <= hz && pv; ++oz) {
        const int uz = cz + oz, gz = (uz + nz) % nz;
        const double gz2 = gap(xi.z, uz, hzs, false);
        if (gz2 > reach2) continue;
        const float dz = fi.z - (float)((double)oz * hzs);
        for (int oy = ly; oy <= hy; ++oy) {
          const int uy = cy + oy, gy = (uy + ny) % ny;
          const double gyz2 = gz2 + gap(xi.y, uy, hys, false);
          if (gyz2 > reach2) continue;
          const float dy = fi.y - (float)((double)oy * hys);
          for (int ox = lx; ox <= hx; ++ox) {
            const int ux = cx + ox, gx = (ux + nx) % nx;
            if (gyz2 + gap(xi.x, ux, hxs, false) > reach2) continue;
            const float dx = fi.x - (float)((double)ox * hxs);
            const int cc = mem * d.ew_ncell + (gz * ny + gy) * nx + gx;
            const int qe = d.ew_start[cc + 1];
            for (int q = d.ew_start[cc] + sub; q < qe; q += EW_RL) {
              if (q == p) continue;
              const float* rj = d.ew_xf + 8 * (long)q;
              const float4 oj = *reinterpret_cast<const float4*>(rj);
              const V3<float> r{dx - oj.x, dy - oj.y, dz - oj.z};
              const float r2 = __builtin_fmaf(r.z, r.z, __builtin_fmaf(r.y, r.y, r.x * r.x));
              if (!(r2 < rc2f)) continue;
              const float4 mj = *reinterpret_cast<const float4*>(rj + 4);
              ew_pair<float>(r, r2, miR, V3<float>{mj.x, mj.y, mj.z}, aR, spR, CR, FR, BR);
            }
          }
        }
      }
    }
  }
  // The FP64 walk, compiled once without the minimum image (every axis wide
  // enough) and once with it, so the common case carries no per-pair selects.
  auto walk = [&](auto narrow) {
    constexpr bool NW = decltype(narrow)::value;
    for (int oz = lz; oz <= hz && pv; ++oz) {
      const int uz = cz + oz, gz = (uz + nz) % nz;
      const double gz2 = gap(xi.z, uz, hzs, NW && wz);
      if (gz2 > reach2) continue;
      const double sz = NW && wz ? 0.0 : (uz < 0 ? Lz : (uz >= nz ? -Lz : 0.0));
      for (int oy = ly; oy <= hy; ++oy) {
        const int uy = cy + oy, gy = (uy + ny) % ny;
        const double gyz2 = gz2 + gap(xi.y, uy, hys, NW && wy);
        if (gyz2 > reach2) continue;
        const double sy = NW && wy ? 0.0 : (uy < 0 ? Ly : (uy >= ny ? -Ly : 0.0));
        for (int ox = lx; ox <= hx; ++ox) {
          const int ux = cx + ox, gx = (ux + nx) % nx;
          if (gyz2 + gap(xi.x, ux, hxs, NW && wx) > reach2) continue;
          const double sx = NW && wx ? 0.0 : (ux < 0 ? Lx : (ux >= nx ? -Lx : 0.0));
          const int cc = mem * d.ew_ncell + (gz * ny + gy) * nx + gx;
          const int qe = d.ew_start[cc + 1];
          for (int q = d.ew_start[cc] + sub; q < qe; q += EW_RL) {
            if (q == p) continue;
            const double* rj = d.ew_xm + 8 * (long)q;
            V3<double> r{(xi.x - rj[0]) + sx, (xi.y - rj[1]) + sy, (xi.z - rj[2]) + sz};
            if constexpr (NW) {
              if (wx) r.x -= Lx * rint(r.x * iLx);  // minimum image
              if (wy) r.y -= Ly * rint(r.y * iLy);
              if (wz) r.z -= Lz * rint(r.z * iLz);
            }
            const double r2 = dot(r, r);
            if (!(r2 < rc2)) continue;
            const V3<double> mj{rj[4], rj[5], rj[6]};
            ew_pair<R>(cvt<R>(r), (R)r2, miR, cvt<R>(mj), aR, spR, CR, FR, BR);
          }
        }
      }
    }
  };
  if (wx || wy || wz)
    walk(std::true_type{});
  else if (!f32walk)
    walk(std::false_type{});
  V3<double> F = cvt<double>(FR), B = cvt<double>(BR);
#pragma unroll
  for (int o = EW_RL / 2; o > 0; o >>= 1) {
    F.x += __shfl_xor(F.x, o); F.y += __shfl_xor(F.y, o); F.z += __shfl_xor(F.z, o);
    B.x += __shfl_xor(B.x, o); B.y += __shfl_xor(B.y, o); B.z += __shfl_xor(B.z, o);
  }
  if (!pv || sub != 0) return;
  B = B + d.ew_self * mi;
  double* o = d.dpart;
  o[i] = F.x; o[N + i] = F.y; o[2 * N + i] = F.z;
  o[3 * N + i] = B.x; o[4 * N + i] = B.y; o[5 * N + i] = B.z;
}

// The k vectors come in segments of at most EW_SEG consecutive vectors of one
// row (fixed n_x, n_y; n_z rising by one), so that exp(i k.x) along a segment
// follows from its first value by repeated rotation through exp(i dkz z),
// dkz = 2 pi / L_z: one sincos per segment instead of per vector (the rotation
// adds an error of a few ulp per step).

// Partial structure factors: block (segment block, chunk); thread = one
// segment; the chunk's particles (at most EW_BLOCK sorted positions of one
// member) with their rotation exp(i dkz z) staged in LDS and read as
// broadcasts.
// exp(i ph) as R: FP64 directly; FP32 from the argument reduced modulo 2 pi in
// FP64 (|k.x| reaches a few hundred radians, where an FP32 argument alone
// would lose 1e-5 of the phase).
template <class R>
__device__ __forceinline__ void ew_phase(double ph, R& sn, R& cs) {
  if constexpr (sizeof(R) == 8) {
    sincos(ph, &sn, &cs);
  } else {
    constexpr double two_pi = 6.283185307179586477, inv_two_pi = 0.15915494309189533577;
    sincosf((float)(ph - two_pi * rint(ph * inv_two_pi)), &sn, &cs);
  }
}

template <class R>
__global__ __launch_bounds__(EW_BLOCK) void k_ew_sk(Dev d) {
  __shared__ double sx[8 * EW_BLOCK];
  const int K = d.ew_K;
  const int sg = blockIdx.x * EW_BLOCK + threadIdx.x;
  const int ch = blockIdx.y;
  const int b = d.ew_chunks[3 * ch], e = d.ew_chunks[3 * ch + 1];
  const int p = b + threadIdx.x;
  if (p < e) {
    const double* rec = d.ew_xm + 8 * (long)p;
    double* o = sx + 8 * threadIdx.x;
    for (int c = 0; c < 3; ++c) {
      o[c] = rec[c];
      o[3 + c] = rec[4 + c];
    }
    sincos(d.ew_dkz * rec[2], &o[7], &o[6]);  // cos, sin of dkz z
  }
  __syncthreads();
  if (sg >= d.ew_SEG) return;
  const int k0 = d.ew_seg[2 * sg], nk = d.ew_seg[2 * sg + 1];
  const double* kv = d.ew_k + 4 * (long)k0;
  const double kx = kv[0], ky = kv[1], kz = kv[2], dkz = d.ew_dkz;
  R Sr[EW_SEG], Si[EW_SEG];
#pragma unroll
  for (int m = 0; m < EW_SEG; ++m) Sr[m] = Si[m] = R(0);
  const int n = e - b;
  for (int q = 0; q < n; ++q) {
    const double* r = sx + 8 * q;
    R sn, cs;
    ew_phase<R>(kx * r[0] + ky * r[1] + kz * r[2], sn, cs);
    R mk = (R)(kx * r[3] + ky * r[4] + kz * r[5]);
    const R dm = (R)(dkz * r[5]), rc = (R)r[6], rs = (R)r[7];
#pragma unroll
    for (int m = 0; m < EW_SEG; ++m) {
      if (m < nk) {
        Sr[m] += mk * cs;
        Si[m] += mk * sn;
      }
      const R c2 = cs * rc - sn * rs;
      sn = sn * rc + cs * rs;
      cs = c2;
      mk += dm;
    }
  }
  double* o = d.ew_Sp + 2 * ((long)ch * K + k0);
#pragma unroll
  for (int m = 0; m < EW_SEG; ++m)
    if (m < nk) {
      o[2 * m] = (double)Sr[m];
      o[2 * m + 1] = (double)Si[m];
    }
}

// S(k) of every member from its chunks' partial sums, times the vector's
// weight (the only use of S(k) is weighted): EW_SR lanes per (member, k), lane
// l adding every EW_SR-th chunk in order, their sums added by a fixed xor tree.
constexpr int EW_SR = 8;
__global__ __launch_bounds__(EW_BLOCK) void k_ew_sreduce(Dev d) {
  const int K = d.ew_K;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long u = t / EW_SR;
  const int l = (int)(t % EW_SR);
  const bool valid = u < (long)d.M * K;
  const long uu = valid ? u : 0;
  const int m = (int)(uu / K), kk = (int)(uu % K);
  double Sr = 0.0, Si = 0.0;
  if (valid)
    for (int ch = d.ew_chunk_off[m] + l; ch < d.ew_chunk_off[m + 1]; ch += EW_SR) {
      const double* s = d.ew_Sp + 2 * ((long)ch * K + kk);
      Sr += s[0];
      Si += s[1];
    }
#pragma unroll
  for (int o = EW_SR / 2; o > 0; o >>= 1) {
    Sr += __shfl_xor(Sr, o);
    Si += __shfl_xor(Si, o);
  }
  if (!valid || l != 0) return;
  const double c = d.ew_k[4 * (long)kk + 3];
  d.ew_S[2 * uu] = c * Sr;
  d.ew_S[2 * uu + 1] = c * Si;
}

// Reciprocal-space force and field. Block = 64 sorted positions of one chunk
// (one per lane; blockIdx.y picks which 64 of its 256) x 8 waves: wave w takes
// every 8th row of k vectors (fixed n_x, n_y), so that a row's vectors and the
// member's weighted S(k) are the same for the whole wave (scalar loads), and
// exp(i k.x) follows along each run of EW_SEG vectors from one sincos by
// rotation through exp(i dkz z). Along a row only k_z changes, so the k_x and
// k_y parts of the sums are taken once per row. The 8 partial sums of a particle are then added
// in wave order through LDS.
constexpr int EW_KP = 64;  // particles per kspace block, one per lane
constexpr int EW_KL = 8;   // waves per kspace block, each its own rows
constexpr int EW_KBLOCK = EW_KP * EW_KL;
template <class R>
__global__ __launch_bounds__(EW_KBLOCK) void k_ew_kspace(Dev d) {
  __shared__ double red[6 * EW_KBLOCK];
  const long N = d.n;
  const int K = d.ew_K;
  const int ch = blockIdx.x;
  const int b = d.ew_chunks[3 * ch], e = d.ew_chunks[3 * ch + 1], mem = d.ew_chunks[3 * ch + 2];
  const int pl = threadIdx.x % EW_KP;
  const int kl = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / EW_KP));
  const int p = b + (int)blockIdx.y * EW_KP + pl;
  const bool pv = p < e;
  V3<double> xi{0.0, 0.0, 0.0}, mi{0.0, 0.0, 0.0};
  if (pv) {
    const double* rec = d.ew_xm + 8 * (long)p;
    xi = V3<double>{rec[0], rec[1], rec[2]};
    mi = V3<double>{rec[4], rec[5], rec[6]};
  }
  double rs_, rc_;
  sincos(d.ew_dkz * xi.z, &rs_, &rc_);
  const R rs = (R)rs_, rc = (R)rc_;
  const R mdz = (R)(mi.z * d.ew_dkz);
  V3<double> F{0.0, 0.0, 0.0}, B{0.0, 0.0, 0.0};
  const double* S = d.ew_S + 2 * (long)mem * K;
  for (int rw = kl; rw < d.ew_ROWS; rw += EW_KL) {
    const int k0 = d.ew_row[2 * rw], nk = d.ew_row[2 * rw + 1];
    const double* kv = d.ew_k + 4 * (long)k0;
    const double* sk = S + 2 * (long)k0;
    const double kx = kv[0], ky = kv[1];
    R mk = (R)(mi.x * kx + mi.y * ky + mi.z * kv[2]);
    R sn = R(0), cs = R(1);
    // sums along the row: a = m.k Im(conj(S) e^{ikx}) and g = Re(conj(S) e^{ikx}),
    // each also weighted by k_z
    R A = R(0), Az = R(0), G = R(0), Gz = R(0);
    for (int m = 0; m < nk; ++m) {
      const R Sr = (R)sk[2 * m], Si = (R)sk[2 * m + 1];
      const double kzd = kv[4 * m + 2];
      const R kzm = (R)kzd;
      // the phase restarts where the structure factors' runs of EW_SEG start
      // (every EW_SEG vectors of a row), with the same operations, so that a
      // particle's own part of S(k) meets the same bits of exp(i k.x) and its
      // self term cancels to rounding
      if (m % EW_SEG == 0) ew_phase<R>(kx * xi.x + ky * xi.y + kzd * xi.z, sn, cs);
      const R a = mk * (sn * Sr - cs * Si);
      const R g = cs * Sr + sn * Si;
      A += a;
      Az += a * kzm;
      G += g;
      Gz += g * kzm;
      const R c2 = cs * rc - sn * rs;
      sn = sn * rc + cs * rs;
      cs = c2;
      mk += mdz;
    }
    F.x += kx * (double)A;
    F.y += ky * (double)A;
    F.z += (double)Az;
    B.x -= kx * (double)G;
    B.y -= ky * (double)G;
    B.z -= (double)Gz;
  }
  double* o6 = red + 6 * threadIdx.x;
  o6[0] = F.x; o6[1] = F.y; o6[2] = F.z; o6[3] = B.x; o6[4] = B.y; o6[5] = B.z;
  __syncthreads();
  if (kl != 0 || !pv) return;
  double t[6] = {0, 0, 0, 0, 0, 0};
  for (int l = 0; l < EW_KL; ++l)
    for (int c = 0; c < 6; ++c) t[c] += red[6 * (l * EW_KP + pl) + c];
  const int i = d.ew_sorted[p];
  double* o = d.dpart;
  o[i] += t[0]; o[N + i] += t[1]; o[2 * N + i] += t[2];
  o[3 * N + i] += t[3]; o[4 * N + i] += t[4]; o[5 * N + i] += t[5];
}

hipError_t launch_ewald(const Dev& d, const hipEvent_t* ev_real, hipStream_t s, const hipEvent_t* ev) {
  const int total = d.M * d.ew_ncell;
  const unsigned pg = (unsigned)((d.n + EW_BLOCK - 1) / EW_BLOCK);
  hipError_t e = launch_fill_i32(d.ew_cnt, total, 0, s);
  if (e != hipSuccess) return e;
  // the event pair (timing mode) brackets the whole sequence
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_ew_bin, dim3(pg), dim3(EW_BLOCK), 0, s, d);
  hipLaunchKernelGGL(k_ew_scan, dim3(1), dim3(1024), 0, s, (const int*)d.ew_cnt, d.ew_start, total);
  hipLaunchKernelGGL(k_ew_scatter, dim3(pg), dim3(EW_BLOCK), 0, s, d);
  hipLaunchKernelGGL(k_ew_rank, dim3(pg), dim3(EW_BLOCK), 0, s, d);
  hipLaunchKernelGGL(k_ew_pack, dim3(pg), dim3(EW_BLOCK), 0, s, d);
  if (d.muf)  // the mixed path
    launch_k(ev_real, k_ew_real<float>,
             dim3((unsigned)((ew_rl<float>() * d.n + EW_BLOCK - 1) / EW_BLOCK)), dim3(EW_BLOCK), s, d);
  else
    launch_k(ev_real, k_ew_real<double>,
             dim3((unsigned)((ew_rl<double>() * d.n + EW_BLOCK - 1) / EW_BLOCK)), dim3(EW_BLOCK), s, d);
  const dim3 skg((unsigned)((d.ew_SEG + EW_BLOCK - 1) / EW_BLOCK), (unsigned)d.ew_TC);
  if (d.muf)  // the mixed path: phases and per-thread sums in FP32
    hipLaunchKernelGGL(k_ew_sk<float>, skg, dim3(EW_BLOCK), 0, s, d);
  else
    hipLaunchKernelGGL(k_ew_sk<double>, skg, dim3(EW_BLOCK), 0, s, d);
  static_assert(EW_BLOCK % EW_SR == 0, "sreduce lane groups within a wave");
  hipLaunchKernelGGL(k_ew_sreduce,
                     dim3((unsigned)(((long)d.M * d.ew_K * EW_SR + EW_BLOCK - 1) / EW_BLOCK)),
                     dim3(EW_BLOCK), 0, s, d);
  static_assert(EW_CHUNK % EW_KP == 0, "kspace block shape");
  const dim3 kg((unsigned)d.ew_TC, EW_CHUNK / EW_KP);
  if (d.muf)
    hipLaunchKernelGGL(k_ew_kspace<float>, kg, dim3(EW_KBLOCK), 0, s, d);
  else
    hipLaunchKernelGGL(k_ew_kspace<double>, kg, dim3(EW_KBLOCK), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev) return hipEventRecord(ev[1], s);
  return hipSuccess;
}

}  // namespace rodmx
