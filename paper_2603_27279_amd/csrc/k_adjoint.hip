// Reverse pass of the time step: gradients of a function of the final state
// with respect to the body dipoles, the field table and the initial state,
// by checkpoint-and-recompute through the recorded steps. All adjoint
// arithmetic is FP64.
//
// One step n -> n+1 of the forward loop (SI "Equations of motion") is
//   v' = v + h F/m, x1 = x + dt v', w' = w + h T/I, q1 = Rich(q, w')   (pre)
//   (F1, T1) = forces(x1, q1, v', w', m_body, field[n+1])             (forces)
//   v1 = v' + h F1/m, w1 = w' + h T1/I                                 (post)
// with h = dt/2, for free particles (clamped ones never move; driven ones
// follow a prescribed rotation). The reverse step takes the cotangent of the
// state at n+1 and returns the one at n:
//   post: v'-bar = v1-bar, F1-bar += h v1-bar / m (likewise for w, T);
//   forces: vector-Jacobian products of every force term (below);
//   pre: the Richardson update differentiated step by step, x-bar passes
//        through, v'-bar += dt x1-bar, F-bar = h v'-bar / m.
// Force terms:
//   bonds   - exact Jacobian columns of the bond function from forward-mode
//             dual numbers (11 inputs: r_f, q1, q2), contracted with the
//             bond's cotangent (F-bar_k - F-bar_{k+1}, T-bar_k + T-bar_{k+1},
//             T-bar_k - T-bar_{k+1});
//   dipoles - closed-form Hessian-vector products of the pair potential
//             U(r, a, b) = (a.b)/r^3 - 3 (a.r)(b.r)/r^5 (force = -dU/dr, field
//             = -dU/da), evaluated once with i as target and once as source;
//   Zeeman, torque m x B, damping, contact, and m = R(q) m_body - by hand.
#include "rod_adjoint.h"
#include "bond_core.h"
#include "dual.h"
#include "particle_body.h"
#include "fixsum.h"

#include <algorithm>

namespace rodmx {

enum AdjMode { ADJ_STEP = 0, ADJ_PREPARE = 1 };

__device__ __forceinline__ V3<double> ldv(const double* p, long N, long i) { return ld3(p, N, i); }

__device__ __forceinline__ Q4<double> qv(V3<double> v) { return {0.0, v.x, v.y, v.z}; }
__device__ __forceinline__ V3<double> vec(Q4<double> q) { return {q.x, q.y, q.z}; }

// ---------------------------------------------------------------- Richardson VJP
// Cotangent of the normalisation y -> y/|y|: (v - n (n.v)) / |y|.
__device__ __forceinline__ Q4<double> jn(Q4<double> y, Q4<double> v) {
  const double s = 1.0 / ::sqrt(qdot(y, y));
  const Q4<double> n = qscale(s, y);
  return qscale(s, qadd(v, qscale(-qdot(n, v), n)));
}

// Given q, the half-step angular velocity w and the cotangent of the updated
// orientation, add the cotangents of q and w.
__device__ void richardson_vjp(Q4<double> q, V3<double> w, double dt, Q4<double> qbar_new,
                               Q4<double>& qbar, V3<double>& wbar) {
  const Q4<double> p{0.0, w.x, w.y, w.z};
  const Q4<double> pc{0.0, -w.x, -w.y, -w.z};
  auto rate = [&](Q4<double> a) { return qscale(0.5, qmul(p, a)); };
  const Q4<double> y1 = qadd(q, qscale(dt, rate(q)));
  const Q4<double> q1 = qnormalize(y1);
  const Q4<double> yh = qadd(q, qscale(0.5 * dt, rate(q)));
  const Q4<double> qh = qnormalize(yh);
  const Q4<double> y2 = qadd(qh, qscale(0.5 * dt, rate(qh)));
  const Q4<double> q2 = qnormalize(y2);
  const Q4<double> yn = qadd(qscale(2.0, q2), qscale(-1.0, q1));
  const Q4<double> ybn = jn(yn, qbar_new);
  const Q4<double> yb2 = jn(y2, qscale(2.0, ybn));
  const Q4<double> yb1 = jn(y1, qscale(-1.0, ybn));
  // y2 = qh + (dt/2) 1/2 p qh
  const Q4<double> qbh = qadd(yb2, qscale(0.25 * dt, qmul(pc, yb2)));
  V3<double> wb = 0.25 * dt * vec(qmul(yb2, qconj(qh)));
  const Q4<double> ybh = jn(yh, qbh);
  // yh = q + (dt/2) 1/2 p q ;  y1 = q + dt 1/2 p q
  qbar = qadd(qbar, qadd(qadd(ybh, qscale(0.25 * dt, qmul(pc, ybh))),
                         qadd(yb1, qscale(0.5 * dt, qmul(pc, yb1)))));
  wb = wb + 0.25 * dt * vec(qmul(ybh, qconj(q))) + 0.5 * dt * vec(qmul(yb1, qconj(q)));
  wbar = wbar + wb;
}

// ---------------------------------------------------------------- local terms
// Post-kick VJP and the per-particle force terms (Zeeman, dipole torque,
// damping). S1 is the state of the level whose forces are reversed; S0 the
// state one level earlier (ADJ_STEP only).
__device__ __forceinline__ void adj_local(const Dev& d, const Adj& a, long i, const double* S0,
                                          const double* S1, int koff, int mode) {
  const long long lvl = *a.lbase + koff;
  const long N = d.n;
  const bool free_p = d.bc[i] == 0;
  const double h = 0.5 * d.dt;
  V3<double> Fe{0, 0, 0}, Te{0, 0, 0}, vb{0, 0, 0}, wb{0, 0, 0};
  if (free_p) {
    const V3<double> cv = ldv(a.cv, N, i), cw = ldv(a.cw, N, i);
    Fe = ldv(a.cF, N, i);
    Te = ldv(a.cT, N, i);
    vb = cv;
    wb = cw;
    if (mode == ADJ_STEP) {
      Fe = Fe + (h * d.minv[i]) * cv;
      Te = Te + (h * d.Iinv[i]) * cw;
      // half-step angular velocity of the step, for the Richardson VJP
      const V3<double> w0 = ldv(S0 + 10 * N, N, i), T0 = ldv(S0 + 16 * N, N, i);
      st3(a.wh, N, i, w0 + (h * d.Iinv[i]) * T0);
    }
  }
  // damping: F = -c m v', T = -c I w'
  vb = vb - (d.damping * d.mass[i]) * Fe;
  wb = wb - (d.damping * d.inertia[i]) * Te;
  const V3<double> x1 = ldv(S1, N, i);
  const V3<double> m = ldv(d.mu, N, i);
  const V3<double> Bd = ldv(S1 + 19 * N, N, i);
  const long long L = d.field_len;
  const long long row = ((lvl % L) + L) % L;
  const double* f = d.field + (row * d.M + d.mem[i]) * 12;
  const V3<double> Be{f[0] + f[3] * x1.x + f[4] * x1.y + f[5] * x1.z,
                      f[1] + f[6] * x1.x + f[7] * x1.y + f[8] * x1.z,
                      f[2] + f[9] * x1.x + f[10] * x1.y + f[11] * x1.z};
  // torque m x (B_dip + B_ext): m-bar += B x T-bar, B-bar = T-bar x m
  const V3<double> Bt = Bd + Be;
  const V3<double> hb = cross(Te, m);
  // Zeeman force G^T m: m-bar += G F-bar
  const V3<double> GF{f[3] * Fe.x + f[4] * Fe.y + f[5] * Fe.z,
                      f[6] * Fe.x + f[7] * Fe.y + f[8] * Fe.z,
                      f[9] * Fe.x + f[10] * Fe.y + f[11] * Fe.z};
  st3(a.mloc, N, i, cross(Bt, Te) + GF);
  // B_ext = B0 + G x1: x-bar += G^T B-bar
  st3(a.xloc, N, i, V3<double>{f[3] * hb.x + f[6] * hb.y + f[9] * hb.z,
                               f[4] * hb.x + f[7] * hb.y + f[10] * hb.z,
                               f[5] * hb.x + f[8] * hb.y + f[11] * hb.z});
  st3(a.h, N, i, hb);
  st3(a.Fe, N, i, Fe);
  st3(a.Te, N, i, Te);
  st3(a.vbar, N, i, vb);
  st3(a.wbar, N, i, wb);
  const double hbv[3] = {hb.x, hb.y, hb.z}, xv[3] = {x1.x, x1.y, x1.z},
               mv[3] = {m.x, m.y, m.z}, Fv[3] = {Fe.x, Fe.y, Fe.z};
  for (int k = 0; k < 3; ++k) a.fieldc[k * N + i] = hbv[k];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) a.fieldc[(3 + 3 * r + c) * N + i] = hbv[r] * xv[c] + mv[r] * Fv[c];
}

// ---------------------------------------------------------------- bonds
// One thread per (input direction, bond): column `dir` of the bond's Jacobian
// by a dual-number evaluation, contracted with the bond cotangent.
__device__ __forceinline__ void adj_bond(const Dev& d, const Adj& a, const double* S1, long t) {
  const long N = d.n;
  if (t >= 11 * N) return;
  const int dir = (int)(t / N);
  const long k = t - (long)dir * N;
  if (!(d.bflags[k] & 1)) return;
  const V3<double> Fb = ldv(a.Fe, N, k) - ldv(a.Fe, N, k + 1);
  const V3<double> Tsb = ldv(a.Te, N, k) + ldv(a.Te, N, k + 1);
  const V3<double> Tbb = ldv(a.Te, N, k) - ldv(a.Te, N, k + 1);
  const V3<double> x1 = ldv(S1, N, k), x2 = ldv(S1, N, k + 1);
  const Q4<double> q1 = ld4(S1 + 6 * N, N, k), q2 = ld4(S1 + 6 * N, N, k + 1);
  const V3<double> rref{d.bref[k], d.bref[N + k], d.bref[2 * N + k]};
  const double r0 = d.bref[3 * N + k];
  const double* K4 = d.rodK + 4 * d.rod[k];
  auto sd = [&](int c) { return dir == c ? 1.0 : 0.0; };
  V3<DD> X1{DD(x1.x), DD(x1.y), DD(x1.z)};
  V3<DD> X2{DD(x2.x, sd(0)), DD(x2.y, sd(1)), DD(x2.z, sd(2))};
  Q4<DD> Q1{DD(q1.w, sd(3)), DD(q1.x, sd(4)), DD(q1.y, sd(5)), DD(q1.z, sd(6))};
  Q4<DD> Q2{DD(q2.w, sd(7)), DD(q2.x, sd(8)), DD(q2.y, sd(9)), DD(q2.z, sd(10))};
  V3<DD> F, Ts, Tbt;
  bond_one<DD, DD>(X1, X2, Q1, Q2, rref, r0, K4, F, Ts, Tbt, nullptr);
  a.bvjp[dir * N + k] = (F.x.d * Fb.x + F.y.d * Fb.y + F.z.d * Fb.z) +
                        (Ts.x.d * Tsb.x + Ts.y.d * Tsb.y + Ts.z.d * Tsb.z) +
                        (Tbt.x.d * Tbb.x + Tbt.y.d * Tbb.y + Tbt.z.d * Tbb.z);
}

// ---------------------------------------------------------------- dipoles
// Squared distance with explicitly rounded operations: the exact selection of
// the contact search and of the dipole cutoff.
__device__ __forceinline__ double r2x(V3<double> p, V3<double> q) {
  double dx = __dsub_rn(p.x, q.x), dy = __dsub_rn(p.y, q.y), dz = __dsub_rn(p.z, q.z);
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}
// Whether pair (i, j) interacts: every pair of a member, or with a cutoff the
// pairs the forward list walk selects.
__device__ __forceinline__ bool dip_pair_on(const Dev& d, V3<double> xi, V3<double> xj) {
  return d.dcut == 0.0 || r2x(xi, xj) < d.dcut * d.dcut;
}

// Gradients of Phi = grad_r U . g + grad_a U . h with respect to r, a and b.
__device__ void phi_grad(V3<double> r, V3<double> am, V3<double> bm, V3<double> g, V3<double> hv,
                         V3<double>& dr, V3<double>& da, V3<double>& db) {
  const double u = rsqrt_nr(dot(r, r));
  const double u2 = u * u, u3 = u2 * u, u5 = u3 * u2, u7 = u5 * u2, u9 = u7 * u2;
  const double A = dot(am, bm), P = dot(am, r), Q = dot(bm, r), G = dot(r, g);
  const double Ga = dot(am, g), Gb = dot(bm, g), Hb = dot(bm, hv), Hr = dot(r, hv);
  const double cr = 15.0 * A * u7 * G - 105.0 * u9 * P * Q * G + 15.0 * u7 * (Q * Ga + P * Gb) -
                    3.0 * u5 * Hb + 15.0 * u7 * Q * Hr;
  const double ca = 15.0 * u7 * Q * G - 3.0 * u5 * Gb;
  const double cb = 15.0 * u7 * P * G - 3.0 * u5 * Ga - 3.0 * u5 * Hr;
  const double cg = -3.0 * A * u5 + 15.0 * u7 * P * Q;
  const double ch = -3.0 * u5 * Q;
  dr = cr * r + ca * am + cb * bm + cg * g + ch * hv;
  da = ca * r - (3.0 * u5 * G) * bm - (3.0 * u5 * Q) * g;
  db = cb * r - (3.0 * u5 * G) * am - (3.0 * u5 * P) * g + u3 * hv;
}

constexpr int ATJ = 256;

// LDS of the fused reverse force kernel: a dipole tile and its reduction, or
// the field-gradient reduction (different workgroups, one union).
union AdjSmem {
  double sj[12][ATJ];
  double red[4][6][64];
  double fred[12][256];
};

__device__ __forceinline__ void adj_dipole_item(const Dev& d, const Adj& a, const double* S1,
                                                const DipWork& wk, AdjSmem& sm) {
  double(*sj)[ATJ] = sm.sj;
  const long N = d.n;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = wk.i0 + lane;
  const bool act = i < wk.i1;
  V3<double> xi{0, 0, 0}, mi{0, 0, 0}, gi{0, 0, 0}, hi{0, 0, 0};
  if (act) {
    xi = ldv(S1, N, i); mi = ldv(d.mu, N, i); gi = ldv(a.Fe, N, i); hi = ldv(a.h, N, i);
  }
  V3<double> xb{0, 0, 0}, mb{0, 0, 0};
  for (int t0 = wk.j0; t0 < wk.j1; t0 += ATJ) {
    const int jn = min(ATJ, wk.j1 - t0);
    if ((int)threadIdx.x < jn) {
      const int j = t0 + threadIdx.x;
      const double* srcs[4] = {S1, d.mu, a.Fe, a.h};
      for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 3; ++c) sj[3 * s + c][threadIdx.x] = srcs[s][c * N + j];
    }
    __syncthreads();
    const int jb = wave * 64, je = min(jb + 64, jn);
    for (int jj = jb; jj < je; ++jj) {
      if (t0 + jj == i) continue;
      const V3<double> xj{sj[0][jj], sj[1][jj], sj[2][jj]};
      if (!dip_pair_on(d, xi, xj)) continue;
      const V3<double> mj{sj[3][jj], sj[4][jj], sj[5][jj]};
      const V3<double> gj{sj[6][jj], sj[7][jj], sj[8][jj]};
      const V3<double> hj{sj[9][jj], sj[10][jj], sj[11][jj]};
      V3<double> dr, da, db;
      phi_grad(xi - xj, mi, mj, gi, hi, dr, da, db);  // i as target
      xb = xb - dr;
      mb = mb - da;
      phi_grad(xj - xi, mj, mi, gj, hj, dr, da, db);  // i as source
      xb = xb + dr;
      mb = mb - db;
    }
    __syncthreads();
  }
  // (the last tile pass ended with a barrier, so the tile may be overwritten)
  const double v6[6] = {xb.x, xb.y, xb.z, mb.x, mb.y, mb.z};
  for (int k = 0; k < 6; ++k) sm.red[wave][k][lane] = v6[k];
  __syncthreads();
  if (wave == 0 && act) {
    double* p = d.dpart + (long)wk.slot * 6 * N;
    for (int k = 0; k < 6; ++k)
      p[k * N + i] = d.C * (((sm.red[0][k][lane] + sm.red[1][k][lane]) + sm.red[2][k][lane]) +
                            sm.red[3][k][lane]);
  }
}

// Small-member layout (as the forward): one wave per target, lanes striding
// over the member's sources, a fixed xor tree across lanes.
__device__ __forceinline__ void adj_dipole_small_item(const Dev& d, const Adj& a, const double* S1,
                                                      const DipWork& wk) {
  const long N = d.n;
  const int lane = threadIdx.x & 63;
  const int i = wk.i0 + (int)(threadIdx.x >> 6);
  if (i >= wk.i1) return;  // the whole wave
  const V3<double> xi = ldv(S1, N, i), mi = ldv(d.mu, N, i), gi = ldv(a.Fe, N, i),
                   hi = ldv(a.h, N, i);
  V3<double> xb{0, 0, 0}, mb{0, 0, 0};
  for (int jb = wk.j0 + lane; jb < wk.j1; jb += 2 * 64) {
    V3<double> xj[2], mj[2], gj[2], hj[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {  // loads first; out-of-range entries read source j0
      const int j = jb + 64 * u < wk.j1 ? jb + 64 * u : wk.j0;
      xj[u] = ldv(S1, N, j); mj[u] = ldv(d.mu, N, j); gj[u] = ldv(a.Fe, N, j); hj[u] = ldv(a.h, N, j);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int j = jb + 64 * u;
      if (j >= wk.j1) break;
      if (j == i || !dip_pair_on(d, xi, xj[u])) continue;
      V3<double> dr, da, db;
      phi_grad(xi - xj[u], mi, mj[u], gi, hi, dr, da, db);  // i as target
      xb = xb - dr;
      mb = mb - da;
      phi_grad(xj[u] - xi, mj[u], mi, gj[u], hj[u], dr, da, db);  // i as source
      xb = xb + dr;
      mb = mb - db;
    }
  }
  double v6[6] = {xb.x, xb.y, xb.z, mb.x, mb.y, mb.z};
#pragma unroll
  for (int k = 0; k < 6; ++k)
    for (int o = 32; o > 0; o >>= 1) v6[k] += __shfl_xor(v6[k], o);
  if (lane == 0) {
    double* p = d.dpart + (long)wk.slot * 6 * N;
    for (int k = 0; k < 6; ++k) p[k * N + i] = d.C * v6[k];
  }
}

// ---------------------------------------------------------------- contact

// x-bar_i += J(d) (F-bar_i - F-bar_j) over the contacts j of i, with
// J(d) = k [ (r_c/r - 1) I - r_c d d^T / r^3 ], d = x_i - x_j. Same search
// as the forward contact kernel (27 lanes per particle, exact sums).
__device__ __forceinline__ void adj_contact(const Dev& d, const Adj& a, const double* S1, long blk) {
  const long N = d.n;
  const int lane = threadIdx.x & 31;
  const long i = (blk * blockDim.x + threadIdx.x) >> 5;
  const bool pv = i < N;
  const long ii = pv ? i : 0;
  const V3<double> xi = ldv(S1, N, ii);
  const V3<double> gi = ldv(a.Fe, N, ii);
  const int mem = d.mem[ii], rod = d.rod[ii];
  const int mlo = d.mrange[2 * mem], mhi = d.mrange[2 * mem + 1];
  const double rc2 = d.rc * d.rc;
  const int cx = cell_coord(xi.x, d.inv_cell), cy = cell_coord(xi.y, d.inv_cell), cz = cell_coord(xi.z, d.inv_cell);
  const int c = lane < 27 ? lane : 0;
  const unsigned key = cell_hash(cx + c % 3 - 1, cy + (c / 3) % 3 - 1, cz + c / 9 - 1, mem, d.cell_mask);
  bool scan = pv && lane < 27;
  for (int o = 0; o < 26; ++o) {
    unsigned ko = __shfl(key, o, 32);
    if (o < lane && ko == key) scan = false;
  }
  Fix3 sum{};
  auto take = [&](int j, int rj, V3<double> xj) {
    if (j == (int)i || j < mlo || j >= mhi) return;
    if (rj == rod && abs(j - (int)i) <= d.depth) return;
    const double r2 = r2x(xi, xj);
    if (!(r2 < rc2)) return;
    const double r = ::sqrt(r2);
    const V3<double> dd = xi - xj;
    const V3<double> gv = gi - ldv(a.Fe, N, j);
    const double s1 = d.kc * (d.rc / r - 1.0);
    const double s2 = d.kc * d.rc * dot(dd, gv) / (r * r2);
    fix_add(sum, s1 * gv - s2 * dd, d.fix_scale[0], d.flags + FLAG_CONTACT_RANGE);
  };
  const CellTab tab = cell_tab(d, d.step[d.lc]);
  if (scan) {
    const CellSlot* sl = tab.slot + (long)key * CELL_CAP;
    const int nb = min(tab.cnt[key], CELL_CAP);
    for (int s = 0; s < nb; ++s) {
      const CellSlot e = sl[s];
      take((int)(e.tag & 0xffffffffll), (int)(e.tag >> 32), V3<double>{e.x, e.y, e.z});
    }
  }
  if (pv && lane == 27) {
    const int no = min(*tab.ovf_cnt, OVF_CAP);
    for (int o = 0; o < no; ++o) {
      const int j = tab.ovf[o];
      take(j, d.rod[j], ldv(S1, N, j));
    }
  }
  sum = half_sum(sum);
  if (pv && lane == 0) st3(d.cF, N, i, fix_value(sum, d.fix_inv[0]));
}

// ---------------------------------------------------------------- field gradient
__device__ __forceinline__ void adj_field(const Dev& d, const Adj& a, int koff, int mem,
                                          double (*red)[256]) {
  const long long lvl = *a.lbase + koff;
  const int b = d.mrange[2 * mem], e = d.mrange[2 * mem + 1];
  const long N = d.n;
  const long long L = d.field_len;
  const long long row = ((lvl % L) + L) % L;
  double s[12];
  for (int k = 0; k < 12; ++k) s[k] = 0.0;
  for (int i = b + threadIdx.x; i < e; i += blockDim.x)
    for (int k = 0; k < 12; ++k) s[k] += a.fieldc[k * N + i];
  for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 12; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 12) a.fieldbar[(row * d.M + mem) * 12 + threadIdx.x] += red[threadIdx.x][0];
}

// ---------------------------------------------------------------- fused launch
// The reverse of the force terms in one launch: dipole work items (either
// layout), bond Jacobian columns, contact, and the per-member field gradient.
// Their outputs are disjoint (slots, per-bond columns, contact x-bar, field
// table), and all read only what the local kernel wrote before.
__global__ __launch_bounds__(256) void k_adj_forces(Dev d, Adj a, const double* S1,
                                                    const DipWork* __restrict__ work, int ndip,
                                                    int nbond, int ncont, int koff) {
  __shared__ AdjSmem sm;
  int b = blockIdx.x;
  if (b < ndip) {
    if (d.dip_small) adj_dipole_small_item(d, a, S1, work[b]);
    else adj_dipole_item(d, a, S1, work[b], sm);
    return;
  }
  b -= ndip;
  if (b < nbond) {
    adj_bond(d, a, S1, (long)b * blockDim.x + threadIdx.x);
    return;
  }
  b -= nbond;
  if (b < ncont) {
    adj_contact(d, a, S1, b);
    return;
  }
  adj_field(d, a, koff, b - ncont, sm.fred);
}

// ---------------------------------------------------------------- gather
// Assemble x-bar and q-bar of the level, push m-bar through m = q m_body q*,
// then reverse the pre kick (ADJ_STEP) or write the initial-state gradients
// (ADJ_PREPARE).
__device__ __forceinline__ void adj_gather(const Dev& d, const Adj& a, long i, const double* S0,
                                           const double* S1, int nslot_max, int mode,
                                           const rod_gradients& gx) {
  const long N = d.n;
  const uint8_t bf = d.bflags[i];
  V3<double> xb = ldv(a.cx, N, i) + ldv(a.xloc, N, i);
  Q4<double> qb = ld4(a.cq, N, i);
  if (bf & 1) {  // bond (i, i+1): i is particle 1
    xb = xb - V3<double>{a.bvjp[i], a.bvjp[N + i], a.bvjp[2 * N + i]};
    qb = qadd(qb, Q4<double>{a.bvjp[3 * N + i], a.bvjp[4 * N + i], a.bvjp[5 * N + i], a.bvjp[6 * N + i]});
  }
  if (bf & 2) {  // bond (i-1, i): i is particle 2
    const long k = i - 1;
    xb = xb + V3<double>{a.bvjp[k], a.bvjp[N + k], a.bvjp[2 * N + k]};
    qb = qadd(qb, Q4<double>{a.bvjp[7 * N + k], a.bvjp[8 * N + k], a.bvjp[9 * N + k], a.bvjp[10 * N + k]});
  }
  V3<double> mbar = ldv(a.mloc, N, i);
  if (d.dipole_on) {
    const int S = d.mslots[d.mem[i]];
    for (int s = 0; s < S && s < nslot_max; ++s) {
      const double* p = d.dpart + (long)s * 6 * N;
      xb = xb + V3<double>{p[i], p[N + i], p[2 * N + i]};
      mbar = mbar + V3<double>{p[3 * N + i], p[4 * N + i], p[5 * N + i]};
    }
  }
  if (d.contact_on) xb = xb + ldv(d.cF, N, i);
  // m = q m_body q*: m_body-bar += q* m-bar q; q-bar += -2 (0, m-bar) q (0, m_body)
  const Q4<double> q1 = ld4(S1 + 6 * N, N, i);
  const V3<double> mbody = ldv(d.mb, N, i);
  st3(a.mbbar, N, i, ldv(a.mbbar, N, i) + qrot_inv(q1, mbar));
  qb = qadd(qb, qscale(-2.0, qmul(qmul(qv(mbar), q1), qv(mbody))));
  const int b = d.bc[i];
  const V3<double> z{0, 0, 0};
  if (mode == ADJ_STEP) {
    V3<double> vb = ldv(a.vbar, N, i), wb = ldv(a.wbar, N, i);
    Q4<double> qn{0, 0, 0, 0};
    if (b == 0) {
      const Q4<double> q0 = ld4(S0 + 6 * N, N, i);
      richardson_vjp(q0, ldv(a.wh, N, i), d.dt, qb, qn, wb);
      vb = vb + d.dt * xb;
      const double h = 0.5 * d.dt;
      st3(a.cx, N, i, xb);
      st3(a.cv, N, i, vb);
      st4(a.cq, N, i, qn);
      st3(a.cw, N, i, wb);
      st3(a.cF, N, i, (h * d.minv[i]) * vb);
      st3(a.cT, N, i, (h * d.Iinv[i]) * wb);
    } else {
      st3(a.cx, N, i, xb);
      st4(a.cq, N, i, b == 1 ? qb : qn);
      st3(a.cv, N, i, z);
      st3(a.cw, N, i, z);
      st3(a.cF, N, i, z);
      st3(a.cT, N, i, z);
    }
  } else {
    if (gx.x0) st3(gx.x0, N, i, xb);
    if (gx.v0) st3(gx.v0, N, i, b == 0 ? ldv(a.vbar, N, i) : z);
    if (gx.w0) st3(gx.w0, N, i, b == 0 ? ldv(a.wbar, N, i) : z);
    if (gx.q0) {
      // q was normalised from the raw input: project out the radial part.
      Q4<double> g{0, 0, 0, 0};
      if (b != 2) g = qadd(qb, qscale(-qdot(q1, qb), q1));
      st4(gx.q0, N, i, g);
    }
  }
}

// Cell list of level lvl is done with: empty it.
__device__ __forceinline__ void clear_cells_of(const Dev& d, long i, long long lvl) {
  if (!d.contact_on) return;
  const CellTab tab = cell_tab(d, lvl);
  if (i == 0) *tab.ovf_cnt = 0;
  if (i < d.n) tab.cnt[d.key[i]] = 0;
}

// One reverse level in one pass per particle, for the state S1 of level
// lbase + koff (view v, whose level counter reads that level):
//  - when S2 (the state one level later) is given, the gather of that later
//    level, which hands over the cotangents of S1 and empties its cell list;
//  - the dipole moment and cell-list entry of S1 (the force evaluation being
//    reversed needs them);
//  - the local VJPs of level koff (kicks, damping, Zeeman, torques).
// Everything a particle reads was written by earlier kernels or by its own
// thread; the cell lists of consecutive levels alternate tables.
__global__ __launch_bounds__(256) void k_adj_level(Dev v, Adj a, const double* S0, const double* S1,
                                                   const double* S2, int koff, int mode,
                                                   int nslot_max) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long N = v.n;
  const long long lvl = v.step[v.lc];
  if (S2) {
    clear_cells_of(v, i, lvl + 1);
    if (i < N) adj_gather(v, a, i, S1, S2, nslot_max, ADJ_STEP, rod_gradients{});
  }
  if (i >= N) return;
  moment_and_cell(v, i, ld4(S1 + 6 * N, N, i), ldv(S1, N, i), ldv(v.mb, N, i), v.mem[i], v.rod[i],
                  lvl);
  adj_local(v, a, i, S0, S1, koff, mode);
}

// The gather of a level on its own (the last of a segment, and the initial
// force evaluation).
__global__ __launch_bounds__(256) void k_adj_gather(Dev v, Adj a, const double* S0, const double* S1,
                                                    int nslot_max, int mode, rod_gradients gx) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  clear_cells_of(v, i, v.step[v.lc]);
  if (i < v.n) adj_gather(v, a, i, S0, S1, nslot_max, mode, gx);
}

__global__ void k_set_level(long long* p, long long v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) { p[0] = v; p[1] = v; }
}
// First level of the segment, and the counters of the reverse views.
__global__ void k_set_base(long long* p, long long* levels, int nlev, long long v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) p[0] = v;
  if (k < nlev) levels[3 * k] = levels[3 * k + 1] = levels[3 * k + 2] = v + k;
}

// ---------------------------------------------------------------- host side
template <class T>
static int adalloc(std::vector<void*>& allocs, T** p, size_t count) {
  void* q = nullptr;
  size_t bytes = std::max<size_t>(count * sizeof(T), 16);
  if (hipMalloc(&q, bytes) != hipSuccess) return rodmx_fail(ROD_E_HIP, "tape allocation failed");
  allocs.push_back(q);
  if (hipMemset(q, 0, bytes) != hipSuccess) return rodmx_fail(ROD_E_HIP, "tape memset failed");
  *p = (T*)q;
  return ROD_OK;
}

#define ACHK(expr)                                                                   \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess) return rodmx_fail(ROD_E_HIP, hipGetErrorString(_e));       \
  } while (0)
#define ATRY(expr)                   \
  do {                               \
    int _r = (expr);                 \
    if (_r != ROD_OK) return _r;     \
  } while (0)

int tape_init(Tape& t, const Dev& d, int every, int capacity, std::vector<void*>& allocs) {
  t.every = every;
  t.capacity = capacity;
  if (capacity <= 0) return ROD_OK;
  const size_t N = d.n;
  const size_t nck = (size_t)capacity / every + 1;
  Adj& a = t.a;
  double* cot = nullptr;
  ATRY(adalloc(allocs, &t.ckpt, nck * STATE_PLANES * N));
  ATRY(adalloc(allocs, &t.seg, (size_t)(every + 1) * SEG_PLANES * N));
  ATRY(adalloc(allocs, &cot, STATE_PLANES * N));
  a.cx = cot; a.cv = cot + 3 * N; a.cq = cot + 6 * N; a.cw = cot + 10 * N;
  a.cF = cot + 13 * N; a.cT = cot + 16 * N;
  ATRY(adalloc(allocs, &a.Fe, 3 * N));
  ATRY(adalloc(allocs, &a.Te, 3 * N));
  ATRY(adalloc(allocs, &a.h, 3 * N));
  ATRY(adalloc(allocs, &a.mloc, 3 * N));
  ATRY(adalloc(allocs, &a.xloc, 3 * N));
  ATRY(adalloc(allocs, &a.vbar, 3 * N));
  ATRY(adalloc(allocs, &a.wbar, 3 * N));
  ATRY(adalloc(allocs, &a.wh, 3 * N));
  ATRY(adalloc(allocs, &a.fieldc, 12 * N));
  ATRY(adalloc(allocs, &a.bvjp, 11 * N));
  ATRY(adalloc(allocs, &a.mbbar, 3 * N));
  ATRY(adalloc(allocs, &a.fieldbar, (size_t)d.field_len * d.M * 12));
  ATRY(adalloc(allocs, &a.scratch, 6 * N));
  ATRY(adalloc(allocs, &a.level, 3));
  ATRY(adalloc(allocs, &a.lbase, 1));
  ATRY(adalloc(allocs, &a.levels, 3 * (size_t)(every + 1)));
  return ROD_OK;
}

// Copy the caller's state into a recorded-state slot (STATE_PLANES N).
static int save_state(const Dev& d, double* dst, hipStream_t s) {
  const size_t N = d.n, b3 = 3 * N * sizeof(double);
  ACHK(hipMemcpyAsync(dst, d.x, b3, hipMemcpyDeviceToDevice, s));
  ACHK(hipMemcpyAsync(dst + 3 * N, d.v, b3, hipMemcpyDeviceToDevice, s));
  ACHK(hipMemcpyAsync(dst + 6 * N, d.q, 4 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
  ACHK(hipMemcpyAsync(dst + 10 * N, d.w, b3, hipMemcpyDeviceToDevice, s));
  ACHK(hipMemcpyAsync(dst + 13 * N, d.F, b3, hipMemcpyDeviceToDevice, s));
  ACHK(hipMemcpyAsync(dst + 16 * N, d.T, b3, hipMemcpyDeviceToDevice, s));
  return ROD_OK;
}

int tape_start(Tape& t, const Dev& d, hipStream_t s, int64_t step) {
  t.active = true;
  t.start_step = step;
  return save_state(d, t.ckpt, s);
}

int tape_before_step(Tape& t, const Dev& d, hipStream_t s, int64_t step) {
  const int64_t k = step - t.start_step;
  if (k >= t.capacity)
    return rodmx_fail(ROD_E_STATE, "tape capacity exceeded: raise tape_capacity or call rod_tape_begin");
  if (k > 0 && k % t.every == 0) return save_state(d, t.ckpt + (size_t)(k / t.every) * STATE_PLANES * d.n, s);
  return ROD_OK;
}

// A view of the device context whose state lives in a recorded-state slot.
static Dev view(const Dev& d, double* S, long long* level) {
  Dev v = d;
  const long N = d.n;
  v.x = S; v.v = S + 3 * N; v.q = S + 6 * N; v.w = S + 10 * N; v.F = S + 13 * N; v.T = S + 16 * N;
  v.step = level;
  return v;
}

static inline unsigned nblk(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Reverse the force evaluation of state S1 (level lbase + koff) and, in
// ADJ_STEP mode, the kicks of the step from S0: one per-particle pass (which
// first completes the later level S2 when given) and one launch for the force
// terms. The gather of S1's own level is left to the next call or to
// reverse_gather. Only device-side values vary between segments, so a full
// segment can be captured once and replayed.
static int reverse_level(Tape& t, const Dev& d, const DipWork* work, int nwork, int max_slots,
                         hipStream_t s, const double* S0, double* S1, const double* S2, int koff,
                         int mode) {
  const long N = d.n;
  Adj& a = t.a;
  Dev v = view(d, S1, a.levels + 3 * koff);
  hipLaunchKernelGGL(k_adj_level, dim3(nblk(N, 256)), dim3(256), 0, s, v, a, S0,
                     (const double*)S1, S2, koff, mode, max_slots);
  ACHK(hipGetLastError());
  const int ndip = d.dipole_on ? nwork : 0;
  const int nbond = (int)nblk(11 * N, 256);
  const int ncont = d.contact_on ? (int)nblk(32 * N, 256) : 0;
  hipLaunchKernelGGL(k_adj_forces, dim3(ndip + nbond + ncont + d.M), dim3(256), 0, s, v, a,
                     (const double*)S1, work, ndip, nbond, ncont, koff);
  ACHK(hipGetLastError());
  return ROD_OK;
}

// The gather of level lbase + koff on its own.
static int reverse_gather(Tape& t, const Dev& d, int max_slots, hipStream_t s, const double* S0,
                          double* S1, int koff, int mode, const rod_gradients& gx) {
  Adj& a = t.a;
  Dev v = view(d, S1, a.levels + 3 * koff);
  hipLaunchKernelGGL(k_adj_gather, dim3(nblk(d.n, 256)), dim3(256), 0, s, v, a, S0,
                     (const double*)S1, max_slots, mode, gx);
  ACHK(hipGetLastError());
  return ROD_OK;
}

// Recompute steps 0..len-1 of a segment from seg[0] (levels from the view's
// counters), with the forward's fused chain: pre, forces, then (kick, forces)
// per further step, and post. Each level's state goes to its own slot; the
// kick closes slot k (full-step v and w, forces, dipole field) and writes the
// advanced state into slot k + 1.
static int recompute(Tape& t, const Dev& d, int precision, const DipWork* work, int nwork,
                     hipStream_t s, int len) {
  const long N = d.n;
  const size_t SP = SEG_PLANES * (size_t)N;
  Dev v = view(d, t.seg + SP, t.a.level);
  v.src = t.seg;  // the pre kernel reads step 0 and writes step 1
  ACHK(launch_pre(v, PRE_STEP, s));
  v.src = nullptr;
  ACHK(launch_force_pass(v, precision, work, nwork, 1, s));
  for (int k = 1; k < len; ++k) {
    double* Sk = t.seg + k * SP;
    v.nx = Sk + SP;
    ACHK(launch_kick(v, Sk + 19 * N, s));
    Dev w = view(d, Sk + SP, t.a.level);
    w.lc = 3 - v.lc;
    v = w;
    ACHK(launch_force_pass(v, precision, work, nwork, 1, s));
  }
  ACHK(launch_post(v, POST_KICK, ROD_TERM_ALL, nullptr, nullptr, t.seg + len * SP + 19 * N, s));
  return ROD_OK;
}

static int reverse_segment(Tape& t, const Dev& d, const DipWork* work, int nwork, int max_slots,
                           hipStream_t s, int len) {
  const size_t SP = SEG_PLANES * (size_t)d.n;
  for (int k = len - 1; k >= 0; --k) {
    double* Sk = t.seg + k * SP;
    const double* S2 = k + 1 < len ? Sk + 2 * SP : nullptr;
    ATRY(reverse_level(t, d, work, nwork, max_slots, s, Sk, Sk + SP, S2, k + 1, ADJ_STEP));
  }
  return reverse_gather(t, d, max_slots, s, t.seg, t.seg + SP, 1, ADJ_STEP, rod_gradients{});
}

template <class F>
static int capture(hipStream_t s, hipGraphExec_t* out, F body) {
  hipGraph_t g = nullptr;
  ACHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = body();
  hipError_t e = hipStreamEndCapture(s, &g);
  if (rc != ROD_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
  ACHK(e);
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  ACHK(e);
  return ROD_OK;
}

void tape_release(Tape& t) {
  if (t.g_recompute) (void)hipGraphExecDestroy(t.g_recompute);
  if (t.g_reverse) (void)hipGraphExecDestroy(t.g_reverse);
  t.g_recompute = t.g_reverse = nullptr;
}

int adjoint_run(Tape& t, const Dev& d, int precision, const DipWork* work, int nwork,
                hipStream_t s, int64_t end_step, const rod_cotangent* gy, rod_gradients* gx) {
  const long N = d.n;
  const int64_t T = end_step - t.start_step;
  if (T <= 0) return rodmx_fail(ROD_E_NOTAPE, "no recorded steps");
  Adj& a = t.a;
  const size_t b3 = 3 * N * sizeof(double);
  ACHK(hipMemsetAsync(a.cx, 0, STATE_PLANES * N * sizeof(double), s));
  if (gy->x) ACHK(hipMemcpyAsync(a.cx, gy->x, b3, hipMemcpyDeviceToDevice, s));
  if (gy->v) ACHK(hipMemcpyAsync(a.cv, gy->v, b3, hipMemcpyDeviceToDevice, s));
  if (gy->q) ACHK(hipMemcpyAsync(a.cq, gy->q, 4 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (gy->w) ACHK(hipMemcpyAsync(a.cw, gy->w, b3, hipMemcpyDeviceToDevice, s));
  ACHK(hipMemsetAsync(a.mbbar, 0, b3, s));
  ACHK(hipMemsetAsync(a.fieldbar, 0, (size_t)d.field_len * d.M * 12 * sizeof(double), s));
  int max_slots = 1;
  {
    std::vector<int> ms(d.M);
    ACHK(hipMemcpy(ms.data(), d.mslots, d.M * sizeof(int), hipMemcpyDeviceToHost));
    for (int m : ms) max_slots = std::max(max_slots, m);
  }
  const int64_t nseg = (T + t.every - 1) / t.every;
  for (int64_t sg = nseg - 1; sg >= 0; --sg) {
    const int64_t s0 = t.start_step + sg * t.every;
    const int len = (int)std::min<int64_t>(t.every, T - sg * t.every);
    // recompute the segment from its checkpoint with the forward kernels
    ACHK(hipMemcpyAsync(t.seg, t.ckpt + (size_t)sg * STATE_PLANES * N,
                        STATE_PLANES * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_set_level, dim3(1), dim3(1), 0, s, a.level, (long long)s0);
    ACHK(hipGetLastError());
    hipLaunchKernelGGL(k_set_base, dim3(nblk(t.every + 1, 256)), dim3(256), 0, s, a.lbase,
                       a.levels, t.every + 1, (long long)s0);
    ACHK(hipGetLastError());
    if (len == t.every) {
      if (!t.g_recompute)
        ATRY(capture(s, &t.g_recompute, [&] { return recompute(t, d, precision, work, nwork, s, len); }));
      if (!t.g_reverse)
        ATRY(capture(s, &t.g_reverse, [&] { return reverse_segment(t, d, work, nwork, max_slots, s, len); }));
      ACHK(hipGraphLaunch(t.g_recompute, s));
      ACHK(hipGraphLaunch(t.g_reverse, s));
    } else {
      ATRY(recompute(t, d, precision, work, nwork, s, len));
      ATRY(reverse_segment(t, d, work, nwork, max_slots, s, len));
    }
  }
  // the initial force evaluation: dipole field of the start state, then its reverse
  {
    double* S = t.seg;
    ACHK(hipMemcpyAsync(S, t.ckpt, STATE_PLANES * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_set_level, dim3(1), dim3(1), 0, s, a.level, (long long)t.start_step);
    ACHK(hipGetLastError());
    hipLaunchKernelGGL(k_set_base, dim3(nblk(t.every + 1, 256)), dim3(256), 0, s, a.lbase,
                       a.levels, t.every + 1, (long long)t.start_step);
    ACHK(hipGetLastError());
    Dev v = view(d, S, a.level);
    ACHK(launch_pre(v, PRE_EVAL, s));
    ACHK(launch_force_pass(v, precision, work, nwork, 1, s));
    ACHK(launch_post(v, POST_EVAL, ROD_TERM_ALL, a.scratch, a.scratch + 3 * N, S + 19 * N, s));
    ATRY(reverse_level(t, d, work, nwork, max_slots, s, S, S, nullptr, 0, ADJ_PREPARE));
    ATRY(reverse_gather(t, d, max_slots, s, S, S, 0, ADJ_PREPARE, *gx));
  }
  if (gx->m_body) ACHK(hipMemcpyAsync(gx->m_body, a.mbbar, b3, hipMemcpyDeviceToDevice, s));
  if (gx->field)
    ACHK(hipMemcpyAsync(gx->field, a.fieldbar, (size_t)d.field_len * d.M * 12 * sizeof(double),
                        hipMemcpyDeviceToDevice, s));
  return ROD_OK;
}

}  // namespace rodmx
