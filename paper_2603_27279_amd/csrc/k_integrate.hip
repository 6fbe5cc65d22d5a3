// Per-particle kernels of the time step: the first half-kick / drift / Richardson
// quaternion update with boundary conditions and dipole rotation (pre), and the
// force gather with Zeeman, damping and external terms followed by the second
// half-kick (post). SI "Equations of motion"; dipoles rotate with the particle
// (main text, magnetised beams); Zeeman force and torque (Methods).
#include "rod.h"
#include "rod_internal.h"
#include "rod_math.h"
#include "particle_body.h"

// Contract a*b+c only within one expression, so that the separate and the
// fused form of a step round identically.
#pragma clang fp contract(on)

namespace rodmx {

// dq/dt = 1/2 (0, w) q for a space-frame angular velocity w.
__device__ __forceinline__ Q4<double> q_rate(Q4<double> q, V3<double> w) {
  return qscale(0.5, qmul(Q4<double>{0.0, w.x, w.y, w.z}, q));
}

// Richardson extrapolation of one full step against two half steps, each
// intermediate renormalised: q(t+dt) = N(2 q2 - q1).
__device__ __forceinline__ Q4<double> richardson(Q4<double> q, V3<double> w, double dt) {
  Q4<double> rq = q_rate(q, w);
  Q4<double> q1 = qnormalize(qadd(q, qscale(dt, rq)));
  Q4<double> qh = qnormalize(qadd(q, qscale(0.5 * dt, rq)));
  Q4<double> q2 = qnormalize(qadd(qh, qscale(0.5 * dt, q_rate(qh, w))));
  return qnormalize(qadd(qscale(2.0, q2), qscale(-1.0, q1)));
}

__device__ __forceinline__ Q4<double> drive_q(const Dev& d, long long lvl) {
  double phi = 2.0 * 3.14159265358979323846 * (double)lvl / (double)d.period;
  double s, c;
  sincos(0.5 * phi, &s, &c);
  return {c, s * d.axis[0], s * d.axis[1], s * d.axis[2]};
}



// Advance particle i from its state at level lvl - 1 (in registers) to level
// lvl: half-kick, drift and quaternion update of free particles; the imposed
// rotation of driven ones. The result goes to the planes of d.nx when set,
// else in place; states of particles that do not move are written only when
// `copy_still` is set (out-of-place step).
__device__ __forceinline__ void advance(const Dev& d, long i, int b, long long lvl, V3<double>& x,
                                        V3<double>& v, Q4<double>& q, V3<double>& w,
                                        V3<double> F, V3<double> T, double minv, double Iinv,
                                        bool copy_still) {
  const long N = d.n;
  // output planes: those of the next recorded state, or in place
  double* const xo = d.nx ? d.nx : d.x;
  double* const vo = d.nx ? d.nx + 3 * N : d.v;
  double* const qo = d.nx ? d.nx + 6 * N : d.q;
  double* const wo = d.nx ? d.nx + 10 * N : d.w;
  if (b == 0) {
    const double h = 0.5 * d.dt;
    v = v + (h * minv) * F;
    x = x + d.dt * v;
    w = w + (h * Iinv) * T;
    q = richardson(q, w, d.dt);
    if (d.use_lists) {  // moved too far since the contact lists were built?
      const V3<double> m = x - ld3(d.xb, N, i);
      const double lim = NBR_MOVE * d.skin;
      const bool far = dot(m, m) > lim * lim;
      const unsigned long long who = __ballot(far);  // one atomic per wave
      if (far && __lane_id() == (unsigned)(__ffsll((long long)who) - 1))
        atomicOr(&d.rebuild[lvl & 1], 1u);
    }
    st3(vo, N, i, v);
    st3(xo, N, i, x);
    st3(wo, N, i, w);
    st4(qo, N, i, q);
  } else {
    if (b == 2) q = drive_q(d, lvl);
    if (copy_still || b == 2) st4(qo, N, i, q);
    if (copy_still) {
      st3(xo, N, i, x);
      st3(vo, N, i, v);
      st3(wo, N, i, w);
    }
  }
}

__device__ __forceinline__ V3<double> pre_particle(const Dev& d, long i, int mode, long long n,
                                                   long long lvl);

__global__ __launch_bounds__(256) void k_pre(Dev d, int mode) {
  const long i = d.i_lo + (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = d.step[0];
  const long long lvl = n + (mode == PRE_STEP ? 1 : 0);  // level of the coming force evaluation
  if (i == 0) d.step[d.lc] = lvl;
  const bool valid = i < d.i_hi;
  V3<double> x{0.0, 0.0, 0.0};
  if (valid) x = pre_particle(d, i, mode, n, lvl);
  chunk_box(d, i, x, valid);
}

// Cell-list entries of the level being evaluated, when its contact lists are
// rebuilt (lazy_cells: the particle kernels left the list empty). Most steps
// keep their lists, and then every workgroup only reads the flag: the grid is
// capped at CELL_INSERT_WGS workgroups (a few per compute unit), each thread
// striding over the particles CELL_INSERT_ILP at a time, so that their loads
// and slot claims are in flight together.
constexpr int CELL_INSERT_WGS = 1024;
constexpr int CELL_INSERT_ILP = 4;
__global__ __launch_bounds__(256) void k_cell_insert(Dev d, int build) {
  const long long lvl = d.step[d.lc];
  if (!build && d.rebuild[lvl & 1] == 0u) return;  // the lists stay
  const long N = d.n;
  const long G = (long)gridDim.x * blockDim.x;
  const CellTab t = cell_tab(d, lvl);
  for (long i0 = (long)blockIdx.x * blockDim.x + threadIdx.x; i0 < N; i0 += CELL_INSERT_ILP * G) {
    V3<double> x[CELL_INSERT_ILP];
    int rod[CELL_INSERT_ILP], slot[CELL_INSERT_ILP];
    unsigned key[CELL_INSERT_ILP];
#pragma unroll
    for (int u = 0; u < CELL_INSERT_ILP; ++u) {
      const long i = i0 + u * G < N ? i0 + u * G : i0;
      x[u] = ld3(d.x, N, i);
      rod[u] = d.rod[i];
      key[u] = cell_key(d, x[u], d.mem[i]);
    }
#pragma unroll
    for (int u = 0; u < CELL_INSERT_ILP; ++u)  // the claims, all in flight
      slot[u] = i0 + u * G < N ? atomicAdd(&t.cnt[key[u]], 1) : 0;
#pragma unroll
    for (int u = 0; u < CELL_INSERT_ILP; ++u)
      if (i0 + u * G < N) cell_place(d, t, i0 + u * G, x[u], rod[u], key[u], slot[u]);
  }
}

hipError_t launch_cell_insert(const Dev& d, int build, hipStream_t s, const hipEvent_t* ev) {
  const long blocks = (d.n + 255) / 256;
  launch_k(ev, k_cell_insert, dim3((unsigned)(blocks < CELL_INSERT_WGS ? blocks : CELL_INSERT_WGS)), dim3(256),
           s, d, build);
  return hipGetLastError();
}

// The pre kernel's work for particle i; returns its position at level lvl.
__device__ __forceinline__ V3<double> pre_particle(const Dev& d, long i, int mode, long long n,
                                                   long long lvl) {
  const long N = d.n;
  const int b = d.bc[i];
  // state read in place, or from separate planes (out-of-place step)
  const double* sx = d.src ? d.src : d.x;
  const double* sv = d.src ? d.src + 3 * N : d.v;
  const double* sq = d.src ? d.src + 6 * N : d.q;
  const double* sw = d.src ? d.src + 10 * N : d.w;
  const double* sF = d.src ? d.src + 13 * N : d.F;
  const double* sT = d.src ? d.src + 16 * N : d.T;
  Q4<double> q = ld4(sq, N, i);
  V3<double> x = ld3(sx, N, i);
  const V3<double> mb = ld3(d.mb, N, i);
  const int mem = d.mem[i], rod = d.rod[i];
  if (mode == PRE_STEP) {
    V3<double> v = ld3(sv, N, i), w = ld3(sw, N, i);
    advance(d, i, b, lvl, x, v, q, w, ld3(sF, N, i), ld3(sT, N, i), d.minv[i], d.Iinv[i],
            d.src != nullptr);
  } else if (mode == PRE_PREPARE) {
    q = qnormalize(q);
    if (b != 0) {
      V3<double> z{0.0, 0.0, 0.0};
      st3(d.v, N, i, z);
      st3(d.w, N, i, z);
    }
    if (b == 2) {
      q = drive_q(d, n);
      double om = 2.0 * 3.14159265358979323846 / ((double)d.period * d.dt);
      st3(d.w, N, i, V3<double>{om * d.axis[0], om * d.axis[1], om * d.axis[2]});
    }
    st4(d.q, N, i, q);
  }
  moment_and_cell(d, i, q, x, mb, mem, rod, lvl, !(d.lazy_cells && mode == PRE_STEP));
  return x;
}

__device__ __forceinline__ bool finite3(V3<double> a) {
  return isfinite(a.x) && isfinite(a.y) && isfinite(a.z);
}

// State of one particle as read at the start of a gather: every load that does
// not depend on another is issued before any arithmetic or store.
struct PIn {
  V3<double> x, v, w, m, mb;
  Q4<double> q;
  double minv, Iinv;
  int b, mem, rod;
};
__device__ __forceinline__ PIn load_particle(const Dev& d, long i) {
  const long N = d.n;
  return {ld3(d.x, N, i), ld3(d.v, N, i), ld3(d.w, N, i), ld3(d.mu, N, i), ld3(d.mb, N, i),
          ld4(d.q, N, i), d.minv[i], d.Iinv[i], d.bc[i], d.mem[i], d.rod[i]};
}

// Dipole force and field of particle i: its S slots added in slot order, in
// FP64, B slots per round trip (FP32 slots of the mixed path: 16; FP64: 8).
// Slots past the member's own count hold zeros.
template <class T, int B>
__device__ __forceinline__ void slot_sum(const T* dp, long N, int s_begin, int s_end, long i,
                                         V3<double>& Fd, V3<double>& Bd) {
  for (int s0 = s_begin; s0 < s_end; s0 += B) {
    T v[B][6];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const T* q = dp + (long)(s0 + k) * 6 * N;
      if (s0 + k < s_end)
#pragma unroll
        for (int c = 0; c < 6; ++c) v[k][c] = q[c * N + i];
    }
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (s0 + k < s_end) {
        Fd = Fd + V3<double>{(double)v[k][0], (double)v[k][1], (double)v[k][2]};
        Bd = Bd + V3<double>{(double)v[k][3], (double)v[k][4], (double)v[k][5]};
      }
  }
}

// The dipole force and field of particle i from slots [s_begin, s_end) when
// `mask` asks for them (zero otherwise). Called first in the particle
// kernels: the slot loads are the longest chain of the gather, and few other
// values are live yet.
__device__ __forceinline__ void dipole_sums(const Dev& d, long i, int mask, V3<double>& Fd,
                                            V3<double>& Bd, int s_begin, int s_end) {
  Fd = V3<double>{0.0, 0.0, 0.0};
  Bd = V3<double>{0.0, 0.0, 0.0};
  if (!((mask & 2) && d.dipole_on)) return;
  if (d.dslotf) slot_sum<float, 8>(d.dslotf, d.n, s_begin, s_end, i, Fd, Bd);
  else slot_sum<double, 8>(d.dpart, d.n, s_begin, s_end, i, Fd, Bd);
}

// Systems below 65,536 particles spread the gather over four waves per 64
// particles (a quarter of the workgroups a particle per thread would give):
// wave w adds the slots [w G, (w + 1) G), G = ceil(S / 4), of each of the 64
// particles, the four partial sums meet in LDS, and wave 0 adds them in wave
// order and completes the kernel alone. Every gather of such a system (fused
// kick and unfused post) sums in this order, so launch forms stay bitwise
// equal; larger systems add the slots one after another.
constexpr int SPLIT_WAVES = 4;
inline bool particle_split(long n) { return n < 65536; }

// Slot sums of particle i in the kernel's layout: all slots (SPLIT false), or
// this wave's group, combined through `part` ([SPLIT_WAVES][64][6]); returns
// false on waves other than the first, which then leave the kernel.
template <bool SPLIT>
__device__ __forceinline__ bool dipole_sums_of(const Dev& d, long i, bool valid, int mask,
                                               V3<double>& Fd, V3<double>& Bd, double* part) {
  if constexpr (!SPLIT) {
    if (valid) dipole_sums(d, i, mask, Fd, Bd, 0, d.max_slots);
    return true;
  } else {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int G = (d.max_slots + SPLIT_WAVES - 1) / SPLIT_WAVES;
    const int sb = min(w * G, d.max_slots), se = min(sb + G, d.max_slots);
    V3<double> f{0.0, 0.0, 0.0}, b{0.0, 0.0, 0.0};
    if (valid) dipole_sums(d, i, mask, f, b, sb, se);
    double* o = part + 6 * (w * 64 + lane);
    o[0] = f.x; o[1] = f.y; o[2] = f.z; o[3] = b.x; o[4] = b.y; o[5] = b.z;
    __syncthreads();
    if (w != 0) return false;
    Fd = V3<double>{0.0, 0.0, 0.0};
    Bd = V3<double>{0.0, 0.0, 0.0};
    for (int u = 0; u < SPLIT_WAVES; ++u) {
      const double* q = part + 6 * (u * 64 + lane);
      Fd = Fd + V3<double>{q[0], q[1], q[2]};
      Bd = Bd + V3<double>{q[3], q[4], q[5]};
    }
    return true;
  }
}

// Total force and torque on particle i from the terms in `mask` at level lvl
// (bond, dipole, Zeeman, contact, damping, external), with the dipole force Fd
// and field Bd from dipole_sums; the dipole field is written to Bo when given.
// HM: the contact law is Hertz-Mindlin, whose contacts also exert a torque (a
// template argument, so that the Hookean kernels carry no extra load). FL: the
// immersed-boundary penalty m_p / dt_fluid (U_p - v_p) with the velocity the
// evaluation sees, also stored to d.ibm_f (only the unfused post kernel).
// Loads are unconditional where the index is valid, so they are all in flight
// together.
template <bool HM, bool FL = false>
__device__ __forceinline__ void gather(const Dev& d, long i, int mask, long long lvl, double* Bo,
                                       const PIn& p, V3<double> Fd, V3<double> Bd, V3<double>& F,
                                       V3<double>& T) {
  const long N = d.n;
  const long im = i > 0 ? i - 1 : 0;
  const uint8_t bf = d.bflags[i];
  const V3<double> bF0 = ld3(d.bF, N, i), bTs0 = ld3(d.bTs, N, i), bTb0 = ld3(d.bTbt, N, i);
  const V3<double> bF1 = ld3(d.bF, N, im), bTs1 = ld3(d.bTs, N, im), bTb1 = ld3(d.bTbt, N, im);
  const V3<double> cF = d.contact_on ? ld3(d.cF, N, i) : V3<double>{0.0, 0.0, 0.0};
  V3<double> cT{0.0, 0.0, 0.0};  // used only with HM
  if constexpr (HM) cT = ld3(d.cT, N, i);
  const double mass = d.mass[i], inertia = d.inertia[i];
  F = V3<double>{0.0, 0.0, 0.0};
  T = V3<double>{0.0, 0.0, 0.0};
  if (mask & 1) {  // bonds: +F, tau_s + tau_bt from bond (i, i+1); -F, tau_s - tau_bt from (i-1, i)
    if (bf & 1) {
      F = F + bF0;
      T = T + bTs0 + bTb0;
    }
    if (bf & 2) {
      F = F - bF1;
      T = T + bTs1 - bTb1;
    }
  }
  const V3<double> m = p.m;
  if ((mask & 2) && d.dipole_on) {  // dipole-dipole: force and torque m x B_dip
    F = F + Fd;
    T = T + cross(m, Bd);
  }
  if (Bo) st3(Bo, N, i, Bd);
  if (mask & 4) {  // Zeeman: B = B0 + G x, f = G^T m, tau = m x B
    long long L = d.field_len;
    long long row = ((lvl % L) + L) % L;
    const double* f = d.field + (row * d.M + p.mem) * 12;
    const V3<double> x = p.x;
    V3<double> B{f[0] + f[3] * x.x + f[4] * x.y + f[5] * x.z,
                 f[1] + f[6] * x.x + f[7] * x.y + f[8] * x.z,
                 f[2] + f[9] * x.x + f[10] * x.y + f[11] * x.z};
    F = F + V3<double>{f[3] * m.x + f[6] * m.y + f[9] * m.z,
                       f[4] * m.x + f[7] * m.y + f[10] * m.z,
                       f[5] * m.x + f[8] * m.y + f[11] * m.z};
    T = T + cross(m, B);
  }
  if ((mask & 8) && d.contact_on) {  // contact (Hertz-Mindlin: also its torque)
    F = F + cF;
    if constexpr (HM) T = T + cT;
  }
  if (mask & 16) {  // global viscous damping with the current (half-step) velocities
    F = F - (d.damping * mass) * p.v;
    T = T - (d.damping * inertia) * p.w;
  }
  if constexpr (FL) {
    const V3<double> Fp = (mass * d.ibm_idt) * (ld3(d.ibm_u, N, i) - p.v);
    F = F + Fp;
    st3(d.ibm_f, N, i, Fp);
  }
  if (mask & 32) {
    if (d.extF) F = F + ld3(d.extF, N, i);
    if (d.extT) T = T + ld3(d.extT, N, i);
  }
}

// Store the forces of the state and apply the second half-kick to free
// particles, updating p.v and p.w (stored when `store_vw`; the fused kick
// overwrites them with the next half-kick anyway). Flags non-finite values.
__device__ __forceinline__ void kick(const Dev& d, long i, V3<double> F, V3<double> T, PIn& p,
                                     bool store_vw) {
  const long N = d.n;
  st3(d.F, N, i, F);
  st3(d.T, N, i, T);
  if (p.b == 0) {
    const double h = 0.5 * d.dt;
    p.v = p.v + (h * p.minv) * F;
    p.w = p.w + (h * p.Iinv) * T;
    if (store_vw) {
      st3(d.v, N, i, p.v);
      st3(d.w, N, i, p.w);
    }
  }
  if (!finite3(F) || !finite3(T) || !finite3(p.x)) atomicOr(&d.flags[FLAG_NONFINITE], 1u);
}

template <bool HM, bool FL, bool SPLIT>
__global__ __launch_bounds__(256) void k_post(Dev d, int mode, int mask, double* Fo, double* To,
                                              double* Bo) {
  __shared__ double part[SPLIT ? 6 * 64 * SPLIT_WAVES : 1];
  const long i = d.i_lo + (SPLIT ? (long)blockIdx.x * 64 + (threadIdx.x & 63)
                                 : (long)blockIdx.x * blockDim.x + threadIdx.x);
  const long N = d.n;
  const long long lvl = d.step[d.lc];  // level of the forces being gathered
  if (i == 0 && (!SPLIT || threadIdx.x < 64)) {
    if (mode == POST_KICK) d.step[0] = lvl;
    *cell_tab(d, lvl).ovf_cnt = 0;  // the contact pass that used the overflow list has finished
    if (d.use_lists) d.rebuild[lvl & 1] = 0u;  // and so has the one that read this flag
  }
  V3<double> Fd, Bd;
  if (!dipole_sums_of<SPLIT>(d, i, i < d.i_hi, mask, Fd, Bd, part)) return;
  if (i >= d.i_hi) return;
  PIn p = load_particle(d, i);
  const int key = d.contact_on ? d.key[i] : 0;
  V3<double> F, T;
  gather<HM, FL>(d, i, mask, lvl, Bo, p, Fd, Bd, F, T);
  if (mode == POST_EVAL) {
    st3(Fo, N, i, F);
    st3(To, N, i, T);
  } else if (mode == POST_KICK) {
    kick(d, i, F, T, p, true);
  } else {  // prepare: forces of the initial state, no kick
    st3(d.F, N, i, F);
    st3(d.T, N, i, T);
    if (!finite3(F) || !finite3(T) || !finite3(p.x)) atomicOr(&d.flags[FLAG_NONFINITE], 1u);
  }
  if (d.contact_on) cell_tab(d, lvl).cnt[key] = 0;  // empty the cell list for the next build
}

// The end of one step and the start of the next in one pass: gather and second
// half-kick at level L = step[lc], then half-kick, drift, rotation, moments and
// cell insertion for level L + 1 (written to step[3 - lc]). The cell list and
// overflow list of level L are emptied while those of level L + 1 are filled.
template <bool HM, bool SPLIT>
__global__ __launch_bounds__(256) void k_kick(Dev d, double* Bo) {
  __shared__ double part[SPLIT ? 6 * 64 * SPLIT_WAVES : 1];
  const long i = d.i_lo + (SPLIT ? (long)blockIdx.x * 64 + (threadIdx.x & 63)
                                 : (long)blockIdx.x * blockDim.x + threadIdx.x);
  const long long L = d.step[d.lc];
  if (i == 0 && (!SPLIT || threadIdx.x < 64)) {
    d.step[3 - d.lc] = L + 1;
    *cell_tab(d, L).ovf_cnt = 0;
    if (d.use_lists) d.rebuild[L & 1] = 0u;
  }
  const bool valid = i < d.i_hi;
  V3<double> x{0.0, 0.0, 0.0};
  V3<double> Fd, Bd;
  if (!dipole_sums_of<SPLIT>(d, i, valid, ROD_TERM_ALL, Fd, Bd, part)) return;
  if (valid) {
    PIn p = load_particle(d, i);
    const int key = d.contact_on ? d.key[i] : 0;
    V3<double> F, T;
    gather<HM>(d, i, ROD_TERM_ALL, L, Bo, p, Fd, Bd, F, T);
    // in place, the next half-kick overwrites v and w; out of place (a recorded
    // state) the full-step v and w stay with level L
    const bool apart = d.nx != nullptr;
    kick(d, i, F, T, p, apart);
    if (d.contact_on) cell_tab(d, L).cnt[key] = 0;
    advance(d, i, p.b, L + 1, p.x, p.v, p.q, p.w, F, T, p.minv, p.Iinv, apart);
    moment_and_cell(d, i, p.q, p.x, p.mb, p.mem, p.rod, L + 1, !d.lazy_cells);
    x = p.x;
  }
  chunk_box(d, i, x, valid);
}

// Per-particle energy terms [9][N]: bond terms attributed to the bond's first
// particle, Zeeman -m.B, dipole -1/2 m.B_dip, contact (pairs halved), kinetic.
__global__ __launch_bounds__(256) void k_energy_part(Dev d, const double* Bdip, double* E) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long N = d.n;
  if (i >= N) return;
  const long long lvl = d.step[d.lc];
  const bool hb = d.bflags[i] & 1;
  for (int t = 0; t < 4; ++t) E[t * N + i] = hb ? d.bE[t * N + i] : 0.0;
  const V3<double> m = ld3(d.mu, N, i);
  long long L = d.field_len;
  long long row = ((lvl % L) + L) % L;
  const double* f = d.field + (row * d.M + d.mem[i]) * 12;
  V3<double> x = ld3(d.x, N, i);
  V3<double> B{f[0] + f[3] * x.x + f[4] * x.y + f[5] * x.z,
               f[1] + f[6] * x.x + f[7] * x.y + f[8] * x.z,
               f[2] + f[9] * x.x + f[10] * x.y + f[11] * x.z};
  E[4 * N + i] = -dot(m, B);
  E[5 * N + i] = d.dipole_on ? -0.5 * dot(m, ld3(Bdip, N, i)) : 0.0;
  E[6 * N + i] = d.contact_on ? d.cE[i] : 0.0;
  V3<double> v = ld3(d.v, N, i), w = ld3(d.w, N, i);
  E[7 * N + i] = 0.5 * d.mass[i] * dot(v, v);
  E[8 * N + i] = 0.5 * d.inertia[i] * dot(w, w);
}

// One block per member: fixed-order tree sum of the member's particle range.
__global__ __launch_bounds__(256) void k_energy_reduce(Dev d, const double* E, double* out) {
  __shared__ double red[256];
  const int mem = blockIdx.x;
  const int b = d.mrange[2 * mem], e = d.mrange[2 * mem + 1];
  const long N = d.n;
  for (int t = 0; t < 9; ++t) {
    double s = 0.0;
    for (int i = b + threadIdx.x; i < e; i += blockDim.x) s += E[t * N + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[mem * 9 + t] = red[0];
    __syncthreads();
  }
}

static inline unsigned blocks_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_pre(const Dev& d, int mode, hipStream_t s, const hipEvent_t* ev) {
  const int bs = particle_block(d.n);
  launch_k(ev, k_pre, dim3(blocks_for(d.i_hi - d.i_lo, bs)), dim3(bs), s, d, mode);
  return hipGetLastError();
}

template <bool SPLIT>
static void post_variant(const Dev& d, int mode, int mask, double* Fo, double* To, double* Bo,
                         hipStream_t s, const hipEvent_t* ev, dim3 g, dim3 b) {
  if (d.ibm_u) {
    if (d.hm) launch_k(ev, k_post<true, true, SPLIT>, g, b, s, d, mode, mask, Fo, To, Bo);
    else launch_k(ev, k_post<false, true, SPLIT>, g, b, s, d, mode, mask, Fo, To, Bo);
  } else if (d.hm) {
    launch_k(ev, k_post<true, false, SPLIT>, g, b, s, d, mode, mask, Fo, To, Bo);
  } else {
    launch_k(ev, k_post<false, false, SPLIT>, g, b, s, d, mode, mask, Fo, To, Bo);
  }
}

hipError_t launch_post(const Dev& d, int mode, int mask, double* Fo, double* To, double* Bo,
                       hipStream_t s, const hipEvent_t* ev) {
  if (particle_split(d.n)) {  // four waves per 64 particles
    post_variant<true>(d, mode, mask, Fo, To, Bo, s, ev, dim3(blocks_for(d.i_hi - d.i_lo, 64)),
                       dim3(64 * SPLIT_WAVES));
  } else {
    const int bs = particle_block(d.n);
    post_variant<false>(d, mode, mask, Fo, To, Bo, s, ev, dim3(blocks_for(d.i_hi - d.i_lo, bs)),
                        dim3(bs));
  }
  return hipGetLastError();
}

hipError_t launch_kick(const Dev& d, double* Bo, hipStream_t s, const hipEvent_t* ev) {
  if (particle_split(d.n)) {
    const dim3 g(blocks_for(d.i_hi - d.i_lo, 64)), b(64 * SPLIT_WAVES);
    if (d.hm) launch_k(ev, k_kick<true, true>, g, b, s, d, Bo);
    else launch_k(ev, k_kick<false, true>, g, b, s, d, Bo);
  } else {
    const int bs = particle_block(d.n);
    const dim3 g(blocks_for(d.i_hi - d.i_lo, bs)), b(bs);
    if (d.hm) launch_k(ev, k_kick<true, false>, g, b, s, d, Bo);
    else launch_k(ev, k_kick<false, false>, g, b, s, d, Bo);
  }
  return hipGetLastError();
}

// Kinetic energy, translational plus rotational, of each member from the
// state's velocities: one block per member, fixed-order tree sum.
__global__ __launch_bounds__(256) void k_kinetic(Dev d, double* out) {
  __shared__ double red[256];
  const int mem = blockIdx.x;
  const int b = d.mrange[2 * mem], e = d.mrange[2 * mem + 1];
  const long N = d.n;
  double s = 0.0;
  for (int i = b + threadIdx.x; i < e; i += blockDim.x) {
    const V3<double> v = ld3(d.v, N, i), w = ld3(d.w, N, i);
    s += 0.5 * d.mass[i] * dot(v, v) + 0.5 * d.inertia[i] * dot(w, w);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[mem] = red[0];
}

// Positions of the listed particles, [n][3].
__global__ __launch_bounds__(256) void k_gather_x(Dev d, const int* idx, int n, double* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const V3<double> x = ld3(d.x, d.n, idx[k]);
  out[3 * k] = x.x; out[3 * k + 1] = x.y; out[3 * k + 2] = x.z;
}

hipError_t launch_kinetic(const Dev& d, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_kinetic, dim3(d.M), dim3(256), 0, s, d, out);
  return hipGetLastError();
}

hipError_t launch_gather_x(const Dev& d, const int* idx, int n, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_x, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, idx, n, out);
  return hipGetLastError();
}

hipError_t launch_energy(const Dev& d, double* Epart, double* out, hipStream_t s) {
  // Epart holds [9][N] energy terms, then [3][N] dipole field, [3][N] and [3][N] scratch.
  double* Bd = Epart + 9 * d.n;
  hipError_t e = launch_post(d, POST_EVAL, 2, Bd + 3 * d.n, Bd + 6 * d.n, Bd, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_part, dim3(blocks_for(d.n, 256)), dim3(256), 0, s, d,
                     (const double*)Bd, Epart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_reduce, dim3(d.M), dim3(256), 0, s, d, (const double*)Epart, out);
  return hipGetLastError();
}

}  // namespace rodmx
