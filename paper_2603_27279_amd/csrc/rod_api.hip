// Host runtime behind the C ABI of include/rod.h: descriptor validation,
// topology and constants, workspace, the step schedule (eager launches or a
// captured HIP graph of several steps), inspection entry points, and the tape
// used by the reverse pass.
#include "rod.h"
#include "rod_internal.h"
#include "lbm.h"
#include "lbm_internal.h"
#include "rod_adjoint.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

static_assert(rodmx::HM_CAP == ROD_HM_MAX_CONTACTS, "Hertz-Mindlin capacity differs from rod.h");
using namespace rodmx;

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPC(expr)                                                                        \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return fail(ROD_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e),       \
                  __FILE__, __LINE__);                                                    \
  } while (0)

#define TRY(expr)                 \
  do {                            \
    int _r = (expr);              \
    if (_r != ROD_OK) return _r;  \
  } while (0)

struct rod_ctx {
  rod_desc desc;            // scalar fields (host pointers cleared after init)
  rod_buffers ub;
  hipStream_t user = nullptr, s = nullptr;
  int dev = 0;                // device current at rod_init
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  Dev d;
  std::vector<void*> allocs;
  double* ibm_buf = nullptr;  // coupled cycles: fluid velocity and penalty force [6][N]
  DipWork* work = nullptr;
  int nwork = 0, max_slots = 1;
  // with a dipole cutoff and a tape: all-pairs items of one slot for the
  // reverse pass (it tests each pair against the cutoff)
  DipWork* adj_work = nullptr;
  int adj_nwork = 0;
  std::vector<void*> plan_allocs;   // dipole work list, slot counts, partial slots
  std::vector<int> mrange_h;        // [2M] member particle ranges
  int plan_small = -1, plan_target = 1024;  // current dipole layout
  std::vector<int> mslots_h;        // [M] source ranges per member of the current layout
  std::vector<int> mlen_h;          // [M] length of those ranges
  // per-rod launch mode (baseline for the batched form)
  int launch_mode = ROD_LAUNCH_BATCHED;
  DipWork* rod_work = nullptr;      // dipole items grouped by rod
  std::vector<int> rod_work_off;    // [R+1]
  std::vector<void*> rod_allocs;
  double* epart = nullptr;
  double* eout = nullptr;
  int* pair_count = nullptr;
  std::vector<int> rod_offset;
  std::vector<int> rod_member_h;
  std::vector<double> bref_h;  // [4N]
  std::vector<double> rodK_h;  // [R][4]
  std::vector<uint8_t> bflags_h;
  std::vector<int> rod_h;
  int64_t h_step = 0;
  hipGraphExec_t gexec = nullptr;
  int gsteps = 0;
  Tape tape;
  hipGraphExec_t tgexec = nullptr;  // one checkpoint interval of steps, for taped runs
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kernel;  // kernel class of each recorded pair
  int ev_used = 0;             // pairs recorded since the last read
  double t_ms[ROD_KERNEL_COUNT] = {0};
  int64_t t_cnt[ROD_KERNEL_COUNT] = {0};
};

static int timing_collect(rod_ctx* c);
constexpr int EV_PAIRS_MAX = 4096;  // pending pairs before they are folded into the sums

// Event pair that the next launch of kernel class `kid` stamps with its own
// start and end (null when timing is off). The pool stays bounded: once
// EV_PAIRS_MAX pairs are pending, the stream is synchronised and their times
// are added to the per-class sums.
static int timing_events(rod_ctx* c, int kid, const hipEvent_t** ev) {
  *ev = nullptr;
  if (!c->timing) return ROD_OK;
  if (c->ev_used >= EV_PAIRS_MAX) TRY(timing_collect(c));
  while ((int)c->ev_pool.size() < 2 * (c->ev_used + 1)) {
    hipEvent_t e;
    HIPC(hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  if ((int)c->ev_kernel.size() < c->ev_used + 1) c->ev_kernel.resize(c->ev_used + 1);
  c->ev_kernel[c->ev_used] = kid;
  *ev = &c->ev_pool[2 * c->ev_used];
  ++c->ev_used;
  return ROD_OK;
}
static int timing_collect(rod_ctx* c) {
  if (c->ev_used == 0) return ROD_OK;
  HIPC(hipStreamSynchronize(c->s));
  for (int k = 0; k < c->ev_used; ++k) {
    float ms = 0.f;
    HIPC(hipEventElapsedTime(&ms, c->ev_pool[2 * k], c->ev_pool[2 * k + 1]));
    c->t_ms[c->ev_kernel[k]] += ms;
    c->t_cnt[c->ev_kernel[k]] += 1;
  }
  c->ev_used = 0;
  return ROD_OK;
}

#define TIMED(c, kid, launch, ...)                     \
  do {                                                 \
    const hipEvent_t* ev_ = nullptr;                   \
    TRY(timing_events((c), (kid), &ev_));              \
    HIPC(launch(__VA_ARGS__, ev_));                    \
  } while (0)

static size_t next_pow2(size_t v) {
  size_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

template <class T>
static int palloc(rod_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  size_t bytes = std::max<size_t>(count * sizeof(T), 16);
  HIPC(hipMalloc(&q, bytes));
  c->plan_allocs.push_back(q);
  HIPC(hipMemset(q, 0, bytes));
  *p = (T*)q;
  return ROD_OK;
}

template <class T>
static int dalloc(rod_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  size_t bytes = std::max<size_t>(count * sizeof(T), 16);
  HIPC(hipMalloc(&q, bytes));
  c->allocs.push_back(q);
  HIPC(hipMemset(q, 0, bytes));
  *p = (T*)q;
  return ROD_OK;
}

// Bounds on one pair's contribution to the contact sums of force, torque and
// energy, which set the quanta of those exact sums: for the Hookean law the
// force k r_c and the energy k r_c^2 / 2 at full overlap (no torque); for
// Hertz-Mindlin the normal force at an overlap of r_c, times 1 + mu since the
// tangential force is limited to mu times the normal one, that tangential force
// on the arm r_c / 2 for the torque, and the normal energy at that overlap. A
// zero bound (no such term) is taken as 1.
static void contact_bounds(const rod_desc* d, double b[3]) {
  const double rc = d->r_contact;
  if (d->contact_model == ROD_CONTACT_HERTZ_MINDLIN) {
    const double E = d->contact_hm[0], nu = d->contact_hm[1], mu = d->contact_hm[2];
    const double Es = E / (2.0 * (1.0 - nu * nu)), Rs = 0.25 * rc;
    const double fn = 4.0 / 3.0 * Es * std::sqrt(Rs * rc) * rc;
    b[0] = (1.0 + mu) * fn;
    b[1] = 0.5 * rc * mu * fn;
    b[2] = 8.0 / 15.0 * Es * std::sqrt(Rs) * rc * rc * std::sqrt(rc);
  } else {
    const double k = std::fabs(d->k_contact);
    b[0] = k * rc;
    b[1] = 0.0;
    b[2] = 0.5 * k * rc * rc;
  }
  for (int q = 0; q < 3; ++q)
    if (b[q] == 0.0) b[q] = 1.0;
}

// Scale exponents of the exact contact sums; fails when a bound is not finite
// or so far from 1 that the scale or a term at its bound leaves FP64's range.
static int contact_scales(const rod_desc* d, int e[3]) {
  double b[3];
  contact_bounds(d, b);
  static const char* what[3] = {"force", "torque", "energy"};
  for (int q = 0; q < 3; ++q) {
    if (!std::isfinite(b[q]) || !(b[q] > 0))
      return fail(ROD_E_INVALID, "the contact law's bound on a pair's %s (%g) is not finite",
                  what[q], b[q]);
    e[q] = FIX_BOUND_EXP - std::ilogb(b[q]);
    if (e[q] < -900 || e[q] > 900)
      return fail(ROD_E_INVALID, "the contact law's bound on a pair's %s (%g) is outside the "
                  "range of the exact contact sums (2^-820 to 2^980)", what[q], b[q]);
  }
  return ROD_OK;
}

static int validate(const rod_desc* d) {
  if (!d) return fail(ROD_E_INVALID, "descriptor is NULL");
  if (d->n_particles < 1 || d->n_rods < 1 || d->n_members < 1)
    return fail(ROD_E_INVALID, "need n_particles, n_rods, n_members >= 1 (got %d, %d, %d)",
                d->n_particles, d->n_rods, d->n_members);
  if (!d->rod_offset || !d->rod_member || !d->rod_params || !d->x_ref || !d->bc)
    return fail(ROD_E_INVALID, "rod_offset, rod_member, rod_params, x_ref and bc are required");
  if (d->rod_offset[0] != 0 || d->rod_offset[d->n_rods] != d->n_particles)
    return fail(ROD_E_INVALID, "rod_offset must start at 0 and end at n_particles");
  for (int r = 0; r < d->n_rods; ++r) {
    if (d->rod_offset[r + 1] <= d->rod_offset[r])
      return fail(ROD_E_INVALID, "rod_offset must be strictly increasing (rod %d)", r);
    int m = d->rod_member[r];
    if (m < 0 || m >= d->n_members || (r > 0 && m < d->rod_member[r - 1]))
      return fail(ROD_E_INVALID, "rod_member must be non-decreasing in [0, n_members) (rod %d)", r);
    const double* p = d->rod_params + 4 * r;
    if (!(p[0] > 0) || !(p[1] > 0) || !(p[2] > 0) || !(p[3] > -1.0))
      return fail(ROD_E_INVALID, "rod %d: need diameter, density, Young > 0 and Poisson > -1", r);
  }
  {
    std::vector<char> used(d->n_members, 0);
    for (int r = 0; r < d->n_rods; ++r) used[d->rod_member[r]] = 1;
    for (int m = 0; m < d->n_members; ++m)
      if (!used[m]) return fail(ROD_E_INVALID, "member %d has no rod", m);
  }
  bool driven = false;
  for (int i = 0; i < d->n_particles; ++i) {
    if (d->bc[i] < 0 || d->bc[i] > 2) return fail(ROD_E_INVALID, "bc[%d] = %d is not 0, 1 or 2", i, d->bc[i]);
    driven |= d->bc[i] == 2;
  }
  if (driven) {
    double a = std::sqrt(d->drive_axis[0] * d->drive_axis[0] + d->drive_axis[1] * d->drive_axis[1] +
                         d->drive_axis[2] * d->drive_axis[2]);
    if (d->drive_period <= 0 || !(a > 0))
      return fail(ROD_E_INVALID, "driven particles need drive_period > 0 and a non-zero axis");
  }
  if (!(d->dt > 0) || !std::isfinite(d->dt)) return fail(ROD_E_INVALID, "dt must be > 0");
  if (!(d->damping >= 0)) return fail(ROD_E_INVALID, "damping must be >= 0");
  if (d->field_len < 1) return fail(ROD_E_INVALID, "field_len must be >= 1");
  if (d->precision != ROD_FP64 && d->precision != ROD_MIXED)
    return fail(ROD_E_INVALID, "precision must be ROD_FP64 or ROD_MIXED");
  if (d->contact_on && !(d->r_contact > 0)) return fail(ROD_E_INVALID, "r_contact must be > 0");
  if (d->exclude_depth < 0) return fail(ROD_E_INVALID, "exclude_depth must be >= 0");
  if (d->graph_steps < 0 || d->tape_every < 0 || d->tape_capacity < 0)
    return fail(ROD_E_INVALID, "graph_steps, tape_every and tape_capacity must be >= 0");
  if (d->bond_damping) {
    bool any = false;
    for (int k = 0; k < 4 * d->n_rods; ++k) {
      const double g = d->bond_damping[k];
      if (!(g >= 0) || !std::isfinite(g))
        return fail(ROD_E_INVALID, "bond damping factors must be finite and >= 0 (rod %d)", k / 4);
      any = any || g != 0;
    }
    if (any && d->tape_capacity > 0)
      return fail(ROD_E_INVALID, "bond damping is not differentiated: no tape with bond damping");
  }
  if (d->contact_model != ROD_CONTACT_HOOKEAN && d->contact_model != ROD_CONTACT_HERTZ_MINDLIN)
    return fail(ROD_E_INVALID, "contact_model must be ROD_CONTACT_HOOKEAN or _HERTZ_MINDLIN");
  if (d->contact_on && d->contact_model == ROD_CONTACT_HERTZ_MINDLIN) {
    const double* h = d->contact_hm;
    for (int k = 0; k < 5; ++k)
      if (!std::isfinite(h[k])) return fail(ROD_E_INVALID, "contact_hm must be finite");
    if (!(h[0] > 0) || !(h[1] > -1.0 && h[1] <= 0.5) || !(h[2] >= 0) || !(h[3] >= 0) ||
        !(h[4] >= 0))
      return fail(ROD_E_INVALID, "Hertz-Mindlin needs E > 0, -1 < nu <= 0.5, mu, g_n, g_t >= 0");
    if (d->tape_capacity > 0)
      return fail(ROD_E_INVALID, "Hertz-Mindlin contact is not differentiated: no tape with it");
  }
  if (d->contact_on) {
    if (!std::isfinite(d->k_contact)) return fail(ROD_E_INVALID, "k_contact must be finite");
    int e[3];
    TRY(contact_scales(d, e));
  }
  if (!(d->dipole_cutoff >= 0) || !std::isfinite(d->dipole_cutoff))
    return fail(ROD_E_INVALID, "dipole_cutoff must be finite and >= 0");
  {
    int nb = 0;
    for (int a = 0; a < 3; ++a) {
      if (!std::isfinite(d->box[a]) || d->box[a] < 0)
        return fail(ROD_E_INVALID, "box lengths must be finite and >= 0");
      nb += d->box[a] > 0;
    }
    if (nb != 0 && nb != 3) return fail(ROD_E_INVALID, "box: all three lengths > 0, or all 0");
    if (nb == 3 && d->dipole_on) {
      const double Lmin = std::min(d->box[0], std::min(d->box[1], d->box[2]));
      if (!(d->ewald_alpha > 0) || !std::isfinite(d->ewald_alpha))
        return fail(ROD_E_INVALID, "ewald_alpha must be finite and > 0");
      if (!(d->ewald_rcut > 0) || !(d->ewald_rcut <= 0.5 * Lmin))
        return fail(ROD_E_INVALID, "ewald_rcut must be in (0, min(box) / 2]");
      if (d->ewald_kmax < 1 || d->ewald_kmax > 64)
        return fail(ROD_E_INVALID, "ewald_kmax must be in [1, 64]");
      if (d->contact_on)
        return fail(ROD_E_INVALID, "a periodic box needs contact_on = 0 (contact is not periodic)");
      if (d->dipole_cutoff > 0)
        return fail(ROD_E_INVALID, "a periodic box takes the Ewald sum: dipole_cutoff must be 0");
      if (d->tape_capacity > 0)
        return fail(ROD_E_INVALID, "the Ewald sum is not differentiated: no tape with a box");
    }
  }
  if (d->dipole_on && d->dipole_cutoff > 0) {
    if (!d->contact_on)
      return fail(ROD_E_INVALID, "a dipole cutoff needs contact_on (it walks the contact cells)");
  }
  if (d->tape_capacity > 0 && d->tape_every < 1)
    return fail(ROD_E_INVALID, "a tape needs tape_every >= 1");
  for (int r = 0; r < d->n_rods; ++r)
    for (int k = d->rod_offset[r]; k + 1 < d->rod_offset[r + 1]; ++k) {
      double dx = d->x_ref[3 * (k + 1)] - d->x_ref[3 * k];
      double dy = d->x_ref[3 * (k + 1) + 1] - d->x_ref[3 * k + 1];
      double dz = d->x_ref[3 * (k + 1) + 2] - d->x_ref[3 * k + 2];
      if (!(dx * dx + dy * dy + dz * dz > 0))
        return fail(ROD_E_INVALID, "zero-length reference bond at particle %d", k);
    }
  return ROD_OK;
}

// Spatial order of the particles of member [b, e) into perm[b, e): by the
// Morton code of positions quantised to 2^21 levels over the member's largest
// extent, ties in particle order, so that consecutive entries are close in space.
static void spatial_order(const std::vector<double>& x, long N, int b, int e, int* perm) {
  double lo[3] = {1e300, 1e300, 1e300}, ext = 0.0;
  for (int a = 0; a < 3; ++a) {
    double hi = -1e300;
    for (int i = b; i < e; ++i) {
      lo[a] = std::min(lo[a], x[a * N + i]);
      hi = std::max(hi, x[a * N + i]);
    }
    ext = std::max(ext, hi - lo[a]);
  }
  const double scale = ext > 0.0 && std::isfinite(ext) ? 2097151.0 / ext : 0.0;
  auto spread = [](uint64_t v) {  // bit k of v to bit 3k
    uint64_t r = 0;
    for (int k = 0; k < 21; ++k) r |= ((v >> k) & 1ull) << (3 * k);
    return r;
  };
  std::vector<std::pair<uint64_t, int>> key((size_t)(e - b));
  for (int i = b; i < e; ++i) {
    uint64_t code = 0;
    for (int a = 0; a < 3; ++a) {
      double t = (x[a * N + i] - lo[a]) * scale;
      t = std::isfinite(t) ? std::min(2097151.0, std::max(0.0, t)) : 0.0;  // (a non-finite state)
      code |= spread((uint64_t)t) << a;
    }
    key[i - b] = {code, i};
  }
  std::sort(key.begin(), key.end());
  for (int i = b; i < e; ++i) perm[i] = key[i - b].second;
}

// Dipole work list. Split layout: blocks of 64 targets against S source ranges
// of the same member, S chosen so the launch holds about target_wgs work items
// (each range at least 128 sources). Small-member layout: blocks of
// DIP_SMALL_I targets against the whole member. small: -1 = automatic, 0 =
// split, 1 = small, 2 = split in the spatial order of the current positions
// (the ranges are then places in that order; see Dev::dperm).
static int build_dipole_plan(rod_ctx* c, int small_req, int target_wgs) {
  const std::vector<int>& mrange = c->mrange_h;
  const int M = c->desc.n_members;
  const long N = c->desc.n_particles;
  long iblocks = 0;
  int max_member = 0;
  for (int m = 0; m < M; ++m) {
    iblocks += (mrange[2 * m + 1] - mrange[2 * m] + 63) / 64;
    max_member = std::max(max_member, mrange[2 * m + 1] - mrange[2 * m]);
  }
  // Small systems: one wave per target, its lanes striding over the member.
  bool small = small_req < 0 ? (iblocks < 512 && max_member <= 2048) : small_req == 1;
  if (max_member > 16384) small = false;
  const bool spatial = small_req == 2;
  if (!c->plan_allocs.empty()) HIPC(hipStreamSynchronize(c->s));  // old plan may be in use
  for (void* p : c->plan_allocs) (void)hipFree(p);
  c->plan_allocs.clear();
  std::vector<DipWork> items;
  std::vector<int> mslots(M, 1), mlen(M, 0);
  int max_slots = 1;
  // with a dipole cutoff the list walk writes slot 0, and with a periodic box the
  // Ewald sum does: there are no work items
  for (int m = 0; m < M && c->d.dcut == 0.0 && !c->d.ew_on; ++m) {
    const int b = mrange[2 * m], e = mrange[2 * m + 1], nm = e - b;
    if (small) {
      for (int i0 = b; i0 < e; i0 += DIP_SMALL_I) {
        DipWork w{};
        w.i0 = i0; w.i1 = std::min(i0 + DIP_SMALL_I, e); w.j0 = b; w.j1 = e; w.slot = 0;
        items.push_back(w);
      }
      continue;
    }
    // enough j ranges to give the launch ~target_wgs work items, each of at least half a tile
    int S = (int)std::min<long>((target_wgs + iblocks - 1) / iblocks, (nm + 127) / 128);
    S = std::max(S, 1);
    const int len = (nm + S - 1) / S;
    S = (nm + len - 1) / len;
    mslots[m] = S;
    mlen[m] = len;
    max_slots = std::max(max_slots, S);
    for (int i0 = b; i0 < e; i0 += 64)
      for (int s = 0; s < S; ++s) {
        DipWork w{};
        w.i0 = i0; w.i1 = std::min(i0 + 64, e);
        w.j0 = b + s * len; w.j1 = std::min(e, b + (s + 1) * len);
        w.slot = s;
        items.push_back(w);
      }
  }
  // the reverse pass of a dipole cutoff: every pair of a member in one slot,
  // each tested against the cutoff (the forward walks its lists instead)
  std::vector<DipWork> adj;
  for (int m = 0; m < M && c->d.dcut > 0.0 && c->desc.tape_capacity > 0; ++m) {
    const int b = mrange[2 * m], e = mrange[2 * m + 1];
    const int bs = small ? DIP_SMALL_I : 64;
    for (int i0 = b; i0 < e; i0 += bs) {
      DipWork w{};
      w.i0 = i0; w.i1 = std::min(i0 + bs, e); w.j0 = b; w.j1 = e; w.slot = 0;
      adj.push_back(w);
    }
  }
  c->adj_nwork = (int)adj.size();
  c->adj_work = nullptr;
  if (!adj.empty()) {
    TRY(palloc(c, &c->adj_work, adj.size()));
    HIPC(hipMemcpy(c->adj_work, adj.data(), adj.size() * sizeof(DipWork), hipMemcpyHostToDevice));
  }
  c->mslots_h = mslots;
  c->mlen_h = mlen;
  c->d.dip_small = small ? 1 : 0;
  c->plan_small = spatial ? 2 : small ? 1 : 0;
  c->d.dperm = nullptr;
  c->d.sbox = nullptr;
  if (spatial && !items.empty()) {  // the order of the positions the plan is built at
    std::vector<double> xh(3 * (size_t)N);
    HIPC(hipStreamSynchronize(c->s));
    HIPC(hipMemcpy(xh.data(), c->d.x, 3 * (size_t)N * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<int> perm((size_t)N);
    for (long i = 0; i < N; ++i) perm[i] = (int)i;
    for (int m = 0; m < M; ++m) spatial_order(xh, N, mrange[2 * m], mrange[2 * m + 1], perm.data());
    int* dp = nullptr;
    TRY(palloc(c, &dp, (size_t)N));
    HIPC(hipMemcpy(dp, perm.data(), (size_t)N * sizeof(int), hipMemcpyHostToDevice));
    c->d.dperm = dp;
    TRY(palloc(c, &c->d.sbox, 6 * (size_t)((N + 63) / 64)));
  }
  c->plan_target = target_wgs;
  c->max_slots = max_slots;
  c->d.max_slots = max_slots;
  c->nwork = (int)items.size();
  TRY(palloc(c, &c->work, std::max<size_t>(1, items.size())));
  if (!items.empty())
    HIPC(hipMemcpy(c->work, items.data(), items.size() * sizeof(DipWork), hipMemcpyHostToDevice));
  int* ms = nullptr;
  TRY(palloc(c, &ms, M));
  HIPC(hipMemcpy(ms, mslots.data(), M * sizeof(int), hipMemcpyHostToDevice));
  c->d.mslots = ms;
  TRY(palloc(c, &c->d.dpart, (size_t)max_slots * 6 * N));
  c->d.dslotf = nullptr;
  if (c->desc.precision == ROD_MIXED && c->desc.dipole_on && c->d.dcut == 0.0 && !c->d.ew_on)
    TRY(palloc(c, &c->d.dslotf, (size_t)max_slots * 6 * N));
  return ROD_OK;
}

// Ewald sum of a periodic box: cells, reciprocal vectors and their weights,
// member-aligned particle chunks, structure-factor buffers.
// k vectors of the half space 0 < |n|^2 <= kmax^2 in rows of fixed (n_x, n_y)
// with n_z rising, and the rows cut into segments of at most 8 vectors
// ([first, count] pairs in *seg).
static void ewald_vectors(const rod_desc* dsc, std::vector<double>* kt,
                          std::vector<int>* seg = nullptr, std::vector<int>* rows = nullptr) {
  const double pi = 3.14159265358979323846;
  const double* L = dsc->box;
  const double V = L[0] * L[1] * L[2], a = dsc->ewald_alpha;
  const int K = dsc->ewald_kmax;
  for (int nx = 0; nx <= K; ++nx)
    for (int ny = -K; ny <= K; ++ny)
      for (int nz = -K; nz <= K; ++nz) {
        const bool half = nx > 0 || (nx == 0 && (ny > 0 || (ny == 0 && nz > 0)));
        if (!half || nx * nx + ny * ny + nz * nz > K * K) continue;
        const double kx = 2.0 * pi * nx / L[0], ky = 2.0 * pi * ny / L[1], kz = 2.0 * pi * nz / L[2];
        const double k2 = kx * kx + ky * ky + kz * kz;
        const int idx = (int)(kt->size() / 4);
        kt->push_back(kx); kt->push_back(ky); kt->push_back(kz);
        kt->push_back(2.0 * 4.0 * pi * dsc->mu0_4pi / V * std::exp(-k2 / (4.0 * a * a)) / k2);
        const bool row_start = idx == 0 || nz == -K ||
                               (*kt)[4 * (idx - 1)] != kx || (*kt)[4 * (idx - 1) + 1] != ky;
        if (seg) {  // a new segment at the start of a row or after EW_SEG vectors
          if (row_start || seg->back() == EW_SEG) {
            seg->push_back(idx);
            seg->push_back(1);
          } else {
            seg->back() += 1;
          }
        }
        if (rows) {
          if (row_start) {
            rows->push_back(idx);
            rows->push_back(1);
          } else {
            rows->back() += 1;
          }
        }
      }
}
static int ewald_count(const rod_desc* dsc, int nc[3], int* K, int* TC) {
  // cells of side >= rcut / EW_REACH: the real-space walk reaches EW_REACH cells each way
  for (int a = 0; a < 3; ++a)
    nc[a] = (int)std::max(1.0, std::min((double)EW_MAX_NC,
                                        std::floor(EW_REACH * dsc->box[a] / dsc->ewald_rcut)));
  std::vector<double> kt;
  ewald_vectors(dsc, &kt);
  *K = (int)(kt.size() / 4);
  std::vector<int> msz(dsc->n_members, 0);
  for (int r = 0; r < dsc->n_rods; ++r)
    msz[dsc->rod_member[r]] += dsc->rod_offset[r + 1] - dsc->rod_offset[r];
  int tc = 0;
  for (int m = 0; m < dsc->n_members; ++m) tc += (msz[m] + EW_CHUNK - 1) / EW_CHUNK;
  *TC = tc;
  return ROD_OK;
}
static int ewald_setup(rod_ctx* c, const rod_desc* dsc, const std::vector<int>& mrange) {
  Dev& d = c->d;
  d.ew_on = dsc->dipole_on && dsc->box[0] > 0 && dsc->box[1] > 0 && dsc->box[2] > 0;
  if (!d.ew_on) return ROD_OK;
  const int M = dsc->n_members, N = dsc->n_particles;
  int K = 0, TC = 0;
  ewald_count(dsc, d.ew_nc, &K, &TC);
  for (int a = 0; a < 3; ++a) d.box[a] = dsc->box[a];
  d.ew_alpha = dsc->ewald_alpha;
  d.ew_rc = dsc->ewald_rcut;
  d.ew_self = dsc->mu0_4pi * 4.0 * std::pow(dsc->ewald_alpha, 3) / (3.0 * std::sqrt(3.14159265358979323846));
  const long ncell = (long)d.ew_nc[0] * d.ew_nc[1] * d.ew_nc[2];
  if (ncell * M > (1L << 26))
    return fail(ROD_E_INVALID, "Ewald cells: %ld per member times %d members exceeds 2^26", ncell, M);
  d.ew_ncell = (int)ncell;
  d.ew_K = K;
  d.ew_TC = TC;
  std::vector<double> kt;
  std::vector<int> seg, rows;
  ewald_vectors(dsc, &kt, &seg, &rows);
  std::vector<int> chunks, coff(M + 1, 0);
  for (int m = 0; m < M; ++m) {
    coff[m] = (int)(chunks.size() / 3);
    for (int b = mrange[2 * m]; b < mrange[2 * m + 1]; b += EW_CHUNK) {
      chunks.push_back(b);
      chunks.push_back(std::min(b + EW_CHUNK, mrange[2 * m + 1]));
      chunks.push_back(m);
    }
  }
  coff[M] = (int)(chunks.size() / 3);
  double* kdev = nullptr;
  int *chd = nullptr, *cod = nullptr, *sgd = nullptr, *rwd = nullptr;
  TRY(dalloc(c, &d.ew_cnt, (size_t)M * ncell));
  TRY(dalloc(c, &d.ew_start, (size_t)M * ncell + 1));
  TRY(dalloc(c, &d.ew_cell, (size_t)N));
  TRY(dalloc(c, &d.ew_slot, (size_t)N));
  TRY(dalloc(c, &d.ew_tmp, (size_t)N));
  TRY(dalloc(c, &d.ew_sorted, (size_t)N));
  TRY(dalloc(c, &d.ew_xm, 8 * (size_t)N));
  d.ew_xf = nullptr;
  if (dsc->precision == ROD_MIXED) TRY(dalloc(c, &d.ew_xf, 8 * (size_t)N));
  TRY(dalloc(c, &kdev, kt.size()));
  TRY(dalloc(c, &chd, chunks.size()));
  TRY(dalloc(c, &cod, coff.size()));
  TRY(dalloc(c, &sgd, seg.size()));
  TRY(dalloc(c, &rwd, rows.size()));
  TRY(dalloc(c, &d.ew_Sp, 2 * (size_t)TC * K));
  TRY(dalloc(c, &d.ew_S, 2 * (size_t)M * K));
  HIPC(hipMemcpy(kdev, kt.data(), kt.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(chd, chunks.data(), chunks.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(cod, coff.data(), coff.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(sgd, seg.data(), seg.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(rwd, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice));
  d.ew_seg = sgd;
  d.ew_SEG = (int)(seg.size() / 2);
  d.ew_row = rwd;
  d.ew_ROWS = (int)(rows.size() / 2);
  d.ew_dkz = 2.0 * 3.14159265358979323846 / dsc->box[2];
  d.ew_k = kdev;
  d.ew_chunks = chd;
  d.ew_chunk_off = cod;
  return ROD_OK;
}

// Cells of the cutoff sort (dipole_list.h): side dcut + skin, from the lower
// corner of the reference lattice less one cell. Each axis gets the key bits
// its extent needs (plus a cell either side), the member field ceil(log2 M);
// keys have at most ceil(log2 N) + 1 bits (the widest axis gives up bits
// first: its cells then share buckets) and at least log2 DL_SCAN.
struct DlGeo { double inv, org[3]; int bits[3]; unsigned axis[3]; int mshift, nb; };
static int ceil_log2(double v) {
  int b = 0;
  while (b < 31 && std::ldexp(1.0, b) < v) ++b;
  return b;
}
static DlGeo dl_geometry(const rod_desc* d) {
  DlGeo g{};
  const double side = d->dipole_cutoff + NBR_SKIN * d->r_contact;
  g.inv = 1.0 / side;
  const int N = d->n_particles;
  for (int a = 0; a < 3; ++a) {
    double lo = d->x_ref[a], hi = d->x_ref[a];
    for (int k = 1; k < N; ++k) {
      lo = std::min(lo, d->x_ref[3 * k + a]);
      hi = std::max(hi, d->x_ref[3 * k + a]);
    }
    g.org[a] = lo - side;
    g.bits[a] = ceil_log2(std::min(std::floor((hi - g.org[a]) * g.inv) + 2.0, 1048576.0));
  }
  const int mbits = ceil_log2((double)d->n_members);
  const int max_bits = std::max(ceil_log2((double)DL_SCAN), ceil_log2((double)N) + 1);
  while (g.bits[0] + g.bits[1] + g.bits[2] + mbits > max_bits) {
    int w = 0;
    for (int a = 1; a < 3; ++a)
      if (g.bits[a] > g.bits[w]) w = a;
    if (g.bits[w] == 0) break;
    --g.bits[w];
  }
  int pos = 0;  // bit l of each axis in turn, lowest first
  for (int l = 0; l < 21; ++l)
    for (int a = 0; a < 3; ++a)
      if (l < g.bits[a]) g.axis[a] |= 1u << pos++;
  g.mshift = pos;
  g.nb = std::max(DL_SCAN, 1 << (pos + mbits));
  return g;
}

static size_t workspace_bytes(const rod_desc* d, int max_slots) {
  size_t N = d->n_particles, R = d->n_rods, M = d->n_members;
  size_t cells = d->contact_on ? next_pow2(std::max<size_t>(1024, 2 * N)) : 1;
  size_t b = 0;
  b += N * (1 + 4 + 4 + 1) + 8 * N * 4 + 8 * N * 4 + 8 * R * 4 + 4 * M * 3;  // topology
  b += 8 * 3 * N + 4 * 3 * N + 8 * 9 * N + 8 * 4 * N;                         // mu, bonds
  b += 8 * (size_t)max_slots * 6 * N + 8 * 4 * N;                               // dipole, contact
  if (d->precision == ROD_MIXED && d->dipole_on) b += 4 * (size_t)max_slots * 6 * N;  // FP32 slots
  b += 2 * (4 * cells + sizeof(CellSlot) * cells * CELL_CAP + 4 * OVF_CAP) + 4 * N;  // cells
  const bool hm = d->contact_on && d->contact_model == ROD_CONTACT_HERTZ_MINDLIN;
  const bool dcut = d->dipole_on && d->dipole_cutoff > 0;
  if (d->contact_on && ((long)N >= CONTACT_LANES_MAX_N || dcut))
    b += (4 * NBR_CAP + 4 + 24) * N;                                            // lists
  if (dcut) b += (4 * DNBR_CAP + 4 + 64) * N;                                   // dipole lists
  if (dcut) {                                                                   // cutoff sort
    const DlGeo g = dl_geometry(d);
    b += 4 * (2 * (size_t)g.nb + 1 + g.nb / DL_SCAN) + (4 * 5 + sizeof(DlRec)) * N;
  }
  if (hm) b += (24 + 8 + 2 * HM_CAP * (4 + 24)) * N;                            // torque, contacts
  if (d->dipole_on && d->box[0] > 0 && d->box[1] > 0 && d->box[2] > 0) {      // Ewald
    int nc[3], K = 0, TC = 0;
    ewald_count(d, nc, &K, &TC);
    const size_t cells = (size_t)nc[0] * nc[1] * nc[2] * M;
    b += 8 * cells + 4 + (4 * 4 + 64) * N + 32 * (size_t)K + 12 * (size_t)TC + 4 * (M + 1) +
         16 * ((size_t)TC + M) * K;
  }
  if (d->precision == ROD_MIXED && d->dipole_on) b += 48 * ((N + 63) / 64);  // chunk boxes
  if (d->dipole_on) b += 4 * N + 48 * ((N + 63) / 64);  // spatial order and its chunk boxes
  if (d->bond_damping) b += 8 * 4 * R + 8 * 2 * 5 * N;                       // bond damping
  b += 8 * 18 * N + 8 * 9 * M;                                                  // energy
  return b;
}

// ------------------------------------------------------------------ schedule
// Contact of one level. Stepping with candidate lists (lazy_cells), the cell
// list is filled first, by a launch that does nothing unless the lists are
// rebuilt (timed as a class of its own, so that the contact time is the walk's).
static int contact_term(rod_ctx* c, const Dev& d, int want_energy, int build) {
  if (d.lazy_cells && !want_energy && !contact_in_forces(d))
    TIMED(c, ROD_KERNEL_CELLS, launch_cell_insert, d, build, c->s);
  TIMED(c, ROD_KERNEL_CONTACT, launch_contact, d, want_energy, build, c->s);
  return ROD_OK;
}

// The Ewald sum, timed as a whole (dipole class) and its real-space walk alone.
static int ewald_term(rod_ctx* c, const Dev& d) {
  const hipEvent_t* evr = nullptr;
  TRY(timing_events(c, ROD_KERNEL_EWALD_REAL, &evr));
  TIMED(c, ROD_KERNEL_DIPOLE, launch_ewald, d, evr, c->s);
  return ROD_OK;
}

// build: rebuild the contact candidate lists of large systems this step.
static int force_terms(rod_ctx* c, const Dev& d, int want_energy, int build) {
  if (!want_energy && c->launch_mode == ROD_LAUNCH_BATCHED) {
    TIMED(c, ROD_KERNEL_FORCES, launch_forces, d, c->desc.precision, c->work, c->nwork, c->s);
    if (c->desc.contact_on && !contact_in_forces(d)) TRY(contact_term(c, d, 0, build));
    if (d.dcut > 0) TIMED(c, ROD_KERNEL_DIPOLE, launch_dipole_cut, d, build, c->s);
    if (d.ew_on) TRY(ewald_term(c, d));
    return ROD_OK;
  }
  TIMED(c, ROD_KERNEL_BOND, launch_bond, d, c->desc.precision, want_energy, c->s);
  if (c->desc.dipole_on && d.dcut > 0)
    TIMED(c, ROD_KERNEL_DIPOLE, launch_dipole_cut, d, build, c->s);
  else if (d.ew_on)
    TRY(ewald_term(c, d));
  else if (c->desc.dipole_on)
    TIMED(c, ROD_KERNEL_DIPOLE, launch_dipole, d, c->desc.precision, c->work, c->nwork, c->s);
  if (c->desc.contact_on) TRY(contact_term(c, d, want_energy, build));
  return ROD_OK;
}
static int force_terms(rod_ctx* c, int want_energy) { return force_terms(c, c->d, want_energy, 1); }

// Evaluations outside stepping (inspection, energies, tuning) leave the
// recorded bond damping measures and Hertz-Mindlin contacts as they are: the
// velocities they see are not the half-step ones of the step's evaluation.
struct NoRecord {
  rod_ctx* c;
  explicit NoRecord(rod_ctx* ctx) : c(ctx) { c->d.hist_write = 0; }
  ~NoRecord() { c->d.hist_write = 1; }
};

// n consecutive steps. Batched: pre, forces, then (kick, forces) for every
// further step, and post; the fused kick ends one step and starts the next, and
// the level counter it reads alternates between step[1] and step[2]. Other
// modes: pre, forces, post per step.
static int enqueue_steps(rod_ctx* c, int64_t n) {
  if (n <= 0) return ROD_OK;
  // contact by candidate lists: the particle kernels of the stepping chain leave
  // the cell list empty, and the contact launch fills it when the lists are
  // rebuilt (the cell list serves nothing else between rebuilds)
  const int lazy = c->d.contact_on && c->d.use_lists && !contact_in_forces(c->d);
  if (c->launch_mode != ROD_LAUNCH_BATCHED) {
    Dev d = c->d;
    d.lazy_cells = lazy;
    for (int64_t k = 0; k < n; ++k) {
      TIMED(c, ROD_KERNEL_PRE, launch_pre, d, PRE_STEP, c->s);
      TRY(force_terms(c, d, 0, k == 0));
      TIMED(c, ROD_KERNEL_POST, launch_post, d, POST_KICK, ROD_TERM_ALL, nullptr, nullptr,
            nullptr, c->s);
    }
    return ROD_OK;
  }
  Dev d = c->d;  // d.lc = 1
  d.lazy_cells = lazy;
  TIMED(c, ROD_KERNEL_PRE, launch_pre, d, PRE_STEP, c->s);
  TRY(force_terms(c, d, 0, 1));
  for (int64_t k = 1; k < n; ++k) {
    TIMED(c, ROD_KERNEL_KICK, launch_kick, d, nullptr, c->s);
    d.lc = 3 - d.lc;
    TRY(force_terms(c, d, 0, 0));
  }
  TIMED(c, ROD_KERNEL_POST, launch_post, d, POST_KICK, ROD_TERM_ALL, nullptr, nullptr, nullptr,
        c->s);
  return ROD_OK;
}

static int enqueue_prepare(rod_ctx* c) {
  HIPC(launch_pre(c->d, PRE_PREPARE, c->s));
  TRY(force_terms(c, 0));
  HIPC(launch_post(c->d, POST_PREPARE, ROD_TERM_ALL, nullptr, nullptr, nullptr, c->s));
  return ROD_OK;
}

// Dipole items of the current layout regrouped by rod: the same source ranges,
// target blocks cut at rod boundaries (each target's sums are unchanged).
static int build_rod_work(rod_ctx* c) {
  if (!c->rod_allocs.empty()) HIPC(hipStreamSynchronize(c->s));
  for (void* p : c->rod_allocs) (void)hipFree(p);
  c->rod_allocs.clear();
  std::vector<DipWork> items;
  c->rod_work_off.assign(1, 0);
  const int bs = c->d.dip_small ? DIP_SMALL_I : 64;
  for (int r = 0; r < c->desc.n_rods; ++r) {
    const int m = c->rod_member_h[r];
    const int b = c->mrange_h[2 * m], e = c->mrange_h[2 * m + 1];
    for (int i0 = c->rod_offset[r]; i0 < c->rod_offset[r + 1]; i0 += bs) {
      const int i1 = std::min(i0 + bs, c->rod_offset[r + 1]);
      if (c->d.dip_small) {
        DipWork w{};
        w.i0 = i0; w.i1 = i1; w.j0 = b; w.j1 = e; w.slot = 0;
        items.push_back(w);
      } else {
        for (int s = 0; s < c->mslots_h[m]; ++s) {
          DipWork w{};
          w.i0 = i0; w.i1 = i1;
          w.j0 = b + s * c->mlen_h[m]; w.j1 = std::min(e, b + (s + 1) * c->mlen_h[m]);
          w.slot = s;
          items.push_back(w);
        }
      }
    }
    c->rod_work_off.push_back((int)items.size());
  }
  void* q = nullptr;
  HIPC(hipMalloc(&q, std::max<size_t>(items.size(), 1) * sizeof(DipWork)));
  c->rod_allocs.push_back(q);
  HIPC(hipMemcpy(q, items.data(), items.size() * sizeof(DipWork), hipMemcpyHostToDevice));
  c->rod_work = (DipWork*)q;
  return ROD_OK;
}

// The plain per-rod loop: every kernel launched once per rod on that rod's particles.
static int enqueue_step_per_rod(rod_ctx* c) {
  const int R = c->desc.n_rods;
  auto rod_dev = [&](int r) {
    Dev dr = c->d;
    dr.far_ok = 0;  // waves do not start on 64-particle chunk boundaries
    dr.dperm = nullptr;  // per-rod work items are particle ranges
    dr.sbox = nullptr;
    dr.i_lo = c->rod_offset[r];
    dr.i_hi = c->rod_offset[r + 1];
    return dr;
  };
  for (int r = 0; r < R; ++r) HIPC(launch_pre(rod_dev(r), PRE_STEP, c->s));
  for (int r = 0; r < R; ++r) HIPC(launch_bond(rod_dev(r), c->desc.precision, 0, c->s));
  if (c->desc.dipole_on && c->d.dcut > 0) {
    HIPC(launch_dipole_sort(c->d, 1, c->s));  // one sort of the whole system
    for (int r = 0; r < R; ++r) HIPC(launch_dipole_cut(rod_dev(r), 1, c->s));
  }
  else if (c->d.ew_on)  // one periodic sum over every member (not separable by rod)
    HIPC(launch_ewald(c->d, nullptr, c->s));
  else if (c->desc.dipole_on)
    for (int r = 0; r < R; ++r)
      HIPC(launch_dipole(rod_dev(r), c->desc.precision, c->rod_work + c->rod_work_off[r],
                         c->rod_work_off[r + 1] - c->rod_work_off[r], c->s));
  if (c->desc.contact_on)
    for (int r = 0; r < R; ++r) HIPC(launch_contact(rod_dev(r), 0, 1, c->s));
  for (int r = 0; r < R; ++r)
    HIPC(launch_post(rod_dev(r), POST_KICK, ROD_TERM_ALL, nullptr, nullptr, nullptr, c->s));
  return ROD_OK;
}

static int enter(rod_ctx* c) {
  HIPC(hipEventRecord(c->ev_in, c->user));
  HIPC(hipStreamWaitEvent(c->s, c->ev_in, 0));
  return ROD_OK;
}
static int leave(rod_ctx* c) {
  HIPC(hipEventRecord(c->ev_out, c->s));
  HIPC(hipStreamWaitEvent(c->user, c->ev_out, 0));
  return ROD_OK;
}

static int capture_steps(rod_ctx* c, int nsteps, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIPC(hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
  int rc = ROD_OK;
  rc = enqueue_steps(c, nsteps);
  hipError_t e = hipStreamEndCapture(c->s, &g);
  if (rc != ROD_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
  if (e != hipSuccess) return fail(ROD_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(ROD_E_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
  return ROD_OK;
}

static int capture_graph(rod_ctx* c) {
  TRY(capture_steps(c, c->desc.graph_steps, &c->gexec));
  c->gsteps = c->desc.graph_steps;
  return ROD_OK;
}

// ------------------------------------------------------------------ C ABI
// ---- static staging of rod_contact_pairs_noalloc
// The pairs that entry point finds are staged in this file-scope device array
// instead of a per-call allocation: a 256-byte header whose first int counts the
// pairs, then [ROD_NOALLOC_MAX_PAIRS][2] int32 pairs. Each GPU the library runs on
// holds its own copy (8 MiB + 256 B) until the process ends. Host code never
// passes the array's name to a kernel or a copy (on the host it is only a
// stand-in): it resolves the device address once per device with
// hipGetSymbolAddress and uses that.
constexpr size_t NOALLOC_HEADER = 256;
constexpr size_t NOALLOC_BYTES =
    NOALLOC_HEADER + 2 * sizeof(int32_t) * (size_t)ROD_NOALLOC_MAX_PAIRS;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEV = 64;
static std::mutex g_scratch_init_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEV];    // device address of `scratch`, per device
static int g_scratch_state[NOALLOC_MAX_DEV];    // 0 unresolved, 1 resolved, -1 failed
static hipError_t g_scratch_err[NOALLOC_MAX_DEV];
static std::mutex g_scratch_use_mu[NOALLOC_MAX_DEV];  // one staging user per device at a time

// Resolve the address of `scratch` on device `dev`, which must be current.
// Called by rod_init; a failure is kept and reported by the entry point.
static void scratch_resolve(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return;
  std::lock_guard<std::mutex> lk(g_scratch_init_mu);
  if (g_scratch_state[dev] != 0) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr) {
    g_scratch_ptr[dev] = ptr;
    g_scratch_state[dev] = 1;
  } else {
    g_scratch_err[dev] = e;
    g_scratch_state[dev] = -1;
  }
}

extern "C" {

const char* rod_last_error(void) { return g_err.c_str(); }

int rod_query_workspace(const rod_desc* d, size_t* bytes) {
  TRY(validate(d));
  if (!bytes) return fail(ROD_E_INVALID, "bytes is NULL");
  *bytes = workspace_bytes(d, 16);
  return ROD_OK;
}

int rod_init(rod_ctx** out, const rod_desc* dsc, const rod_buffers* b, void* hip_stream,
             int32_t forces_valid) {
  if (!out) return fail(ROD_E_INVALID, "out is NULL");
  *out = nullptr;
  TRY(validate(dsc));
  if (!b || !b->x || !b->v || !b->q || !b->w || !b->force || !b->torque || !b->m_body || !b->field)
    return fail(ROD_E_INVALID, "x, v, q, w, force, torque, m_body and field buffers are required");
  rod_ctx* c = new rod_ctx();
  auto cleanup = [&](int rc) {
    rod_free(c);
    return rc;
  };
  c->desc = *dsc;
  c->ub = *b;
  c->user = (hipStream_t)hip_stream;
  const int N = dsc->n_particles, R = dsc->n_rods, M = dsc->n_members;
  c->h_step = dsc->step0;
  int rc;
  if (hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess)
    return cleanup(fail(ROD_E_HIP, "stream/event creation failed"));
  if (hipGetDevice(&c->dev) != hipSuccess) return cleanup(fail(ROD_E_HIP, "hipGetDevice failed"));
  scratch_resolve(c->dev);

  // ---- topology and constants (host)
  c->rod_offset.assign(dsc->rod_offset, dsc->rod_offset + R + 1);
  c->rod_member_h.assign(dsc->rod_member, dsc->rod_member + R);
  std::vector<int> rod(N), mem(N);
  std::vector<uint8_t> bfl(N, 0);
  std::vector<int8_t> bc(dsc->bc, dsc->bc + N);
  std::vector<double> minv(N), Iinv(N), mass(N), inertia(N), bref(4 * (size_t)N, 0.0),
      rodK(4 * (size_t)R);
  std::vector<int> mrange(2 * M);
  for (int m = 0; m < M; ++m) { mrange[2 * m] = N; mrange[2 * m + 1] = 0; }
  const double pi = 3.14159265358979323846;
  for (int r = 0; r < R; ++r) {
    const double* p = dsc->rod_params + 4 * r;
    const double dd = p[0], rho = p[1], E = p[2], nu = p[3];
    const double A = pi * dd * dd / 4.0, I = pi * dd * dd * dd * dd / 64.0,
                 J = pi * dd * dd * dd * dd / 32.0, G = E / (2.0 * (1.0 + nu));
    rodK[4 * r + 0] = E * A;         // K_r = EA / L
    rodK[4 * r + 1] = 12.0 * E * I;  // K_s = 12 EI / L^3
    rodK[4 * r + 2] = G * J;         // K_t = GJ / L
    rodK[4 * r + 3] = E * I;         // K_b = EI / L
    const double pm = rho * pi * dd * dd * dd / 6.0;           // solid sphere
    const double pI = 0.4 * pm * (0.5 * dd) * (0.5 * dd);      // 2/5 m R^2
    const int m = dsc->rod_member[r];
    for (int i = dsc->rod_offset[r]; i < dsc->rod_offset[r + 1]; ++i) {
      rod[i] = r; mem[i] = m;
      mass[i] = pm; inertia[i] = pI; minv[i] = 1.0 / pm; Iinv[i] = 1.0 / pI;
      if (i + 1 < dsc->rod_offset[r + 1]) {
        bfl[i] |= 1; bfl[i + 1] |= 2;
        double rx = dsc->x_ref[3 * (i + 1)] - dsc->x_ref[3 * i];
        double ry = dsc->x_ref[3 * (i + 1) + 1] - dsc->x_ref[3 * i + 1];
        double rz = dsc->x_ref[3 * (i + 1) + 2] - dsc->x_ref[3 * i + 2];
        bref[i] = rx; bref[N + i] = ry; bref[2 * (size_t)N + i] = rz;
        bref[3 * (size_t)N + i] = std::sqrt(rx * rx + ry * ry + rz * rz);
      }
    }
    mrange[2 * m] = std::min(mrange[2 * m], dsc->rod_offset[r]);
    mrange[2 * m + 1] = std::max(mrange[2 * m + 1], dsc->rod_offset[r + 1]);
  }
  c->bref_h = bref;
  c->rodK_h = rodK;
  c->bflags_h = bfl;
  c->rod_h = rod;

  // ---- device workspace
  Dev& d = c->d;
  d = Dev{};
  d.n = N; d.R = R; d.M = M;
  d.i_lo = 0; d.i_hi = N;
  d.x = b->x; d.v = b->v; d.q = b->q; d.w = b->w; d.F = b->force; d.T = b->torque;
  d.mb = b->m_body; d.field = b->field; d.extF = b->ext_force; d.extT = b->ext_torque;
  uint8_t* bflags; int *rod_d, *mem_d, *mrange_d; int8_t* bc_d;
  double *minv_d, *Iinv_d, *mass_d, *inertia_d, *bref_d, *rodK_d;
  if ((rc = dalloc(c, &bflags, N)) || (rc = dalloc(c, &rod_d, N)) || (rc = dalloc(c, &mem_d, N)) ||
      (rc = dalloc(c, &bc_d, N)) || (rc = dalloc(c, &minv_d, N)) || (rc = dalloc(c, &Iinv_d, N)) ||
      (rc = dalloc(c, &mass_d, N)) || (rc = dalloc(c, &inertia_d, N)) ||
      (rc = dalloc(c, &bref_d, 4 * (size_t)N)) || (rc = dalloc(c, &rodK_d, 4 * (size_t)R)) ||
      (rc = dalloc(c, &mrange_d, 2 * (size_t)M)))
    return cleanup(rc);
  struct Up { void* dst; const void* src; size_t bytes; } ups[] = {
      {bflags, bfl.data(), (size_t)N}, {rod_d, rod.data(), 4 * (size_t)N},
      {mem_d, mem.data(), 4 * (size_t)N}, {bc_d, bc.data(), (size_t)N},
      {minv_d, minv.data(), 8 * (size_t)N}, {Iinv_d, Iinv.data(), 8 * (size_t)N},
      {mass_d, mass.data(), 8 * (size_t)N}, {inertia_d, inertia.data(), 8 * (size_t)N},
      {bref_d, bref.data(), 32 * (size_t)N}, {rodK_d, rodK.data(), 32 * (size_t)R},
      {mrange_d, mrange.data(), 8 * (size_t)M}};
  for (auto& u : ups)
    if (hipMemcpy(u.dst, u.src, u.bytes, hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(ROD_E_HIP, "upload failed"));
  d.bflags = bflags; d.rod = rod_d; d.mem = mem_d; d.bc = bc_d;
  d.minv = minv_d; d.Iinv = Iinv_d; d.mass = mass_d; d.inertia = inertia_d;
  d.bref = bref_d; d.rodK = rodK_d; d.mrange = mrange_d;
  float* muf = nullptr;
  if ((rc = dalloc(c, &d.mu, 3 * (size_t)N)) || (rc = dalloc(c, &muf, 3 * (size_t)N)) ||
      (rc = dalloc(c, &d.bF, 3 * (size_t)N)) || (rc = dalloc(c, &d.bTs, 3 * (size_t)N)) ||
      (rc = dalloc(c, &d.bTbt, 3 * (size_t)N)) || (rc = dalloc(c, &d.bE, 4 * (size_t)N)) ||
      (rc = dalloc(c, &d.cF, 3 * (size_t)N)) || (rc = dalloc(c, &d.cE, (size_t)N)) ||
      (rc = dalloc(c, &d.key, (size_t)N)) || (rc = dalloc(c, &d.ovf_list, 2 * (size_t)OVF_CAP)) ||
      (rc = dalloc(c, &d.ovf_cnt, 2)) || (rc = dalloc(c, &d.flags, FLAG_COUNT)) ||
      (rc = dalloc(c, &d.step, 3)) ||
      (rc = dalloc(c, &c->epart, 18 * (size_t)N)) || (rc = dalloc(c, &c->eout, 9 * (size_t)M)) ||
      (rc = dalloc(c, &c->pair_count, 1)))
    return cleanup(rc);
  d.muf = dsc->precision == ROD_MIXED ? muf : nullptr;
  if (dsc->precision == ROD_MIXED && dsc->dipole_on) {
    if ((rc = dalloc(c, &d.cbox, 6 * (size_t)((N + 63) / 64)))) return cleanup(rc);
    d.far_ok = 1;
  }
  size_t cells = dsc->contact_on ? next_pow2(std::max<size_t>(1024, 2 * (size_t)N)) : 1;
  if ((rc = dalloc(c, &d.cell_cnt, 2 * cells)) ||
      (rc = dalloc(c, &d.cell_slot, 2 * cells * CELL_CAP)))
    return cleanup(rc);
  d.cell_mask = (unsigned)(cells - 1);
  d.dt = dsc->dt; d.damping = dsc->damping; d.C = dsc->mu0_4pi; d.kc = dsc->k_contact;
  d.rc = dsc->r_contact; d.inv_cell = dsc->contact_on ? 1.0 / dsc->r_contact : 0.0;
  for (int q = 0; q < 3; ++q) { d.fix_scale[q] = 1.0; d.fix_inv[q] = 1.0; }
  if (dsc->contact_on) {
    int e[3];
    if ((rc = contact_scales(dsc, e))) return cleanup(rc);
    for (int q = 0; q < 3; ++q) {
      d.fix_scale[q] = std::ldexp(1.0, e[q]);
      d.fix_inv[q] = std::ldexp(1.0, -e[q]);
    }
  }
  d.depth = dsc->exclude_depth; d.field_len = dsc->field_len;
  d.hm = dsc->contact_on && dsc->contact_model == ROD_CONTACT_HERTZ_MINDLIN;
  d.dcut = dsc->dipole_on && dsc->dipole_cutoff > 0 ? dsc->dipole_cutoff : 0.0;
  d.use_lists = dsc->contact_on && ((long)N >= CONTACT_LANES_MAX_N || d.dcut > 0);
  d.lazy_cells = 0;  // set in the stepping chain's copy
  d.skin = NBR_SKIN * dsc->r_contact;
  // with lists the 27 cells around a particle must cover the list cutoff r_c + skin
  if (d.use_lists) d.inv_cell = 1.0 / (dsc->r_contact + d.skin);
  d.dnbr = nullptr; d.dnbr_cnt = nullptr; d.xm = nullptr;
  d.dl_cnt = d.dl_aux = d.dl_start = d.dl_bkt = d.dl_slot = d.dl_tmp = d.dl_sorted = d.dl_pos = nullptr;
  d.dl_rec = nullptr;
  d.dl_nb = 0;
  if (d.dcut > 0) {
    const DlGeo g = dl_geometry(dsc);
    d.dl_inv = g.inv;
    for (int a = 0; a < 3; ++a) {
      d.dl_org[a] = g.org[a]; d.dl_bits[a] = g.bits[a]; d.dl_axis[a] = g.axis[a];
    }
    d.dl_mshift = g.mshift;
    d.dl_nb = g.nb;
    if ((rc = dalloc(c, &d.dl_cnt, (size_t)g.nb)) || (rc = dalloc(c, &d.dl_aux, (size_t)g.nb / DL_SCAN)) ||
        (rc = dalloc(c, &d.dl_start, (size_t)g.nb + 1)) || (rc = dalloc(c, &d.dl_bkt, (size_t)N)) ||
        (rc = dalloc(c, &d.dl_slot, (size_t)N)) || (rc = dalloc(c, &d.dl_tmp, (size_t)N)) ||
        (rc = dalloc(c, &d.dl_sorted, (size_t)N)) || (rc = dalloc(c, &d.dl_pos, (size_t)N)) ||
        (rc = dalloc(c, &d.dl_rec, (size_t)N)))
      return cleanup(rc);
  }
  d.ibm_u = nullptr; d.ibm_f = nullptr; d.ibm_idt = 1.0;
  if (d.dcut > 0 && ((rc = dalloc(c, &d.dnbr, (size_t)DNBR_CAP * N)) ||
                     (rc = dalloc(c, &d.dnbr_cnt, (size_t)N)) ||
                     (rc = dalloc(c, &d.xm, 8 * (size_t)N))))
    return cleanup(rc);
  if (d.dcut > 0 && hipMemset(d.dnbr_cnt, 0, sizeof(int) * (size_t)N) != hipSuccess)
    return cleanup(fail(ROD_E_HIP, "memset failed"));
  if ((rc = ewald_setup(c, dsc, mrange))) return cleanup(rc);
  if (d.use_lists &&
      ((rc = dalloc(c, &d.nbr, (size_t)NBR_CAP * N)) || (rc = dalloc(c, &d.nbr_cnt, (size_t)N)) ||
       (rc = dalloc(c, &d.xb, 3 * (size_t)N)) || (rc = dalloc(c, &d.rebuild, 2))))
    return cleanup(rc);
  d.dipole_on = dsc->dipole_on != 0; d.contact_on = dsc->contact_on != 0;
  d.cT = nullptr; d.hc_cnt = nullptr; d.hc_j = nullptr; d.hc_s = nullptr;
  if (d.hm) {
    const double E = dsc->contact_hm[0], nu = dsc->contact_hm[1];
    d.hm_Es = E / (2.0 * (1.0 - nu * nu));
    d.hm_Gs = E / (4.0 * (2.0 - nu) * (1.0 + nu));
    d.hm_Rs = 0.25 * dsc->r_contact;
    d.hm_mu = dsc->contact_hm[2]; d.hm_gn = dsc->contact_hm[3]; d.hm_gt = dsc->contact_hm[4];
    if ((rc = dalloc(c, &d.cT, 3 * (size_t)N)) || (rc = dalloc(c, &d.hc_cnt, 2 * (size_t)N)) ||
        (rc = dalloc(c, &d.hc_j, 2 * (size_t)HM_CAP * N)) ||
        (rc = dalloc(c, &d.hc_s, 6 * (size_t)HM_CAP * N)))
      return cleanup(rc);
  }
  // the first evaluation (at step0) has no previous level; all of stepping's
  // and rod_init's evaluations record their measures and contacts
  d.hist_from = dsc->step0 + 1;
  d.hist_write = 1;
  d.bdamp = nullptr;
  d.hist = nullptr;
  if (dsc->bond_damping) {
    bool any = false;
    for (int k = 0; k < 4 * R; ++k) any = any || dsc->bond_damping[k] != 0;
    if (any) {
      double* g = nullptr;
      if ((rc = dalloc(c, &g, 4 * (size_t)R)) || (rc = dalloc(c, &d.hist, 2 * 5 * (size_t)N)))
        return cleanup(rc);
      if (hipMemcpy(g, dsc->bond_damping, 32 * (size_t)R, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(ROD_E_HIP, "upload failed"));
      d.bdamp = g;
    }
  }
  {
    double a = std::sqrt(dsc->drive_axis[0] * dsc->drive_axis[0] +
                         dsc->drive_axis[1] * dsc->drive_axis[1] +
                         dsc->drive_axis[2] * dsc->drive_axis[2]);
    for (int k = 0; k < 3; ++k) d.axis[k] = a > 0 ? dsc->drive_axis[k] / a : 0.0;
  }
  d.period = dsc->drive_period > 0 ? dsc->drive_period : 1;
  d.lc = 1;
  long long s0[3] = {dsc->step0, dsc->step0, dsc->step0};
  if (hipMemcpy(d.step, s0, sizeof(s0), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(ROD_E_HIP, "upload failed"));
  c->mrange_h = mrange;
  if ((rc = build_dipole_plan(c, -1, 1024))) return cleanup(rc);
  // descriptor host pointers are not kept
  c->desc.rod_offset = nullptr; c->desc.rod_member = nullptr; c->desc.rod_params = nullptr;
  c->desc.x_ref = nullptr; c->desc.bc = nullptr; c->desc.bond_damping = nullptr;
  if ((rc = tape_init(c->tape, c->d, dsc->tape_every, dsc->tape_capacity, c->allocs))) {
    return cleanup(fail(rc, "tape allocation failed"));
  }

  // ---- initial state: normalise q, boundary conditions, forces of level step0
  if ((rc = enter(c))) return cleanup(rc);
  if (forces_valid) {
    if (hipSuccess != launch_pre(c->d, PRE_PREPARE, c->s)) return cleanup(fail(ROD_E_HIP, "launch failed"));
    // bond damping and Hertz-Mindlin contact: record the measures and contacts
    // of this level (the forces are the caller's)
    if (c->d.bdamp && hipSuccess != launch_bond(c->d, dsc->precision, 0, c->s))
      return cleanup(fail(ROD_E_HIP, "launch failed"));
    if (c->d.hm && hipSuccess != launch_contact(c->d, 0, 1, c->s))
      return cleanup(fail(ROD_E_HIP, "launch failed"));
  } else if ((rc = enqueue_prepare(c))) {
    return cleanup(rc);
  }
  if ((rc = leave(c))) return cleanup(rc);
  if (forces_valid && d.contact_on) {
    // pre built the cell list without a force pass; empty it again
    if (hipStreamSynchronize(c->s) != hipSuccess) return cleanup(fail(ROD_E_HIP, "sync failed"));
    if (hipMemset(d.cell_cnt, 0, 2 * cells * sizeof(int)) != hipSuccess ||
        hipMemset(d.ovf_cnt, 0, 2 * sizeof(int)) != hipSuccess)
      return cleanup(fail(ROD_E_HIP, "memset failed"));
  }
  *out = c;
  return ROD_OK;
}

int rod_step(rod_ctx* c, int64_t n) {
  if (!c) return fail(ROD_E_INVALID, "context is NULL");
  if (n < 0) return fail(ROD_E_INVALID, "n_steps must be >= 0");
  if (n == 0) return ROD_OK;
  TRY(enter(c));
  if (c->tape.active) {
    // Checkpoint every tape_every steps; whole checkpoint intervals replay a graph.
    const int every = c->tape.every;
    int64_t k = 0;
    while (k < n) {
      const int64_t rel = c->h_step + k - c->tape.start_step;
      TRY(tape_before_step(c->tape, c->d, c->s, c->h_step + k));
      if (!c->timing && rel % every == 0 && n - k >= every && rel + every <= c->tape.capacity) {
        if (!c->tgexec) TRY(capture_steps(c, every, &c->tgexec));
        HIPC(hipGraphLaunch(c->tgexec, c->s));
        k += every;
      } else {
        TRY(enqueue_steps(c, 1));
        k += 1;
      }
    }
  } else if (c->launch_mode == ROD_LAUNCH_PER_ROD) {
    for (int64_t k = 0; k < n; ++k) TRY(enqueue_step_per_rod(c));
  } else {
    int64_t left = n;
    if (!c->timing && c->desc.graph_steps > 0 && left >= c->desc.graph_steps) {
      if (!c->gexec) TRY(capture_graph(c));
      while (left >= c->gsteps) {
        HIPC(hipGraphLaunch(c->gexec, c->s));
        left -= c->gsteps;
      }
    }
    TRY(enqueue_steps(c, left));
  }
  c->h_step += n;
  TRY(leave(c));
  return ROD_OK;
}

int rod_sync(rod_ctx* c) {
  if (!c) return fail(ROD_E_INVALID, "context is NULL");
  HIPC(hipStreamSynchronize(c->s));
  unsigned f[FLAG_COUNT];
  HIPC(hipMemcpy(f, c->d.flags, sizeof(f), hipMemcpyDeviceToHost));
  unsigned any = 0;
  for (int k = 0; k < FLAG_COUNT; ++k) any |= f[k];
  if (any) {
    unsigned z[FLAG_COUNT] = {};
    HIPC(hipMemcpy(c->d.flags, z, sizeof(z), hipMemcpyHostToDevice));
    if (f[FLAG_NONFINITE]) return fail(ROD_E_NONFINITE, "non-finite force, torque or position");
    if (f[FLAG_CONTACT_RANGE])
      return fail(ROD_E_OVERFLOW, "a contact pair's force, torque or energy was non-finite or "
                  "2^28 times the contact law's bound or more: outside the range of the exact "
                  "contact sums");
    if (f[FLAG_HM_OVF])
      return fail(ROD_E_OVERFLOW, "a particle had more than %d Hertz-Mindlin contacts", HM_CAP);
    if (f[FLAG_DIP_OVF])
      return fail(ROD_E_OVERFLOW, "a particle had more than %d neighbours within the dipole "
                  "cutoff and skin", DNBR_CAP);
    return fail(ROD_E_OVERFLOW, "contact search capacity exceeded: more than %d particles "
                "landed in full cells", OVF_CAP);
  }
  return ROD_OK;
}

int rod_get_step(rod_ctx* c, int64_t* step) {
  if (!c || !step) return fail(ROD_E_INVALID, "NULL argument");
  HIPC(hipStreamSynchronize(c->s));
  long long s = 0;
  HIPC(hipMemcpy(&s, c->d.step, sizeof(s), hipMemcpyDeviceToHost));
  if (s != c->h_step) return fail(ROD_E_STATE, "device step %lld differs from host %lld", s, (long long)c->h_step);
  *step = s;
  return ROD_OK;
}

int rod_eval_forces(rod_ctx* c, int32_t terms, double* F, double* T, double* B) {
  if (!c || !F || !T) return fail(ROD_E_INVALID, "NULL argument");
  if (terms < 0 || terms > ROD_TERM_ALL) return fail(ROD_E_INVALID, "bad term mask %d", terms);
  NoRecord keep(c);
  TRY(enter(c));
  HIPC(launch_pre(c->d, PRE_EVAL, c->s));
  TRY(force_terms(c, 0));
  HIPC(launch_post(c->d, POST_EVAL, terms, F, T, B, c->s));
  TRY(leave(c));
  return ROD_OK;
}

int rod_energy(rod_ctx* c, double* out, int32_t on_device) {
  if (!c || !out) return fail(ROD_E_INVALID, "NULL argument");
  NoRecord keep(c);
  TRY(enter(c));
  HIPC(launch_pre(c->d, PRE_EVAL, c->s));
  TRY(force_terms(c, 1));
  HIPC(launch_energy(c->d, c->epart, c->eout, c->s));
  const size_t bytes = 9 * sizeof(double) * c->d.M;
  if (on_device) {
    HIPC(hipMemcpyAsync(out, c->eout, bytes, hipMemcpyDeviceToDevice, c->s));
    TRY(leave(c));
  } else {
    HIPC(hipMemcpyAsync(out, c->eout, bytes, hipMemcpyDeviceToHost, c->s));
    TRY(leave(c));
    HIPC(hipStreamSynchronize(c->s));
  }
  return ROD_OK;
}

int rod_topology(rod_ctx* c, int32_t* ij, double* rref, double* K, int32_t cap, int32_t* count) {
  if (!c || !count) return fail(ROD_E_INVALID, "NULL argument");
  const long N = c->d.n;
  int B = 0;
  for (long k = 0; k < N; ++k) {
    if (!(c->bflags_h[k] & 1)) continue;
    if (B < cap) {
      if (ij) { ij[2 * B] = (int)k; ij[2 * B + 1] = (int)k + 1; }
      const double r0 = c->bref_h[3 * N + k];
      if (rref) for (int a = 0; a < 3; ++a) rref[3 * B + a] = c->bref_h[a * N + k];
      if (K) {
        const double* k4 = &c->rodK_h[4 * c->rod_h[k]];
        K[4 * B + 0] = k4[0] / r0;
        K[4 * B + 1] = k4[1] / (r0 * r0 * r0);
        K[4 * B + 2] = k4[2] / r0;
        K[4 * B + 3] = k4[3] / r0;
      }
    }
    ++B;
  }
  *count = B;
  return ROD_OK;
}

int rod_contact_pairs(rod_ctx* c, int32_t* pairs, int32_t cap, int32_t* count) {
  if (!c || !count || (cap > 0 && !pairs)) return fail(ROD_E_INVALID, "NULL argument");
  *count = 0;
  if (!c->desc.contact_on) return ROD_OK;
  int32_t* dp = nullptr;
  const int dcap = std::max(cap, 1);
  HIPC(hipMalloc(&dp, 2 * sizeof(int32_t) * dcap));
  int rc = ROD_OK;
  do {
    if ((rc = enter(c))) break;
    if (hipMemsetAsync(c->pair_count, 0, sizeof(int), c->s) != hipSuccess ||
        launch_pre(c->d, PRE_EVAL, c->s) != hipSuccess ||
        launch_contact_pairs(c->d, dp, cap, c->pair_count, c->s) != hipSuccess ||
        launch_clear_cells(c->d, c->s) != hipSuccess) {
      rc = fail(ROD_E_HIP, "launch failed");
      break;
    }
    if ((rc = leave(c))) break;
    int cnt = 0;
    if (hipStreamSynchronize(c->s) != hipSuccess ||
        hipMemcpy(&cnt, c->pair_count, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
      rc = fail(ROD_E_HIP, "readback failed");
      break;
    }
    int nw = std::min(cnt, cap);
    if (nw > 0) {
      if (hipMemcpy(pairs, dp, 2 * sizeof(int32_t) * nw, hipMemcpyDeviceToHost) != hipSuccess) {
        rc = fail(ROD_E_HIP, "readback failed");
        break;
      }
      std::vector<std::pair<int, int>> v(nw);
      for (int k = 0; k < nw; ++k) v[k] = {pairs[2 * k], pairs[2 * k + 1]};
      std::sort(v.begin(), v.end());
      for (int k = 0; k < nw; ++k) { pairs[2 * k] = v[k].first; pairs[2 * k + 1] = v[k].second; }
    }
    *count = cnt;
  } while (0);
  (void)hipFree(dp);
  return rc;
}

// The pairs of one search, sorted in place (i, then j ascending), with no
// allocation: a pair is two adjacent int32 of the caller's array.
namespace {
struct PairI32 { int32_t i, j; };
static_assert(sizeof(PairI32) == 2 * sizeof(int32_t), "pair layout");
}  // namespace

int rod_contact_pairs_noalloc(rod_ctx* c, int32_t* pairs, int32_t cap, int32_t* count) {
  if (!c || !count || (cap > 0 && !pairs)) return fail(ROD_E_INVALID, "NULL argument");
  if (cap < 0 || cap > ROD_NOALLOC_MAX_PAIRS)
    return fail(ROD_E_INVALID, "cap %d is outside [0, %d], the static staging capacity", cap,
                ROD_NOALLOC_MAX_PAIRS);
  *count = 0;
  if (!c->desc.contact_on) return ROD_OK;
  if (c->dev < 0 || c->dev >= NOALLOC_MAX_DEV)
    return fail(ROD_E_INVALID, "device %d has no static staging (at most %d devices)", c->dev,
                NOALLOC_MAX_DEV);
  if (g_scratch_state[c->dev] != 1)
    return fail(ROD_E_HIP, "static staging of device %d is unavailable: %s", c->dev,
                hipGetErrorString(g_scratch_err[c->dev]));
  std::lock_guard<std::mutex> lk(g_scratch_use_mu[c->dev]);
  int32_t* dcount = (int32_t*)g_scratch_ptr[c->dev];
  int32_t* dpairs = (int32_t*)((char*)g_scratch_ptr[c->dev] + NOALLOC_HEADER);
  TRY(enter(c));
  if (launch_fill_i32(dcount, 1, 0, c->s) != hipSuccess ||
      launch_pre(c->d, PRE_EVAL, c->s) != hipSuccess ||
      launch_contact_pairs(c->d, dpairs, cap, dcount, c->s) != hipSuccess ||
      launch_clear_cells(c->d, c->s) != hipSuccess)
    return fail(ROD_E_HIP, "launch failed");
  TRY(leave(c));
  int cnt = 0;
  HIPC(hipStreamSynchronize(c->s));
  HIPC(hipMemcpy(&cnt, dcount, sizeof(int32_t), hipMemcpyDeviceToHost));
  const int nw = std::min(cnt, cap);
  if (nw > 0) {
    HIPC(hipMemcpy(pairs, dpairs, 2 * sizeof(int32_t) * (size_t)nw, hipMemcpyDeviceToHost));
    PairI32* pv = reinterpret_cast<PairI32*>(pairs);
    std::sort(pv, pv + nw, [](const PairI32& a, const PairI32& b) {
      return a.i != b.i ? a.i < b.i : a.j < b.j;
    });
  }
  *count = cnt;
  return ROD_OK;
}

// Contact history of the current level: parity h_step & 1 of the per-level
// planes, which the level's force evaluation wrote and the next step reads.
int rod_get_contact_history(rod_ctx* c, int32_t* count, int32_t* partner, double* disp) {
  if (!c || !count || !partner || !disp) return fail(ROD_E_INVALID, "NULL argument");
  if (!c->d.hm) return fail(ROD_E_STATE, "the context has no Hertz-Mindlin contact");
  const long N = c->d.n, p = c->h_step & 1;
  std::vector<int> cnt(N), pj((size_t)HM_CAP * N);
  std::vector<double> ps((size_t)3 * HM_CAP * N);
  HIPC(hipStreamSynchronize(c->s));
  HIPC(hipMemcpy(cnt.data(), c->d.hc_cnt + p * N, sizeof(int) * N, hipMemcpyDeviceToHost));
  HIPC(hipMemcpy(pj.data(), c->d.hc_j + p * HM_CAP * N, sizeof(int) * HM_CAP * N,
                 hipMemcpyDeviceToHost));
  HIPC(hipMemcpy(ps.data(), c->d.hc_s + p * 3 * HM_CAP * N, sizeof(double) * 3 * HM_CAP * N,
                 hipMemcpyDeviceToHost));
  for (long i = 0; i < N; ++i) {
    const int n = std::min(std::max(cnt[i], 0), HM_CAP);
    count[i] = n;
    for (int k = 0; k < HM_CAP; ++k) {
      const bool on = k < n;
      partner[i * HM_CAP + k] = on ? pj[(size_t)k * N + i] : 0;
      for (int a = 0; a < 3; ++a)
        disp[(i * HM_CAP + k) * 3 + a] = on ? ps[((size_t)a * HM_CAP + k) * N + i] : 0.0;
    }
  }
  return ROD_OK;
}

int rod_set_contact_history(rod_ctx* c, const int32_t* count, const int32_t* partner,
                            const double* disp) {
  if (!c || !count || !partner || !disp) return fail(ROD_E_INVALID, "NULL argument");
  if (!c->d.hm) return fail(ROD_E_STATE, "the context has no Hertz-Mindlin contact");
  const long N = c->d.n, p = c->h_step & 1;
  std::vector<int> cnt(N), pj((size_t)HM_CAP * N, 0);
  std::vector<double> ps((size_t)3 * HM_CAP * N, 0.0);
  for (long i = 0; i < N; ++i) {
    const int n = count[i];
    if (n < 0 || n > HM_CAP)
      return fail(ROD_E_INVALID, "count[%ld] = %d is outside [0, %d]", i, n, HM_CAP);
    cnt[i] = n;
    for (int k = 0; k < n; ++k) {
      const int j = partner[i * HM_CAP + k];
      if (j < 0 || j >= N || j == i)
        return fail(ROD_E_INVALID, "partner[%ld][%d] = %d is not another particle", i, k, j);
      pj[(size_t)k * N + i] = j;
      for (int a = 0; a < 3; ++a) {
        const double v = disp[(i * HM_CAP + k) * 3 + a];
        if (!std::isfinite(v))
          return fail(ROD_E_INVALID, "disp[%ld][%d] is not finite", i, k);
        ps[((size_t)a * HM_CAP + k) * N + i] = v;
      }
    }
  }
  HIPC(hipStreamSynchronize(c->s));
  HIPC(hipMemcpy(c->d.hc_cnt + p * N, cnt.data(), sizeof(int) * N, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(c->d.hc_j + p * HM_CAP * N, pj.data(), sizeof(int) * HM_CAP * N,
                 hipMemcpyHostToDevice));
  HIPC(hipMemcpy(c->d.hc_s + p * 3 * HM_CAP * N, ps.data(), sizeof(double) * 3 * HM_CAP * N,
                 hipMemcpyHostToDevice));
  return ROD_OK;
}

int rod_tape_begin(rod_ctx* c) {
  if (!c) return fail(ROD_E_INVALID, "context is NULL");
  if (c->tape.capacity <= 0) return fail(ROD_E_NOTAPE, "context was created without a tape");
  TRY(enter(c));
  TRY(enqueue_prepare(c));
  TRY(tape_start(c->tape, c->d, c->s, c->h_step));
  TRY(leave(c));
  return ROD_OK;
}

int rod_grad(rod_ctx* c, const rod_cotangent* gy, rod_gradients* gx) {
  if (!c || !gy || !gx) return fail(ROD_E_INVALID, "NULL argument");
  if (!c->tape.active || c->h_step == c->tape.start_step)
    return fail(ROD_E_NOTAPE, "no recorded steps: call rod_tape_begin, then rod_step");
  TRY(enter(c));
  const bool cut = c->d.dcut > 0.0;
  TRY(adjoint_run(c->tape, c->d, c->desc.precision, cut ? c->adj_work : c->work,
                  cut ? c->adj_nwork : c->nwork, c->s, c->h_step, gy, gx));
  TRY(leave(c));
  return ROD_OK;
}

int rod_timing(rod_ctx* c, int32_t enable) {
  if (!c) return fail(ROD_E_INVALID, "context is NULL");
  TRY(timing_collect(c));
  c->timing = enable != 0;
  for (int k = 0; k < ROD_KERNEL_COUNT; ++k) { c->t_ms[k] = 0.0; c->t_cnt[k] = 0; }
  return ROD_OK;
}

int rod_kernel_times(rod_ctx* c, double* ms, int64_t* launches) {
  if (!c) return fail(ROD_E_INVALID, "context is NULL");
  TRY(timing_collect(c));
  for (int k = 0; k < ROD_KERNEL_COUNT; ++k) {
    if (ms) ms[k] = c->t_ms[k];
    if (launches) launches[k] = c->t_cnt[k];
    c->t_ms[k] = 0.0;
    c->t_cnt[k] = 0;
  }
  return ROD_OK;
}

// ------------------------------------------------------------------ autotuner
static void drop_graphs(rod_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->tgexec) (void)hipGraphExecDestroy(c->tgexec);
  c->gexec = c->tgexec = nullptr;
  c->gsteps = 0;
  tape_release(c->tape);
}

// Microseconds per force evaluation (pre, forces, gather) of the current layout.
static int time_eval(rod_ctx* c, double* us) {
  double* F = c->epart;  // scratch: [3N] force and [3N] torque
  double* T = c->epart + 3 * c->d.n;
  NoRecord keep(c);
  auto eval = [&]() -> int {
    HIPC(launch_pre(c->d, PRE_EVAL, c->s));
    TRY(force_terms(c, 0));
    HIPC(launch_post(c->d, POST_EVAL, ROD_TERM_ALL, F, T, nullptr, c->s));
    return ROD_OK;
  };
  hipEvent_t a, b;
  HIPC(hipEventCreate(&a));
  HIPC(hipEventCreate(&b));
  int rc = ROD_OK;
  float ms = 0.f;
  int reps = 3;
  for (int k = 0; k < 3 && rc == ROD_OK; ++k) rc = eval();  // warm-up
  for (int round = 0; round < 2 && rc == ROD_OK; ++round) {
    if (hipEventRecord(a, c->s) != hipSuccess) { rc = fail(ROD_E_HIP, "event record failed"); break; }
    for (int k = 0; k < reps && rc == ROD_OK; ++k) rc = eval();
    if (rc != ROD_OK) break;
    if (hipEventRecord(b, c->s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess) { rc = fail(ROD_E_HIP, "event timing failed"); break; }
    // aim at ~5 ms of timed work (at most 200 evaluations)
    const double per = std::max(1e-3, (double)ms / reps);
    if (round == 0) reps = (int)std::min(200.0, std::max(3.0, 5.0 / per));
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc == ROD_OK) *us = 1e3 * (double)ms / reps;
  return rc;
}

static std::string tune_key(rod_ctx* c) {
  hipDeviceProp_t p;
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
    arch = p.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the member sizes
  for (size_t k = 0; k + 1 < c->mrange_h.size(); k += 2) {
    uint64_t v = (uint64_t)(c->mrange_h[k + 1] - c->mrange_h[k]);
    for (int b = 0; b < 8; ++b) { h ^= (v >> (8 * b)) & 0xff; h *= 1099511628211ull; }
  }
  char buf[256];
  snprintf(buf, sizeof(buf), "%s|prec=%d|N=%ld|M=%d|sizes=%016llx", arch.c_str(),
           c->desc.precision, c->d.n, c->d.M, (unsigned long long)h);
  return buf;
}

extern "C" int rod_launch_mode(rod_ctx* c, int32_t mode) {
  if (!c) return fail(ROD_E_INVALID, "context is NULL");
  if (mode != ROD_LAUNCH_BATCHED && mode != ROD_LAUNCH_PER_ROD && mode != ROD_LAUNCH_SEPARATE)
    return fail(ROD_E_INVALID, "mode must be one of ROD_LAUNCH_BATCHED, _PER_ROD, _SEPARATE");
  if (c->tape.active) return fail(ROD_E_STATE, "launch mode change while a tape is recorded");
  if (mode == c->launch_mode) return ROD_OK;
  TRY(enter(c));
  if (mode == ROD_LAUNCH_PER_ROD) TRY(build_rod_work(c));
  HIPC(hipStreamSynchronize(c->s));  // captured steps of the old mode may still run
  drop_graphs(c);
  c->launch_mode = mode;
  TRY(leave(c));
  return ROD_OK;
}

extern "C" int rod_dipole_layout(rod_ctx* c, int32_t small, int32_t target_wgs) {
  if (!c) return fail(ROD_E_INVALID, "context is NULL");
  if (small < -1 || small > 2 || target_wgs < 1)
    return fail(ROD_E_INVALID, "small must be -1, 0, 1 or 2 and target_wgs >= 1");
  if (c->tape.active) return fail(ROD_E_STATE, "layout change while a tape is recorded");
  TRY(enter(c));
  TRY(build_dipole_plan(c, small, target_wgs));
  if (c->launch_mode == ROD_LAUNCH_PER_ROD) TRY(build_rod_work(c));
  drop_graphs(c);
  TRY(leave(c));
  return ROD_OK;
}

static const char* layout_name(int small) {
  return small == 1 ? "small-member layout" : small == 2 ? "spatial split layout" : "split layout";
}

extern "C" int rod_autotune(rod_ctx* c, const char* cache_path, int32_t force, char* report,
                            int32_t report_len) {
  if (!c) return fail(ROD_E_INVALID, "context is NULL");
  if (c->tape.active) return fail(ROD_E_STATE, "autotune while a tape is recorded");
  std::string rep, key = tune_key(c);
  int small = -1, target = 0;
  bool cached = false;
  double best_us = 0.0;
  if (cache_path && !force) {  // look the problem up in the cache
    if (FILE* f = fopen(cache_path, "r")) {
      char line[512], k[300];
      while (fgets(line, sizeof(line), f)) {
        int s_, t_;
        double u_;
        if (sscanf(line, "{\"key\": \"%299[^\"]\", \"small\": %d, \"target_wgs\": %d, \"us_per_eval\": %lf",
                   k, &s_, &t_, &u_) == 4 && key == k) {
          small = s_; target = t_; best_us = u_;
          cached = true;
        }
      }
      fclose(f);
    }
  }
  TRY(enter(c));
  if (!cached) {
    struct Cand { int small, target; };
    std::vector<Cand> cands;
    int max_member = 0;
    for (size_t k = 0; k + 1 < c->mrange_h.size(); k += 2)
      max_member = std::max(max_member, c->mrange_h[k + 1] - c->mrange_h[k]);
    if (c->desc.dipole_on && c->d.dcut == 0.0 && !c->d.ew_on) {  // (a cutoff or a box: no layout)
      if (max_member <= 16384) cands.push_back({1, 0});
      for (int sp : {0, 2})  // particle order, spatial order
        for (int t : {512, 1024, 2048, 4096, 8192, 16384, 32768}) cands.push_back({sp, t});
    } else {
      cands.push_back({0, 1024});
    }
    best_us = 1e300;
    // split targets that give the same work list (in the same order) are timed once
    std::vector<std::pair<int, int>> seen;
    struct Timed { int small, target; double us; };
    std::vector<Timed> timed;
    for (const Cand& cd : cands) {
      TRY(build_dipole_plan(c, cd.small, cd.target));
      if (cd.small != 1) {
        const std::pair<int, int> k{cd.small, c->nwork};
        if (std::find(seen.begin(), seen.end(), k) != seen.end()) continue;
        seen.push_back(k);
      }
      double us = 0.0;
      TRY(time_eval(c, &us));
      char line[160];
      snprintf(line, sizeof(line), "%s target_wgs=%d work_items=%d slots=%d: %.2f us/eval\n",
               layout_name(cd.small), cd.target, c->nwork, c->max_slots, us);
      rep += line;
      timed.push_back({cd.small, cd.target, us});
      best_us = std::min(best_us, us);
    }
    // Candidates within 1% of the fastest are taken as equal, and the first of
    // them in the candidate order wins, so that timing noise between runs does
    // not flip the choice between near-equal layouts.
    for (const Timed& t : timed)
      if (t.us <= 1.01 * best_us) {
        small = t.small; target = t.target; best_us = t.us;
        break;
      }
    if (cache_path) {
      if (FILE* f = fopen(cache_path, "a")) {
        fprintf(f, "{\"key\": \"%s\", \"small\": %d, \"target_wgs\": %d, \"us_per_eval\": %.3f}\n",
                key.c_str(), small, target, best_us);
        fclose(f);
      }
    }
  } else {
    rep += "cached choice\n";
  }
  if (c->plan_small != small || c->plan_target != target) TRY(build_dipole_plan(c, small, target));
  if (c->launch_mode == ROD_LAUNCH_PER_ROD) TRY(build_rod_work(c));
  drop_graphs(c);
  TRY(leave(c));
  char line[256];
  snprintf(line, sizeof(line), "chosen: %s target_wgs=%d work_items=%d slots=%d (%.2f us/eval) key=%s\n",
           layout_name(small), target, c->nwork, c->max_slots, best_us, key.c_str());
  rep += line;
  if (report && report_len > 0) {
    strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return ROD_OK;
}

// ------------------------------------------------------------------ ramp
namespace {
struct TmpDev {  // device memory of one call
  void* p = nullptr;
  ~TmpDev() { if (p) (void)hipFree(p); }
};
}  // namespace

// Rods immersed in a lattice (Methods, "Immersed boundary coupling"). Per
// cycle: moments of the lattice, its velocity interpolated at every particle,
// then n_sub rod steps whose post kernel adds the penalty force and records it,
// each followed by the spreading of -F_p / n_sub at the new positions, then one
// lattice step with that force field. Everything runs on the rod stream; the
// lattice stream is drained first and made to wait for the result.
extern "C" int rod_lbm_cycles(rod_ctx* c, lbm_ctx* l, int32_t n_sub, int64_t n_cycles) {
  if (!c || !l) return fail(ROD_E_INVALID, "NULL argument");
  if (n_sub < 1 || n_cycles < 0) return fail(ROD_E_INVALID, "need n_sub >= 1 and n_cycles >= 0");
  if (std::fabs(c->desc.dt * n_sub - 1.0) > 1e-12)
    return fail(ROD_E_INVALID, "the rod time step times n_sub must be the lattice step 1 (dt = %g)", c->desc.dt);
  if (c->tape.active) return fail(ROD_E_STATE, "coupled cycles while a tape is recorded");
  if (n_cycles == 0) return ROD_OK;
  const long N = c->d.n, cells = l->L.cells;
  if (!l->work) HIPC(hipMalloc(&l->work, sizeof(double) * 7 * (size_t)cells));
  if (!c->ibm_buf) HIPC(hipMalloc(&c->ibm_buf, sizeof(double) * 6 * (size_t)N));
  double* rho = l->work;
  double* u = rho + cells;
  double* g = u + 3 * cells;
  Dev d = c->d;
  d.ibm_u = c->ibm_buf;
  d.ibm_f = c->ibm_buf + 3 * N;
  d.ibm_idt = 1.0;
  HIPC(hipStreamSynchronize(l->s));
  TRY(enter(c));
  for (int64_t k = 0; k < n_cycles; ++k) {
    HIPC(lbmx::launch_lbm_moments(l, rho, u, c->s));
    HIPC(lbmx::launch_ibm_interp(l, u, d.x, N, c->ibm_buf, c->s));
    HIPC(lbmx::launch_fill0(g, 3 * cells, c->s));
    for (int32_t sub = 0; sub < n_sub; ++sub) {
      TIMED(c, ROD_KERNEL_PRE, launch_pre, d, PRE_STEP, c->s);
      TRY(force_terms(c, d, 0, 1));
      TIMED(c, ROD_KERNEL_POST, launch_post, d, POST_KICK, ROD_TERM_ALL, nullptr, nullptr, nullptr,
            c->s);
      HIPC(lbmx::launch_ibm_spread(l, d.x, d.ibm_f, N, 1.0 / n_sub, g, c->s));
    }
    HIPC(lbmx::launch_lbm_step(l, g, c->s));
  }
  c->h_step += n_cycles * n_sub;
  HIPC(hipEventRecord(c->ev_out, c->s));
  HIPC(hipStreamWaitEvent(l->s, c->ev_out, 0));
  TRY(leave(c));
  return ROD_OK;
}

extern "C" int rod_ramp(rod_ctx* c, const double* fields, int32_t n_inc, int32_t max_steps,
                        int32_t check_every, double ke_tol, const int32_t* watch, int32_t n_watch,
                        double* x_watch, int32_t* steps, double* ke) {
  if (!c || !fields) return fail(ROD_E_INVALID, "NULL argument");
  if (n_inc < 1 || check_every < 1 || max_steps < 1 || n_watch < 0 || std::isnan(ke_tol))
    return fail(ROD_E_INVALID, "need n_inc, check_every, max_steps >= 1, n_watch >= 0, ke_tol a number");
  if (c->desc.field_len != 1) return fail(ROD_E_INVALID, "the ramp needs field_len = 1");
  if (n_watch > 0 && (!watch || !x_watch)) return fail(ROD_E_INVALID, "watch and x_watch are required");
  for (int32_t a = 0; a < n_watch; ++a)
    if (watch[a] < 0 || watch[a] >= c->d.n) return fail(ROD_E_INVALID, "watch index %d out of range", watch[a]);
  if (c->tape.active) return fail(ROD_E_STATE, "ramp while a tape is recorded");
  const int M = c->d.M;
  const size_t fbytes = sizeof(double) * 12 * (size_t)M;
  TmpDev dk, dw, dx;
  HIPC(hipMalloc(&dk.p, sizeof(double) * M));
  if (n_watch > 0) {
    HIPC(hipMalloc(&dw.p, sizeof(int32_t) * n_watch));
    HIPC(hipMalloc(&dx.p, 3 * sizeof(double) * n_watch));
    HIPC(hipMemcpy(dw.p, watch, sizeof(int32_t) * n_watch, hipMemcpyHostToDevice));
  }
  std::vector<double> e(M);
  for (int32_t k = 0; k < n_inc; ++k) {
    TRY(enter(c));
    HIPC(hipMemcpyAsync(const_cast<double*>(c->d.field), fields + (size_t)k * 12 * M, fbytes,
                        hipMemcpyHostToDevice, c->s));
    TRY(leave(c));
    int32_t taken = 0;
    while (taken < max_steps) {
      const int32_t chunk = std::min(check_every, max_steps - taken);
      TRY(rod_step(c, chunk));
      taken += chunk;
      TRY(enter(c));
      HIPC(launch_kinetic(c->d, (double*)dk.p, c->s));
      HIPC(hipMemcpyAsync(e.data(), dk.p, sizeof(double) * M, hipMemcpyDeviceToHost, c->s));
      TRY(leave(c));
      TRY(rod_sync(c));  // waits for the copy and reports non-finite state or overflow
      bool rest = true;
      for (int m = 0; m < M; ++m) rest = rest && e[m] <= ke_tol;
      if (rest) break;
    }
    if (steps) steps[k] = taken;
    if (ke) std::copy(e.begin(), e.end(), ke + (size_t)k * M);
    if (n_watch > 0) {
      TRY(enter(c));
      HIPC(launch_gather_x(c->d, (const int*)dw.p, n_watch, (double*)dx.p, c->s));
      HIPC(hipMemcpyAsync(x_watch + (size_t)k * 3 * n_watch, dx.p, 3 * sizeof(double) * n_watch,
                          hipMemcpyDeviceToHost, c->s));
      TRY(leave(c));
      HIPC(hipStreamSynchronize(c->s));
    }
  }
  return ROD_OK;
}

int rod_free(rod_ctx* c) {
  if (!c) return ROD_OK;
  if (c->s) (void)hipStreamSynchronize(c->s);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (void* p : c->plan_allocs) (void)hipFree(p);
  for (void* p : c->rod_allocs) (void)hipFree(p);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->tgexec) (void)hipGraphExecDestroy(c->tgexec);
  tape_release(c->tape);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->ibm_buf) (void)hipFree(c->ibm_buf);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->s) (void)hipStreamDestroy(c->s);
  delete c;
  return ROD_OK;
}

}  // extern "C"

// Used by the adjoint module to report errors in the same channel.
int rodmx_fail(int code, const char* msg) { return fail(code, "%s", msg); }
