// Internal declarations shared by the kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstdint>

namespace rodmx {

// One entry of the hashed cell list: the particle's position at insertion and
// a tag holding its index (low 32 bits) and rod (high 32 bits).
struct alignas(32) CellSlot { double x, y, z; long long tag; };

// A particle of the cutoff sort at its sorted position: position, index and
// the high bits of its cell's coordinates.
struct alignas(32) DlRec { double x, y, z; int i; unsigned tag; };

// Device-side view of one context: every pointer is a device pointer, fixed for
// the lifetime of the context, so that captured graphs can be replayed.
struct Dev {
  long n;           // particles
  long i_lo, i_hi;  // particle range served by the per-particle kernels (normally 0, n)
  int R, M;         // rods, members
  // caller-owned state (SoA planes)
  double *x, *v, *q, *w, *F, *T;
  const double* src;       // if set, the pre kernel reads the state from these planes
                           // (x, v, q, w, F, T as in a recorded state) instead of in place
  double* nx;              // if set, the kick kernel writes the next level's x, v, q, w to
                           // these planes (same layout) instead of in place
  const double *mb, *field, *extF, *extT;
  // topology and constants
  const uint8_t* bflags;   // bit0: bond (k, k+1); bit1: bond (k-1, k)
  const int* rod;          // rod of each particle
  const int* mem;          // member of each particle
  const int8_t* bc;        // boundary condition of each particle
  const double *minv, *Iinv, *mass, *inertia;
  const double* bref;      // [4N]: reference bond vector planes x, y, z and its length r0
  const double* rodK;      // [R][4]: EA, 12EI, GJ, EI
  const int* mrange;       // [2M]: member particle range [begin, end)
  // per-step work buffers
  double* mu;              // [3N] global dipole moments
  float* muf;              // [3N] FP32 copy for the mixed dipole kernel
  double *bF, *bTs, *bTbt; // [3N] per-bond outputs (index = first particle)
  double* bE;              // [4N] per-bond energies (energy evaluation only)
  double* dpart;           // [S][6][N] dipole partial sums (F then B), one slot per j range
                           // (FP64 path; the reverse pass keeps its cotangent sums here)
  float* dslotf;           // [S][6][N] the same partial sums on the mixed path (FP32), else null
  const double* bdamp;     // [R][4] bond damping factors g_r, g_s, g_t, g_b, or null (none)
  double* hist;            // [2][5][N] bond damping measures per level parity (bond k at k)
  const int* mslots;       // [M]: j ranges (partial slots) of each member
  int max_slots;           // largest entry of mslots; slots a member does not use stay zero
  double* cF;              // [3N] contact force
  double* cE;              // [N] contact energy per particle (energy evaluation only)
  // Hashed cell lists, one for even and one for odd time levels, so that a
  // kernel can empty the list of one level while it fills that of the next.
  int* cell_cnt;           // [2][cells] particles hashed to each cell
  CellSlot* cell_slot;     // [2][cells][CELL_CAP] position and tag of each listed particle
  int* key;                // [N] cell of each particle at its last insertion
  int* ovf_list;           // [2][OVF_CAP] particles whose cell was full
  int* ovf_cnt;            // [2] entries of the overflow lists (reset by the particle kernel)
  unsigned cell_mask;      // cells - 1 (power of two)
  // Contact candidate lists of large systems (use_lists): see contact_listed.
  int use_lists;
  // Stepping of a system whose contact search walks candidate lists: the
  // particle kernels leave the cell list empty and k_cell_insert fills it
  // only when the lists are rebuilt (set in the stepping chain's copy only).
  int lazy_cells;
  int* nbr;                // [NBR_CAP][N] candidates of each particle at the last build
  int* nbr_cnt;            // [N] candidates listed, or -1 when more than NBR_CAP
  double* xb;              // [3N] positions at the last build
  unsigned* rebuild;       // [2] per level parity: some particle moved too far since the build
  double skin;             // list cutoff is r_c + skin
  unsigned* flags;         // [FLAG_COUNT]: [0] non-finite state, [1] a dipole list was full,
                           // [2] overflow list full,
                           // [3] a particle had more Hertz-Mindlin contacts than HM_CAP,
                           // [4] a contact sum's term left the range of its exact sum
  long long* step;         // [3]: [0] time level of the state (written by the particle
                           // kernel); [1], [2] level of the force evaluation in flight,
                           // in the entry named by lc. No kernel writes what it reads.
  int lc;                  // 1 or 2: entry of step[] holding the level of the forces
  // parameters
  double dt, damping, C, kc, rc, inv_cell;
  // Exact contact sums (contact_body.h, Fix128): per quantity (force, torque,
  // energy) the power of two that maps the contact law's bound on one pair's
  // term to 2^80, and its inverse.
  double fix_scale[3], fix_inv[3];
  int depth, field_len, dipole_on, contact_on;
  int dip_small;           // dipole work items use the small-member layout (4 i per item)
  // Bounding boxes of consecutive 64-particle chunks at the level being
  // evaluated (x, y, z low then high), written where positions are set; the
  // mixed dipole kernel uses them to pick far sub-tiles (far_ok; off in the
  // per-rod loop, whose waves do not start on chunk boundaries).
  double* cbox;            // [(N + 63) / 64][6]
  int far_ok;
  // Split layout in spatial order (rod_dipole_layout with small = 2): the
  // work items' target and source ranges are positions in a space-filling-curve
  // order of each member's particles, dperm[position] = particle, so that 64
  // consecutive positions are close in space and most sub-tiles pass the far
  // test; sbox holds the boxes of consecutive 64-position chunks, written before
  // each launch of the dipole work items. Both null: positions are particles.
  const int* dperm;        // [N]
  double* sbox;            // [(N + 63) / 64][6]
  double axis[3];
  long long period;
  // ---- per-level history (bond damping, Hertz-Mindlin) and Hertz-Mindlin state
  // Levels from hist_from on find the previous level's bond damping measures
  // and Hertz-Mindlin contacts (the first evaluation of a run has none). Only
  // the evaluations of stepping (and of rod_init) record them (hist_write).
  long long hist_from;
  int hist_write;
  // Hertz-Mindlin contact (hm): E*, G*, R*, friction and dashpot coefficients,
  // the contact torque, and each particle's contacts per level parity: count,
  // partner and tangential displacement (seen from the particle).
  int hm;
  double hm_Es, hm_Gs, hm_Rs, hm_mu, hm_gn, hm_gt;
  double* cT;              // [3N] contact torque (hm)
  int* hc_cnt;             // [2][N]
  int* hc_j;               // [2][HM_CAP][N]
  double* hc_s;            // [2][3][HM_CAP][N]
  // Dipole cutoff (dcut > 0; 0: all pairs of a member): each particle's
  // neighbours within dcut + skin, found at a rebuild from the particles
  // sorted by cell (dipole_list.h). Cells of side 1 / dl_inv >= dcut + skin
  // from the origin dl_org; a bucket is the member shifted by dl_mshift above
  // the coordinates' low dl_bits[a] bits, deposited at the bits of dl_axis[a].
  double dcut;
  double dl_inv;
  double dl_org[3];
  int dl_bits[3];
  unsigned dl_axis[3];
  int dl_mshift;
  int dl_nb;               // buckets (a power of two, a multiple of DL_SCAN)
  int* dl_cnt;             // [nb] particles per bucket (zero between rebuilds)
  int* dl_aux;             // [nb / DL_SCAN] count of each scan block
  int* dl_start;           // [nb + 1] first sorted position of each bucket
  int* dl_bkt;             // [N] bucket of each particle
  int* dl_slot;            // [N] its counting slot in the bucket
  int* dl_tmp;             // [N] particles by bucket in counting order
  int* dl_sorted;          // [N] particle at each sorted position
  int* dl_pos;             // [N] sorted position of each particle
  DlRec* dl_rec;            // [N] position, index and cell tag at each sorted position
  int* dnbr;               // [DNBR_CAP][N] by sorted position
  int* dnbr_cnt;           // [N] by sorted position
  double* xm;              // [N][8]: x, y, z, m_x, m_y, m_z, 0, 0 of the level (cutoff), or null
  // Periodic box with the Ewald sum of the dipoles (ew_on; k_ewald.hip): box
  // lengths, splitting parameter, real-space cutoff, the self-field
  // coefficient C 4 a^3 / (3 sqrt(pi)); member-major cells of side >= ew_rc / EW_REACH,
  // ew_nc per axis; particles sorted by cell with an interleaved copy of their
  // wrapped positions and moments; the reciprocal vectors of the half space
  // with their coefficients, particle chunks (sorted ranges of one member) and
  // the partial and summed structure factors.
  int ew_on;
  double box[3];
  double ew_alpha, ew_rc, ew_self;
  int ew_nc[3];
  int ew_ncell;            // cells per member
  int* ew_cnt;             // [M ncell] particles per cell
  int* ew_start;           // [M ncell + 1] first sorted position of each cell
  int* ew_cell;            // [N] cell of each particle
  int* ew_slot;            // [N] its place in the cell's count
  int* ew_tmp;             // [N] particles grouped by cell in counting-slot order
  int* ew_sorted;          // [N] particles by cell, each cell's in ascending index
  double* ew_xm;           // [N][8] wrapped x, y, z, 0, m_x, m_y, m_z, 0 in sorted order
  float* ew_xf;            // [N][8] mixed path: the position's offset from the centre of its
                           // cell, 0, m_x, m_y, m_z, 0 (FP32) in sorted order; else NULL
  const double* ew_k;      // [K][4] k_x, k_y, k_z, 2 (4 pi C / V) exp(-k^2 / 4 a^2) / k^2
  int ew_K;
  const int* ew_seg;       // [SEG][2] first vector and count (<= EW_SEG) of runs along k_z
  int ew_SEG;
  const int* ew_row;       // [ROWS][2] first vector and count of each row (fixed n_x, n_y)
  int ew_ROWS;
  double ew_dkz;           // 2 pi / L_z, the k_z step along a run
  const int* ew_chunks;    // [TC][3] sorted range [begin, end) of at most 256 and the member
  const int* ew_chunk_off; // [M + 1] first chunk of each member
  int ew_TC;
  double* ew_Sp;           // [TC][K][2] structure factor of each chunk
  double* ew_S;            // [M][K][2] structure factor of each member times the k weight
  // Immersed-boundary penalty (set only on the copy a coupled cycle launches
  // with): fluid velocity at the particles [3][N], the penalty force of the
  // evaluation written to ibm_f [3][N], stiffness m_p * ibm_idt.
  const double* ibm_u;
  double* ibm_f;
  double ibm_idt;
};

constexpr int CELL_CAP = 8;
constexpr int OVF_CAP = 4096;
constexpr int NBR_CAP = 32;                     // candidates per particle list
constexpr long CONTACT_LANES_MAX_N = 65536;     // below: lane-parallel cell search, above: lists
constexpr double NBR_SKIN = 0.25;               // skin as a fraction of r_c
constexpr double NBR_MOVE = 0.45;               // rebuild past this fraction of the skin
                                                // (below 1/2, a margin for rounding)
constexpr int HM_CAP = 32;                      // Hertz-Mindlin contacts kept per particle
constexpr int DNBR_CAP = 256;                   // dipole list entries per particle (cutoff)
constexpr int DL_SCAN = 2048;                   // buckets per block of the cutoff sort's sums
enum { FLAG_NONFINITE = 0, FLAG_DIP_OVF = 1, FLAG_LIST_OVF = 2, FLAG_HM_OVF = 3,
       FLAG_CONTACT_RANGE = 4, FLAG_COUNT = 5 };
// Exponent that maps a pair-term bound b to 2^80 in the exact contact sums.
constexpr int FIX_BOUND_EXP = 80;

// Cell of a coordinate (cells of side 1/inv), clamped so runaway coordinates
// stay hashable.
__device__ __forceinline__ int cell_coord(double x, double inv) {
  double c = floor(x * inv);
  c = fmin(fmax(c, -1.0e9), 1.0e9);
  return (int)c;
}

// Bucket of cell (cx, cy, cz) of member `mem`: a row (cy, cz, mem) starts at a
// hashed base and runs linearly in cx, so that the three cells of a row of a
// 3x3x3 neighbourhood share cache lines. Distinct cells may share a bucket (the
// search checks every candidate's distance), which costs only extra checks.
__device__ __forceinline__ unsigned cell_hash(int cx, int cy, int cz, int mem, unsigned mask) {
  const unsigned row = (unsigned)cy * 73856093u ^ (unsigned)cz * 19349663u ^
                       (unsigned)mem * 83492791u;
  return ((unsigned)cx + row) & mask;
}

// Cell list of time level `lvl`.
struct CellTab { int* cnt; CellSlot* slot; int* ovf; int* ovf_cnt; };
__device__ __forceinline__ CellTab cell_tab(const Dev& d, long long lvl) {
  const long p = (long)(lvl & 1);
  const long cells = (long)d.cell_mask + 1;
  return {d.cell_cnt + p * cells, d.cell_slot + p * cells * CELL_CAP, d.ovf_list + p * OVF_CAP,
          d.ovf_cnt + p};
}

enum PreMode { PRE_PREPARE = 0, PRE_STEP = 1, PRE_EVAL = 2 };
enum PostMode { POST_PREPARE = 0, POST_KICK = 1, POST_EVAL = 2 };

// One dipole work item: an i block [i0, i1) of at most 64 particles of one
// member against j in [j0, j1) of the same member,
// written to partial slot `slot`.
struct DipWork { int i0, i1, j0, j1, slot, pad0, pad1, pad2; };


// Targets per work item of the small-member layout (one wave of a 256-thread
// workgroup each).
constexpr int DIP_SMALL_I = 4;

// Threads per block of the per-particle kernels: small blocks spread small
// systems over more compute units.
inline int particle_block(long n) { return n < 65536 ? 64 : 256; }

// Kernel launchers (each enqueues on `s`; return the launch status).
// Launch that, given `ev`, has the runtime stamp ev[0] and ev[1] with the
// kernel's own start and end (timing mode); a plain launch otherwise.
template <typename... KArgs, typename... Args>
inline void launch_k(const hipEvent_t* ev, void (*kernel)(KArgs...), dim3 g, dim3 b,
                     hipStream_t s, Args... args) {
  if (ev)
    hipExtLaunchKernelGGL(kernel, g, b, 0u, s, ev[0], ev[1], 0u, static_cast<KArgs>(args)...);
  else
    hipLaunchKernelGGL(kernel, g, b, 0, s, static_cast<KArgs>(args)...);
}

hipError_t launch_pre(const Dev& d, int mode, hipStream_t s, const hipEvent_t* ev = nullptr);
// Cell-list entries of the current level for a rebuild of the contact lists
// (nothing unless the lists are stale or `build`); the stepping chain of a
// system with lazy_cells.
hipError_t launch_cell_insert(const Dev& d, int build, hipStream_t s,
                              const hipEvent_t* ev = nullptr);
// Kinetic energy of each member into out[M]; positions of idx[0..n) into out[n][3].
hipError_t launch_kinetic(const Dev& d, double* out, hipStream_t s);
hipError_t launch_gather_x(const Dev& d, const int* idx, int n, double* out, hipStream_t s);
hipError_t launch_bond(const Dev& d, int precision, int want_energy, hipStream_t s,
                       const hipEvent_t* ev = nullptr);
hipError_t launch_dipole(const Dev& d, int precision, const DipWork* work, int nwork,
                         hipStream_t s, const hipEvent_t* ev = nullptr);
// Dipole interaction with a cutoff (d.dcut > 0) from the Verlet lists; build:
// rebuild them regardless of motion.
hipError_t launch_dipole_cut(const Dev& d, int build, hipStream_t s,
                             const hipEvent_t* ev = nullptr);
// The cutoff sort alone (when the lists are stale or `build`), over the whole
// system: launched once before the per-rod loop's list walks.
hipError_t launch_dipole_sort(const Dev& d, int build, hipStream_t s);
// Boxes of the 64-position chunks of the spatial order (d.dperm) into d.sbox;
// nothing without a spatial order.
hipError_t launch_spatial_boxes(const Dev& d, hipStream_t s);
// Ewald sum of the dipoles of a periodic box (d.ew_on): writes the dipole
// force and field to slot 0 of the FP64 partial sums.
// ev_real (timing mode, else NULL): the runtime stamps the real-space walk's own
// start and end on it; ev brackets the whole sum.
hipError_t launch_ewald(const Dev& d, const hipEvent_t* ev_real, hipStream_t s,
                        const hipEvent_t* ev = nullptr);
constexpr int EW_CHUNK = 256;   // particles per structure-factor chunk
constexpr int EW_SEG = 8;       // k vectors per run of one row (one sincos per run)
constexpr int EW_MAX_NC = 256;  // cells per box axis at most
constexpr int EW_REACH = 3;     // real-space cells of side >= rc / EW_REACH
// build: rebuild contact candidate lists (large systems) regardless of motion.
hipError_t launch_contact(const Dev& d, int want_energy, int build, hipStream_t s,
                          const hipEvent_t* ev = nullptr);
// Dipole, bond and contact forces of a step in one launch.
// Whether the contact search runs inside the fused force launch (lane-parallel
// cell search of smaller systems, either law) or in a launch of its own
// (candidate lists of large systems).
inline bool contact_in_forces(const Dev& d) { return d.n < CONTACT_LANES_MAX_N; }
hipError_t launch_forces(const Dev& d, int precision, const DipWork* work, int nwork,
                         hipStream_t s, const hipEvent_t* ev = nullptr);
// The whole force pass of a level: launch_forces, and for systems whose contact
// search is not part of it, launch_contact. build: rebuild the candidate lists.
hipError_t launch_force_pass(const Dev& d, int precision, const DipWork* work, int nwork,
                             int build, hipStream_t s);
hipError_t launch_post(const Dev& d, int mode, int mask, double* Fout, double* Tout,
                       double* Bout, hipStream_t s, const hipEvent_t* ev = nullptr);
// Second half-kick of the step whose forces are in flight (level step[lc]) fused
// with the first half-kick, drift and rotation of the next step; writes the next
// level into step[3 - lc].
// Bo: where to write the dipole field of the gathered level (or nullptr).
hipError_t launch_kick(const Dev& d, double* Bo, hipStream_t s, const hipEvent_t* ev = nullptr);
hipError_t launch_energy(const Dev& d, double* Epart, double* out, hipStream_t s);
hipError_t launch_contact_pairs(const Dev& d, int* pairs, int cap, int* count, hipStream_t s);
hipError_t launch_clear_cells(const Dev& d, hipStream_t s);
// Fill p[0..n) with v.
hipError_t launch_fill_i32(int* p, int n, int v, hipStream_t s);

}  // namespace rodmx
