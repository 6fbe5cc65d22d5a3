/* rod.h - C ABI of the MI355X (gfx950) library for the per-timestep
 * force-and-integrate loop of the bonded-particle model of magneto-elastic rods.
 *
 * One time step of the loop (paper, SI "Equations of motion"):
 *   v(t+dt/2) = v + dt/2 f/m,  x(t+dt) = x + dt v(t+dt/2),
 *   w(t+dt/2) = w + dt/2 tau/I, q(t+dt) by Richardson extrapolation of
 *   dq/dt = 1/2 (0, w) q with renormalisation after every substep;
 *   forces at t+dt; v(t+dt) = v(t+dt/2) + dt/2 f/m, w likewise.
 * The forces are the sum of
 *   - bonds: central-frame decomposition into stretch, shear, twist and bend
 *     (main text eq:bpm-fr, eq:bpm-fst, eq:bpm-tst, eq:bpm-tb, eq:bpm-tt,
 *     eq:bpm-vector; SI "Symmetric rotational decomposition"), spring
 *     constants K_r = EA/L, K_s = 12EI/L^3, K_t = GJ/L, K_b = EI/L;
 *   - dipoles that rotate with their particle (m = R(q) m_body, section on
 *     magnetised beams): Zeeman force grad(m.B) and torque m x B, and the
 *     all-pairs dipole-dipole force and torque within an ensemble member
 *     (Methods, "Magnetic interactions"), open boundaries, no cutoff;
 *   - Hookean normal contact k (r_c - r) between pairs closer than r_c that
 *     are not bonded within `exclude_depth` (Methods, "Contact"), found with a
 *     hashed cell list (above 65,536 particles through per-particle candidate
 *     lists built from it; the selected pairs are the same);
 *   - global viscous damping -c m v, -c I w with the half-step velocities;
 *   - optional constant external forces and torques.
 *
 * Conventions
 *   - All device arrays are structure-of-arrays (SoA) planes of length N:
 *     a "[3N]" vector array holds x-components [0,N), y [N,2N), z [2N,3N);
 *     quaternions "[4N]" hold the planes w, x, y, z (Hamilton product,
 *     active rotation v' = q v q*).
 *   - Particles of a rod are contiguous; consecutive particles of a rod are
 *     bonded; rods of a member are contiguous; members never interact.
 *   - Every function returns ROD_OK (0) or a negative error code and never
 *     throws; rod_last_error() returns a message for the calling thread.
 *   - Work is enqueued on the stream given to rod_init; functions that return
 *     host data synchronise that stream first.
 *   - The library keeps non-owning pointers to the caller's device buffers:
 *     they must stay valid until rod_free. It allocates its own workspace.
 */
#ifndef ROD_H
#define ROD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ROD_OK = 0,
  ROD_E_INVALID = -1,   /* bad argument or descriptor */
  ROD_E_HIP = -2,       /* a HIP runtime call failed */
  ROD_E_NONFINITE = -3, /* a force, position or quaternion became NaN/inf */
  ROD_E_NOTAPE = -4,    /* rod_grad without a recorded forward run */
  ROD_E_OVERFLOW = -5,  /* contact search capacity exceeded */
  ROD_E_STATE = -6      /* call not valid in the current context state */
};

enum { ROD_FP64 = 0, ROD_MIXED = 1 };

/* Force terms, as a bitmask for rod_eval_forces. */
enum {
  ROD_TERM_BOND = 1, ROD_TERM_DIPOLE = 2, ROD_TERM_ZEEMAN = 4,
  ROD_TERM_CONTACT = 8, ROD_TERM_DAMP = 16, ROD_TERM_EXT = 32, ROD_TERM_ALL = 63
};

/* Boundary condition of a particle. */
enum { ROD_BC_FREE = 0, ROD_BC_CLAMPED = 1, ROD_BC_DRIVEN = 2 };

/* Contact law (rod_desc.contact_model). */
enum { ROD_CONTACT_HOOKEAN = 0, ROD_CONTACT_HERTZ_MINDLIN = 1 };

/* Tangential-history capacity of a Hertz-Mindlin particle: contacts it can
   hold at once (more: ROD_E_OVERFLOW at rod_sync). */
#define ROD_HM_MAX_CONTACTS 32

/* Host-side description; copied by rod_init (the caller may free it after). */
typedef struct rod_desc {
  int32_t n_particles;        /* N >= 1 */
  int32_t n_rods;             /* R >= 1 */
  int32_t n_members;          /* M >= 1 */
  const int32_t* rod_offset;  /* host [R+1], strictly increasing, [0] = 0, [R] = N */
  const int32_t* rod_member;  /* host [R], non-decreasing, values 0..M-1, every member used */
  const double* rod_params;   /* host [R][4]: diameter d > 0, density > 0, Young E > 0, Poisson nu > -1 */
  const double* x_ref;        /* host [N][3] (AoS): reference lattice; bond k has r_i = x_ref[k+1]-x_ref[k],
                                 reference orientations are the identity */
  const int8_t* bc;           /* host [N]: ROD_BC_* */
  double drive_axis[3];       /* unit axis of driven particles */
  int64_t drive_period;       /* steps per turn of driven particles: q(n) = R(axis, 2 pi n / P); 0 = none */
  int32_t field_len;          /* L >= 1 rows of the field table (row n mod L is used at time level n) */
  double dt;                  /* time step > 0 */
  double damping;             /* global viscous damping c >= 0 */
  double mu0_4pi;             /* dipole prefactor mu0 / 4 pi */
  double k_contact;           /* contact stiffness */
  double r_contact;           /* contact distance r_c > 0 (cells of side r_c, or 1.25 r_c with lists) */
  int32_t dipole_on;          /* 0 / 1 */
  int32_t contact_on;         /* 0 / 1 */
  int32_t exclude_depth;      /* same-rod pairs with |i - j| <= depth never contact (>= 0) */
  int32_t precision;          /* ROD_FP64 or ROD_MIXED (FP32 pair/bond arithmetic, FP64 state and sums) */
  int64_t step0;              /* time level of the initial state */
  int32_t graph_steps;        /* steps per captured HIP graph; 0 = launch eagerly */
  int32_t tape_every;         /* checkpoint interval for rod_grad (0 = no gradient support) */
  int32_t tape_capacity;      /* maximum number of steps rod_grad can reverse (0 = no tape) */
  const double* bond_damping; /* host [R][4] or NULL: bond damping factors g_r, g_s, g_t, g_b >= 0
                                 of each rod's bonds (Methods, "Damping"). Radial: g_r times the
                                 relative velocity along the bond axis joins the radial force.
                                 Shear: K_s gamma becomes K_s gamma + g_s gamma-dot in f_s and
                                 tau_s. Twist and bend: g_t psi-dot and g_b theta-dot join the
                                 torques. The rates are differences of these measures between the
                                 current and the previous force evaluation of the run, over dt
                                 (the twist change taken modulo 2 pi; the bend vector per component
                                 in the bond frame). rod_init records the initial state's measures,
                                 and its evaluation has no rates (with forces_valid the caller's
                                 forces are kept and only the measures are taken); an evaluation
                                 at that same level finds zero rates. Velocities are those of the
                                 force evaluation (half-step while stepping). Factors must be
                                 finite and >= 0 (else ROD_E_INVALID). Not differentiated: nonzero
                                 factors with tape_capacity > 0 are refused (ROD_E_INVALID). */
  int32_t contact_model;      /* ROD_CONTACT_HOOKEAN: k_contact (r_c - r) along the line of centres.
                                 ROD_CONTACT_HERTZ_MINDLIN (Methods, "Contact"), as for two equal
                                 elastic spheres of diameter r_c: R* = r_c / 4, overlap
                                 delta = r_c - r, a = sqrt(R* delta), E* = E / (2 (1 - nu^2)),
                                 G* = E / (4 (2 - nu)(1 + nu)); normal force
                                 max(0, 4/3 E* a delta - g_n v_n); tangential force
                                 -8 G* a s - g_t v_t limited to mu times the normal force, with v the
                                 contact-point velocity of the pair (centre velocities plus spins)
                                 and s the contact's tangential displacement: zero for a new contact,
                                 otherwise the previous evaluation's s turned into the current
                                 tangent plane plus v_t dt (reset to hold the limited force when the
                                 limit acts). The torque (-r/2 n) x F_t acts on both particles.
                                 Each particle keeps its contacts of the last two levels (at most
                                 ROD_HM_MAX_CONTACTS each); as with bond damping, rod_init records
                                 the initial contacts (all new) and a restart starts them afresh. Not
                                 differentiated: with tape_capacity > 0 it is refused. */
  double contact_hm[5];       /* Hertz-Mindlin: contact modulus E > 0, Poisson ratio -1 < nu <= 0.5,
                                 friction coefficient mu >= 0, normal and tangential viscous damping
                                 g_n, g_t >= 0 */
  double dipole_cutoff;       /* 0: the dipole-dipole sum runs over every pair of a member. > 0: only
                                 pairs with r^2 = (dx dx + dy dy) + dz dz < cutoff^2 (exact FP64
                                 selection) interact, through the same pair law (the truncated pair
                                 interaction of the paper's simulations, for very large systems).
                                 Needs contact_on: each particle keeps a list of the member's
                                 particles within cutoff + r_contact / 4, rebuilt with the contact
                                 lists from the particles sorted by cell (cells of that side); at
                                 most 256 per particle (more: ROD_E_OVERFLOW at rod_sync). FP64 on
                                 both paths; the sort fixes the list order and the sums, so a run
                                 repeated gives the same bits. With a tape, rod_grad
                                 differentiates the truncated sum (pairs selected by the
                                 recorded distances); its reverse pass visits every pair of a
                                 member (one slot) and tests each against the cutoff. */
  double box[3];              /* Periodic box lengths L_x, L_y, L_z, all > 0; or all 0 (open
                                 boundaries). With a box and dipole_on, the dipole-dipole
                                 interaction is the Ewald sum of each member's periodic system
                                 (the long-range solvers offered beside the truncated pair style:
                                 Introduction; SI "Magnetic dipoles"), with conducting boundaries
                                 at infinity: real-space pairs by the minimum image closer than
                                 ewald_rcut, with the erfc-screened dipole terms; reciprocal
                                 vectors k = 2 pi (n_x/L_x, n_y/L_y, n_z/L_z), 0 < |n|^2 <=
                                 ewald_kmax^2, weighted by (4 pi C / V) exp(-k^2/4a^2) / k^2 with
                                 a = ewald_alpha; the self field C 4 a^3 / (3 sqrt(pi)) m_i.
                                 Positions need not be wrapped into the box. The real-space
                                 pair law, the reciprocal phases (from FP64 arguments reduced
                                 modulo 2 pi) and their per-thread sums are FP32 on the mixed
                                 path, and so are its separations and cutoff test when every
                                 axis holds at least seven cells, of side rcut / 3 to rcut
                                 (taken from the positions' offsets to their cells' centres);
                                 the
                                 sums across lanes, chunks and rows and the self field are FP64
                                 on both paths; sums in a fixed order (deterministic). Needs
                                 contact_on = 0 (contact is not periodic), dipole_cutoff = 0 and
                                 no tape (ROD_E_INVALID otherwise). The accuracy is the caller's
                                 choice of a, ewald_rcut and ewald_kmax: erfc(a rc) and
                                 exp(-(pi kmax / (a L))^2) bound the two truncations. */
  double ewald_alpha;         /* Ewald splitting parameter a > 0 (with a box) */
  double ewald_rcut;          /* real-space cutoff, 0 < rc <= min(L) / 2 (with a box) */
  int32_t ewald_kmax;         /* reciprocal cutoff, 1 <= kmax <= 64 (with a box) */
} rod_desc;

/* Caller-owned device buffers (SoA, float64). */
typedef struct rod_buffers {
  double* x;                  /* [3N] positions, updated in place */
  double* v;                  /* [3N] velocities */
  double* q;                  /* [4N] orientations (normalised by rod_init) */
  double* w;                  /* [3N] angular velocities (space frame) */
  double* force;              /* [3N] total force of the current time level (part of the state) */
  double* torque;             /* [3N] total torque of the current time level */
  const double* m_body;       /* [3N] body-frame dipole moments */
  const double* field;        /* [L][M][12] rows: B0 (3), G (3x3 row-major); B(x) = B0 + G x */
  const double* ext_force;    /* [3N] or NULL */
  const double* ext_torque;   /* [3N] or NULL */
} rod_buffers;

typedef struct rod_ctx rod_ctx; /* opaque; owned by the library, released by rod_free */

/* Bytes of device workspace rod_init would allocate for this description. */
int rod_query_workspace(const rod_desc* d, size_t* bytes);

/* Validate `d`, build the topology (bonds, spring constants, masses) and the
 * workspace, normalise q, impose the boundary conditions of level step0 and,
 * unless `forces_valid` is non-zero, evaluate force/torque of that level into
 * the caller's buffers. `hip_stream` is a hipStream_t (NULL = default stream).
 * On error *out is set to NULL. */
int rod_init(rod_ctx** out, const rod_desc* d, const rod_buffers* b, void* hip_stream,
             int32_t forces_valid);

/* Advance n_steps >= 0 time steps (asynchronous on the stream). When the
 * context records a tape, at most tape_capacity steps may follow rod_tape_begin. */
int rod_step(rod_ctx* c, int64_t n_steps);

/* Current time level (synchronises). */
int rod_get_step(rod_ctx* c, int64_t* step);

/* Wait for the stream and report device-side error flags (non-finite state,
 * contact capacity overflow) raised since the last check. */
int rod_sync(rod_ctx* c);

/* Evaluate the selected force terms (ROD_TERM_* mask) at the current state
 * into device buffers F[3N] and T[3N]; damping uses the current v and w; the
 * field row is that of the current level. Does not change the state.
 * B_dip (device [3N] or NULL) receives the dipole field at each particle. */
int rod_eval_forces(rod_ctx* c, int32_t terms, double* F, double* T, double* B_dip);

/* Energies per member, 9 doubles each: stretch, shear, twist, bend
 * (eq:total-energy), Zeeman -m.B, dipole-dipole, contact 1/2 k (r_c - r)^2,
 * translational and rotational kinetic energy. `out` is [M][9]; host memory
 * (synchronises) when out_on_device = 0, device memory otherwise. */
int rod_energy(rod_ctx* c, double* out, int32_t out_on_device);

/* Bond topology as built (host outputs, each may be NULL): ij [cap][2] particle
 * pairs, rref [cap][3] reference vectors, K [cap][4] = K_r, K_s, K_t, K_b.
 * *count receives the number of bonds; at most cap entries are written. */
int rod_topology(rod_ctx* c, int32_t* ij, double* rref, double* K, int32_t cap, int32_t* count);

/* Contact pairs (i < j, ascending) found by the cell list at the current state
 * (host output, synchronises); *count receives the total, at most cap written. */
int rod_contact_pairs(rod_ctx* c, int32_t* pairs, int32_t cap, int32_t* count);

/* Hertz-Mindlin contact history of the current time level (Methods, "Contact":
 * the tangential spring of a contact builds up over the contact's lifetime, so
 * a run continued from a saved state must carry it to equal the uncut run).
 * rod_get_contact_history writes, for every particle i, its contact count
 * count[i] (host [N], at most ROD_HM_MAX_CONTACTS), its partners
 * partner[i][k] (host [N][ROD_HM_MAX_CONTACTS]) and the tangential
 * displacement of each contact seen from i, disp[i][k][3] (host
 * [N][ROD_HM_MAX_CONTACTS][3]); entries past the count are zero. It
 * synchronises. rod_set_contact_history installs such a history as the current
 * level's, replacing what the context recorded there (a context created with
 * forces_valid from a saved state records that state's contacts as new ones):
 * the next step then continues each listed contact's displacement. Errors:
 * ROD_E_INVALID (NULL arguments, a count outside [0, ROD_HM_MAX_CONTACTS], a
 * partner outside [0, N) or equal to its particle, a non-finite
 * displacement), ROD_E_STATE (the context has no Hertz-Mindlin contact),
 * ROD_E_HIP. */
int rod_get_contact_history(rod_ctx* c, int32_t* count, int32_t* partner, double* disp);
int rod_set_contact_history(rod_ctx* c, const int32_t* count, const int32_t* partner,
                            const double* disp);

/* Largest `cap` of rod_contact_pairs_noalloc (its static staging holds this
 * many pairs). */
#define ROD_NOALLOC_MAX_PAIRS 1048576

/* For callers that cannot allocate device memory (tight serving or polling
 * loops, harnesses that forbid hipMalloc): rod_contact_pairs without a per-call
 * allocation. The same search and output: the contact pairs (i < j) of the
 * current state, sorted ascending into `pairs` (host [cap][2]); *count receives
 * the total, at most cap are written (synchronises). The pairs are staged in a
 * static device array of the library, 8 MiB + 256 B on each GPU it runs on,
 * held until the process ends; the call allocates no device or host memory.
 * Errors: ROD_E_INVALID for NULL arguments or cap outside
 * [0, ROD_NOALLOC_MAX_PAIRS]; ROD_E_HIP if the array's device address could not
 * be resolved when the context was created, or a launch or copy failed.
 * Every call on one GPU shares that GPU's array: calls from threads of one
 * process are serialised by a lock per device; calls that bypass it (e.g. from
 * another copy of the library in the same process) would race. */
int rod_contact_pairs_noalloc(rod_ctx* c, int32_t* pairs, int32_t cap, int32_t* count);

/* Gradient support (reverse mode through recorded steps).
 * rod_tape_begin marks the current state as the start of the recorded run
 * (and stores it as the first checkpoint); subsequent rod_step calls record
 * checkpoints every tape_every steps, up to tape_capacity steps. */
int rod_tape_begin(rod_ctx* c);

typedef struct rod_cotangent {  /* device [3N]/[4N] cotangents of the final state; NULL = zero */
  const double* x; const double* v; const double* q; const double* w;
} rod_cotangent;

typedef struct rod_gradients {  /* device outputs (overwritten); NULL = not wanted */
  double* m_body;               /* [3N] */
  double* field;                /* [L][M][12] */
  double* x0; double* v0; double* q0; double* w0;  /* [3N], [3N], [4N] (raw q0), [3N] */
} rod_gradients;

/* Reverse the recorded steps: given cotangents of the state at the end of the
 * recorded run, write the gradients with respect to the body dipoles, the
 * field table and the state at rod_tape_begin (q0 taken before the
 * normalisation rod_init applies when the tape starts at rod_init's state).
 * The forward state is not changed. Returns ROD_E_NOTAPE without a tape. */
int rod_grad(rod_ctx* c, const rod_cotangent* gy, rod_gradients* gx);

/* Kernel timing with HIP events on the library's own stream.
 * While enabled (enable != 0), rod_step launches every step eagerly (no graph)
 * and hands each kernel launch a pair of events that the runtime stamps with
 * that kernel's own start and end (hipExtLaunchKernel), so launch gaps are
 * not counted. rod_kernel_times synchronises, adds up the elapsed time of all
 * timed launches since the last read per kernel class and resets the sums:
 * ms[ROD_KERNEL_COUNT] (milliseconds) and launches[ROD_KERNEL_COUNT] (host
 * arrays, may be NULL). The library holds at most 4096 pending event pairs;
 * beyond that a timed launch first synchronises the stream and folds the
 * pending times into the sums. */
enum {
  ROD_KERNEL_PRE = 0,     /* half-kick, drift, quaternion update, dipole rotation, cell list */
  ROD_KERNEL_BOND = 1,    /* bond forces and torques */
  ROD_KERNEL_DIPOLE = 2,  /* all-pairs dipole-dipole */
  ROD_KERNEL_CONTACT = 3, /* contact (cell list, or candidate lists) */
  ROD_KERNEL_POST = 4,    /* force gather, Zeeman, damping, second half-kick */
  ROD_KERNEL_FORCES = 5,  /* dipole, bond and (below 65536 particles) contact in one launch */
  ROD_KERNEL_KICK = 6,    /* post of one step fused with pre of the next */
  ROD_KERNEL_CELLS = 7,   /* cell-list fill before the contact launch when stepping with
                             candidate lists (empty unless the lists are rebuilt) */
  ROD_KERNEL_EWALD_REAL = 8, /* the Ewald sum's real-space walk alone (with a box; its time is
                                also part of ROD_KERNEL_DIPOLE, which covers the whole sum) */
  ROD_KERNEL_COUNT = 9
};
int rod_timing(rod_ctx* c, int32_t enable);
int rod_kernel_times(rod_ctx* c, double* ms, int64_t* launches);

/* Autotuner for the work layout of the all-pairs dipole kernel (the dominant
 * kernel). Candidates: the small-member layout (one wave per target, four
 * targets per workgroup; members of at most 16384 particles), then the split
 * layout in particle order and in spatial order (64 targets per workgroup,
 * each member's sources split into enough ranges to give the launch 512 ...
 * 32768 work items; distinct work lists are timed once). Each candidate is
 * timed with HIP events on the library's stream over repeated force
 * evaluations at the current state (the state is not changed); the fastest is
 * applied, candidates within 1% of it counting as equal (the first of them in
 * the order above wins, so that timing noise does not flip the choice). With a
 * non-NULL cache_path (a JSON-lines file) the choice is looked up first
 * (unless force != 0) under a key of GPU architecture, precision and member
 * sizes, and a new choice is appended. A text report is copied into `report`
 * (report_len bytes, may be NULL). Invalidates captured graphs; not allowed
 * while a tape is recorded (ROD_E_STATE). */
int rod_autotune(rod_ctx* c, const char* cache_path, int32_t force, char* report,
                 int32_t report_len);

/* Launch mode of rod_step. ROD_LAUNCH_BATCHED (default): each kernel serves all
 * rods and members in one launch (graph-captured when graph_steps > 0); the
 * dipole and bond forces of a step share one launch, and so does contact below
 * 65536 particles (above, the candidate-list search is a launch of its own,
 * timed as ROD_KERNEL_CONTACT); between two consecutive steps of one call the
 * closing half-kick and the next step's opening half-kick, drift and rotation
 * share one launch.
 * ROD_LAUNCH_SEPARATE: as batched, with the three force terms launched as
 * separate kernels and no kick fusion (per-term timing).
 * ROD_LAUNCH_PER_ROD: the plain per-rod loop, every kernel launched once per
 * rod on that rod's particles, eagerly; kept as the baseline the batched form
 * is measured against. Batched and
 * separate give bitwise identical states; so does the per-rod loop in FP64,
 * while on the mixed path it always takes the exact position differences in
 * the dipole sum and agrees with the batched launch to rounding. */
enum { ROD_LAUNCH_BATCHED = 0, ROD_LAUNCH_PER_ROD = 1, ROD_LAUNCH_SEPARATE = 2 };
int rod_launch_mode(rod_ctx* c, int32_t mode);

/* Set the dipole work layout directly: small = 1 small-member layout (ignored
 * for members above 16384 particles), 0 split layout aiming at target_wgs
 * work items, 2 the split layout over each member's particles taken in a
 * space-filling-curve (Morton) order of their positions at this call (on the
 * mixed path more of its sub-tiles of sources are far from their targets and
 * take the cheaper position differences; sums are as deterministic as in
 * particle order, but rounded in another order), -1 the default rule.
 * Invalidates captured graphs. */
int rod_dipole_layout(rod_ctx* c, int32_t small, int32_t target_wgs);

/* Quasi-static field ramp: the loading protocol of the magnetised beams in
 * non-uniform fields and of the helical rods with dipole-dipole interactions
 * (results sections "Magnetized beams in non-uniform fields" and "Helical rods
 * with dipole-dipole interactions"): a field parameter is raised (and lowered)
 * in increments and the damped system comes to rest at each one.
 * For each of n_inc settings in turn, the context's field table (which must
 * have field_len = 1; the caller's buffer is overwritten and holds the last
 * setting on return) takes fields[k] (host [n_inc][M][12]: B0 then G,
 * row-major, per member). From the first force evaluation after it is set the
 * system steps (graphs as for rod_step) in chunks of check_every steps until,
 * after a chunk, the kinetic energy of every member (translational plus
 * rotational, from the state's velocities) is at most ke_tol, or max_steps
 * steps have been taken; a negative ke_tol runs every setting for max_steps.
 * Then the positions of the particles in watch (host [n_watch]) are written to
 * x_watch (host [n_inc][n_watch][3]), the steps taken to steps (host
 * [n_inc], nullable) and the members' kinetic energies to ke (host
 * [n_inc][M], nullable). The ramp synchronises after every chunk.
 * Errors: ROD_E_INVALID (NULL arguments, n_inc < 1, check_every < 1,
 * max_steps < 1, ke_tol not a number, field_len != 1, a watch index outside
 * [0, N)); ROD_E_STATE (a tape is being recorded); ROD_E_NONFINITE and
 * ROD_E_OVERFLOW as reported by rod_sync after a chunk (the ramp stops there;
 * outputs of earlier settings are written). */
int rod_ramp(rod_ctx* c, const double* fields, int32_t n_inc, int32_t max_steps,
             int32_t check_every, double ke_tol, const int32_t* watch, int32_t n_watch,
             double* x_watch, int32_t* steps, double* ke);

/* Measured arithmetic ceiling of the current GPU, for roofline fractions
 * reported beside the vendor peaks: a launch of 16 workgroups of 256 threads
 * per compute unit, each thread running 16 independent fused multiply-add
 * chains for 2048 iterations in vector registers (no memory traffic in the
 * loop). precision ROD_MIXED times FP32 FMAs (unpacked, as the library's own
 * arithmetic), ROD_FP64 FP64 FMAs. `sink` is a device buffer of one element of
 * that type, written only for an impossible result (it keeps the chains live).
 * Runs on hip_stream (NULL = default), synchronises, and writes the best of
 * five timed launches to *tflops (2 flops per FMA). Errors: ROD_E_INVALID
 * (NULL argument, unknown precision), ROD_E_HIP. Needs no context. */
int rod_probe_fma(int32_t precision, void* sink, void* hip_stream, double* tflops);

/* Release the context and its workspace (synchronises). NULL is accepted. */
int rod_free(rod_ctx* c);

/* Message of the last error on the calling thread ("" if none). */
const char* rod_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ROD_H */
