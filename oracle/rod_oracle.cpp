// Plain FP64 CPU oracle of the per-timestep force-and-integrate loop of the
// bonded-particle model for magneto-elastic rods.
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library. It shares no code, header
// or constant with the GPU library; both read the same seeded inputs.
//
// Style: straight loops in the order the paper states the steps, double
// precision, compiled with -ffp-contract=off. The scalar type is a template
// parameter so that the same code, instantiated with a dual number, yields exact
// forward-mode directional derivatives (JVPs) of a whole trajectory.
//
// Paper sections followed (main text unless marked SI):
//   bond model        "Bonded-particle model for elastic rods": eq. after the
//                     definition of r_i/r_f (relative displacement in C),
//                     eq:bpm-fr, eq:bpm-fst, eq:bpm-tst, eq:bpm-tb, eq:bpm-tt,
//                     eq:bpm-vector; spring constants below eq:bpm-vector;
//                     SI "Symmetric rotational decomposition" (eq:quat-h,
//                     u = q_C* q2, u = m* u0 m, u = t2 b2, u* = t1 b1,
//                     b = b2 b1*, t = t2 t1*).
//   energy            eq:total-energy.
//   magnetisation     "Magnetized beams in non-uniform fields": m = R m_body.
//   Zeeman / dipoles  Methods "Magnetic interactions".
//   contact           Methods "Contact": the workloads' Hookean normal law, or
//                     the paper's Hertz-Mindlin law (Hertz normal force,
//                     Mindlin tangential spring with a Coulomb limit and a
//                     per-contact tangential displacement history).
//   bond damping      Methods "Damping": radial term from the relative
//                     velocity along the bond axis; shear, twist and bend terms
//                     from finite-difference rates of the stored measures.
//   integrator        SI "Equations of motion" (velocity Verlet, Richardson
//                     quaternion update, renormalisation after each substep,
//                     solid-sphere inertia).
//   dipole cutoff     the truncated pair interaction of the paper's
//                     simulations (pairs closer than the cutoff only).
//   field ramp        the quasi-static loading protocol of "Magnetized beams
//                     in non-uniform fields" and of the helical rods with
//                     dipole-dipole interactions (settings in turn, each held
//                     with damped dynamics until the system is at rest).
//
// Readings where the paper is silent (each is listed in the design notes):
//   shortest-arc central frame; gamma via atan2 with the gamma/sigma limit at
//   sigma = 0; shortest-arc form of eq:quat-h with an x-axis fallback; twist
//   psi = psi2 - psi1 = 4 atan2(u_z, u_w); log map of b with b_w >= 0;
//   mass-proportional global damping with the half-step velocities; clamped
//   particles never move; driven particles have q = R(axis, 2 pi n / P).
//
// Parity pinned by: closed-form bond modes, invariants (objectivity, exchange,
// Newton's third law, angular momentum), a rotation-matrix re-derivation of the
// bond, Euler-Bernoulli cantilever limits, closed-form dipole pairs, finite
// differences of the energies, brute-force contact vs a k-d tree, integrator
// convergence order, finite differences of the dual-number JVP, closed forms of
// each bond damping mode and the damped oscillator, Hertz contact and impact
// theory with Mindlin stick-slip, the dipole cutoff's limits and partial sums,
// and the magnetic cantilever at every increment of a ramp.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <type_traits>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

// ---------------------------------------------------------------- scalars
struct Dual {  // value + one tangent component
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, s > 0 ? a.d / (2.0 * s) : 0.0);
}
inline Dual atan2(Dual y, Dual x) {
  double den = x.v * x.v + y.v * y.v;
  return Dual(std::atan2(y.v, x.v), den > 0 ? (x.v * y.d - y.v * x.d) / den : 0.0);
}
inline Dual sin(Dual a) { return Dual(std::sin(a.v), std::cos(a.v) * a.d); }
inline Dual cos(Dual a) { return Dual(std::cos(a.v), -std::sin(a.v) * a.d); }
inline double val(Dual a) { return a.v; }
inline double val(double a) { return a; }
using std::sqrt; using std::atan2; using std::sin; using std::cos;

// ---------------------------------------------------------------- vectors
template <class T> struct V3 { T x, y, z; };
template <class T> struct Q4 { T w, x, y, z; };  // Hamilton quaternion, w scalar

template <class T> V3<T> v3(T x, T y, T z) { return V3<T>{x, y, z}; }
template <class T> V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> T norm(V3<T> a) { return sqrt(dot(a, a)); }
template <class T> V3<T> lift(V3<double> a) { return {T(a.x), T(a.y), T(a.z)}; }

template <class T> Q4<T> qmul(Q4<T> a, Q4<T> b) {
  return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
          a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
          a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
template <class T> Q4<T> qconj(Q4<T> a) { return {a.w, -a.x, -a.y, -a.z}; }
template <class T> T qdot(Q4<T> a, Q4<T> b) { return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> Q4<T> qscale(T s, Q4<T> a) { return {s * a.w, s * a.x, s * a.y, s * a.z}; }
template <class T> Q4<T> qadd(Q4<T> a, Q4<T> b) { return {a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> Q4<T> qnormalize(Q4<T> a) { return qscale(T(1.0) / sqrt(qdot(a, a)), a); }
// Active rotation of a vector: q v q*.
template <class T> V3<T> qrot(Q4<T> q, V3<T> v) {
  Q4<T> p{T(0.0), v.x, v.y, v.z};
  Q4<T> r = qmul(qmul(q, p), qconj(q));
  return {r.x, r.y, r.z};
}

// ---------------------------------------------------------------- model
struct Bond {
  int i, j;             // particle 1 = i, particle 2 = j
  V3<double> rref;      // reference bond vector r_i (global = reference C frame)
  double Kr, Ks, Kt, Kb;
  double gr = 0, gs = 0, gt = 0, gb = 0;  // damping factors (Methods "Damping")
};

// Bond damping of one evaluation: the deformation measures of the previous
// time level (gamma, psi, theta-vector in C'; null: no rates yet), where the
// current ones go, the relative velocity v2 - v1 and the time step.
struct Damp {
  const double* hprev;
  double* hnow;
  V3<double> dv;
  double dt;
};

struct Model {
  int n = 0, R = 0, M = 0;
  std::vector<int> rod_of, member_of;
  std::vector<int> member_begin, member_end;  // particle ranges per member
  std::vector<double> mass, inertia;
  std::vector<Bond> bonds;
  std::vector<int8_t> bc;
  V3<double> drive_axis{1, 0, 0};
  int64_t drive_period = 0;
  double dt = 0, damping = 0, C = 1, kc = 0, rc = 0;
  int dipole_on = 0, contact_on = 0, depth = 1;
  const double* ext_force = nullptr;
  const double* ext_torque = nullptr;
  int field_len = 1;
  bool bond_damp = false;  // some bond has a non-zero damping factor
  // Contact law: 0 Hookean normal; 1 Hertz-Mindlin with contact modulus E,
  // Poisson ratio nu, friction coefficient mu, normal and tangential viscous
  // damping coefficients gn, gt.
  int contact_model = 0;
  double hmE = 0, hmNu = 0, hmMu = 0, hmGn = 0, hmGt = 0;
  // Dipole-dipole cutoff: 0 for every pair of a member; otherwise only pairs
  // with r^2 = (dx dx + dy dy) + dz dz < dcut^2 interact.
  double dcut = 0;
  // Periodic box (all three lengths > 0; else open boundaries): the dipole sum
  // is the Ewald sum of each member's periodic system, with splitting
  // parameter alpha, real-space cutoff rcut and reciprocal vectors
  // k = 2 pi (n_x / L_x, n_y / L_y, n_z / L_z), 0 < |n|^2 <= kmax^2.
  bool periodic = false;
  double box[3] = {0, 0, 0};
  double ew_alpha = 0, ew_rcut = 0;
  int ew_kmax = 0;
  // Immersed-boundary penalty (Methods, "Immersed boundary coupling"): the fluid
  // velocity interpolated at each particle ([N][3], or null: no coupling), the
  // fluid time step (kappa_p = m_p / fluid_dt) and where the forces go ([N][3]).
  const double* fluid_u = nullptr;
  double fluid_dt = 1.0;
  double* fluid_F = nullptr;
};

// Tangential displacement history of Hertz-Mindlin contacts: for particle i,
// its contacts j at one evaluation and the displacement s of each, seen from i.
struct CEntry {
  int j;
  V3<double> s;
};
using CHist = std::vector<std::vector<CEntry>>;

}  // namespace orc

extern "C" {

// Mirrors the workload dictionary (AoS arrays as the generator writes them).
struct orc_system {
  int32_t n, n_rods, n_members;
  const int32_t* rod_offset;   // [R+1]
  const int32_t* rod_member;   // [R]
  const double* rod_params;    // [R][4] diameter, density, Young, Poisson
  const double* x_ref;         // [N][3]
  const int8_t* bc;            // [N]
  double drive_axis[3];
  int64_t drive_period;
  int32_t field_len;
  const double* ext_force;     // [N][3] or NULL
  const double* ext_torque;    // [N][3] or NULL
  double dt, damping, mu0_4pi, k_contact, r_contact;
  int32_t dipole_on, contact_on, exclude_depth;
  const double* bond_damping;  // [R][4] g_r, g_s, g_t, g_b, or NULL
  int32_t contact_model;       // 0 Hookean, 1 Hertz-Mindlin
  double contact_hm[5];        // Hertz-Mindlin: E, nu, mu, g_n, g_t
  double dipole_cutoff;        // 0: all pairs of a member; > 0: pairs closer than this
  const double* fluid_u;       // [N][3] fluid velocity at the particles, or NULL
  double fluid_dt;             // fluid time step (penalty stiffness m_p / fluid_dt)
  double* fluid_F;             // [N][3] penalty force of the last evaluation, or NULL
  double box[3];               // periodic box lengths (all > 0), or zeros: open boundaries
  double ewald_alpha;          // Ewald splitting parameter
  double ewald_rcut;           // real-space cutoff of the Ewald sum
  int32_t ewald_kmax;          // reciprocal vectors with 0 < |n|^2 <= kmax^2
};

}  // extern "C"

namespace orc {

// Spring constants of a cylindrical bond of length L and diameter d
// (main text below eq:bpm-vector; SI "Deriving the spring constants").
static void spring_constants(double d, double E, double nu, double L, Bond& b) {
  const double pi = 3.14159265358979323846;
  double A = pi * d * d / 4.0;
  double I = pi * d * d * d * d / 64.0;
  double J = pi * d * d * d * d / 32.0;
  double G = E / (2.0 * (1.0 + nu));
  b.Kr = E * A / L;
  b.Ks = 12.0 * E * I / (L * L * L);
  b.Kt = G * J / L;
  b.Kb = E * I / L;
}

static Model build_model(const orc_system* s) {
  Model m;
  m.n = s->n; m.R = s->n_rods; m.M = s->n_members;
  m.rod_of.assign(m.n, -1);
  m.member_of.assign(m.n, -1);
  m.member_begin.assign(m.M, m.n);
  m.member_end.assign(m.M, 0);
  m.mass.assign(m.n, 0.0);
  m.inertia.assign(m.n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int r = 0; r < m.R; ++r) {
    int mem = s->rod_member[r];
    double d = s->rod_params[4 * r + 0], rho = s->rod_params[4 * r + 1];
    double E = s->rod_params[4 * r + 2], nu = s->rod_params[4 * r + 3];
    for (int p = s->rod_offset[r]; p < s->rod_offset[r + 1]; ++p) {
      m.rod_of[p] = r;
      m.member_of[p] = mem;
      // Solid sphere of diameter d (SI "Equations of motion"): I = 2/5 m R^2.
      m.mass[p] = rho * pi * d * d * d / 6.0;
      m.inertia[p] = 0.4 * m.mass[p] * (0.5 * d) * (0.5 * d);
      m.member_begin[mem] = std::min(m.member_begin[mem], p);
      m.member_end[mem] = std::max(m.member_end[mem], p + 1);
      // Consecutive particles of a rod are bonded; the reference bond is the
      // unperturbed lattice vector, with reference orientations equal to 1.
      if (p + 1 < s->rod_offset[r + 1]) {
        Bond b;
        b.i = p; b.j = p + 1;
        b.rref = {s->x_ref[3 * (p + 1)] - s->x_ref[3 * p],
                  s->x_ref[3 * (p + 1) + 1] - s->x_ref[3 * p + 1],
                  s->x_ref[3 * (p + 1) + 2] - s->x_ref[3 * p + 2]};
        spring_constants(d, E, nu, norm(b.rref), b);
        if (s->bond_damping) {
          b.gr = s->bond_damping[4 * r + 0]; b.gs = s->bond_damping[4 * r + 1];
          b.gt = s->bond_damping[4 * r + 2]; b.gb = s->bond_damping[4 * r + 3];
          m.bond_damp = m.bond_damp || b.gr != 0 || b.gs != 0 || b.gt != 0 || b.gb != 0;
        }
        m.bonds.push_back(b);
      }
    }
  }
  m.bc.assign(s->bc, s->bc + m.n);
  m.drive_axis = {s->drive_axis[0], s->drive_axis[1], s->drive_axis[2]};
  m.drive_period = s->drive_period;
  m.dt = s->dt; m.damping = s->damping; m.C = s->mu0_4pi;
  m.kc = s->k_contact; m.rc = s->r_contact;
  m.dipole_on = s->dipole_on; m.contact_on = s->contact_on; m.depth = s->exclude_depth;
  m.ext_force = s->ext_force; m.ext_torque = s->ext_torque;
  m.field_len = s->field_len > 0 ? s->field_len : 1;
  m.contact_model = s->contact_model;
  m.hmE = s->contact_hm[0]; m.hmNu = s->contact_hm[1]; m.hmMu = s->contact_hm[2];
  m.hmGn = s->contact_hm[3]; m.hmGt = s->contact_hm[4];
  m.dcut = s->dipole_cutoff;
  m.periodic = s->box[0] > 0 && s->box[1] > 0 && s->box[2] > 0;
  for (int a = 0; a < 3; ++a) m.box[a] = s->box[a];
  m.ew_alpha = s->ewald_alpha; m.ew_rcut = s->ewald_rcut; m.ew_kmax = s->ewald_kmax;
  m.fluid_u = s->fluid_u; m.fluid_dt = s->fluid_dt > 0 ? s->fluid_dt : 1.0; m.fluid_F = s->fluid_F;
  return m;
}

// ---------------------------------------------------------------- one bond
// Forces and torques of one bond between particles 1 and 2, following the
// symmetric decomposition step by step. Outputs, all in the global frame:
//   F   = f_r + f_s acting on particle 1 (particle 2 receives -F),
//   Ts  = tau_s (both particles),
//   Tbt = tau_b + tau_t acting on particle 1 (particle 2 receives -Tbt),
//   e   = the four terms of eq:total-energy.
// With `dmp`, the damping terms of Methods "Damping" are added and the current
// measures are stored (see Damp).
template <class T>
void bond_eval(V3<T> x1, V3<T> x2, Q4<T> q1, Q4<T> q2, const Bond& bd,
               V3<T>& F, V3<T>& Ts, V3<T>& Tbt, T e[4], const Damp* dmp = nullptr) {
  const T zero(0.0), one(1.0), half(0.5);
  // Bond vectors r_f (current) and r_i (reference), global frame.
  V3<T> rf = x2 - x1;
  double r0 = norm(bd.rref);
  V3<T> ri_hat = lift<T>((1.0 / r0) * bd.rref);

  // Central frame q_C: spherical midpoint of q1 and q2 on the short arc.
  if (val(qdot(q1, q2)) < 0.0) q2 = qscale(T(-1.0), q2);
  Q4<T> qc = qnormalize(qadd(q1, q2));

  // r_f seen from the moving central frame: q_C* r_f q_C.
  V3<T> rho = qrot(qconj(qc), rf);
  T r = norm(rho);
  V3<T> rh = (one / r) * rho;

  // Radial force (eq:bpm-fr), in C; radial damping adds g_r times the relative
  // velocity along the bond axis, (v2 - v1) . r_f-hat = (q_C* (v2 - v1) q_C) . r-hat.
  T frad = T(bd.Kr) * (r - T(r0));
  if (dmp) frad = frad + T(bd.gr) * dot(qrot(qconj(qc), lift<T>(dmp->dv)), rh);
  V3<T> fr = frad * rh;

  // Shear angle gamma between r_i-hat and r_f-hat[C]; t = c/|c|, s = t x r_f-hat.
  // f_s = K_s r gamma s and tau_s = 1/2 K_s r^2 gamma t (eq:bpm-fst, eq:bpm-tst),
  // written with g = gamma/|c| so that the straight bond (c = 0) is its limit.
  V3<T> c = cross(ri_hat, rh);
  T sigma = norm(c);
  T cg = dot(ri_hat, rh);
  T gamma = atan2(sigma, cg);
  T g = val(sigma) > 0.0 ? gamma / sigma : one / cg;
  // Shear damping: K_s gamma becomes K_s gamma + g_s gamma-dot in f_s and tau_s,
  // gamma-dot = (gamma^n - gamma^(n-1)) / dt; no term where s-hat is undefined.
  T ks = T(bd.Ks) * g;
  if (dmp && dmp->hprev && val(sigma) > 0.0)
    ks = ks + T(bd.gs) * ((gamma - T(dmp->hprev[0])) / T(dmp->dt)) / sigma;
  V3<T> fs = (r * ks) * cross(c, rh);
  V3<T> ts = (half * r * r * ks) * c;

  // Quaternion m turning the z-axis of C onto r_f-hat[C] (eq:quat-h, written as
  // the shortest-arc quaternion normalize(1 + z, -y, x, 0)).
  Q4<T> mq;
  if (val(one + rh.z) > 1e-12)
    mq = qnormalize(Q4<T>{one + rh.z, -rh.y, rh.x, zero});
  else
    mq = Q4<T>{zero, one, zero, zero};

  // Half rotation u0 = q_C* q2 (= q1* q_C), expressed in C': u = m* u0 m.
  Q4<T> u0 = qmul(qconj(qc), q2);
  Q4<T> u = qmul(qmul(qconj(mq), u0), mq);

  // Swing-twist with bend before twist: u = t2 b2, u* = t1 b1, t1 = t2*.
  T tn = sqrt(u.w * u.w + u.z * u.z);
  Q4<T> t2{u.w / tn, zero, zero, u.z / tn};
  T psi = T(4.0) * atan2(u.z, u.w);   // psi2 - psi1 with psi1 = -psi2
  Q4<T> b2 = qmul(qconj(t2), u);
  Q4<T> b1 = qmul(t2, qconj(u));
  Q4<T> b = qmul(b2, qconj(b1));       // effective bend b = b2 b1*

  // Axis-angle vector theta b-hat of b (short arc).
  if (val(b.w) < 0.0) b = qscale(T(-1.0), b);
  V3<T> bv{b.x, b.y, b.z};
  T bn = norm(bv);
  T theta = T(2.0) * atan2(bn, b.w);
  T fac = val(bn) > 0.0 ? theta / bn : T(2.0) / b.w;
  V3<T> th = fac * bv;

  // Bending and twisting torques in C' (eq:bpm-tb, eq:bpm-tt).
  V3<T> tbt{T(bd.Kb) * th.x, T(bd.Kb) * th.y, T(bd.Kb) * th.z + T(bd.Kt) * psi};
  // Twist and bend damping: g_t psi-dot and g_b theta-dot (per component in C'),
  // the twist change taken modulo 2 pi (psi wraps at +-pi).
  if (dmp && dmp->hprev) {
    const double twopi = 6.28318530717958647692;
    T dpsi = psi - T(dmp->hprev[1]);
    dpsi = dpsi - T(twopi * std::round(val(dpsi) / twopi));
    const T idt(1.0 / dmp->dt);
    tbt = tbt + V3<T>{T(bd.gb) * (th.x - T(dmp->hprev[2])) * idt,
                      T(bd.gb) * (th.y - T(dmp->hprev[3])) * idt,
                      T(bd.gb) * (th.z - T(dmp->hprev[4])) * idt + T(bd.gt) * dpsi * idt};
  }
  if (dmp && dmp->hnow) {
    dmp->hnow[0] = val(gamma); dmp->hnow[1] = val(psi);
    dmp->hnow[2] = val(th.x); dmp->hnow[3] = val(th.y); dmp->hnow[4] = val(th.z);
  }

  // Back to the global frame: v[O] = q_C v[C] q_C*, v[O] = q_C m v[C'] m* q_C*.
  F = qrot(qc, fr + fs);
  Ts = qrot(qc, ts);
  Tbt = qrot(qmul(qc, mq), tbt);

  // eq:total-energy.
  T dr = r - T(r0);
  e[0] = half * T(bd.Kr) * dr * dr;
  e[1] = half * T(bd.Ks) * r * r * gamma * gamma;
  e[2] = half * T(bd.Kt) * psi * psi;
  e[3] = half * T(bd.Kb) * theta * theta;
}

// ---------------------------------------------------------------- state views
template <class T> V3<T> ld3(const T* a, int p) { return {a[3 * p], a[3 * p + 1], a[3 * p + 2]}; }
template <class T> Q4<T> ld4(const T* a, int p) { return {a[4 * p], a[4 * p + 1], a[4 * p + 2], a[4 * p + 3]}; }
template <class T> void st3(T* a, int p, V3<T> v) { a[3 * p] = v.x; a[3 * p + 1] = v.y; a[3 * p + 2] = v.z; }
template <class T> void st4(T* a, int p, Q4<T> q) { a[4 * p] = q.w; a[4 * p + 1] = q.x; a[4 * p + 2] = q.y; a[4 * p + 3] = q.z; }
template <class T> void add3(T* a, int p, V3<T> v) { a[3 * p] += v.x; a[3 * p + 1] += v.y; a[3 * p + 2] += v.z; }

// External field of a member at step n: B(x) = B0 + G x (G row-major).
template <class T> struct Field { V3<T> B0; T G[9]; };
template <class T> Field<T> field_at(const Model& md, const T* field, int64_t n, int mem) {
  int64_t L = md.field_len;
  int64_t idx = ((n % L) + L) % L;
  const T* f = field + (idx * md.M + mem) * 12;
  Field<T> F;
  F.B0 = {f[0], f[1], f[2]};
  for (int k = 0; k < 9; ++k) F.G[k] = f[3 + k];
  return F;
}
template <class T> V3<T> field_B(const Field<T>& f, V3<T> x) {
  return {f.B0.x + f.G[0] * x.x + f.G[1] * x.y + f.G[2] * x.z,
          f.B0.y + f.G[3] * x.x + f.G[4] * x.y + f.G[5] * x.z,
          f.B0.z + f.G[6] * x.x + f.G[7] * x.y + f.G[8] * x.z};
}

enum { T_BOND = 1, T_DIPOLE = 2, T_ZEEMAN = 4, T_CONTACT = 8, T_DAMP = 16, T_EXT = 32, T_ALL = 63,
       T_FLUID = 64 };

static bool excluded(const Model& md, int i, int j) {
  if (md.member_of[i] != md.member_of[j]) return true;
  return md.rod_of[i] == md.rod_of[j] && std::abs(i - j) <= md.depth;
}

// Dipole moments in the global frame: m = R(q) m_body (magnetisation rotates
// with the particle).
template <class T>
void dipoles(const Model& md, const T* q, const T* mbody, std::vector<T>& mu) {
  mu.assign(3 * md.n, T(0.0));
  for (int p = 0; p < md.n; ++p) st3(mu.data(), p, qrot(ld4(q, p), ld3(mbody, p)));
}

// Total force and torque at one time level.
//   x, q: positions and orientations;  v, w: the velocities used by damping;
//   mu: global dipole moments; field: external field table; n: time level.
// Bdip (optional) receives the dipole field at each particle.
// ---------------------------------------------------------------- Ewald
// Periodic dipole-dipole interaction by Ewald summation: the long-range
// solvers the paper's LAMMPS implementation offers beside the truncated pair
// style (Introduction; SI "Magnetic dipoles"), for a member whose particles
// repeat in a box L_x x L_y x L_z, with conducting boundaries at infinity (no
// surface term). With C = mu0/4pi, r = x_i - x_j + n L over every image, the
// interaction splits at alpha into
//   real space, pairs (and images of a particle itself) closer than rcut:
//     U = C sum (mi.mj) B(r) - (mi.r)(mj.r) C(r), with
//     B = [erfc(a r) + 2 a r/sqrt(pi) e] / r^3,
//     C = [3 erfc(a r) + 2 a r/sqrt(pi) (3 + 2 a^2 r^2) e] / r^5,
//     D = [15 erfc(a r) + 2 a r/sqrt(pi) (15 + 10 a^2 r^2 + 4 a^4 r^4) e] / r^7,
//     e = exp(-a^2 r^2): the screened forms of 1/r^3, 3/r^5, 15/r^7;
//   reciprocal space, k = 2 pi n / L, n != 0, |n|^2 <= kmax^2:
//     U = (2 pi C / V) sum_k g(k) |S(k)|^2, g = exp(-k^2 / 4 a^2) / k^2,
//     S(k) = sum_j (mj.k) exp(i k.x_j);
//   self: U = -C 2 a^3 / (3 sqrt(pi)) sum |m_i|^2.
// Force F_i = -dU/dx_i, field B_i = -dU/dm_i (so that U = -1/2 sum m_i.B_i and
// the torque is m_i x B_i):
//   real: F_i += C [(mi.mj) C r + C ((mj.r) mi + (mi.r) mj) - (mi.r)(mj.r) D r],
//         B_i += C [C (mj.r) r - B mj];
//   reciprocal: F_i += (4 pi C / V) g (mi.k) k Im[exp(i k.x_i) S*(k)],
//               B_i -= (4 pi C / V) g k Re[exp(i k.x_i) S*(k)];
//   self: B_i += C 4 a^3 / (3 sqrt(pi)) m_i.
// Every image within rcut is taken (rcut may exceed half the box); the
// reciprocal sum runs over all k of the sphere, k and -k alike.
// F, Bd: [N][3] (added to); U: [M] (added to) or null.
static void ewald_dipoles(const Model& md, const double* x, const double* mu, double* F,
                          double* Bd, double* U) {
  const double pi = 3.14159265358979323846;
  const double C = md.C, a = md.ew_alpha, rc2 = md.ew_rcut * md.ew_rcut;
  const double L[3] = {md.box[0], md.box[1], md.box[2]};
  const double V = L[0] * L[1] * L[2];
  const double sp = 2.0 * a / std::sqrt(pi);
  for (int mem = 0; mem < md.M; ++mem) {
    const int b = md.member_begin[mem], e = md.member_end[mem];
    double Um = 0.0;
    // real space
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : Um)
    for (int i = b; i < e; ++i) {
      const V3<double> xi = ld3(x, i), mi = ld3(mu, i);
      V3<double> Fi{0, 0, 0}, Bi{0, 0, 0};
      for (int j = b; j < e; ++j) {
        const V3<double> mj = ld3(mu, j);
        const V3<double> r0 = xi - ld3(x, j);
        const double r0a[3] = {r0.x, r0.y, r0.z};
        int lo[3], hi[3];
        for (int ax = 0; ax < 3; ++ax) {
          lo[ax] = (int)std::ceil((-md.ew_rcut - r0a[ax]) / L[ax]);
          hi[ax] = (int)std::floor((md.ew_rcut - r0a[ax]) / L[ax]);
        }
        for (int nx = lo[0]; nx <= hi[0]; ++nx)
          for (int ny = lo[1]; ny <= hi[1]; ++ny)
            for (int nz = lo[2]; nz <= hi[2]; ++nz) {
              if (i == j && nx == 0 && ny == 0 && nz == 0) continue;
              const V3<double> r{r0.x + nx * L[0], r0.y + ny * L[1], r0.z + nz * L[2]};
              const double r2 = dot(r, r);
              if (!(r2 < rc2)) continue;
              const double rr = std::sqrt(r2), ar = a * rr, ex = std::exp(-ar * ar);
              const double ec = std::erfc(ar);
              const double Bf = (ec + sp * rr * ex) / (r2 * rr);
              const double Cf = (3.0 * ec + sp * rr * (3.0 + 2.0 * ar * ar) * ex) / (r2 * r2 * rr);
              const double Df = (15.0 * ec + sp * rr * (15.0 + 10.0 * ar * ar + 4.0 * ar * ar * ar * ar) * ex) /
                                (r2 * r2 * r2 * rr);
              const double dmi = dot(mi, r), dmj = dot(mj, r), mm = dot(mi, mj);
              Fi = Fi + C * ((mm * Cf) * r + Cf * (dmj * mi + dmi * mj) - (dmi * dmj * Df) * r);
              Bi = Bi + C * ((Cf * dmj) * r - Bf * mj);
              Um += 0.5 * C * (mm * Bf - dmi * dmj * Cf);
            }
      }
      add3(F, i, Fi);
      add3(Bd, i, Bi);
    }
    // reciprocal space
    const int K = md.ew_kmax;
    for (int nx = -K; nx <= K; ++nx)
      for (int ny = -K; ny <= K; ++ny)
        for (int nz = -K; nz <= K; ++nz) {
          const int n2 = nx * nx + ny * ny + nz * nz;
          if (n2 == 0 || n2 > K * K) continue;
          const V3<double> k{2.0 * pi * nx / L[0], 2.0 * pi * ny / L[1], 2.0 * pi * nz / L[2]};
          const double k2 = dot(k, k);
          const double g = std::exp(-k2 / (4.0 * a * a)) / k2;
          double Sr = 0.0, Si = 0.0;
          for (int j = b; j < e; ++j) {
            const double mk = dot(ld3(mu, j), k), ph = dot(k, ld3(x, j));
            Sr += mk * std::cos(ph);
            Si += mk * std::sin(ph);
          }
          Um += 2.0 * pi * C / V * g * (Sr * Sr + Si * Si);
          const double c = 4.0 * pi * C / V * g;
          for (int i = b; i < e; ++i) {
            const double ph = dot(k, ld3(x, i));
            const double cs = std::cos(ph), sn = std::sin(ph);
            const double mk = dot(ld3(mu, i), k);
            add3(F, i, (c * mk * (sn * Sr - cs * Si)) * k);
            add3(Bd, i, (-c * (cs * Sr + sn * Si)) * k);
          }
        }
    // self
    const double cs = C * 4.0 * a * a * a / (3.0 * std::sqrt(pi));
    for (int i = b; i < e; ++i) {
      const V3<double> mi = ld3(mu, i);
      add3(Bd, i, cs * mi);
      Um -= 0.5 * cs * dot(mi, mi);
    }
    if (U) U[mem] += Um;
  }
}

// ---------------------------------------------------------------- Hertz-Mindlin
// One Hertz-Mindlin contact seen from particle i, its partner j closer than r_c
// (Methods, "Contact", which names the law; its constants are the textbook
// ones for two equal elastic spheres of diameter r_c):
//   n = (x_i - x_j) / r, overlap delta = r_c - r, R* = r_c / 4,
//   E* = E / (2 (1 - nu^2)), G* = E / (4 (2 - nu)(1 + nu)), a = sqrt(R* delta);
//   normal: F_n = max(0, 4/3 E* a delta - g_n v_n), v_n = (v_rel . n);
//   contact-point velocity of i relative to j: the two centres' velocities plus
//     w x (branch vector) of each, the branch vectors being -r/2 n and +r/2 n:
//     v_rel = (v_i - v_j) - r/2 (w_i + w_j) x n, tangential part v_t;
//   tangential (Mindlin): s, the tangential displacement of the contact, is
//     turned into the current tangent plane (keeping its length) and advanced
//     by v_t dt; a contact absent from the previous evaluation starts at s = 0;
//     F_t = -8 G* a s - g_t v_t, limited to |F_t| <= mu F_n (where the limit
//     acts, s is reset to the displacement that holds the limited force);
//   force on i: F_n n + F_t (j receives the opposite); torque on i and on j:
//     (-r/2 n) x F_t.
// sprev: s of the previous evaluation, or null for a new contact. Writes the
// new s to snow and the normal elastic energy 8/15 E* sqrt(R*) delta^(5/2) to e.
static void hertz_mindlin(const Model& md, V3<double> xi, V3<double> xj, V3<double> vi,
                          V3<double> vj, V3<double> wi, V3<double> wj, const V3<double>* sprev,
                          V3<double>& F, V3<double>& Tq, V3<double>& snow, double& e) {
  const V3<double> d = xi - xj;
  const double r = std::sqrt((d.x * d.x + d.y * d.y) + d.z * d.z);
  const V3<double> n = (1.0 / r) * d;
  const double delta = md.rc - r;
  const double Rs = 0.25 * md.rc;
  const double Es = md.hmE / (2.0 * (1.0 - md.hmNu * md.hmNu));
  const double Gs = md.hmE / (4.0 * (2.0 - md.hmNu) * (1.0 + md.hmNu));
  const double a = std::sqrt(Rs * delta);
  const double kn = 4.0 / 3.0 * Es * a, kt = 8.0 * Gs * a;

  const V3<double> vrel = (vi - vj) - (0.5 * r) * cross(wi + wj, n);
  const double vn = dot(vrel, n);
  const V3<double> vt = vrel - vn * n;
  const double Fn = std::max(0.0, kn * delta - md.hmGn * vn);

  V3<double> sv{0.0, 0.0, 0.0};
  if (sprev) {
    V3<double> sp = *sprev;
    V3<double> st = sp - dot(sp, n) * n;  // into the current tangent plane
    const double lt = norm(st), lp = norm(sp);
    if (lt > 0.0) st = (lp / lt) * st;
    sv = st + md.dt * vt;
  }
  V3<double> Ft = (-kt) * sv - md.hmGt * vt;
  const double ft = norm(Ft), fmax = md.hmMu * Fn;
  if (ft > fmax) {
    Ft = (fmax / ft) * Ft;
    sv = (-1.0 / kt) * (Ft + md.hmGt * vt);
  }
  F = Fn * n + Ft;
  Tq = cross((-0.5 * r) * n, Ft);
  snow = sv;
  e = 8.0 / 15.0 * Es * std::sqrt(Rs) * delta * delta * std::sqrt(delta);
}

// hprev / hnow: [B][5] bond damping measures of the previous and the current
// level (see Damp); used when the model has bond damping (FP64 only).
// cprev / cnow: Hertz-Mindlin contact histories of the previous evaluation
// (null: none, every contact is new) and of this one (written when non-null).
template <class T>
void forces(const Model& md, const T* x, const T* q, const T* v, const T* w,
            const T* mu, const T* field, int64_t n, int mask, T* F, T* Tq,
            T* Bdip = nullptr, const double* hprev = nullptr, double* hnow = nullptr,
            const CHist* cprev = nullptr, CHist* cnow = nullptr) {
  const int N = md.n;
  for (int k = 0; k < 3 * N; ++k) { F[k] = T(0.0); Tq[k] = T(0.0); }

  // Bonds: each bond adds its forces to its two particles (eq:bpm-vector).
  if (mask & T_BOND) {
    const int B = (int)md.bonds.size();
    std::vector<V3<T>> bF(B), bTs(B), bTbt(B);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < B; ++k) {
      const Bond& bd = md.bonds[k];
      T e[4];
      if constexpr (std::is_same<T, double>::value) {
        if (md.bond_damp) {
          Damp dm{hprev ? hprev + 5 * k : nullptr, hnow ? hnow + 5 * k : nullptr,
                  ld3(v, bd.j) - ld3(v, bd.i), md.dt};
          bond_eval(ld3(x, bd.i), ld3(x, bd.j), ld4(q, bd.i), ld4(q, bd.j), bd,
                    bF[k], bTs[k], bTbt[k], e, &dm);
          continue;
        }
      }
      bond_eval(ld3(x, bd.i), ld3(x, bd.j), ld4(q, bd.i), ld4(q, bd.j), bd,
                bF[k], bTs[k], bTbt[k], e);
    }
    for (int k = 0; k < B; ++k) {
      const Bond& bd = md.bonds[k];
      add3(F, bd.i, bF[k]);
      add3(Tq, bd.i, bTs[k] + bTbt[k]);
      add3(F, bd.j, T(-1.0) * bF[k]);
      add3(Tq, bd.j, bTs[k] - bTbt[k]);
    }
  }

  // Dipole-dipole, every ordered pair i != j of a member (Methods, "Magnetic
  // interactions"), or with a cutoff only the pairs closer than it (the
  // truncated pair interaction the paper's simulations use). With
  // r = x_i - x_j, U = C/r^3 [mi.mj - 3 (mi.r^)(mj.r^)];
  // F_i = -dU/dx_i; the field of j at x_i is C (3 (mj.r) r / r^5 - mj / r^3);
  // the torque is m_i x B_i.
  std::vector<T> Bd(3 * N, T(0.0));
  if ((mask & T_DIPOLE) && md.dipole_on && md.periodic) {
    if constexpr (std::is_same<T, double>::value) {
      std::vector<double> Fe(3 * N, 0.0);
      ewald_dipoles(md, x, mu, Fe.data(), Bd.data(), nullptr);
      for (int i = 0; i < N; ++i) {
        add3(F, i, ld3(Fe.data(), i));
        add3(Tq, i, cross(ld3(mu, i), ld3(Bd.data(), i)));
      }
    }
  } else if ((mask & T_DIPOLE) && md.dipole_on) {
    const T C(md.C);
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < N; ++i) {
      int mem = md.member_of[i];
      V3<T> xi = ld3(x, i), mi = ld3(mu, i);
      V3<T> Fi{T(0.0), T(0.0), T(0.0)}, Bi{T(0.0), T(0.0), T(0.0)};
      for (int j = md.member_begin[mem]; j < md.member_end[mem]; ++j) {
        if (j == i) continue;
        V3<T> mj = ld3(mu, j);
        V3<T> r = xi - ld3(x, j);
        T r2 = dot(r, r);
        if (md.dcut > 0.0 && !(val(r2) < md.dcut * md.dcut)) continue;
        T rinv = T(1.0) / sqrt(r2);
        T rinv3 = rinv * rinv * rinv;
        T rinv5 = rinv3 * rinv * rinv;
        T a = dot(mi, r), b = dot(mj, r), cmm = dot(mi, mj);
        V3<T> fij = (T(3.0) * C * rinv5) *
                    ((cmm * r + b * mi + a * mj) - (T(5.0) * a * b * rinv * rinv) * r);
        V3<T> bij = (T(3.0) * C * b * rinv5) * r - (C * rinv3) * mj;
        Fi = Fi + fij;
        Bi = Bi + bij;
      }
      st3(Bd.data(), i, Bi);
      add3(F, i, Fi);
      add3(Tq, i, cross(mi, Bi));
    }
  }
  if (Bdip) for (int k = 0; k < 3 * N; ++k) Bdip[k] = Bd[k];

  // Zeeman: U = -m.B, f = grad(m.B) = G^T m, tau = m x B.
  if (mask & T_ZEEMAN) {
    for (int p = 0; p < N; ++p) {
      Field<T> f = field_at(md, field, n, md.member_of[p]);
      V3<T> mp = ld3(mu, p);
      V3<T> B = field_B(f, ld3(x, p));
      V3<T> fz{f.G[0] * mp.x + f.G[3] * mp.y + f.G[6] * mp.z,
               f.G[1] * mp.x + f.G[4] * mp.y + f.G[7] * mp.z,
               f.G[2] * mp.x + f.G[5] * mp.y + f.G[8] * mp.z};
      add3(F, p, fz);
      add3(Tq, p, cross(mp, B));
    }
  }

  // Hertz-Mindlin contact: the same pairs as below, each seen from both ends.
  if constexpr (std::is_same<T, double>::value) {
    if ((mask & T_CONTACT) && md.contact_on && md.contact_model == 1) {
      const double rc2 = md.rc * md.rc;
      if (cnow) cnow->assign(N, {});
#pragma omp parallel for schedule(dynamic, 64)
      for (int i = 0; i < N; ++i) {
        int mem = md.member_of[i];
        V3<double> Fi{0.0, 0.0, 0.0}, Ti{0.0, 0.0, 0.0};
        for (int j = md.member_begin[mem]; j < md.member_end[mem]; ++j) {
          if (j == i || excluded(md, i, j)) continue;
          V3<double> d = ld3(x, i) - ld3(x, j);
          double r2 = (d.x * d.x + d.y * d.y) + d.z * d.z;
          if (!(r2 < rc2)) continue;
          const V3<double>* sp = nullptr;
          if (cprev)
            for (const CEntry& c : (*cprev)[i])
              if (c.j == j) sp = &c.s;
          V3<double> f, t, sn;
          double e;
          hertz_mindlin(md, ld3(x, i), ld3(x, j), ld3(v, i), ld3(v, j), ld3(w, i), ld3(w, j),
                        sp, f, t, sn, e);
          Fi = Fi + f;
          Ti = Ti + t;
          if (cnow) (*cnow)[i].push_back({j, sn});
        }
        add3(F, i, Fi);
        add3(Tq, i, Ti);
      }
    }
  }

  // Contact: brute force over all pairs of a member that are not excluded;
  // pairs with r^2 = (dx dx + dy dy) + dz dz < r_c^2 repel with k (r_c - r).
  if ((mask & T_CONTACT) && md.contact_on && md.contact_model == 0) {
    const double rc2 = md.rc * md.rc;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < N; ++i) {
      int mem = md.member_of[i];
      V3<T> Fi{T(0.0), T(0.0), T(0.0)};
      for (int j = md.member_begin[mem]; j < md.member_end[mem]; ++j) {
        if (j == i || excluded(md, i, j)) continue;
        V3<T> d = ld3(x, i) - ld3(x, j);
        T r2 = (d.x * d.x + d.y * d.y) + d.z * d.z;
        if (!(val(r2) < rc2)) continue;
        T r = sqrt(r2);
        Fi = Fi + (T(md.kc) * (T(md.rc) - r) / r) * d;
      }
      add3(F, i, Fi);
    }
  }

  // Global viscous damping (mass-proportional) with the supplied velocities.
  if (mask & T_DAMP) {
    for (int p = 0; p < N; ++p) {
      add3(F, p, T(-md.damping * md.mass[p]) * ld3(v, p));
      add3(Tq, p, T(-md.damping * md.inertia[p]) * ld3(w, p));
    }
  }
  // Immersed-boundary penalty force kappa_p (U_p - v_p), kappa_p = m_p / fluid_dt,
  // with the velocities the evaluation sees (half-step ones while stepping).
  if constexpr (std::is_same<T, double>::value) {
    if ((mask & T_FLUID) && md.fluid_u) {
      for (int p = 0; p < N; ++p) {
        const V3<double> Fp = (md.mass[p] / md.fluid_dt) * (ld3(md.fluid_u, p) - ld3(v, p));
        add3(F, p, Fp);
        if (md.fluid_F) st3(md.fluid_F, p, Fp);
      }
    }
  }
  if (mask & T_EXT) {
    for (int p = 0; p < N; ++p) {
      if (md.ext_force) add3(F, p, lift<T>(V3<double>{md.ext_force[3 * p], md.ext_force[3 * p + 1], md.ext_force[3 * p + 2]}));
      if (md.ext_torque) add3(Tq, p, lift<T>(V3<double>{md.ext_torque[3 * p], md.ext_torque[3 * p + 1], md.ext_torque[3 * p + 2]}));
    }
  }
}

// ---------------------------------------------------------------- integrator
// dq/dt = 1/2 (0, w) q for the space-frame angular velocity w.
template <class T> Q4<T> qrate(Q4<T> q, V3<T> w) {
  return qscale(T(0.5), qmul(Q4<T>{T(0.0), w.x, w.y, w.z}, q));
}

// Richardson update of q over dt with the half-step angular velocity; every
// intermediate quaternion is renormalised.
template <class T> Q4<T> richardson(Q4<T> q, V3<T> w, double dt) {
  Q4<T> q1 = qnormalize(qadd(q, qscale(T(dt), qrate(q, w))));
  Q4<T> qh = qnormalize(qadd(q, qscale(T(0.5 * dt), qrate(q, w))));
  Q4<T> q2 = qnormalize(qadd(qh, qscale(T(0.5 * dt), qrate(qh, w))));
  return qnormalize(qadd(qscale(T(2.0), q2), qscale(T(-1.0), q1)));
}

template <class T> Q4<T> drive_q(const Model& md, int64_t n) {
  const double pi = 3.14159265358979323846;
  double phi = 2.0 * pi * (double)n / (double)md.drive_period;
  double s = std::sin(0.5 * phi);
  return {T(std::cos(0.5 * phi)), T(s * md.drive_axis.x), T(s * md.drive_axis.y), T(s * md.drive_axis.z)};
}

template <class T> struct State {
  std::vector<T> x, v, q, w, F, Tq;
  int64_t step = 0;
  std::vector<double> hist;  // [B][5] bond damping measures of the last force evaluation
  bool hist_valid = false;
  CHist chist;               // Hertz-Mindlin contacts of the last force evaluation
  bool chist_valid = false;
};

// Boundary-condition state of driven particles at time level n.
template <class T> void apply_drive(const Model& md, State<T>& s, int64_t n) {
  if (md.drive_period == 0) return;
  const double pi = 3.14159265358979323846;
  double Om = 2.0 * pi / ((double)md.drive_period * md.dt);
  for (int p = 0; p < md.n; ++p) {
    if (md.bc[p] != 2) continue;
    st4(s.q.data(), p, drive_q<T>(md, n));
    st3(s.v.data(), p, V3<T>{T(0.0), T(0.0), T(0.0)});
    st3(s.w.data(), p, lift<T>(Om * md.drive_axis));
  }
}

// Forces of level n; with bond damping the rates are taken against the
// measures of the previous evaluation (none yet: no rates), which are then
// replaced by this level's. Hertz-Mindlin contacts likewise continue from the
// contacts of the previous evaluation (none yet: every contact is new).
template <class T>
void eval_forces(const Model& md, State<T>& s, const T* mbody, const T* field, int64_t n) {
  std::vector<T> mu;
  dipoles(md, s.q.data(), mbody, mu);
  std::vector<double> hnow(md.bond_damp ? 5 * md.bonds.size() : 0);
  const bool hm = md.contact_on && md.contact_model == 1;
  CHist cnow;
  forces(md, s.x.data(), s.q.data(), s.v.data(), s.w.data(), mu.data(), field, n,
         T_ALL | T_FLUID, s.F.data(), s.Tq.data(), (T*)nullptr,
         md.bond_damp && s.hist_valid ? s.hist.data() : nullptr,
         md.bond_damp ? hnow.data() : nullptr,
         hm && s.chist_valid ? &s.chist : nullptr, hm ? &cnow : nullptr);
  if (md.bond_damp) {
    s.hist.swap(hnow);
    s.hist_valid = true;
  }
  if (hm) {
    s.chist.swap(cnow);
    s.chist_valid = true;
  }
}

// Bond damping measures and Hertz-Mindlin contacts of a given state (a
// continued run that brings none): they are taken from its own configuration,
// as a first evaluation would (no rates; every contact new, s = 0), its forces
// left as they are, so that its first step continues from them.
template <class T>
void record_measures(const Model& md, State<T>& s, const T* mbody, const T* field, int64_t n,
                     bool bonds, bool contacts) {
  std::vector<T> mu, Ft(3 * md.n), Tt(3 * md.n);
  dipoles(md, s.q.data(), mbody, mu);
  std::vector<double> hnow(5 * md.bonds.size());
  CHist cnow;
  forces(md, s.x.data(), s.q.data(), s.v.data(), s.w.data(), mu.data(), field, n,
         (bonds ? T_BOND : 0) | (contacts ? T_CONTACT : 0), Ft.data(), Tt.data(), (T*)nullptr,
         nullptr, bonds ? hnow.data() : nullptr, nullptr, contacts ? &cnow : nullptr);
  if (bonds) {
    s.hist.swap(hnow);
    s.hist_valid = true;
  }
  if (contacts) {
    s.chist.swap(cnow);
    s.chist_valid = true;
  }
}

// One velocity-Verlet step n -> n+1 (SI "Equations of motion").
template <class T>
void step(const Model& md, State<T>& s, const T* mbody, const T* field) {
  const double dt = md.dt;
  const int64_t n1 = s.step + 1;
  for (int p = 0; p < md.n; ++p) {
    if (md.bc[p] != 0) continue;  // clamped and driven particles are not integrated
    T im(1.0 / md.mass[p]), iI(1.0 / md.inertia[p]);
    V3<T> vh = ld3(s.v.data(), p) + (T(0.5 * dt) * im) * ld3(s.F.data(), p);
    V3<T> xn = ld3(s.x.data(), p) + T(dt) * vh;
    V3<T> wh = ld3(s.w.data(), p) + (T(0.5 * dt) * iI) * ld3(s.Tq.data(), p);
    Q4<T> qn = richardson(ld4(s.q.data(), p), wh, dt);
    st3(s.v.data(), p, vh);
    st3(s.x.data(), p, xn);
    st3(s.w.data(), p, wh);
    st4(s.q.data(), p, qn);
  }
  apply_drive(md, s, n1);
  eval_forces(md, s, mbody, field, n1);  // forces at t + dt, damping with v(t+dt/2)
  for (int p = 0; p < md.n; ++p) {
    if (md.bc[p] != 0) continue;
    T im(1.0 / md.mass[p]), iI(1.0 / md.inertia[p]);
    st3(s.v.data(), p, ld3(s.v.data(), p) + (T(0.5 * dt) * im) * ld3(s.F.data(), p));
    st3(s.w.data(), p, ld3(s.w.data(), p) + (T(0.5 * dt) * iI) * ld3(s.Tq.data(), p));
  }
  s.step = n1;
}

// Prepare a state from raw inputs: normalise q, impose boundary conditions of
// time level `step`, and evaluate the forces of that level.
template <class T>
void prepare(const Model& md, State<T>& s, const T* mbody, const T* field) {
  for (int p = 0; p < md.n; ++p) {
    st4(s.q.data(), p, qnormalize(ld4(s.q.data(), p)));
    if (md.bc[p] != 0) {
      st3(s.v.data(), p, V3<T>{T(0.0), T(0.0), T(0.0)});
      st3(s.w.data(), p, V3<T>{T(0.0), T(0.0), T(0.0)});
    }
  }
  apply_drive(md, s, s.step);
  s.hist_valid = false;   // the first evaluation seeds the bond damping measures
  s.chist_valid = false;  // and the Hertz-Mindlin contacts
  eval_forces(md, s, mbody, field, s.step);
}

}  // namespace orc

using namespace orc;

// ---------------------------------------------------------------- C entry points
extern "C" {

// Bond list of the topology: pairs (i, j), reference vectors and K_r, K_s, K_t, K_b.
int orc_bonds(const orc_system* s, int32_t* ij, double* rref, double* K, int cap) {
  Model md = build_model(s);
  int B = (int)md.bonds.size();
  for (int k = 0; k < B && k < cap; ++k) {
    const Bond& b = md.bonds[k];
    ij[2 * k] = b.i; ij[2 * k + 1] = b.j;
    rref[3 * k] = b.rref.x; rref[3 * k + 1] = b.rref.y; rref[3 * k + 2] = b.rref.z;
    K[4 * k] = b.Kr; K[4 * k + 1] = b.Ks; K[4 * k + 2] = b.Kt; K[4 * k + 3] = b.Kb;
  }
  return B;
}

// Mass and moment of inertia per particle.
void orc_mass(const orc_system* s, double* mass, double* inertia) {
  Model md = build_model(s);
  for (int p = 0; p < md.n; ++p) { mass[p] = md.mass[p]; inertia[p] = md.inertia[p]; }
}

// One bond in isolation (for closed-form and invariant tests).
void orc_bond_single(const double* x1, const double* x2, const double* q1, const double* q2,
                     const double* rref, const double* K, double* F, double* Ts, double* Tbt,
                     double* e) {
  Bond b;
  b.i = 0; b.j = 1;
  b.rref = {rref[0], rref[1], rref[2]};
  b.Kr = K[0]; b.Ks = K[1]; b.Kt = K[2]; b.Kb = K[3];
  V3<double> f, ts, tbt;
  bond_eval(ld3(x1, 0), ld3(x2, 0), ld4(q1, 0), ld4(q2, 0), b, f, ts, tbt, e);
  st3(F, 0, f); st3(Ts, 0, ts); st3(Tbt, 0, tbt);
}

// One Hertz-Mindlin contact in isolation (for closed-form tests): positions,
// velocities and spins of i and j, the previous tangential displacement (null:
// a new contact); returns the force and torque on i and the new displacement.
void orc_hm_single(const orc_system* s, const double* xi, const double* xj, const double* vi,
                   const double* vj, const double* wi, const double* wj, const double* sprev,
                   double* F, double* Tq, double* snew, double* e) {
  Model md = build_model(s);
  V3<double> f, t, sn, sp;
  if (sprev) sp = ld3(sprev, 0);
  hertz_mindlin(md, ld3(xi, 0), ld3(xj, 0), ld3(vi, 0), ld3(vj, 0), ld3(wi, 0), ld3(wj, 0),
                sprev ? &sp : nullptr, f, t, sn, *e);
  st3(F, 0, f); st3(Tq, 0, t); st3(snew, 0, sn);
}

// Force and torque of the selected terms (bitmask: 1 bond, 2 dipole, 4 Zeeman,
// 8 contact, 16 damping, 32 external) at the state given, field index n.
// Bdip (nullable) receives the dipole field at each particle.
// hprev / hnow (nullable): bond damping measures [B][5] of the previous level
// and of this one.
void orc_forces(const orc_system* s, const double* x, const double* q, const double* v,
                const double* w, const double* mbody, const double* field, int64_t n,
                int32_t mask, double* F, double* Tq, double* Bdip, const double* hprev,
                double* hnow) {
  Model md = build_model(s);
  std::vector<double> mu;
  dipoles(md, q, mbody, mu);
  forces(md, x, q, v, w, mu.data(), field, n, mask, F, Tq, Bdip, hprev, hnow);
}

// Energies per member, 9 terms: stretch, shear, twist, bend (eq:total-energy),
// Zeeman -m.B, dipole-dipole, contact (Hookean 1/2 k (r_c - r)^2, or the
// normal Hertz energy; the tangential springs are not counted), translational
// and rotational kinetic energy.
void orc_energy(const orc_system* s, const double* x, const double* q, const double* v,
                const double* w, const double* mbody, const double* field, int64_t n,
                double* out) {
  Model md = build_model(s);
  for (int k = 0; k < 9 * md.M; ++k) out[k] = 0.0;
  for (const Bond& bd : md.bonds) {
    V3<double> f, ts, tbt;
    double e[4];
    bond_eval(ld3(x, bd.i), ld3(x, bd.j), ld4(q, bd.i), ld4(q, bd.j), bd, f, ts, tbt, e);
    for (int t = 0; t < 4; ++t) out[9 * md.member_of[bd.i] + t] += e[t];
  }
  std::vector<double> mu;
  dipoles(md, q, mbody, mu);
  for (int p = 0; p < md.n; ++p) {
    int mem = md.member_of[p];
    Field<double> f = field_at(md, field, n, mem);
    out[9 * mem + 4] -= dot(ld3(mu.data(), p), field_B(f, ld3(x, p)));
    out[9 * mem + 7] += 0.5 * md.mass[p] * dot(ld3(v, p), ld3(v, p));
    out[9 * mem + 8] += 0.5 * md.inertia[p] * dot(ld3(w, p), ld3(w, p));
  }
  if (md.dipole_on && md.periodic) {  // Ewald energy of each member's periodic system
    std::vector<double> Fe(3 * md.n, 0.0), Be(3 * md.n, 0.0), Ue(md.M, 0.0);
    ewald_dipoles(md, x, mu.data(), Fe.data(), Be.data(), Ue.data());
    for (int mem = 0; mem < md.M; ++mem) out[9 * mem + 5] += Ue[mem];
  }
  for (int i = 0; i < md.n; ++i) {
    int mem = md.member_of[i];
    for (int j = i + 1; j < md.member_end[mem]; ++j) {
      V3<double> r = ld3(x, i) - ld3(x, j);
      if (md.dipole_on && !md.periodic &&
          (md.dcut == 0.0 || (r.x * r.x + r.y * r.y) + r.z * r.z < md.dcut * md.dcut)) {
        double rr = norm(r);
        V3<double> rh = (1.0 / rr) * r;
        V3<double> mi = ld3(mu.data(), i), mj = ld3(mu.data(), j);
        out[9 * mem + 5] += md.C / (rr * rr * rr) * (dot(mi, mj) - 3.0 * dot(mi, rh) * dot(mj, rh));
      }
      if (md.contact_on && !excluded(md, i, j)) {
        double r2 = (r.x * r.x + r.y * r.y) + r.z * r.z;
        if (r2 < md.rc * md.rc) {
          double ov = md.rc - std::sqrt(r2);
          if (md.contact_model == 1) {  // Hertz: 8/15 E* sqrt(R*) delta^(5/2)
            const double Es = md.hmE / (2.0 * (1.0 - md.hmNu * md.hmNu));
            out[9 * mem + 6] += 8.0 / 15.0 * Es * std::sqrt(0.25 * md.rc) * ov * ov * std::sqrt(ov);
          } else {
            out[9 * mem + 6] += 0.5 * md.kc * ov * ov;
          }
        }
      }
    }
  }
}

// Contact pairs (i < j) by brute force over all pairs; returns the count and
// writes at most `cap` pairs.
int orc_contact_pairs(const orc_system* s, const double* x, int32_t* pairs, int cap) {
  Model md = build_model(s);
  const double rc2 = md.rc * md.rc;
  int cnt = 0;
  for (int i = 0; i < md.n; ++i)
    for (int j = i + 1; j < md.n; ++j) {
      if (excluded(md, i, j)) continue;
      V3<double> d = ld3(x, i) - ld3(x, j);
      double r2 = (d.x * d.x + d.y * d.y) + d.z * d.z;
      if (r2 < rc2) {
        if (cnt < cap) { pairs[2 * cnt] = i; pairs[2 * cnt + 1] = j; }
        ++cnt;
      }
    }
  return cnt;
}

// Prepare the initial state (normalise q, boundary conditions, forces of level
// `step`) and advance it by nsteps. Arrays are AoS and updated in place;
// F and Tq receive the forces of the final level.
// hist (nullable, [B][5]): bond damping measures of the last evaluation,
// written at the end; read when continuing a prepared state with hist_in set
// (without it the continued state's own measures are recorded first).
// hc_cnt [N], hc_j [N][hc_cap], hc_s [N][hc_cap][3] (nullable): the
// Hertz-Mindlin contacts of the last evaluation (partner, tangential
// displacement), written at the end and read when continuing with hc_in set, so
// that a run cut in pieces keeps its tangential springs. Returns 0, or -1 when a
// particle has more than hc_cap contacts to write.
int orc_run(const orc_system* s, double* x, double* v, double* q, double* w, double* F,
            double* Tq, const double* mbody, const double* field, int64_t step0,
            int64_t nsteps, int32_t prepared, double* hist, int32_t hist_in, int32_t* hc_cnt,
            int32_t* hc_j, double* hc_s, int32_t hc_cap, int32_t hc_in) {
  Model md = build_model(s);
  State<double> st;
  st.x.assign(x, x + 3 * md.n); st.v.assign(v, v + 3 * md.n);
  st.q.assign(q, q + 4 * md.n); st.w.assign(w, w + 3 * md.n);
  st.F.assign(3 * md.n, 0.0); st.Tq.assign(3 * md.n, 0.0);
  st.step = step0;
  const size_t HB = 5 * md.bonds.size();
  if (prepared) {
    st.F.assign(F, F + 3 * md.n); st.Tq.assign(Tq, Tq + 3 * md.n);
    const bool have = md.bond_damp && hist && hist_in;
    if (have) {
      st.hist.assign(hist, hist + HB);
      st.hist_valid = true;
    }
    bool hm = md.contact_on && md.contact_model == 1;
    if (hm && hc_cnt && hc_in) {  // the contacts as the previous piece left them
      st.chist.assign(md.n, {});
      for (int i = 0; i < md.n; ++i)
        for (int k = 0; k < hc_cnt[i]; ++k) {
          const int64_t e = (int64_t)i * hc_cap + k;
          st.chist[i].push_back(CEntry{hc_j[e], V3<double>{hc_s[3 * e], hc_s[3 * e + 1], hc_s[3 * e + 2]}});
        }
      st.chist_valid = true;
      hm = false;
    }
    if ((md.bond_damp && !have) || hm)
      record_measures(md, st, mbody, field, step0, md.bond_damp && !have, hm);
  } else {
    prepare(md, st, mbody, field);
  }
  for (int64_t k = 0; k < nsteps; ++k) step(md, st, mbody, field);
  if (md.bond_damp && hist && st.hist.size() == HB) std::copy(st.hist.begin(), st.hist.end(), hist);
  if (hc_cnt && st.chist_valid && (int)st.chist.size() == md.n) {
    for (int i = 0; i < md.n; ++i) {
      if ((int)st.chist[i].size() > hc_cap) return -1;
      hc_cnt[i] = (int32_t)st.chist[i].size();
      for (int k = 0; k < hc_cnt[i]; ++k) {
        const int64_t e = (int64_t)i * hc_cap + k;
        hc_j[e] = st.chist[i][k].j;
        hc_s[3 * e] = st.chist[i][k].s.x; hc_s[3 * e + 1] = st.chist[i][k].s.y; hc_s[3 * e + 2] = st.chist[i][k].s.z;
      }
    }
  }
  std::copy(st.x.begin(), st.x.end(), x); std::copy(st.v.begin(), st.v.end(), v);
  std::copy(st.q.begin(), st.q.end(), q); std::copy(st.w.begin(), st.w.end(), w);
  std::copy(st.F.begin(), st.F.end(), F); std::copy(st.Tq.begin(), st.Tq.end(), Tq);
  return 0;
}

// Forward-mode directional derivative of a whole run. Inputs are the raw
// initial state, body dipoles and field table with their tangents (d*); the
// run starts from `prepare` (q0 normalised first). Outputs: the final state
// (x, v, q, w) and its tangent.
void orc_run_jvp(const orc_system* s, const double* x0, const double* v0, const double* q0,
                 const double* w0, const double* mbody, const double* field,
                 const double* dx0, const double* dv0, const double* dq0, const double* dw0,
                 const double* dmbody, const double* dfield, int64_t step0, int64_t nsteps,
                 double* xT, double* vT, double* qT, double* wT,
                 double* dxT, double* dvT, double* dqT, double* dwT) {
  Model md = build_model(s);
  const int N = md.n;
  const int64_t FL = (int64_t)md.field_len * md.M * 12;
  auto mk = [](const double* a, const double* da, int64_t len) {
    std::vector<Dual> r(len);
    for (int64_t k = 0; k < len; ++k) r[k] = Dual(a[k], da ? da[k] : 0.0);
    return r;
  };
  State<Dual> st;
  st.x = mk(x0, dx0, 3 * N); st.v = mk(v0, dv0, 3 * N);
  st.q = mk(q0, dq0, 4 * N); st.w = mk(w0, dw0, 3 * N);
  st.F.assign(3 * N, Dual()); st.Tq.assign(3 * N, Dual());
  st.step = step0;
  std::vector<Dual> mb = mk(mbody, dmbody, 3 * N), fd = mk(field, dfield, FL);
  prepare(md, st, mb.data(), fd.data());
  for (int64_t k = 0; k < nsteps; ++k) step(md, st, mb.data(), fd.data());
  for (int k = 0; k < 3 * N; ++k) {
    xT[k] = st.x[k].v; dxT[k] = st.x[k].d;
    vT[k] = st.v[k].v; dvT[k] = st.v[k].d;
    wT[k] = st.w[k].v; dwT[k] = st.w[k].d;
  }
  for (int k = 0; k < 4 * N; ++k) { qT[k] = st.q[k].v; dqT[k] = st.q[k].d; }
}

// Dipole force, dipole field and contact force of selected particles only, by
// the same direct sums over their member (for spot checks of large systems).
void orc_rows(const orc_system* s, const double* x, const double* q, const double* mbody,
              const int32_t* rows, int32_t nrows, double* Fdip, double* Bdip, double* Fc) {
  Model md = build_model(s);
  std::vector<double> mu;
  dipoles(md, q, mbody, mu);
  const double C = md.C, rc2 = md.rc * md.rc;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < nrows; ++k) {
    const int i = rows[k];
    const int mem = md.member_of[i];
    V3<double> xi = ld3(x, i), mi = ld3(mu.data(), i);
    V3<double> Fi{0, 0, 0}, Bi{0, 0, 0}, Fci{0, 0, 0};
    for (int j = md.member_begin[mem]; j < md.member_end[mem]; ++j) {
      if (j == i) continue;
      V3<double> r = xi - ld3(x, j);
      if (md.dipole_on && (md.dcut == 0.0 || dot(r, r) < md.dcut * md.dcut)) {
        V3<double> mj = ld3(mu.data(), j);
        double r2 = dot(r, r);
        double rinv = 1.0 / std::sqrt(r2);
        double rinv3 = rinv * rinv * rinv, rinv5 = rinv3 * rinv * rinv;
        double a = dot(mi, r), b = dot(mj, r), cmm = dot(mi, mj);
        Fi = Fi + (3.0 * C * rinv5) * ((cmm * r + b * mi + a * mj) - (5.0 * a * b * rinv * rinv) * r);
        Bi = Bi + (3.0 * C * b * rinv5) * r - (C * rinv3) * mj;
      }
      if (md.contact_on && !excluded(md, i, j)) {
        double r2 = (r.x * r.x + r.y * r.y) + r.z * r.z;
        if (r2 < rc2) {
          double rr = std::sqrt(r2);
          Fci = Fci + (md.kc * (md.rc - rr) / rr) * r;
        }
      }
    }
    st3(Fdip, k, Fi); st3(Bdip, k, Bi); st3(Fc, k, Fci);
  }
}

// Quasi-static field ramp (the loading protocol of "Magnetized beams in
// non-uniform fields" and of the helical rods with dipole-dipole interactions):
// the field takes each of n_inc settings in turn ([n_inc][M][12], B0 and G per
// member); from the first force evaluation after it is set, the system steps
// with its damping, in chunks of check_every steps, until the kinetic energy
// of every member (translational plus rotational, summed in particle order)
// is at most ke_tol after a chunk, or max_steps have been taken (a negative
// ke_tol never counts as rest). Then the
// positions of the watched particles are recorded ([n_inc][n_watch][3]), with
// the steps taken and the kinetic energies ([n_inc][M]). The state arrays hold
// a prepared state on entry (its forces evaluated with the field before the
// ramp) and the final one on return; bond damping measures and Hertz-Mindlin
// contacts carry over from increment to increment.
void orc_ramp(const orc_system* s, double* x, double* v, double* q, double* w, double* F,
              double* Tq, const double* mbody, const double* fields, int32_t n_inc,
              int32_t max_steps, int32_t check_every, double ke_tol, int64_t step0,
              int32_t prepared, const int32_t* watch, int32_t n_watch, double* x_watch,
              int32_t* steps, double* ke) {
  Model md = build_model(s);
  const int64_t FM = (int64_t)md.M * 12;
  std::vector<double> field(fields, fields + FM);  // the setting in force
  State<double> st;
  st.x.assign(x, x + 3 * md.n); st.v.assign(v, v + 3 * md.n);
  st.q.assign(q, q + 4 * md.n); st.w.assign(w, w + 3 * md.n);
  st.F.assign(3 * md.n, 0.0); st.Tq.assign(3 * md.n, 0.0);
  st.step = step0;
  if (prepared) {
    st.F.assign(F, F + 3 * md.n); st.Tq.assign(Tq, Tq + 3 * md.n);
    const bool hm = md.contact_on && md.contact_model == 1;
    if (md.bond_damp || hm) record_measures(md, st, mbody, field.data(), step0, md.bond_damp, hm);
  } else {
    prepare(md, st, mbody, field.data());
  }
  for (int32_t k = 0; k < n_inc; ++k) {
    std::copy(fields + k * FM, fields + (k + 1) * FM, field.begin());
    int32_t taken = 0;
    std::vector<double> e(md.M, 0.0);
    while (taken < max_steps) {
      const int32_t chunk = std::min(check_every, max_steps - taken);
      for (int32_t t = 0; t < chunk; ++t) step(md, st, mbody, field.data());
      taken += chunk;
      std::fill(e.begin(), e.end(), 0.0);
      for (int p = 0; p < md.n; ++p)
        e[md.member_of[p]] += 0.5 * md.mass[p] * dot(ld3(st.v.data(), p), ld3(st.v.data(), p)) +
                              0.5 * md.inertia[p] * dot(ld3(st.w.data(), p), ld3(st.w.data(), p));
      bool rest = true;
      for (int m = 0; m < md.M; ++m) rest = rest && e[m] <= ke_tol;
      if (rest) break;
    }
    if (steps) steps[k] = taken;
    if (ke) std::copy(e.begin(), e.end(), ke + (int64_t)k * md.M);
    for (int32_t a = 0; a < n_watch; ++a)
      for (int c = 0; c < 3; ++c) x_watch[((int64_t)k * n_watch + a) * 3 + c] = st.x[3 * watch[a] + c];
  }
  std::copy(st.x.begin(), st.x.end(), x); std::copy(st.v.begin(), st.v.end(), v);
  std::copy(st.q.begin(), st.q.end(), q); std::copy(st.w.begin(), st.w.end(), w);
  std::copy(st.F.begin(), st.F.end(), F); std::copy(st.Tq.begin(), st.Tq.end(), Tq);
}

// Threads the OpenMP loops of this library use.
// Threads of the parallel loops from now on (n >= 1), for timing the oracle on
// a given number of host cores.
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
