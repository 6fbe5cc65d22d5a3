"""Pins of the FP64 oracle against what the paper and the mathematics fix.

CPU only. Each test names the passage it relies on. None of these tests
compares the oracle with itself: closed forms, invariants, an independent
rotation-matrix derivation of the bond, Euler-Bernoulli beam limits, the
paper's printed cantilever energy error, finite differences of independently
coded energies, a k-d tree neighbour search, and integrator convergence orders.
"""
import os

import numpy as np
import pytest
from scipy.linalg import expm, logm
from scipy.spatial import cKDTree

import oracle
import workloads

RNG = np.random.default_rng(12345)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- helpers
def qaxis(axis, ang):
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    return np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * a])


def qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def rotmat(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def rand_quat(scale=1.0):
    return qaxis(RNG.normal(size=3), scale * RNG.uniform(-1, 1))


K4 = np.array([2.0, 3.0, 5.0, 7.0])  # K_r, K_s, K_t, K_b (distinct on purpose)
ID = np.array([1.0, 0, 0, 0])


def rel(a, b):
    return np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300)


def single_rod(n, spacing=1.0, d=1.0, rho=1.0, E=1.0, nu=0.5, axis=(1, 0, 0), **kw):
    x, off, mem = workloads.straight_rods([n], [(0, 0, 0)], axis, spacing=spacing)
    bc = np.zeros(n, np.int8)
    bc[0] = 1
    w = workloads._base(x, off, mem, [d, rho, E, nu], np.zeros((n, 3)), bc,
                        workloads._field_const(1, (0, 0, 0)), dipole_on=False,
                        contact_on=False)
    w.update(kw)
    return w


# ----------------------------------------------------------------- bond: closed forms
def test_bond_pure_stretch():
    """eq:bpm-fr and eq:total-energy: stretching by delta gives F1 = K_r delta r-hat."""
    L, dl = 1.3, 0.11
    for ax in (np.array([1.0, 0, 0]), np.array([0, 0, 1.0]), np.array([1.0, 2, -2]) / 3):
        F, Ts, Tbt, e = oracle.bond_single(np.zeros(3), (L + dl) * ax, ID, ID, L * ax, K4)
        np.testing.assert_allclose(F, K4[0] * dl * ax, atol=1e-14)
        np.testing.assert_allclose(Ts, 0, atol=1e-14)
        np.testing.assert_allclose(Tbt, 0, atol=1e-14)
        np.testing.assert_allclose(e, [0.5 * K4[0] * dl ** 2, 0, 0, 0], atol=1e-15)


def test_bond_pure_transverse():
    """eq:bpm-fst / eq:bpm-tst: a transverse offset s gives gamma = atan2(s, L),
    f_s = K_s r gamma s-hat, tau_s = 1/2 K_s r^2 gamma t-hat on both particles."""
    L = 1.0
    for s in (1e-6, 0.05, 0.4):
        x2 = np.array([L, s, 0.0])
        F, Ts, Tbt, e = oracle.bond_single(np.zeros(3), x2, ID, ID, [L, 0, 0], K4)
        r = np.hypot(L, s)
        g = np.arctan2(s, L)
        Fexp = K4[0] * (r - L) * x2 / r + K4[1] * g * np.array([-s, L, 0.0])
        np.testing.assert_allclose(F, Fexp, rtol=1e-13, atol=1e-18)
        np.testing.assert_allclose(Ts, [0, 0, 0.5 * K4[1] * r * r * g], rtol=1e-13)
        np.testing.assert_allclose(Tbt, 0, atol=1e-15)
        np.testing.assert_allclose(e, [0.5 * K4[0] * (r - L) ** 2, 0.5 * K4[1] * r * r * g * g, 0, 0],
                                   rtol=1e-12, atol=1e-30)


@pytest.mark.parametrize("psi", [1e-5, 0.3, 1.0, 3.0])
def test_bond_symmetric_twist(psi):
    """eq:bpm-tt: equal and opposite rotations about the bond axis give
    tau_t = K_t psi along the axis, no force."""
    F, Ts, Tbt, e = oracle.bond_single(np.zeros(3), [1.0, 0, 0], qaxis([1, 0, 0], -psi / 2),
                                       qaxis([1, 0, 0], psi / 2), [1.0, 0, 0], K4)
    np.testing.assert_allclose(Tbt, [K4[2] * psi, 0, 0], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(F, 0, atol=1e-14)
    np.testing.assert_allclose(Ts, 0, atol=1e-14)
    np.testing.assert_allclose(e[2], 0.5 * K4[2] * psi ** 2, rtol=1e-12)


def test_bond_twist_wraps_past_pi():
    """Shortest-arc central frame: the per-bond relative twist is taken in
    (-pi, pi], so a twist of pi + 0.2 acts as -(pi - 0.2)."""
    psi = np.pi + 0.2
    F, Ts, Tbt, e = oracle.bond_single(np.zeros(3), [1.0, 0, 0], qaxis([1, 0, 0], -psi / 2),
                                       qaxis([1, 0, 0], psi / 2), [1.0, 0, 0], K4)
    np.testing.assert_allclose(Tbt, [K4[2] * (psi - 2 * np.pi), 0, 0], rtol=1e-12)


@pytest.mark.parametrize("axis", [(0, 1, 0), (0, 0, 1), (0, 1, 1)])
@pytest.mark.parametrize("theta", [1e-5, 0.2, 1.2])
def test_bond_symmetric_bend(axis, theta):
    """eq:bpm-tb: equal and opposite rotations about an axis normal to the bond
    give tau_b = K_b theta about that axis, no force and no shear."""
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    F, Ts, Tbt, e = oracle.bond_single(np.zeros(3), [1.0, 0, 0], qaxis(a, -theta / 2),
                                       qaxis(a, theta / 2), [1.0, 0, 0], K4)
    np.testing.assert_allclose(Tbt, K4[3] * theta * a, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(F, 0, atol=1e-14)
    np.testing.assert_allclose(Ts, 0, atol=1e-14)
    np.testing.assert_allclose(e[3], 0.5 * K4[3] * theta ** 2, rtol=1e-12, atol=1e-14 * K4[3] * theta)


# ----------------------------------------------------------------- bond: invariants
def rand_bond_state(amp=0.3):
    rref = RNG.normal(size=3)
    rref *= RNG.uniform(0.8, 1.5) / np.linalg.norm(rref)
    x1 = RNG.normal(size=3)
    x2 = x1 + rref + amp * RNG.normal(size=3) * 0.3
    q1, q2 = rand_quat(amp), rand_quat(amp)
    return x1, x2, q1, q2, rref


def test_bond_zero_for_rigid_copies_of_reference():
    """SI null space of the stiffness matrix: any rigid motion of the reference
    bond gives zero force and torque."""
    for _ in range(20):
        rref = RNG.normal(size=3)
        Q = rand_quat(3.0)
        a = RNG.normal(size=3) * 5
        R = rotmat(Q)
        F, Ts, Tbt, e = oracle.bond_single(a, a + R @ rref, Q, Q, rref, K4)
        assert np.max(np.abs(np.concatenate([F, Ts, Tbt]))) < 1e-13
        assert np.max(np.abs(e)) < 1e-25


def test_bond_objectivity():
    """Rigid motion of the current state rotates every output with it."""
    for _ in range(20):
        x1, x2, q1, q2, rref = rand_bond_state()
        Q = rand_quat(3.0)
        R = rotmat(Q)
        a = RNG.normal(size=3)
        F, Ts, Tbt, e = oracle.bond_single(x1, x2, q1, q2, rref, K4)
        F2, Ts2, Tbt2, e2 = oracle.bond_single(R @ x1 + a, R @ x2 + a, qmul(Q, q1), qmul(Q, q2),
                                               rref, K4)
        np.testing.assert_allclose(F2, R @ F, atol=1e-12)
        np.testing.assert_allclose(Ts2, R @ Ts, atol=1e-12)
        np.testing.assert_allclose(Tbt2, R @ Tbt, atol=1e-12)
        np.testing.assert_allclose(e2, e, rtol=1e-10, atol=1e-14)


def test_bond_exchange_symmetry():
    """SI symmetric decomposition: exchanging particles 1 and 2 swaps their
    forces and torques."""
    for _ in range(20):
        x1, x2, q1, q2, rref = rand_bond_state()
        F, Ts, Tbt, e = oracle.bond_single(x1, x2, q1, q2, rref, K4)
        F2, Ts2, Tbt2, e2 = oracle.bond_single(x2, x1, q2, q1, -rref, K4)
        np.testing.assert_allclose(F2, -F, atol=1e-12)
        np.testing.assert_allclose(Ts2, Ts, atol=1e-12)
        np.testing.assert_allclose(Tbt2, -Tbt, atol=1e-12)
        np.testing.assert_allclose(e2, e, rtol=1e-10, atol=1e-14)


def test_bond_newton_and_angular_momentum():
    """eq:bpm-vector with eq:bpm-tst: zero net force and zero net torque about
    the origin (tau_s = 1/2 r_f x f_s balances the moment of the force pair)."""
    for _ in range(20):
        x1, x2, q1, q2, rref = rand_bond_state()
        F, Ts, Tbt, _ = oracle.bond_single(x1, x2, q1, q2, rref, K4)
        L = (Ts + Tbt) + (Ts - Tbt) + np.cross(x1, F) + np.cross(x2, -F)
        assert np.max(np.abs(L)) < 1e-12 * max(1.0, np.max(np.abs(F)) * np.linalg.norm(x1))


def _shortest_rot(a, b):
    """Rotation matrix of the shortest arc taking unit a onto unit b (Rodrigues)."""
    v = np.cross(a, b)
    s = np.linalg.norm(v)
    c = np.dot(a, b)
    if s < 1e-300:
        return np.eye(3)
    k = v / s
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    ang = np.arctan2(s, c)
    return np.eye(3) + np.sin(ang) * Kx + (1 - np.cos(ang)) * Kx @ Kx


def _swing_twist_bend_first(A):
    """A = T S with T about z and S a swing (axis normal to z): S^T is the
    shortest arc from z to A^T z."""
    z = np.array([0, 0, 1.0])
    S = _shortest_rot(z, A.T @ z).T
    return A @ S.T, S


def _axis_angle_vec(R):
    W = logm(R).real
    return np.array([W[2, 1], W[0, 2], W[1, 0]])


def bond_by_matrices(x1, x2, q1, q2, rref, K):
    """The bond model re-derived with rotation matrices, the paper's literal
    arccos / unit-vector forms and library matrix exp/log."""
    Kr, Ks, Kt, Kb = K
    R1, R2 = rotmat(q1), rotmat(q2)
    RC = R1 @ expm(0.5 * logm(R1.T @ R2).real)      # geodesic midpoint
    rho = RC.T @ (x2 - x1)
    r = np.linalg.norm(rho)
    rh = rho / r
    r0 = np.linalg.norm(rref)
    rih = rref / r0
    fr = Kr * (r - r0) * rh
    gamma = np.arccos(np.clip(np.dot(rih, rh), -1, 1))
    t = np.cross(rih, rh)
    t /= np.linalg.norm(t)
    s = np.cross(t, rh)
    fs = Ks * r * gamma * s
    ts = 0.5 * np.cross(rho, fs)                     # first form of eq:bpm-tst
    RM = _shortest_rot(np.array([0, 0, 1.0]), rh)
    U = RM.T @ (RC.T @ R2) @ RM
    T2, S2 = _swing_twist_bend_first(U)
    T1, S1 = _swing_twist_bend_first(U.T)
    psi = np.arctan2(T2[1, 0], T2[0, 0]) - np.arctan2(T1[1, 0], T1[0, 0])
    th = _axis_angle_vec(S2 @ S1.T)
    tbt = Kb * th + Kt * psi * np.array([0, 0, 1.0])
    return RC @ (fr + fs), RC @ ts, RC @ RM @ tbt


def test_bond_matches_rotation_matrix_derivation():
    """An independent matrix formulation of the whole bond agrees."""
    for _ in range(25):
        x1, x2, q1, q2, rref = rand_bond_state(0.6)
        F, Ts, Tbt, _ = oracle.bond_single(x1, x2, q1, q2, rref, K4)
        F2, Ts2, Tbt2 = bond_by_matrices(x1, x2, q1, q2, rref, K4)
        scale = max(np.max(np.abs(np.concatenate([F, Ts, Tbt]))), 1e-3)
        assert np.max(np.abs(F - F2)) < 1e-10 * scale
        assert np.max(np.abs(Ts - Ts2)) < 1e-10 * scale
        assert np.max(np.abs(Tbt - Tbt2)) < 1e-10 * scale


# ----------------------------------------------------------------- Euler-Bernoulli limits
def _EI(d=1.0, E=1.0):
    return E * np.pi * d ** 4 / 64


def test_eb_static_residual_tip_load():
    """SI eq:beam-stiffness-matrix / eq:bpm-general-planar: the linearised chain
    is the cubic-Hermite beam, which is nodally exact for a tip load. On the
    exact deflection and slope of P x^2 (3L - x) / (6EI), interior particles are
    in equilibrium and the tip bond pulls back with -P."""
    n, l = 11, 1.0
    Lt = (n - 1) * l
    w = single_rod(n, spacing=l)
    EI = _EI()
    P = 1e-8
    xs = np.arange(n) * l
    y = P * xs ** 2 * (3 * Lt - xs) / (6 * EI)
    slope = P * (6 * Lt * xs - 3 * xs ** 2) / (6 * EI)
    # keep every bond at its reference length (no second-order stretch)
    xa = np.concatenate([[0.0], np.cumsum(np.sqrt(l * l - np.diff(y) ** 2))])
    x = np.stack([xa, y, np.zeros(n)], 1)
    q = np.array([qaxis([0, 0, 1], np.arctan(s)) for s in slope])
    F, T = oracle.forces(w, x, q, mask=oracle.BOND)
    # bending degrees of freedom (transverse force, torque about z): exact up
    # to O(P^2); the axial force is the shear force projected by the slope.
    assert np.max(np.abs(F[1:-1, 1])) < 1e-6 * P
    assert np.max(np.abs(T[1:-1, 2])) < 1e-6 * P * l
    np.testing.assert_allclose(F[-1, 1], -P, rtol=1e-6)
    assert abs(T[-1, 2]) < 1e-6 * P * l
    assert np.max(np.abs(F[:, 0])) < 2 * np.max(np.abs(slope)) * P
    assert np.max(np.abs(F[:, 2])) + np.max(np.abs(T[:, :2])) < 1e-6 * P


def test_eb_axial_and_torsion_static():
    """Axial tip force stretches each bond by P/K_r (K_r = EA/L); a tip torque
    twists each bond by T/K_t (K_t = GJ/L, G = E / (2 (1 + nu)))."""
    n, l, d, E, nu = 8, 1.0, 1.0, 1.0, 0.5
    w = single_rod(n, spacing=l, d=d, E=E, nu=nu)
    A = np.pi * d * d / 4
    J = np.pi * d ** 4 / 32
    G = E / (2 * (1 + nu))
    P, Tt = 1e-3, 1e-3
    xs = np.arange(n) * l * (1 + P / (E * A))
    x = np.stack([xs, np.zeros(n), np.zeros(n)], 1)
    q = np.tile(ID, (n, 1))
    F, T = oracle.forces(w, x, q, mask=oracle.BOND)
    assert np.max(np.abs(F[1:-1])) < 1e-15
    np.testing.assert_allclose(F[-1], [-P, 0, 0], rtol=1e-12, atol=1e-18)
    x = np.stack([np.arange(n) * l, np.zeros(n), np.zeros(n)], 1)
    q = np.array([qaxis([1, 0, 0], k * Tt * l / (G * J)) for k in range(n)])
    F, T = oracle.forces(w, x, q, mask=oracle.BOND)
    assert np.max(np.abs(T[1:-1])) < 1e-15
    np.testing.assert_allclose(T[-1], [-Tt, 0, 0], rtol=1e-12, atol=1e-18)


@pytest.mark.slow
def test_eb_cantilever_tip_load_damped_to_rest():
    """SI static cantilever: damped dynamics under a small tip load settle on the
    nodal Euler-Bernoulli deflection P x^2 (3L - x) / (6EI) (nodal exactness)."""
    for nb in (4, 10):
        Lt = 10.0
        w = single_rod(nb + 1, spacing=Lt / nb, damping=0.02, dt=0.1)
        EI = _EI()
        P = 1e-4 * 3 * EI / Lt ** 2
        ef = np.zeros((nb + 1, 3))
        ef[-1, 1] = P
        w["ext_force"] = ef
        st = oracle.run(w, 40000)
        xs = np.arange(nb + 1) * Lt / nb
        y = P * xs ** 2 * (3 * Lt - xs) / (6 * EI)
        np.testing.assert_allclose(st["x"][:, 1], y, rtol=1e-6, atol=1e-12)


@pytest.mark.slow
def test_eb_magnetic_cantilever_small_field():
    """Zeeman torque m x B with m rotating with the particle (Methods; magnetised
    beams): a weak field normal to an axially magnetised cantilever loads each
    free node with the moment mu = m B, and the tip deflects by
    sum_k mu x_k (2L - x_k) / (2EI)."""
    nb, Lt, m, B = 10, 10.0, 1e-3, 1e-2
    w = single_rod(nb + 1, spacing=Lt / nb, damping=0.02, dt=0.1)
    w["m_body"] = np.tile([m, 0, 0], (nb + 1, 1))
    w["field"] = workloads._field_const(1, (0, B, 0))
    st = oracle.run(w, 40000)
    EI = _EI()
    xs = np.arange(1, nb + 1) * Lt / nb
    tip = np.sum(m * B * xs * (2 * Lt - xs) / (2 * EI))
    np.testing.assert_allclose(st["x"][-1, 1], tip, rtol=1e-4)


@pytest.mark.slow
def test_printed_cantilever_energy_error():
    """SI static cantilever: with the tip load sized for a 10% tip deflection,
    the bond energy differs from P^2 L^3 / (6EI) by about 1.5% at N = 4 and
    does not decrease further (golden/cantilever_energy.txt)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "cantilever_energy.txt"))
    for nb, printed, lo, hi in rows:
        nb = int(nb)
        Lt, d = 100.0, 1.0
        w = single_rod(nb + 1, spacing=Lt / nb, d=d, damping=2e-3, dt=0.5)
        EI = _EI(d)
        P = 0.1 * Lt * 3 * EI / Lt ** 3
        ef = np.zeros((nb + 1, 3))
        ef[-1, 1] = P
        w["ext_force"] = ef
        st = oracle.run(w, 400000)
        U = oracle.energy(w, st["x"], st["q"])[0, :4].sum()
        err = abs(U / (P * P * Lt ** 3 / (6 * EI)) - 1)
        assert lo < err < hi, (nb, err, printed)


# ----------------------------------------------------------------- dipoles, Zeeman, contact
def two_particles(x2, m1, m2, B=(0, 0, 0), G=None, dip=True, contact=False, rods=2):
    x = np.array([[0.0, 0, 0], np.asarray(x2, float)])
    if rods == 2:
        off, mem = np.array([0, 1, 2], np.int32), np.array([0, 0], np.int32)
        params = [[1.0, 1.0, 1.0, 0.5]] * 2
    else:
        off, mem = np.array([0, 2], np.int32), np.array([0], np.int32)
        params = [[1.0, 1.0, 1.0, 0.5]]
    w = workloads._base(x, off, mem, params, np.array([m1, m2], float), np.zeros(2, np.int8),
                        workloads._field_const(1, B, G), dipole_on=dip, contact_on=contact)
    return w, x, np.tile(ID, (2, 1))


def test_dipole_pair_closed_forms():
    """Methods, dipole-dipole energy: coaxial, side-by-side and perpendicular pairs."""
    m, d = 0.7, 1.3
    # coaxial head-to-tail: attractive 6 m^2/d^4, U = -2 m^2/d^3
    w, x, q = two_particles([d, 0, 0], [m, 0, 0], [m, 0, 0])
    F, T = oracle.forces(w, x, q, mask=oracle.DIPOLE)
    np.testing.assert_allclose(F[0], [6 * m * m / d ** 4, 0, 0], rtol=1e-14)
    np.testing.assert_allclose(F[1], -F[0], rtol=1e-14)
    np.testing.assert_allclose(T, 0, atol=1e-16)
    np.testing.assert_allclose(oracle.energy(w, x, q)[0, 5], -2 * m * m / d ** 3, rtol=1e-14)
    # side by side: repulsive 3 m^2/d^4, U = +m^2/d^3
    w, x, q = two_particles([0, d, 0], [m, 0, 0], [m, 0, 0])
    F, T = oracle.forces(w, x, q, mask=oracle.DIPOLE)
    np.testing.assert_allclose(F[0], [0, -3 * m * m / d ** 4, 0], rtol=1e-14)
    np.testing.assert_allclose(oracle.energy(w, x, q)[0, 5], m * m / d ** 3, rtol=1e-14)
    # perpendicular: m_i = m x, m_j = m y, r_ij = x_i - x_j = -d x (particle 0 at origin)
    w, x, q = two_particles([d, 0, 0], [m, 0, 0], [0, m, 0])
    F, T = oracle.forces(w, x, q, mask=oracle.DIPOLE)
    np.testing.assert_allclose(F[0], [0, -3 * m * m / d ** 4, 0], rtol=1e-14, atol=1e-18)
    np.testing.assert_allclose(T[0], [0, 0, -m * m / d ** 3], rtol=1e-14, atol=1e-18)
    np.testing.assert_allclose(T[1], [0, 0, -2 * m * m / d ** 3], rtol=1e-14, atol=1e-18)
    # total angular momentum balance: sum tau + x x F = 0 (tau_i != -tau_j)
    L = T.sum(0) + np.cross(x, F).sum(0)
    assert np.max(np.abs(L)) < 1e-15


def _cluster(n=6, seed=7, contact=False, B=(0, 0, 0), G=None):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 2.5, size=(n, 3))
    mb = rng.normal(size=(n, 3)) * 0.5
    off = np.arange(n + 1, dtype=np.int32)
    w = workloads._base(x, off, np.zeros(n, np.int32), [[1.0, 1, 1, 0.5]] * n, mb,
                        np.zeros(n, np.int8), workloads._field_const(1, B, G),
                        contact_on=contact, r_contact=1.2, k_contact=3.0)
    q = np.array([rand_quat(2.0) for _ in range(n)])
    return w, x, q


def _fd_check(w, x, q, mask, terms, h=1e-6):
    """Force = -dU/dx and torque.e = -dU/dphi (rotating particle p about e)."""
    F, T = oracle.forces(w, x, q, mask=mask)
    U = lambda xx, qq: oracle.energy(w, xx, qq)[0, terms].sum()
    n = x.shape[0]
    for p in range(n):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[p, a] += h
            xm[p, a] -= h
            fd = -(U(xp, q) - U(xm, q)) / (2 * h)
            assert abs(fd - F[p, a]) < 1e-7 * max(1.0, np.abs(F).max()), (p, a, fd, F[p, a])
            e = np.eye(3)[a]
            qp, qm = q.copy(), q.copy()
            qp[p] = qmul(qaxis(e, h), q[p])
            qm[p] = qmul(qaxis(e, -h), q[p])
            fd = -(U(x, qp) - U(x, qm)) / (2 * h)
            assert abs(fd - T[p, a]) < 1e-7 * max(1.0, np.abs(T).max()), (p, a, fd, T[p, a])


def test_dipole_force_torque_are_energy_derivatives():
    w, x, q = _cluster()
    _fd_check(w, x, q, oracle.DIPOLE, [5])


def test_zeeman_force_torque_are_energy_derivatives():
    """U = -m.B with B = B0 + G x: f = G^T m, tau = m x B."""
    G = np.array([[-0.5, 0.2, 0.0], [0.1, 1.0, 0.3], [0.0, -0.4, -0.5]])
    w, x, q = _cluster(B=(0.3, -0.7, 0.2), G=G)
    w["dipole_on"] = False
    _fd_check(w, x, q, oracle.ZEEMAN, [4])


def test_contact_force_is_energy_derivative_and_closed_form():
    w, x, q = _cluster(contact=True, seed=3)
    w["dipole_on"] = False
    assert len(oracle.contact_pairs(w, x)) > 0
    _fd_check(w, x, q, oracle.CONTACT, [6])
    w2, x2, q2 = two_particles([0.8, 0, 0], [0, 0, 0], [0, 0, 0], dip=False, contact=True)
    F, T = oracle.forces(w2, x2, q2, mask=oracle.CONTACT)
    np.testing.assert_allclose(F[0], [-10 * 0.2, 0, 0], rtol=1e-14)


def test_contact_pairs_match_kdtree_and_exclusions():
    """Brute-force pairs equal a k-d tree query, minus excluded same-rod pairs
    (|i - j| <= depth) and pairs of different members."""
    rng = np.random.default_rng(11)
    for depth in (0, 1, 3):
        lens = [7, 5, 9, 6]
        x = rng.uniform(0, 4.0, size=(sum(lens), 3))
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
        mem = np.array([0, 0, 1, 1], np.int32)
        n = x.shape[0]
        w = workloads._base(x, off, mem, [[1.0, 1, 1, 0.5]] * 4, np.zeros((n, 3)),
                            np.zeros(n, np.int8), workloads._field_const(2, (0, 0, 0)),
                            contact_on=True, r_contact=1.0, exclude_depth=depth)
        got = {tuple(p) for p in oracle.contact_pairs(w, x)}
        rod = np.repeat(np.arange(4), lens)
        member = mem[rod]
        exp = set()
        for i, j in cKDTree(x).query_pairs(1.0):
            i, j = min(i, j), max(i, j)
            if member[i] != member[j]:
                continue
            if rod[i] == rod[j] and j - i <= depth:
                continue
            exp.add((i, j))
        assert got == exp


# ----------------------------------------------------------------- integrator
def test_free_rotation_second_order():
    """SI equations of motion: the Richardson update of q under constant omega
    converges to exp(1/2 omega t) q0 with an error quadratic in dt."""
    om = np.array([0.3, -1.1, 0.7])
    errs = []
    for dt in (0.02, 0.01, 0.005):
        x = np.zeros((1, 3))
        w = workloads._base(x, np.array([0, 1], np.int32), np.array([0], np.int32),
                            [1.0, 1, 1, 0.5], np.zeros((1, 3)), np.zeros(1, np.int8),
                            workloads._field_const(1, (0, 0, 0)), damping=0.0, dt=dt,
                            dipole_on=False)
        w["w0"] = om[None, :].copy()
        q0 = rand_quat(2.0)
        w["q0"] = q0[None, :].copy()
        t = 2.0
        st = oracle.run(w, int(round(t / dt)))
        qe = qmul(qaxis(om, np.linalg.norm(om) * t), q0)
        qn = st["q"][0] * np.sign(np.dot(st["q"][0], qe))
        errs.append(np.linalg.norm(qn - qe))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_radial_bond_period():
    """Velocity Verlet of a free two-particle bond: relative stretch oscillates
    with omega = sqrt(2 K_r / m) (K_r = EA/L, m = rho pi d^3 / 6)."""
    w = single_rod(2, damping=0.0, dt=0.005, dipole_on=False)
    w["bc"] = np.zeros(2, np.int8)
    w["x0"] = w["x_ref"].copy()
    w["x0"][1, 0] += 1e-3
    Kr = 1.0 * np.pi / 4 / 1.0
    m = np.pi / 6
    om = np.sqrt(2 * Kr / m)
    period = 2 * np.pi / om
    nper = period / w["dt"]
    half = oracle.run(w, int(round(nper / 2)))
    full = oracle.run(w, int(round(nper)))
    s_half = half["x"][1, 0] - half["x"][0, 0] - 1
    s_full = full["x"][1, 0] - full["x"][0, 0] - 1
    np.testing.assert_allclose(s_half, -1e-3, rtol=2e-3)
    np.testing.assert_allclose(s_full, 1e-3, rtol=2e-3)


# ----------------------------------------------------------------- global damping, inertia
# SI "Equations of motion": a solid sphere of diameter d and density rho has
# m = rho pi d^3 / 6 and I = 2/5 m (d/2)^2. Methods "Damping" leaves the form of
# the global damping open; the reading taken is -c m v and -c I w evaluated with
# the half-step velocities when forces are computed (the first evaluation with
# v0, w0). The two constants are written out here, not taken from the oracle.
def _sphere(d, rho):
    m = rho * np.pi * d ** 3 / 6.0
    return m, 0.4 * m * (0.5 * d) ** 2


def _free_sphere(d, rho, **kw):
    w = workloads._base(np.zeros((1, 3)), np.array([0, 1], np.int32), np.array([0], np.int32),
                        [d, rho, 1.0, 0.5], np.zeros((1, 3)), np.zeros(1, np.int8),
                        workloads._field_const(1, (0, 0, 0)), dipole_on=False)
    w.update(kw)
    return w


@pytest.mark.parametrize("nst", [1, 2, 7, 60])
def test_global_damping_decay_closed_form(nst):
    """A force-free sphere under global damping c: the half-step velocity of
    velocity Verlet shrinks by exactly (1 - c dt) per step after a first
    factor (1 - c dt / 2), since each force evaluation sees the half-step
    velocity (-c m v and -c I w: the rate is c whatever the mass and inertia).
    So v_n = v0 (1 - c dt/2)^2 (1 - c dt)^(n-1), x_n = x0 + dt v0 (1 - c dt/2)
    sum_k (1 - c dt)^k, and the state's force and torque are -c m v_half and
    -c I w_half with m and I of the sphere."""
    d, rho, c, dt = 1.3, 2.1, 0.7, 0.01
    m, I = _sphere(d, rho)
    v0 = np.array([0.3, -0.2, 0.5])
    w0 = np.array([0.4, 0.1, -0.9])
    w = _free_sphere(d, rho, damping=c, dt=dt)
    w["v0"] = v0[None, :].copy()
    w["w0"] = w0[None, :].copy()
    st = oracle.run(w, nst)
    a, b = 1.0 - 0.5 * c * dt, 1.0 - c * dt
    half = a * b ** (nst - 1)  # v_half of the last step over v0
    np.testing.assert_allclose(st["v"][0], v0 * half * a, rtol=1e-13)
    np.testing.assert_allclose(st["w"][0], w0 * half * a, rtol=1e-13)
    disp = dt * a * sum(b ** k for k in range(nst))
    np.testing.assert_allclose(st["x"][0], v0 * disp, rtol=1e-13)
    np.testing.assert_allclose(st["F"][0], -c * m * v0 * half, rtol=1e-13)
    np.testing.assert_allclose(st["T"][0], -c * I * w0 * half, rtol=1e-13)


def test_sphere_mass_and_inertia_under_constant_load():
    """A constant external force and torque on a free sphere, no damping:
    velocity Verlet gives v_n = n dt F / m and w_n = n dt T / I exactly, with
    the solid-sphere m and I."""
    d, rho, dt, nst = 0.8, 3.0, 0.02, 25
    m, I = _sphere(d, rho)
    Fe, Te = np.array([0.2, -0.5, 0.1]), np.array([-0.03, 0.07, 0.02])
    w = _free_sphere(d, rho, damping=0.0, dt=dt)
    w["ext_force"] = Fe[None, :].copy()
    w["ext_torque"] = Te[None, :].copy()
    st = oracle.run(w, nst)
    np.testing.assert_allclose(st["v"][0], nst * dt * Fe / m, rtol=1e-12)
    np.testing.assert_allclose(st["w"][0], nst * dt * Te / I, rtol=1e-12)
    np.testing.assert_allclose(st["x"][0], 0.5 * (nst * dt) ** 2 * Fe / m, rtol=1e-12)


def test_twist_bond_period():
    """Two free spheres twisted symmetrically about their bond and released
    without damping: each carries -+K_t psi (P3), so the relative twist obeys
    psi'' = -2 K_t psi / I and oscillates with omega = sqrt(2 K_t / I),
    K_t = G J / L, G = E / (2 (1 + nu)), J = pi d^4 / 32 (eq:bpm-tt and the
    spring constants), I of the solid sphere."""
    d, rho, E, nu = 1.0, 1.0, 1.0, 0.5
    w = single_rod(2, d=d, rho=rho, E=E, nu=nu, damping=0.0, dt=0.005)
    w["bc"] = np.zeros(2, np.int8)
    psi0 = 1e-3
    w["x0"] = w["x_ref"].copy()
    w["q0"] = np.stack([qaxis([1, 0, 0], -psi0 / 2), qaxis([1, 0, 0], psi0 / 2)])
    Kt = E / (2 * (1 + nu)) * np.pi * d ** 4 / 32 / 1.0
    _, I = _sphere(d, rho)
    nper = 2 * np.pi / np.sqrt(2 * Kt / I) / w["dt"]

    def twist(st):
        r = qmul(np.array([1.0, -1, -1, -1]) * st["q"][0], st["q"][1])
        return 2 * np.arctan2(r[1], r[0])
    np.testing.assert_allclose(twist(oracle.run(w, int(round(nper / 2)))), -psi0, rtol=2e-3)
    np.testing.assert_allclose(twist(oracle.run(w, int(round(nper)))), psi0, rtol=2e-3)


def _total_energy(w, st):
    return oracle.energy(w, st["x"], st["q"], st["v"], st["w"], step=st["step"]).sum()


@pytest.mark.slow
def test_nve_conservative_subset_bounded():
    """Without bonds and damping, dipoles + static Zeeman + contact form a
    potential system: velocity Verlet keeps the total energy within a bounded
    O(dt^2) band with no secular drift."""
    rng = np.random.default_rng(5)
    g = np.stack(np.meshgrid(np.arange(3), np.arange(2), np.arange(4), indexing="ij"), -1)
    x = 1.3 * g.reshape(-1, 3) + rng.normal(0, 0.05, size=(24, 3))
    n = x.shape[0]
    off = np.arange(n + 1, dtype=np.int32)
    w = workloads._base(x, off, np.zeros(n, np.int32), [[1.0, 1, 1, 0.5]] * n,
                        rng.normal(size=(n, 3)) * 0.04, np.zeros(n, np.int8),
                        workloads._field_const(1, (0.2, 0.1, -0.3)), damping=0.0,
                        contact_on=True, exclude_depth=0)
    w["v0"] = rng.normal(0, 0.2, size=(n, 3))
    spans = []
    for dt in (0.002, 0.001):
        w["dt"] = dt
        st = None
        E = []
        for k in range(40):
            st = oracle.run(w, int(round(0.5 / dt)), state=st)
            E.append(_total_energy(w, st))
        E = np.array(E)
        E0 = _total_energy(w, oracle.run(w, 0))
        spans.append(np.max(np.abs(E - E0)))
        assert abs(E[-10:].mean() - E[:10].mean()) < 3 * spans[-1]
    assert 3.0 < spans[0] / spans[1] < 5.0, spans


def test_nve_full_bond_small_amplitude():
    """Forces are not exact gradients of eq:total-energy (Discussion), so NVE
    energy is only approximately conserved: bounded to 1e-3 relative over 1000
    steps at 1e-3 amplitude."""
    w = workloads.cantilever(n=12, m=0.0, B=(0, 0, 0), damping=0.0, seed=9)
    w["v0"] = np.random.default_rng(2).normal(size=(12, 3)) * 1e-3
    w["v0"][0] = 0
    st0 = oracle.run(w, 0)
    E0 = _total_energy(w, st0)
    st = oracle.run(w, 1000)
    assert abs(_total_energy(w, st) - E0) <= 1e-3 * abs(E0)


def test_clamped_and_driven_particles():
    """Clamped particles never move; driven particles follow R(axis, 2 pi n / P)."""
    w = workloads.twisted_rod(n=16, period=100, contact_on=False)
    st = oracle.run(w, 37)
    np.testing.assert_array_equal(st["x"][0], w["x0"][0])
    np.testing.assert_array_equal(st["x"][-1], w["x0"][-1])
    np.testing.assert_allclose(st["q"][-1], qaxis([1, 0, 0], 2 * np.pi * 37 / 100), atol=1e-15)
    np.testing.assert_array_equal(st["q"][0], ID)


# ----------------------------------------------------------------- JVP
def test_jvp_matches_central_differences():
    """The dual-number JVP of a whole run equals central differences of the run."""
    w = workloads.adjoint_rod(n=8, steps=30)
    rng = np.random.default_rng(3)
    tan = {k: rng.normal(size=np.shape(w[k])) for k in ("x0", "v0", "q0", "w0", "m_body")}
    tan["field"] = rng.normal(size=w["field"].shape)
    for k in ("x0", "v0", "q0", "w0"):
        tan[k][0] = 0.0
    nst = 30
    _, dT = oracle.run_jvp(w, nst, tan)
    h = 1e-6

    def shifted(sgn):
        w2 = dict(w)
        for k in ("x0", "v0", "q0", "w0", "m_body", "field"):
            w2[k] = w[k] + sgn * h * tan[k]
        return oracle.run(w2, nst)
    sp, sm = shifted(1), shifted(-1)
    for k in ("x", "v", "q", "w"):
        fd = (sp[k] - sm[k]) / (2 * h)
        assert rel(dT[k], fd) < 1e-6, k


# ----------------------------------------------------------------- bond damping
# Methods "Damping": f_r += g_r (dv . r_f-hat); f_s += g_s r_f gamma-dot (tau_s
# accordingly); tau_t += g_t psi-dot; tau_b += g_b theta-dot, the rates being
# finite differences of the stored measures between time levels.
G4 = np.array([0.3, 0.7, 1.1, 1.3])  # g_r, g_s, g_t, g_b (distinct on purpose)


def two_bond(x2, q1, q2, g=G4, v2=(0, 0, 0), dt=0.01):
    """Two free particles 1 (at the origin) and 2 (at x2), reference bond x-hat;
    returns the workload and the state arrays."""
    w = single_rod(2, dt=dt, damping=0.0, bond_damping=np.array([g], float))
    w["bc"] = np.zeros(2, np.int8)
    x = np.array([[0.0, 0, 0], np.asarray(x2, float)])
    q = np.array([q1, q2], float)
    v = np.array([[0.0, 0, 0], np.asarray(v2, float)])
    return w, x, q, v


def damped_minus_plain(w, x, q, v, hist):
    """Bond force and torque with damping minus without, and this level's measures."""
    Fd, Td, h = oracle.forces(w, x, q, v=v, mask=oracle.BOND, hist=hist, hist_out=True)
    w0 = dict(w)
    w0["bond_damping"] = None
    Fp, Tp = oracle.forces(w0, x, q, v=v, mask=oracle.BOND)
    return Fd - Fp, Td - Tp, h


@pytest.mark.parametrize("u", [0.37, -1.2])
def test_bond_damping_radial_dashpot(u):
    """Separating (or approaching) along the axis at relative speed u: particle 1
    is pulled by g_r u x-hat, particle 2 by the opposite; no torque. A relative
    velocity across the bond gives no radial term."""
    w, x, q, v = two_bond([1.1, 0, 0], ID, ID, v2=(u, 0, 0))
    _, _, h = oracle.forces(w, x, q, v=v, mask=oracle.BOND, hist_out=True)
    dF, dT, _ = damped_minus_plain(w, x, q, v, h)  # same measures: no angular rates
    np.testing.assert_allclose(dF[0], [G4[0] * u, 0, 0], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(dF[1], [-G4[0] * u, 0, 0], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(dT, 0.0, atol=1e-15)
    w, x, q, v = two_bond([1.1, 0, 0], ID, ID, v2=(0, u, 0.5 * u))
    dF, dT, _ = damped_minus_plain(w, x, q, v, h)
    np.testing.assert_allclose(dF, 0.0, atol=1e-15)


def test_bond_damping_shear_rate():
    """Pure transverse offset s (P2 geometry): the shear angle goes from
    gamma_a = atan(s_a / L) to gamma_b; the extra force on particle 1 is
    g_s gamma-dot (-s, L, 0) and the extra tau_s is 1/2 g_s r^2 gamma-dot z-hat on
    both particles."""
    L, sa, sb, dt = 1.0, 0.05, 0.08, 0.01
    wa, xa, qa, va = two_bond([L, sa, 0], ID, ID, dt=dt)
    _, _, ha = oracle.forces(wa, xa, qa, v=va, mask=oracle.BOND, hist_out=True)
    w, x, q, v = two_bond([L, sb, 0], ID, ID, dt=dt)
    dF, dT, hb = damped_minus_plain(w, x, q, v, ha)
    ga, gb = np.arctan2(sa, L), np.arctan2(sb, L)
    np.testing.assert_allclose([ha[0, 0], hb[0, 0]], [ga, gb], rtol=1e-14)
    gdot = (gb - ga) / dt
    r2 = L * L + sb * sb
    np.testing.assert_allclose(dF[0], G4[1] * gdot * np.array([-sb, L, 0]), rtol=1e-12)
    np.testing.assert_allclose(dF[1], -dF[0], rtol=1e-14)
    for p in (0, 1):
        np.testing.assert_allclose(dT[p], [0, 0, 0.5 * G4[1] * r2 * gdot], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("pa,pb", [(0.2, 0.25), (-0.4, -0.1), (3.0, -3.0)])
def test_bond_damping_twist_rate(pa, pb):
    """Symmetric twist (P3 geometry) from psi_a to psi_b: the extra torque on
    particle 1 is g_t psi-dot about the bond axis, psi-dot the change taken
    modulo 2 pi over dt (the last case crosses the wrap at pi)."""
    dt = 0.01
    wa, xa, qa, va = two_bond([1, 0, 0], qaxis([1, 0, 0], -pa / 2), qaxis([1, 0, 0], pa / 2), dt=dt)
    _, _, ha = oracle.forces(wa, xa, qa, v=va, mask=oracle.BOND, hist_out=True)
    w, x, q, v = two_bond([1, 0, 0], qaxis([1, 0, 0], -pb / 2), qaxis([1, 0, 0], pb / 2), dt=dt)
    dF, dT, hb = damped_minus_plain(w, x, q, v, ha)
    np.testing.assert_allclose([ha[0, 1], hb[0, 1]], [pa, pb], rtol=1e-13)
    dpsi = (pb - pa + np.pi) % (2 * np.pi) - np.pi
    np.testing.assert_allclose(dT[0], [G4[2] * dpsi / dt, 0, 0], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dT[1], -dT[0], rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(dF, 0.0, atol=1e-14)


@pytest.mark.parametrize("axis", [(0, 1, 0), (0, 0, 1), (0, 1, 1)])
def test_bond_damping_bend_rate(axis):
    """Symmetric bend (P4 geometry) from theta_a to theta_b about a transverse
    axis: the extra torque on particle 1 is g_b (theta_b - theta_a) / dt along
    that axis, the opposite on particle 2, and no force."""
    ta, tb, dt = 0.1, 0.13, 0.01
    ax = np.asarray(axis, float) / np.linalg.norm(axis)
    wa, xa, qa, va = two_bond([1, 0, 0], qaxis(ax, -ta / 2), qaxis(ax, ta / 2), dt=dt)
    _, _, ha = oracle.forces(wa, xa, qa, v=va, mask=oracle.BOND, hist_out=True)
    w, x, q, v = two_bond([1, 0, 0], qaxis(ax, -tb / 2), qaxis(ax, tb / 2), dt=dt)
    dF, dT, _ = damped_minus_plain(w, x, q, v, ha)
    np.testing.assert_allclose(dT[0], G4[3] * (tb - ta) / dt * ax, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(dT[1], -dT[0], rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(dF, 0.0, atol=1e-13)


def test_bond_damping_radial_oscillator_envelope():
    """Particle 0 clamped, particle 1 pulled out along the bond by delta and
    released, only radial damping: m x'' = -K_r x - g_r x', whose amplitude
    decays as exp(-g_r t / 2m) (textbook damped oscillator). The peaks over 4000
    steps follow it to 1e-3."""
    g = 0.05
    w = single_rod(2, damping=0.0, bond_damping=np.array([[g, 0, 0, 0]]))
    w["x0"] = w["x_ref"].copy()
    w["x0"][1, 0] += 0.01
    m = oracle.mass(w)[0][1]
    st, xs = None, []
    for _ in range(4000):
        st = oracle.run(w, 1, state=st)
        xs.append(st["x"][1, 0] - 1.0)
    xs = np.array(xs)
    t = w["dt"] * np.arange(1, len(xs) + 1)
    pk = [k for k in range(1, len(xs) - 1) if xs[k] > xs[k - 1] and xs[k] >= xs[k + 1]]
    assert len(pk) >= 3
    env = xs[pk] / xs[pk[0]]
    ref = np.exp(-g * (t[pk] - t[pk[0]]) / (2 * m))
    np.testing.assert_allclose(env, ref, rtol=1e-3)


def test_bond_damping_dissipates_and_plain_bonds_conserve():
    """A free-ended rod bent and twisted at rest by small amounts (the regime of
    the energy check of the plain bond model), no global damping: with bond
    damping its total energy falls (by more than a third over 1500 steps, never
    rising by more than the integrator's O(dt^2) wobble); without, every sample
    stays within 2e-3 of the start (the plain bond model conserves energy only
    approximately, see test_nve_full_bond_small_amplitude)."""
    def total(w, st):
        e = oracle.energy(w, st["x"], st["q"], v=st["v"], om=st["w"])
        return float(np.sum(e[:, [0, 1, 2, 3, 7, 8]]))
    base = single_rod(6, damping=0.0)
    rng = np.random.default_rng(3)
    base["x0"] = base["x_ref"] + 1e-3 * rng.normal(size=(6, 3)) * (base["bc"] == 0)[:, None]
    base["q0"] = np.array([qaxis(rng.normal(size=3), 5e-3) for _ in range(6)])
    out = {}
    for label, g in (("plain", None), ("damped", np.array([[0.2, 0.2, 0.2, 0.2]]))):
        w = dict(base)
        w["bond_damping"] = g
        st = oracle.run(w, 0)
        es = [total(w, st)]
        for _ in range(15):
            st = oracle.run(w, 100, state=st)
            es.append(total(w, st))
        out[label] = np.array(es)
    e = out["plain"]
    assert np.max(np.abs(e - e[0])) <= 2e-3 * e[0]
    e = out["damped"]
    assert e[-1] < e[0] * (2.0 / 3.0)
    assert np.all(np.diff(e) <= 1e-3 * e[0])


def test_bond_damping_continued_runs():
    """A damped run cut in two is the uncut run, whether the second part gets
    the measures the first left or records them from the state it is given
    (they are that state's own)."""
    w = single_rod(8, damping=0.0)
    rng = np.random.default_rng(11)
    w["x0"] = w["x_ref"] + 0.05 * rng.normal(size=(8, 3)) * (w["bc"] == 0)[:, None]
    w["q0"] = np.array([qaxis(rng.normal(size=3), 0.2) for _ in range(8)])
    w["v0"] = 0.1 * rng.normal(size=(8, 3)) * (w["bc"] == 0)[:, None]
    w["bond_damping"] = np.array([[0.4, 0.3, 0.2, 0.1]])
    whole = oracle.run(w, 20)
    half = oracle.run(w, 10)
    bare = {k: v for k, v in half.items() if k != "hist"}
    for st in (half, bare):
        cont = oracle.run(w, 10, state=st)
        assert cont["step"] == 20
        for k in ("x", "v", "q", "w", "F", "T"):
            np.testing.assert_array_equal(cont[k], whole[k])
    # with measures that are not the state's (all zero) the run differs
    zero = dict(half, hist=np.zeros_like(half["hist"]))
    assert np.max(np.abs(oracle.run(w, 10, state=zero)["x"] - whole["x"])) > 1e-6
