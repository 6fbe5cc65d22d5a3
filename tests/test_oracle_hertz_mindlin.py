"""Pins of the oracle's Hertz-Mindlin contact (Methods, "Contact") against
textbook contact mechanics of two equal elastic spheres:

- the Hertz normal force and energy, 4/3 E* sqrt(R*) delta^(3/2) and its
  integral, with E* = E / (2 (1 - nu^2)) and R* = r_c / 4;
- the duration of a head-on elastic Hertz impact, (2 delta_max / v) times
  2/5 B(2/5, 1/2), and its restitution (1 without damping, below 1 with it);
- Mindlin stick then Coulomb slip of a spinning sphere held against a clamped
  one: |F_t| = min(k_t L u dt + g_t u, mu F_n) at level L, k_t = 8 G* a;
- no tangential force under rolling without slip or rigid motion of a pair;
- exact conservation of linear and angular momentum in a frictional clump.
"""
import numpy as np
import pytest
from scipy.special import beta

import oracle
import workloads

CONTACT = 8


def spheres(xs, bc=None, hm=(10.0, 0.3, 0.5, 0.0, 0.0), dt=0.01, **kw):
    """Single-particle rods (d = 1, rho = 1) of one member, Hertz-Mindlin
    contact at r_c = 1, no dipoles, no field, no global damping."""
    xs = np.asarray(xs, float)
    n = len(xs)
    x, off, mem = workloads.straight_rods([1] * n, xs, (1, 0, 0))
    bc = np.zeros(n, np.int8) if bc is None else np.asarray(bc, np.int8)
    return workloads._base(x, off, mem, np.tile([1.0, 1.0, 1.0, 0.5], (n, 1)), np.zeros((n, 3)),
                           bc, workloads._field_const(1, (0, 0, 0)), dipole_on=False,
                           contact_on=True, contact_model="hertz_mindlin",
                           contact_hm=np.asarray(hm, float), damping=0.0, dt=dt, **kw)


def estar(E, nu):
    return E / (2.0 * (1.0 - nu * nu))


def gstar(E, nu):
    G = E / (2.0 * (1.0 + nu))
    return G / (2.0 * (2.0 - nu))


RS = 0.25  # R* of two spheres of diameter 1


@pytest.mark.parametrize("delta", [1e-3, 0.02, 0.1, 0.3])
def test_hertz_normal_force_and_energy(delta):
    E, nu = 7.0, 0.35
    rng = np.random.default_rng(int(delta * 1e4))
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    r = 1.0 - delta
    xs = [[0.2, -0.1, 0.3], np.array([0.2, -0.1, 0.3]) - r * n]
    w = spheres(xs, bc=[1, 1], hm=(E, nu, 0.5, 0.0, 0.0))
    q = np.tile([1.0, 0, 0, 0], (2, 1))
    F, T = oracle.forces(w, w["x0"], q, mask=CONTACT)
    d = w["x0"][0] - w["x0"][1]
    rr = np.linalg.norm(d)
    n, delta = d / rr, 1.0 - rr  # as placed, to rounding
    Fn = 4.0 / 3.0 * estar(E, nu) * np.sqrt(RS) * delta ** 1.5
    np.testing.assert_allclose(F[0], Fn * n, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(F[1], -Fn * n, rtol=1e-13, atol=1e-16)
    np.testing.assert_array_equal(T, 0.0)
    U = 8.0 / 15.0 * estar(E, nu) * np.sqrt(RS) * delta ** 2.5
    e = oracle.energy(w, w["x0"], q)
    assert abs(e[0, 6] - U) <= 1e-13 * U
    # the force is minus the derivative of that energy along the line of centres
    h = 1e-6 * max(delta, 1e-2)
    Ue = []
    for s in (+1, -1):
        xx = np.array(w["x0"]).copy()
        xx[1] = xx[0] - (r + s * h) * n
        Ue.append(oracle.energy(w, xx, q)[0, 6])
    assert abs(-(Ue[0] - Ue[1]) / (2 * h) - Fn) <= 1e-6 * Fn


def _collide(hm, u=0.1, dt=2e-4, gap=1e-3):
    """Two free spheres meeting head-on, each at speed u; returns (time in
    contact, speed of separation afterwards)."""
    w = spheres([[0, 0, 0], [1.0 + gap, 0, 0]], hm=hm, dt=dt)
    w["v0"] = np.array([[u, 0, 0], [-u, 0, 0]])
    st = oracle.run(w, 0)
    inside, seen = 0, False
    for _ in range(200000):
        st = oracle.run(w, 1, state=st)
        r = np.linalg.norm(st["x"][1] - st["x"][0])
        if r < 1.0:
            inside += 1
            seen = True
        elif seen:
            break
    return inside * dt, st["v"][1, 0] - st["v"][0, 0]  # speed of separation


def test_hertz_impact_duration_and_restitution():
    E, nu = 100.0, 0.5
    u = 0.1
    t, vout = _collide((E, nu, 0.5, 0.0, 0.0), u=u)
    v = 2 * u
    mstar = 0.5 * np.pi / 6.0
    dmax = (15.0 * mstar * v * v / (16.0 * estar(E, nu) * np.sqrt(RS))) ** 0.4
    tc = 2.0 * dmax / v * 0.4 * beta(0.4, 0.5)
    assert abs(t - tc) <= 3 * 2e-4 + 1e-3 * tc, (t, tc)
    assert abs(vout / v - 1.0) <= 1e-4
    # a normal dashpot takes energy out of the impact
    _, vd = _collide((E, nu, 0.5, 0.5, 0.0), u=u)
    assert 0.0 < vd < 0.99 * v


def test_mindlin_stick_then_coulomb_slip():
    """A driven sphere spinning about z at a fixed overlap with a clamped one:
    the contact point slides at u = (r/2) Omega along +y (seen from the driven
    sphere). The tangential displacement grows by u dt per level from zero, so
    |F_t| = k_t L u dt + g_t u until it reaches mu F_n, where it stays."""
    E, nu, mu, gt = 10.0, 0.3, 0.5, 0.01
    r, dt, P = 0.95, 0.01, 1000
    w = spheres([[0, 0, 0], [r, 0, 0]], bc=[2, 1], hm=(E, nu, mu, 0.0, gt), dt=dt,
                drive_axis=np.array([0.0, 0.0, 1.0]), drive_period=P)
    delta = 1.0 - r
    a = np.sqrt(RS * delta)
    Fn = 4.0 / 3.0 * estar(E, nu) * a * delta
    kt = 8.0 * gstar(E, nu) * a
    u = 0.5 * r * 2 * np.pi / (P * dt)
    capped = False
    for L in (0, 1, 3, 5, 6, 10, 50):
        st = oracle.run(w, L)
        ft = min(kt * L * u * dt + gt * u, mu * Fn)
        capped = capped or ft == mu * Fn
        F0 = np.array([-Fn, -ft, 0.0])
        np.testing.assert_allclose(st["F"][0], F0, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(st["F"][1], -F0, rtol=1e-12, atol=1e-15)
        Tz = np.array([0.0, 0.0, -0.5 * r * ft])
        np.testing.assert_allclose(st["T"][0], Tz, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(st["T"][1], Tz, rtol=1e-12, atol=1e-15)
    assert capped and kt * 3 * u * dt + gt * u < mu * Fn  # both regimes were seen


def test_no_tangential_force_without_slip():
    """Rolling without slip, rigid motion of the pair and a common velocity
    leave only the normal force (the contact-point velocities agree)."""
    rng = np.random.default_rng(4)
    E, nu = 10.0, 0.3
    hm = (E, nu, 0.8, 0.3, 0.7)
    for _ in range(5):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        r = 0.9
        c = rng.normal(size=3)
        xs = np.array([c + 0.5 * r * n, c - 0.5 * r * n])
        w = spheres(xs, hm=hm)
        q = np.tile([1.0, 0, 0, 0], (2, 1))
        Fn = 4.0 / 3.0 * estar(E, nu) * np.sqrt(RS * 0.1) * 0.1
        wi, wj = rng.normal(size=3), rng.normal(size=3)
        vj = rng.normal(size=3)
        cases = [
            # rolling: v_i - v_j = r/2 (w_i + w_j) x n, and no normal motion
            (np.array([vj + 0.5 * r * np.cross(wi + wj, n), vj]), np.array([wi, wj])),
        ]
        Om = rng.normal(size=3)
        vc = rng.normal(size=3)
        # rigid motion of the pair: v = vc + Om x (x - c), w = Om for both
        cases.append((np.array([vc + np.cross(Om, xs[0] - c), vc + np.cross(Om, xs[1] - c)]),
                      np.array([Om, Om])))
        for v, om in cases:
            F, T = oracle.forces(w, xs, q, v=v, om=om, mask=CONTACT)
            np.testing.assert_allclose(F[0], Fn * n, rtol=1e-12, atol=1e-13)
            np.testing.assert_allclose(F[1], -Fn * n, rtol=1e-12, atol=1e-13)
            np.testing.assert_allclose(T, 0.0, atol=1e-13)
        # a sliding pair at the first evaluation: only the tangential dashpot,
        # opposite to the sliding velocity of the contact point
        v = np.array([vj + 0.3 * np.cross(n, rng.normal(size=3)), vj])
        F, _ = oracle.forces(w, xs, q, v=v, om=np.zeros((2, 3)), mask=CONTACT)
        vt = (v[0] - v[1]) - np.dot(v[0] - v[1], n) * n
        Ft = F[0] - np.dot(F[0], n) * n
        assert np.dot(Ft, vt) < 0
        assert abs(np.dot(Ft, vt) / (np.linalg.norm(Ft) * np.linalg.norm(vt)) + 1.0) < 1e-12


def test_frictional_clump_conserves_momentum():
    """Spheres thrown together in a box with friction and both dashpots: the
    pair forces are opposite and each pair puts the same torque on both
    spheres, so linear and angular momentum (orbital plus spin) are conserved
    to rounding; the pairs do slide (the Coulomb limit is reached)."""
    rng = np.random.default_rng(9)
    n = 40
    xs = rng.uniform(0, 3.2, size=(n, 3))
    w = spheres(xs, hm=(20.0, 0.3, 0.3, 0.5, 0.5), dt=0.005)
    w["v0"] = rng.normal(0, 0.5, (n, 3))
    w["w0"] = rng.normal(0, 2.0, (n, 3))
    m, I = oracle.mass(w)

    def momenta(st):
        p = (m[:, None] * st["v"]).sum(0)
        Lm = (np.cross(st["x"], m[:, None] * st["v"]) + I[:, None] * st["w"]).sum(0)
        return p, Lm

    st0 = oracle.run(w, 0)
    st = oracle.run(w, 300)
    p0, L0 = momenta(st0)
    p1, L1 = momenta(st)
    scale = (m[:, None] * np.abs(st0["v"])).sum() * (1 + np.abs(st0["x"]).max())
    assert np.max(np.abs(p1 - p0)) <= 1e-12 * scale
    assert np.max(np.abs(L1 - L0)) <= 1e-12 * scale
    assert len(oracle.contact_pairs(w, st0["x"])) > 10
    assert np.max(np.abs(st["w"] - st0["w"])) > 0.1  # friction turned the spins


def test_hookean_model_is_the_default():
    w = spheres([[0, 0, 0], [0.9, 0, 0]], bc=[1, 1])
    w["contact_model"] = "hookean"
    F, _ = oracle.forces(w, w["x0"], np.tile([1.0, 0, 0, 0], (2, 1)), mask=CONTACT)
    np.testing.assert_allclose(F[0], [-w["k_contact"] * 0.1, 0, 0], rtol=1e-14)


def test_oblique_impact_keeps_friction_in_the_tangent_plane():
    """Two spinning spheres meet off-centre with high friction and no normal
    dashpot. The contact normal turns during the impact; the tangential
    displacement is turned with it, so at every level the force along the
    line of centres is the Hertz force of the overlap alone, while the
    tangential force is present and within the Coulomb limit."""
    E, nu, mu = 50.0, 0.3, 1.0
    dt = 0.002
    w = spheres([[0, 0, 0], [1.001, 0.5, 0.1]], hm=(E, nu, mu, 0.0, 0.2), dt=dt)
    w["v0"] = np.array([[0.4, 0.0, 0.0], [-0.4, 0.0, 0.0]])
    w["w0"] = np.array([[0.0, 0.0, 3.0], [1.0, 0.0, -2.0]])
    seen, turned = 0, []
    for L in range(0, 400, 8):
        st = oracle.run(w, L)
        d = st["x"][0] - st["x"][1]
        r = np.linalg.norm(d)
        if r >= 1.0:
            if seen:
                break
            continue
        n = d / r
        turned.append(n)
        delta = 1.0 - r
        Fn = 4.0 / 3.0 * estar(E, nu) * np.sqrt(RS * delta) * delta
        F = st["F"][0]
        assert abs(np.dot(F, n) - Fn) <= 1e-12 * np.linalg.norm(F), L
        Ft = F - np.dot(F, n) * n
        assert np.linalg.norm(Ft) <= mu * Fn * (1 + 1e-12)
        seen += 1
    assert seen >= 5
    assert np.linalg.norm(Ft) > 1e-3 * Fn
    assert np.degrees(np.arccos(np.clip(np.dot(turned[0], turned[-1]), -1, 1))) > 5


def test_turned_displacement_keeps_its_length():
    """A stuck contact whose normal has turned: with no sliding the previous
    displacement is turned into the new tangent plane at its own length, so
    the tangential force keeps its magnitude, -k_t |s|, and is normal to n."""
    E, nu = 10.0, 0.3
    w = spheres([[0, 0, 0], [0.9, 0, 0]], hm=(E, nu, 10.0, 0.0, 0.0))
    rng = np.random.default_rng(2)
    for _ in range(5):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        xi, xj = 0.45 * n, -0.45 * n
        sp = 1e-3 * rng.normal(size=3)  # a displacement from an earlier tangent plane
        F, T, sn, e = oracle.hm_single(w, xi, xj, sprev=sp)
        a = np.sqrt(RS * 0.1)
        kt = 8.0 * gstar(E, nu) * a
        assert abs(np.dot(sn, n)) <= 1e-15
        np.testing.assert_allclose(np.linalg.norm(sn), np.linalg.norm(sp), rtol=1e-13)
        st = sp - np.dot(sp, n) * n  # the turn is the projection, stretched back
        np.testing.assert_allclose(sn, st * np.linalg.norm(sp) / np.linalg.norm(st), rtol=1e-12)
        Ft = F - np.dot(F, n) * n
        np.testing.assert_allclose(Ft, -kt * sn, rtol=1e-12, atol=1e-18)
        np.testing.assert_allclose(T, np.cross(-0.45 * n, Ft), rtol=1e-12, atol=1e-18)


def test_continued_runs_keep_the_tangential_springs():
    """A run cut in pieces carries its contacts and their tangential
    displacements in the state: the stick phase of the driven sphere keeps
    growing as k_t L u dt across the cuts (a reset would drop it to g_t u), and
    a frictional clump run in three pieces is the uncut run."""
    E, nu, mu, gt = 10.0, 0.3, 0.5, 0.01
    r, dt, P = 0.95, 0.01, 1000
    w = spheres([[0, 0, 0], [r, 0, 0]], bc=[2, 1], hm=(E, nu, mu, 0.0, gt), dt=dt,
                drive_axis=np.array([0.0, 0.0, 1.0]), drive_period=P)
    st = oracle.run(w, 2)
    for _ in range(2):
        st = oracle.run(w, 1, state=st)
    np.testing.assert_array_equal(st["F"], oracle.run(w, 4)["F"])
    rng = np.random.default_rng(10)
    n = 30
    w = spheres(rng.uniform(0, 2.9, size=(n, 3)), hm=(20.0, 0.3, 0.3, 0.5, 0.5), dt=0.005)
    w["v0"] = rng.normal(0, 0.5, (n, 3))
    w["w0"] = rng.normal(0, 2.0, (n, 3))
    whole = oracle.run(w, 90)
    st = oracle.run(w, 30)
    assert st["hc_cnt"].sum() > 10
    st = oracle.run(w, 30, state=st)
    st = oracle.run(w, 30, state=st)
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(st[k], whole[k])
