"""Pins of the oracle's periodic dipole sum (Ewald summation; the long-range
solvers named beside the truncated pair style in the Introduction and SI
"Magnetic dipoles"). CPU only. What fixes the result independently of the
code: the splitting parameter must drop out; a simple cubic lattice of equal
dipoles feels the Lorentz field 4 pi C m / (3 a^3) (the field of a spherical
cavity, since the lattice sum over a sphere vanishes by cubic symmetry, plus
the conducting-boundary term); forces equal the absolutely convergent direct
sum over images, and fields and energy the spherically summed ones after the
boundary term; a small cluster in a huge box is the open-boundary all-pairs
sum; forces and fields are derivatives of the energy; the energy is
-1/2 sum m.B; total force vanishes; shifting particles by box vectors or all
of them by any vector changes nothing."""
import numpy as np
import pytest

import oracle
import workloads

DIP = oracle.DIPOLE


def periodic(x, m, box, alpha, rcut, kmax, C=1.0):
    """Single-particle rods (no bonds) in one member, dipoles only."""
    n = len(x)
    xx, off, mem = workloads.straight_rods([1] * n, x, (1, 0, 0))
    w = workloads._base(xx, off, mem, np.tile([1.0, 1, 1, 0.5], (n, 1)), np.asarray(m, float),
                        np.zeros(n, np.int8), workloads._field_const(1, (0, 0, 0)),
                        dipole_on=True, contact_on=False, damping=0.0, mu0_4pi=C,
                        box=np.asarray(box, float), ewald_alpha=alpha, ewald_rcut=rcut,
                        ewald_kmax=kmax, name="periodic")
    w["x0"] = np.asarray(x, float).copy()
    return w


def evaluate(w):
    q = w["q0"]
    F, T, B = oracle.forces(w, w["x0"], q, mask=DIP, with_field=True)
    U = oracle.energy(w, w["x0"], q)[0, 5]
    return F, T, B, U


def converged(box, alpha):
    """rcut and kmax at which the real and reciprocal tails are below 1e-16."""
    rcut = 6.0 / alpha
    kmax = int(np.ceil(6.2 * alpha * max(box) / np.pi))
    return rcut, kmax


RNG = np.random.default_rng(2024)
BOX = (4.0, 5.0, 4.5)
X6 = RNG.uniform(0, 1, (6, 3)) * np.array(BOX)
M6 = RNG.normal(0, 0.3, (6, 3))


def self_energy(m, alpha, C=1.0):
    """Magnitude of the self part of the Ewald energy, C 2 a^3 / (3 sqrt(pi)) sum |m|^2."""
    return C * 2 * alpha ** 3 / (3 * np.sqrt(np.pi)) * np.sum(np.asarray(m) ** 2)


def rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def test_splitting_parameter_drops_out():
    res = []
    for alpha in (0.9, 1.3):
        rcut, kmax = converged(BOX, alpha)
        res.append(evaluate(periodic(X6, M6, BOX, alpha, rcut, kmax)))
    (F1, T1, B1, U1), (F2, T2, B2, U2) = res
    assert rel(F1, F2) < 1e-12 and rel(T1, T2) < 1e-12 and rel(B1, B2) < 1e-12
    # the energy is a small difference of its real, reciprocal and self parts:
    # rounding is measured against the largest part (the self energy at 1.3)
    assert abs(U1 - U2) < 1e-13 * self_energy(M6, 1.3)


@pytest.mark.parametrize("rep", [1, 2])
def test_simple_cubic_lattice_lorentz_field(rep):
    a, m = 1.7, np.array([0.3, -0.5, 0.8])
    g = np.stack(np.meshgrid(*[np.arange(rep)] * 3, indexing="ij"), -1).reshape(-1, 3)
    x = a * (g + 0.25)
    box = (rep * a,) * 3
    rcut, kmax = converged(box, 2.2 / a)
    F, T, B, U = evaluate(periodic(x, np.tile(m, (len(x), 1)), box, 2.2 / a, rcut, kmax, C=0.7))
    Bl = 4 * np.pi * 0.7 * m / (3 * a ** 3)
    np.testing.assert_allclose(B, np.tile(Bl, (len(x), 1)), rtol=1e-12, atol=1e-14)
    assert np.max(np.abs(F)) < 1e-13 * np.linalg.norm(m) ** 2 / a ** 4
    assert np.max(np.abs(T)) < 1e-13 * np.linalg.norm(m) ** 2 / a ** 3
    np.testing.assert_allclose(U, -len(x) * 2 * np.pi * 0.7 * np.dot(m, m) / (3 * a ** 3), rtol=1e-12)


def _image_sums(x, m, box, R):
    """Direct sums over every image closer than R (spherical order): force,
    field and energy with bare dipole-dipole terms (C = 1)."""
    L = np.array(box)
    nmax = int(np.ceil(R / L.min())) + 1
    g = np.arange(-nmax, nmax + 1)
    shifts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) * L
    n = len(x)
    F, B, U = np.zeros((n, 3)), np.zeros((n, 3)), 0.0
    for i in range(n):
        for j in range(n):
            r = x[i] - x[j] + shifts
            if i == j:
                r = r[np.any(shifts != 0, axis=1)]
            r2 = np.sum(r * r, 1)
            keep = np.sum(shifts[:len(r)] ** 2, 1) < R * R if i != j else \
                np.sum(shifts[np.any(shifts != 0, axis=1)] ** 2, 1) < R * R
            r, r2 = r[keep], r2[keep]
            rr = np.sqrt(r2)
            a, b, mm = r @ m[i], r @ m[j], m[i] @ m[j]
            F[i] += np.sum((3 / rr ** 5)[:, None] * (mm * r + b[:, None] * m[i] + a[:, None] * m[j]
                                                   - (5 * a * b / r2)[:, None] * r), 0)
            B[i] += np.sum((3 * b / rr ** 5)[:, None] * r - (1 / rr ** 3)[:, None] * m[j], 0)
            U += 0.5 * np.sum(mm / rr ** 3 - 3 * a * b / rr ** 5)
    return F, B, U


def test_forces_equal_direct_image_sum():
    """Forces decay as r^-4, so their image sum converges absolutely (here as
    R^-3: 2e-6 at R = 10 boxes, 2e-7 at 20); fields and energy converge only
    conditionally (as 1/R) and are pinned by the lattice and cluster cases."""
    x, m = X6[:4], M6[:4]
    alpha = 1.1
    rcut, kmax = converged(BOX, alpha)
    F, T, B, U = evaluate(periodic(x, m, BOX, alpha, rcut, kmax))
    Fd, _, _ = _image_sums(x, m, BOX, 22 * max(BOX))
    assert rel(F, Fd) < 1e-6


def test_small_cluster_in_huge_box_is_the_open_sum():
    x, m = X6[:5] * 0.6 + 100.0, M6[:5]
    box = (2000.0, 2000.0, 2000.0)
    alpha = 6.0 / 1000.0
    rcut, kmax = converged(box, alpha)
    rcut = min(rcut, 1000.0)
    w = periodic(x, m, box, alpha, rcut, kmax)
    F, T, B, U = evaluate(w)
    wo = dict(w, box=None)
    Fo, To, Bo = oracle.forces(wo, x, w["q0"], mask=DIP, with_field=True)
    assert rel(F, Fo) < 1e-6 and rel(T, To) < 1e-6 and rel(B, Bo) < 1e-6


def test_force_field_and_energy_are_consistent():
    """F = -dU/dx and B = -dU/dm (central differences), U = -1/2 sum m.B,
    total force zero, torque m x B."""
    alpha = 1.2
    rcut, kmax = converged(BOX, alpha)
    w = periodic(X6, M6, BOX, alpha, rcut, kmax)
    F, T, B, U = evaluate(w)
    assert abs(U + 0.5 * np.sum(M6 * B)) < 1e-13 * self_energy(M6, alpha)
    assert np.max(np.abs(F.sum(0))) < 1e-12 * np.max(np.abs(F))
    np.testing.assert_allclose(T, np.cross(M6, B), rtol=0, atol=1e-13 * np.max(np.abs(T)))
    h = 1e-6
    for i in (0, 3):
        for a in range(3):
            for key, sgn_out in (("x0", F), ("m_body", B)):
                up, dn = dict(w), dict(w)
                up[key] = w[key].copy(); dn[key] = w[key].copy()
                up[key][i, a] += h; dn[key][i, a] -= h
                Uu = oracle.energy(up, up["x0"], w["q0"], mbody=up["m_body"])[0, 5]
                Ud = oracle.energy(dn, dn["x0"], w["q0"], mbody=dn["m_body"])[0, 5]
                fd = -(Uu - Ud) / (2 * h)
                assert abs(fd - sgn_out[i, a]) < 1e-7 * np.max(np.abs(sgn_out)), (key, i, a)


def test_shifts_by_box_vectors_and_translations_change_nothing():
    alpha = 1.0
    rcut, kmax = converged(BOX, alpha)
    base = evaluate(periodic(X6, M6, BOX, alpha, rcut, kmax))
    shift = np.array([[1, 0, -2], [0, 3, 0], [-1, -1, 1], [0, 0, 0], [2, 0, 0], [0, -4, 5]]) * np.array(BOX)
    moved = evaluate(periodic(X6 + shift, M6, BOX, alpha, rcut, kmax))
    trans = evaluate(periodic(X6 + np.array([0.37, -1.9, 2.6]), M6, BOX, alpha, rcut, kmax))
    for a, b, c in zip(base[:3], moved[:3], trans[:3]):
        assert rel(b, a) < 1e-12 and rel(c, a) < 1e-12
    assert abs(moved[3] - base[3]) < 1e-12 * abs(base[3])
