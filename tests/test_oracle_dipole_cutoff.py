"""Pins of the oracle's dipole-dipole cutoff (the truncated pair interaction
of the paper's simulations): a cutoff wider than the member is the all-pairs
sum, a pair just inside the cutoff has the closed-form coaxial force and
energy and one just outside none, an on-axis chain's field is the partial
sum of 2 C m / k^3 over the neighbours inside the cutoff, the truncated
interaction still balances force and angular momentum, and the dual-number run
through a cutoff is the derivative of the run."""
import numpy as np
import pytest

import oracle
import workloads
from test_oracle_pins import ID, two_particles


def chain(n, m=0.3, spacing=1.0):
    x, off, mem = workloads.straight_rods([n], [(0.0, 0.0, 0.0)], (1, 0, 0), spacing=spacing)
    w = workloads._base(x, off, mem, [[1.0, 1.0, 1.0, 0.5]], np.tile([m, 0.0, 0.0], (n, 1)),
                        np.zeros(n, np.int8), workloads._field_const(1, (0, 0, 0)))
    return w, x, np.tile(ID, (n, 1))


def test_wide_cutoff_is_all_pairs():
    rng = np.random.default_rng(5)
    n = 40
    x = rng.uniform(0, 4, (n, 3))
    xs, off, mem = workloads.straight_rods([1] * n, x, (1, 0, 0))
    w = workloads._base(xs, off, mem, np.tile([1.0, 1, 1, 0.5], (n, 1)), rng.normal(0, 0.2, (n, 3)),
                        np.zeros(n, np.int8), workloads._field_const(1, (0, 0, 0)))
    q = np.tile(ID, (n, 1))
    F0, T0 = oracle.forces(w, x, q, mask=oracle.DIPOLE)
    wc = dict(w, dipole_cutoff=100.0)
    F1, T1 = oracle.forces(wc, x, q, mask=oracle.DIPOLE)
    np.testing.assert_array_equal(F0, F1)
    np.testing.assert_array_equal(T0, T1)
    np.testing.assert_array_equal(oracle.energy(w, x, q), oracle.energy(wc, x, q))


@pytest.mark.parametrize("side", [-1, 1])
def test_pair_at_the_cutoff(side):
    m, rd = 0.7, 2.5
    d = rd * (1 + side * 1e-9)
    w, x, q = two_particles([d, 0, 0], [m, 0, 0], [m, 0, 0])
    w["dipole_cutoff"] = rd
    F, T = oracle.forces(w, x, q, mask=oracle.DIPOLE)
    E = oracle.energy(w, x, q)[0, 5]
    if side < 0:  # inside: the coaxial pair, attractive 6 m^2 / d^4, U = -2 m^2 / d^3
        np.testing.assert_allclose(F[0], [6 * m * m / d ** 4, 0, 0], rtol=1e-14)
        np.testing.assert_allclose(E, -2 * m * m / d ** 3, rtol=1e-14)
    else:
        np.testing.assert_array_equal(F, 0.0)
        assert E == 0.0
    np.testing.assert_allclose(T, 0, atol=1e-16)


@pytest.mark.parametrize("rd", [1.5, 3.5, 7.2])
def test_chain_field_is_the_partial_sum(rd):
    """Head-to-tail chain along x: the neighbour k sites away adds 2 C m / k^3
    to the field along the chain; with the cutoff only k < rd count, so the
    end particle's torque-free field is 2 m sum_{k < rd} 1/k^3 and its force
    6 m^2 sum 1/k^4 towards the chain."""
    n, m = 12, 0.3
    w, x, q = chain(n, m)
    w["dipole_cutoff"] = rd
    F, T, B = oracle.forces(w, x, q, mask=oracle.DIPOLE, with_field=True)
    ks = np.arange(1, n)
    ks = ks[ks < rd]
    np.testing.assert_allclose(B[0], [2 * m * np.sum(1.0 / ks ** 3), 0, 0], rtol=1e-13)
    np.testing.assert_allclose(F[0], [6 * m * m * np.sum(1.0 / ks ** 4), 0, 0], rtol=1e-13)


def test_truncated_interaction_balances():
    rng = np.random.default_rng(8)
    n = 60
    x = rng.uniform(0, 5, (n, 3))
    xs, off, mem = workloads.straight_rods([1] * n, x, (1, 0, 0))
    w = workloads._base(xs, off, mem, np.tile([1.0, 1, 1, 0.5], (n, 1)), rng.normal(0, 0.3, (n, 3)),
                        np.zeros(n, np.int8), workloads._field_const(1, (0, 0, 0)),
                        dipole_cutoff=1.8)
    q = np.array([[np.cos(a), *(np.sin(a) * v / np.linalg.norm(v))]
                  for a, v in zip(rng.uniform(0, 1.5, n), rng.normal(size=(n, 3)))])
    F, T = oracle.forces(w, x, q, mask=oracle.DIPOLE)
    scale = np.abs(F).max() * (1 + np.abs(x).max())
    assert np.abs(F.sum(0)).max() <= 1e-13 * scale
    assert np.abs((np.cross(x, F) + T).sum(0)).max() <= 1e-13 * scale
    Fa, _ = oracle.forces(dict(w, dipole_cutoff=0.0), x, q, mask=oracle.DIPOLE)
    assert np.abs(Fa - F).max() > 1e-3 * np.abs(Fa).max()  # the cutoff does cut


def test_jvp_through_the_cutoff_matches_central_differences():
    """A rod of 10 with a cutoff of 2.5: pairs up to two neighbours apart (about
    1 and 2 apart) interact, the next (about 3 apart) do not, and no distance
    comes near 2.5 over the run. The dual-number run (pairs selected by the
    primal distances) equals central differences of the run, and differs from
    the all-pairs one."""
    from test_oracle_pins import rel
    w = workloads.adjoint_rod(n=10, steps=30, dipole_cutoff=2.5)
    rng = np.random.default_rng(8)
    tan = {k: rng.normal(size=np.shape(w[k])) for k in ("x0", "v0", "q0", "w0", "m_body")}
    tan["field"] = rng.normal(size=w["field"].shape)
    for k in ("x0", "v0", "q0", "w0"):
        tan[k][0] = 0.0
    nst = 30
    st, dT = oracle.run_jvp(w, nst, tan)
    d = np.linalg.norm(st["x"][:, None, :] - st["x"][None, :, :], axis=-1)
    assert np.all(np.abs(d - 2.5) > 0.2)
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
    _, dA = oracle.run_jvp(dict(w, dipole_cutoff=0.0), nst, tan)
    assert rel(dA["x"], dT["x"]) > 1e-6  # the cutoff matters
