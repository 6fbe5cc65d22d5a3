"""Pins of the oracle's quasi-static field ramp (the loading protocol of the
paper's magnetised beams in non-uniform fields and of its magnetic helix): the
field takes one setting after another and the damped system comes to rest at
each. Pinned by the plain integrator (a ramp of one setting with no rest test
is that many steps), chunk invariance, the Euler-Bernoulli closed form of a
magnetic cantilever at every increment, and reversibility of an elastic
ramp."""
import numpy as np

import oracle
import workloads
from test_oracle_pins import _EI, single_rod


def cantilever(nb=10, Lt=10.0, m=1e-3, damping=0.05, dt=0.1):
    w = single_rod(nb + 1, spacing=Lt / nb, damping=damping, dt=dt)
    w["m_body"] = np.tile([m, 0, 0], (nb + 1, 1))
    w["field"] = workloads._field_const(1, (0, 0, 0))
    return w


def uniform(Bs):
    f = np.zeros((len(Bs), 1, 12))
    f[:, 0, 1] = Bs  # B along y, no gradient
    return f


def test_one_setting_without_rest_test_is_plain_stepping():
    w = cantilever()
    f = uniform([0.01])
    w["field"] = f[:1]
    r = oracle.ramp(w, f, max_steps=700, check_every=100, ke_tol=-1.0, watch=[10, 3])
    o = oracle.run(w, 700)
    assert r["steps"].tolist() == [700]
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(r["state"][k], o[k])
    np.testing.assert_array_equal(r["x_watch"][0], o["x"][[10, 3]])
    m, I = oracle.mass(w)
    ke = 0.5 * (m * (o["v"] ** 2).sum(1)).sum() + 0.5 * (I * (o["w"] ** 2).sum(1)).sum()
    np.testing.assert_allclose(r["ke"][0, 0], ke, rtol=1e-12)


def test_chunks_do_not_change_the_run():
    w = cantilever()
    f = uniform([0.0, 0.005, 0.01])
    w["field"] = f[:1]
    a = oracle.ramp(w, f, max_steps=300, check_every=7, ke_tol=-1.0, watch=[10])
    b = oracle.ramp(w, f, max_steps=300, check_every=300, ke_tol=-1.0, watch=[10])
    assert a["steps"].tolist() == b["steps"].tolist() == [300] * 3
    for k in ("x", "v", "q", "w"):
        np.testing.assert_array_equal(a["state"][k], b["state"][k])
    np.testing.assert_array_equal(a["x_watch"], b["x_watch"])


def test_magnetic_cantilever_follows_the_static_solution():
    """Each increment comes to rest (kinetic energy below the tolerance before
    the step limit) at the Euler-Bernoulli deflection of its own field,
    sum_k m B x_k (2L - x_k) / (2EI), linear in B."""
    nb, Lt, m = 10, 10.0, 1e-3
    w = cantilever(nb, Lt, m)
    Bs = np.linspace(0.0, 0.01, 6)
    f = uniform(Bs)
    w["field"] = f[:1]
    # at rest: a kinetic energy of 1e-20 leaves the slowest mode an amplitude
    # of order 1e-8, far below the 1e-4 of the deflection compared
    r = oracle.ramp(w, f, max_steps=200000, check_every=200, ke_tol=1e-20, watch=[nb])
    xs = np.arange(1, nb + 1) * Lt / nb
    tip = Bs * np.sum(m * xs * (2 * Lt - xs) / (2 * _EI()))
    assert np.all(r["steps"] % 200 == 0) and np.all(r["steps"] < 200000)
    assert np.all(r["ke"][:, 0] <= 1e-20)
    assert r["steps"][0] == 200  # at rest from the start: one chunk
    np.testing.assert_allclose(r["x_watch"][:, 0, 1], tip, rtol=1e-4, atol=1e-9)


def test_elastic_ramp_is_reversible():
    """Without dipole-dipole attraction or contact the rest shape depends on
    the field alone: loading and unloading pass through the same states."""
    w = cantilever(m=2e-2)
    Bs = np.concatenate([np.linspace(0, 0.05, 6), np.linspace(0.05, 0, 6)[1:]])
    f = uniform(Bs)
    w["field"] = f[:1]
    r = oracle.ramp(w, f, max_steps=80000, check_every=200, ke_tol=1e-18, watch=[10])
    up, down = r["x_watch"][:6, 0], r["x_watch"][5:, 0][::-1]
    np.testing.assert_allclose(up, down, atol=1e-7 * np.abs(up).max())
    assert np.abs(up[-1, 1]) > 0.1  # the large-field shape is far from linear
