"""The quasi-static field ramp (rod_ramp) against the oracle's: fixed-length
settings, the rest test, the constant-gradient beam of the magnetised-beam
results, the magnetic helix (dipoles, Hertz-Mindlin contact and its history
carried across settings), graph invariance and argument checks."""
import numpy as np
import pytest

import oracle
import workloads
from paper_2603_27279_amd import RodSim
from paper_2603_27279_amd._lib import ROD_E_INVALID, ROD_E_STATE, RodError
from test_oracle_ramp import cantilever, uniform
from test_oracle_pins import _EI

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "mixed": 1e-4}


def run_both(w, f, prec="fp64", graph_steps=0, **kw):
    w = dict(w, field=f[:1])
    sim = RodSim(w, precision=prec, graph_steps=graph_steps)
    g = sim.ramp(f, **kw)
    s = sim.state()
    sim.free()
    o = oracle.ramp(w, f, **kw)
    return g, o, s


def close(g, o, x0, prec):
    motion = max(np.max(np.abs(o["x_watch"] - x0)), 1e-300)
    err = np.max(np.abs(g["x_watch"] - o["x_watch"])) / motion
    assert err <= TOL[prec], err


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fixed_length_settings(prec):
    w = cantilever()
    f = uniform([0.002, 0.006, 0.01, 0.004])
    g, o, _ = run_both(w, f, prec, max_steps=300, check_every=70, ke_tol=-1.0, watch=[10, 5, 0])
    assert g["steps"].tolist() == o["steps"].tolist() == [300] * 4
    close(g, o, w["x0"][[10, 5, 0]], prec)
    np.testing.assert_allclose(g["ke"], o["ke"], rtol=1e-6 if prec == "mixed" else 1e-9)


def test_rest_test_and_the_static_solution():
    nb, Lt, m = 10, 10.0, 1e-3
    w = cantilever(nb, Lt, m)
    Bs = np.linspace(0.0, 0.01, 6)
    f = uniform(Bs)
    g, o, _ = run_both(w, f, "fp64", max_steps=200000, check_every=200, ke_tol=1e-20,
                       watch=[nb])
    assert g["steps"].tolist() == o["steps"].tolist()
    assert np.all(g["steps"] < 200000) and np.all(g["ke"] <= 1e-20)
    xs = np.arange(1, nb + 1) * Lt / nb
    tip = Bs * np.sum(m * xs * (2 * Lt - xs) / (2 * _EI()))
    np.testing.assert_allclose(g["x_watch"][:, 0, 1], tip, rtol=1e-4, atol=1e-9)
    close(g, o, w["x0"][[nb]], "fp64")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_constant_gradient_beam(prec):
    """The beam of the magnetised-beam results magnetised along +y in the field
    of the potential -(b/mu0) (y^2/2 - ((x - L/2)^2 + z^2)/4):
    B = b (-(x - L/2)/2, y, -z/2), gradient b diag(-1/2, 1, -1/2)."""
    nb, Lt = 20, 20.0
    w = cantilever(nb, Lt, damping=0.05, dt=0.1)
    w["m_body"] = np.tile([0.0, 0.02, 0.0], (nb + 1, 1))
    bs = [0.0, 2e-4, 5e-4, 1e-3]
    f = np.zeros((len(bs), 1, 12))
    for k, b in enumerate(bs):
        f[k, 0, 0] = b * Lt / 4  # B0 = b (L/4, 0, 0)
        f[k, 0, 3], f[k, 0, 7], f[k, 0, 11] = -b / 2, b, -b / 2
    g, o, _ = run_both(w, f, prec, max_steps=400, check_every=100, ke_tol=-1.0,
                       watch=[nb, nb // 2])
    close(g, o, w["x0"][[nb, nb // 2]], prec)
    assert np.max(np.abs(o["x_watch"][-1] - w["x0"][[nb, nb // 2]])) > 1e-3


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_magnetic_helix_settings(prec):
    w = workloads.magnetic_helix()
    f = workloads.helix_ramp_fields(w, [0.0, 1.5, 3.0])
    g, o, _ = run_both(w, f, prec, max_steps=500, check_every=250, ke_tol=-1.0,
                       watch=[0, 51, 103])
    close(g, o, w["x0"][[0, 51, 103]], prec)
    np.testing.assert_array_equal(g["x_watch"][:, 0], np.tile(w["x0"][0], (3, 1)))  # clamped


def test_graphs_do_not_change_the_ramp():
    w = workloads.magnetic_helix()
    f = workloads.helix_ramp_fields(w, [0.0, 2.0])
    kw = dict(max_steps=300, check_every=100, ke_tol=-1.0, watch=[103])
    a, _, sa = run_both(w, f, "mixed", graph_steps=0, **kw)
    b, _, sb = run_both(w, f, "mixed", graph_steps=50, **kw)
    np.testing.assert_array_equal(a["x_watch"], b["x_watch"])
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(sa[k], sb[k])


def test_ramp_arguments():
    w = cantilever()
    f = uniform([0.01])
    sim = RodSim(dict(w, field=f[:1]), precision="fp64")
    for kw, code in ((dict(watch=[11]), ROD_E_INVALID), (dict(watch=[-1]), ROD_E_INVALID),
                     (dict(check_every=0), ROD_E_INVALID), (dict(max_steps=0), ROD_E_INVALID),
                     (dict(ke_tol=float("nan")), ROD_E_INVALID)):
        args = dict(max_steps=10, check_every=5, ke_tol=-1.0, watch=[0]) | kw
        with pytest.raises(RodError) as e:
            sim.ramp(f, **args)
        assert e.value.code == code, kw
    sim.free()
    two = dict(w, field=np.concatenate([f, f]))  # a two-row field table
    sim = RodSim(two, precision="fp64")
    with pytest.raises(RodError) as e:
        sim.ramp(f, max_steps=10, check_every=5, ke_tol=-1.0)
    assert e.value.code == ROD_E_INVALID
    sim.free()
    sim = RodSim(dict(w, field=f[:1]), precision="fp64", tape_every=5, tape_capacity=20)
    sim.tape_begin()
    with pytest.raises(RodError) as e:
        sim.ramp(f, max_steps=10, check_every=5, ke_tol=-1.0)
    assert e.value.code == ROD_E_STATE
    sim.free()
