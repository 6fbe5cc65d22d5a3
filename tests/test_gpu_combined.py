"""Hertz-Mindlin contact, bond damping and the dipole cutoff together against
the FP64 oracle. They share the cell table, the list rebuild rule and the
per-level history planes: below the list size the Hertz-Mindlin search runs
in the force launch on cells widened for the lists; above it both searches
walk lists rebuilt by the same flag."""
import numpy as np
import pytest

import oracle
import workloads
from paper_2603_27279_amd import RodSim, TERM_ALL
from test_gpu_parity import TRAJ_TOL, coil, rel_inf
from test_gpu_hertz_mindlin import HM, spinning

pytestmark = pytest.mark.gpu


def everything(w):
    w = dict(w)
    w["contact_model"] = "hertz_mindlin"
    w["contact_hm"] = np.asarray(HM, float)
    w["bond_damping"] = np.tile([0.4, 0.2, 0.3, 0.1], (len(w["rod_member"]), 1))
    w["dipole_cutoff"] = 3.0
    return w


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_small_system_100_steps(prec):
    w = everything(spinning(coil(members=2), 12, vel=0.05, spin=0.2))
    sim = RodSim(w, precision=prec, graph_steps=20)
    sim.step(100)
    sim.sync()
    g = sim.state()
    o = oracle.run(w, 100)
    o0 = oracle.run(w, 0)
    tol = TRAJ_TOL[prec]
    for k in ("x", "q"):
        m = max(np.max(np.abs(o[k] - o0[k])), 1e-300)
        assert np.max(np.abs(g[k] - o[k])) / m <= tol, (prec, k)
    for k in ("v", "w", "F", "T"):
        assert rel_inf(g[k], o[k]) <= tol, (prec, k, rel_inf(g[k], o[k]))
    sim.free()


def test_large_system_5_steps():
    rng = np.random.default_rng(21)
    members, rods, length = 70, 10, 100
    lens = [length] * (members * rods)
    origins = [(0.0, 1.05 * (r % rods), 0.0) for r in range(members * rods)]
    x, off, mem = workloads.straight_rods(lens, origins, (1, 0, 0),
                                          member=np.repeat(np.arange(members), rods))
    n = x.shape[0]
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (members * rods, 1)),
                        rng.normal(0, 0.05, (n, 3)), np.zeros(n, np.int8),
                        workloads._field_const(members, (0, 0, 0.5)), contact_on=True,
                        precision="fp64", name="combined_large")
    w["x0"] = x + rng.normal(0, 0.05, x.shape)
    w = everything(spinning(w, 22, vel=0.05, spin=0.3))
    assert n >= 65536
    sim = RodSim(w, precision="fp64")
    st = oracle.run(w, 0)
    Fo, To = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=TERM_ALL, hist=st["hist"])
    F, T = sim.eval_forces(TERM_ALL)
    assert rel_inf(F.cpu().numpy().T, Fo) <= 1e-12
    assert rel_inf(T.cpu().numpy().T, To) <= 1e-12
    sim.step(5)
    g = sim.state()
    o = oracle.run(w, 5)
    motion = np.max(np.abs(o["x"] - st["x"]))
    assert np.max(np.abs(g["x"] - o["x"])) / motion <= TRAJ_TOL["fp64"]
    for k in ("F", "T"):
        assert rel_inf(g[k], o[k]) <= TRAJ_TOL["fp64"], (k, rel_inf(g[k], o[k]))
    sim.free()
