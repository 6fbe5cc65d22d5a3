"""Bond damping on the HIP path (Methods, "Damping") against the FP64 oracle.

The rates are finite differences of each bond's shear angle, twist and bend
vector between consecutive force evaluations, so these tests follow the
measures through whole runs: trajectories with several damping factors per
rod, evaluations at the initial level (no rates), every launch form and graph
chunking, and restarts from a saved state.
"""
import numpy as np
import pytest

import oracle
import workloads
from paper_2603_27279_amd import RodSim, TERM_ALL, TERM_BOND
from test_gpu_parity import TOL, TRAJ_TOL, coil, perturb, rel_inf

pytestmark = pytest.mark.gpu


def damped(w, g):
    w = dict(w)
    w["bond_damping"] = np.broadcast_to(np.asarray(g, float), (len(w["rod_member"]), 4)).copy()
    w["damping"] = 0.0  # bond damping is the only dissipation
    return w


def _cilia():
    w = perturb(workloads.cilia_carpet(grid=(4, 4), pitch=3.0, len_range=(5, 40)), 2)
    rng = np.random.default_rng(17)
    g = rng.uniform(0.0, 0.6, (len(w["rod_member"]), 4))
    g[::5] = 0.0          # some rods undamped
    g[1::7, 1] = 0.0      # and some modes off
    return damped(w, g)


CASES = {
    "twisted": lambda: damped(perturb(workloads.twisted_rod(n=300, period=200), 1),
                              [0.5, 0.3, 0.2, 0.2]),
    "cilia": _cilia,
    "coil2": lambda: damped(coil(members=2), [0.4, 0.2, 0.3, 0.1]),
}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(CASES))
def test_damped_trajectory_100_steps(case, prec):
    w = CASES[case]()
    sim = RodSim(w, precision=prec)
    sim.step(100)
    g = sim.state()
    o = oracle.run(w, 100)
    o0 = oracle.run(w, 0)
    tol = TRAJ_TOL[prec]
    motion = max(np.max(np.abs(o["x"] - o0["x"])), 1e-300)
    for k in ("x", "q"):
        m = max(np.max(np.abs(o[k] - o0[k])), 1e-300)
        assert np.max(np.abs(g[k] - o[k])) / m <= tol, (case, prec, k)
    for k in ("v", "w", "F", "T"):
        assert rel_inf(g[k], o[k]) <= tol, (case, prec, k, rel_inf(g[k], o[k]))
    # the damping is seen: the undamped run lies far outside the tolerance
    plain = dict(w)
    plain["bond_damping"] = None
    u = oracle.run(plain, 100)
    assert np.max(np.abs(u["x"] - o["x"])) / motion > 100 * tol
    sim.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_initial_level_has_no_rates(prec):
    """rod_init's evaluation and any later one at the same level take no rates
    (both equal the oracle's evaluation against the level's own measures); the
    radial term, which needs no history, is present."""
    w = CASES["cilia"]()
    sim = RodSim(w, precision=prec)
    st = oracle.run(w, 0)
    g = sim.state()
    assert rel_inf(g["F"], st["F"]) <= TOL[prec]
    assert rel_inf(g["T"], st["T"]) <= TOL[prec]
    for mask in (TERM_BOND, TERM_ALL):
        Fo, To = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=mask, hist=st["hist"])
        for _ in range(2):  # a repeated evaluation changes nothing
            F, T = sim.eval_forces(mask)
            F, T = F.cpu().numpy().T, T.cpu().numpy().T
            assert rel_inf(F, Fo, 1e-300) <= TOL[prec], (prec, mask)
            assert rel_inf(T, To, 1e-300) <= TOL[prec], (prec, mask)
    plain = dict(w)
    plain["bond_damping"] = None
    Fp, _ = oracle.forces(plain, st["x"], st["q"], st["v"], st["w"], mask=TERM_BOND)
    Fo, _ = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=TERM_BOND, hist=st["hist"])
    assert np.max(np.abs(Fo - Fp)) > 1e-3 * np.max(np.abs(Fp))
    sim.free()


def test_eval_after_steps_matches_the_steps_measures():
    """After k steps an evaluation at level k takes its rates against level k-1,
    the measures the step itself used; with the oracle's measures of level k-1
    and the same state, the bond forces agree."""
    w = CASES["twisted"]()
    k = 7
    sim = RodSim(w, precision="fp64")
    sim.step(k)
    g = sim.state()
    prev = oracle.run(w, k - 1)
    F, T = sim.eval_forces(TERM_BOND)
    F, T = F.cpu().numpy().T, T.cpu().numpy().T
    Fo, To = oracle.forces(w, g["x"], g["q"], g["v"], g["w"], step=k, mask=TERM_BOND,
                           hist=prev["hist"])
    # the measures of level k-1 differ between the two runs by their trajectory
    # difference (< 1e-12 of the motion); the rates divide it by dt
    assert rel_inf(F, Fo) <= 1e-9, rel_inf(F, Fo)
    assert rel_inf(T, To) <= 1e-9, rel_inf(T, To)
    sim.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_damped_launch_forms_and_graphs_bitwise(prec):
    """Batched launches in graphs of any size, eager batched and separate
    launches keep the measures in the same parity planes: bitwise equal."""
    w = CASES["cilia"]()
    runs = []
    for mode, gsteps in (("batched", 0), ("batched", 1), ("batched", 7), ("separate", 10)):
        sim = RodSim(w, precision=prec, graph_steps=gsteps)
        sim.launch_mode(mode)
        for n in (13, 10, 1, 6):
            sim.step(n)
        runs.append(sim.state())
        sim.free()
    for r in runs[1:]:
        assert r["step"] == 30
        for k in ("x", "v", "q", "w", "F", "T"):
            np.testing.assert_array_equal(r[k], runs[0][k])
    if prec == "fp64":
        sim = RodSim(w, precision=prec)
        sim.launch_mode("per_rod")
        sim.step(30)
        s = sim.state()
        for k in ("x", "v", "q", "w", "F", "T"):
            np.testing.assert_array_equal(s[k], runs[0][k])
        sim.free()


@pytest.mark.parametrize("damp", [False, True])
def test_restart_from_saved_state(damp):
    """A context started at level 20 from a saved state and its forces
    (forces_valid) continues as the run that saved it (restart normalises q
    again: agreement to rounding), and as the oracle continued from that state,
    which records the state's own measures as the restart does."""
    w = CASES["twisted"]()
    if not damp:
        w["bond_damping"] = None
    a = RodSim(w, precision="fp64", graph_steps=5)
    a.step(20)
    s = a.state()
    w2 = dict(w, x0=s["x"], v0=s["v"], q0=s["q"], w0=s["w"])
    b = RodSim(w2, precision="fp64", graph_steps=5, step0=20, forces=(s["F"], s["T"]))
    assert b.get_step() == 20
    a.step(15)
    b.step(15)
    sa, sb = a.state(), b.state()
    assert sa["step"] == sb["step"] == 35
    o = oracle.run(w, 15, state={k: s[k] for k in ("x", "v", "q", "w", "F", "T", "step")})
    assert o["step"] == 35
    motion = max(np.max(np.abs(o["x"] - s["x"])), 1e-300)
    for ref, tol in ((sa, 1e-12), (o, TRAJ_TOL["fp64"])):
        assert np.max(np.abs(sb["x"] - ref["x"])) / motion <= tol
        assert np.max(np.abs(sb["q"] - ref["q"])) <= tol
        for k in ("v", "w", "F", "T"):
            assert rel_inf(sb[k], ref[k]) <= tol, (damp, k, rel_inf(sb[k], ref[k]))
    a.free(); b.free()


def test_zero_factors_are_the_undamped_model():
    w = CASES["twisted"]()
    z = dict(w, bond_damping=np.zeros((1, 4)))
    p = dict(w, bond_damping=None)
    out = []
    for v in (z, p):
        sim = RodSim(v, precision="fp64")
        sim.step(10)
        out.append(sim.state())
        sim.free()
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(out[0][k], out[1][k])
