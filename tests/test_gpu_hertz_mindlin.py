"""Hertz-Mindlin contact on the HIP path (Methods, "Contact") against the FP64
oracle: forces and torques at the initial level (every contact new), energies,
100-step trajectories in which contacts carry their tangential displacement
from level to level, launch forms and graph chunking, inspection that leaves
the contact history alone, restarts, systems past the lane-parallel search
size, and the per-particle contact capacity."""
import numpy as np
import pytest

import oracle
import workloads
from paper_2603_27279_amd import RodSim, TERM_ALL, TERM_CONTACT
from paper_2603_27279_amd._lib import ROD_E_OVERFLOW, RodError
from test_gpu_parity import TOL, TRAJ_TOL, clump, coil, perturb, rel_inf

pytestmark = pytest.mark.gpu

# E, nu, mu, g_n, g_t: stiff enough that the dipole-laden clump below keeps
# at most 14 contacts per particle (well under the capacity of 32)
HM = (200.0, 0.3, 0.5, 0.2, 0.2)


def hertz_mindlin(w, hm=HM):
    w = dict(w)
    w["contact_model"] = "hertz_mindlin"
    w["contact_hm"] = np.asarray(hm, float)
    return w


def spinning(w, seed, vel=0.3, spin=1.0):
    """Random velocities and spins on free particles, so that contacts slide."""
    rng = np.random.default_rng(seed)
    free = (w["bc"] == 0)[:, None]
    w = dict(w)
    w["v0"] = vel * rng.normal(size=(w["n"], 3)) * free
    w["w0"] = spin * rng.normal(size=(w["n"], 3)) * free
    return w


def spheres(n=60, box=4.0, seed=3):
    """Single-particle rods thrown into a box: many short frictional contacts."""
    rng = np.random.default_rng(seed)
    x, off, mem = workloads.straight_rods([1] * n, rng.uniform(0, box, (n, 3)), (1, 0, 0))
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (n, 1)), np.zeros((n, 3)),
                        np.zeros(n, np.int8), workloads._field_const(1, (0, 0, 0)),
                        dipole_on=False, contact_on=True, damping=0.0, precision="fp64",
                        name="spheres")
    return spinning(w, seed + 1, vel=0.5, spin=2.0)


CASES = {
    "clump": lambda: hertz_mindlin(spinning(clump(box=4.5), 11)),
    "coil2": lambda: hertz_mindlin(spinning(coil(members=2), 12, vel=0.05, spin=0.2)),
    "spheres": lambda: hertz_mindlin(spheres()),
}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(CASES))
def test_initial_level_forces(case, prec):
    w = CASES[case]()
    sim = RodSim(w, precision=prec)
    st = oracle.run(w, 0)
    assert len(oracle.contact_pairs(w, st["x"])) > 10
    for mask in (TERM_CONTACT, TERM_ALL):
        Fo, To = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=mask)
        F, T = sim.eval_forces(mask)
        F, T = F.cpu().numpy().T, T.cpu().numpy().T
        tol = 1e-12 if mask == TERM_CONTACT else TOL[prec]
        assert rel_inf(F, Fo, 1e-300) <= tol, (case, prec, mask, rel_inf(F, Fo))
        assert rel_inf(T, To, 1e-300) <= tol, (case, prec, mask, rel_inf(T, To))
    g = sim.state()
    assert rel_inf(g["F"], st["F"]) <= TOL[prec]
    assert rel_inf(g["T"], st["T"]) <= TOL[prec]
    E = sim.energy()
    Eo = oracle.energy(w, g["x"], g["q"], g["v"], g["w"])
    assert np.all(np.abs(E[:, 6] - Eo[:, 6]) <= 1e-12 * np.abs(Eo[:, 6]) + 1e-300)
    assert np.all(Eo[:, 6] > 0)
    sim.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(CASES))
def test_trajectory_100_steps(case, prec):
    w = CASES[case]()
    sim = RodSim(w, precision=prec)
    sim.step(100)
    sim.sync()
    g = sim.state()
    o = oracle.run(w, 100)
    o0 = oracle.run(w, 0)
    tol = TRAJ_TOL[prec]
    for k in ("x", "q"):
        m = max(np.max(np.abs(o[k] - o0[k])), 1e-300)
        assert np.max(np.abs(g[k] - o[k])) / m <= tol, (case, prec, k)
    for k in ("v", "w", "F", "T"):
        assert rel_inf(g[k], o[k]) <= tol, (case, prec, k, rel_inf(g[k], o[k]))
    if prec == "fp64":
        # the tangential history matters: the oracle continued one step at a
        # time with the contacts dropped from its state each time (they restart
        # at every level) ends far from this run; carrying them it is the run
        st = o0
        for _ in range(100):
            st = oracle.run(w, 1, state={k: v for k, v in st.items() if not k.startswith("hc_")})
        motion = np.max(np.abs(o["x"] - o0["x"]))
        assert np.max(np.abs(st["x"] - o["x"])) / motion > 100 * tol
        st = o0
        for _ in range(4):
            st = oracle.run(w, 25, state=st)
        np.testing.assert_array_equal(st["x"], o["x"])
    sim.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_launch_forms_and_graphs_bitwise(prec):
    w = CASES["clump"]()
    runs = []
    for mode, gsteps in (("batched", 0), ("batched", 1), ("batched", 7), ("separate", 10),
                         ("per_rod", 0)):
        sim = RodSim(w, precision=prec, graph_steps=gsteps)
        sim.launch_mode(mode)
        for n in (13, 10, 1, 6):
            sim.step(n)
        runs.append(sim.state())
        sim.free()
    for r in runs[1:] if prec == "fp64" else runs[1:4]:
        assert r["step"] == 30
        for k in ("x", "v", "q", "w", "F", "T"):
            np.testing.assert_array_equal(r[k], runs[0][k])


def test_inspection_leaves_the_contacts_alone():
    """Force and energy evaluations and autotuning between steps see full-step
    velocities; they must not overwrite the contacts the next step continues."""
    w = CASES["spheres"]()
    a = RodSim(w, precision="fp64", graph_steps=5)
    b = RodSim(w, precision="fp64", graph_steps=5)
    a.step(10)
    a.eval_forces(TERM_ALL)
    a.energy()
    a.autotune()
    a.step(10)
    b.step(20)
    sa, sb = a.state(), b.state()
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(sa[k], sb[k])
    a.free(); b.free()


def test_restart_starts_contacts_afresh():
    """A context started from a saved state (forces_valid) records that
    state's contacts as new ones, as the oracle continued from it does."""
    w = CASES["clump"]()
    a = RodSim(w, precision="fp64")
    a.step(20)
    s = a.state()
    w2 = dict(w, x0=s["x"], v0=s["v"], q0=s["q"], w0=s["w"])
    b = RodSim(w2, precision="fp64", step0=20, forces=(s["F"], s["T"]))
    b.step(15)
    g = b.state()
    o = oracle.run(w, 15, state={k: s[k] for k in ("x", "v", "q", "w", "F", "T", "step")})
    motion = np.max(np.abs(o["x"] - s["x"]))
    assert g["step"] == o["step"] == 35
    assert np.max(np.abs(g["x"] - o["x"])) / motion <= TRAJ_TOL["fp64"]
    for k in ("v", "w", "F", "T"):
        assert rel_inf(g[k], o[k]) <= TRAJ_TOL["fp64"], (k, rel_inf(g[k], o[k]))
    a.free(); b.free()


def test_restart_carries_the_contact_history():
    """rod_get_contact_history at step 20 matches the oracle's continued state
    (partners and tangential displacements); a context started from the saved
    state with that history installed (rod_set_contact_history) runs 15 more
    steps as the uncut 35-step run, to the rounding of the quaternion
    renormalisation rod_init applies (without the history forces differ by
    about 30% after those steps), and as the oracle's run continued from its
    own step-20 state."""
    w = hertz_mindlin(spheres())
    a = RodSim(w, precision="fp64")
    a.step(20)
    s = a.state()
    h = a.contact_history()
    o20 = oracle.run(w, 20)
    assert np.sum(h["count"]) > 10
    np.testing.assert_array_equal(h["count"], o20["hc_cnt"])
    scale = max(np.max(np.abs(o20["hc_s"])), 1e-300)
    for i in range(w["n"]):
        mine = {int(j): h["disp"][i, k] for k, j in enumerate(h["partner"][i, :h["count"][i]])}
        theirs = {int(j): o20["hc_s"][i, k] for k, j in enumerate(o20["hc_j"][i, :o20["hc_cnt"][i]])}
        assert mine.keys() == theirs.keys(), i
        for j in mine:
            assert np.max(np.abs(mine[j] - theirs[j])) <= 1e-9 * scale, (i, j)
    assert np.any(np.abs(h["disp"]) > 0)  # sliding contacts carry a displacement
    a.step(15)
    uncut = a.state()
    w2 = dict(w, x0=s["x"], v0=s["v"], q0=s["q"], w0=s["w"])
    b = RodSim(w2, precision="fp64", step0=20, forces=(s["F"], s["T"]))
    b.set_contact_history(h)
    b.step(15)
    g = b.state()
    motion = np.max(np.abs(uncut["x"] - s["x"]))
    assert np.max(np.abs(g["x"] - uncut["x"])) <= 1e-12 * motion
    for k in ("v", "q", "w", "F", "T"):
        assert rel_inf(g[k], uncut[k]) <= 1e-12, (k, rel_inf(g[k], uncut[k]))
    o = oracle.run(w, 15, state=o20)
    motion = np.max(np.abs(o["x"] - o20["x"]))
    assert np.max(np.abs(g["x"] - o["x"])) / motion <= TRAJ_TOL["fp64"]
    for k in ("v", "w", "F", "T"):
        assert rel_inf(g[k], o[k]) <= TRAJ_TOL["fp64"], k
    # bad histories are refused on the host
    bad = dict(h, count=h["count"].copy())
    bad["count"][0] = 17
    with pytest.raises(RodError):
        b.set_contact_history(bad)
    a.free(); b.free()


def test_large_system_uses_the_cell_walk():
    """Above the lane-parallel search size (70,000 particles) the Hertz-Mindlin
    search walks the cells in its own launch: forces at the initial level and
    after 5 steps agree with the oracle."""
    rng = np.random.default_rng(12)
    members, rods, length = 70, 10, 100
    lens = [length] * (members * rods)
    origins = [(0.0, 1.05 * (r % rods), 0.0) for r in range(members * rods)]
    x, off, mem = workloads.straight_rods(lens, origins, (1, 0, 0),
                                          member=np.repeat(np.arange(members), rods))
    n = x.shape[0]
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (members * rods, 1)),
                        rng.normal(0, 0.02, (n, 3)), np.zeros(n, np.int8),
                        workloads._field_const(members, (0, 0, 0.5)), contact_on=True,
                        exclude_depth=1, precision="fp64", name="hm_large", dipole_on=False)
    w["x0"] = x + rng.normal(0, 0.05, x.shape)
    w = hertz_mindlin(spinning(w, 13, vel=0.05, spin=0.3))
    assert n >= 65536
    sim = RodSim(w, precision="fp64")
    st = oracle.run(w, 0)
    Fo, To = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=TERM_CONTACT)
    F, T = sim.eval_forces(TERM_CONTACT)
    assert rel_inf(F.cpu().numpy().T, Fo) <= 1e-12
    assert rel_inf(T.cpu().numpy().T, To) <= 1e-12
    assert np.count_nonzero(np.abs(To).sum(1)) > 1000
    sim.step(5)
    g = sim.state()
    o = oracle.run(w, 5)
    motion = np.max(np.abs(o["x"] - st["x"]))
    assert np.max(np.abs(g["x"] - o["x"])) / motion <= TRAJ_TOL["fp64"]
    for k in ("F", "T"):
        assert rel_inf(g[k], o[k]) <= TRAJ_TOL["fp64"], (k, rel_inf(g[k], o[k]))
    sim.free()


def test_contact_capacity_is_reported():
    """A particle buried among 40 overlapping neighbours has more contacts than
    a particle keeps (32): rod_sync reports ROD_E_OVERFLOW; 24 neighbours fit."""
    for k, fits in ((24, True), (40, False)):
        # neighbours on a sphere of radius 0.8 around the origin (Fibonacci points)
        i = np.arange(k) + 0.5
        phi = np.arccos(1 - 2 * i / k)
        th = np.pi * (1 + 5 ** 0.5) * i
        pts = 0.8 * np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
        xs = np.concatenate([[[0.0, 0.0, 0.0]], pts]) + 5.0
        x, off, mem = workloads.straight_rods([1] * (k + 1), xs, (1, 0, 0))
        n = k + 1
        w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (n, 1)), np.zeros((n, 3)),
                            np.ones(n, np.int8), workloads._field_const(1, (0, 0, 0)),
                            dipole_on=False, contact_on=True, precision="fp64")
        w = hertz_mindlin(w)
        assert (len(oracle.contact_pairs(w, xs)) >= k)
        sim = RodSim(w, precision="fp64")
        if fits:
            sim.step(3)
            sim.sync()
        else:
            with pytest.raises(RodError) as e:
                sim.step(3)
                sim.sync()
            assert e.value.code == ROD_E_OVERFLOW
        sim.free()
