"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: topology and contact pair sets bit-exact; per-step forces within 1e-12
(FP64 path) and 1e-5 (mixed path) of ||ref||_inf per quantity; 100-step
trajectories within 1e-9 / 1e-4 of the motion; energies within 1e-12.
"""
import numpy as np
import pytest

import oracle
import workloads
from paper_2603_27279_amd import (RodSim, TERM_ALL, TERM_BOND, TERM_CONTACT, TERM_DAMP,
                                  TERM_DIPOLE, TERM_EXT, TERM_ZEEMAN)
from paper_2603_27279_amd._lib import ROD_E_NONFINITE, RodError

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}
TRAJ_TOL = {"fp64": 1e-9, "mixed": 1e-4}


def rel_inf(a, ref, floor=0.0):
    den = max(np.max(np.abs(ref)) if ref.size else 0.0, floor)
    num = np.max(np.abs(a - ref)) if ref.size else 0.0
    return num / den if den > 0 else num


def qaxis(axis, ang):
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    return np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * a])


def perturb(w, seed, dx=0.05, rot=0.3, vel=0.05):
    """Move a workload away from its reference: position noise, random
    orientations and velocities on free particles."""
    rng = np.random.default_rng(seed)
    w = dict(w)
    free = w["bc"] == 0
    n = w["n"]
    w["x0"] = w["x0"] + dx * rng.normal(size=(n, 3)) * free[:, None]
    q = np.array([qaxis(rng.normal(size=3), rot * rng.uniform(-1, 1)) for _ in range(n)])
    w["q0"] = np.where(free[:, None], q, w["q0"])
    w["v0"] = vel * rng.normal(size=(n, 3)) * free[:, None]
    w["w0"] = vel * rng.normal(size=(n, 3)) * free[:, None]
    return w


def coil(n=400, members=1, seed=21, pitch=0.8, radius=1.5):
    """Rods wound on a tight helix: turns lie closer than the contact distance."""
    lam = 1.0 / np.hypot(radius, pitch / (2 * np.pi))
    rods = []
    for m in range(members):
        k = np.arange(n)
        ph = k * lam
        rods.append(np.stack([radius * np.cos(ph), radius * np.sin(ph), pitch * ph / (2 * np.pi)], 1))
    x, off, mem = workloads.straight_rods([n] * members, [(0, 0, 0)] * members, (1, 0, 0),
                                          member=np.arange(members))
    bc = np.zeros(n * members, np.int8)
    bc[off[:-1]] = 1
    mb = np.tile([0.0, 0.0, 0.04], (n * members, 1))
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (members, 1)), mb, bc,
                        workloads._field_const(members, (0.1, 0.3, -0.2)), contact_on=True,
                        precision="mixed", name="coil")
    w["x0"] = np.concatenate(rods, 0) + np.random.default_rng(seed).normal(0, 1e-3, (n * members, 3))
    return w


def clump(n_rods=20, L=10, box=3.5, seed=5):
    """Short rods dropped at random into a small box: dense contacts and full cells."""
    rng = np.random.default_rng(seed)
    lens = [L] * n_rods
    x, off, mem = workloads.straight_rods(lens, [(0, 0, 0)] * n_rods, (1, 0, 0))
    n = x.shape[0]
    bc = np.zeros(n, np.int8)
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (n_rods, 1)),
                        rng.normal(0, 0.02, (n, 3)), bc, workloads._field_const(1, (0, 0, 0.5)),
                        contact_on=True, exclude_depth=2, precision="fp64", name="clump")
    w["x0"] = rng.uniform(0, box, size=(n, 3))
    return w


CASES = {
    "cantilever": lambda: workloads.cantilever(n=20),
    "twisted": lambda: perturb(workloads.twisted_rod(n=300, period=200), 1),
    "coil2": lambda: coil(members=2),
    "cilia": lambda: perturb(workloads.cilia_carpet(grid=(4, 4), pitch=3.0, len_range=(5, 40)), 2),
    "ensemble": lambda: perturb(workloads.ensemble(members=3, n=300), 3),
    "clump": lambda: clump(),
    "gradient_field": lambda: perturb(workloads.cantilever(
        n=50, B=(0.2, 1.0, -0.3)), 4) | {"field": np.concatenate(
            [[0.2, 1.0, -0.3], [-0.5, 0.1, 0.0, 0.2, 1.0, 0.0, 0.0, 0.3, -0.5]])[None, None, :]},
}


def oracle_prepared(w):
    return oracle.run(w, 0)


MASKS = [("bond", TERM_BOND), ("dipole", TERM_DIPOLE), ("zeeman", TERM_ZEEMAN),
         ("contact", TERM_CONTACT), ("damping", TERM_DAMP), ("all", TERM_ALL)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(CASES))
def test_forces_per_term(case, prec):
    w = CASES[case]()
    sim = RodSim(w, precision=prec)
    st = oracle_prepared(w)
    gs = sim.state()
    np.testing.assert_allclose(gs["q"], st["q"], atol=1e-15)
    for name, mask in MASKS:
        Fo, To = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=mask)
        F, T = sim.eval_forces(mask)
        F, T = F.cpu().numpy().T, T.cpu().numpy().T
        floor = 1e-300
        assert rel_inf(F, Fo, floor) <= TOL[prec], (case, prec, name, rel_inf(F, Fo, floor))
        assert rel_inf(T, To, floor) <= TOL[prec], (case, prec, name, rel_inf(T, To, floor))
    # the state's own force/torque (evaluated by rod_init) equals the full sum
    Fo, To = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=TERM_ALL)
    assert rel_inf(gs["F"], Fo) <= TOL[prec]
    assert rel_inf(gs["T"], To) <= TOL[prec]
    sim.free()


@pytest.mark.parametrize("case", ["cantilever", "twisted", "coil2", "clump", "ensemble"])
def test_topology_and_contact_pairs_exact(case):
    w = CASES[case]()
    sim = RodSim(w, precision="fp64")
    ij, rr, K = sim.topology()
    oij, orr, oK = oracle.bonds(w)
    np.testing.assert_array_equal(ij, oij)
    np.testing.assert_array_equal(rr, orr)
    np.testing.assert_allclose(K, oK, rtol=1e-15)
    st = oracle_prepared(w)
    pairs = sim.contact_pairs()
    opairs = oracle.contact_pairs(w, st["x"]) if w["contact_on"] else np.zeros((0, 2), np.int32)
    np.testing.assert_array_equal(pairs, opairs)
    if case in ("coil2", "clump"):
        assert len(opairs) > 20
    sim.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["cantilever", "twisted", "coil2", "cilia", "ensemble", "clump"])
def test_trajectory_100_steps(case, prec):
    w = CASES[case]()
    sim = RodSim(w, precision=prec)
    sim.step(100)
    sim.sync()
    g = sim.state()
    o = oracle.run(w, 100)
    o0 = oracle.run(w, 0)
    assert g["step"] == 100
    tol = TRAJ_TOL[prec]
    for k in ("x", "q"):
        motion = max(np.max(np.abs(o[k] - o0[k])), 1e-300)
        assert np.max(np.abs(g[k] - o[k])) / motion <= tol, (case, prec, k)
    for k in ("v", "w", "F", "T"):
        assert rel_inf(g[k], o[k]) <= tol, (case, prec, k, rel_inf(g[k], o[k]))
    sim.free()


@pytest.mark.parametrize("case", ["cantilever", "twisted", "coil2", "ensemble", "clump"])
def test_energy_terms(case):
    w = CASES[case]()
    sim = RodSim(w, precision="fp64")
    sim.step(7)
    g = sim.state()
    E = sim.energy()
    Eo = oracle.energy(w, g["x"], g["q"], g["v"], g["w"], step=7)
    scale = np.abs(Eo).sum(axis=1, keepdims=True)
    assert np.all(np.abs(E - Eo) <= 1e-12 * scale + 1e-300), (E, Eo)
    sim.free()


def test_graph_replay_matches_eager_bitwise():
    w = CASES["twisted"]()
    a = RodSim(w, precision="mixed", graph_steps=10)
    b = RodSim(w, precision="mixed", graph_steps=0)
    for n in (25, 10, 3):
        a.step(n)
        b.step(n)
    sa, sb = a.state(), b.state()
    assert sa["step"] == sb["step"] == 38
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(sa[k], sb[k])
    a.free(); b.free()


def test_runs_are_deterministic():
    w = CASES["clump"]()
    out = []
    for _ in range(2):
        s = RodSim(w, precision="fp64")
        s.step(20)
        out.append(s.state())
        s.free()
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(out[0][k], out[1][k])


def test_edge_cases_single_particles_and_short_rods():
    """Rods of 1 and 2 particles, a member holding a single particle, N not a
    multiple of any tile size."""
    lens = [1, 2, 1, 3, 1]
    x, off, _ = workloads.straight_rods(lens, [(0, 0, 0), (0, 2, 0), (0, 4, 0), (0, 6, 0), (5, 0, 0)],
                                        (1, 0, 0))
    mem = np.array([0, 0, 0, 0, 1], np.int32)
    n = x.shape[0]
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (5, 1)),
                        np.random.default_rng(0).normal(0, 0.1, (n, 3)), np.zeros(n, np.int8),
                        workloads._field_const(2, (0, 0.3, 0)), contact_on=True)
    w = perturb(w, 9)
    for prec in ("fp64", "mixed"):
        sim = RodSim(w, precision=prec)
        sim.step(30)
        g = sim.state()
        o = oracle.run(w, 30)
        assert rel_inf(g["x"] - w["x0"], o["x"] - w["x0"]) <= TRAJ_TOL[prec]
        sim.free()


def test_nonfinite_state_is_reported():
    w = workloads.cantilever(n=20)
    sim = RodSim(w, precision="fp64")
    sim.x[0, 5] = float("nan")
    sim.step(1)
    with pytest.raises(RodError) as e:
        sim.sync()
    assert e.value.code == ROD_E_NONFINITE
    sim.free()


# ---------------------------------------------------------------- full sizes
FULL = {
    "twisted_rod": lambda: workloads.make("twisted_rod"),
    "cilia_carpet": lambda: workloads.make("cilia_carpet"),
    "rod_array": lambda: workloads.make("rod_array"),
    "ensemble": lambda: workloads.make("ensemble"),
}


# the dipole layouts the autotuner picks for these workloads on this GPU (None:
# the default rule)
BENCH_LAYOUT = {"twisted_rod": (0, 1024), "cilia_carpet": (2, 32768), "rod_array": (2, 32768),
                "ensemble": (0, 16384)}


@pytest.mark.parametrize("name,layout", [(n, None) for n in FULL] + list(BENCH_LAYOUT.items()))
def test_full_size_sampled_rows(name, layout):
    """Full-size workloads in the launch configuration of the benchmark (mixed
    path, graph replay, the default layout and the one the autotuner picks):
    after 20 steps, bond, Zeeman and damping forces of every particle, and
    dipole force/field and contact force of 48 sampled particles, match the
    oracle at the GPU's state."""
    w = FULL[name]()
    sim = RodSim(w, precision="mixed", graph_steps=10)
    if layout is not None:
        sim.dipole_layout(*layout)
    sim.step(20)
    sim.sync()
    g = sim.state()
    qn = g["q"]
    for mask in (TERM_BOND, TERM_ZEEMAN, TERM_DAMP):
        F, T = sim.eval_forces(mask)
        Fo, To = oracle.forces(w, g["x"], qn, g["v"], g["w"], step=20, mask=mask)
        assert rel_inf(F.cpu().numpy().T, Fo) <= TOL["mixed"], (name, mask)
        assert rel_inf(T.cpu().numpy().T, To) <= TOL["mixed"], (name, mask)
    rows = np.sort(np.random.default_rng(0).choice(w["n"], 48, replace=False))
    rows[0] = 0
    rows[-1] = w["n"] - 1
    F, T, B = sim.eval_forces(TERM_DIPOLE, with_field=True)
    Fc, _ = sim.eval_forces(TERM_CONTACT)
    Fo, Bo, Fco = oracle.rows(w, g["x"], qn, rows)
    F, B, Fc = F.cpu().numpy().T[rows], B.cpu().numpy().T[rows], Fc.cpu().numpy().T[rows]
    assert rel_inf(F, Fo) <= TOL["mixed"], (name, rel_inf(F, Fo))
    assert rel_inf(B, Bo) <= TOL["mixed"], (name, rel_inf(B, Bo))
    assert np.max(np.abs(Fc - Fco)) <= 1e-12 * max(1.0, np.max(np.abs(Fco)))
    sim.free()


def _check_trajectory(g, o, o0, prec, label):
    tol = TRAJ_TOL[prec]
    for k in ("x", "q"):
        motion = max(np.max(np.abs(o[k] - o0[k])), 1e-300)
        assert np.max(np.abs(g[k] - o[k])) / motion <= tol, (label, k)
    for k in ("v", "w", "F", "T"):
        assert rel_inf(g[k], o[k]) <= tol, (label, k, rel_inf(g[k], o[k]))


def test_full_size_twisted_rod_trajectory():
    """The benchmark's workload as the benchmark runs it (N = 4096, mixed path,
    autotuned layout, 50-step graphs, fused launches): 100 steps against the
    oracle's trajectory."""
    w = workloads.make("twisted_rod")
    sim = RodSim(w, precision="mixed", graph_steps=50)
    sim.autotune()
    sim.step(100)
    sim.sync()
    g = sim.state()
    assert g["step"] == 100
    _check_trajectory(g, oracle.run(w, 100), oracle.run(w, 0), "mixed", "twisted_rod")
    sim.free()


def _member(w, m):
    """Member m of a workload as a system of its own (members never interact)."""
    off = w["rod_offset"]
    rods = np.nonzero(w["rod_member"] == m)[0]
    a, b = off[rods[0]], off[rods[-1] + 1]
    sub = dict(w)
    sub.update(n=int(b - a), rod_offset=(off[rods[0]:rods[-1] + 2] - a).astype(np.int32),
               rod_member=np.zeros(len(rods), np.int32), n_members=1,
               rod_params=w["rod_params"][rods], field=w["field"][:, m:m + 1, :])
    for k in ("x_ref", "x0", "v0", "w0", "q0", "m_body", "bc"):
        sub[k] = w[k][a:b]
    return sub, a, b


def test_full_size_ensemble_members_trajectory():
    """The 64 x 4096 ensemble stepped as one batched launch (20 steps, graphs of
    5); members 0, 31 and 63 checked against the oracle run on each member alone."""
    w = workloads.make("ensemble")
    sim = RodSim(w, precision="mixed", graph_steps=5)
    sim.autotune()
    sim.step(20)
    sim.sync()
    g = sim.state()
    for m in (0, 31, 63):
        sub, a, b = _member(w, m)
        gm = {k: g[k][a:b] for k in ("x", "q", "v", "w", "F", "T")}
        _check_trajectory(gm, oracle.run(sub, 20), oracle.run(sub, 0), "mixed", f"member {m}")
    sim.free()


def test_cantilever_full_run_fp64():
    """The plain FP64 configuration as stated: 20-particle cantilever, 1000 steps."""
    w = workloads.make("cantilever")
    sim = RodSim(w, precision="fp64", graph_steps=50)
    sim.step(1000)
    sim.sync()
    g = sim.state()
    assert g["step"] == 1000
    _check_trajectory(g, oracle.run(w, 1000), oracle.run(w, 0), "fp64", "cantilever")
    sim.free()
