"""Dipole work layouts and the autotuner: every layout gives the oracle's
forces; tuning does not change the state; the cache round-trips."""
import numpy as np
import pytest

import oracle
import workloads
from paper_2603_27279_amd import RodSim, TERM_ALL, TERM_DIPOLE
from paper_2603_27279_amd._lib import ROD_E_INVALID, ROD_E_STATE, RodError

pytestmark = pytest.mark.gpu


def rel_inf(a, ref):
    return np.max(np.abs(a - ref)) / np.max(np.abs(ref))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
@pytest.mark.parametrize("layout", [(1, 1024), (0, 64), (0, 1024), (0, 8192), (0, 65536), (2, 64),
                                    (2, 1024)])
def test_every_layout_matches_oracle(layout, prec, tol):
    w = workloads.ensemble(members=3, n=700)
    w["x0"] = w["x0"] + np.random.default_rng(1).normal(0, 0.05, w["x0"].shape) * (w["bc"] == 0)[:, None]
    sim = RodSim(w, precision=prec)
    sim.dipole_layout(*layout)
    st = oracle.run(w, 0)
    for mask in (TERM_DIPOLE, TERM_ALL):
        F, T = sim.eval_forces(mask)
        Fo, To = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=mask)
        assert rel_inf(F.cpu().numpy().T, Fo) <= tol
        assert rel_inf(T.cpu().numpy().T, To) <= tol
    sim.step(10)
    o = oracle.run(w, 10)
    g = sim.state()
    motion = np.max(np.abs(o["x"] - w["x0"]))
    assert np.max(np.abs(g["x"] - o["x"])) / motion <= (1e-9 if prec == "fp64" else 1e-4)
    sim.free()


def test_autotune_keeps_state_and_caches(tmp_path):
    w = workloads.twisted_rod(n=1500)
    cache = tmp_path / "tune.jsonl"
    a = RodSim(w, precision="mixed", graph_steps=10)
    a.step(15)
    before = a.state()
    rep = a.autotune(cache)
    after = a.state()
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(before[k], after[k])
    assert "chosen" in rep and cache.exists()
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and '"key"' in lines[0]
    a.step(25)  # graphs are recaptured after the layout change
    o = oracle.run(w, 40)
    motion = np.max(np.abs(o["x"] - w["x0"]))
    assert np.max(np.abs(a.state()["x"] - o["x"])) / motion <= 1e-4
    # two fresh contexts that take the cached choice run identically
    runs = []
    for _ in range(2):
        b = RodSim(w, precision="mixed", graph_steps=10)
        assert "cached choice" in b.autotune(cache)
        b.step(40)
        runs.append(b.state())
        b.free()
    for k in ("x", "v", "q", "w"):
        np.testing.assert_array_equal(runs[0][k], runs[1][k])
    a.free()


def test_dipole_layout_arguments_are_checked():
    w = workloads.twisted_rod(n=300)
    sim = RodSim(w, precision="mixed")
    for bad in ((3, 64), (-2, 64), (0, 0)):
        with pytest.raises(RodError) as e:
            sim.dipole_layout(*bad)
        assert e.value.code == ROD_E_INVALID
    sim.step(3)
    sim.free()


def test_autotune_refused_while_taping():
    w = workloads.adjoint_rod(n=32)
    sim = RodSim(w, precision="fp64", tape_every=5, tape_capacity=20)
    sim.tape_begin()
    with pytest.raises(RodError) as e:
        sim.autotune()
    assert e.value.code == ROD_E_STATE
    sim.free()


def _many_rods():
    """A small cilia carpet: 30 rods of uneven length in one member, so rods do
    not start on block boundaries and contact can join neighbouring rods."""
    w = workloads.cilia_carpet(grid=(6, 5), pitch=3.0, len_range=(5, 70), seed=7)
    rng = np.random.default_rng(8)
    w["x0"] = w["x0"] + rng.normal(0, 0.05, w["x0"].shape) * (w["bc"] == 0)[:, None]
    return w


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("layout", [(1, 1024), (0, 64), (0, 4096)])
def test_launch_modes_match(layout, prec):
    """Batched and separate launches use the same work items: bitwise equal.
    The per-rod loop cuts target blocks at rod boundaries; in FP64 it is still
    bitwise equal, on the mixed path a block may take the exact-difference path
    where the batched block took the far-tile one, so it agrees to rounding."""
    w = _many_rods()
    states = []
    for mode in ("batched", "separate", "per_rod"):
        sim = RodSim(w, precision=prec, graph_steps=0 if mode == "per_rod" else 10)
        sim.dipole_layout(*layout)
        sim.launch_mode(mode)
        sim.step(30)
        states.append(sim.state())
        sim.free()
    o = oracle.run(w, 30)
    motion = np.max(np.abs(o["x"] - w["x0"]))
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(states[0][k], states[1][k])
        if prec == "fp64":
            np.testing.assert_array_equal(states[0][k], states[2][k])
    if prec == "mixed":
        assert np.max(np.abs(states[2]["x"] - states[0]["x"])) / motion <= 1e-5
        for k in ("F", "T"):
            assert rel_inf(states[2][k], states[0][k]) <= 1e-5
    assert np.max(np.abs(states[0]["x"] - o["x"])) / motion <= (1e-9 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("target", [64, 4096])
def test_spatial_layout_launch_modes(prec, target):
    """The split layout over the spatial order of the particles: batched and
    separate launches bitwise equal, the trajectory within the oracle's bound,
    and the state of the particle-order layout to rounding (the sums are the
    same terms added in another order)."""
    w = _many_rods()
    states, energies = [], []
    for small, mode in ((2, "batched"), (2, "separate"), (0, "batched"), (2, "per_rod")):
        sim = RodSim(w, precision=prec, graph_steps=0 if mode == "per_rod" else 10)
        sim.dipole_layout(small, target)
        sim.launch_mode(mode)
        sim.step(30)
        states.append(sim.state())
        energies.append(sim.energy())
        sim.free()
    o = oracle.run(w, 30)
    motion = np.max(np.abs(o["x"] - w["x0"]))
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(states[0][k], states[1][k])
    np.testing.assert_array_equal(energies[0], energies[1])
    # particle order, and the per-rod loop (whose work items are particle ranges)
    for other in (states[2], states[3]):
        assert np.max(np.abs(states[0]["x"] - other["x"])) / motion <= (1e-12 if prec == "fp64" else 1e-5)
    np.testing.assert_allclose(energies[0], energies[2], rtol=1e-12 if prec == "fp64" else 1e-5,
                               atol=1e-12 * np.max(np.abs(energies[2])))
    assert np.max(np.abs(states[0]["x"] - o["x"])) / motion <= (1e-9 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("make", [workloads.magnetic_helix, workloads.coiled_rods])
def test_spatial_layout_with_contacts(make):
    """Systems with contacts in the force launch (the helix's Hertz-Mindlin law,
    coiled rods' Hookean turns): the spatial order steps like particle order to
    rounding, and its batched and separate launches are bitwise equal."""
    w = make()
    states = []
    for small, mode in ((2, "batched"), (2, "separate"), (0, "batched")):
        sim = RodSim(w, precision="mixed", graph_steps=10)
        sim.dipole_layout(small, 64)
        sim.launch_mode(mode)
        sim.step(40)
        states.append(sim.state())
        sim.free()
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(states[0][k], states[1][k])
    motion = np.max(np.abs(states[2]["x"] - w["x0"]))
    assert np.max(np.abs(states[0]["x"] - states[2]["x"])) / motion <= 1e-5
    for k in ("F", "T"):
        assert rel_inf(states[0][k], states[2][k]) <= 1e-4, k


def test_spatial_layout_without_work_items():
    """A dipole cutoff walks lists and holds no work items: asking for the
    spatial order changes nothing."""
    w = dict(_many_rods(), dipole_cutoff=3.0)
    runs = []
    for layout in ((0, 1024), (2, 1024)):
        sim = RodSim(w, precision="mixed", graph_steps=10)
        sim.dipole_layout(*layout)
        sim.step(12)
        runs.append(sim.state())
        sim.free()
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(runs[0][k], runs[1][k])


def _twisted_small():
    w = workloads.twisted_rod(n=300, period=200)
    rng = np.random.default_rng(9)
    w["x0"] = w["x0"] + rng.normal(0, 0.05, w["x0"].shape) * (w["bc"] == 0)[:, None]
    return w


@pytest.mark.parametrize("graph_steps", [0, 1, 2, 7])
def test_fused_step_chains_match_separate_bitwise(graph_steps):
    """Batched stepping fuses the end of one step with the start of the next and
    alternates level counters; any chunking and graph size gives the state of
    unfused separate launches."""
    w = _twisted_small()
    a = RodSim(w, precision="mixed", graph_steps=graph_steps)
    b = RodSim(w, precision="mixed", graph_steps=0)
    b.launch_mode("separate")
    for n in (25, 10, 1, 3):
        a.step(n)
        b.step(n)
    sa, sb = a.state(), b.state()
    assert sa["step"] == sb["step"] == 39
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(sa[k], sb[k])
    a.free(); b.free()


def test_timing_mode_runs_the_same_steps():
    w = _twisted_small()
    a = RodSim(w, precision="mixed", graph_steps=5)
    b = RodSim(w, precision="mixed", graph_steps=5)
    for s in (a, b):
        s.dipole_layout(0, 64)  # split layout: dipole work inside the fused force kernel
    a.timing(True)
    a.step(13)
    kt = a.kernel_times()
    a.timing(False)
    b.step(13)
    assert kt["pre"][1] == 1 and kt["post"][1] == 1
    assert kt["forces"][1] == 13 and kt["kick"][1] == 12
    assert all(kt[k][1] == 0 for k in ("bond", "dipole", "contact"))
    assert all(ms > 0 for ms, c in kt.values() if c)
    sa, sb = a.state(), b.state()
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(sa[k], sb[k])
    a.free(); b.free()


def test_timing_counts_survive_the_event_pool_bound():
    """More timed launches than the library keeps pending event pairs for: the
    sums are folded on the way and every launch is still counted."""
    w = _twisted_small()
    a = RodSim(w, precision="mixed")
    a.dipole_layout(0, 64)
    a.timing(True)
    a.step(2500)  # 5000 timed launches
    kt = a.kernel_times()
    a.timing(False)
    assert kt["pre"][1] == 1 and kt["post"][1] == 1
    assert kt["forces"][1] == 2500 and kt["kick"][1] == 2499
    assert all(ms > 0 for ms, c in kt.values() if c)
    a.free()


def _dense_large(members=70, rods=10, length=100, seed=12):
    """70,000 particles (above the size where contact switches to candidate
    lists): per member ten parallel rods 1.05 apart with random velocities, so
    rods collide and lists go stale part-way through a call. Members overlap in
    space but never interact; the oracle's brute-force contact stays cheap."""
    rng = np.random.default_rng(seed)
    origins, member = [], []
    for m in range(members):
        for r in range(rods):
            origins.append((0.0, 1.05 * (r % 2), 1.05 * (r // 2)))
            member.append(m)
    x, off, mem = workloads.straight_rods([length] * len(origins), origins, (1.0, 0.0, 0.0),
                                          member=np.array(member))
    n = x.shape[0]
    bc = np.zeros(n, np.int8)
    w = workloads._base(x, off, mem, np.tile([1.0, 1.0, 1.0, 0.5], (len(origins), 1)),
                        np.zeros((n, 3)), bc, workloads._field_const(members, (0.0, 0.0, 0.0)),
                        dipole_on=False, contact_on=True, precision="fp64", name="dense_large")
    w["v0"] = rng.normal(0.0, 0.4, (n, 3))
    return w


def test_contact_lists_match_cell_search_bitwise():
    w = _dense_large()
    assert w["n"] >= 65536
    a = RodSim(w, precision="fp64", graph_steps=0)   # lists reused within the call
    b = RodSim(w, precision="fp64", graph_steps=10)  # one build per graph replay
    c = RodSim(w, precision="fp64", graph_steps=0)   # a build at every step
    a.step(40)
    b.step(40)
    for _ in range(40):
        c.step(1)
    for s in (a, b, c):
        s.sync()  # raises if a cell or the overflow list ran out of room
    sa, sb, sc = a.state(), b.state(), c.state()
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(sa[k], sc[k])
        np.testing.assert_array_equal(sb[k], sc[k])
    o = oracle.run(w, 40)
    motion = np.max(np.abs(o["x"] - w["x0"]))
    assert motion > 0.5  # particles moved past the skin: lists were rebuilt mid-call
    assert np.max(np.abs(sa["x"] - o["x"])) / motion <= 1e-9
    for s in (a, b, c):
        s.free()


def test_autotune_cache_holds_small_layout_choice(tmp_path):
    """A cached small-member choice (whose target_wgs is 0) is taken from the cache."""
    w = workloads.twisted_rod(n=1500)
    a = RodSim(w, precision="mixed")
    key = a.autotune().strip().splitlines()[-1].split("key=")[1].strip()
    cache = tmp_path / "tune.jsonl"
    cache.write_text('{"key": "%s", "small": 1, "target_wgs": 0, "us_per_eval": 1.000}\n' % key)
    rep = a.autotune(cache)
    assert "cached choice" in rep
    assert "chosen: small-member layout" in rep
    a.step(10)
    o = oracle.run(w, 10)
    motion = np.max(np.abs(o["x"] - w["x0"]))
    assert np.max(np.abs(a.state()["x"] - o["x"])) / motion <= 1e-4
    a.free()
