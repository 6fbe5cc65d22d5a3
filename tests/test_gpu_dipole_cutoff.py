"""The dipole-dipole interaction with a cutoff on the HIP path against the FP64
oracle: forces at the initial level, 100-step trajectories (lists rebuilt as
particles move past the skin), a cutoff wider than the members against the
all-pairs kernels, every launch form, a system past the lane-parallel contact
size, cells that share a sort bucket, and the per-particle list capacity. Sums
run in list order, fixed by the cell sort: a run repeated gives the same bits;
launch forms whose lists are rebuilt at other steps agree to rounding."""
import numpy as np
import pytest

import oracle
import workloads
from paper_2603_27279_amd import RodSim, TERM_ALL, TERM_DIPOLE
from paper_2603_27279_amd._lib import ROD_E_OVERFLOW, RodError
from test_gpu_parity import TOL, TRAJ_TOL, clump, coil, perturb, rel_inf

pytestmark = pytest.mark.gpu

CASES = {
    "twisted": lambda: dict(perturb(workloads.twisted_rod(n=300, period=200), 1), dipole_cutoff=3.0),
    "cilia": lambda: dict(perturb(workloads.cilia_carpet(grid=(4, 4), pitch=3.0, len_range=(5, 40)), 2),
                          dipole_cutoff=2.5),
    "coil2": lambda: dict(coil(members=2), dipole_cutoff=4.0),
    "clump": lambda: dict(clump(), dipole_cutoff=1.7),
}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(CASES))
def test_forces_at_the_initial_level(case, prec):
    w = CASES[case]()
    sim = RodSim(w, precision=prec)
    st = oracle.run(w, 0)
    for mask in (TERM_DIPOLE, TERM_ALL):
        Fo, To = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=mask)
        F, T = sim.eval_forces(mask)
        F, T = F.cpu().numpy().T, T.cpu().numpy().T
        tol = 1e-12 if mask == TERM_DIPOLE else TOL[prec]
        assert rel_inf(F, Fo, 1e-300) <= tol, (case, prec, mask, rel_inf(F, Fo))
        assert rel_inf(T, To, 1e-300) <= tol, (case, prec, mask, rel_inf(T, To))
    Fa, _ = oracle.forces(dict(w, dipole_cutoff=0.0), st["x"], st["q"], mask=TERM_DIPOLE)
    assert np.abs(Fa - Fo).max() > 1e-6 * np.abs(Fa).max()  # the cutoff matters here
    E = sim.energy()
    Eo = oracle.energy(w, st["x"], st["q"], st["v"], st["w"])
    assert np.all(np.abs(E[:, 5] - Eo[:, 5]) <= 1e-12 * np.abs(Eo[:, 5]) + 1e-300)
    sim.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(CASES))
def test_trajectory_100_steps(case, prec):
    w = CASES[case]()
    sim = RodSim(w, precision=prec, graph_steps=25)
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
    sim.free()


def test_wide_cutoff_matches_all_pairs():
    """A cutoff wider than every member gives the all-pairs kernels' result to
    rounding (different summation order and reciprocal square root)."""
    w = perturb(workloads.ensemble(members=3, n=8), 3)
    a = RodSim(dict(w, dipole_cutoff=9.0), precision="fp64")
    b = RodSim(w, precision="fp64")
    Fa, Ta = a.eval_forces(TERM_DIPOLE)
    Fb, Tb = b.eval_forces(TERM_DIPOLE)
    assert rel_inf(Fa.cpu().numpy(), Fb.cpu().numpy()) <= 1e-13
    assert rel_inf(Ta.cpu().numpy(), Tb.cpu().numpy()) <= 1e-13
    a.step(50); b.step(50)
    sa, sb = a.state(), b.state()
    motion = np.max(np.abs(sb["x"] - w["x0"]))
    assert np.max(np.abs(sa["x"] - sb["x"])) / motion <= 1e-10
    a.free(); b.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_launch_forms_agree(prec):
    w = CASES["cilia"]()
    runs = []
    for mode, gsteps in (("batched", 0), ("batched", 7), ("separate", 10), ("per_rod", 0)):
        sim = RodSim(w, precision=prec, graph_steps=gsteps)
        sim.launch_mode(mode)
        for n in (13, 10, 1, 6):
            sim.step(n)
        runs.append(sim.state())
        sim.free()
    motion = np.max(np.abs(runs[0]["x"] - w["x0"]))
    for r in runs[1:]:
        assert r["step"] == 30
        assert np.max(np.abs(r["x"] - runs[0]["x"])) / motion <= 1e-11
        for k in ("F", "T"):
            assert rel_inf(r[k], runs[0][k]) <= (1e-10 if prec == "fp64" else 1e-5)


def test_large_system():
    """70,000 particles: contact and dipole lists both in use."""
    rng = np.random.default_rng(12)
    members, rods, length = 70, 10, 100
    lens = [length] * (members * rods)
    origins = [(0.0, 1.05 * (r % rods), 0.0) for r in range(members * rods)]
    x, off, mem = workloads.straight_rods(lens, origins, (1, 0, 0),
                                          member=np.repeat(np.arange(members), rods))
    n = x.shape[0]
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (members * rods, 1)),
                        rng.normal(0, 0.05, (n, 3)), np.zeros(n, np.int8),
                        workloads._field_const(members, (0, 0, 0.5)), contact_on=True,
                        precision="mixed", name="cutoff_large", dipole_cutoff=3.0)
    w["x0"] = x + rng.normal(0, 0.05, x.shape)
    assert n >= 65536
    sim = RodSim(w, precision="mixed")
    st = oracle.run(w, 0)
    Fo, To = oracle.forces(w, st["x"], st["q"], mask=TERM_DIPOLE)
    F, T = sim.eval_forces(TERM_DIPOLE)
    assert rel_inf(F.cpu().numpy().T, Fo) <= 1e-12
    assert rel_inf(T.cpu().numpy().T, To) <= 1e-12
    sim.step(5)
    g = sim.state()
    o = oracle.run(w, 5)
    motion = np.max(np.abs(o["x"] - st["x"]))
    assert np.max(np.abs(g["x"] - o["x"])) / motion <= TRAJ_TOL["mixed"]
    sim.free()


def test_list_capacity_is_reported():
    """400 particles in a box of side 5 with a cutoff of 7: every particle has
    all 399 others within reach, more than a list holds."""
    rng = np.random.default_rng(4)
    n = 400
    xs = rng.uniform(0, 5, (n, 3))
    x, off, mem = workloads.straight_rods([1] * n, xs, (1, 0, 0))
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (n, 1)), rng.normal(0, 0.01, (n, 3)),
                        np.ones(n, np.int8), workloads._field_const(1, (0, 0, 0)), contact_on=True,
                        precision="fp64", dipole_cutoff=7.0)
    sim = RodSim(w, precision="fp64")
    with pytest.raises(RodError) as e:
        sim.step(2)
        sim.sync()
    assert e.value.code == ROD_E_OVERFLOW
    sim.free()


def _bundle(stretch=1.0, shift=(0.0, 0.0, 0.0), seed=21):
    """A 3 x 3 bundle of rods of 100 particles along z on a unit reference
    lattice (pitch 1.1); the state is that lattice stretched along z and
    shifted, so that the cell sort's key bits, chosen for the reference
    lattice, no longer cover it."""
    rng = np.random.default_rng(seed)
    origins = [(1.1 * (r % 3), 1.1 * (r // 3), 0.0) for r in range(9)]
    x, off, mem = workloads.straight_rods([100] * 9, origins, (0, 0, 1))
    n = x.shape[0]
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (9, 1)), rng.normal(0, 0.05, (n, 3)),
                        np.zeros(n, np.int8), workloads._field_const(1, (0, 0, 0.5)), contact_on=True,
                        precision="fp64", name="cutoff_bundle", dipole_cutoff=3.0)
    x0 = x.copy()
    x0[:, 2] *= stretch
    w["x0"] = x0 + np.asarray(shift) + rng.normal(0, 0.05, x.shape)
    return w


@pytest.mark.parametrize("stretch,shift", [(1.0, (0.0, 0.0, 0.0)), (2.5, (0.0, 0.0, 0.0)),
                                           (1.0, (1.0e4, 0.0, -3.0e3))])
def test_cells_sharing_a_bucket(stretch, shift):
    """The sort's key keeps 6 bits of the cell coordinate along the bundle (64
    cells of side 3.25, enough for the reference lattice). Stretched 2.5 times,
    cells 64 apart share buckets; shifted by 10^4, the high bits of every
    cell's coordinates leave the tag's range and cells are told apart by their
    coordinates. The dipole forces and fields match the oracle in each case."""
    w = _bundle(stretch, shift)
    sim = RodSim(w, precision="fp64")
    st = oracle.run(w, 0)
    Fo, To = oracle.forces(w, st["x"], st["q"], mask=TERM_DIPOLE)
    F, T = sim.eval_forces(TERM_DIPOLE)
    assert rel_inf(F.cpu().numpy().T, Fo, 1e-300) <= 1e-12
    assert rel_inf(T.cpu().numpy().T, To, 1e-300) <= 1e-12
    assert np.abs(Fo).max() > 0
    sim.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_runs_repeat_bit_for_bit(prec):
    """The same run twice (graphs of 7 steps, lists rebuilt as particles move)
    ends in the same state, bit for bit."""
    w = CASES["cilia"]()
    runs = []
    for _ in range(2):
        sim = RodSim(w, precision=prec, graph_steps=7)
        for n in (13, 10, 1, 6):
            sim.step(n)
        runs.append(sim.state())
        sim.free()
    for k in ("x", "v", "q", "w", "F", "T"):
        np.testing.assert_array_equal(runs[0][k], runs[1][k], err_msg=k)


@pytest.mark.parametrize("grid,npr", [((32, 16), 512), ((64, 64), 1024)])
def test_full_size_sampled_rows(grid, npr):
    """The rod array at the benchmark's sizes with a cutoff of 3 (262,144
    particles, and the 4.2M-particle array of the memory-bound legs), mixed
    path, graphs of 10: after 20 steps (lists rebuilt at the call's first step
    and whenever a particle passes 0.45 of the skin), the dipole force and field
    of 48 sampled particles match the oracle's truncated sums at the GPU's
    state."""
    w = workloads.rod_array(grid=grid, n_per_rod=npr, dipole_on=True, dipole_cutoff=3.0)
    sim = RodSim(w, precision="mixed", graph_steps=10)
    sim.step(20)
    sim.sync()
    g = sim.state()
    rows = np.sort(np.random.default_rng(1).choice(w["n"], 48, replace=False))
    rows[0] = 0
    rows[-1] = w["n"] - 1
    F, T, B = sim.eval_forces(TERM_DIPOLE, with_field=True)
    Fo, Bo, _ = oracle.rows(w, g["x"], g["q"], rows)
    F, B = F.cpu().numpy().T[rows], B.cpu().numpy().T[rows]
    assert rel_inf(F, Fo) <= 1e-12, rel_inf(F, Fo)
    assert rel_inf(B, Bo) <= 1e-12, rel_inf(B, Bo)
    sim.free()

