"""The Ewald sum of the dipoles in a periodic box (the long-range solvers
beside the truncated pair style; Introduction, SI "Magnetic dipoles") on the
HIP path against the FP64 oracle: per-term forces, torques, fields and
energies at the initial level (one and two members, boxes two and more cells
wide, positions outside the box), 100-step trajectories, the Lorentz field of a
simple cubic lattice, bitwise agreement of graphs, launch forms and repeated
runs (FP64 and mixed), and the per-rod loop."""
import numpy as np
import pytest

import oracle
import workloads
from paper_2603_27279_amd import (RodSim, TERM_ALL, TERM_BOND, TERM_DIPOLE, TERM_ZEEMAN,
                                  TERM_DAMP)
from test_gpu_parity import TOL, TRAJ_TOL, perturb, rel_inf

pytestmark = pytest.mark.gpu

CASES = {
    # rcut = 7 in a 14 x 16 x 18 box: 2 x 2 x 2 cells
    "one_member": lambda: perturb(workloads.periodic_rods(n_rods=8, length=16), 5, dx=0.02,
                                  rot=0.1, vel=0.02),
    # two independent periodic systems in one launch
    "two_members": lambda: workloads.periodic_rods(n_rods=6, length=12, members=2, seed=9),
    # rcut = 3 in 14 x 16 x 18: 4 x 5 x 6 cells; rods reach out of the box
    "many_cells": lambda: workloads.periodic_rods(n_rods=10, length=14, rcut=3.0, seed=10),
    # every axis at least seven cells wide (the walk without minimum images,
    # FP32 separations from cell offsets on the mixed path), two members
    "wide_two_members": lambda: workloads.periodic_rods(n_rods=6, length=12, members=2,
                                                        rcut=3.0, seed=11),
}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(CASES))
def test_initial_level_per_term(case, prec):
    w = CASES[case]()
    assert np.any(w["x0"] < 0) or np.any(w["x0"] > w["box"])  # unwrapped positions
    sim = RodSim(w, precision=prec)
    st = oracle.run(w, 0)
    # the real-space pair law and the reciprocal phases are FP32 on the mixed
    # path (the sums across lanes, chunks and rows and the self term FP64 on both)
    Fo, To, Bo = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=TERM_DIPOLE,
                               with_field=True)
    F, T, B = sim.eval_forces(TERM_DIPOLE, with_field=True)
    F, T, B = (a.cpu().numpy().T for a in (F, T, B))
    for a, b, name in ((F, Fo, "F"), (T, To, "T"), (B, Bo, "B")):
        assert rel_inf(a, b) <= TOL[prec], (case, prec, name, rel_inf(a, b))
    for name, mask in (("bond", TERM_BOND), ("zeeman", TERM_ZEEMAN), ("damping", TERM_DAMP),
                       ("all", TERM_ALL)):
        Fo, To = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=mask)
        F, T = sim.eval_forces(mask)
        assert rel_inf(F.cpu().numpy().T, Fo, 1e-300) <= TOL[prec], (case, prec, name)
        assert rel_inf(T.cpu().numpy().T, To, 1e-300) <= TOL[prec], (case, prec, name)
    E = sim.energy()
    Eo = oracle.energy(w, st["x"], st["q"], st["v"], st["w"])
    assert np.all(np.abs(E[:, 5] - Eo[:, 5]) <= TOL[prec] * np.abs(Eo[:, 5])), (E[:, 5], Eo[:, 5])
    sim.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("kmax", [1, 2, 9])
def test_short_reciprocal_rows(kmax, prec):
    """Reciprocal tables whose rows of k vectors hold one to three vectors
    (kmax 1 and 2: a few rows, fewer than the force pass's waves per block) and
    rows just past one run of eight (kmax 9: up to 19 vectors) against the
    oracle with the same truncation, per term and the field."""
    w = workloads.periodic_rods(n_rods=8, length=16, kmax=kmax, seed=12)
    sim = RodSim(w, precision=prec)
    st = oracle.run(w, 0)
    Fo, To, Bo = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=TERM_DIPOLE,
                               with_field=True)
    F, T, B = (a.cpu().numpy().T for a in sim.eval_forces(TERM_DIPOLE, with_field=True))
    sim.free()
    for a, b, name in ((F, Fo, "F"), (T, To, "T"), (B, Bo, "B")):
        assert rel_inf(a, b) <= TOL[prec], (kmax, prec, name, rel_inf(a, b))


@pytest.fixture(scope="module")
def bench_leg_reference():
    """The periodic rods of the bench leg at full size (32 x 32 rods of 32
    particles in a 64 x 64 x 40 box, rcut 16, 12 x 12 x 7 cells, 10,239
    reciprocal vectors), with the parameters the leg uses, and the oracle's
    dipole force, torque and field at the initial level (one evaluation, about
    half a minute on the host)."""
    import bench
    w = workloads.rod_array(grid=(32, 32), n_per_rod=32, pitch=2.0, contact_on=False)
    box, rcut = (64.0, 64.0, 40.0), 16.0
    alpha = 3.6 / rcut
    w.update(box=np.asarray(box, float), ewald_rcut=rcut, ewald_alpha=alpha,
             ewald_kmax=int(np.ceil(3.6 * alpha * max(box) / np.pi)))
    assert w["n"] == 32768 and bench.ewald_leg.__defaults__[:4] == (32, 32, box, rcut)
    # the initial level as the library prepares it: unit quaternions; the
    # dipole term reads only positions and orientations
    q = np.asarray(w["q0"], dtype=np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    x = np.asarray(w["x0"], dtype=np.float64)
    z = np.zeros_like(x)
    return w, oracle.forces(w, x, q, z, z, mask=TERM_DIPOLE, with_field=True)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_bench_leg_workload_full_size(prec, bench_leg_reference):
    """The bench leg's workload at full size against the oracle: the dipole
    force, torque and field of every particle, on the launch configuration the
    leg times (wide cells: on the mixed path the FP32 cell-offset walk)."""
    w, (Fo, To, Bo) = bench_leg_reference
    sim = RodSim(w, precision=prec)
    F, T, B = (a.cpu().numpy().T for a in sim.eval_forces(TERM_DIPOLE, with_field=True))
    sim.free()
    for a, b, name in ((F, Fo, "F"), (B, Bo, "B")):
        assert rel_inf(a, b) <= TOL[prec], (prec, name, rel_inf(a, b))
    # T = m x B: the rods' moments lie nearly along their own field, so the
    # torque is a small part of |m| |B| and carries B's rounding at that scale;
    # it is held to the bar relative to max(|T|, |m| |B|)
    mB = np.max(np.linalg.norm(w["m_body"], axis=1)) * np.max(np.linalg.norm(Bo, axis=1))
    assert rel_inf(T, To, mB) <= TOL[prec], (prec, "T", rel_inf(T, To, mB),
                                             np.max(np.abs(To)) / mB)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_trajectory_100_steps(prec):
    w = CASES["one_member"]()
    sim = RodSim(w, precision=prec, graph_steps=25)
    sim.step(100)
    sim.sync()
    g = sim.state()
    o = oracle.run(w, 100)
    motion = np.max(np.abs(o["x"] - w["x0"]))
    assert motion > 1e-3
    assert np.max(np.abs(g["x"] - o["x"])) <= TRAJ_TOL[prec] * motion
    rot = np.max(np.abs(o["q"] - w["q0"]))
    assert np.max(np.abs(g["q"] - o["q"])) <= TRAJ_TOL[prec] * rot
    for k in ("v", "w"):
        assert rel_inf(g[k], o[k]) <= TRAJ_TOL[prec] * 10, k
    sim.free()


@pytest.mark.parametrize("rep", [1, 3])
def test_simple_cubic_lattice_lorentz_field(rep):
    """Equal dipoles on a simple cubic lattice (a rep^3 block of single-particle
    rods in a box of rep lattice constants): each feels 4 pi C m / (3 a^3), no
    force and no torque, energy -2 pi C |m|^2 / (3 a^3) per particle. With the
    real-space cutoff at half the box, both truncations below 1e-16 need a
    splitting parameter whose self field (C 4 a^3 / (3 sqrt(pi)) m) is up to
    400 times the result at rep = 1; the reciprocal sum cancels it to within
    rounding of about 1e-13 of that size, hence 2e-11 relative."""
    a, m, C = 2.0, np.array([0.03, -0.05, 0.04]), 0.8
    g = np.stack(np.meshgrid(*[np.arange(rep)] * 3, indexing="ij"), -1).reshape(-1, 3)
    x = a * (g + 0.3)
    n = len(x)
    xx, off, mem = workloads.straight_rods([1] * n, x, (1, 0, 0))
    L = rep * a
    w = workloads._base(xx, off, mem, np.tile([1.0, 1, 1, 0.5], (n, 1)), np.tile(m, (n, 1)),
                        np.zeros(n, np.int8), workloads._field_const(1, (0, 0, 0)),
                        contact_on=False, mu0_4pi=C, box=np.array([L, L, L]),
                        ewald_alpha=6.0 / (0.5 * L), ewald_rcut=0.5 * L,
                        ewald_kmax=int(np.ceil(6.2 * 12.0 / np.pi)))
    w["x0"] = x.copy()
    sim = RodSim(w, precision="fp64")
    F, T, B = sim.eval_forces(TERM_DIPOLE, with_field=True)
    F, T, B = (v.cpu().numpy().T for v in (F, T, B))
    Bl = 4 * np.pi * C * m / (3 * a ** 3)
    np.testing.assert_allclose(B, np.tile(Bl, (n, 1)), rtol=2e-11, atol=1e-15)
    # zero to the rounding of a field that is 2e-11 of its own size: F and T
    # below 1e-11 of |m| |B| (over a)
    scale = np.linalg.norm(m) * np.linalg.norm(Bl)
    assert np.max(np.abs(F)) < 1e-11 * scale / a
    assert np.max(np.abs(T)) < 1e-11 * scale
    E = sim.energy()
    np.testing.assert_allclose(E[0, 5], -n * 2 * np.pi * C * np.dot(m, m) / (3 * a ** 3), rtol=2e-11)
    sim.free()


def test_graphs_launch_forms_and_repeats_bitwise():
    """The cell sort orders each cell by particle index and every sum runs in a
    fixed order: eager and graph-replayed steps, the fused and separate force
    launches, and two runs give the same bits; the per-rod loop (one Ewald sum
    per step) agrees with them bitwise too."""
    w = CASES["many_cells"]()
    runs = []
    for gs, mode in ((0, "batched"), (10, "batched"), (0, "separate"), (0, "per_rod"),
                     (10, "batched")):
        s = RodSim(w, precision="fp64", graph_steps=gs)
        s.launch_mode(mode)
        s.step(30)
        s.sync()
        runs.append(s.state())
        s.free()
    for r in runs[1:]:
        for k in ("x", "v", "q", "w", "F", "T"):
            np.testing.assert_array_equal(r[k], runs[0][k])


def test_mixed_path_graphs_launch_forms_and_repeats_bitwise():
    """The mixed path's FP32 real-space sums run in the same fixed order: eager
    and graph-replayed steps, the fused and separate force launches and two runs
    give the same bits."""
    w = CASES["many_cells"]()
    runs = []
    for gs, mode in ((0, "batched"), (10, "batched"), (0, "separate"), (10, "batched")):
        s = RodSim(w, precision="mixed", graph_steps=gs)
        s.launch_mode(mode)
        s.step(30)
        s.sync()
        runs.append(s.state())
        s.free()
    for r in runs[1:]:
        for k in ("x", "v", "q", "w", "F", "T"):
            np.testing.assert_array_equal(r[k], runs[0][k])


@pytest.mark.parametrize("mode", ["batched", "separate"])
def test_timing_classes_of_the_sum(mode):
    """In timing mode the whole sum is timed as the dipole class and its
    real-space walk alone as its own class, once per force evaluation, the walk
    taking part of the sum's time; timing leaves the results unchanged."""
    w = CASES["many_cells"]()
    ref = RodSim(w, precision="mixed")
    ref.step(6)
    st_ref = ref.state()
    ref.free()
    s = RodSim(w, precision="mixed")
    s.launch_mode(mode)
    s.timing(True)
    s.step(6)
    kt = s.kernel_times()
    s.timing(False)
    st = s.state()
    s.free()
    assert kt["ewald_real"][1] == kt["dipole"][1] >= 6
    assert 0 < kt["ewald_real"][0] < kt["dipole"][0]
    for k in ("x", "v", "q", "w"):
        np.testing.assert_array_equal(st[k], st_ref[k])


def test_descriptor_checks():
    """Box and Ewald parameters are validated before any device work."""
    from paper_2603_27279_amd._lib import ROD_E_INVALID, RodError
    w = CASES["one_member"]()
    for over, msg in ((dict(ewald_rcut=7.5), "ewald_rcut"), (dict(ewald_kmax=0), "ewald_kmax"),
                      (dict(contact_on=True), "contact"), (dict(dipole_cutoff=2.0), "dipole_cutoff")):
        with pytest.raises(RodError) as e:
            RodSim(dict(w, **over), precision="fp64")
        assert e.value.code == ROD_E_INVALID and msg in str(e.value)
