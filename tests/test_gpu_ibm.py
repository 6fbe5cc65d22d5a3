"""Immersed-boundary coupling of rods and lattice (rod_lbm_cycles) against the
FP64 oracle's coupled driver: rod states and populations after several cycles,
for both force launch forms, a carpet of rods spanning many blocks with
positions that wrap around the periodic lattice, a carpet of cilia on
clamped bases with a driven tip in a turning field (periodic, between no-slip
walls, one of them moving, and under a free-slip top), conservation of rods'
plus fluid momentum over many cycles, and the argument checks."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import lbm
from paper_2603_27279_amd import Lattice, RodSim
from paper_2603_27279_amd._lib import ROD_E_INVALID, RodError
from test_gpu_parity import TRAJ_TOL, rel_inf

pytestmark = pytest.mark.gpu


def rods(lens, origins, nsub, seed, field=(0, 0, 0.2), direction=(1, 0, 0), **kw):
    """Free magnetised rods (lattice units), rod dt = 1 / nsub, no damping."""
    rng = np.random.default_rng(seed)
    x, off, mem = workloads.straight_rods(lens, origins, direction)
    n, R = x.shape[0], len(lens)
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (R, 1)), np.tile([0, 0, 0.05], (n, 1)),
                        np.zeros(n, np.int8), workloads._field_const(1, field), damping=0.0,
                        dt=1.0 / nsub, precision="fp64", **kw)
    w["v0"] = 0.01 * rng.normal(size=(n, 3))
    w["x0"] = x + rng.normal(0, 0.02, x.shape)
    return w


def fluid(shape, seed, amp=0.005):
    rng = np.random.default_rng(seed)
    return lbm.equilibrium(1 + 0.01 * rng.random(shape), amp * rng.normal(size=(3,) + shape))


def run_gpu(w, f0, ncycles, nsub, tau, g=(0.0, 0.0, 0.0), mode="batched", prec="fp64",
            walls=0, lid=(0.0, 0.0)):
    sim = RodSim(w, precision=prec)
    sim.launch_mode(mode)
    lat = Lattice(f0, tau=tau, force=g, walls_z=walls, lid=lid)
    sim.lbm_cycles(lat, nsub, ncycles)
    sim.sync()
    st = sim.state()
    f = lat.populations().cpu().numpy()
    sim.free(); lat.free()
    return st, f


def compare(st, f, w, f0, ncycles, nsub, tau, g=(0.0, 0.0, 0.0), prec="fp64", ftol=1e-13,
            walls=0, lid=(0.0, 0.0)):
    ost, of = lbm.coupled(w, f0, ncycles, nsub, tau, g=g, walls=walls, lid=lid)
    assert st["step"] == ncycles * nsub
    motion = np.max(np.abs(ost["x"] - w["x0"]))
    assert np.max(np.abs(st["x"] - ost["x"])) / motion <= TRAJ_TOL[prec]
    for k in ("v", "w", "F", "T"):
        assert rel_inf(st[k], ost[k]) <= TRAJ_TOL[prec], (k, rel_inf(st[k], ost[k]))
    # populations ~ w_i rho: absolute agreement to rounding of the spread sums
    assert np.max(np.abs(f - of)) <= ftol, np.max(np.abs(f - of))
    # the rods moved the fluid
    assert np.max(np.abs(of - lbm.run(f0, ncycles, tau, g=g, walls=walls, lid=lid))) > 1e-9


@pytest.mark.parametrize("mode", ["batched", "separate"])
def test_two_rods_match_oracle(mode):
    nsub, tau = 4, 0.8
    w = rods([6, 6], [(3.2, 4.1, 4.3), (3.7, 6.4, 5.1)], nsub, 1)
    f0 = fluid((12, 12, 14), 2)
    st, f = run_gpu(w, f0, 3, nsub, tau, mode=mode)
    compare(st, f, w, f0, 3, nsub, tau)


def test_mixed_precision_rods():
    """The mixed path's FP32 pair arithmetic feeds the penalty force through
    the velocities; the fluid sees it at that precision."""
    nsub, tau = 4, 0.8
    w = rods([8, 8, 8], [(3.2, 4.1, 4.3), (3.7, 6.4, 5.1), (2.5, 8.8, 7.9)], nsub, 12)
    f0 = fluid((12, 12, 14), 13)
    st, f = run_gpu(w, f0, 3, nsub, tau, prec="mixed")
    compare(st, f, w, f0, 3, nsub, tau, prec="mixed", ftol=1e-8)


def test_hertz_mindlin_contacts():
    """Two rods overlapping by 0.05 with Hertz-Mindlin contact and friction:
    the contact torques and the penalty force share the post kernel."""
    nsub, tau = 8, 0.8
    w = rods([7, 7], [(3.0, 4.0, 5.0), (3.0, 4.95, 5.0)], nsub, 14, contact_on=True,
             contact_model="hertz_mindlin", contact_hm=np.array([20.0, 0.3, 0.5, 0.0, 0.0]))
    f0 = fluid((12, 12, 14), 15)
    ost = oracle.run(w, 0)
    Fc, Tc = oracle.forces(w, ost["x"], ost["q"], ost["v"], ost["w"], mask=8)
    assert np.abs(Fc).max() > 0  # the rods touch
    st, f = run_gpu(w, f0, 2, nsub, tau)
    compare(st, f, w, f0, 2, nsub, tau)


def test_carpet_wraps_around_the_lattice():
    """48 rods of 10 to 30 particles (about 1,000, several blocks) along y,
    many of them crossing the periodic boundary, with a uniform body force."""
    rng = np.random.default_rng(5)
    lens = list(rng.integers(10, 31, 48))
    origins = [(1.3 + 2.1 * (r % 8), 7.0 + 3.3 * rng.random(), 1.7 + 3.9 * (r // 8)) for r in range(48)]
    nsub, tau, g = 2, 0.7, (2e-6, 0.0, -1e-6)
    w = rods(lens, origins, nsub, 6, direction=(0, 1, 0))
    f0 = fluid((24, 20, 18), 7)
    assert np.max(w["x0"][:, 1]) > 20  # past the lattice's y extent: wraps
    st, f = run_gpu(w, f0, 2, nsub, tau, g=g)
    compare(st, f, w, f0, 2, nsub, tau, g=g)


def test_momentum_conserved_over_many_cycles():
    """Bonds, dipoles and a uniform field exert no net force, so the rods'
    and the fluid's momentum plus half a rod step of the last penalty force
    (the velocity-Verlet share not yet in the velocities) stays constant."""
    nsub, tau = 5, 0.9
    lens = [20] * 8
    origins = [(2.0 + 3.0 * r, 5.0, 6.0 + 1.5 * r) for r in range(8)]
    w = rods(lens, origins, nsub, 8)
    shape = (20, 18, 32)
    f0 = fluid(shape, 9, amp=0.01)
    m, _ = oracle.mass(w)
    Cf = lbm.C.astype(float)
    sim = RodSim(w, precision="fp64")
    lat = Lattice(f0, tau=tau)

    def Q():
        st = sim.state()
        f = lat.populations().cpu().numpy()
        Pf = np.einsum("id,i...->d...", Cf, f).reshape(3, -1).sum(1)
        Pr = (m[:, None] * st["v"]).sum(0)
        return Pf + Pr + 0.5 * w["dt"] * st["F"].sum(0), Pr

    q0, pr0 = Q()
    for _ in range(4):
        sim.lbm_cycles(lat, nsub, 10)
        q, pr = Q()
        scale = np.abs(np.einsum("id,i...->d...", Cf, f0)).sum()
        assert np.max(np.abs(q - q0)) <= 1e-12 * scale, (q - q0, scale)
    assert np.max(np.abs(pr - pr0)) > 1e-3 * np.max(np.abs(pr0))
    sim.free(); lat.free()


def test_argument_checks():
    w = rods([4], [(2.0, 2.0, 2.0)], 4, 10)
    sim = RodSim(w, precision="fp64")
    f0 = fluid((8, 8, 8), 11)
    lat = Lattice(f0, tau=0.8)
    with pytest.raises(RodError) as e:
        sim.lbm_cycles(lat, 3, 1)  # dt = 1/4, not 1/3
    assert e.value.code == ROD_E_INVALID
    with pytest.raises(RodError) as e:
        sim.lbm_cycles(lat, 0, 1)
    assert e.value.code == ROD_E_INVALID
    sim.lbm_cycles(lat, 4, 0)  # nothing to do
    assert sim.state()["step"] == 0
    sim.free(); lat.free()


def carpet(nsub, seed, bottom=1.2):
    """A 3 x 3 carpet of cilia (6 to 10 particles, lattice units) standing on
    clamped bases near the bottom wall, the middle one's tip driven (turned
    about z), with velocities on the fixed particles that the coupling must
    ignore, in a field turning in the x-z plane (a table of 8 rows)."""
    rng = np.random.default_rng(seed)
    lens = list(rng.integers(6, 11, 9))
    origins = [(3.0 + 2.5 * (r % 3), 3.5 + 2.5 * (r // 3), bottom) for r in range(9)]
    x, off, mem = workloads.straight_rods(lens, origins, (0, 0, 1))
    n = x.shape[0]
    bc = np.zeros(n, np.int8)
    bc[off[:-1]] = 1
    bc[off[5] - 1] = 2  # tip of rod 4
    ph = 2 * np.pi * np.arange(8) / 8
    field = np.zeros((8, 1, 12))
    field[:, 0, 0], field[:, 0, 2] = 0.3 * np.cos(ph), 0.3 * np.sin(ph)
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (9, 1)),
                        np.tile([0, 0, 0.05], (n, 1)), bc, field, damping=0.0, dt=1.0 / nsub,
                        drive_axis=np.array([0.0, 0.0, 1.0]), drive_period=40, precision="fp64")
    w["x0"] = x + rng.normal(0, 0.02, x.shape) * (bc == 0)[:, None]
    w["v0"] = 0.01 * rng.normal(size=(n, 3))  # fixed particles' velocities included
    return w


@pytest.mark.parametrize("walls,lid", [(1, (0.0, 0.0)), (1, (0.002, 0.0)), (2, (0.0, 0.0))])
def test_carpet_between_walls(walls, lid):
    """Cilia on clamped bases 1.2 lattice units above a no-slip bottom (their
    stencils reach past it), a driven tip and a turning field: in a channel
    with no-slip walls (one of them moving), and under a free-slip top (the
    paper's cilia pumping box)."""
    nsub, tau = 4, 0.8
    w = carpet(nsub, 21)
    f0 = fluid((12, 12, 14), 22)
    st, f = run_gpu(w, f0, 3, nsub, tau, walls=walls, lid=lid)
    fixed = w["bc"] != 0
    np.testing.assert_array_equal(st["x"][w["bc"] == 1], w["x0"][w["bc"] == 1])
    assert np.all(st["v"][fixed] == 0)
    compare(st, f, w, f0, 3, nsub, tau, walls=walls, lid=lid)


def test_carpet_in_a_periodic_lattice_with_fixed_particles():
    """The same carpet in a lattice periodic in every axis (its stencils wrap
    to the top): clamped and driven particles carry the penalty force of
    their stored velocity into the fluid as the oracle's coupled run does."""
    nsub, tau = 4, 0.8
    w = carpet(nsub, 23, bottom=0.6)
    f0 = fluid((12, 12, 14), 24)
    st, f = run_gpu(w, f0, 3, nsub, tau)
    compare(st, f, w, f0, 3, nsub, tau)
