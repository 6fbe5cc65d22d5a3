"""The lattice Boltzmann kernel (include/lbm.h) against the FP64 oracle:
populations after many steps from an off-equilibrium start, periodic, between
no-slip walls (one of them moving), and under a free-slip top, with a body
force, on boxes with ragged and single-cell sides; the moments; force-driven
Poiseuille flow in a full and a half channel and Couette flow under a moving
lid against their closed forms."""
import numpy as np
import pytest

from oracle import lbm
from paper_2603_27279_amd import Lattice

pytestmark = pytest.mark.gpu


def start(shape, seed):
    rng = np.random.default_rng(seed)
    f = lbm.equilibrium(1 + 0.05 * rng.random(shape), 0.03 * rng.normal(size=(3,) + shape))
    return f + 1e-3 * rng.random(f.shape) * lbm.W.reshape(19, 1, 1, 1)


# every lattice shape with periodic z; the walled variants (no-slip bottom and
# top, a moving lid, a free-slip top) on shapes with cells between the walls
CASES = [(shape, walls, lid)
         for walls, lid in [(0, (0.0, 0.0)), (1, (0.0, 0.0)), (1, (0.02, -0.01)), (2, (0.0, 0.0))]
         for shape in [(7, 6, 9), (20, 33, 47), (5, 1, 1), (1, 3, 2)]
         if not (walls and shape[0] < 2)]


@pytest.mark.parametrize("shape,walls,lid", CASES)
def test_populations_match_oracle(shape, walls, lid):
    f0 = start(shape, sum(shape))
    g = (2e-5, -1e-5, 3e-5)
    lat = Lattice(f0, tau=0.7, force=g, walls_z=walls, lid=lid)
    steps = 30
    lat.step(steps)
    got = lat.populations().cpu().numpy()
    want = lbm.run(f0, steps, 0.7, g=g, walls=walls, lid=lid)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    rho, u = lat.moments()
    rw, uw = lbm.moments(want, g)
    np.testing.assert_allclose(rho.cpu().numpy(), rw, rtol=1e-13)
    np.testing.assert_allclose(u.cpu().numpy(), uw, rtol=1e-9, atol=1e-14)
    lat.free()


def test_poiseuille_on_the_gpu():
    nz = 16
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3
    gx = 1e-6
    f0 = lbm.equilibrium(np.ones((nz, 4, 4)), np.zeros((3, nz, 4, 4)))
    lat = Lattice(f0, tau=tau, force=(gx, 0, 0), walls_z=True)
    lat.step(20000)
    _, u = lat.moments()
    u = u.cpu().numpy()
    zz = np.arange(nz)
    want = gx / (2 * nu) * (zz + 0.5) * (nz - 0.5 - zz)
    np.testing.assert_allclose(u[0, :, 2, 1], want, rtol=1e-8)
    # no flow across: the transverse components stay at the rounding of sums of
    # populations of order one
    assert np.max(np.abs(u[1:])) <= 1e-14
    lat.free()


def test_half_channel_and_couette_on_the_gpu():
    """A no-slip bottom under a free-slip top with a body force gives the lower
    half of the Poiseuille parabola of a channel of height 2 nz; no-slip walls
    with the top one moving at U give the linear Couette profile."""
    nz = 10
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3
    gx = 1e-6
    f0 = lbm.equilibrium(np.ones((nz, 4, 4)), np.zeros((3, nz, 4, 4)))
    lat = Lattice(f0, tau=tau, force=(gx, 0, 0), walls_z=2)
    lat.step(25000)
    u = lat.moments()[1].cpu().numpy()
    zz = np.arange(nz)
    np.testing.assert_allclose(u[0, :, 1, 3], gx / (2 * nu) * (zz + 0.5) * (2 * nz - 0.5 - zz),
                               rtol=1e-8)
    lat.free()
    U = 1e-3
    lat = Lattice(f0, tau=0.9, walls_z=1, lid=(0.0, U))
    lat.step(15000)
    u = lat.moments()[1].cpu().numpy()
    np.testing.assert_allclose(u[1, :, 2, 0], U * (zz + 0.5) / nz, rtol=1e-9)
    lat.free()
