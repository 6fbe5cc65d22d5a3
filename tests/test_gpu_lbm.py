"""The lattice Boltzmann kernel (include/lbm.h) against the FP64 oracle:
populations after many steps from an off-equilibrium start, with and without
bounce-back walls and body force, on boxes with ragged and single-cell sides,
the moments, and force-driven Poiseuille flow against its closed form."""
import numpy as np
import pytest

from oracle import lbm
from paper_2603_27279_amd import Lattice

pytestmark = pytest.mark.gpu


def start(shape, seed):
    rng = np.random.default_rng(seed)
    f = lbm.equilibrium(1 + 0.05 * rng.random(shape), 0.03 * rng.normal(size=(3,) + shape))
    return f + 1e-3 * rng.random(f.shape) * lbm.W.reshape(19, 1, 1, 1)


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape", [(7, 6, 9), (20, 33, 47), (5, 1, 1), (1, 3, 2)])
def test_populations_match_oracle(shape, walls):
    if walls and shape[0] < 2:
        pytest.skip("a walled box needs cells between the walls in z")
    f0 = start(shape, sum(shape))
    g = (2e-5, -1e-5, 3e-5)
    lat = Lattice(f0, tau=0.7, force=g, walls_z=walls)
    steps = 30
    lat.step(steps)
    got = lat.populations().cpu().numpy()
    want = lbm.run(f0, steps, 0.7, g=g, walls=walls)
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
