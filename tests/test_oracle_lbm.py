"""Pins of the lattice Boltzmann oracle (D3Q19, BGK, Guo forcing; Methods,
"Lattice Boltzmann method") against closed forms: the equilibrium's moments,
exact conservation of mass and of momentum plus the applied force, the decay
rate of a Taylor-Green vortex, nu (kx^2 + ky^2) with nu = (tau - 1/2)/3, and
force-driven Poiseuille flow between halfway bounce-back walls at the
relaxation time where that scheme reproduces the parabola exactly."""
import numpy as np
import pytest

from oracle import lbm


def test_equilibrium_moments():
    rng = np.random.default_rng(1)
    rho = 1 + 0.1 * rng.random((3, 4, 5))
    u = 0.05 * rng.normal(size=(3, 3, 4, 5))
    f = lbm.equilibrium(rho, u)
    C = lbm.C.astype(float)
    np.testing.assert_allclose(f.sum(0), rho, rtol=1e-14)
    np.testing.assert_allclose(np.einsum("id,i...->d...", C, f), rho * u, rtol=1e-13, atol=1e-16)
    P = np.einsum("id,ie,i...->de...", C, C, f)
    want = rho * (np.einsum("d...,e...->de...", u, u) + np.eye(3)[:, :, None, None, None] / 3)
    np.testing.assert_allclose(P, want, rtol=1e-13, atol=1e-16)
    assert lbm.W.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_array_equal(lbm.C[lbm.OPP], -lbm.C)


def test_uniform_equilibrium_is_a_fixed_point():
    f = lbm.equilibrium(np.full((4, 5, 6), 1.3), np.zeros((3, 4, 5, 6)) + np.array([0.02, -0.01, 0.03]).reshape(3, 1, 1, 1))
    g = lbm.run(f, 20, tau=0.8)
    np.testing.assert_allclose(g, f, rtol=1e-14, atol=1e-17)


def test_mass_and_momentum_balance():
    rng = np.random.default_rng(2)
    shape = (6, 5, 7)
    f = lbm.equilibrium(1 + 0.05 * rng.random(shape), 0.03 * rng.normal(size=(3,) + shape))
    f += 1e-4 * rng.random(f.shape)  # off equilibrium
    g = np.array([1e-5, -2e-5, 3e-5])
    t = 25
    out = lbm.run(f, t, tau=0.7, g=g)
    C = lbm.C.astype(float)
    ncell = np.prod(shape)
    assert abs(out.sum() - f.sum()) <= 1e-12 * f.sum()
    P0 = np.einsum("id,i...->d...", C, f).reshape(3, -1).sum(1)
    P1 = np.einsum("id,i...->d...", C, out).reshape(3, -1).sum(1)
    np.testing.assert_allclose(P1 - P0, t * ncell * g, rtol=1e-9, atol=1e-13)


def test_taylor_green_decay():
    n, tau, U = 32, 0.8, 1e-3
    nu = (tau - 0.5) / 3
    k = 2 * np.pi / n
    z, y, x = np.meshgrid(np.arange(2), np.arange(n), np.arange(n), indexing="ij")
    u = np.zeros((3, 2, n, n))
    u[0] = U * np.sin(k * x) * np.cos(k * y)
    u[1] = -U * np.cos(k * x) * np.sin(k * y)
    f = lbm.equilibrium(np.ones((2, n, n)), u)
    t = 300
    out = lbm.run(f, t, tau)
    _, ut = lbm.moments(out, (0, 0, 0))
    amp0 = np.sum(u[0] * u[0])
    amp1 = np.sum(ut[0] * u[0])
    rate = -np.log(amp1 / amp0) / t
    assert rate == pytest.approx(2 * nu * k * k, rel=5e-3)


def test_poiseuille_between_bounce_back_walls():
    """Body force g along x, walls at z = -1/2 and nz - 1/2: the steady
    profile is u(z) = g / (2 nu) (z + 1/2) (nz - 1/2 - z), exactly so with
    halfway bounce-back at tau = 1/2 + sqrt(3/16)."""
    nz = 12
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3
    gx = 1e-6
    f = lbm.equilibrium(np.ones((nz, 2, 2)), np.zeros((3, nz, 2, 2)))
    out = lbm.run(f, 12000, tau, g=(gx, 0, 0), walls=True)
    _, u = lbm.moments(out, (gx, 0, 0))
    zz = np.arange(nz)
    want = gx / (2 * nu) * (zz + 0.5) * (nz - 0.5 - zz)
    np.testing.assert_allclose(u[0, :, 0, 0], want, rtol=1e-8)
    # any other relaxation time moves the effective wall (a slip that grows with tau)
    out2 = lbm.run(f, 12000, 1.5, g=(gx, 0, 0), walls=True)
    _, u2 = lbm.moments(out2, (gx, 0, 0))
    want2 = gx / (2 * (1.0 / 3)) * (zz + 0.5) * (nz - 0.5 - zz)
    assert np.max(np.abs(u2[0, :, 0, 0] / want2 - 1)) > 1e-3


def test_peskin_delta_moments():
    """The four-point delta sums to one and has zero first moment at any
    offset, so a uniform field interpolates exactly and a spread point force
    keeps its total and its point of application."""
    rng = np.random.default_rng(3)
    shape = (9, 8, 10)
    for X in rng.uniform(0, 8, (6, 3)):
        idx, W = lbm.stencil(X, shape)
        assert W.sum() == pytest.approx(1.0, abs=1e-14)
        o = np.arange(4)
        base = np.floor(X).astype(int) - 1
        for d, sh in ((0, (1, 1, 4)), (1, (1, 4, 1)), (2, (4, 1, 1))):  # W is [z, y, x]
            pos = (base[d] + o).reshape(sh)
            assert abs(np.sum(W * (pos - X[d]))) <= 1e-14
        U0 = np.array([0.01, -0.02, 0.03])
        u = U0.reshape(3, 1, 1, 1) * np.ones((3,) + shape)
        np.testing.assert_allclose(lbm.interpolate(u, X[None]), U0[None], rtol=1e-14)
        F = rng.normal(size=(1, 3))
        gfield = lbm.spread(F, X[None], shape)
        np.testing.assert_allclose(gfield.reshape(3, -1).sum(1), F[0], rtol=1e-13)


def test_coupled_cycle_conserves_momentum():
    """Free rods in a periodic lattice: bonds and dipoles are internal, the
    penalty force is paid back to the fluid, so P_rods + P_fluid +
    (dt/2) sum F_p (the velocity-Verlet share of the last evaluation's penalty
    force not yet in the rods' velocities) stays constant; the exchange is
    real (both momenta change)."""
    import workloads
    rng = np.random.default_rng(4)
    n = 6
    x, off, mem = workloads.straight_rods([n, n], [(3.2, 4.1, 4.3), (3.7, 6.4, 5.1)], (1, 0, 0))
    nsub = 4
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (2, 1)), np.tile([0, 0, 0.05], (2 * n, 1)),
                        np.zeros(2 * n, np.int8), workloads._field_const(1, (0, 0, 0.2)),
                        damping=0.0, dt=1.0 / nsub, precision="fp64")
    w["v0"] = 0.01 * rng.normal(size=(2 * n, 3))
    shape = (12, 12, 14)
    f = lbm.equilibrium(np.ones(shape), 0.005 * rng.normal(size=(3,) + shape))
    import oracle
    m, _ = oracle.mass(w)
    Cf = lbm.C.astype(float)

    def Q(st, f):
        Pf = np.einsum("id,i...->d...", Cf, f).reshape(3, -1).sum(1)
        Pr = (m[:, None] * st["v"]).sum(0)
        Fp = st.get("fluid_F", np.zeros((2 * n, 3))).sum(0)
        return Pf + Pr + 0.5 * w["dt"] * Fp, Pf, Pr

    st0 = oracle.run(w, 0)
    q0, pf0, pr0 = Q(st0, f)
    st, f1 = lbm.coupled(w, f, 3, nsub, tau=0.8, state=st0)
    q1, pf1, pr1 = Q(st, f1)
    np.testing.assert_allclose(q1, q0, rtol=0, atol=1e-13 * np.abs(pf0).sum())
    assert np.max(np.abs(pr1 - pr0)) > 1e-4 * np.max(np.abs(pr0))


def test_half_channel_poiseuille_under_a_free_slip_top():
    """No-slip bottom at z = -1/2, free-slip top at z = nz - 1/2 (walls = 2):
    specular reflection at the top makes the lattice the lower half of a
    bounce-back channel of height 2 nz mirrored about z = nz - 1/2, so the
    steady profile is u(z) = g / (2 nu) (z + 1/2) (2 nz - 1/2 - z), exact at
    tau = 1/2 + sqrt(3/16) as for the full channel; its shear vanishes at the
    top plane."""
    nz = 8
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3
    gx = 1e-6
    f = lbm.equilibrium(np.ones((nz, 2, 2)), np.zeros((3, nz, 2, 2)))
    out = lbm.run(f, 20000, tau, g=(gx, 0, 0), walls=2)
    _, u = lbm.moments(out, (gx, 0, 0))
    zz = np.arange(nz)
    want = gx / (2 * nu) * (zz + 0.5) * (2 * nz - 0.5 - zz)
    np.testing.assert_allclose(u[0, :, 0, 0], want, rtol=1e-8)
    # the full channel of height 2 nz gives the same lower half, population by population
    f2 = lbm.equilibrium(np.ones((2 * nz, 2, 2)), np.zeros((3, 2 * nz, 2, 2)))
    full = lbm.run(f2, 300, tau, g=(gx, 0, 0), walls=1)
    half = lbm.run(f, 300, tau, g=(gx, 0, 0), walls=2)
    np.testing.assert_allclose(half, full[:, :nz], rtol=1e-13, atol=1e-19)


def test_free_slip_top_keeps_mass():
    """Both walls of walls = 2 send every population back into the lattice,
    so mass is exact from a random non-equilibrium state."""
    rng = np.random.default_rng(6)
    shape = (6, 4, 5)
    f = lbm.equilibrium(1 + 0.05 * rng.random(shape), 0.02 * rng.normal(size=(3,) + shape))
    out = lbm.run(f, 40, tau=0.9, walls=2)
    assert abs(out.sum() - f.sum()) <= 1e-12 * f.sum()


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.3])
def test_couette_flow_under_a_moving_lid(tau):
    """No-slip walls with the top one moving at U along x (walls = 1, lid):
    the steady profile is linear, u(z) = U (z + 1/2) / nz, for any tau (the
    moving halfway bounce-back wall reproduces a linear profile exactly)."""
    nz, U = 10, 1e-3
    f = lbm.equilibrium(np.ones((nz, 2, 2)), np.zeros((3, nz, 2, 2)))
    out = lbm.run(f, 12000, tau, walls=1, lid=(U, 0.0))
    _, u = lbm.moments(out, (0, 0, 0))
    zz = np.arange(nz)
    np.testing.assert_allclose(u[0, :, 0, 0], U * (zz + 0.5) / nz, rtol=1e-9)
    np.testing.assert_allclose(u[2], 0.0, atol=1e-10 * U)


def test_stencil_at_walls():
    """With walls in z the stencil drops the nodes beyond them: away from the
    walls (z in [2, nz - 3]) interpolation and spreading are the periodic
    ones; near a wall a uniform field interpolates to itself times the weight
    left inside, and a spread force keeps that share of its total."""
    rng = np.random.default_rng(7)
    shape = (9, 8, 10)
    U0 = np.array([0.01, -0.02, 0.03])
    u = U0.reshape(3, 1, 1, 1) * np.ones((3,) + shape)
    for z in (2.0, 3.7, 5.9):
        X = np.array([rng.uniform(0, 10), rng.uniform(0, 8), z])
        F = rng.normal(size=(1, 3))
        np.testing.assert_array_equal(lbm.spread(F, X[None], shape, walls=1),
                                      lbm.spread(F, X[None], shape))
        np.testing.assert_array_equal(lbm.interpolate(u, X[None], walls=1),
                                      lbm.interpolate(u, X[None]))
    for z in (-0.3, 0.4, 0.9, 7.5, 8.2):
        X = np.array([rng.uniform(0, 10), rng.uniform(0, 8), z])
        _, W = lbm.stencil(X, shape, walls=1)
        inside = W.sum()
        zz = np.floor(z) - 1 + np.arange(4)
        want = np.sum(lbm.peskin4(zz - z) * ((zz >= 0) & (zz < 9)))
        assert inside == pytest.approx(want, abs=1e-15) and inside < 1.0
        np.testing.assert_allclose(lbm.interpolate(u, X[None], walls=1), inside * U0[None], rtol=1e-13)
        F = rng.normal(size=(1, 3))
        g = lbm.spread(F, X[None], shape, walls=1)
        np.testing.assert_allclose(g.reshape(3, -1).sum(1), inside * F[0], rtol=1e-12)
