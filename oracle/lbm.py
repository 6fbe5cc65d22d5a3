"""Plain FP64 lattice Boltzmann oracle (D3Q19, BGK, Guo forcing).

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests may
use it. It shares no code with the GPU library.

Follows the paper's fluid solver (Methods, "Lattice Boltzmann method"): the
populations relax towards the second-order equilibrium with one relaxation
time tau (BGK), a uniform body force enters through Guo's forcing term with the
half-force velocity shift, and streaming moves each population one link. Axes
are periodic; the z axis may instead be bounded by walls at z = -1/2 and
z = nz - 1/2 (walls = 1: no-slip at both, halfway bounce-back: a population
that would leave through a wall comes back reversed at the node it left; the
top wall may move tangentially with velocity lid = (u_x, u_y), which takes
6 w_i rho (c_i . lid) from the reflected population, rho the node's density;
walls = 2: a no-slip bottom and a free-slip top, where a population comes back
with its z component reversed and its tangential components kept). Results,
"Fluid pumping by magnetic cilia arrays", bounds its fluid by a no-slip bottom
and a free-slip top; "Fluid-structure interaction" by no-slip channel walls.
Lattice units: dx = dt = 1, c_s^2 = 1/3, kinematic viscosity nu = (tau - 1/2) / 3.

Step order: moments, collision with forcing (post-collision populations),
streaming. Arrays are [19, nz, ny, nx].
"""
import numpy as np

# D3Q19 velocities: rest, 6 faces, 12 edges; weights 1/3, 1/18, 1/36.
C = np.array([[0, 0, 0],
              [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
              [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
              [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
OPP = np.array([0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17])
# direction with the z component reversed (specular reflection at a free-slip wall)
FLIPZ = np.array([int(np.flatnonzero(np.all(C == C[i] * np.array([1, 1, -1]), axis=1))[0])
                  for i in range(19)])


def equilibrium(rho, u):
    """f_i^eq = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u); rho [..], u [3, ..]."""
    cu = np.einsum("id,d...->i...", C.astype(np.float64), u)
    uu = np.sum(u * u, axis=0)
    return W.reshape((19,) + (1,) * rho.ndim) * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)


def _force(g, shape):
    """A uniform force [3] or a force field [3, nz, ny, nx], as a field."""
    g = np.asarray(g, float)
    return g.reshape(3, 1, 1, 1) * np.ones((1,) + shape) if g.ndim == 1 else g


def moments(f, g):
    """Density and velocity with the half-force shift: rho u = sum_i f_i c_i + g/2
    (g: body force density, uniform [3] or a field [3, nz, ny, nx])."""
    rho = f.sum(axis=0)
    mom = np.einsum("id,i...->d...", C.astype(np.float64), f)
    u = (mom + 0.5 * _force(g, f.shape[1:])) / rho
    return rho, u


def collide(f, tau, g):
    """BGK relaxation plus Guo's forcing term
    F_i = (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i . u) c_i] . g."""
    rho, u = moments(f, g)
    feq = equilibrium(rho, u)
    g = _force(g, f.shape[1:])
    Cf = C.astype(np.float64)
    cu = np.einsum("id,d...->i...", Cf, u)
    cg = np.einsum("id,d...->i...", Cf, g)
    ug = np.sum(u * g, axis=0)
    Fi = (1 - 0.5 / tau) * W.reshape(19, 1, 1, 1) * (3 * (cg - ug) + 9 * cu * cg)
    return f - (f - feq) / tau + Fi


def stream(fs, walls, rho=None, lid=(0.0, 0.0)):
    """Each population moves one link along c_i (periodic wrap). With walls
    (see the module text) the populations that would cross z = -1/2 come back
    reversed at the node they left; those that would cross z = nz - 1/2 come
    back reversed (walls = 1, less 6 w_i rho (c_i . lid), rho [nz, ny, nx] the
    nodes' densities) or with their z component reversed (walls = 2)."""
    out = np.empty_like(fs)
    nz = fs.shape[1]
    walls = int(walls)
    for i in range(19):
        cx, cy, cz = C[i]
        out[i] = np.roll(fs[i], shift=(cz, cy, cx), axis=(0, 1, 2))
    if walls:
        for i in range(19):
            cz = C[i][2]
            if cz == 1 and walls == 2:  # free-slip top: back at z = nz - 1, z reversed
                out[FLIPZ[i], nz - 1] = fs[i, nz - 1]
            elif cz == 1:  # no-slip top: back at z = nz - 1 as OPP[i]
                cl = C[i][0] * lid[0] + C[i][1] * lid[1]
                out[OPP[i], nz - 1] = fs[i, nz - 1] - 6.0 * W[i] * rho[nz - 1] * cl
            elif cz == -1:  # left through the bottom wall: back at z = 0 as OPP[i]
                out[OPP[i], 0] = fs[i, 0]
    return out


def run(f, nsteps, tau, g=(0.0, 0.0, 0.0), walls=False, lid=(0.0, 0.0)):
    """nsteps of collide then stream from populations f [19, nz, ny, nx];
    walls = 0 (or False) periodic, 1 (or True) no-slip walls in z with an
    optional lid velocity of the top one, 2 no-slip bottom and free-slip top."""
    f = np.array(f, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        rho = f.sum(axis=0)
        f = stream(collide(f, tau, g), walls, rho, lid)
    return f


# ---------------------------------------------------------------- immersed boundary
# Methods, "Immersed boundary coupling": fluid velocity interpolated at each
# particle with a smoothed discrete delta, and the reaction force spread back
# with the same delta. The paper does not name its delta; this is Peskin's
# four-point function (phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4 r^2)) / 8 for
# |r| <= 1, (5 - 2|r| - sqrt(-7 + 12|r| - 4 r^2)) / 8 for 1 <= |r| <= 2,
# 0 beyond), a product over the three axes, with nodes at integer
# coordinates, periodic in x and y, and in z unless the lattice has walls
# there: then the nodes beyond a wall (z < 0 or z > nz - 1) take no part, so
# the fluid velocity beyond a wall counts as zero in the interpolation and
# the share of a spread force that would fall there goes to the wall.


def peskin4(r):
    r = np.abs(np.asarray(r, float))
    out = np.zeros_like(r)
    a = r <= 1
    out[a] = (3 - 2 * r[a] + np.sqrt(1 + 4 * r[a] - 4 * r[a] ** 2)) / 8
    b = (r > 1) & (r <= 2)
    out[b] = (5 - 2 * r[b] - np.sqrt(-7 + 12 * r[b] - 4 * r[b] ** 2)) / 8
    return out


def stencil(X, shape, walls=0):
    """The 4 x 4 x 4 lattice nodes around position X (x, y, z) and their
    weights: lists of (iz, iy, ix) index arrays (wrapped) and weights; with
    walls in z, nodes beyond them get weight 0 (their index is clamped)."""
    nz, ny, nx = shape
    base = np.floor(np.asarray(X, float)).astype(np.int64) - 1  # x, y, z
    o = np.arange(4)
    wx = peskin4(base[0] + o - X[0])
    wy = peskin4(base[1] + o - X[1])
    wz = peskin4(base[2] + o - X[2])
    ix, iy = (base[0] + o) % nx, (base[1] + o) % ny
    if walls:
        zz = base[2] + o
        wz = np.where((zz >= 0) & (zz < nz), wz, 0.0)
        iz = np.clip(zz, 0, nz - 1)
    else:
        iz = (base[2] + o) % nz
    W = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
    return np.ix_(iz, iy, ix), W


def interpolate(u, X, walls=0):
    """U(X) = sum over nodes of u(x) delta(x - X), u [3, nz, ny, nx], X [P, 3]."""
    shape = u.shape[1:]
    out = np.zeros((len(X), 3))
    for p, Xp in enumerate(X):
        idx, W = stencil(Xp, shape, walls)
        for d in range(3):
            out[p, d] = np.sum(u[d][idx] * W)
    return out


def spread(F, X, shape, walls=0):
    """Force density field [3, nz, ny, nx] of point forces F [P, 3] at X [P, 3]."""
    g = np.zeros((3,) + tuple(shape))
    for p, Xp in enumerate(X):
        idx, W = stencil(Xp, shape, walls)
        for d in range(3):
            np.add.at(g[d], idx, F[p, d] * W)
    return g


def coupled(w, f, ncycles, nsub, tau, g=(0.0, 0.0, 0.0), state=None, walls=0,
            lid=(0.0, 0.0)):
    """Rods of workload w immersed in the lattice f (Methods, "Immersed boundary
    coupling"), positions in lattice units, the rods' dt = 1 / nsub of the fluid
    step. Each cycle: the fluid velocity (with the half-force shift of the
    uniform force g) is interpolated at every particle once; then nsub rod
    steps, each evaluation adding the penalty force m_p (U_p - v_p) (fluid time
    step 1) and each spreading the reaction -F_p / nsub at the particles'
    positions of that evaluation; then one fluid step with g plus the spread
    forces. The state before the first cycle carries no penalty force.
    ``walls``, ``lid``: the lattice's walls in z (see ``run``) and the stencil
    truncated at them. Returns (rod state, populations)."""
    import oracle as rod_oracle
    shape = f.shape[1:]
    st = rod_oracle.run(w, 0) if state is None else state
    for _ in range(ncycles):
        _, u = moments(f, g)
        U = interpolate(u, st["x"], walls)
        wf = dict(w, fluid_u=U, fluid_dt=1.0)
        field = np.zeros((3,) + tuple(shape))
        for _s in range(nsub):
            st = rod_oracle.run(wf, 1, state=st)
            field += spread(-st["fluid_F"] / nsub, st["x"], shape, walls)
        f = run(f, 1, tau, g=_force(g, shape) + field, walls=walls, lid=lid)
    return st, f
