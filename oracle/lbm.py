"""Plain FP64 lattice Boltzmann oracle (D3Q19, BGK, Guo forcing).

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests may
use it. It shares no code with the GPU library.

Follows the paper's fluid solver (Methods, "Lattice Boltzmann method"): the
populations relax towards the second-order equilibrium with one relaxation
time tau (BGK), a uniform body force enters through Guo's forcing term with the
half-force velocity shift, and streaming moves each population one link. Axes
are periodic; the z axis may instead be bounded by halfway bounce-back walls
at z = -1/2 and z = nz - 1/2 (a population that would leave through a wall
comes back reversed at the node it left). Lattice units: dx = dt = 1,
c_s^2 = 1/3, kinematic viscosity nu = (tau - 1/2) / 3.

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


def equilibrium(rho, u):
    """f_i^eq = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u); rho [..], u [3, ..]."""
    cu = np.einsum("id,d...->i...", C.astype(np.float64), u)
    uu = np.sum(u * u, axis=0)
    return W.reshape((19,) + (1,) * rho.ndim) * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)


def moments(f, g):
    """Density and velocity with the half-force shift: rho u = sum_i f_i c_i + g/2
    (g: body force density, [3])."""
    rho = f.sum(axis=0)
    mom = np.einsum("id,i...->d...", C.astype(np.float64), f)
    u = (mom + 0.5 * np.asarray(g, float).reshape(3, 1, 1, 1)) / rho
    return rho, u


def collide(f, tau, g):
    """BGK relaxation plus Guo's forcing term
    F_i = (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i . u) c_i] . g."""
    rho, u = moments(f, g)
    feq = equilibrium(rho, u)
    g = np.asarray(g, float).reshape(3, 1, 1, 1)
    Cf = C.astype(np.float64)
    cu = np.einsum("id,d...->i...", Cf, u)
    cg = np.einsum("id,d...->i...", Cf, g * np.ones_like(u))
    ug = np.sum(u * g, axis=0)
    Fi = (1 - 0.5 / tau) * W.reshape(19, 1, 1, 1) * (3 * (cg - ug) + 9 * cu * cg)
    return f - (f - feq) / tau + Fi


def stream(fs, walls):
    """Each population moves one link along c_i (periodic wrap); with walls,
    the populations that would cross z = -1/2 or z = nz - 1/2 are reflected
    into the opposite direction at the node they left."""
    out = np.empty_like(fs)
    nz = fs.shape[1]
    for i in range(19):
        cx, cy, cz = C[i]
        out[i] = np.roll(fs[i], shift=(cz, cy, cx), axis=(0, 1, 2))
    if walls:
        for i in range(19):
            cz = C[i][2]
            if cz == 1:    # left through the top wall: back at z = nz - 1 as OPP[i]
                out[OPP[i], nz - 1] = fs[i, nz - 1]
            elif cz == -1:  # left through the bottom wall: back at z = 0 as OPP[i]
                out[OPP[i], 0] = fs[i, 0]
    return out


def run(f, nsteps, tau, g=(0.0, 0.0, 0.0), walls=False):
    """nsteps of collide then stream from populations f [19, nz, ny, nx]."""
    f = np.array(f, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        f = stream(collide(f, tau, g), walls)
    return f
