"""Seeded synthetic workloads for the magneto-elastic rod loop.

This module holds geometry, seeds and input layout only. It contains none of the
model's mechanics (no spring constants, masses, bond topology, forces or
integration): the oracle and the GPU library each derive those from the fields
below on their own.

Every workload is a plain ``dict`` of numpy arrays and scalars:

================  ===========================  =====================================
key               dtype / shape                meaning
================  ===========================  =====================================
n                 int                          number of particles N
rod_offset        int32 [R+1]                  rod r owns particles rod_offset[r]..rod_offset[r+1]-1
rod_member        int32 [R]                    ensemble member of each rod (members never interact)
n_members         int                          M
rod_params        float64 [R, 4]               particle diameter d, density rho, Young E, Poisson nu
x_ref             float64 [N, 3]               unperturbed reference lattice (bonds are built from it)
x0, v0, w0        float64 [N, 3]               initial position, velocity, angular velocity
q0                float64 [N, 4]               initial orientation quaternion (w, x, y, z)
m_body            float64 [N, 3]               dipole moment in the body frame
bc                int8 [N]                     0 free, 1 clamped, 2 driven (position fixed, prescribed rotation)
drive_axis        float64 [3]                  rotation axis of driven particles (unit)
drive_period      int                          steps per full turn of driven particles (0: none)
field             float64 [L, M, 12]           per step (index n mod L) and member: B0 (3) then G (3x3,
                                               row-major); the external field is B(x) = B0 + G x
ext_force         float64 [N, 3] or None       constant external force per particle
ext_torque        float64 [N, 3] or None       constant external torque per particle
dt, damping       float                        time step; global viscous damping coefficient c
mu0_4pi           float                        dipole prefactor mu0 / (4 pi)
dipole_on         bool                         dipole-dipole interaction within a member
dipole_cutoff     float                        0: every pair of a member; > 0: pairs closer than this
box               float64 [3] or None          periodic box lengths: the dipole sum is then the Ewald
                                               sum of each member's periodic system (None: open)
ewald_alpha       float                        Ewald splitting parameter (with a box)
ewald_rcut        float                        Ewald real-space cutoff (with a box)
ewald_kmax        int                          Ewald reciprocal vectors 2 pi n / L, 0 < |n|^2 <= kmax^2
contact_on        bool                         contact between non-excluded pairs
contact_model     str                          "hookean" (normal, k_contact) or "hertz_mindlin"
contact_hm        float64 [5] or None          Hertz-Mindlin: contact modulus E, Poisson nu, friction
                                               mu, normal and tangential damping g_n, g_t
k_contact         float                        Hookean contact stiffness
r_contact         float                        contact distance (pairs closer than this interact)
bond_damping      float64 [R, 4] or None       bond damping factors g_r, g_s, g_t, g_b per rod
exclude_depth     int                          same-rod pairs with |i-j| <= depth never contact
steps             int                          run length of the workload
precision         str                          "fp64" or "mixed" (path the workload is specified for)
================  ===========================  =====================================

Perturbation recipe: positions are ``x_ref + N(0, sigma^2)`` per component on
free particles, drawn as one ``(N, 3)`` normal array from the workload's seed
after every other random draw of that workload.
"""
from __future__ import annotations

import numpy as np

__all__ = ["make", "CONFIGS", "straight_rods", "cilia_carpet", "rod_array",
           "ensemble", "adjoint_rod", "cantilever", "twisted_rod", "magnetic_helix",
           "helix_ramp_fields", "coiled_rods", "periodic_rods"]


def _field_const(n_members, b0, g=None, length=1):
    f = np.zeros((length, n_members, 12), dtype=np.float64)
    f[:, :, 0:3] = np.asarray(b0, dtype=np.float64)
    if g is not None:
        f[:, :, 3:12] = np.asarray(g, dtype=np.float64).reshape(9)
    return f


def _base(x_ref, rod_offset, rod_member, rod_params, m_body, bc, field, **kw):
    n = x_ref.shape[0]
    w = dict(
        n=int(n),
        rod_offset=np.asarray(rod_offset, dtype=np.int32),
        rod_member=np.asarray(rod_member, dtype=np.int32),
        n_members=int(np.max(rod_member)) + 1 if len(rod_member) else 0,
        rod_params=np.asarray(rod_params, dtype=np.float64).reshape(-1, 4),
        x_ref=np.ascontiguousarray(x_ref, dtype=np.float64),
        x0=np.ascontiguousarray(x_ref, dtype=np.float64).copy(),
        v0=np.zeros((n, 3)), w0=np.zeros((n, 3)),
        q0=np.tile(np.array([1.0, 0.0, 0.0, 0.0]), (n, 1)),
        m_body=np.ascontiguousarray(m_body, dtype=np.float64),
        bc=np.asarray(bc, dtype=np.int8),
        drive_axis=np.array([1.0, 0.0, 0.0]), drive_period=0,
        field=np.ascontiguousarray(field, dtype=np.float64),
        ext_force=None, ext_torque=None, bond_damping=None,
        contact_model="hookean", contact_hm=None, dipole_cutoff=0.0,
        box=None, ewald_alpha=0.0, ewald_rcut=0.0, ewald_kmax=0,
        dt=0.01, damping=0.1, mu0_4pi=1.0,
        dipole_on=True, contact_on=False, k_contact=10.0, r_contact=1.0,
        exclude_depth=1, steps=100, precision="fp64", name="custom",
    )
    w.update(kw)
    return w


def _perturb(w, rng, sigma):
    free = (w["bc"] == 0)
    noise = rng.normal(0.0, sigma, size=(w["n"], 3))
    w["x0"] = w["x_ref"] + noise * free[:, None]
    return w


def straight_rods(lengths, origins, axis, spacing=1.0, member=None):
    """Rods of ``lengths[r]`` particles starting at ``origins[r]`` along unit ``axis``."""
    axis = np.asarray(axis, dtype=np.float64)
    pts, offs = [], [0]
    for L, o in zip(lengths, origins):
        k = np.arange(L, dtype=np.float64)[:, None]
        pts.append(np.asarray(o, dtype=np.float64)[None, :] + spacing * k * axis[None, :])
        offs.append(offs[-1] + int(L))
    x = np.concatenate(pts, axis=0) if pts else np.zeros((0, 3))
    if member is None:
        member = np.zeros(len(lengths), dtype=np.int32)
    return x, np.asarray(offs, dtype=np.int32), np.asarray(member, dtype=np.int32)


def cantilever(n=20, seed=1, m=0.05, B=(0.0, 1.0, 0.0), sigma=1e-3, **kw):
    """One straight clamped rod of ``n`` unit spheres along +x (the plain FP64 case)."""
    rng = np.random.default_rng(seed)
    x, off, mem = straight_rods([n], [(0.0, 0.0, 0.0)], (1.0, 0.0, 0.0))
    bc = np.zeros(n, np.int8)
    bc[0] = 1
    mb = np.tile([m, 0.0, 0.0], (n, 1))
    w = _base(x, off, mem, [1.0, 1.0, 1.0, 0.5], mb, bc, _field_const(1, B),
              steps=1000, precision="fp64", name=f"cantilever_n{n}")
    w.update(kw)
    return _perturb(w, rng, sigma)


def twisted_rod(n=4096, seed=2, m=0.02, period=10_000, sigma=1e-3, **kw):
    """Clamped-clamped rod along +x; the far end turns about x once per ``period`` steps."""
    rng = np.random.default_rng(seed)
    x, off, mem = straight_rods([n], [(0.0, 0.0, 0.0)], (1.0, 0.0, 0.0))
    bc = np.zeros(n, np.int8)
    bc[0] = 1
    bc[n - 1] = 2
    mb = np.tile([m, 0.0, 0.0], (n, 1))
    w = _base(x, off, mem, [1.0, 1.0, 1.0, 0.5], mb, bc, _field_const(1, (0, 0, 0)),
              drive_axis=np.array([1.0, 0.0, 0.0]), drive_period=int(period),
              contact_on=True, k_contact=10.0, r_contact=1.0, exclude_depth=1,
              steps=20_000, precision="mixed", name=f"twisted_rod_n{n}")
    w.update(kw)
    return _perturb(w, rng, sigma)


def cilia_carpet(grid=(32, 32), pitch=8.0, len_range=(16, 128), seed=3, m=0.03,
                 period=2000, sigma=1e-3, **kw):
    """Rods clamped at z=0 on a square grid, along +z, lengths uniform in ``len_range``
    (inclusive); the field turns in the x-z plane with |B| = 1 once per ``period`` steps."""
    rng = np.random.default_rng(seed)
    gx, gy = grid
    R = gx * gy
    lengths = rng.integers(len_range[0], len_range[1] + 1, size=R)
    origins = [(pitch * i, pitch * j, 0.0) for i in range(gx) for j in range(gy)]
    x, off, mem = straight_rods(lengths, origins, (0.0, 0.0, 1.0))
    n = x.shape[0]
    bc = np.zeros(n, np.int8)
    bc[off[:-1]] = 1
    mb = np.tile([0.0, 0.0, m], (n, 1))
    ph = 2.0 * np.pi * np.arange(period) / period
    field = np.zeros((period, 1, 12))
    field[:, 0, 0] = np.cos(ph)
    field[:, 0, 2] = np.sin(ph)
    w = _base(x, off, mem, np.tile([1.0, 1.0, 1.0, 0.5], (R, 1)), mb, bc, field,
              contact_on=True, steps=10_000, precision="mixed",
              name=f"cilia_carpet_{gx}x{gy}")
    w.update(kw)
    return _perturb(w, rng, sigma)


def adjoint_rod(n=256, seed=4, m_sigma=0.05, B=(0.0, 0.0, 1.0), E=10.0, sigma=1e-3, **kw):
    """Clamped rod along +x with random body-frame dipoles and a random tip target
    inside the ball of radius 0.5 * (n - 1) around the clamp.

    Young's modulus defaults to 10: with E = 1, dipoles of this spread in a unit
    field turn neighbouring particles by up to pi relative to each other, where
    the short-arc central frame of the bond model flips and the run diverges."""
    rng = np.random.default_rng(seed)
    x, off, mem = straight_rods([n], [(0.0, 0.0, 0.0)], (1.0, 0.0, 0.0))
    bc = np.zeros(n, np.int8)
    bc[0] = 1
    mb = rng.normal(0.0, m_sigma, size=(n, 3))
    rad = 0.5 * (n - 1)
    while True:
        t = rng.uniform(-rad, rad, size=3)
        if np.dot(t, t) <= rad * rad:
            break
    w = _base(x, off, mem, [1.0, 1.0, E, 0.5], mb, bc, _field_const(1, B),
              steps=2000, precision="fp64", name=f"adjoint_rod_n{n}",
              target=t + x[0], tape_every=100)
    w.update(kw)
    return _perturb(w, rng, sigma)


def rod_array(grid=(32, 16), n_per_rod=512, pitch=2.0, seed=5, m=0.05, B_max=2.0,
              half_sweep=20_000, sigma=1e-3, **kw):
    """Parallel rods along +z clamped at z=0 on a lateral grid; B_z is swept as a
    triangle -B_max -> +B_max -> -B_max over 2 * half_sweep steps."""
    rng = np.random.default_rng(seed)
    gx, gy = grid
    R = gx * gy
    origins = [(pitch * i, pitch * j, 0.0) for i in range(gx) for j in range(gy)]
    x, off, mem = straight_rods([n_per_rod] * R, origins, (0.0, 0.0, 1.0))
    n = x.shape[0]
    bc = np.zeros(n, np.int8)
    bc[off[:-1]] = 1
    mb = np.tile([0.0, 0.0, m], (n, 1))
    s = np.arange(2 * half_sweep, dtype=np.float64)
    bz = np.where(s <= half_sweep, -B_max + 2 * B_max * s / half_sweep,
                  B_max - 2 * B_max * (s - half_sweep) / half_sweep)
    field = np.zeros((2 * half_sweep, 1, 12))
    field[:, 0, 2] = bz
    w = _base(x, off, mem, np.tile([1.0, 1.0, 1.0, 0.5], (R, 1)), mb, bc, field,
              contact_on=True, steps=2 * half_sweep, precision="mixed",
              name=f"rod_array_{gx}x{gy}x{n_per_rod}")
    w.update(kw)
    return _perturb(w, rng, sigma)


def ensemble(members=64, n=4096, seed=55, E_range=(0.5, 2.0), m_range=(0.01, 0.05),
             B=(0.0, 1.0, 0.0), sigma=1e-3, **kw):
    """``members`` independent clamped rods of ``n`` particles along +x, one per member,
    with per-member Young's modulus and dipole strength drawn uniformly."""
    rng = np.random.default_rng(seed)
    E = rng.uniform(*E_range, size=members)
    mm = rng.uniform(*m_range, size=members)
    x, off, mem = straight_rods([n] * members, [(0.0, 0.0, 0.0)] * members,
                                (1.0, 0.0, 0.0), member=np.arange(members))
    N = x.shape[0]
    bc = np.zeros(N, np.int8)
    bc[off[:-1]] = 1
    mb = np.zeros((N, 3))
    mb[:, 0] = np.repeat(mm, n)
    params = np.stack([np.ones(members), np.ones(members), E, np.full(members, 0.5)], 1)
    w = _base(x, off, mem, params, mb, bc, _field_const(members, B),
              contact_on=True, steps=1000, precision="mixed",
              name=f"ensemble_{members}x{n}")
    w.update(kw)
    return _perturb(w, rng, sigma)


def magnetic_helix(gamma=4e-4, n_bonds=103, length=103.0, turns=1.64, pitch_angle=0.96,
                   d=2.0, E=1.0, nu=0.5, rho=1.0, friction=0.5, damping=2e-3, bond_damping=0.5,
                   dt=0.1, **kw):
    """The helical rod with intra-rod dipole attraction of the paper's results
    ("Helical rods with dipole-dipole interactions"): arc length ``length`` in
    ``n_bonds`` bonds, length / (2 pi R) = ``turns``, pitch angle psi =
    ``pitch_angle`` pi / 2, r(s) = (R cos Ks, R sin Ks, -s cos psi) with
    K = sin(psi) / R, hanging from the clamped base particle at the origin
    (z = 0), the screw axis along z. Rod diameter ``d``; each particle stands for
    a cylindrical segment of the rod and carries the moment M A l along +z, with
    the magnetisation M from gamma = mu0 M^2 / E. Hertz-Mindlin contact at
    r_c = d between particles more than three apart along the rod; the field is
    set by ``helix_ramp_fields``. Global damping ``damping`` and bond damping
    ``bond_damping`` on all four modes: with global damping alone (2e-3) the
    stretched helix develops a growing high-frequency bond oscillation near
    lambda_m = 3, in the oracle and on the GPU alike; bond damping removes it."""
    R = length / (2.0 * np.pi * turns)
    psi = pitch_angle * np.pi / 2.0
    K = np.sin(psi) / R
    s = np.arange(n_bonds + 1) * (length / n_bonds)
    x = np.stack([R * np.cos(K * s), R * np.sin(K * s), -s * np.cos(psi)], 1)
    n = n_bonds + 1
    mu0 = 4.0 * np.pi  # mu0 / 4 pi = 1
    M = np.sqrt(gamma * E / mu0)
    A, l = np.pi * d * d / 4.0, length / n_bonds
    mb = np.tile([0.0, 0.0, M * A * l], (n, 1))
    bc = np.zeros(n, np.int8)
    bc[0] = 1
    w = _base(x, np.array([0, n], np.int32), np.zeros(1, np.int32), [d, rho, E, nu], mb, bc,
              _field_const(1, (0, 0, 0)), dipole_on=True, contact_on=True, r_contact=d,
              exclude_depth=3, contact_model="hertz_mindlin",
              contact_hm=np.array([E, nu, friction, 0.0, 0.0]), damping=damping, dt=dt,
              bond_damping=np.full((1, 4), float(bond_damping)),
              steps=1000, precision="fp64", name=f"magnetic_helix_g{gamma:g}",
              helix=dict(gamma=gamma, E=E, d=d, length=length, mu0=mu0))
    w.update(kw)
    return w


def helix_ramp_fields(w, lams):
    """Field settings [n_inc, 1, 12] of the helix ramp: the potential
    -(b / mu0) ((x^2 + y^2) / 4 - z^2 / 2) gives B = b (x/2, y/2, -z), a constant
    gradient b diag(1/2, 1/2, -1) along the screw axis, with the prefactor
    b = sqrt(mu0 / (gamma E)) (E I / A) (lambda_m / L)^3 for each lambda_m."""
    h = w["helix"]
    EI_A = h["E"] * h["d"] ** 2 / 16.0  # I / A = d^2 / 16 for a circular section
    lams = np.asarray(lams, dtype=np.float64)
    b = np.sqrt(h["mu0"] / (h["gamma"] * h["E"])) * EI_A * (lams / h["length"]) ** 3
    f = np.zeros((len(lams), 1, 12))
    f[:, 0, 3] = 0.5 * b
    f[:, 0, 7] = 0.5 * b
    f[:, 0, 11] = -b
    return f


# Full-size workloads (name -> builder with defaults).
def coiled_rods(n=400, members=2, pitch=0.8, radius=1.5, seed=21, m=0.04, sigma=1e-3, **kw):
    """Clamped rods wound on a tight helix whose turns lie closer than the contact
    distance, one rod per member: many contacts from the first step."""
    lam = 1.0 / np.hypot(radius, pitch / (2 * np.pi))
    ph = np.arange(n) * lam
    turn = np.stack([radius * np.cos(ph), radius * np.sin(ph), pitch * ph / (2 * np.pi)], 1)
    x, off, mem = straight_rods([n] * members, [(0.0, 0.0, 0.0)] * members, (1.0, 0.0, 0.0),
                                member=np.arange(members))
    x = np.tile(turn, (members, 1))
    bc = np.zeros(n * members, np.int8)
    bc[off[:-1]] = 1
    w = _base(x, off, mem, np.tile([1.0, 1.0, 1.0, 0.5], (members, 1)),
              np.tile([0.0, 0.0, m], (n * members, 1)), bc,
              _field_const(members, (0.1, 0.3, -0.2)), contact_on=True, precision="mixed",
              name=f"coiled_rods_{members}x{n}")
    w.update(kw)
    return _perturb(w, np.random.default_rng(seed), sigma)


def periodic_rods(n_rods=12, length=20, box=(14.0, 16.0, 18.0), members=1, seed=8, m=0.05,
                  rcut=None, alpha=None, kmax=None, sigma=1e-3, **kw):
    """Straight rods of ``length`` particles at random positions and directions
    in a periodic box (some reaching out of it: positions are not wrapped),
    dipoles along each rod, ``members`` independent copies' worth of rods per
    member, no contact. Ewald parameters: rcut half the smallest box length,
    alpha = 3.6 / rcut and kmax = ceil(3.6 alpha max(L) / pi) unless given
    (both truncated tails near exp(-13))."""
    rng = np.random.default_rng(seed)
    L = np.asarray(box, dtype=np.float64)
    R = n_rods * members
    pts, offs, dirs = [], [0], []
    for r in range(R):
        # rods of one member are placed at least 1.2 apart (periodic images
        # included) so that no two particles start overlapping
        first = (r // n_rods) * n_rods
        placed = np.concatenate(pts[first:], 0) if r > first else np.zeros((0, 3))
        for _ in range(1000):
            o = rng.uniform(0.0, 1.0, 3) * L
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            c = o[None, :] + np.arange(length, dtype=np.float64)[:, None] * u[None, :]
            if not len(placed):
                break
            dd = c[:, None, :] - placed[None, :, :]
            dd -= L * np.rint(dd / L)
            if np.min(np.sum(dd * dd, -1)) >= 1.44:
                break
        else:
            raise ValueError("periodic_rods: no room for another rod; use a larger box")
        pts.append(c)
        dirs.append(u)
        offs.append(offs[-1] + length)
    x = np.concatenate(pts, 0)
    n = x.shape[0]
    mb = m * np.repeat(np.asarray(dirs), length, axis=0)  # along each rod
    mem = np.repeat(np.arange(members, dtype=np.int32), n_rods)
    rc = 0.5 * float(L.min()) if rcut is None else float(rcut)
    a = 3.6 / rc if alpha is None else float(alpha)
    km = int(np.ceil(3.6 * a * float(L.max()) / np.pi)) if kmax is None else int(kmax)
    w = _base(x, np.asarray(offs, np.int32), mem, np.tile([1.0, 1.0, 1.0, 0.5], (R, 1)), mb,
              np.zeros(n, np.int8), _field_const(members, (0.0, 0.2, 0.1)), contact_on=False,
              box=L, ewald_alpha=a, ewald_rcut=rc, ewald_kmax=km, precision="fp64",
              steps=1000, name=f"periodic_rods_{R}x{length}")
    w.update(kw)
    return _perturb(w, rng, sigma)


CONFIGS = {
    "cantilever": cantilever,       # 20 particles, FP64, 1000 steps
    "twisted_rod": twisted_rod,     # N = 4096, contact + dipoles, 2e4 steps
    "cilia_carpet": cilia_carpet,   # 1024 rods, ~73.7k particles, 1e4 steps
    "adjoint_rod": adjoint_rod,     # N = 256, T = 2000, gradients
    "rod_array": rod_array,         # 512 x 512 = 262,144 particles
    "ensemble": ensemble,           # 64 members x 4096
}


def make(name, **kw):
    """Build the named workload; keyword arguments override its sizes and values."""
    return CONFIGS[name](**kw)
