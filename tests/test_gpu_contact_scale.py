"""Contact sums at non-unit scales (Methods, "Contact"; the unit systems the
paper recommends put contact forces far from 1): the exact 128-bit sums take
their quantum from the contact law's bound on one pair's term, so per-particle
contact forces and torques keep the FP64 bar relative to each particle's own
force, whatever the stiffness; a term far past that bound is reported instead
of wrapping."""
import numpy as np
import pytest

import oracle
import workloads
from paper_2603_27279_amd import RodSim, TERM_CONTACT
from paper_2603_27279_amd._lib import ROD_E_OVERFLOW, RodError
from test_gpu_parity import clump

pytestmark = pytest.mark.gpu


def per_particle_rel(F, Fo, floor):
    """max_i |F_i - Fo_i|_inf / max(|Fo_i|_inf, floor_i) over particles with a
    nonzero floor; particles whose floor is 0 must match exactly."""
    num = np.max(np.abs(F - Fo), axis=1)
    den = np.maximum(np.max(np.abs(Fo), axis=1), floor)
    zero = floor == 0
    assert np.all(num[zero] == 0.0)
    return float(np.max(num[~zero] / den[~zero])) if np.any(~zero) else 0.0


def hookean_term_sums(w, x):
    """Sum over its contacts of |k (r_c - r)| per particle (a bound on the size of
    the terms the particle's sum cancels; contacts from the brute-force pairs)."""
    S = np.zeros(w["n"])
    for i, j in oracle.contact_pairs(w, x):
        f = abs(w["k_contact"]) * (w["r_contact"] - np.linalg.norm(x[i] - x[j]))
        S[i] += f
        S[j] += f
    return S


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("kc", [1e6, 1e-6])
def test_hookean_per_particle_at_extreme_stiffness(kc, prec):
    w = clump(box=4.0)
    w["k_contact"] = kc
    w["dt"] = 1e-5 if kc > 1 else 0.01
    sim = RodSim(w, precision=prec)
    st = oracle.run(w, 0)
    S = hookean_term_sums(w, st["x"])
    assert np.count_nonzero(S) > 20
    F, _ = sim.eval_forces(TERM_CONTACT)
    Fo, _ = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=TERM_CONTACT)
    err = per_particle_rel(F.cpu().numpy().T, Fo, 1e-3 * S)
    assert err <= 1e-12, err
    # energies: the contact term per member
    E = sim.energy()
    Eo = oracle.energy(w, st["x"], st["q"], st["v"], st["w"])
    assert abs(E[0, 6] - Eo[0, 6]) <= 1e-12 * abs(Eo[0, 6])
    # a few steps (stiff contacts push the clump apart) on the FP64 path
    if prec == "fp64":
        sim.step(20)
        sim.sync()
        g = sim.state()
        o = oracle.run(w, 20)
        motion = np.max(np.abs(o["x"] - w["x0"]))
        assert motion > 0
        assert np.max(np.abs(g["x"] - o["x"])) <= 1e-9 * motion
        S = hookean_term_sums(w, o["x"])
        Fo, _ = oracle.forces(w, o["x"], o["q"], o["v"], o["w"], mask=TERM_CONTACT)
        F, _ = sim.eval_forces(TERM_CONTACT)
        # the states differ by rounding, so the forces by rounding times the stiffness
        assert per_particle_rel(F.cpu().numpy().T, Fo, 1e-3 * S + 1e-300) <= 1e-9
    sim.free()


def hm_pair(E, delta=1e-3, mu=0.5, gn=0.0, gt=0.0, seed=4):
    """Two free unit spheres overlapping by delta (contact distance 1) along a
    random direction, sliding and spinning against each other."""
    rng = np.random.default_rng(seed)
    n_hat = rng.normal(size=3)
    n_hat /= np.linalg.norm(n_hat)
    x = np.stack([np.zeros(3), (1.0 - delta) * n_hat])
    x, off, mem = workloads.straight_rods([1, 1], x, (1, 0, 0))
    w = workloads._base(x, off, mem, np.tile([1.0, 1, 1, 0.5], (2, 1)), np.zeros((2, 3)),
                        np.zeros(2, np.int8), workloads._field_const(1, (0, 0, 0)),
                        dipole_on=False, contact_on=True, damping=0.0, precision="fp64",
                        contact_model="hertz_mindlin",
                        contact_hm=np.array([E, 0.3, mu, gn, gt]), exclude_depth=0,
                        name="hm_pair")
    w["x0"] = x.copy()
    tang = np.cross(n_hat, rng.normal(size=3))
    w["v0"] = np.stack([np.zeros(3), 1e-4 * tang / np.linalg.norm(tang)])
    w["w0"] = np.stack([1e-3 * rng.normal(size=3), 1e-3 * rng.normal(size=3)])
    return w


@pytest.mark.parametrize("E,dt", [(1e-3, 0.01), (1.0, 0.01), (1e9, 1e-6)])
def test_hertz_mindlin_pair_per_particle(E, dt):
    """A Hertz-Mindlin pair at an overlap of 1e-3: at E = 1e-3 its force is
    about 1e-8, far below the 2^-48 quantum of a fixed absolute scale relative
    to the FP64 bar; at E = 1e9 it is about 1e4. Force, torque and the contact's
    history over 30 steps follow the oracle to 1e-12 per particle."""
    w = hm_pair(E, gn=1e-4 * E, gt=1e-4 * E)
    w["dt"] = dt
    sim = RodSim(w, precision="fp64")
    st = oracle.run(w, 0)
    F, T = sim.eval_forces(TERM_CONTACT)
    Fo, To = oracle.forces(w, st["x"], st["q"], st["v"], st["w"], mask=TERM_CONTACT)
    F, T = F.cpu().numpy().T, T.cpu().numpy().T
    for a, b in ((F, Fo), (T, To)):
        den = np.max(np.abs(b), axis=1)
        assert np.all(den > 0)
        assert np.max(np.max(np.abs(a - b), axis=1) / den) <= 1e-12
    for k in (1, 30):
        sim.step(k if k == 1 else k - 1)
        sim.sync()
        g = sim.state()
        o = oracle.run(w, k)
        for key in ("F", "T"):
            den = np.max(np.abs(o[key]), axis=1)
            num = np.max(np.abs(g[key] - o[key]), axis=1)
            if k == 1:
                assert np.all(den > 0), key  # still in contact after one step
            # once the dashpot has pushed the spheres apart both sides are 0
            assert np.all(num[den == 0] == 0.0), (E, k, key)
            assert np.all(num[den > 0] <= 1e-12 * den[den > 0]), (E, k, key)
    sim.free()


def test_term_past_the_bound_is_reported():
    """A normal dashpot force 2^28 times the law's bound on a pair's force (a
    huge g_n on an approaching pair) leaves the exact sums' range: rod_sync
    reports ROD_E_OVERFLOW and no garbage force is summed."""
    w = hm_pair(1.0, gn=1e12)
    n_hat = w["x0"][1] / np.linalg.norm(w["x0"][1])
    w["v0"] = np.stack([np.zeros(3), -0.5 * n_hat])  # approaching
    sim = RodSim(w, precision="fp64")
    with pytest.raises(RodError) as e:
        sim.sync()
    assert e.value.code == ROD_E_OVERFLOW
    assert "exact contact sums" in str(e.value)
    F, _ = sim.eval_forces(TERM_CONTACT)
    assert np.all(np.isfinite(F.cpu().numpy()))
    sim.free()
