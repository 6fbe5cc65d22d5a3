"""Python front of the FP64 CPU oracle (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package. It compiles ``rod_oracle.cpp`` with g++ (plain C++17, OpenMP over
independent rows, no FMA contraction) and calls it through ctypes. Nothing here
is shared with, or imported by, the GPU library.

Arrays cross in the workload's own layout: AoS ``[N, 3]`` / ``[N, 4]`` float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rod_oracle.cpp")
_LIB = os.path.join(_HERE, "librod_oracle.so")
_lib = None

BOND, DIPOLE, ZEEMAN, CONTACT, DAMP, EXT, ALL = 1, 2, 4, 8, 16, 32, 63
FLUID = 64  # immersed-boundary penalty force (with a fluid velocity given)
HC_CAP = 32  # Hertz-Mindlin contacts per particle a continued state can carry
ENERGY_TERMS = ("stretch", "shear", "twist", "bend", "zeeman", "dipole", "contact",
                "kinetic", "rotational")


def build(force=True):
    """Compile the oracle library in place."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _System(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("n_rods", C.c_int32), ("n_members", C.c_int32),
        ("rod_offset", C.c_void_p), ("rod_member", C.c_void_p),
        ("rod_params", C.c_void_p), ("x_ref", C.c_void_p), ("bc", C.c_void_p),
        ("drive_axis", C.c_double * 3), ("drive_period", C.c_int64),
        ("field_len", C.c_int32), ("ext_force", C.c_void_p), ("ext_torque", C.c_void_p),
        ("dt", C.c_double), ("damping", C.c_double), ("mu0_4pi", C.c_double),
        ("k_contact", C.c_double), ("r_contact", C.c_double),
        ("dipole_on", C.c_int32), ("contact_on", C.c_int32), ("exclude_depth", C.c_int32),
        ("bond_damping", C.c_void_p),
        ("contact_model", C.c_int32), ("contact_hm", C.c_double * 5),
        ("dipole_cutoff", C.c_double),
        ("fluid_u", C.c_void_p), ("fluid_dt", C.c_double), ("fluid_F", C.c_void_p),
        ("box", C.c_double * 3), ("ewald_alpha", C.c_double), ("ewald_rcut", C.c_double),
        ("ewald_kmax", C.c_int32),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class System:
    """ctypes view of a workload dict; keeps every array alive while in use."""

    def __init__(self, w):
        self.w = w
        self.n = int(w["n"])
        keep = dict(
            rod_offset=np.ascontiguousarray(w["rod_offset"], dtype=np.int32),
            rod_member=np.ascontiguousarray(w["rod_member"], dtype=np.int32),
            rod_params=_f64(w["rod_params"]),
            x_ref=_f64(w["x_ref"]),
            bc=np.ascontiguousarray(w["bc"], dtype=np.int8),
            field=_f64(w["field"]),
            ext_force=None if w.get("ext_force") is None else _f64(w["ext_force"]),
            ext_torque=None if w.get("ext_torque") is None else _f64(w["ext_torque"]),
            bond_damping=None if w.get("bond_damping") is None else _f64(w["bond_damping"]),
        )
        self.keep = keep
        s = _System()
        s.n = self.n
        s.n_rods = len(keep["rod_member"])
        s.n_members = int(w["n_members"])
        s.rod_offset = _p(keep["rod_offset"])
        s.rod_member = _p(keep["rod_member"])
        s.rod_params = _p(keep["rod_params"])
        s.x_ref = _p(keep["x_ref"])
        s.bc = _p(keep["bc"])
        s.drive_axis = (C.c_double * 3)(*[float(a) for a in w["drive_axis"]])
        s.drive_period = int(w["drive_period"])
        s.field_len = int(keep["field"].shape[0])
        s.ext_force = _p(keep["ext_force"])
        s.ext_torque = _p(keep["ext_torque"])
        s.dt = float(w["dt"]); s.damping = float(w["damping"]); s.mu0_4pi = float(w["mu0_4pi"])
        s.k_contact = float(w["k_contact"]); s.r_contact = float(w["r_contact"])
        s.dipole_on = int(bool(w["dipole_on"])); s.contact_on = int(bool(w["contact_on"]))
        s.exclude_depth = int(w["exclude_depth"])
        s.bond_damping = _p(keep["bond_damping"])
        s.dipole_cutoff = float(w.get("dipole_cutoff") or 0.0)
        fu = w.get("fluid_u")
        keep["fluid_u"] = None if fu is None else _f64(fu, (self.n, 3))
        keep["fluid_F"] = np.zeros((max(self.n, 1), 3))
        s.fluid_u = _p(keep["fluid_u"])
        s.fluid_dt = float(w.get("fluid_dt") or 1.0)
        s.fluid_F = _p(keep["fluid_F"])
        box = w.get("box")
        if box is not None:
            s.box = (C.c_double * 3)(*[float(a) for a in box])
            s.ewald_alpha = float(w["ewald_alpha"])
            s.ewald_rcut = float(w["ewald_rcut"])
            s.ewald_kmax = int(w["ewald_kmax"])
        s.contact_model = contact_model(w)
        if s.contact_model == 1:
            s.contact_hm = (C.c_double * 5)(*[float(a) for a in w["contact_hm"]])
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)

    @property
    def field(self):
        return self.keep["field"]


def bonds(w):
    """Topology: (ij [B,2] int32, rref [B,3], K [B,4] = K_r, K_s, K_t, K_b)."""
    lib = _load()
    sy = System(w)
    cap = max(sy.n, 1)
    ij = np.zeros((cap, 2), np.int32)
    rr = np.zeros((cap, 3))
    K = np.zeros((cap, 4))
    lib.orc_bonds.restype = C.c_int
    B = lib.orc_bonds(sy.ref, _p(ij), _p(rr), _p(K), C.c_int(cap))
    return ij[:B].copy(), rr[:B].copy(), K[:B].copy()


def mass(w):
    lib = _load()
    sy = System(w)
    m = np.zeros(sy.n)
    I = np.zeros(sy.n)
    lib.orc_mass(sy.ref, _p(m), _p(I))
    return m, I


def bond_single(x1, x2, q1, q2, rref, K):
    """One bond: returns (F on particle 1, tau_s, tau_b + tau_t on particle 1, energies[4])."""
    lib = _load()
    a = [_f64(v) for v in (x1, x2, q1, q2, rref, K)]
    F, Ts, Tbt, e = np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(4)
    lib.orc_bond_single(*[_p(v) for v in a], _p(F), _p(Ts), _p(Tbt), _p(e))
    return F, Ts, Tbt, e


CONTACT_MODELS = {"hookean": 0, "hertz_mindlin": 1}


def contact_model(w):
    """0 for the Hookean normal law, 1 for Hertz-Mindlin (``contact_hm`` =
    contact modulus E, Poisson ratio nu, friction mu, damping g_n, g_t)."""
    return CONTACT_MODELS[w.get("contact_model", "hookean")]


def has_bond_damping(w):
    g = w.get("bond_damping")
    return g is not None and bool(np.any(np.asarray(g) != 0))


def forces(w, x, q, v=None, om=None, mbody=None, step=0, mask=ALL, with_field=False,
           hist=None, hist_out=False):
    """Force and torque [N,3] of the terms in ``mask`` at the given state.

    With bond damping, ``hist`` holds the measures [B, 5] (shear angle, twist,
    bend vector in C') of the previous level (None: no rates), and
    ``hist_out=True`` also returns this level's measures."""
    lib = _load()
    sy = System(w)
    n = sy.n
    x = _f64(x, (n, 3)); q = _f64(q, (n, 4))
    v = np.zeros((n, 3)) if v is None else _f64(v, (n, 3))
    om = np.zeros((n, 3)) if om is None else _f64(om, (n, 3))
    mb = _f64(w["m_body"] if mbody is None else mbody, (n, 3))
    F, T, B = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
    nb = max(1, n)
    hin = None if hist is None else _f64(hist)
    hout = np.zeros((nb, 5))
    lib.orc_forces(sy.ref, _p(x), _p(q), _p(v), _p(om), _p(mb), _p(sy.field),
                   C.c_int64(step), C.c_int32(mask), _p(F), _p(T), _p(B), _p(hin), _p(hout))
    out = (F, T, B) if with_field else (F, T)
    if hist_out:
        nbond = len(bonds(w)[0])
        out = out + (hout[:nbond].copy(),)
    return out


def hm_single(w, xi, xj, vi=(0, 0, 0), vj=(0, 0, 0), wi=(0, 0, 0), wj=(0, 0, 0), sprev=None):
    """One Hertz-Mindlin contact of a workload's law: (force on i, torque on i,
    new tangential displacement, normal elastic energy)."""
    lib = _load()
    sy = System(w)
    a = [_f64(v, (3,)) for v in (xi, xj, vi, vj, wi, wj)]
    sp = None if sprev is None else _f64(sprev, (3,))
    F, T, sn, e = np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(1)
    lib.orc_hm_single(sy.ref, *[_p(v) for v in a], _p(sp), _p(F), _p(T), _p(sn), _p(e))
    return F, T, sn, float(e[0])


def energy(w, x, q, v=None, om=None, mbody=None, step=0):
    """Energies [M, 9] (see ENERGY_TERMS)."""
    lib = _load()
    sy = System(w)
    n = sy.n
    x = _f64(x, (n, 3)); q = _f64(q, (n, 4))
    v = np.zeros((n, 3)) if v is None else _f64(v, (n, 3))
    om = np.zeros((n, 3)) if om is None else _f64(om, (n, 3))
    mb = _f64(w["m_body"] if mbody is None else mbody, (n, 3))
    out = np.zeros((int(w["n_members"]), 9))
    lib.orc_energy(sy.ref, _p(x), _p(q), _p(v), _p(om), _p(mb), _p(sy.field),
                   C.c_int64(step), _p(out))
    return out


def contact_pairs(w, x):
    """Sorted contact pairs (i < j) [P, 2] int32 by brute force."""
    lib = _load()
    sy = System(w)
    x = _f64(x, (sy.n, 3))
    lib.orc_contact_pairs.restype = C.c_int
    cnt = lib.orc_contact_pairs(sy.ref, _p(x), None, C.c_int(0))
    out = np.zeros((max(cnt, 1), 2), np.int32)
    lib.orc_contact_pairs(sy.ref, _p(x), _p(out), C.c_int(cnt))
    return out[:cnt].copy()


def run(w, nsteps, state=None, step0=0, mbody=None):
    """Advance a workload. ``state`` (dict x, v, q, w, F, T) continues a previous
    run; otherwise the initial state is prepared from x0, v0, q0, w0.
    Returns the new state dict (AoS arrays) with its step index."""
    lib = _load()
    sy = System(w)
    n = sy.n
    if state is None:
        st = dict(x=_f64(w["x0"]).copy(), v=_f64(w["v0"]).copy(), q=_f64(w["q0"]).copy(),
                  w=_f64(w["w0"]).copy(), F=np.zeros((n, 3)), T=np.zeros((n, 3)), step=step0)
        prepared = 0
    else:
        st = {k: (np.array(v, dtype=np.float64, copy=True) if k != "step" else v)
              for k, v in state.items()}
        prepared = 1
    # bond damping measures of the last evaluation; a continued state without
    # them has its own recorded before the first step
    hist_in = int(prepared and "hist" in st)
    if "hist" not in st:
        st["hist"] = np.zeros((max(1, n), 5))
    # Hertz-Mindlin contacts of the last evaluation (partner, tangential
    # displacement), carried by a continued state like the damping measures
    hc_in = int(prepared and "hc_cnt" in st)
    hc = (np.ascontiguousarray(st.get("hc_cnt", np.zeros(n)), dtype=np.int32),
          np.ascontiguousarray(st.get("hc_j", np.zeros((n, HC_CAP))), dtype=np.int32),
          np.ascontiguousarray(st.get("hc_s", np.zeros((n, HC_CAP, 3))), dtype=np.float64))
    mb = _f64(w["m_body"] if mbody is None else mbody, (n, 3))
    rc = lib.orc_run(sy.ref, _p(st["x"]), _p(st["v"]), _p(st["q"]), _p(st["w"]), _p(st["F"]),
                     _p(st["T"]), _p(mb), _p(sy.field), C.c_int64(int(st["step"])),
                     C.c_int64(int(nsteps)), C.c_int32(prepared), _p(st["hist"]), C.c_int32(hist_in),
                     _p(hc[0]), _p(hc[1]), _p(hc[2]), C.c_int32(HC_CAP), C.c_int32(hc_in))
    if rc != 0:
        raise RuntimeError(f"a particle has more than {HC_CAP} Hertz-Mindlin contacts")
    if int(w.get("contact_on", 0)) and contact_model(w) == 1:
        st["hc_cnt"], st["hc_j"], st["hc_s"] = hc
    st["step"] = int(st["step"]) + int(nsteps)
    if w.get("fluid_u") is not None:
        st["fluid_F"] = sy.keep["fluid_F"][:n].copy()  # penalty forces of the last evaluation
    return st


def ramp(w, fields, max_steps, check_every, ke_tol, watch=(), state=None, step0=0):
    """Quasi-static field ramp: for each field setting ``fields[k]`` ([M, 12],
    B0 then G per member) step until every member's kinetic energy is at most
    ``ke_tol`` after a chunk of ``check_every`` steps (at most ``max_steps``;
    a negative ``ke_tol`` runs every setting for ``max_steps``).
    ``state`` continues a previous run (prepared, forces of its last field);
    otherwise the initial state is prepared with the first setting.
    Returns dict(x_watch [n_inc, n_watch, 3], steps [n_inc], ke [n_inc, M],
    state)."""
    lib = _load()
    sy = System(w)
    n, M = sy.n, int(w["n_members"])
    fields = _f64(fields, (-1, M, 12))
    n_inc = fields.shape[0]
    if state is None:
        st = dict(x=_f64(w["x0"]).copy(), v=_f64(w["v0"]).copy(), q=_f64(w["q0"]).copy(),
                  w=_f64(w["w0"]).copy(), F=np.zeros((n, 3)), T=np.zeros((n, 3)), step=step0)
        prepared = 0
    else:
        st = {k: (np.array(v, dtype=np.float64, copy=True) if k != "step" else v)
              for k, v in state.items() if k != "hist" and not k.startswith("hc_")}
        prepared = 1
    watch = np.ascontiguousarray(watch, dtype=np.int32)
    xw = np.zeros((n_inc, max(len(watch), 1), 3))
    steps = np.zeros(n_inc, np.int32)
    ke = np.zeros((n_inc, M))
    mb = _f64(w["m_body"], (n, 3))
    lib.orc_ramp(sy.ref, _p(st["x"]), _p(st["v"]), _p(st["q"]), _p(st["w"]), _p(st["F"]),
                 _p(st["T"]), _p(mb), _p(fields), C.c_int32(n_inc), C.c_int32(int(max_steps)),
                 C.c_int32(int(check_every)), C.c_double(float(ke_tol)),
                 C.c_int64(int(st["step"])), C.c_int32(prepared), _p(watch),
                 C.c_int32(len(watch)), _p(xw), _p(steps), _p(ke))
    st["step"] = int(st["step"]) + int(steps.sum())
    return dict(x_watch=xw[:, :len(watch)], steps=steps, ke=ke, state=st)


def run_jvp(w, nsteps, tangent, step0=0):
    """Forward-mode derivative of ``run`` from the raw initial inputs.

    ``tangent`` maps any of x0, v0, q0, w0, m_body, field to a direction array.
    Returns (final state dict, final tangent dict) with keys x, v, q, w.
    Bond damping is not differentiated (its rates depend on stored history). With a
    dipole cutoff the selection of pairs is taken from the primal distances (the
    derivative of the truncated sum away from the cutoff)."""
    if has_bond_damping(w):
        raise NotImplementedError("the forward-mode run does not differentiate bond damping")
    if w["contact_on"] and contact_model(w) != 0:
        raise NotImplementedError("the forward-mode run does not differentiate Hertz-Mindlin contact")
    if w.get("box") is not None:
        raise NotImplementedError("the forward-mode run does not differentiate the Ewald sum")
    lib = _load()
    sy = System(w)
    n = sy.n
    ins = [_f64(w[k]) for k in ("x0", "v0", "q0", "w0", "m_body")] + [sy.field]
    dins = [None if tangent.get(k) is None else _f64(tangent[k], np.shape(a))
            for k, a in zip(("x0", "v0", "q0", "w0", "m_body", "field"), ins)]
    out = [np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 4)), np.zeros((n, 3))]
    dout = [np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 4)), np.zeros((n, 3))]
    lib.orc_run_jvp(sy.ref, *[_p(a) for a in ins], *[_p(a) for a in dins],
                    C.c_int64(step0), C.c_int64(int(nsteps)),
                    _p(out[0]), _p(out[1]), _p(out[2]), _p(out[3]),
                    _p(dout[0]), _p(dout[1]), _p(dout[2]), _p(dout[3]))
    keys = ("x", "v", "q", "w")
    return dict(zip(keys, out)), dict(zip(keys, dout))


def rows(w, x, q, rows, mbody=None):
    """Dipole force, dipole field and contact force [len(rows), 3] of selected particles."""
    if w.get("box") is not None:
        raise NotImplementedError("rows are open-boundary sums; a periodic box has no row form")
    lib = _load()
    sy = System(w)
    n = sy.n
    x = _f64(x, (n, 3)); q = _f64(q, (n, 4))
    mb = _f64(w["m_body"] if mbody is None else mbody, (n, 3))
    r = np.ascontiguousarray(rows, dtype=np.int32)
    F, B, Fc = np.zeros((len(r), 3)), np.zeros((len(r), 3)), np.zeros((len(r), 3))
    lib.orc_rows(sy.ref, _p(x), _p(q), _p(mb), _p(r), C.c_int32(len(r)), _p(F), _p(B), _p(Fc))
    return F, B, Fc
