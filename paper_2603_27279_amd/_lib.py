"""ctypes declarations of the C ABI in include/rod.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librodmx.so")

ROD_OK, ROD_E_INVALID, ROD_E_HIP, ROD_E_NONFINITE, ROD_E_NOTAPE, ROD_E_OVERFLOW, ROD_E_STATE = \
    0, -1, -2, -3, -4, -5, -6
ROD_FP64, ROD_MIXED = 0, 1
TERM_BOND, TERM_DIPOLE, TERM_ZEEMAN, TERM_CONTACT, TERM_DAMP, TERM_EXT, TERM_ALL = \
    1, 2, 4, 8, 16, 32, 63

ROD_NOALLOC_MAX_PAIRS = 1048576  # include/rod.h
ROD_HM_MAX_CONTACTS = 32  # include/rod.h

KERNELS = ("pre", "bond", "dipole", "contact", "post", "forces", "kick", "cells", "ewald_real")

_P = C.c_void_p


class RodDesc(C.Structure):
    _fields_ = [
        ("n_particles", C.c_int32), ("n_rods", C.c_int32), ("n_members", C.c_int32),
        ("rod_offset", _P), ("rod_member", _P), ("rod_params", _P), ("x_ref", _P), ("bc", _P),
        ("drive_axis", C.c_double * 3), ("drive_period", C.c_int64), ("field_len", C.c_int32),
        ("dt", C.c_double), ("damping", C.c_double), ("mu0_4pi", C.c_double),
        ("k_contact", C.c_double), ("r_contact", C.c_double),
        ("dipole_on", C.c_int32), ("contact_on", C.c_int32), ("exclude_depth", C.c_int32),
        ("precision", C.c_int32), ("step0", C.c_int64), ("graph_steps", C.c_int32),
        ("tape_every", C.c_int32), ("tape_capacity", C.c_int32),
        ("bond_damping", _P),
        ("contact_model", C.c_int32), ("contact_hm", C.c_double * 5),
        ("dipole_cutoff", C.c_double),
        ("box", C.c_double * 3), ("ewald_alpha", C.c_double), ("ewald_rcut", C.c_double),
        ("ewald_kmax", C.c_int32),
    ]


class RodBuffers(C.Structure):
    _fields_ = [(k, _P) for k in ("x", "v", "q", "w", "force", "torque", "m_body", "field",
                                   "ext_force", "ext_torque")]


class RodCotangent(C.Structure):
    _fields_ = [(k, _P) for k in ("x", "v", "q", "w")]


class RodGradients(C.Structure):
    _fields_ = [(k, _P) for k in ("m_body", "field", "x0", "v0", "q0", "w0")]


class LbmDesc(C.Structure):
    """Mirrors lbm_desc of include/lbm.h."""
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("tau", C.c_double),
                ("force", C.c_double * 3), ("walls_z", C.c_int32),
                ("lid_velocity", C.c_double * 2)]


class RodError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rod error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load librodmx.so (built in place); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the HIP library is required; there is no fallback)")
    lib = C.CDLL(LIB_PATH)
    i32, i64 = C.c_int32, C.c_int64
    sig = {
        "rod_query_workspace": [C.POINTER(RodDesc), C.POINTER(C.c_size_t)],
        "rod_init": [C.POINTER(_P), C.POINTER(RodDesc), C.POINTER(RodBuffers), _P, i32],
        "rod_step": [_P, i64],
        "rod_get_step": [_P, C.POINTER(i64)],
        "rod_sync": [_P],
        "rod_eval_forces": [_P, i32, _P, _P, _P],
        "rod_energy": [_P, _P, i32],
        "rod_topology": [_P, _P, _P, _P, i32, C.POINTER(i32)],
        "rod_contact_pairs": [_P, _P, i32, C.POINTER(i32)],
        "rod_contact_pairs_noalloc": [_P, _P, i32, C.POINTER(i32)],
        "rod_get_contact_history": [_P, _P, _P, _P],
        "rod_set_contact_history": [_P, _P, _P, _P],
        "rod_tape_begin": [_P],
        "rod_grad": [_P, C.POINTER(RodCotangent), C.POINTER(RodGradients)],
        "rod_free": [_P],
        "rod_timing": [_P, i32],
        "rod_kernel_times": [_P, _P, _P],
        "rod_autotune": [_P, C.c_char_p, i32, C.c_char_p, i32],
        "rod_dipole_layout": [_P, i32, i32],
        "rod_launch_mode": [_P, i32],
        "rod_probe_fma": [i32, _P, _P, C.POINTER(C.c_double)],
        "rod_ramp": [_P, _P, i32, i32, i32, C.c_double, _P, i32, _P, _P, _P],
        "lbm_init": [C.POINTER(_P), C.POINTER(LbmDesc), _P, _P],
        "lbm_step": [_P, i64],
        "lbm_populations": [_P, _P],
        "lbm_moments": [_P, _P, _P],
        "lbm_free": [_P],
        "rod_lbm_cycles": [_P, _P, i32, i64],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.rod_last_error.argtypes = []
    lib.rod_last_error.restype = C.c_char_p
    lib.lbm_last_error.argtypes = []
    lib.lbm_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def check(code):
    if code != ROD_OK:
        msg = load().rod_last_error().decode(errors="replace")
        raise RodError(code, msg)
    return code
