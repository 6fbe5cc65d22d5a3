"""Python binding of the rod library: same entry points as the C ABI, with
torch tensors supplying device memory and the current HIP stream.

Only argument marshalling happens here: every step of the loop runs in the HIP
kernels of librodmx.so. Device state is SoA: vectors are ``[3, N]`` float64
tensors, quaternions ``[4, N]``.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L

_PRECISION = {"fp64": L.ROD_FP64, "mixed": L.ROD_MIXED}
_CONTACT_MODEL = {"hookean": 0, "hertz_mindlin": 1}  # ROD_CONTACT_*


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _soa(torch, a, dev):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T), device=dev)


class RodSim:
    """One simulation context built from a workload dictionary (see ``workloads``).

    ``precision``: "fp64" or "mixed" (default: the workload's).
    ``graph_steps``: steps per captured HIP graph (0 = eager launches).
    ``tape_every`` / ``tape_capacity``: checkpointing for ``grad``.
    ``step0``: the time level of the initial state (drive phase, restarts).
    ``forces``: (F, T) [n, 3] of the initial state, e.g. a saved state's; they
    are taken as they are (``forces_valid``) instead of being evaluated.
    """

    def __init__(self, w, precision=None, graph_steps=0, tape_every=0, tape_capacity=0,
                 device="cuda", step0=0, stream=None, forces=None):
        import torch
        self.torch = torch
        self.lib = L.load()
        self.w = w
        n = int(w["n"])
        self.n = n
        dev = torch.device(device)
        self.device = dev
        self.x = _soa(torch, w["x0"], dev)
        self.v = _soa(torch, w["v0"], dev)
        self.q = _soa(torch, w["q0"], dev)
        self.om = _soa(torch, w["w0"], dev)
        if forces is None:
            self.F = torch.zeros((3, n), dtype=torch.float64, device=dev)
            self.T = torch.zeros((3, n), dtype=torch.float64, device=dev)
        else:
            self.F, self.T = _soa(torch, forces[0], dev), _soa(torch, forces[1], dev)
        self.m_body = _soa(torch, w["m_body"], dev)
        self.field = torch.as_tensor(np.ascontiguousarray(w["field"], dtype=np.float64), device=dev)
        self.ext_force = None if w.get("ext_force") is None else _soa(torch, w["ext_force"], dev)
        self.ext_torque = None if w.get("ext_torque") is None else _soa(torch, w["ext_torque"], dev)
        prec = _PRECISION[precision or w.get("precision", "fp64")]
        self.precision = prec
        self._host = dict(
            rod_offset=np.ascontiguousarray(w["rod_offset"], dtype=np.int32),
            rod_member=np.ascontiguousarray(w["rod_member"], dtype=np.int32),
            rod_params=np.ascontiguousarray(w["rod_params"], dtype=np.float64),
            x_ref=np.ascontiguousarray(w["x_ref"], dtype=np.float64),
            bc=np.ascontiguousarray(w["bc"], dtype=np.int8),
            bond_damping=(None if w.get("bond_damping") is None else
                          np.ascontiguousarray(w["bond_damping"], dtype=np.float64).reshape(-1, 4)),
        )
        d = L.RodDesc()
        d.n_particles = n
        d.n_rods = len(self._host["rod_member"])
        d.n_members = int(w["n_members"])
        for k in ("rod_offset", "rod_member", "rod_params", "x_ref", "bc"):
            setattr(d, k, self._host[k].ctypes.data_as(C.c_void_p))
        d.drive_axis = (C.c_double * 3)(*[float(a) for a in w["drive_axis"]])
        d.drive_period = int(w["drive_period"])
        d.field_len = int(self.field.shape[0])
        d.dt = float(w["dt"]); d.damping = float(w["damping"]); d.mu0_4pi = float(w["mu0_4pi"])
        d.k_contact = float(w["k_contact"]); d.r_contact = float(w["r_contact"])
        d.dipole_on = int(bool(w["dipole_on"])); d.contact_on = int(bool(w["contact_on"]))
        d.exclude_depth = int(w["exclude_depth"])
        d.precision = prec
        d.step0 = int(step0)
        d.graph_steps = int(graph_steps)
        d.tape_every = int(tape_every)
        d.tape_capacity = int(tape_capacity)
        bd = self._host["bond_damping"]
        d.bond_damping = None if bd is None else bd.ctypes.data_as(C.c_void_p)
        d.contact_model = _CONTACT_MODEL[w.get("contact_model", "hookean")]
        d.dipole_cutoff = float(w.get("dipole_cutoff") or 0.0)
        if w.get("box") is not None:
            d.box = (C.c_double * 3)(*[float(a) for a in w["box"]])
            d.ewald_alpha = float(w["ewald_alpha"])
            d.ewald_rcut = float(w["ewald_rcut"])
            d.ewald_kmax = int(w["ewald_kmax"])
        if w.get("contact_hm") is not None:
            d.contact_hm = (C.c_double * 5)(*[float(a) for a in w["contact_hm"]])
        self.desc = d
        b = L.RodBuffers()
        b.x, b.v, b.q, b.w = _ptr(self.x), _ptr(self.v), _ptr(self.q), _ptr(self.om)
        b.force, b.torque = _ptr(self.F), _ptr(self.T)
        b.m_body, b.field = _ptr(self.m_body), _ptr(self.field)
        b.ext_force, b.ext_torque = _ptr(self.ext_force), _ptr(self.ext_torque)
        self.bufs = b
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        self.stream = s
        ctx = C.c_void_p()
        L.check(self.lib.rod_init(C.byref(ctx), C.byref(d), C.byref(b),
                                  C.c_void_p(s.cuda_stream), int(forces is not None)))
        self.ctx = ctx

    # ------------------------------------------------------------------ C ABI
    def step(self, n=1):
        L.check(self.lib.rod_step(self.ctx, int(n)))

    def sync(self):
        L.check(self.lib.rod_sync(self.ctx))

    def get_step(self):
        s = C.c_int64()
        L.check(self.lib.rod_get_step(self.ctx, C.byref(s)))
        return s.value

    def eval_forces(self, terms=L.TERM_ALL, with_field=False):
        torch = self.torch
        F = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        T = torch.empty_like(F)
        B = torch.empty_like(F) if with_field else None
        L.check(self.lib.rod_eval_forces(self.ctx, int(terms), _ptr(F), _ptr(T), _ptr(B)))
        return (F, T, B) if with_field else (F, T)

    def energy(self):
        out = np.zeros((int(self.w["n_members"]), 9))
        L.check(self.lib.rod_energy(self.ctx, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def topology(self):
        cnt = C.c_int32()
        L.check(self.lib.rod_topology(self.ctx, None, None, None, 0, C.byref(cnt)))
        B = cnt.value
        ij = np.zeros((max(B, 1), 2), np.int32)
        rr = np.zeros((max(B, 1), 3))
        K = np.zeros((max(B, 1), 4))
        L.check(self.lib.rod_topology(self.ctx, ij.ctypes.data_as(C.c_void_p),
                                      rr.ctypes.data_as(C.c_void_p),
                                      K.ctypes.data_as(C.c_void_p), B, C.byref(cnt)))
        return ij[:B], rr[:B], K[:B]

    def contact_pairs(self):
        cnt = C.c_int32()
        L.check(self.lib.rod_contact_pairs(self.ctx, None, 0, C.byref(cnt)))
        P = cnt.value
        out = np.zeros((max(P, 1), 2), np.int32)
        L.check(self.lib.rod_contact_pairs(self.ctx, out.ctypes.data_as(C.c_void_p), P,
                                           C.byref(cnt)))
        return out[:P]

    def contact_history(self):
        """rod_get_contact_history: dict(count [N], partner [N, 16], disp [N, 16, 3])."""
        n, K = self.n, L.ROD_HM_MAX_CONTACTS
        h = dict(count=np.zeros(n, np.int32), partner=np.zeros((n, K), np.int32),
                 disp=np.zeros((n, K, 3)))
        L.check(self.lib.rod_get_contact_history(self.ctx, *[h[k].ctypes.data_as(C.c_void_p)
                                                             for k in ("count", "partner", "disp")]))
        return h

    def set_contact_history(self, h):
        """rod_set_contact_history from a dict as contact_history returns."""
        a = [np.ascontiguousarray(h["count"], dtype=np.int32),
             np.ascontiguousarray(h["partner"], dtype=np.int32),
             np.ascontiguousarray(h["disp"], dtype=np.float64)]
        L.check(self.lib.rod_set_contact_history(self.ctx, *[v.ctypes.data_as(C.c_void_p) for v in a]))

    def contact_pairs_noalloc(self, cap):
        """rod_contact_pairs_noalloc: at most ``cap`` pairs (sorted) and the total count."""
        cnt = C.c_int32()
        out = np.zeros((max(int(cap), 1), 2), np.int32)
        L.check(self.lib.rod_contact_pairs_noalloc(self.ctx, out.ctypes.data_as(C.c_void_p),
                                                   int(cap), C.byref(cnt)))
        return out[:min(cnt.value, int(cap))], cnt.value

    def ramp(self, fields, max_steps, check_every, ke_tol, watch=()):
        """Quasi-static field ramp (rod_ramp): ``fields`` [n_inc, M, 12] settings
        in turn, each held until every member's kinetic energy is at most
        ``ke_tol`` after a chunk of ``check_every`` steps (at most ``max_steps``;
        negative ``ke_tol``: always ``max_steps``). Needs a one-row field table.
        Returns dict(x_watch [n_inc, n_watch, 3], steps [n_inc], ke [n_inc, M])."""
        M = int(self.w["n_members"])
        f = np.ascontiguousarray(fields, dtype=np.float64).reshape(-1, M, 12)
        watch = np.ascontiguousarray(watch, dtype=np.int32).reshape(-1)
        n_inc, nw = f.shape[0], len(watch)
        xw = np.zeros((n_inc, max(nw, 1), 3))
        steps = np.zeros(n_inc, np.int32)
        ke = np.zeros((n_inc, M))
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        L.check(self.lib.rod_ramp(self.ctx, p(f), n_inc, int(max_steps), int(check_every),
                                  float(ke_tol), p(watch) if nw else None, nw, p(xw), p(steps),
                                  p(ke)))
        return dict(x_watch=xw[:, :nw], steps=steps, ke=ke)

    def lbm_cycles(self, lattice, n_sub, n_cycles):
        """Immersed-boundary coupling (rod_lbm_cycles): ``n_cycles`` lattice
        steps of ``lattice`` (a paper_2603_27279_amd.Lattice), ``n_sub`` rod
        steps each, rod dt = 1 / n_sub, positions in lattice units."""
        L.check(self.lib.rod_lbm_cycles(self.ctx, lattice.ctx, int(n_sub), int(n_cycles)))

    def tape_begin(self):
        L.check(self.lib.rod_tape_begin(self.ctx))

    def grad(self, gx=None, gv=None, gq=None, gw=None, want=("m_body", "field", "x0", "v0",
                                                            "q0", "w0")):
        """Reverse the recorded steps; returns a dict of gradient tensors."""
        torch = self.torch
        cot = L.RodCotangent(_ptr(gx), _ptr(gv), _ptr(gq), _ptr(gw))
        shapes = dict(m_body=(3, self.n), field=tuple(self.field.shape), x0=(3, self.n),
                      v0=(3, self.n), q0=(4, self.n), w0=(3, self.n))
        outs = {k: torch.zeros(shapes[k], dtype=torch.float64, device=self.device) for k in want}
        g = L.RodGradients(*[_ptr(outs.get(k)) for k in ("m_body", "field", "x0", "v0", "q0",
                                                         "w0")])
        L.check(self.lib.rod_grad(self.ctx, C.byref(cot), C.byref(g)))
        return outs

    def timing(self, enable=True):
        """Have every kernel launch stamp HIP events with its own start and end
        (steps run eagerly while on)."""
        L.check(self.lib.rod_timing(self.ctx, int(bool(enable))))

    def kernel_times(self):
        """{kernel: (total_ms, launches)} since the last read."""
        ms = np.zeros(len(L.KERNELS))
        cnt = np.zeros(len(L.KERNELS), dtype=np.int64)
        L.check(self.lib.rod_kernel_times(self.ctx, ms.ctypes.data_as(C.c_void_p),
                                          cnt.ctypes.data_as(C.c_void_p)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(L.KERNELS)}

    def autotune(self, cache_path=None, force=False):
        """Time the dipole work layouts at the current state and apply the fastest;
        returns the tuner's report."""
        buf = C.create_string_buffer(4096)
        path = None if cache_path is None else str(cache_path).encode()
        L.check(self.lib.rod_autotune(self.ctx, path, int(bool(force)), buf, len(buf)))
        return buf.value.decode()

    LAUNCH_MODES = {"batched": 0, "per_rod": 1, "separate": 2}

    def launch_mode(self, mode="batched"):
        """'batched' (default: all rods per launch, force terms fused), 'separate'
        (force terms as separate kernels) or 'per_rod' (the plain per-rod loop)."""
        L.check(self.lib.rod_launch_mode(self.ctx, self.LAUNCH_MODES[mode]))

    def dipole_layout(self, small=-1, target_wgs=1024):
        """Choose the dipole work layout explicitly (see rod_dipole_layout)."""
        L.check(self.lib.rod_dipole_layout(self.ctx, int(small), int(target_wgs)))

    def free(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            L.check(self.lib.rod_free(self.ctx))
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # ------------------------------------------------------------------ helpers
    def state(self):
        """Host copy of the state in the workload layout (AoS numpy arrays)."""
        self.torch.cuda.synchronize(self.device)
        t = lambda a: a.detach().cpu().numpy().T.copy()
        return dict(x=t(self.x), v=t(self.v), q=t(self.q), w=t(self.om), F=t(self.F),
                    T=t(self.T), step=self.get_step())


# Entry points under the C names, for callers that prefer the flat API.
def rod_init(w, **kw):
    return RodSim(w, **kw)


def rod_step(sim, n=1):
    sim.step(n)


def rod_energy(sim):
    return sim.energy()


def rod_grad(sim, **kw):
    return sim.grad(**kw)


def rod_free(sim):
    sim.free()


def _rod_trajectory_function():
    import torch

    class RodTrajectory(torch.autograd.Function):
        """(m_body, field, x0, v0, q0, w0) -> (x_T, v_T, q_T, w_T) after T steps of the
        workload's loop; backward runs the checkpointed reverse pass (rod_grad).

        Tensors are device float64 in the binding's SoA layout ([3, N], [4, N],
        field [L, M, 12])."""

        @staticmethod
        def forward(ctx, m_body, field, x0, v0, q0, w0, workload, nsteps, every, precision):
            sim = RodSim(workload, precision=precision, tape_every=every,
                         tape_capacity=max(int(nsteps), 1))
            with torch.no_grad():
                sim.m_body.copy_(m_body.detach())
                sim.field.copy_(field.detach())
                sim.x.copy_(x0.detach())
                sim.v.copy_(v0.detach())
                sim.q.copy_(q0.detach())
                sim.om.copy_(w0.detach())
            sim.tape_begin()
            sim.step(int(nsteps))
            ctx.sim = sim
            return sim.x.clone(), sim.v.clone(), sim.q.clone(), sim.om.clone()

        @staticmethod
        def backward(ctx, gx, gv, gq, gw):
            sim = ctx.sim
            cont = lambda t: None if t is None else t.contiguous()
            g = sim.grad(gx=cont(gx), gv=cont(gv), gq=cont(gq), gw=cont(gw))
            sim.free()
            ctx.sim = None
            return (g["m_body"], g["field"], g["x0"], g["v0"], g["q0"], g["w0"],
                    None, None, None, None)

    return RodTrajectory


_RT = None


def rod_trajectory(m_body, field, x0, v0, q0, w0, workload, nsteps, every=100, precision="fp64"):
    """Differentiable run of the loop (see RodTrajectory): returns (x_T, v_T, q_T, w_T).

    The tape starts from the given state with tape_begin, so forces of the first
    level are evaluated from (x0, q0, v0, w0); q0 is normalised first."""
    global _RT
    if _RT is None:
        _RT = _rod_trajectory_function()
    return _RT.apply(m_body, field, x0, v0, q0, w0, workload, nsteps, every, precision)
