"""Binding of the lattice Boltzmann solver of include/lbm.h (argument
marshalling only; the HIP kernels do the work). Populations are [19, nz, ny, nx]
in the velocity order of lbm.h."""
import ctypes as C

import numpy as np

from . import _lib as L


def _check(code):
    if code != L.ROD_OK:
        raise L.RodError(code, L.load().lbm_last_error().decode(errors="replace"))


class Lattice:
    """D3Q19 BGK lattice with Guo forcing on the GPU.

    ``f0``: initial populations [19, nz, ny, nx] (numpy or a device tensor);
    ``tau``: relaxation time; ``force``: uniform body force density;
    ``walls_z``: 0 (or False) periodic in z; 1 (or True) no-slip walls below
    z = 0 and above nz - 1; 2 a no-slip bottom and a free-slip top;
    ``lid``: (u_x, u_y) of a moving top wall (walls_z = 1)."""

    def __init__(self, f0, tau, force=(0.0, 0.0, 0.0), walls_z=False, lid=(0.0, 0.0),
                 device="cuda"):
        import torch
        self.torch = torch
        self.lib = L.load()
        f0 = torch.as_tensor(np.ascontiguousarray(f0, dtype=np.float64) if isinstance(f0, np.ndarray)
                             else f0, dtype=torch.float64, device=device).contiguous()
        assert f0.ndim == 4 and f0.shape[0] == 19
        self.shape = tuple(f0.shape[1:])
        nz, ny, nx = self.shape
        d = L.LbmDesc()
        d.nx, d.ny, d.nz = nx, ny, nz
        d.tau = float(tau)
        d.force = (C.c_double * 3)(*[float(g) for g in force])
        d.walls_z = int(walls_z)
        d.lid_velocity = (C.c_double * 2)(*[float(v) for v in lid])
        self.desc = d
        self.device = f0.device
        self.stream = torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        _check(self.lib.lbm_init(C.byref(ctx), C.byref(d), C.c_void_p(f0.data_ptr()),
                                 C.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx
        self._f0 = f0  # kept until the copy has run

    def step(self, n=1):
        _check(self.lib.lbm_step(self.ctx, int(n)))

    def populations(self):
        out = self.torch.empty((19,) + self.shape, dtype=self.torch.float64, device=self.device)
        _check(self.lib.lbm_populations(self.ctx, C.c_void_p(out.data_ptr())))
        return out

    def moments(self):
        rho = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        u = self.torch.empty((3,) + self.shape, dtype=self.torch.float64, device=self.device)
        _check(self.lib.lbm_moments(self.ctx, C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr())))
        return rho, u

    def free(self):
        if getattr(self, "ctx", None):
            _check(self.lib.lbm_free(self.ctx))
            self.ctx = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
