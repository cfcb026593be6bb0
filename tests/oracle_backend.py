"""A float64 CPU backend with the Operator's apply_A / apply_AT interface,
computed by the oracle (test infrastructure: lets the autograd wrapper and
the server's scheduler run without a GPU)."""
import numpy as np
import torch

from oracle import hlib, operators as ops
from oracle.geometry import Geometry as OGeom


class OracleBackend:
    def __init__(self, nx, ny, nz, nt, dx=1e-4, c=1500.0, cfl=0.3, nz_sim=0):
        self.g = OGeom(nx, ny, nz, nt, dx, dx, dx, cfl * dx / c, c, nz_sim)
        self.Hh = hlib.H_half(self.g)
        self.x_shape = (nz, ny, nx)
        self.d_shape = (nt, ny, nx)

    def _apply(self, fn, t):
        a = t.detach().cpu().numpy().astype(np.float64)
        if a.ndim == 4:
            out = np.stack([fn(self.Hh, s) for s in a])
        else:
            out = fn(self.Hh, a)
        return torch.from_numpy(out).to(dtype=t.dtype, device=t.device)

    def apply_A(self, x):
        return self._apply(ops.A_fft, x)

    def apply_AT(self, y):
        return self._apply(ops.AT_fft, y)
