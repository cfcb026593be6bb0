"""Independent 3D solver of the homogeneous wave equation on a periodic grid.

Test infrastructure only (see ``oracle/__init__``).

This is the stand-in for the PDE solver the paper validates its operator
against (Sec. 3.1, Table 1): it never forms the kernel library.  The object
is embedded at z-indices 0..Nz-1 of an Nx x Ny x nz_sim periodic grid and
the field is advanced in time with the k-space corrected second-order scheme

    P^{n+1}(k) = 2 cos(c dt |k|) P^n(k) - P^{n-1}(k),   P^1 = cos(c dt |k|) P^0,

which reproduces the exact band-limited solution cos(n c dt |k|) P^0 of
eq. 1-2 (zero initial velocity).  The recorded data is the real field on the
plane z = 0 at every step.  Wavenumbers are recomputed here on purpose, with
no helper shared with the library code.
"""
from __future__ import annotations

import numpy as np


def simulate(x: np.ndarray, dx: float, dy: float, dz: float, dt: float,
             c: float, nt: int, nz_sim: int) -> np.ndarray:
    """Sensor-plane time series d[n, j, i] for the initial pressure x[l, j, i]."""
    nz, ny, nx = x.shape
    assert nz_sim >= nz
    vol = np.zeros((nz_sim, ny, nx))
    vol[:nz] = x
    kz = 2.0 * np.pi * np.fft.fftfreq(nz_sim, d=dz)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=dy)
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=dx)
    K = np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    two_cos = 2.0 * np.cos(c * dt * K)
    d = np.empty((nt, ny, nx))
    p_prev = None
    p_cur = np.fft.fftn(vol)
    for n in range(nt):
        field = np.fft.ifftn(p_cur)
        d[n] = field[0].real
        if n == 0:
            p_next = 0.5 * two_cos * p_cur
        else:
            p_next = two_cos * p_cur - p_prev
        p_prev, p_cur = p_cur, p_next
    return d
