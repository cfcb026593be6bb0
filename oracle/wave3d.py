"""Independent 3D solver of the homogeneous wave equation on a periodic grid.

Test infrastructure only (see ``oracle/__init__``).

This is the stand-in for the PDE solver the paper validates its operator
against (Sec. 3.1, Table 1): it never forms the kernel library.  The object
is embedded at z-indices 0..Nz-1 of an Nx x Ny x nz_sim periodic grid and
the field is advanced in time with the k-space corrected second-order scheme

    P^{n+1}(k) = 2 cos(c dt |k|) P^n(k) - P^{n-1}(k),   P^1 = cos(c dt |k|) P^0,

which reproduces the exact band-limited solution cos(n c dt |k|) P^0 of
eq. 1-2 (zero initial velocity).  The recorded data is the real field on the
plane z = 0 at every step (or on any set of depth planes).  Wavenumbers are
recomputed here on purpose, with no helper shared with the library code.

Recording every depth plane of one run started from a unit point source on
the sensor plane gives the whole kernel library at once (the reciprocity
argument of the library discussion in Sec. 3.2): in a homogeneous medium the
field at depth z_l due to a source at depth 0 equals the field at depth 0
due to a source at z_l.
"""
from __future__ import annotations

import numpy as np


def simulate(x: np.ndarray, dx: float, dy: float, dz: float, dt: float,
             c: float, nt: int, nz_sim: int, planes=None) -> np.ndarray:
    """Sensor-plane time series d[n, j, i] for the initial pressure x[l, j, i];
    with `planes` (depth indices), the field recorded on each of those planes
    instead: d[n, a, j, i] for plane planes[a]."""
    nz, ny, nx = x.shape
    assert nz_sim >= nz
    vol = np.zeros((nz_sim, ny, nx))
    vol[:nz] = x
    kz = 2.0 * np.pi * np.fft.fftfreq(nz_sim, d=dz)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=dy)
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=dx)
    K = np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    two_cos = 2.0 * np.cos(c * dt * K)
    rec = [0] if planes is None else list(planes)
    d = np.empty((nt, len(rec), ny, nx))
    p_prev = None
    p_cur = np.fft.fftn(vol)
    for n in range(nt):
        field = np.fft.ifftn(p_cur)
        d[n] = field[rec].real
        if n == 0:
            p_next = 0.5 * two_cos * p_cur
        else:
            p_next = two_cos * p_cur - p_prev
        p_prev, p_cur = p_cur, p_next
    return d[:, 0] if planes is None else d
