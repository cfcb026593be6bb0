"""Grids and wavenumbers of the discrete planar geometry.

Test infrastructure only (see ``oracle/__init__``).

The object lives on G_rho = G_xy x G_z and the data on G_d = G_xy x T
(paper Sec. 2.2).  Readings used here where the paper leaves things open:

* the sensor plane is depth index l = 0 (z_l = l*dz), and the time grid is
  t_n = n*dt for n = 0..Nt-1 (it includes t = 0);
* the transverse boundary is periodic at Nx x Ny (circular convolution), or,
  for the zero-padded linear convolution, periodic at a period of at least
  2Nx x 2Ny with the object padded and the data cropped (``linear_grid``;
  ``doubled`` is exactly 2Nx x 2Ny);
* the simulated medium is periodic in z with period nz_sim >= Nz; by default
  nz_sim is the smallest power of two >= Nz + ceil(c*dt*(Nt-1)/dz) + 1, so
  that the wrapped image of the object cannot reach the sensor within the
  record;
* wavenumbers are in numpy ``fftfreq`` order (Nyquist bin at -N/2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Geometry:
    nx: int
    ny: int
    nz: int
    nt: int
    dx: float
    dy: float
    dz: float
    dt: float
    c: float
    nz_sim: int = 0  # 0 selects the default rule below

    @property
    def nq(self) -> int:
        """z-period of the simulated medium, in grid points."""
        if self.nz_sim:
            return int(self.nz_sim)
        reach = math.ceil(self.c * self.dt * (self.nt - 1) / self.dz)
        need = self.nz + reach + 1
        return 1 << max(0, math.ceil(math.log2(need)))

    @property
    def n_half(self) -> int:
        """Number of r2c half-spectrum columns along x."""
        return self.nx // 2 + 1


def kx_full(g: Geometry) -> np.ndarray:
    """k_x for every DFT index m = 0..Nx-1 (rad/m)."""
    return 2.0 * np.pi * np.fft.fftfreq(g.nx, d=g.dx)


def ky_full(g: Geometry) -> np.ndarray:
    """k_y for every DFT index p = 0..Ny-1 (rad/m)."""
    return 2.0 * np.pi * np.fft.fftfreq(g.ny, d=g.dy)


def kz_full(g: Geometry) -> np.ndarray:
    """k_z for every index q = 0..nz_sim-1 of the periodic z-grid (rad/m)."""
    return 2.0 * np.pi * np.fft.fftfreq(g.nq, d=g.dz)


def doubled(g: Geometry) -> Geometry:
    """The 2Nx x 2Ny periodic grid on which the zero-padded linear
    convolution of the Nx x Ny window is taken (same physics and z-period)."""
    from dataclasses import replace
    return replace(g, nx=2 * g.nx, ny=2 * g.ny, nz_sim=g.nq)


def transform_sizes():
    """Periods the zero-padded convolution may be taken on (any period >= 2N
    keeps every source-sensor offset of an N-point window from wrapping;
    these are the ones with fast transforms): 2^a 3^b with b <= 3, multiples
    of 4 in [16, 1024], and at least 48 when b > 0."""
    return sorted(v for v in (2 ** a * 3 ** b for a in range(2, 11) for b in range(4))
                  if 16 <= v <= 1024 and (v & (v - 1) == 0 or v >= 48))


def linear_grid(g: Geometry) -> Geometry:
    """The periodic grid of the zero-padded linear convolution of an Nx x Ny
    window: along each axis the smallest of ``transform_sizes`` that is
    >= max(16, 2N), so no source-sensor offset inside the window wraps
    (equals ``doubled`` when N is a power of two >= 8)."""
    from dataclasses import replace

    def size(n):
        return min(p for p in transform_sizes() if p >= max(16, 2 * n))
    return replace(g, nx=size(g.nx), ny=size(g.ny), nz_sim=g.nq)


def time_axis(g: Geometry) -> np.ndarray:
    return np.arange(g.nt, dtype=np.float64) * g.dt


def paper_like(nx, ny, nz, nt, dx=100e-6, c=1500.0, cfl=0.3, nz_sim=0) -> Geometry:
    """Geometry with dx = dy = dz and dt = cfl*dx/c, the physics of the
    synthetic workloads used throughout the tests."""
    return Geometry(nx=nx, ny=ny, nz=nz, nt=nt, dx=dx, dy=dx, dz=dx,
                    dt=cfl * dx / c, c=c, nz_sim=nz_sim)
