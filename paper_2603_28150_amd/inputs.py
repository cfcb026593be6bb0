"""Seeded synthetic inputs: objects (initial pressure) and noise.

This module holds none of the operator's arithmetic; it only draws arrays.
Both the GPU path and the CPU reference consume what it produces, so it
depends on numpy alone.  Shapes follow the operator's layouts: objects are
[Nz, Ny, Nx] (x fastest), data-shaped arrays are [Nt, Ny, Nx].

Objects stand in for the paper's workloads, which are not available:
* ``gaussian_blobs``: a few isotropic Gaussian absorbers, a small-scale
  stand-in for bead phantoms (Sec. 3.3);
* ``vascular_phantom``: random polyline tubes roughly parallel to the sensor,
  shaped like the wire phantom and in-vivo vasculature (Sec. 3.3-3.4);
* ``gaussian_random``: i.i.d. N(0, 1) voxels, the "Gaussian random
  initial-pressure distributions" of the forward-model validation (Sec. 3.1).
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def gaussian_random(shape, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(shape)


def _periodic_delta(coord: np.ndarray, centre: float, n: int) -> np.ndarray:
    d = coord - centre
    return d - n * np.round(d / n)


def gaussian_blobs(shape, seed: int, n_blobs: int = 4, sigma=(1.0, 3.0),
                   amp=(0.2, 1.0)) -> np.ndarray:
    """Sum of isotropic Gaussian blobs (sigma in voxels) with centres uniform
    in the volume; periodic distance in x and y, truncated in z."""
    nz, ny, nx = shape
    g = rng(seed)
    z = np.arange(nz)[:, None, None]
    y = np.arange(ny)[None, :, None]
    x = np.arange(nx)[None, None, :]
    out = np.zeros(shape)
    for _ in range(n_blobs):
        cz, cy, cx = g.uniform(0, nz), g.uniform(0, ny), g.uniform(0, nx)
        s = g.uniform(*sigma)
        a = g.uniform(*amp)
        r2 = (z - cz) ** 2 + _periodic_delta(y, cy, ny) ** 2 + _periodic_delta(x, cx, nx) ** 2
        out += a * np.exp(-0.5 * r2 / (s * s))
    return out


def vascular_phantom(shape, seed: int, n_tubes: int = 40, radius=(1.0, 3.0),
                     amp=(0.2, 1.0), n_segments: int = 6,
                     seg_len=(0.1, 0.3), turn_deg: float = 20.0) -> np.ndarray:
    """Random polyline tubes in a zero background.

    Each tube starts at a uniform point with z in [0.1, 0.9]*Nz and takes
    ``n_segments`` straight segments of length U(seg_len)*Nx; the initial
    direction is a random unit vector whose z component is damped by 0.3
    (vessels run roughly parallel to the sensor plane) and it turns by a
    N(0, turn_deg) rotation per segment.  A voxel at distance dist from the
    segment axis gets a * clip(r + 0.5 - dist, 0, 1); tubes combine by max.
    Distances wrap in x and y; z is clipped to the volume.
    """
    nz, ny, nx = shape
    g = rng(seed)
    out = np.zeros(shape)
    for _ in range(n_tubes):
        r = g.uniform(*radius)
        a = g.uniform(*amp)
        p = np.array([g.uniform(0.1, 0.9) * nz, g.uniform(0, ny), g.uniform(0, nx)])
        d = g.standard_normal(3)
        d[0] *= 0.3
        d /= np.linalg.norm(d)
        for _ in range(n_segments):
            length = g.uniform(*seg_len) * nx
            q = p + length * d
            _stamp_segment(out, p, q, r, a)
            p = q
            p[0] = min(max(p[0], 0.0), nz - 1.0)
            # random small rotation of the direction
            axis = g.standard_normal(3)
            axis -= axis.dot(d) * d
            axis /= np.linalg.norm(axis) + 1e-30
            ang = np.deg2rad(g.normal(0.0, turn_deg))
            d = np.cos(ang) * d + np.sin(ang) * axis
            d[0] *= 0.3 if abs(d[0]) > 0.5 else 1.0
            d /= np.linalg.norm(d)
    return out


def _stamp_segment(out, p, q, r, a):
    nz, ny, nx = out.shape
    lo = np.floor(np.minimum(p, q) - r - 1).astype(int)
    hi = np.ceil(np.maximum(p, q) + r + 1).astype(int)
    zs = np.arange(max(lo[0], 0), min(hi[0], nz - 1) + 1)
    if zs.size == 0:
        return
    ys = np.arange(lo[1], hi[1] + 1)
    xs = np.arange(lo[2], hi[2] + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    P = np.stack([Z, Y, X], axis=-1).astype(np.float64)
    seg = q - p
    L2 = float(seg.dot(seg)) or 1e-30
    t = np.clip(((P - p) @ seg) / L2, 0.0, 1.0)
    closest = p + t[..., None] * seg
    dist = np.linalg.norm(P - closest, axis=-1)
    val = a * np.clip(r + 0.5 - dist, 0.0, 1.0)
    yi = np.mod(ys, ny)
    xi = np.mod(xs, nx)
    sub = out[np.ix_(zs, yi, xi)]
    np.maximum(sub, val, out=sub)
    out[np.ix_(zs, yi, xi)] = sub


def noise_like(shape, seed: int) -> np.ndarray:
    """Standard normal noise; the caller scales it to the wanted level
    (sigma = nu * RMS(clean data): nu = 0.01 for 1 %, 10^(-20/20) for 20 dB)."""
    return rng(seed).standard_normal(shape)


NOISE_1PCT = 0.01
NOISE_20DB = 10.0 ** (-20.0 / 20.0)


def bandpass_fir(ntaps: int, f_lo: float, f_hi: float, dt: float) -> np.ndarray:
    """Causal band-pass impulse response for a sensor model: a Hann-windowed
    difference of two sinc low-passes (cut-offs f_lo < f_hi in Hz, sampling
    step dt), delayed by (ntaps-1)/2 samples and scaled to unit gain at the
    band centre.  Filter design only; it is an input of the operator."""
    n = np.arange(ntaps) - (ntaps - 1) / 2.0
    w = 0.5 - 0.5 * np.cos(2.0 * np.pi * np.arange(ntaps) / (ntaps - 1))
    h = (2 * f_hi * dt * np.sinc(2 * f_hi * dt * n) - 2 * f_lo * dt * np.sinc(2 * f_lo * dt * n)) * w
    fc = 0.5 * (f_lo + f_hi)
    gain = abs(np.sum(h * np.exp(-2j * np.pi * fc * dt * np.arange(ntaps))))
    return h / gain

