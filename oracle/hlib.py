"""Kernel library H^[k, l, n] of the depth-dependent transverse model.

Test infrastructure only (see ``oracle/__init__``).

The paper obtains one impulse response per depth, h_z(r_perp, t), by
simulating a unit point absorber at that depth and recording the field on
the sensor plane (Sec. 2.1, and the library discussion of Sec. 3.2).  Here
the simulation is done exactly: on the periodic grid the semi-discrete wave
field is p^(k, t) = cos(c |k| t) p0^(k) (eq. 1-2 with zero initial velocity),
so the field on the sensor plane z = 0 due to a unit absorber at depth z_l is,
in the transverse Fourier domain,

    H^[(m,p), l, n] = (1/nq) * sum_q cos(c t_n |k(m,p,q)|) * exp(-2 pi i q l / nq)

with |k|^2 = kx(m)^2 + ky(p)^2 + kz(q)^2.  The q-sum is evaluated directly
(no FFT); the result is real because the summand is even in q, and the
imaginary part is checked to vanish.  The real-space kernels h_l(i, j, n) of
eq. 7 are the inverse 2D DFT of H^ over (m, p), evaluated with dense DFT
matrices.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, kx_full, ky_full, kz_full, time_axis


def H_hat(g: Geometry, m_idx, p_idx, chunk: int = 256) -> np.ndarray:
    """H^ for the transverse frequencies (m_idx[i], p_idx[i]).

    m_idx, p_idx are DFT indices in [0, Nx) and [0, Ny).  Returns a float64
    array [K, Nz, Nt].  Raises if the imaginary part of the direct sum is not
    at rounding level.
    """
    m_idx = np.asarray(m_idx, dtype=np.int64).ravel()
    p_idx = np.asarray(p_idx, dtype=np.int64).ravel()
    assert m_idx.shape == p_idx.shape
    kx, ky, kz = kx_full(g), ky_full(g), kz_full(g)
    t = time_axis(g)
    nq = g.nq
    q = np.arange(nq)
    l = np.arange(g.nz)
    # exp(-2 pi i q l / nq) / nq, the DFT over the periodic z-grid evaluated
    # at the depths of the object grid
    E = np.exp(-2j * np.pi * np.outer(q, l) / nq) / nq  # [nq, nz]
    # the phases are real: real and imaginary parts of the sum as two real
    # matrix products
    Er, Ei = np.ascontiguousarray(E.real), np.ascontiguousarray(E.imag)
    out = np.empty((m_idx.size, g.nz, g.nt), dtype=np.float64)
    for s in range(0, m_idx.size, chunk):
        mm = m_idx[s:s + chunk]
        pp = p_idx[s:s + chunk]
        kperp2 = kx[mm] ** 2 + ky[pp] ** 2                        # [K]
        kabs = np.sqrt(kperp2[:, None] + kz[None, :] ** 2)         # [K, nq]
        phase = np.cos(g.c * t[None, :, None] * kabs[:, None, :])  # [K, nt, nq]
        Sr = phase @ Er                                            # [K, nt, nz]
        Si = phase @ Ei
        scale = max(1.0, float(np.abs(Sr).max()))
        if np.abs(Si).max() > 1e-13 * scale:
            raise AssertionError("imaginary part of H^ is not at rounding level")
        out[s:s + chunk] = np.transpose(Sr, (0, 2, 1))
    return out


def H_full(g: Geometry) -> np.ndarray:
    """H^ on the full transverse DFT grid: float64 [Ny, Nx, Nz, Nt]."""
    p, m = np.meshgrid(np.arange(g.ny), np.arange(g.nx), indexing="ij")
    return H_hat(g, m.ravel(), p.ravel()).reshape(g.ny, g.nx, g.nz, g.nt)


def H_half(g: Geometry) -> np.ndarray:
    """H^ on the r2c half spectrum (m = 0..Nx/2): float64 [Ny, Nx/2+1, Nz, Nt]."""
    p, m = np.meshgrid(np.arange(g.ny), np.arange(g.n_half), indexing="ij")
    return H_hat(g, m.ravel(), p.ravel()).reshape(g.ny, g.n_half, g.nz, g.nt)


def dft_matrix(n: int, sign: float) -> np.ndarray:
    """Dense DFT matrix F[a, b] = exp(sign * 2 pi i a b / n)."""
    a = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(a, a) / n)


def h_space(g: Geometry, Hf: np.ndarray | None = None) -> np.ndarray:
    """Real-space kernels h[l, j, i, n] (eq. 7): the inverse 2D DFT of H^
    over the transverse frequencies, by dense DFT matrices."""
    if Hf is None:
        Hf = H_full(g)
    Fy_inv = dft_matrix(g.ny, +1.0)
    Fx_inv = dft_matrix(g.nx, +1.0)
    # h[j, i, l, n] = 1/(NxNy) sum_{p,m} e^{+2 pi i p j/Ny} H[p,m,l,n] e^{+2 pi i m i/Nx}
    h = np.einsum("jp,pmln,im->jiln", Fy_inv, Hf, Fx_inv, optimize=True)
    h /= g.nx * g.ny
    if np.abs(h.imag).max() > 1e-12 * max(1.0, np.abs(h.real).max()):
        raise AssertionError("real-space kernels are not real")
    return np.ascontiguousarray(np.transpose(h.real, (2, 0, 1, 3)))


def with_sensor_response(H: np.ndarray, r) -> np.ndarray:
    """Library seen through sensors with the causal impulse response r (taps
    at t = 0, dt, ...), folded in along the time axis (the last one):
    H'[..., n] = sum_{j <= min(n, len(r)-1)} r[j] H[..., n-j]; nothing is
    recorded before t = 0.  r = [1] gives the ideal point sensors."""
    r = np.asarray(r, dtype=np.float64)
    nt = H.shape[-1]
    out = np.zeros(H.shape, dtype=np.result_type(H, r))
    for j in range(min(len(r), nt)):
        out[..., j:] += r[j] * H[..., :nt - j]
    return out

