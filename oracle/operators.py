"""Forward operator A (the paper's H) and its adjoint A^T (the paper's H*).

Test infrastructure only (see ``oracle/__init__``).

Array layouts (C order, x fastest): object x[l, j, i] of shape [Nz, Ny, Nx],
data d[n, j, i] of shape [Nt, Ny, Nx].  All arithmetic is float64.

Three independent realisations of the same discrete operator:

* ``A_direct`` / ``AT_direct``: eq. 7 written out as a sum over depths of 2D
  circular convolutions with the real-space kernels h_l, and eq. 11 as the
  matching sum over time of 2D circular correlations (periodic transverse
  boundary, so shifts wrap).  Tiny grids only.
* ``A_dft`` / ``AT_dft``: the three steps of the FFT realisation of
  Sec. 3.2 (transverse DFT of every depth slice, per-frequency
  multiply-accumulate over depth, inverse transverse DFT of every time
  sample) with dense DFT matrices on the full spectrum; the adjoint runs the
  same steps with conj(H^) and the sum over time.
* ``A_fft`` / ``AT_fft``: the same with numpy's r2c/c2r FFTs (pocketfft) on
  the half spectrum, the only form fast enough for long iterations on large
  grids.

For the zero-padded linear convolution of Sec. 2.3, ``A_direct_linear``
writes the sum over signed source-sensor offsets out, and ``A_linear`` /
``AT_linear`` pad, apply the periodic operator of the doubled grid and crop.

The inner products are the unweighted Euclidean ones of eq. 10, so A^T is the
plain matrix transpose.
"""
from __future__ import annotations

import numpy as np

from .hlib import dft_matrix


# ---------------------------------------------------------------- direct sums
def A_direct(h: np.ndarray, x: np.ndarray) -> np.ndarray:
    """d[n, j, i] = sum_l sum_{i',j'} h[l, j-j', i-i', n] x[l, j', i'] (eq. 7)."""
    nz, ny, nx, nt = h.shape
    assert x.shape == (nz, ny, nx)
    d = np.zeros((nt, ny, nx))
    for b in range(ny):
        for a in range(nx):
            xs = np.roll(x, shift=(b, a), axis=(1, 2))        # x[l, j-b, i-a]
            d += np.tensordot(h[:, b, a, :], xs, axes=([0], [0]))
    return d


def AT_direct(h: np.ndarray, d: np.ndarray) -> np.ndarray:
    """g[l, j', i'] = sum_n sum_{i,j} h[l, j-j', i-i', n] d[n, j, i] (eq. 11)."""
    nz, ny, nx, nt = h.shape
    assert d.shape == (nt, ny, nx)
    g = np.zeros((nz, ny, nx))
    for b in range(ny):
        for a in range(nx):
            ds = np.roll(d, shift=(-b, -a), axis=(1, 2))      # d[n, j'+b, i'+a]
            g += np.tensordot(h[:, b, a, :], ds, axes=([1], [0]))
    return g


# ------------------------------------------------------ dense DFT (full grid)
def A_dft(Hf: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A by dense DFT matrices.  Hf: H^ on the full grid [Ny, Nx, Nz, Nt]."""
    ny, nx, nz, nt = Hf.shape
    Fy, Fx = dft_matrix(ny, -1.0), dft_matrix(nx, -1.0)
    X = np.einsum("pj,lji,mi->pml", Fy, x, Fx, optimize=True)      # step (i)
    D = np.einsum("pmln,pml->pmn", Hf, X, optimize=True)            # step (ii)
    d = np.einsum("jp,pmn,im->nji", Fy.conj(), D, Fx.conj(), optimize=True)  # (iii)
    d /= nx * ny
    if np.abs(d.imag).max() > 1e-12 * max(1e-300, np.abs(d.real).max()):
        raise AssertionError("A_dft output is not real")
    return d.real


def AT_dft(Hf: np.ndarray, d: np.ndarray) -> np.ndarray:
    """A^T by dense DFT matrices: same steps, conj(H^), sum over time."""
    ny, nx, nz, nt = Hf.shape
    Fy, Fx = dft_matrix(ny, -1.0), dft_matrix(nx, -1.0)
    R = np.einsum("pj,nji,mi->pmn", Fy, d, Fx, optimize=True)
    G = np.einsum("pmln,pmn->pml", Hf.conj(), R, optimize=True)
    g = np.einsum("jp,pml,im->lji", Fy.conj(), G, Fx.conj(), optimize=True)
    g /= nx * ny
    if np.abs(g.imag).max() > 1e-12 * max(1e-300, np.abs(g.real).max()):
        raise AssertionError("AT_dft output is not real")
    return g.real


# --------------------------------------------------- pocketfft, half spectrum
def contract_A(Hk: np.ndarray, Xk: np.ndarray) -> np.ndarray:
    """Step (ii) of A (Sec. 3.2, eq. 16): D^[k, n] = sum_l H^[k, l, n] X^[k, l]
    for every frequency k, as one (1 x nz) by (nz x nt) matrix product per
    frequency.  Hk: real or complex [K, nz, nt]; Xk: complex [K, nz]."""
    if np.iscomplexobj(Hk):
        return np.matmul(Xk[:, None, :], Hk)[:, 0, :]
    Xs = np.stack([Xk.real, Xk.imag], axis=1)             # [K, 2, nz]
    Ds = np.matmul(Xs, Hk)                                 # [K, 2, nt]
    return Ds[:, 0, :] + 1j * Ds[:, 1, :]


def contract_AT(Hk: np.ndarray, Rk: np.ndarray) -> np.ndarray:
    """Step (ii) of A^T (eq. 11): G^[k, l] = sum_n conj(H^[k, l, n]) R^[k, n],
    one (nz x nt) by (nt x 1) product per frequency.  Hk: [K, nz, nt]; Rk:
    complex [K, nt]."""
    if np.iscomplexobj(Hk):
        return np.matmul(np.conj(Hk), Rk[:, :, None])[:, :, 0]
    Rs = np.stack([Rk.real, Rk.imag], axis=2)             # [K, nt, 2]
    Gs = np.matmul(Hk, Rs)                                 # [K, nz, 2]
    return Gs[:, :, 0] + 1j * Gs[:, :, 1]


def A_fft(Hh: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A with r2c/c2r FFTs.  Hh: H^ on the half spectrum [Ny, Nx/2+1, Nz, Nt]."""
    ny, nh, nz, nt = Hh.shape
    nx = x.shape[-1]
    X = np.fft.rfft2(x, axes=(1, 2))                       # [nz, ny, nh]
    D = contract_A(Hh.reshape(ny * nh, nz, nt), X.reshape(nz, ny * nh).T)   # [K, nt]
    return np.fft.irfft2(D.T.reshape(nt, ny, nh), s=(ny, nx), axes=(1, 2))


def AT_fft(Hh: np.ndarray, d: np.ndarray) -> np.ndarray:
    """A^T with r2c/c2r FFTs (conj(H^) = H^ up to rounding, kept explicit)."""
    ny, nh, nz, nt = Hh.shape
    nx = d.shape[-1]
    R = np.fft.rfft2(d, axes=(1, 2))                       # [nt, ny, nh]
    G = contract_AT(Hh.reshape(ny * nh, nz, nt), R.reshape(nt, ny * nh).T)  # [K, nz]
    return np.fft.irfft2(G.T.reshape(nz, ny, nh), s=(ny, nx), axes=(1, 2))


# ------------------------------------ zero-padded linear convolution (Sec. 2.3)
# The object and the data live on the Ny x Nx window; the kernels are those of
# the doubled periodic grid (2Ny x 2Nx), indexed by the signed offset between
# sensor and source, which stays inside (-Ny, Ny) x (-Nx, Nx).
def pad2(f: np.ndarray, py: int, px: int) -> np.ndarray:
    """Zero-pad the last two axes of f to (py, px) (data at the low indices)."""
    out = np.zeros(f.shape[:-2] + (py, px))
    out[..., :f.shape[-2], :f.shape[-1]] = f
    return out


def A_direct_linear(h2: np.ndarray, x: np.ndarray) -> np.ndarray:
    """d[n, j, i] = sum_l sum_{j', i' in window} h2[l, j-j', i-i', n] x[l, j', i']
    with negative offsets read from the doubled grid's kernel at +2N.
    h2: [nz, 2Ny, 2Nx, nt]; tiny grids only."""
    nz, py, px, nt = h2.shape
    _, ny, nx = x.shape
    d = np.zeros((nt, ny, nx))
    for b in range(-(ny - 1), ny):
        for a in range(-(nx - 1), nx):
            hb = h2[:, b % py, a % px, :]                     # [nz, nt]
            js, je = max(0, -b), min(ny, ny - b)              # source rows j' with j'+b in window
            is_, ie = max(0, -a), min(nx, nx - a)
            d[:, js + b:je + b, is_ + a:ie + a] += np.tensordot(hb, x[:, js:je, is_:ie], axes=([0], [0]))
    return d


def A_linear(Hh2: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A with the zero-padded linear convolution: pad, A on the doubled grid
    (Hh2 = H^ of the doubled grid, half spectrum), crop."""
    py, nh2 = Hh2.shape[:2]
    _, ny, nx = x.shape
    return A_fft(Hh2, pad2(x, py, 2 * (nh2 - 1)))[:, :ny, :nx]


def AT_linear(Hh2: np.ndarray, d: np.ndarray) -> np.ndarray:
    """A^T of A_linear: pad the data, A^T on the doubled grid, crop."""
    py, nh2 = Hh2.shape[:2]
    _, ny, nx = d.shape
    return AT_fft(Hh2, pad2(d, py, 2 * (nh2 - 1)))[:, :ny, :nx]


# --------------------------------------------------- sensor response along t
def filter_t(d: np.ndarray, r) -> np.ndarray:
    """Causal filtering of data d[n, j, i] along time: sum_j r[j] d[n-j]."""
    r = np.asarray(r, dtype=np.float64)
    nt = d.shape[0]
    out = np.zeros(d.shape)
    for j in range(min(len(r), nt)):
        out[j:] += r[j] * d[:nt - j]
    return out


def filter_t_adjoint(d: np.ndarray, r) -> np.ndarray:
    """Adjoint of filter_t (anti-causal correlation): sum_j r[j] d[n+j]."""
    r = np.asarray(r, dtype=np.float64)
    nt = d.shape[0]
    out = np.zeros(d.shape)
    for j in range(min(len(r), nt)):
        out[:nt - j] += r[j] * d[j:]
    return out


# ------------------------------------------------- scan-grid sampling operator
def sample(d: np.ndarray, sx: int, sy: int) -> np.ndarray:
    """S: the data at every sx-th column and sy-th row of the sensor grid."""
    return np.ascontiguousarray(d[..., ::sy, ::sx])


def sample_adjoint(ds: np.ndarray, sx: int, sy: int, ny: int, nx: int) -> np.ndarray:
    """S^T: scan-grid data placed back on the sensor grid, zeros elsewhere."""
    out = np.zeros(ds.shape[:-2] + (ny, nx))
    out[..., ::sy, ::sx] = ds
    return out


# ----------------------------------------- single frequencies of large grids
def dft_at(f: np.ndarray, m_idx, p_idx) -> np.ndarray:
    """Forward 2D DFT of every slice of f[s, j, i] at the frequencies
    (m_idx[k], p_idx[k]) by direct sums: returns complex [K, S]."""
    s, ny, nx = f.shape
    m_idx = np.asarray(m_idx).ravel()
    p_idx = np.asarray(p_idx).ravel()
    ey = np.exp(-2j * np.pi * np.outer(p_idx, np.arange(ny)) / ny)   # [K, ny]
    ex = np.exp(-2j * np.pi * np.outer(m_idx, np.arange(nx)) / nx)   # [K, nx]
    out = np.empty((m_idx.size, s), dtype=np.complex128)
    for k in range(m_idx.size):
        out[k] = np.einsum("j,sji,i->s", ey[k], f, ex[k], optimize=True)
    return out


def A_at_freqs(Hk: np.ndarray, x: np.ndarray, m_idx, p_idx) -> np.ndarray:
    """Spectrum of A x at the given frequencies: D^[k, n] = sum_l H^[k,l,n] X^[k,l]."""
    X = dft_at(x, m_idx, p_idx)                            # [K, nz]
    return contract_A(Hk, X)


def AT_at_freqs(Hk: np.ndarray, d: np.ndarray, m_idx, p_idx) -> np.ndarray:
    """Spectrum of A^T d at the given frequencies: G^[k, l] = sum_n H^[k,l,n] R^[k,n]."""
    R = dft_at(d, m_idx, p_idx)                            # [K, nt]
    return contract_AT(Hk, R)
