"""Step size, FISTA / projected gradient and dense matrices.

Test infrastructure only (see ``oracle/__init__``).

The inverse problem of Sec. 2.3 (eq. 12-14): minimise
f(x) + g(x), f(x) = 1/2 ||A x - d||^2 and g(x) = lambda ||x||_1 + i_{R+}(x),
by FISTA (Beck and Teboulle) with the gradient of eq. 15,
grad f(x) = A^T (A x - d).  Readings where the paper gives no detail: a
constant step tau, t_1 = 1, x_0 = 0, z_1 = x_0, no restart and no
backtracking, a fixed iteration count; the proximal map of tau*g is
max(v - tau*lambda, 0) under non-negativity and soft thresholding
otherwise; momentum off gives the projected (proximal) gradient method.
The momentum weights are computed in float64 on the host.
"""
from __future__ import annotations

import math

import numpy as np


def momentum_weights(niter: int, momentum: bool = True) -> list[float]:
    """beta_k for k = 1..niter: t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
    beta_k = (t_k - 1) / t_{k+1}, with t_1 = 1; all zero without momentum."""
    betas, t = [], 1.0
    for _ in range(niter):
        if not momentum:
            betas.append(0.0)
            continue
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        betas.append((t - 1.0) / t_next)
        t = t_next
    return betas


def prox(v: np.ndarray, tau: float, lam: float, nonneg: bool) -> np.ndarray:
    """Proximal map of tau * (lambda ||.||_1 + i_{R+}) (eq. 14)."""
    if nonneg:
        return np.maximum(v - tau * lam, 0.0)
    return np.sign(v) * np.maximum(np.abs(v) - tau * lam, 0.0)


def fista(A, AT, d, x_shape, niter: int, tau: float, lam: float = 0.0,
          nonneg: bool = True, momentum: bool = True, x0=None, z0=None,
          x_prev0=None, k0: int = 0, record=None):
    """FISTA iterates.  Returns the list [x_1, ..., x_niter] (float64).

    Starting state defaults to x_0 = z_1 = 0; (x_prev0, z0, k0) let a caller
    resume from iteration k0 (the momentum weight used at step k0+1 is
    beta_{k0+1}).  ``record(k, z, x)`` is called after every step if given.
    """
    x_prev = np.zeros(x_shape) if x_prev0 is None else np.array(x_prev0, dtype=np.float64)
    z = np.zeros(x_shape) if z0 is None else np.array(z0, dtype=np.float64)
    betas = momentum_weights(k0 + niter, momentum)[k0:]
    out = []
    for it in range(niter):
        g = AT(A(z) - d)
        x = prox(z - tau * g, tau, lam, nonneg)
        z = x + betas[it] * (x - x_prev)
        x_prev = x
        out.append(x)
        if record is not None:
            record(k0 + it + 1, z, x)
    return out


def objective(A, d, x, lam: float = 0.0) -> float:
    r = A(x) - d
    return 0.5 * float(np.vdot(r, r).real) + lam * float(np.abs(x).sum())


def power_iteration(A, AT, v0: np.ndarray, niter: int) -> list[float]:
    """Rayleigh quotients L_i = <v, A^T A v> with ||v|| = 1, v <- A^T A v / ||A^T A v||."""
    v = v0 / np.linalg.norm(v0)
    Ls = []
    for _ in range(niter):
        w = AT(A(v))
        Ls.append(float(np.vdot(v, w).real))
        v = w / np.linalg.norm(w)
    return Ls


def norm_exact(Hh: np.ndarray) -> float:
    """||A||^2 = max over transverse frequencies of the largest eigenvalue of
    H^_k^T H^_k (A is block diagonal in the transverse Fourier basis)."""
    ny, nh, nz, nt = Hh.shape
    Hk = Hh.reshape(ny * nh, nz, nt)
    G = np.einsum("kln,kmn->klm", Hk, Hk)
    return float(np.linalg.eigvalsh(G)[:, -1].max())


def dense_matrix(op, in_shape) -> np.ndarray:
    """Dense matrix of a linear map, built column by column."""
    n = int(np.prod(in_shape))
    cols = []
    e = np.zeros(n)
    for i in range(n):
        e[:] = 0.0
        e[i] = 1.0
        cols.append(np.asarray(op(e.reshape(in_shape))).ravel())
    return np.stack(cols, axis=1)
