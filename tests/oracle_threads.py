"""The oracle's kernel library built on several host threads.

Test infrastructure: splits the half-spectrum frequencies into blocks and
calls the oracle's direct q-sum (``oracle.hlib.H_hat``) on each block from a
thread pool (numpy releases the GIL inside its cosines and matrix products),
with the BLAS pool held to one thread per caller.  Every frequency is still
computed on its own by the oracle; only the order in which blocks are done
changes.  Sized for the host of the GPU machine (at most 16 threads).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
from threadpoolctl import threadpool_limits

from oracle import hlib


def host_threads() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def H_half(g, block: int = 128) -> np.ndarray:
    """float64 [Ny, Nx/2+1, Nz, Nt], equal to ``oracle.hlib.H_half(g)``."""
    nh = g.nx // 2 + 1
    nk = g.ny * nh
    out = np.empty((nk, g.nz, g.nt))
    k = np.arange(nk)
    m, p = k % nh, k // nh

    def run(s):
        out[s:s + block] = hlib.H_hat(g, m[s:s + block], p[s:s + block], chunk=block)

    with threadpool_limits(1), ThreadPoolExecutor(host_threads()) as ex:
        list(ex.map(run, range(0, nk, block)))
    return out.reshape(g.ny, nh, g.nz, g.nt)
