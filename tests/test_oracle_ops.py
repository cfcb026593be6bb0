"""Pins of the oracle's forward operator A and adjoint A^T (CPU only)."""
import json
import os

import numpy as np
import pytest

from oracle.geometry import Geometry, paper_like
from oracle import hlib, operators as ops, wave3d, solvers
from paper_2603_28150_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def small():
    g = paper_like(12, 8, 5, 20)        # ragged, non-square, nz_sim = 16
    Hf = hlib.H_full(g)
    Hh = hlib.H_half(g)
    h = hlib.h_space(g, Hf)
    return g, Hf, Hh, h


def test_three_forms_of_A_agree(small):
    g, Hf, Hh, h = small
    x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=11)
    d1 = ops.A_direct(h, x)
    d2 = ops.A_dft(Hf, x)
    d3 = ops.A_fft(Hh, x)
    assert rel(d2, d1) < 1e-13
    assert rel(d3, d1) < 1e-13


def test_three_forms_of_AT_agree(small):
    g, Hf, Hh, h = small
    y = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=12)
    g1 = ops.AT_direct(h, y)
    g2 = ops.AT_dft(Hf, y)
    g3 = ops.AT_fft(Hh, y)
    assert rel(g2, g1) < 1e-13
    assert rel(g3, g1) < 1e-13


def test_dot_test(small):
    # <A x, y> = <x, A^T y> for the Euclidean products of eq. 10
    g, Hf, Hh, h = small
    for seed in range(5):
        x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=100 + seed)
        y = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=200 + seed)
        Ax = ops.A_fft(Hh, x)
        ATy = ops.AT_fft(Hh, y)
        lhs, rhs = np.vdot(Ax, y), np.vdot(x, ATy)
        assert abs(lhs - rhs) / (np.linalg.norm(Ax) * np.linalg.norm(y)) < 1e-12


def test_dense_transpose_brute_force():
    # A^T equals the transpose of the dense matrix of A (8^2 x 4 x 16)
    g = paper_like(8, 8, 4, 16)
    Hh = hlib.H_half(g)
    M = solvers.dense_matrix(lambda v: ops.A_fft(Hh, v), (g.nz, g.ny, g.nx))
    MT = solvers.dense_matrix(lambda v: ops.AT_fft(Hh, v), (g.nt, g.ny, g.nx))
    assert np.abs(MT - M.T).max() < 1e-13 * np.abs(M).max()


def test_shift_equivariance_and_impulse(small):
    g, Hf, Hh, h = small
    x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=13)
    d = ops.A_fft(Hh, x)
    xs = np.roll(x, shift=(3, 5), axis=(1, 2))
    ds = ops.A_fft(Hh, xs)
    assert rel(ds, np.roll(d, shift=(3, 5), axis=(1, 2))) < 1e-13
    # t = 0 shows the absorbers on the sensor plane only
    assert np.abs(d[0] - x[0]).max() < 1e-13 * np.abs(x).max()
    # a unit absorber at (0, 0, l) yields the kernel h_l
    for l in range(g.nz):
        e = np.zeros_like(x)
        e[l, 0, 0] = 1.0
        dl = ops.A_fft(Hh, e)
        assert np.abs(np.transpose(dl, (1, 2, 0)) - h[l]).max() < 1e-13


def test_linearity(small):
    g, Hf, Hh, h = small
    a = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=14)
    b = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=15)
    lhs = ops.A_fft(Hh, 2.0 * a - 3.0 * b)
    rhs = 2.0 * ops.A_fft(Hh, a) - 3.0 * ops.A_fft(Hh, b)
    assert rel(lhs, rhs) < 1e-13


def test_table1_analogue_against_independent_wave_solver():
    """Sec. 3.1, Table 1: the convolution operator reproduces a wave solver
    with matched discretisation and boundaries at rounding level, over 100
    Gaussian random objects."""
    with open(os.path.join(GOLDEN, "table1_forward_equivalence.json")) as f:
        paper = json.load(f)
    g = paper_like(16, 16, 8, 24)
    Hh = hlib.H_half(g)
    r2, rinf = [], []
    for s in range(100):
        x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=3000 + s)
        dm = ops.A_fft(Hh, x)
        dw = wave3d.simulate(x, g.dx, g.dy, g.dz, g.dt, g.c, g.nt, g.nq)
        r2.append(np.linalg.norm(dm - dw) / np.linalg.norm(dw))
        rinf.append(np.abs(dm - dw).max() / np.abs(dw).max())
    # rounding level: within 10x of the paper's max (FP64 throughout)
    assert np.median(r2) < 10 * paper["rel_l2"]["max"]
    assert max(r2) < 10 * paper["rel_l2"]["max"]
    assert max(rinf) < 10 * paper["rel_linf"]["max"]


def test_gaussian_pulse_matches_continuous_wave_equation():
    """Continuum pin of the physics and of every grid constant (dx, dy, dz,
    c, dt, time and depth origins): for a well-resolved Gaussian initial
    pressure the spherically symmetric solution of eq. 1-2 is
    p(R,t) = [(R-ct) p0(R-ct) + (R+ct) p0(R+ct)] / (2R).
    The discrete model must reproduce it at the sensor plane while no
    periodic image of the pulse can have arrived."""
    dx, dy, dz, c = 100e-6, 80e-6, 100e-6, 1500.0
    g = Geometry(nx=64, ny=64, nz=32, nt=112, dx=dx, dy=dy, dz=dz,
                 dt=0.3 * dx / c, c=c)
    sig = 250e-6
    cx, cy, z0 = 32 * dx, 32 * dy, 16 * dz
    zz = (np.arange(g.nz) * dz)[:, None, None]
    yy = (np.arange(g.ny) * dy)[None, :, None]
    xx = (np.arange(g.nx) * dx)[None, None, :]
    x = np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2 + (zz - z0) ** 2) / (2 * sig ** 2))
    d = ops.A_fft(hlib.H_half(g), x)

    def p0(r):
        return np.exp(-r ** 2 / (2 * sig ** 2))

    t = np.arange(g.nt) * g.dt
    checked = 0
    for (i, j) in [(32, 32), (35, 32), (32, 36), (28, 29), (38, 38)]:
        R = np.sqrt((i * dx - cx) ** 2 + (j * dy - cy) ** 2 + z0 ** 2)
        # nearest periodic image (transverse or in z)
        imgs = [np.sqrt((i * dx - cx - a * g.nx * dx) ** 2 + (j * dy - cy - b * g.ny * dy) ** 2 + z0 ** 2)
                for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]
        imgs.append(g.nq * dz - z0)
        t_lim = (min(imgs) - 8 * sig) / c
        sel = t < t_lim
        assert t_lim > (R + 3 * sig) / c      # the window holds the whole pulse peak
        exact = ((R - c * t) * p0(R - c * t) + (R + c * t) * p0(R + c * t)) / (2 * R)
        err = np.abs(d[sel, j, i] - exact[sel]).max() / np.abs(exact).max()
        assert err < 1e-7, (i, j, err)
        checked += 1
    assert checked == 5


def test_sampled_frequency_helpers(small):
    g, Hf, Hh, h = small
    x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=16)
    y = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=17)
    m = np.array([0, 3, 6, 1])
    p = np.array([0, 7, 4, 2])
    Hk = hlib.H_hat(g, m, p)
    D = ops.A_at_freqs(Hk, x, m, p)
    Dref = np.fft.rfft2(ops.A_fft(Hh, x), axes=(1, 2))[:, p, m].T
    assert np.abs(D - Dref).max() < 1e-12 * np.abs(Dref).max()
    G = ops.AT_at_freqs(Hk, y, m, p)
    Gref = np.fft.rfft2(ops.AT_fft(Hh, y), axes=(1, 2))[:, p, m].T
    assert np.abs(G - Gref).max() < 1e-12 * np.abs(Gref).max()
