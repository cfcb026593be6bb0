"""Pins of the oracle's zero-padded linear convolution (Sec. 2.3): the
pad / doubled-grid / crop form against the direct sum over signed offsets,
the adjoint and transpose identities, and the physics: a pulse whose
wavefront reaches the edges of the window reproduces the free-space
closed-form solution there, where the periodic operator of the same window
already shows the wrapped wavefront."""
import numpy as np
import pytest

from oracle import hlib, operators as ops
from oracle.geometry import Geometry, doubled, linear_grid, paper_like, transform_sizes
from paper_2603_28150_amd import inputs


@pytest.mark.parametrize("shape", [(8, 8, 3, 12), (8, 4, 2, 9), (4, 8, 3, 7), (6, 5, 3, 10), (5, 7, 2, 9),
                                   (20, 8, 2, 6), (24, 40, 2, 5), (36, 4, 1, 4)])
def test_linear_fft_form_equals_direct_offset_sums(shape):
    # power-of-two windows on the doubled grid, other windows on the
    # smallest transform size holding twice the window (48 x 16, 48 x 96 and
    # 72 x 16 for the last three: periods 3 * 2^a and 9 * 2^a)
    nx, ny, nz, nt = shape
    g = paper_like(nx, ny, nz, nt)
    g2 = linear_grid(g)
    assert g2.nx >= 2 * nx and g2.ny >= 2 * ny
    if nx & (nx - 1) == 0 and ny & (ny - 1) == 0 and min(nx, ny) >= 8:
        assert g2 == doubled(g)
    Hf2 = hlib.H_full(g2)
    h2 = hlib.h_space(g2, Hf2)                        # [nz, 2ny, 2nx, nt]
    Hh2 = hlib.H_half(g2)
    x = inputs.gaussian_random((nz, ny, nx), seed=701)
    d_direct = ops.A_direct_linear(h2, x)
    d_fft = ops.A_linear(Hh2, x)
    assert np.abs(d_fft - d_direct).max() <= 1e-12 * np.abs(d_direct).max()
    # the linear operator is not the periodic one of the window
    d_per = ops.A_fft(hlib.H_half(g), x)
    assert np.abs(d_per - d_fft).max() > 1e-3 * np.abs(d_fft).max()


def test_linear_grid_sizes_for_the_paper_shapes():
    # the wire phantom (202^2) and the in vivo grid (384 x 326): the period
    # holds twice the window, is one of the fast transform sizes, and no
    # smaller such size would
    sizes = transform_sizes()
    for n, want in [(202, 432), (326, 768), (384, 768), (16, 32), (20, 48), (100, 216), (512, 1024), (34, 72)]:
        p = linear_grid(paper_like(n, n, 1, 2)).nx
        assert p == want and p >= 2 * n and p in sizes
        assert not [q for q in sizes if 2 * n <= q < p]


def test_linear_adjoint_and_dense_transpose():
    g = paper_like(8, 4, 3, 10)
    Hh2 = hlib.H_half(doubled(g))
    n_in, n_out = g.nz * g.ny * g.nx, g.nt * g.ny * g.nx
    A = np.empty((n_out, n_in))
    for c in range(n_in):
        e = np.zeros(n_in)
        e[c] = 1.0
        A[:, c] = ops.A_linear(Hh2, e.reshape(g.nz, g.ny, g.nx)).ravel()
    AT = np.empty((n_in, n_out))
    for c in range(n_out):
        e = np.zeros(n_out)
        e[c] = 1.0
        AT[:, c] = ops.AT_linear(Hh2, e.reshape(g.nt, g.ny, g.nx)).ravel()
    assert np.abs(AT - A.T).max() <= 1e-13 * np.abs(A).max()
    x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=702)
    y = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=703)
    lhs = np.vdot(ops.A_linear(Hh2, x), y)
    rhs = np.vdot(x, ops.AT_linear(Hh2, y))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(ops.A_linear(Hh2, x)) * np.linalg.norm(y)


def test_linear_pulse_near_edge_matches_free_space():
    """Gaussian pulse (sigma 2.5 cells) in a 32 x 32 window, 6 sigma from every
    face so that the window holds it whole.  The free-space solution
    [(R-ct) p0(R-ct) + (R+ct) p0(R+ct)] / (2R) must hold at sensor points up
    to the window's edges until an image of the doubled grid (period 64) or
    of the z-period could arrive; the periodic operator of the window
    (period 32) departs from it, its image reaching the edge points together
    with the direct wave."""
    dx, dy, dz, c = 100e-6, 100e-6, 100e-6, 1500.0
    g = Geometry(nx=32, ny=32, nz=32, nt=128, dx=dx, dy=dy, dz=dz, dt=0.3 * dx / c, c=c)
    g2 = doubled(g)
    sig = 250e-6
    cx, cy, z0 = 15 * dx, 15 * dy, 16 * dz
    zz = (np.arange(g.nz) * dz)[:, None, None]
    yy = (np.arange(g.ny) * dy)[None, :, None]
    xx = (np.arange(g.nx) * dx)[None, None, :]
    x = np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2 + (zz - z0) ** 2) / (2 * sig ** 2))
    d_lin = ops.A_linear(hlib.H_half(g2), x)
    d_per = ops.A_fft(hlib.H_half(g), x)

    def p0(r):
        return np.exp(-r ** 2 / (2 * sig ** 2))

    t = np.arange(g.nt) * g.dt
    periodic_departs = False
    for (i, j) in [(15, 15), (30, 15), (15, 30), (28, 26), (2, 15)]:
        R = np.sqrt((i * dx - cx) ** 2 + (j * dy - cy) ** 2 + z0 ** 2)
        exact = ((R - c * t) * p0(R - c * t) + (R + c * t) * p0(R + c * t)) / (2 * R)

        def t_limit(px, py):
            imgs = [np.sqrt((i * dx - cx - a * px * dx) ** 2 + (j * dy - cy - b * py * dy) ** 2 + z0 ** 2)
                    for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]
            imgs.append(g.nq * dz - z0)
            return (min(imgs) - 8 * sig) / c

        sel = t < t_limit(64, 64)
        assert t_limit(64, 64) > (R + 3 * sig) / c      # the window holds the pulse peak
        err = np.abs(d_lin[sel, j, i] - exact[sel]).max() / np.abs(exact).max()
        assert err < 1e-7, (i, j, err)
        err_per = np.abs(d_per[sel, j, i] - exact[sel]).max() / np.abs(exact).max()
        periodic_departs |= err_per > 1e-3
    assert periodic_departs
