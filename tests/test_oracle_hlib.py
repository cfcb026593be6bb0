"""Pins of the oracle's kernel library H^ (CPU only).

Each test fixes H^ with something other than the oracle's own formula:
an exact identity, a closed form derived by hand, a symmetry of the
physics, or a library routine computing the same sum another way.
"""
import math

import numpy as np
import pytest

from oracle.geometry import Geometry, paper_like
from oracle import hlib

TINY = paper_like(32, 32, 16, 64)          # 32^2 x 16 x 64, nz_sim = 64


def test_default_nz_sim_rule():
    # the wrapped image cannot reach the sensor within the record
    assert TINY.nq == 64
    assert paper_like(256, 256, 128, 512).nq == 512
    assert paper_like(128, 128, 64, 256).nq == 256
    assert paper_like(128, 128, 96, 384).nq == 256
    assert paper_like(16, 16, 16, 32).nq == 32


def test_t0_is_kronecker_delta_in_depth():
    # at t = 0 the field is the initial pressure itself: the sensor plane
    # sees only the absorber placed on it (eq. 2, z_0 = sensor plane)
    H = hlib.H_half(TINY)
    expect = np.zeros(TINY.nz)
    expect[0] = 1.0
    err = np.abs(H[:, :, :, 0] - expect).max()
    assert err < 1e-14


@pytest.mark.parametrize("nq", [64, 63])
def test_kperp_zero_is_dalembert_with_periodic_sinc(nq):
    # closed form for k_perp = 0: the 1D d'Alembert solution on a periodic
    # z-grid of nq points with a band-limited (periodic sinc) pulse
    g = Geometry(nx=8, ny=8, nz=16, nt=64, dx=1e-4, dy=1e-4, dz=1e-4,
                 dt=0.3e-4 / 1500.0, c=1500.0, nz_sim=nq)
    H = hlib.H_hat(g, [0], [0])[0]                      # [nz, nt]

    def D(u):
        if abs(math.sin(math.pi * u / nq)) < 1e-12:
            return 1.0
        if nq % 2 == 0:
            return math.sin(math.pi * u) / math.tan(math.pi * u / nq) / nq
        return math.sin(math.pi * u) / math.sin(math.pi * u / nq) / nq

    expect = np.empty_like(H)
    for l in range(g.nz):
        for n in range(g.nt):
            s = g.c * n * g.dt / g.dz
            expect[l, n] = 0.5 * (D(l - s) + D(l + s))
    assert np.abs(H - expect).max() < 1e-13


def test_real_even_and_radial():
    g = Geometry(nx=16, ny=16, nz=6, nt=24, dx=1e-4, dy=1e-4, dz=1e-4,
                 dt=2e-8, c=1500.0)
    Hf = hlib.H_full(g)                        # raises if Im H^ is not ~0
    # even in m and in p
    Hm = Hf[:, (-np.arange(16)) % 16]
    Hp = Hf[(-np.arange(16)) % 16]
    assert np.abs(Hf - Hm).max() < 1e-14
    assert np.abs(Hf - Hp).max() < 1e-14
    # m <-> p on a square grid with dx = dy
    assert np.abs(Hf - np.transpose(Hf, (1, 0, 2, 3))).max() < 1e-14
    # depends on kx^2 + ky^2 only: (3,4) and (5,0) share |k_perp|
    assert np.abs(Hf[4, 3] - Hf[0, 5]).max() < 1e-13


def test_anisotropic_grid_breaks_only_the_swap():
    g = Geometry(nx=16, ny=8, nz=4, nt=16, dx=1e-4, dy=1.3e-4, dz=1e-4,
                 dt=2e-8, c=1500.0)
    Hf = hlib.H_full(g)
    assert np.abs(Hf - Hf[:, (-np.arange(16)) % 16]).max() < 1e-14
    assert np.abs(Hf - Hf[(-np.arange(8)) % 8]).max() < 1e-14
    assert np.abs(Hf[1, 2] - Hf[2, 1]).max() > 1e-3


def test_depth_sum_matches_numpy_fft():
    # the direct q-sum equals the library FFT over the periodic z-grid
    g = TINY
    m, p = 5, 27
    H = hlib.H_hat(g, [m], [p])[0]
    kx = 2 * np.pi * np.fft.fftfreq(g.nx, g.dx)[m]
    ky = 2 * np.pi * np.fft.fftfreq(g.ny, g.dy)[p]
    kz = 2 * np.pi * np.fft.fftfreq(g.nq, g.dz)
    t = np.arange(g.nt) * g.dt
    cosk = np.cos(g.c * t[:, None] * np.sqrt(kx ** 2 + ky ** 2 + kz[None, :] ** 2))
    F = np.fft.fft(cosk, axis=1) / g.nq                  # [nt, nq]
    assert np.abs(F.imag).max() < 1e-14
    assert np.abs(F.real[:, :g.nz].T - H).max() < 1e-14


def test_space_kernels_are_impulse_responses():
    # h_l is the sensor response to a unit absorber at (0, 0, l): at t = 0 it
    # is the absorber itself when l = 0 and nothing otherwise
    g = paper_like(8, 8, 4, 16)
    h = hlib.h_space(g)
    assert h.shape == (4, 8, 8, 16)
    e = np.zeros((8, 8))
    e[0, 0] = 1.0
    assert np.abs(h[0, :, :, 0] - e).max() < 1e-14
    assert np.abs(h[1:, :, :, 0]).max() < 1e-14


def test_library_by_reciprocity_from_one_point_source_run():
    # one run of the independent k-space stepper from a unit point source on
    # the sensor plane, recorded on every depth plane: by reciprocity (source
    # and receiver depths exchanged in a homogeneous medium) the recorded
    # planes, transformed over (x, y), are the whole library (the library
    # construction discussed in Sec. 3.2)
    from oracle import wave3d
    g = paper_like(8, 12, 5, 24)
    src = np.zeros((g.nz, g.ny, g.nx))
    src[0, 0, 0] = 1.0
    planes = wave3d.simulate(src, g.dx, g.dy, g.dz, g.dt, g.c, g.nt, g.nq, planes=range(g.nz))
    Hrec = np.fft.fft2(planes, axes=(2, 3))                     # [n, l, p, m]
    Hf = hlib.H_full(g)                                         # [p, m, l, n]
    assert np.abs(Hrec.imag).max() < 1e-13
    assert np.abs(np.transpose(Hrec.real, (2, 3, 1, 0)) - Hf).max() < 1e-13 * np.abs(Hf).max()
    # the plane-0 record alone is the d'Alembert/t = 0 structure: the depth-0 kernel
    d0 = wave3d.simulate(src, g.dx, g.dy, g.dz, g.dt, g.c, g.nt, g.nq)
    assert np.array_equal(d0, planes[:, 0])
