"""Pins of the oracle's sensor response folded into the library along t:
identity and delay taps, folding equals filtering the data of A (and the
correlation on the data side for A^T), on both transverse boundaries."""
import numpy as np

from oracle import hlib, operators as ops
from oracle.geometry import doubled, paper_like
from paper_2603_28150_amd import inputs


def test_identity_and_delay_taps():
    g = paper_like(8, 8, 4, 16)
    H = hlib.H_half(g)
    assert np.array_equal(hlib.with_sensor_response(H, [1.0]), H)
    Hd = hlib.with_sensor_response(H, [0.0, 0.0, 1.0])
    assert np.array_equal(Hd[..., 2:], H[..., :-2])
    assert not Hd[..., :2].any()


def test_folding_equals_filtering_the_data():
    g = paper_like(16, 8, 5, 40)
    H = hlib.H_half(g)
    r = inputs.gaussian_random((9,), seed=901)
    Hr = hlib.with_sensor_response(H, r)
    x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=902)
    d = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=903)
    y = ops.A_fft(Hr, x)
    assert np.abs(y - ops.filter_t(ops.A_fft(H, x), r)).max() <= 1e-12 * np.abs(y).max()
    gr = ops.AT_fft(Hr, d)
    assert np.abs(gr - ops.AT_fft(H, ops.filter_t_adjoint(d, r))).max() <= 1e-12 * np.abs(gr).max()
    # filter_t_adjoint is the adjoint of filter_t
    lhs = np.vdot(ops.filter_t(d, r), d[::-1])
    rhs = np.vdot(d, ops.filter_t_adjoint(d[::-1], r))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(d) ** 2 * np.abs(r).sum()


def test_folding_on_the_linear_boundary_and_bandpass_taps():
    g = paper_like(8, 8, 4, 48)
    H2 = hlib.H_half(doubled(g))
    r = inputs.bandpass_fir(17, 1e6, 25e6, g.dt)
    x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=904)
    y = ops.A_linear(hlib.with_sensor_response(H2, r), x)
    assert np.abs(y - ops.filter_t(ops.A_linear(H2, x), r)).max() <= 1e-12 * np.abs(y).max()
    # a long enough design passes the band centre with unit gain and blocks DC
    r63 = inputs.bandpass_fir(63, 5e6, 20e6, g.dt)
    gain = lambda f: abs(np.sum(r63 * np.exp(-2j * np.pi * f * g.dt * np.arange(63))))
    assert abs(gain(12.5e6) - 1.0) < 1e-12
    assert gain(0.0) < 0.01 and gain(24e6) < 0.01 and abs(gain(5e6) - 0.5) < 0.01
