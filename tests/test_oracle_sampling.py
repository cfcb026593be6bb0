"""Pins of the oracle's scan-grid sampling operator S (data recorded at every
sx-th column and sy-th row of the sensor grid) and of S A / A^T S^T."""
import numpy as np

from oracle import hlib, operators as ops
from oracle.geometry import paper_like
from paper_2603_28150_amd import inputs


def test_sampling_operator_identities():
    d = inputs.gaussian_random((5, 12, 16), seed=950)
    for sx, sy in [(1, 1), (2, 1), (1, 3), (4, 2)]:
        ds = ops.sample(d, sx, sy)
        assert ds.shape == (5, 12 // sy, 16 // sx)
        assert np.array_equal(ops.sample(ops.sample_adjoint(ds, sx, sy, 12, 16), sx, sy), ds)   # S S^T = I
        m = ops.sample_adjoint(ops.sample(d, sx, sy), sx, sy, 12, 16)                          # S^T S: a mask
        assert np.array_equal(ops.sample_adjoint(ops.sample(m, sx, sy), sx, sy, 12, 16), m)
        e = inputs.gaussian_random(ds.shape, seed=951)
        assert abs(np.vdot(ops.sample(d, sx, sy), e) - np.vdot(d, ops.sample_adjoint(e, sx, sy, 12, 16))) < 1e-12
    # the samples are the grid points i = sx*i', j = sy*j'
    assert ops.sample(d, 4, 3)[2, 1, 3] == d[2, 3, 12]


def test_sampled_operator_dense_transpose():
    g = paper_like(8, 4, 2, 6)
    H = hlib.H_half(g)
    sx, sy = 2, 2
    A = lambda v: ops.sample(ops.A_fft(H, v), sx, sy)
    AT = lambda v: ops.AT_fft(H, ops.sample_adjoint(v, sx, sy, g.ny, g.nx))
    n_in, shp_out = g.nz * g.ny * g.nx, (g.nt, g.ny // sy, g.nx // sx)
    M = np.stack([A(np.eye(n_in)[c].reshape(g.nz, g.ny, g.nx)).ravel() for c in range(n_in)], axis=1)
    MT = np.stack([AT(np.eye(int(np.prod(shp_out)))[c].reshape(shp_out)).ravel()
                   for c in range(int(np.prod(shp_out)))], axis=1)
    assert np.abs(MT - M.T).max() <= 1e-13 * np.abs(M).max()
