"""GPU parity of periodic grids whose transverse lengths are not fast FFT
sizes (the paper's 202 and 326 among them): those axes run chirp-z
transforms (a circular convolution of power-of-two length M >= 2N - 1 done
with M-point FFTs).  Library, A, A^T, the adjoint identity, the stage call
pat_spectrum against numpy's DFT, batches and FISTA, all against the float64
oracle, which transforms any length directly."""
import numpy as np
import pytest
import torch

from oracle import hlib, operators as ops, quant, solvers
from oracle.geometry import Geometry as OGeom
from paper_2603_28150_amd import inputs
from paper_2603_28150_amd.op import Geometry, Operator

pytestmark = pytest.mark.gpu

CASES = {
    "202x202": Geometry.paper_like(202, 202, 3, 12),                        # M = 512 both axes
    "326x16": Geometry(326, 16, 3, 11, 1e-4, 1.2e-4, 1e-4, 2e-8, 1500.0),   # chirp x (M = 1024), fast y
    "16x326": Geometry(16, 326, 3, 11, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),     # fast x, chirp y
    "18x50": Geometry(18, 50, 5, 19, 1e-4, 1.1e-4, 1e-4, 2e-8, 1500.0),     # M = 64 and 128
    "510x24": Geometry(510, 24, 2, 9, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),      # longest chirp-z axis
    "202x96": Geometry(202, 96, 4, 15, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),     # chirp x, radix-3 y
}


def og(g: Geometry) -> OGeom:
    return OGeom(g.nx, g.ny, g.nz, g.nt, g.dx, g.dy, g.dz, g.dt, g.c, g.nz_sim)


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


_cache = {}


def setup(name, h_dtype="f32"):
    key = (name, h_dtype)
    if key not in _cache:
        g = CASES[name]
        _cache[key] = (g, Operator(g, h_dtype), hlib.H_half(og(g)))
    return _cache[key]


@pytest.mark.parametrize("name", list(CASES))
def test_chirp_z_operator_matches_oracle(name):
    g, op, Hh = setup(name)
    assert op.nk == g.ny * (g.nx // 2 + 1)
    Hg = host(op.export_H())
    Ho = Hh.reshape(op.nk, g.nz, g.nt)
    assert np.abs(Hg - Ho).max() <= 1e-7 * np.abs(Ho).max()
    x = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=1201)
    y = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=1202)
    assert rel(host(op.apply_A(dev(x))), ops.A_fft(Hh, x)) < 1e-5
    assert rel(host(op.apply_AT(dev(y))), ops.AT_fft(Hh, y)) < 1e-5
    assert op.adjoint_check(dev(x), dev(y)) < 1e-5


@pytest.mark.parametrize("name", ["202x202", "326x16", "18x50"])
def test_chirp_z_spectrum_stage_is_the_dft(name):
    # pat_spectrum of S slices: row r of the spectrum array holds frequency
    # k_of_row[r] = p * (nx/2 + 1) + m of every slice (numpy's rfft2 in float64)
    g, op, _ = setup(name)
    S = 5
    f = inputs.gaussian_random((S, g.ny, g.nx), seed=1210)
    spec = op.spectrum_buffer(S).zero_()       # padding entries are never written
    op.spectrum(dev(f), S, spec)
    got = host(spec)
    ref = np.fft.rfft2(f, axes=(1, 2)).reshape(S, -1)        # [S, nk], k = p*nh + m
    rows = np.array(op.spectrum_rows())
    live = rows >= 0
    G = got[live][:, :S, 0] + 1j * got[live][:, :S, 1]       # [rows, S]
    R = ref[:, rows[live]].T
    assert np.abs(G - R).max() <= 1e-5 * np.abs(R).max()
    # and back: the inverse stage call returns the slices
    back = torch.empty((S, g.ny, g.nx), device="cuda")
    op.inverse_spectrum(spec, S, back)
    assert rel(host(back), f) < 1e-5


def test_chirp_z_batches_and_16bit_library():
    g, op, Hh = setup("202x96")
    xs = np.stack([inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=1220 + b) for b in range(3)])
    ys = host(op.apply_A(dev(xs)))                               # matrix cores
    for b in range(3):
        assert rel(ys[b], ops.A_fft(Hh, xs[b])) < 1e-5
        assert rel(ys[b], host(op.apply_A(dev(xs[b])))) < 1e-5
    for kind in ("bf16", "f16"):
        ob = Operator(g, kind)
        Hq, _ = quant.quantise(Hh, kind)
        yb = host(ob.apply_A(dev(xs)))                           # 16-bit tiles, matrix cores
        for b in range(3):
            assert rel(yb[b], ops.A_fft(Hq, xs[b])) < 2e-5, (kind, b)
            assert rel(yb[b], ops.A_fft(Hh, xs[b])) < 5e-3, (kind, b)
        assert rel(host(ob.apply_A(dev(xs[0]))), ops.A_fft(Hq, xs[0])) < 2e-5


def test_chirp_z_fista_matches_oracle():
    g, op, Hh = setup("18x50")
    A = lambda v: ops.A_fft(Hh, v)
    AT = lambda v: ops.AT_fft(Hh, v)
    clean = A(inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=1230))
    d = clean + 0.01 * np.sqrt(np.mean(clean ** 2)) * inputs.noise_like(clean.shape, seed=1231)
    tau = float(np.float32(0.9 / solvers.norm_exact(Hh)))
    xs = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), 8, tau, 1e-3, nonneg=True)
    for k in (1, 8):
        assert rel(host(op.recon_fista(dev(d), k, tau, 1e-3, nonneg=True)), xs[k - 1]) < 1e-5, k


@pytest.mark.parametrize("n", [20, 22, 26, 34, 62, 66, 98, 130, 254, 258, 386, 414, 506])
def test_chirp_z_lengths_sweep(n):
    # every convolution length (64 ... 1024) along x and along y, on thin
    # grids: A against the oracle and the adjoint identity
    for g in (Geometry(n, 16, 2, 5, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),
              Geometry(16, n, 2, 5, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0)):
        op = Operator(g)
        Hh = hlib.H_half(og(g))
        x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=1240 + n)
        y = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=1241 + n)
        assert rel(host(op.apply_A(dev(x))), ops.A_fft(Hh, x)) < 1e-5, (g.nx, g.ny)
        assert rel(host(op.apply_AT(dev(y))), ops.AT_fft(Hh, y)) < 1e-5, (g.nx, g.ny)
        assert op.adjoint_check(dev(x), dev(y)) < 1e-5
