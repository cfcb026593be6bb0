"""GPU parity of the zero-padded linear convolution (Sec. 2.3) and of the
larger transforms it needs (512 and 1024 points, and the 2^a 3^b sizes), through
the C ABI, against the float64 oracle, on power-of-two windows and on the
paper's grid shapes.

The linear operator pads the object into the periodic grid of the smallest
transform size holding twice the window, applies the operator of that grid
and crops the data; the HIP path never stores the
padding (the transforms skip the zero rows and columns on the way in and the
cropped ones on the way out).  Bars as in the periodic parity tests: library
1e-7, A, A^T and FISTA iterates 1e-5 (float32), 2e-5 against the oracle
applying the same 16-bit library."""
import numpy as np
import pytest
import torch

from oracle import hlib, operators as ops, quant, solvers
from oracle.geometry import Geometry as OGeom, linear_grid
from paper_2603_28150_amd import _lib, inputs
from paper_2603_28150_amd.op import Geometry, Operator

pytestmark = pytest.mark.gpu

LINEAR = {
    "tiny": Geometry.paper_like(16, 16, 16, 64, boundary="linear"),          # 32^2 transforms
    "ragged": Geometry(32, 16, 13, 37, 1e-4, 1.3e-4, 1e-4, 2e-8, 1500.0, 0, "linear"),  # 64 x 32
    "mid": Geometry.paper_like(64, 64, 40, 130, boundary="linear"),         # 128^2
    "big": Geometry.paper_like(256, 256, 4, 24, boundary="linear"),         # 512^2
    # the paper's grid shapes (wire phantom 202^2, in vivo 384 x 326): rows
    # that are not a multiple of 4 long, 512^2 and 1024^2 transforms
    "wire202": Geometry.paper_like(202, 202, 17, 48, boundary="linear"),       # 432^2
    "invivo384x326": Geometry.paper_like(384, 326, 4, 24, boundary="linear"),   # 768^2
    "w20x40": Geometry.paper_like(20, 40, 6, 30, boundary="linear"),            # 48 x 96
    "w100x30": Geometry.paper_like(100, 30, 5, 24, boundary="linear"),          # 216 x 72
    # smallest windows: a 4-point line of sensors (16 x 16 transforms), 5 x 3
    "line4x1": Geometry(4, 1, 3, 9, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0, 0, "linear"),
    "w5x3": Geometry(5, 3, 2, 7, 1e-4, 1.1e-4, 1e-4, 2e-8, 1500.0, 0, "linear"),
}
PERIODIC_LARGE = {
    "512x16": Geometry(512, 16, 5, 19, 1e-4, 1.2e-4, 1e-4, 2e-8, 1500.0),
    "16x512": Geometry(16, 512, 4, 21, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),
    "512x512": Geometry.paper_like(512, 512, 4, 24),
    "1024x16": Geometry(1024, 16, 3, 17, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),
    "16x1024": Geometry(16, 1024, 3, 17, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),
    # transform sizes 3 * 2^a (radix-3 stages)
    "48x96": Geometry(48, 96, 5, 19, 1e-4, 1.2e-4, 1e-4, 2e-8, 1500.0),
    "192x192": Geometry.paper_like(192, 192, 6, 30),
    "384x16": Geometry(384, 16, 3, 17, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),
    "16x768": Geometry(16, 768, 3, 17, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),
    "768x768": Geometry.paper_like(768, 768, 2, 12),
    # 9 * 2^a and 27 * 2^a (two and three radix-3 stages)
    "72x108": Geometry(72, 108, 5, 19, 1e-4, 1.2e-4, 1e-4, 2e-8, 1500.0),
    "144x216": Geometry.paper_like(144, 216, 4, 20),
    "288x16": Geometry(288, 16, 3, 17, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),
    "432x576": Geometry.paper_like(432, 576, 2, 10),
    "16x864": Geometry(16, 864, 3, 17, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),
    "864x32": Geometry(864, 32, 2, 9, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0),
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


def linear_setup(name, h_dtype="f32"):
    key = (name, h_dtype)
    if key not in _cache:
        g = LINEAR[name]
        _cache[key] = (g, Operator(g, h_dtype), hlib.H_half(linear_grid(og(g))))
    return _cache[key]


@pytest.mark.parametrize("name", list(LINEAR))
def test_linear_library_is_that_of_the_padded_grid(name):
    g, op, Hh2 = linear_setup(name)
    assert op.nk == Hh2.shape[0] * Hh2.shape[1]
    Hg = host(op.export_H())
    Ho = Hh2.reshape(op.nk, g.nz, g.nt)
    assert np.abs(Hg - Ho).max() <= 1e-7 * np.abs(Ho).max()


@pytest.mark.parametrize("name", list(LINEAR))
def test_linear_apply_and_adjoint_match_oracle(name):
    g, op, Hh2 = linear_setup(name)
    x = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=801)
    y = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=802)
    assert rel(host(op.apply_A(dev(x))), ops.A_linear(Hh2, x)) < 1e-5
    assert rel(host(op.apply_AT(dev(y))), ops.AT_linear(Hh2, y)) < 1e-5
    assert op.adjoint_check(dev(x), dev(y)) < 1e-5


def test_linear_batch_equals_single_objects():
    g, op, Hh2 = linear_setup("ragged")
    xs = np.stack([inputs.gaussian_random((g.nz, g.ny, g.nx), seed=810 + b) for b in range(3)])
    ys = host(op.apply_A(dev(xs)))
    for b in range(3):
        # a batch runs on the matrix cores (float16 terms, 2^-22 relative)
        assert rel(ys[b], host(op.apply_A(dev(xs[b])))) < 1e-5
        assert rel(ys[b], ops.A_linear(Hh2, xs[b])) < 1e-5


def test_wide_transforms_match_narrow_ones_bit_for_bit():
    # 2,112 slices on the 202 x 202 window (432^2 transforms): the row passes
    # take their workgroups in tiles of 4 rows (202 rows: a partial last
    # tile) and the column passes slice blocks fastest; every slice's spectrum
    # is the one a call on 640 of the slices computes (row-major order),
    # bit for bit, and the inverse returns the slices
    g = LINEAR["wire202"]
    op = Operator(g, "f32")
    S, Sn = 2112, 640
    x = dev(inputs.gaussian_random((S, g.ny, g.nx), seed=821))
    B_ws = -(-S // g.nt)
    wide = op.spectrum_buffer(S)
    op.spectrum(x, S, wide, B_ws=B_ws)
    narrow = op.spectrum_buffer(Sn)
    used = torch.tensor([r for r, k in enumerate(op.spectrum_rows()) if k >= 0], device="cuda")
    for s0 in (0, S - Sn):
        op.spectrum(x[s0:s0 + Sn].contiguous(), Sn, narrow, B_ws=B_ws)
        assert torch.equal(wide[used, s0:s0 + Sn], narrow[used, :Sn]), s0
    back = torch.empty_like(x)
    op.inverse_spectrum(wide, S, back, B_ws=B_ws)
    assert rel(host(back), host(x)) < 1e-6


@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_linear_16bit_library(kind):
    g, op, Hh2 = linear_setup("tiny", kind)
    Hq, _ = quant.quantise(Hh2, kind)
    x = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=820)
    d = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=821)
    assert rel(host(op.apply_A(dev(x))), ops.A_linear(Hq, x)) < 2e-5
    assert rel(host(op.apply_AT(dev(d))), ops.AT_linear(Hq, d)) < 2e-5
    assert rel(host(op.apply_A(dev(x))), ops.A_linear(Hh2, x)) < 5e-3
    xb = np.stack([inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=822 + b) for b in range(4)])
    yb = host(op.apply_A(dev(xb)))                     # batch: matrix cores
    for b in range(4):
        assert rel(yb[b], ops.A_linear(Hq, xb[b])) < 2e-5


def test_linear_power_iteration_matches_oracle():
    # no Gram blocks here: every power step is A^T (A v) through both transforms
    g, op, Hh2 = linear_setup("ragged")
    v0 = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=832)
    L, trace = op.power_norm(dev(v0), 20)
    Lo = solvers.power_iteration(lambda v: ops.A_linear(Hh2, v), lambda v: ops.AT_linear(Hh2, v), v0, 20)
    assert np.max(np.abs(np.array(trace) - Lo) / np.array(Lo)) < 1e-5
    assert L == trace[-1]


def test_linear_fista_matches_oracle_and_rejects_normal_step():
    g, op, Hh2 = linear_setup("tiny")
    A = lambda v: ops.A_linear(Hh2, v)
    AT = lambda v: ops.AT_linear(Hh2, v)
    x_true = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=830)
    clean = A(x_true)
    d = clean + 0.01 * np.sqrt(np.mean(clean ** 2)) * inputs.noise_like(clean.shape, seed=831)
    tau = float(np.float32(0.9 / solvers.norm_exact(Hh2)))   # ||A_lin|| <= ||A_padded||
    K = 12
    xs = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), K, tau, 1e-3, nonneg=True)
    for k in (1, 4, K):
        assert rel(host(op.recon_fista(dev(d), k, tau, 1e-3, nonneg=True)), xs[k - 1]) < 1e-5, k
    _, tr = op.recon_fista(dev(d), K, tau, 1e-3, nonneg=True, trace=True)
    betas = solvers.momentum_weights(K)
    zs = [np.zeros_like(xs[0])]
    for k in range(1, K):
        zs.append(xs[k - 1] + betas[k - 1] * (xs[k - 1] - (xs[k - 2] if k >= 2 else 0.0)))
    fo = np.array([0.5 * np.sum((A(z_) - d) ** 2) for z_ in zs])
    assert np.max(np.abs(host(tr) - fo) / fo) < 1e-5
    x = torch.zeros((1,) + op.x_shape, device="cuda")
    with pytest.raises(_lib.PatError):
        op.fista_step_normal(x, x, torch.zeros_like(x), [0.0], [tau], [0.0], [True])


@pytest.mark.parametrize("name", list(PERIODIC_LARGE))
def test_periodic_large_and_radix3_transforms(name):
    g = PERIODIC_LARGE[name]
    op = Operator(g)
    Hh = hlib.H_half(og(g))
    x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=840)
    y = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=841)
    assert rel(host(op.apply_A(dev(x))), ops.A_fft(Hh, x)) < 1e-5
    assert rel(host(op.apply_AT(dev(y))), ops.AT_fft(Hh, y)) < 1e-5
    assert op.adjoint_check(dev(x), dev(y)) < 1e-5
