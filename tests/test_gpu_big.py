"""GPU parity at the full 256^2 x 128 x 512 operator (the benchmark workload),
checked where the oracle can afford it: the kernel library and the output
spectra at sampled transverse frequencies (direct DFT sums, float64), plus
the adjoint identity with float64 dot products on the GPU."""
import numpy as np
import pytest
import torch

from oracle import hlib, operators as ops
from oracle.geometry import Geometry as OGeom
from paper_2603_28150_amd import inputs
from paper_2603_28150_amd.op import Geometry, Operator

pytestmark = pytest.mark.gpu

BIG = Geometry.paper_like(256, 256, 128, 512)
# (m, p): DC, axes, Nyquist corners, a class with four members and random ones
M = np.array([0, 128, 0, 128, 3, 7, 100, 41, 129 - 1, 17])
P = np.array([0, 0, 128, 128, 250, 3, 9, 200, 77, 17])


@pytest.fixture(scope="module")
def big():
    op = Operator(BIG)
    o = OGeom(BIG.nx, BIG.ny, BIG.nz, BIG.nt, BIG.dx, BIG.dy, BIG.dz, BIG.dt, BIG.c)
    Hk = hlib.H_hat(o, M, P)
    return op, Hk


def test_big_kernel_library_at_sampled_frequencies(big):
    op, Hk = big
    nh = BIG.nx // 2 + 1
    for i, (m, p) in enumerate(zip(M, P)):
        Hg = op.export_H(int(p * nh + m), 1)[0].cpu().numpy().astype(np.float64)
        assert np.abs(Hg - Hk[i]).max() <= 1e-7 * np.abs(Hk[i]).max()


def test_big_forward_and_adjoint_spectra(big):
    op, Hk = big
    x = inputs.gaussian_random((BIG.nz, BIG.ny, BIG.nx), seed=90)
    y = op.apply_A(torch.from_numpy(x.astype(np.float32)).cuda())
    Dg = ops.dft_at(y.cpu().numpy().astype(np.float64), M, P)       # [K, nt]
    Do = ops.A_at_freqs(Hk, x, M, P)
    scale = np.linalg.norm(Do) / np.sqrt(len(M))
    for i in range(len(M)):
        assert np.linalg.norm(Dg[i] - Do[i]) < 1e-5 * scale, (M[i], P[i])
    r = inputs.gaussian_random((BIG.nt, BIG.ny, BIG.nx), seed=91)
    g = op.apply_AT(torch.from_numpy(r.astype(np.float32)).cuda())
    Gg = ops.dft_at(g.cpu().numpy().astype(np.float64), M, P)
    Go = ops.AT_at_freqs(Hk, r, M, P)
    scale = np.linalg.norm(Go) / np.sqrt(len(M))
    for i in range(len(M)):
        assert np.linalg.norm(Gg[i] - Go[i]) < 1e-5 * scale, (M[i], P[i])


def test_big_adjoint_identity(big):
    op, _ = big
    x = torch.from_numpy(inputs.gaussian_random((BIG.nz, BIG.ny, BIG.nx), seed=92).astype(np.float32)).cuda()
    y = torch.from_numpy(inputs.gaussian_random((BIG.nt, BIG.ny, BIG.nx), seed=93).astype(np.float32)).cuda()
    assert op.adjoint_check(x, y) < 1e-5


@pytest.mark.parametrize("kind,B", [("bf16", 4), ("f16", 4), ("bf16", 16)])
def test_big_16bit_library_batch(kind, B):
    # full-size 16-bit library on the matrix cores, batches of 4 and of 16 (the
    # benchmark's launch shape): every object within the 16-bit bound of the
    # exact oracle at sampled frequencies
    op = Operator(BIG, kind)
    o = OGeom(BIG.nx, BIG.ny, BIG.nz, BIG.nt, BIG.dx, BIG.dy, BIG.dz, BIG.dt, BIG.c)
    Hk = hlib.H_hat(o, M, P)
    xs = np.stack([inputs.gaussian_random((BIG.nz, BIG.ny, BIG.nx), seed=94 + b) for b in range(B)])
    ys = op.apply_A(torch.from_numpy(xs.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    for b in (range(B) if B <= 4 else (0, 7, B - 1)):
        Dg = ops.dft_at(ys[b], M, P)
        Do = ops.A_at_freqs(Hk, xs[b], M, P)
        assert np.linalg.norm(Dg - Do) / np.linalg.norm(Do) < 5e-3


def test_big_float32_batch_of_16(big):
    # the batch form of the benchmark (16 objects, float32 library on the
    # matrix cores): sampled objects of the batch against the oracle's
    # spectra at the sampled frequencies, forward and adjoint
    op, Hk = big
    B = 16
    xs = np.stack([inputs.gaussian_random((BIG.nz, BIG.ny, BIG.nx), seed=700 + b) for b in range(B)])
    ys = op.apply_A(torch.from_numpy(xs.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    rs = np.stack([inputs.gaussian_random((BIG.nt, BIG.ny, BIG.nx), seed=800 + b) for b in (0, 5, 15)])
    rb = np.zeros((B, BIG.nt, BIG.ny, BIG.nx), np.float32)
    rb[[0, 5, 15]] = rs
    gs = op.apply_AT(torch.from_numpy(rb).cuda()).cpu().numpy().astype(np.float64)
    for i, b in enumerate((0, 5, 15)):
        Dg = ops.dft_at(ys[b], M, P)
        Do = ops.A_at_freqs(Hk, xs[b], M, P)
        assert np.linalg.norm(Dg - Do) / np.linalg.norm(Do) < 1e-5, b
        Gg = ops.dft_at(gs[b], M, P)
        Go = ops.AT_at_freqs(Hk, rs[i], M, P)
        assert np.linalg.norm(Gg - Go) / np.linalg.norm(Go) < 1e-5, b
    assert np.abs(gs[1]).max() == 0.0                # zero data, zero image


def test_paper_in_vivo_grid_full_size():
    # the in vivo grid of the paper (384 x 326 x 96 at 50 um, 384 samples here)
    # on the linear boundary, 768^2 transforms, as the benchmark runs it: the
    # adjoint identity with float64 dots, and one object of a batch of 2
    # (matrix cores) against the same object alone (VALU kernel)
    g = Geometry.paper_like(384, 326, 96, 384, dx=50e-6, boundary="linear")
    op = Operator(g)
    assert op.nk == 768 * 385
    x = torch.from_numpy(inputs.vascular_phantom(op.x_shape, seed=95).astype(np.float32)).cuda()
    y = torch.from_numpy(inputs.gaussian_random(op.d_shape, seed=96).astype(np.float32)).cuda()
    assert op.adjoint_check(x, y) < 1e-5
    x2 = torch.stack([x, torch.flip(x, dims=(0,))])
    y2 = op.apply_A(x2)
    y1 = op.apply_A(x)
    assert float(torch.linalg.norm(y2[0] - y1) / torch.linalg.norm(y1)) < 1e-5


def test_big_linear_boundary_full_size():
    # the linear-boundary form as the benchmark runs it (256^2 window, 128 x
    # 512, 512^2 transforms): adjoint identity with float64 dots, and an
    # object in a batch of 2 against the same object alone
    g = Geometry.paper_like(256, 256, 128, 512, boundary="linear")
    op = Operator(g)
    x = torch.from_numpy(inputs.vascular_phantom(op.x_shape, seed=97).astype(np.float32)).cuda()
    y = torch.from_numpy(inputs.gaussian_random(op.d_shape, seed=98).astype(np.float32)).cuda()
    assert op.adjoint_check(x, y) < 1e-5
    y2 = op.apply_A(torch.stack([x, x.flip(0)]))
    y1 = op.apply_A(x)
    assert float(torch.linalg.norm(y2[0] - y1) / torch.linalg.norm(y1)) < 1e-5


def test_big_fista_gram_path_equals_explicit_path(big):
    # at the benchmark size the FISTA iterate through the nz x nz Gram blocks
    # (pat_recon_fista) equals the explicit A-then-A^T iteration, step by
    # step (both checked against the oracle at small sizes; here they pin each
    # other where the oracle cannot follow), and the data misfit falls
    op, _ = big
    x0 = torch.from_numpy(inputs.vascular_phantom(op.x_shape, seed=99).astype(np.float32)).cuda()
    d = op.apply_A(x0)
    d = d + 0.05 * float(d.std()) * torch.from_numpy(
        inputs.noise_like(op.d_shape, seed=100).astype(np.float32)).cuda()
    v0 = torch.from_numpy(inputs.gaussian_random(op.x_shape, seed=101).astype(np.float32)).cuda()
    L, _ = op.power_norm(v0, 30)      # a random start: A^T A is block diagonal in k
    tau = 0.9 / L
    K = 4
    xe = torch.zeros((1,) + op.x_shape, device="cuda")
    ze = torch.zeros_like(xe)
    tk = 1.0
    for k in range(K):
        tn = (1.0 + (1.0 + 4.0 * tk * tk) ** 0.5) / 2.0
        op.fista_step(d[None], xe, ze, [(tk - 1.0) / tn], [tau], [0.0], [True])
        tk = tn
    xg, tr = op.recon_fista(d, K, tau, 0.0, nonneg=True, trace=True)
    assert float(torch.linalg.norm(xg - xe[0]) / torch.linalg.norm(xe[0])) < 1e-5
    tr = tr.cpu().numpy()
    assert tr[-1] < 0.8 * tr[0]
