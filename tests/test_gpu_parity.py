"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (relative l2 unless stated): kernel library 1e-7 (float32 storage),
A, A^T and every FISTA iterate 1e-5 (float32 arithmetic), 16-bit library
5e-3 against the exact oracle and 2e-5 against the oracle applying the same
quantised library.  The adjoint check uses float64 dot products on the GPU.
"""
import numpy as np
import pytest
import torch

from oracle import hlib, operators as ops, quant, solvers
from oracle.geometry import Geometry as OGeom
from paper_2603_28150_amd import _lib, inputs
from paper_2603_28150_amd.op import Geometry, Operator

pytestmark = pytest.mark.gpu

TINY = Geometry.paper_like(32, 32, 16, 64)                       # radial fold
RAGGED = Geometry(32, 16, 13, 37, 1e-4, 1.3e-4, 1e-4, 2e-8, 1500.0)  # quadrant fold, ragged
MID = Geometry.paper_like(64, 64, 40, 130)                       # several tiles per row
GEOMS = {"tiny": TINY, "ragged": RAGGED, "mid": MID}
# depth and time axes that are multiples of 32: both products of the batched
# float32 path take the branch-free operand loads (K a multiple of 16, N of 32)
EXTRA = {"square": Geometry.paper_like(32, 32, 32, 64),
         # A^T's k axis (time) over three chunks of 128, the last partial
         "long": Geometry.paper_like(32, 32, 32, 320)}


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
        g = GEOMS[name] if name in GEOMS else EXTRA[name]
        Hh = hlib.H_half(og(g))
        _cache[key] = (g, Operator(g, h_dtype), Hh)
    return _cache[key]


@pytest.mark.parametrize("name", list(GEOMS))
def test_kernel_library_matches_oracle(name):
    g, op, Hh = setup(name)
    Hg = host(op.export_H())
    Ho = Hh.reshape(op.nk, g.nz, g.nt)
    assert np.abs(Hg - Ho).max() <= 1e-7 * np.abs(Ho).max()
    assert rel(Hg, Ho) < 1e-7


@pytest.mark.parametrize("name", list(GEOMS))
def test_forward_matches_oracle(name):
    g, op, Hh = setup(name)
    x = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=21)
    y = host(op.apply_A(dev(x)))
    assert rel(y, ops.A_fft(Hh, x)) < 1e-5
    xr = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=22)
    assert rel(host(op.apply_A(dev(xr))), ops.A_fft(Hh, xr)) < 1e-5


@pytest.mark.parametrize("name", list(GEOMS))
def test_adjoint_matches_oracle(name):
    g, op, Hh = setup(name)
    y = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=23)
    assert rel(host(op.apply_AT(dev(y))), ops.AT_fft(Hh, y)) < 1e-5


@pytest.mark.parametrize("name", list(GEOMS))
def test_adjoint_identity_on_gpu(name):
    g, op, Hh = setup(name)
    x = dev(inputs.gaussian_random((g.nz, g.ny, g.nx), seed=24))
    y = dev(inputs.gaussian_random((g.nt, g.ny, g.nx), seed=25))
    assert op.adjoint_check(x, y) < 1e-5


def test_direct_sum_form_on_tiny_grid():
    # the GPU agrees with eq. 7 written as circular convolution sums too
    g = Geometry.paper_like(16, 16, 6, 20)
    op = Operator(g)
    o = og(g)
    h = hlib.h_space(o)
    x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=26)
    assert rel(host(op.apply_A(dev(x))), ops.A_direct(h, x)) < 1e-5
    y = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=27)
    assert rel(host(op.apply_AT(dev(y))), ops.AT_direct(h, y)) < 1e-5


def test_batch_matches_single_and_is_repeatable():
    g, op, Hh = setup("ragged")
    xs = np.stack([inputs.gaussian_random((g.nz, g.ny, g.nx), seed=30 + b) for b in range(3)])
    yb = op.apply_A(dev(xs))
    yb2 = op.apply_A(dev(xs))
    assert torch.equal(yb, yb2)                      # same stream, same bits: no races
    for b in range(3):
        assert rel(host(yb[b]), ops.A_fft(Hh, xs[b])) < 1e-5
        # a batch runs on the matrix cores (float16 terms, 2^-22 relative)
        assert rel(host(yb[b]), host(op.apply_A(dev(xs[b])))) < 1e-5
    ds = np.stack([inputs.gaussian_random((g.nt, g.ny, g.nx), seed=40 + b) for b in range(3)])
    gb = op.apply_AT(dev(ds))
    for b in range(3):
        assert rel(host(gb[b]), ops.AT_fft(Hh, ds[b])) < 1e-5


@pytest.mark.parametrize("shape", [(16, 16, 1, 1), (16, 16, 1, 7), (16, 32, 3, 1), (256, 16, 2, 3)])
def test_degenerate_sizes(shape):
    nx, ny, nz, nt = shape
    g = Geometry(nx, ny, nz, nt, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0)
    op = Operator(g)
    Hh = hlib.H_half(og(g))
    x = inputs.gaussian_random((nz, ny, nx), seed=50)
    y = host(op.apply_A(dev(x)))
    assert rel(y, ops.A_fft(Hh, x)) < 1e-5
    # t = 0 sees only the sensor-plane slice
    assert np.abs(y[0] - x[0]).max() < 1e-5 * np.abs(x).max()
    d = inputs.gaussian_random((nt, ny, nx), seed=51)
    assert rel(host(op.apply_AT(dev(d))), ops.AT_fft(Hh, d)) < 1e-5


def test_invalid_arguments_raise():
    g, op, Hh = setup("tiny")
    x = dev(np.zeros((g.nz, g.ny, g.nx)))
    y = torch.empty((g.nt, g.ny, g.nx), device="cuda")
    ws = op.workspace(1)
    L = _lib.load()
    assert L.pat_apply_A(op.handle, x.data_ptr(), y.data_ptr(), 0, ws.data_ptr(), ws.numel(), None) == -1
    assert L.pat_apply_A(op.handle, x.data_ptr(), y.data_ptr(), 1, ws.data_ptr(), 16, None) == -1
    assert L.pat_apply_A(op.handle, x.data_ptr() + 4, y.data_ptr(), 1, ws.data_ptr(), ws.numel(), None) == -1
    # batches whose spectrum rows would exceed 2^30 slices are refused on the host
    import ctypes
    n = ctypes.c_size_t()
    assert L.pat_workspace_bytes(op.handle, 1 << 24, ctypes.byref(n)) == 0
    assert L.pat_workspace_bytes(op.handle, 1 << 25, ctypes.byref(n)) == -1
    assert L.pat_contract(op.handle, 0, x.data_ptr(), y.data_ptr(), 1 << 25, None) == -1
    with pytest.raises(_lib.PatError):
        Operator(Geometry(41, 32, 4, 4, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0))


def test_power_iteration_matches_oracle():
    g, op, Hh = setup("tiny")
    v0 = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=1002)
    L, trace = op.power_norm(dev(v0), 30)
    Lo = solvers.power_iteration(lambda v: ops.A_fft(Hh, v), lambda v: ops.AT_fft(Hh, v), v0, 30)
    assert np.max(np.abs(np.array(trace) - Lo) / np.array(Lo)) < 1e-5
    assert L == trace[-1]
    assert L <= solvers.norm_exact(Hh) * (1 + 1e-5)


def _problem(name, seed_obj=0, seed_noise=1, nu=inputs.NOISE_1PCT):
    g, op, Hh = setup(name)
    p0 = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=seed_obj)
    clean = ops.A_fft(Hh, p0)
    d = clean + nu * np.sqrt(np.mean(clean ** 2)) * inputs.noise_like(clean.shape, seed=seed_noise)
    return g, op, Hh, d


def test_fista_every_iterate_matches_oracle():
    # the tiny workload: 4 blobs, 1 % noise, 20 iterations with non-negativity
    g, op, Hh, d = _problem("tiny")
    A = lambda v: ops.A_fft(Hh, v)
    AT = lambda v: ops.AT_fft(Hh, v)
    tau = 1.0 / solvers.power_iteration(A, AT, inputs.gaussian_random((g.nz, g.ny, g.nx), seed=1002), 30)[-1]
    tau = float(np.float32(tau))
    K = 20
    xs = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), K, tau, 0.0, nonneg=True)
    # GPU trajectory one step at a time through the batched step entry point
    dd = dev(d)[None]
    x = torch.zeros((1, g.nz, g.ny, g.nx), device="cuda")
    z = torch.zeros_like(x)
    betas = solvers.momentum_weights(K)
    for k in range(K):
        op.fista_step(dd, x, z, [betas[k]], [tau], [0.0], [True])
        assert rel(host(x[0]), xs[k]) < 1e-5, k
        assert host(x[0]).min() >= 0.0
    # the whole-loop entry point (gradient through the Gram blocks of the
    # library, per frequency) lands on the same iterates
    for k in (1, 2, 5, K):
        assert rel(host(op.recon_fista(dev(d), k, tau, 0.0, nonneg=True)), xs[k - 1]) < 1e-5, k
    xf, tr = op.recon_fista(dev(d), K, tau, 0.0, nonneg=True, momentum=True, trace=True)
    # trace: 1/2 ||A z_k - d||^2 at the gradient point of step k
    zs = [np.zeros_like(xs[0])]
    for k in range(1, K):
        zs.append(xs[k - 1] + betas[k - 1] * (xs[k - 1] - (xs[k - 2] if k >= 2 else 0.0)))
    fo = np.array([0.5 * np.sum((A(z_) - d) ** 2) for z_ in zs])
    # the trace comes from the Gram identity 1/2(<z, g> - <z, A^T d> + ||d||^2)
    # without forming A z; its error scales with the starting objective
    # 1/2 ||d||^2 = fo[0], not with the current one
    assert np.max(np.abs(host(tr) - fo)) < 1e-5 * fo[0]


def test_fista_teacher_forced_step():
    # one oracle step from the GPU's own state lands on the GPU's next iterate
    g, op, Hh, d = _problem("ragged", nu=inputs.NOISE_20DB)
    A = lambda v: ops.A_fft(Hh, v)
    AT = lambda v: ops.AT_fft(Hh, v)
    tau = float(np.float32(0.9 / solvers.norm_exact(Hh)))
    dd = dev(d)[None]
    x = torch.zeros((1, g.nz, g.ny, g.nx), device="cuda")
    z = torch.zeros_like(x)
    betas = solvers.momentum_weights(12)
    for k in range(12):
        xp, zp = host(x[0]), host(z[0])
        op.fista_step(dd, x, z, [betas[k]], [tau], [1e-3], [True])
        xo = solvers.fista(A, AT, d, xp.shape, 1, tau, 1e-3, nonneg=True, z0=zp, x_prev0=xp, k0=k)[0]
        assert rel(host(x[0]), xo) < 1e-5, k


def test_projected_gradient_soft_threshold():
    g, op, Hh, d = _problem("mid", seed_obj=5, seed_noise=6)
    A = lambda v: ops.A_fft(Hh, v)
    AT = lambda v: ops.AT_fft(Hh, v)
    tau = float(np.float32(1.0 / solvers.norm_exact(Hh)))
    xs = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), 8, tau, 0.01, nonneg=False, momentum=False)
    xg = op.recon_fista(dev(d), 8, tau, 0.01, nonneg=False, momentum=False)
    assert rel(host(xg), xs[-1]) < 1e-5


def test_batched_fista_step_isolates_objects():
    # three problems with different tau/lambda/nonneg in one batched step equal
    # the same problems stepped alone
    g, op, Hh = setup("tiny")
    ds = np.stack([_problem("tiny", seed_obj=60 + b, seed_noise=70 + b)[3] for b in range(3)])
    taus = [0.3, 0.5, 0.7]
    lams = [0.0, 0.01, 0.0]
    nn = [True, False, True]
    xb = torch.zeros((3, g.nz, g.ny, g.nx), device="cuda")
    zb = torch.zeros_like(xb)
    bad = torch.zeros(3, dtype=torch.int32, device="cuda")
    for k in range(4):
        op.fista_step(dev(ds), xb, zb, [0.1 * k] * 3, taus, lams, nn, nonfinite=bad)
    for b in range(3):
        x1 = torch.zeros((1, g.nz, g.ny, g.nx), device="cuda")
        z1 = torch.zeros_like(x1)
        for k in range(4):
            op.fista_step(dev(ds[b])[None], x1, z1, [0.1 * k], [taus[b]], [lams[b]], [nn[b]])
        assert rel(host(xb[b]), host(x1[0])) < 1e-5   # batch on the matrix cores
    assert int(bad.sum()) == 0


@pytest.mark.parametrize("name", ["tiny", "ragged"])  # update fused into the last transform pass (16
def test_nonfinite_iterates_flag_only_their_object(name):  # depths) and separate (13)
    # a step of 3e38 for object 1 overflows its iterate to +-inf wherever its
    # gradient is not tiny (the threshold tau * lambda stays 0); the flag is
    # raised for it alone and the other objects step as they do alone
    # (explicit and normal step)
    g, op, Hh = setup(name)
    B = 3
    ds = np.stack([inputs.gaussian_random((g.nt, g.ny, g.nx), seed=80 + b) for b in range(B)])
    tau = float(np.float32(0.5 / solvers.norm_exact(Hh)))
    taus = [tau, float(np.float32(3e38)), tau]
    atd = op.apply_AT(dev(ds))
    for normal in (False, True):
        x = torch.zeros((B, g.nz, g.ny, g.nx), device="cuda")
        z = dev(np.stack([inputs.gaussian_random((g.nz, g.ny, g.nx), seed=90 + b) for b in range(B)]))
        bad = torch.zeros(B, dtype=torch.int32, device="cuda")
        if normal:
            op.fista_step_normal(atd, x, z, [0.5] * B, taus, [0.0] * B, [False] * B, nonfinite=bad)
        else:
            op.fista_step(dev(ds), x, z, [0.5] * B, taus, [0.0] * B, [False] * B, nonfinite=bad)
        assert bad.tolist() == [0, 1, 0], normal
        for b in (0, 2):
            x1 = torch.zeros((1, g.nz, g.ny, g.nx), device="cuda")
            z1 = dev(inputs.gaussian_random((g.nz, g.ny, g.nx), seed=90 + b))[None]
            if normal:
                op.fista_step_normal(atd[b:b + 1].contiguous(), x1, z1, [0.5], [tau], [0.0], [False])
            else:
                op.fista_step(dev(ds[b])[None], x1, z1, [0.5], [tau], [0.0], [False])
            assert torch.isfinite(x[b]).all()
            assert rel(host(x[b]), host(x1[0])) < 1e-5, (normal, b)


@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_quantised_library(kind):
    g = TINY
    op = Operator(g, kind)
    Hh = setup("tiny")[2]
    Hq, s = quant.quantise(Hh, kind)
    Hg = host(op.export_H()).reshape(Hh.shape)
    # identical up to rare last-place differences of the 16-bit format
    ulp = 2.0 ** -8 if kind == "bf16" else 2.0 ** -11
    diff = np.abs(Hg - Hq)
    # entries whose exact value is 0 (e.g. t = 0 off the sensor plane) hold
    # float64 rounding noise on both sides: compare those absolutely
    top = np.abs(Hq).max()
    big = np.abs(Hq) > 1e-12 * top
    assert np.all(diff[~big] <= 1e-12 * top)
    assert np.mean(diff[big] > 0) < 1e-3
    assert np.all(diff[big] <= ulp * np.abs(Hq[big]) * 1.01)
    x = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=80)
    y = host(op.apply_A(dev(x)))
    assert rel(y, ops.A_fft(Hq, x)) < 2e-5
    assert rel(y, ops.A_fft(Hh, x)) < 5e-3
    d = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=81)
    gq = host(op.apply_AT(dev(d)))
    assert rel(gq, ops.AT_fft(Hq, d)) < 2e-5
    assert rel(gq, ops.AT_fft(Hh, d)) < 5e-3
    assert op.adjoint_check(dev(x), dev(d)) < 1e-5


@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_quantised_long_rows(kind):
    # 1,100 samples: A's 16-bit rows of 138 16-byte chunks are split over two
    # workgroups per item (the single-object path); against the oracle
    # applying the same quantised library
    g = Geometry(16, 16, 8, 1100, 1e-4, 1e-4, 1e-4, 2e-8, 1500.0)
    op = Operator(g, kind)
    Hq, _ = quant.quantise(hlib.H_half(og(g)), kind)
    x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=85)
    d = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=86)
    assert rel(host(op.apply_A(dev(x))), ops.A_fft(Hq, x)) < 2e-5
    assert rel(host(op.apply_AT(dev(d))), ops.AT_fft(Hq, d)) < 2e-5
    assert op.adjoint_check(dev(x), dev(d)) < 1e-5


@pytest.mark.parametrize("name", ["tiny", "ragged"])
def test_stage_calls_compose_apply_and_row_map(name):
    g, op, Hh = setup(name)
    x = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=95)
    xd = dev(x)
    Xs = op.spectrum_buffer(g.nz)
    op.spectrum(xd, g.nz, Xs)
    rows = op.spectrum_rows()
    assert sorted(k for k in rows if k >= 0) == list(range(op.nk))
    ref = np.fft.rfft2(x, axes=(1, 2))              # [nz, ny, nx/2+1]
    nh = g.nx // 2 + 1
    Xh = Xs.cpu().numpy().astype(np.float64)
    for r, k in enumerate(rows):
        if k < 0:
            continue
        p, m = divmod(k, nh)
        got = Xh[r, :g.nz, 0] + 1j * Xh[r, :g.nz, 1]
        assert np.abs(got - ref[:, p, m]).max() <= 1e-5 * np.abs(ref).max()
    Ds = op.spectrum_buffer(g.nt)
    op.contract(Xs, Ds, adjoint=False)
    y = torch.empty(op.d_shape, device="cuda")
    op.inverse_spectrum(Ds, g.nt, y)
    assert torch.equal(y, op.apply_A(xd))


@pytest.mark.parametrize("kind", ["bf16", "f16"])
@pytest.mark.parametrize("name,B", [("tiny", 16), ("ragged", 3), ("mid", 2), ("tiny", 19)])
def test_quantised_batched_matrix_core_path(kind, name, B):
    # 16-bit libraries run batches on the matrix cores; every object of a
    # batch must match the oracle applying the same quantised library (2e-5)
    # and the exact oracle (5e-3), and agree with its own single-object apply
    # (the VALU kernel on float32 spectra) to the hi + lo bf16 split of the
    # spectra that the matrix-core path makes: 2^-17 relative per element
    g = GEOMS[name]
    op = Operator(g, kind)
    Hh = setup(name)[2]
    Hq, _ = quant.quantise(Hh, kind)
    xs = np.stack([inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=300 + b) for b in range(B)])
    ys = host(op.apply_A(dev(xs)))
    ds = np.stack([inputs.gaussian_random((g.nt, g.ny, g.nx), seed=400 + b) for b in range(B)])
    gs = host(op.apply_AT(dev(ds)))
    for b in range(B):
        assert rel(ys[b], ops.A_fft(Hq, xs[b])) < 2e-5, b
        assert rel(ys[b], ops.A_fft(Hh, xs[b])) < 5e-3, b
        assert rel(gs[b], ops.AT_fft(Hq, ds[b])) < 2e-5, b
        assert rel(gs[b], ops.AT_fft(Hh, ds[b])) < 5e-3, b
    for b in (0, B - 1):
        assert rel(ys[b], host(op.apply_A(dev(xs[b])))) < 1e-5
        assert rel(gs[b], host(op.apply_AT(dev(ds[b])))) < 1e-5
    assert op.adjoint_check(dev(xs[0]), dev(ds[0])) < 1e-5


@pytest.mark.parametrize("name,B", [("tiny", 16), ("ragged", 4), ("mid", 5), ("ragged", 2), ("tiny", 9), ("mid", 11),
                                    ("tiny", 5), ("square", 3), ("square", 8), ("square", 13)])
def test_float32_batched_path(name, B):
    # float32 batches run on the matrix cores (library rows and spectra each
    # split into two float16 terms under power-of-two scales): every object
    # matches the oracle to the
    # float32 bar, and its own single-object apply (the VALU kernel) to 1e-5;
    # the ragged shapes (13 and 37 along k) end in a partial k-step, the mid
    # one spans two k-chunks for A^T; 9, 11 and 13 objects (72, 88 and 104
    # member-object pairs) need a second, partial column group of 64 pairs,
    # 3 and 5 objects (24 and 40 pairs) one group of 32 pairs; the square
    # shape takes the branch-free operand loads for A and A^T (tiny for A)
    g, op, Hh = setup(name)
    xs = np.stack([inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=500 + b) for b in range(B)])
    ds = np.stack([inputs.gaussian_random((g.nt, g.ny, g.nx), seed=600 + b) for b in range(B)])
    yb = op.apply_A(dev(xs))
    gb = op.apply_AT(dev(ds))
    assert torch.equal(yb, op.apply_A(dev(xs)))      # repeatable bits
    ys, gs = host(yb), host(gb)
    for b in range(B):
        assert rel(ys[b], ops.A_fft(Hh, xs[b])) < 1e-5, b
        assert rel(gs[b], ops.AT_fft(Hh, ds[b])) < 1e-5, b
    for b in (0, B - 1):
        assert rel(ys[b], host(op.apply_A(dev(xs[b])))) < 1e-5
        assert rel(gs[b], host(op.apply_AT(dev(ds[b])))) < 1e-5


@pytest.mark.parametrize("name,B", [("long", 5), ("long", 9), ("mid", 5), ("mid", 9)])
def test_float32_batched_path_scales(name, B):
    # the float16 terms of the batched float32 path carry a power of two per
    # (member, object) pair and per library row: objects 2^-40 to 2^40 in
    # one batch each keep the float32 bar, and data that grow (or shrink)
    # by 2^30 along time, or start with all-zero chunks, make later k-chunks
    # lower a pair's exponent, which rescales its partial sums of A^T;
    # 5 objects take 40-pair column groups, 9 objects 64-pair groups; the long
    # shape takes the branch-free operand loads, the mid one the bounded ones
    g, op, Hh = setup(name)
    e = [(-40, -20, 0, 20, 40)[b % 5] for b in range(B)]
    xs = np.stack([inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=700 + b) * 2.0 ** e[b] for b in range(B)])
    t = np.arange(g.nt, dtype=np.float64) / g.nt
    shapes = [2.0 ** (30 * t), 2.0 ** (-30 * t), (t >= 0.5).astype(np.float64), np.ones_like(t)]
    ds = np.stack([inputs.gaussian_random((g.nt, g.ny, g.nx), seed=800 + b) * shapes[b % 4][:, None, None]
                   * 2.0 ** e[b] for b in range(B)])
    ys, gs = host(op.apply_A(dev(xs))), host(op.apply_AT(dev(ds)))
    for b in range(B):
        assert rel(ys[b], ops.A_fft(Hh, xs[b])) < 1e-5, b
        assert rel(gs[b], ops.AT_fft(Hh, ds[b])) < 1e-5, b
        assert np.isfinite(ys[b]).all() and np.isfinite(gs[b]).all()


@pytest.mark.parametrize("name,kind", [("ragged", "f32"), ("mid", "f32"), ("tiny", "bf16"), ("tiny", "f16")])
def test_gram_fista_matches_oracle(name, kind):
    # FISTA through the per-frequency normal operator on every fold and
    # precision: quadrant (ragged), radial (mid; tiny with 4-member items in 16 bits, against the
    # oracle applying the same quantised library)
    g = GEOMS[name]
    op = Operator(g, kind) if kind != "f32" else setup(name)[1]
    Hh = setup(name)[2]
    if kind != "f32":
        Hh, _ = quant.quantise(Hh, kind)
    p0 = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=600)
    clean = ops.A_fft(Hh, p0)
    d = clean + inputs.NOISE_20DB * np.sqrt(np.mean(clean ** 2)) * inputs.noise_like(clean.shape, seed=601)
    A = lambda v: ops.A_fft(Hh, v)
    AT = lambda v: ops.AT_fft(Hh, v)
    tau = float(np.float32(0.95 / solvers.norm_exact(Hh)))
    xs = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), 15, tau, 2e-3, nonneg=True)
    for k in (3, 15):
        assert rel(host(op.recon_fista(dev(d), k, tau, 2e-3, nonneg=True)), xs[k - 1]) < 1e-5, k


def test_normal_step_matches_explicit_step_and_oracle():
    # batched FISTA steps through the Gram blocks (A^T d given) against the
    # explicit A then A^T step and against the oracle, three objects
    g, op, Hh = setup("mid")
    ds = np.stack([_problem("mid", seed_obj=700 + b, seed_noise=710 + b)[3] for b in range(3)])
    atd = op.apply_AT(dev(ds))
    taus = [float(np.float32(f / solvers.norm_exact(Hh))) for f in (0.5, 0.8, 1.0)]
    lams, nn = [0.0, 1e-3, 0.0], [True, True, False]
    xe = torch.zeros((3, g.nz, g.ny, g.nx), device="cuda")
    ze, xn, zn = torch.zeros_like(xe), torch.zeros_like(xe), torch.zeros_like(xe)
    betas = solvers.momentum_weights(6)
    for k in range(6):
        op.fista_step(dev(ds), xe, ze, [betas[k]] * 3, taus, lams, nn)
        op.fista_step_normal(atd, xn, zn, [betas[k]] * 3, taus, lams, nn)
    A = lambda v: ops.A_fft(Hh, v)
    AT = lambda v: ops.AT_fft(Hh, v)
    for b in range(3):
        xo = solvers.fista(A, AT, ds[b], (g.nz, g.ny, g.nx), 6, taus[b], lams[b], nonneg=nn[b])[-1]
        assert rel(host(xn[b]), xo) < 1e-5, b
        assert rel(host(xn[b]), host(xe[b])) < 1e-5, b


@pytest.mark.parametrize("nz,nt", [(8, 2048), (2048, 8)], ids=["nt2048", "nz2048"])
@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_longest_depth_and_time_axes(nz, nt, kind):
    # the longest axes the library accepts (2048 samples or depths; nz_sim
    # 1024 and 4096 by the default rule), one object and a batch of two
    g = Geometry.paper_like(16, 16, nz, nt)
    op = Operator(g, kind)
    Hh = hlib.H_half(og(g))
    if kind != "f32":
        Hh, _ = quant.quantise(Hh, kind)
    bar = 1e-5 if kind == "f32" else 2e-5
    xs = np.stack([inputs.gaussian_random((nz, 16, 16), seed=900 + b) for b in range(2)])
    ds = np.stack([inputs.gaussian_random((nt, 16, 16), seed=910 + b) for b in range(2)])
    y1 = host(op.apply_A(dev(xs[0])))
    g1 = host(op.apply_AT(dev(ds[0])))
    assert rel(y1, ops.A_fft(Hh, xs[0])) < bar
    assert rel(g1, ops.AT_fft(Hh, ds[0])) < bar
    y2 = host(op.apply_A(dev(xs)))
    g2 = host(op.apply_AT(dev(ds)))
    for b in range(2):
        assert rel(y2[b], ops.A_fft(Hh, xs[b])) < bar, b
        assert rel(g2[b], ops.AT_fft(Hh, ds[b])) < bar, b
