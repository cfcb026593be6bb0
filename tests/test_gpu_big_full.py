"""GPU parity at the full 256^2 x 128 x 512 operator against the FP64 oracle
with its whole library on the host (17.3 GB, half spectrum).

* A and A^T element-wise: every output sample, and every one of the 33,024
  half-spectrum frequencies on its own (Sec. 3.2, steps (i)-(iii); eq. 11);
  the same for objects of a batch of 16 on the matrix cores.
* FISTA (Sec. 2.3, eq. 12-15) on the benchmark's problem (vascular phantom,
  20 dB noise, step from 30 power iterations on the GPU): one oracle step from
  the GPU's own state at k = 1, 50 and 100 lands on the GPU's next iterate,
  and the whole-loop entry point equals the stepped iterate after 100 steps.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle_threads
from oracle import operators as ops, solvers
from oracle.geometry import Geometry as OGeom
from paper_2603_28150_amd import inputs
from paper_2603_28150_amd.op import Geometry, Operator

pytestmark = pytest.mark.gpu

BIG = Geometry.paper_like(256, 256, 128, 512)
SHAPE = (BIG.nz, BIG.ny, BIG.nx)
DSHAPE = (BIG.nt, BIG.ny, BIG.nx)


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def big():
    o = OGeom(BIG.nx, BIG.ny, BIG.nz, BIG.nt, BIG.dx, BIG.dy, BIG.dz, BIG.dt, BIG.c)
    Hh = oracle_threads.H_half(o)
    op = Operator(BIG)
    yield op, Hh
    del op, Hh
    torch.cuda.empty_cache()


def per_frequency_ok(yg, yo, bound=1e-5):
    """Every half-spectrum frequency of yg within bound of yo, relative to
    that frequency's own norm or, where it is below the mean, to the mean."""
    Fg = np.fft.rfft2(yg, axes=(1, 2)).reshape(yg.shape[0], -1)
    Fo = np.fft.rfft2(yo, axes=(1, 2)).reshape(yo.shape[0], -1)
    err = np.linalg.norm(Fg - Fo, axis=0)
    ref = np.linalg.norm(Fo, axis=0)
    floor = np.linalg.norm(Fo) / np.sqrt(Fo.shape[1])
    worst = float(np.max(err / np.maximum(ref, floor)))
    return worst < bound, worst


def test_big_A_and_AT_every_frequency(big):
    op, Hh = big
    x = inputs.gaussian_random(SHAPE, seed=1401)
    yg, yo = host(op.apply_A(dev(x))), ops.A_fft(Hh, x)
    assert rel(yg, yo) < 1e-5
    ok, worst = per_frequency_ok(yg, yo)
    assert ok, worst
    r = inputs.gaussian_random(DSHAPE, seed=1402)
    gg, go = host(op.apply_AT(dev(r))), ops.AT_fft(Hh, r)
    assert rel(gg, go) < 1e-5
    ok, worst = per_frequency_ok(gg, go)
    assert ok, worst


def test_big_batch_of_16_every_frequency(big):
    # the batched form (16 objects, float32 library on the matrix cores):
    # the first and last object of the batch, forward and adjoint
    op, Hh = big
    xs = np.stack([inputs.vascular_phantom(SHAPE, seed=2001 + b) for b in (0, 15)])
    xb = torch.zeros((16,) + SHAPE, device="cuda")
    xb[0], xb[15] = dev(xs[0]), dev(xs[1])
    yb = op.apply_A(xb)
    rs = np.stack([inputs.gaussian_random(DSHAPE, seed=1410 + b) for b in (0, 15)])
    rb = torch.zeros((16,) + DSHAPE, device="cuda")
    rb[0], rb[15] = dev(rs[0]), dev(rs[1])
    gb = op.apply_AT(rb)
    for i, b in enumerate((0, 15)):
        yg, yo = host(yb[b]), ops.A_fft(Hh, xs[i])
        assert rel(yg, yo) < 1e-5, b
        assert per_frequency_ok(yg, yo)[0], b
        gg, go = host(gb[b]), ops.AT_fft(Hh, rs[i])
        assert rel(gg, go) < 1e-5, b
        assert per_frequency_ok(gg, go)[0], b
    assert float(yb[7].abs().max()) == 0.0


def test_big_fista_teacher_forced_steps(big):
    op, Hh = big
    A = lambda v: ops.A_fft(Hh, v)
    AT = lambda v: ops.AT_fft(Hh, v)
    p0 = inputs.vascular_phantom(SHAPE, seed=1001)
    clean = A(p0)
    d = clean + inputs.NOISE_20DB * np.sqrt(np.mean(clean ** 2)) * inputs.noise_like(DSHAPE, seed=1501)
    dd = dev(d)
    L, _ = op.power_norm(dev(inputs.gaussian_random(SHAPE, seed=1002)), 30)
    tau = float(np.float32(1.0 / L))
    K = 100
    betas = solvers.momentum_weights(K)
    atd = op.apply_AT(dd)[None]
    x = torch.zeros((1,) + SHAPE, device="cuda")
    z = torch.zeros_like(x)
    states = {}
    for k in range(1, K + 1):
        if k in (1, 50, 100):
            states[k] = [host(x[0]), host(z[0])]
        op.fista_step_normal(atd, x, z, [betas[k - 1]], [tau], [0.0], [True])
        if k in states:
            states[k].append(host(x[0]))
    assert rel(host(op.recon_fista(dd, K, tau, 0.0, nonneg=True)), states[K][2]) < 1e-5

    def forced(k):
        xp, zp, xg = states[k]
        xo = solvers.fista(A, AT, d, SHAPE, 1, tau, 0.0, nonneg=True, z0=zp, x_prev0=xp, k0=k - 1)[0]
        return rel(xg, xo)

    with ThreadPoolExecutor(3) as ex:
        errs = dict(zip(states, ex.map(forced, states)))
    print("FISTA 256x256x128x512 teacher-forced rel. l2 error:", errs, flush=True)
    assert max(errs.values()) < 1e-5, errs
