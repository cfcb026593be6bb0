"""GPU parity of the sensor response folded into the library along t: the
library, A, A^T and FISTA against the float64 oracle (which folds by direct
causal convolution of its library along t), for random taps, a band-pass
design, 16-bit storage and the linear boundary."""
import numpy as np
import pytest
import torch

from oracle import hlib, operators as ops, quant, solvers
from oracle.geometry import Geometry as OGeom, doubled
from paper_2603_28150_amd import inputs
from paper_2603_28150_amd.op import Geometry, Operator

pytestmark = pytest.mark.gpu

_dt = 0.3 * 100e-6 / 1500.0
TAPS = {
    "random9": tuple(inputs.gaussian_random((9,), seed=910)),
    "bandpass63": tuple(inputs.bandpass_fir(63, 5e6, 20e6, _dt)),
    "single": (0.7,),
}
CASES = {
    "tiny-random9": (Geometry.paper_like(32, 32, 16, 64, ir=TAPS["random9"]), "random9"),
    "ragged-bandpass63": (Geometry(32, 16, 13, 97, 1e-4, 1.3e-4, 1e-4, 2e-8, 1500.0, 0, "periodic",
                                   TAPS["bandpass63"]), "bandpass63"),
    "mid-single": (Geometry.paper_like(64, 64, 40, 130, ir=TAPS["single"]), "single"),
    "linear-random9": (Geometry.paper_like(16, 16, 16, 64, boundary="linear", ir=TAPS["random9"]), "random9"),
}


def og(g: Geometry) -> OGeom:
    o = OGeom(g.nx, g.ny, g.nz, g.nt, g.dx, g.dy, g.dz, g.dt, g.c, g.nz_sim)
    return doubled(o) if g.boundary == "linear" else o


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_ops(g, H):
    if g.boundary == "linear":
        return (lambda v: ops.A_linear(H, v)), (lambda v: ops.AT_linear(H, v))
    return (lambda v: ops.A_fft(H, v)), (lambda v: ops.AT_fft(H, v))


_cache = {}


def setup(name):
    if name not in _cache:
        g, taps = CASES[name]
        Hr = hlib.with_sensor_response(hlib.H_half(og(g)), TAPS[taps])
        _cache[name] = (g, Operator(g), Hr)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_filtered_library_and_operator_match_oracle(name):
    g, op, Hr = setup(name)
    Hg = host(op.export_H())
    Ho = Hr.reshape(op.nk, g.nz, g.nt)
    assert np.abs(Hg - Ho).max() <= 1e-7 * np.abs(Ho).max()
    A, AT = oracle_ops(g, Hr)
    x = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=920)
    d = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=921)
    assert rel(host(op.apply_A(dev(x))), A(x)) < 1e-5
    assert rel(host(op.apply_AT(dev(d))), AT(d)) < 1e-5
    assert op.adjoint_check(dev(x), dev(d)) < 1e-5


def test_filtered_fista_gram_path_matches_oracle():
    g, op, Hr = setup("tiny-random9")
    A, AT = oracle_ops(g, Hr)
    clean = A(inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=930))
    d = clean + 0.01 * np.sqrt(np.mean(clean ** 2)) * inputs.noise_like(clean.shape, seed=931)
    tau = float(np.float32(0.9 / solvers.norm_exact(Hr)))
    xs = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), 10, tau, 1e-3, nonneg=True)
    for k in (1, 10):
        assert rel(host(op.recon_fista(dev(d), k, tau, 1e-3, nonneg=True)), xs[k - 1]) < 1e-5, k


@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_filtered_16bit_library(kind):
    g, _, Hr = setup("tiny-random9")
    op = Operator(g, kind)
    Hq, _ = quant.quantise(Hr, kind)
    x = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=940)
    assert rel(host(op.apply_A(dev(x))), ops.A_fft(Hq, x)) < 2e-5
    assert rel(host(op.apply_A(dev(x))), ops.A_fft(Hr, x)) < 5e-3
