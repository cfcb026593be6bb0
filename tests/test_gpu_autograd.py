"""Differentiation form on the GPU: backward of A is the HIP adjoint."""
import numpy as np
import pytest
import torch

from oracle import hlib, operators as ops
from oracle.geometry import paper_like
from paper_2603_28150_amd import autograd as pad, inputs
from paper_2603_28150_amd.op import Geometry, Operator

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_backward_is_oracle_adjoint():
    g = Geometry.paper_like(64, 64, 32, 128)
    op = Operator(g)
    Hh = hlib.H_half(paper_like(64, 64, 32, 128))
    x = torch.from_numpy(inputs.gaussian_random(op.x_shape, seed=3201).astype(np.float32)).cuda().requires_grad_(True)
    y = inputs.gaussian_random(op.d_shape, seed=3202)
    r = pad.forward(op, x) - torch.from_numpy(y.astype(np.float32)).cuda()
    (0.5 * (r * r).sum()).backward()
    x64 = x.detach().cpu().numpy().astype(np.float64)
    expect = ops.AT_fft(Hh, ops.A_fft(Hh, x64) - y)
    assert rel(x.grad.cpu().numpy().astype(np.float64), expect) < 1e-5


def test_directional_derivative_exact_on_gpu():
    g = Geometry.paper_like(128, 128, 64, 256)
    op = Operator(g)
    x = torch.from_numpy(inputs.vascular_phantom(op.x_shape, seed=3001).astype(np.float32)).cuda()
    v = torch.from_numpy(inputs.gaussian_random(op.x_shape, seed=3002).astype(np.float32)).cuda()
    y = torch.from_numpy(inputs.gaussian_random(op.d_shape, seed=3003).astype(np.float32)).cuda()
    h = float(x.norm() / v.norm())

    def f(u):
        r = (op.apply_A(u) - y).double()
        return 0.5 * float((r * r).sum())

    xr = x.clone().requires_grad_(True)
    r = pad.forward(op, xr) - y
    (0.5 * (r * r).sum()).backward()
    lhs = (f(x + h * v) - f(x - h * v)) / (2 * h)
    rhs = float((xr.grad.double() * v.double()).sum())
    assert abs(lhs - rhs) <= 1e-5 * abs(rhs)


def test_adam_tv_reconstruction_runs():
    # the differentiation workload: 128^2 x 64 x 256, 1/2||Ax-y||^2 + 1e-3 TV, Adam, 200 steps
    g = Geometry.paper_like(128, 128, 64, 256)
    op = Operator(g)
    p0 = torch.from_numpy(inputs.vascular_phantom(op.x_shape, seed=3001).astype(np.float32)).cuda()
    y = op.apply_A(p0)
    x, losses = pad.fit_adam_tv(op, y, steps=200, lr=1e-2, tv_weight=1e-3)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.05 * losses[0]
    assert float(torch.linalg.norm(x - p0) / torch.linalg.norm(p0)) < 1.0
