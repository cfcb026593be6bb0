"""The autograd wrapper: forward A, backward A^T (CPU, float64 oracle backend)."""
import numpy as np
import torch

from paper_2603_28150_amd import autograd as pad, inputs
from tests.oracle_backend import OracleBackend


def test_gradcheck_forward_and_adjoint():
    be = OracleBackend(16, 16, 16, 32)
    x = torch.from_numpy(inputs.gaussian_random(be.x_shape, seed=3101)).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda v: pad.forward(be, v), (x,), fast_mode=True)
    y = torch.from_numpy(inputs.gaussian_random(be.d_shape, seed=3102)).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda v: pad.adjoint(be, v), (y,), fast_mode=True)


def test_data_term_gradient_is_adjoint_of_residual():
    be = OracleBackend(16, 16, 8, 24)
    x = torch.from_numpy(inputs.gaussian_random(be.x_shape, seed=1)).requires_grad_(True)
    y = torch.from_numpy(inputs.gaussian_random(be.d_shape, seed=2))
    r = pad.forward(be, x) - y
    (0.5 * (r * r).sum()).backward()
    expect = be.apply_AT(be.apply_A(x.detach()) - y)
    assert torch.allclose(x.grad, expect, rtol=0, atol=1e-12 * float(expect.abs().max()))


def test_central_difference_is_exact_for_the_quadratic():
    # f(x + h v) - f(x - h v) = 2 h <grad f(x), v> for f = 1/2 ||A x - y||^2
    be = OracleBackend(16, 16, 8, 24)
    x = torch.from_numpy(inputs.gaussian_random(be.x_shape, seed=3))
    v = torch.from_numpy(inputs.gaussian_random(be.x_shape, seed=4))
    y = torch.from_numpy(inputs.gaussian_random(be.d_shape, seed=5))
    f = lambda u: 0.5 * float(((be.apply_A(u) - y) ** 2).sum())
    h = float(x.norm() / v.norm())
    xr = x.clone().requires_grad_(True)
    r = pad.forward(be, xr) - y
    (0.5 * (r * r).sum()).backward()
    lhs = (f(x + h * v) - f(x - h * v)) / (2 * h)
    rhs = float((xr.grad * v).sum())
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_adam_tv_decreases_the_objective():
    be = OracleBackend(16, 16, 8, 16)
    p0 = inputs.gaussian_blobs(be.x_shape, seed=3001)
    y = be.apply_A(torch.from_numpy(p0))
    x, losses = pad.fit_adam_tv(be, y, steps=30, lr=1e-2)
    assert losses[-1] < 0.5 * losses[0]
    assert x.shape == be.x_shape


def test_tv_closed_form():
    # a single step edge in x of height a over the full (y, z) extent: periodic
    # TV along x counts two jumps per row
    x = torch.zeros(2, 4, 8, dtype=torch.float64)
    x[..., 3:6] = 2.0
    tv = pad.tv_iso(x, eps=0.0)
    assert abs(float(tv) - 2 * 4 * 2 * 2.0) < 1e-12
