"""A as a differentiable torch operation whose backward is A^T.

f(x) = 1/2 ||A x - y||^2 has gradient A^T (A x - y) (eq. 15), so the
backward of y = A x for an upstream gradient g is A^T g: the hand-written
adjoint kernel, not a traced transpose.  The backend is anything with
``apply_A`` / ``apply_AT`` methods taking and returning tensors (the HIP
``Operator``; tests also plug in a float64 CPU backend).
"""
from __future__ import annotations

import torch


class PatA(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, backend) -> torch.Tensor:
        ctx.backend = backend
        return backend.apply_A(x.contiguous())

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        return ctx.backend.apply_AT(gy.contiguous()), None


class PatAT(torch.autograd.Function):
    """A^T as a differentiable operation (its backward is A)."""

    @staticmethod
    def forward(ctx, y: torch.Tensor, backend) -> torch.Tensor:
        ctx.backend = backend
        return backend.apply_AT(y.contiguous())

    @staticmethod
    def backward(ctx, gx: torch.Tensor):
        return ctx.backend.apply_A(gx.contiguous()), None


def forward(backend, x: torch.Tensor) -> torch.Tensor:
    """y = A x, differentiable in x."""
    return PatA.apply(x, backend)


def adjoint(backend, y: torch.Tensor) -> torch.Tensor:
    """x = A^T y, differentiable in y."""
    return PatAT.apply(y, backend)


def tv_iso(x: torch.Tensor, eps: float = 1e-6) -> torch.Tensor:
    """Isotropic total variation sum sqrt(|grad x|^2 + eps^2) of x[..., z, y, x]:
    forward differences, periodic in x and y, zero last difference in z."""
    dx = torch.roll(x, -1, dims=-1) - x
    dy = torch.roll(x, -1, dims=-2) - x
    dz = torch.zeros_like(x)
    dz[..., :-1, :, :] = x[..., 1:, :, :] - x[..., :-1, :, :]
    return torch.sqrt(dx * dx + dy * dy + dz * dz + eps * eps).sum()


def fit_adam_tv(backend, y: torch.Tensor, steps: int = 200, lr: float = 1e-2,
                tv_weight: float = 1e-3, x0: torch.Tensor | None = None, callback=None):
    """Minimise 1/2 ||A x - y||^2 + tv_weight * TV(x) with Adam from x0 (default 0).
    Returns (x, list of loss values)."""
    shape = backend.x_shape
    x = torch.zeros(shape, dtype=y.dtype, device=y.device) if x0 is None else x0.clone()
    x.requires_grad_(True)
    opt = torch.optim.Adam([x], lr=lr)
    losses = []
    for k in range(steps):
        opt.zero_grad(set_to_none=True)
        r = forward(backend, x) - y
        loss = 0.5 * (r * r).sum() + tv_weight * tv_iso(x)
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
        if callback is not None:
            callback(k, x)
    return x.detach(), losses
