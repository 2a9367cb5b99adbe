"""torch.autograd Functions over the library's kernels.

* RadonFwd: y = M R x; its backward is the adjoint product (and vice versa for
  RadonAdj), as R^T M^T is the transpose of M R (Section 3 stores both).
* NormalOp: out = alpha R^T M^T M R x + lambda K^T K x + sigma x; the operator
  is symmetric, so its backward is the same product.
* UnrolledCG: x_n = CG_n(rhs) from x_0 = 0 on that operator, differentiated
  through every iteration (the step lengths and beta_k depend on rhs, so the
  map is nonlinear); the library keeps checkpoints every `ckpt` iterations and
  replays each segment during the reverse sweep.

Losses of the gradient workload (a learned-prior setting built on the
resolvent system eq:PD_resolve of Section 2, alpha <- tau*alpha, lambda = 0,
sigma = 1):
  L1(mu, f) = 1/2 ||M R mu - f||^2,
  L2(mu, f) = 1/2 ||M R u - f||^2 with u = CG_n(mu + tau alpha R^T M^T f).
"""
from __future__ import annotations

import torch

__all__ = ["RadonFwd", "RadonAdj", "NormalOp", "UnrolledCG", "unrolled_cg", "loss_data",
           "loss_unrolled"]


def _c(t):
    return t if t.is_contiguous() else t.contiguous()


class RadonFwd(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op, x):
        ctx.op, ctx.shape = op, x.shape
        return op.fwd(_c(x))

    @staticmethod
    def backward(ctx, gy):
        return None, ctx.op.adj(_c(gy)).reshape(ctx.shape)


class RadonAdj(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op, y):
        ctx.op, ctx.shape = op, y.shape
        return op.adj(_c(y))

    @staticmethod
    def backward(ctx, gx):
        return None, ctx.op.fwd(_c(gx)).reshape(ctx.shape)


class NormalOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op, x, alpha, lam, sigma):
        ctx.op, ctx.coef, ctx.shape = op, (alpha, lam, sigma), x.shape
        return op.normal(_c(x), alpha, lam, sigma)

    @staticmethod
    def backward(ctx, g):
        return None, ctx.op.normal(_c(g), *ctx.coef).reshape(ctx.shape), None, None, None


class UnrolledCG(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op, rhs, alpha, lam, sigma, n_iter, ckpt):
        x, tape = op.cg_unrolled(_c(rhs), alpha, lam, sigma, n_iter, ckpt)
        ctx.op, ctx.args, ctx.tape, ctx.shape = op, (alpha, lam, sigma, n_iter, ckpt), tape, rhs.shape
        return x

    @staticmethod
    def backward(ctx, gx):
        g = ctx.op.cg_unrolled_vjp(ctx.tape, _c(gx), *ctx.args)
        return None, g.reshape(ctx.shape), None, None, None, None, None


def unrolled_cg(op, rhs, alpha: float, lam: float = 0.0, sigma: float = 1.0, n: int = 10,
                ckpt: int = 5):
    """x = CG_n(rhs) on alpha R^T M^T M R + lam K^T K + sigma I, differentiable in rhs."""
    return UnrolledCG.apply(op, rhs, float(alpha), float(lam), float(sigma), int(n), int(ckpt))


def loss_data(op, mu, f):
    """Per-image 1/2 ||M R mu - f||^2 (shape [batch])."""
    r = RadonFwd.apply(op, mu) - f.reshape(-1, op.rows)
    return 0.5 * (r * r).sum(dim=1)


def loss_unrolled(op, mu, f, tau_alpha: float, n: int = 10, ckpt: int = 5):
    """Per-image 1/2 ||M R CG_n(mu + tau_alpha R^T M^T f) - f||^2 on the
    resolvent operator tau_alpha R^T M^T M R + I."""
    fb = f.reshape(-1, op.rows)
    rhs = mu.reshape(-1, op.nn) + tau_alpha * RadonAdj.apply(op, fb)
    u = unrolled_cg(op, rhs, tau_alpha, 0.0, 1.0, n, ckpt)
    r = RadonFwd.apply(op, u) - fb
    return 0.5 * (r * r).sum(dim=1)
