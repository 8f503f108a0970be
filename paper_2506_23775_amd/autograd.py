"""torch.autograd integration of the circuit cost.

``circuit_cost(gates, circuit, target)`` returns f(G) = -Re Tr[U^dagger C(G)]
as a differentiable scalar.  Gradients use the paper's convention
grad f = d_x f + i d_y f (Sec. "Riemannian optimization"), which is also the
gradient PyTorch accumulates for a real loss of complex leaves, so
``gates.grad`` is the Euclidean gradient computed by ``rq_grad``.  The
gradient is itself differentiable: its vector-Jacobian product is the
Euclidean Hessian applied to the incoming vector (the Hessian is symmetric in
real coordinates), evaluated by ``rq_hvp``; ``torch.autograd.grad`` with
``create_graph=True`` therefore yields Hessian-vector products.

All arithmetic runs in librq's kernels; this module only routes tensors.
"""

from __future__ import annotations

import torch

from . import rq


def _ctx_args(ctx):
    return ctx.circuit, ctx.target, ctx.range, ctx.chunk


class _EuclideanGradient(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gates, circuit, target, rng, chunk):
        ctx.circuit, ctx.target, ctx.range, ctx.chunk = circuit, target, rng, chunk
        ctx.save_for_backward(gates)
        _, eg, _ = rq.rq_grad(circuit, target, gates.detach(), range=rng, chunk=chunk)
        return eg.to(device=gates.device, dtype=gates.dtype)

    @staticmethod
    def backward(ctx, v):
        (gates,) = ctx.saved_tensors
        circuit, target, rng, chunk = _ctx_args(ctx)
        out = rq.rq_hvp(circuit, target, gates.detach(), v.detach(), range=rng, chunk=chunk)
        ehvp = out[3].to(device=gates.device, dtype=gates.dtype)
        return ehvp, None, None, None, None


class _Cost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gates, circuit, target, rng, chunk):
        ctx.circuit, ctx.target, ctx.range, ctx.chunk = circuit, target, rng, chunk
        ctx.save_for_backward(gates)
        f = rq.rq_cost(circuit, target, gates.detach(), range=rng, chunk=chunk)
        return f.to(device=gates.device, dtype=torch.float64).reshape(())

    @staticmethod
    def backward(ctx, gout):
        (gates,) = ctx.saved_tensors
        circuit, target, rng, chunk = _ctx_args(ctx)
        eg = _EuclideanGradient.apply(gates, circuit, target, rng, chunk)
        return gout.to(eg.dtype) * eg, None, None, None, None


def circuit_cost(gates: torch.Tensor, circuit: "rq.Circuit", target: "rq.Target",
                 range=None, chunk=None) -> torch.Tensor:
    """Differentiable f(G) for complex [P, 4, 4] gates (any device)."""
    if not gates.is_complex():
        raise TypeError("gates must be a complex tensor [P, 4, 4]")
    return _Cost.apply(gates, circuit, target, range, chunk)


def euclidean_gradient(gates: torch.Tensor, circuit, target, range=None, chunk=None):
    """Differentiable Euclidean gradient (its VJP is the Euclidean HVP)."""
    return _EuclideanGradient.apply(gates, circuit, target, range, chunk)
