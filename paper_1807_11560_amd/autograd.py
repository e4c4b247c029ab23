"""torch.autograd form of the registration energy (paper §3.2: the energy
E(v0) = 1/2 <L~ v0, v0> + sigma^-2 ||m(1) - I1||^2 subject to the band
EPDiff and state equations), differentiated exactly: argument marshalling
over the C-ABI.

``energy(problem, v0, I0, I1, ws)`` returns E(v0) as a 0-dim float64 tensor
that autograd can differentiate with respect to the complex64 band field v0.

  forward   lddmm_energy: shooting, transport and the energy reductions on
            the GPU, no adjoint work;
  backward  lddmm_gradient_exact: the reverse sweep of every Euler and
            transport step of the forward (the derivative of the discrete
            energy, which finite differences of ``energy`` see), then
            lddmm_apply_symbol turns the V-metric gradient g_V into the l2
            gradient L~ g_V, which under torch's convention for real
            functions of complex tensors is dE/dRe(v0) + i dE/dIm(v0).

The backward transports the state again rather than keeping it from the
forward: with ``problem.checkpoint = c`` only every c-th state is kept and
each segment is transported again during the sweep, so one workspace of
``lddmm_workspace_bytes`` for that problem serves both passes (at
160x192x160 / band 32^3 / 20 steps, c = 5: under a third of the unchecked
layout).  The images receive no gradient.
"""

import torch

from . import lddmm as L


class LDDMMShootSSD(torch.autograd.Function):
    """Energy of one registration problem as a differentiable function of v0."""

    @staticmethod
    def forward(ctx, v0, I0, I1, problem, ws):
        e3 = L.energy(problem, I0, I1, v0, ws)
        ctx.save_for_backward(v0, I0, I1)
        ctx.problem, ctx.ws = problem, ws
        return e3[0].clone()

    @staticmethod
    def backward(ctx, grad_e):
        v0, I0, I1 = ctx.saved_tensors
        g, _ = L.gradient_exact(ctx.problem, I0, I1, v0.detach(), ctx.ws)
        g_l2 = L.apply_symbol(ctx.problem, L.SYMBOL_L, g, ctx.ws)
        return grad_e.to(torch.float32) * g_l2, None, None, None, None


def energy(problem, v0, I0, I1, ws):
    """E(v0) as a differentiable 0-dim tensor (see the module doc)."""
    return LDDMMShootSSD.apply(v0, I0, I1, problem, ws)
