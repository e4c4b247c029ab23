"""torch.autograd form of the registration energy (paper §3.2 energy, its
gradient by the adjoint Jacobi sweep): argument marshalling over the C-ABI.

``energy(problem, v0, I0, I1, ws)`` returns E(v0) = 1/2 <L~ v0, v0> +
sigma^-2 ||m(1) - I1||^2 as a 0-dim float64 tensor that autograd can
differentiate with respect to the complex64 band field v0.  The forward pass
is lddmm_gradient (shooting, transport, energy, adjoint Jacobi sweep, all on
the GPU); the backward pass returns grad_E times the l2 gradient L~ g_V
(lddmm_apply_symbol on the V-metric gradient), which under torch's convention
for real functions of complex tensors is dE/dRe(v0) + i dE/dIm(v0).  The
gradient is the paper's method (the adjoint Jacobi equations), not the exact
derivative of the discrete energy: they agree at v0 = 0, and away from it the
band truncation of the coadjoint transport leaves a gap that does not shrink
with the number of time steps.  The images receive no gradient.

The whole trajectory of one call stays in the workspace (no checkpointing:
at 160x192x160, band 32^3 and 20 steps it is under 3 GiB of the 288 GiB of
HBM), and lddmm_hessvec may follow on the same workspace.
"""

import torch

from . import lddmm as L


class LDDMMShootSSD(torch.autograd.Function):
    """Energy of one registration problem as a differentiable function of v0."""

    @staticmethod
    def forward(ctx, v0, I0, I1, problem, ws):
        g, e3 = L.gradient(problem, I0, I1, v0, ws)
        ctx.save_for_backward(L.apply_symbol(problem, L.SYMBOL_L, g, ws))
        return e3[0].clone()

    @staticmethod
    def backward(ctx, grad_e):
        (g_l2,) = ctx.saved_tensors
        return (grad_e.to(torch.float32) * g_l2, None, None, None, None)


def energy(problem, v0, I0, I1, ws):
    """E(v0) as a differentiable 0-dim tensor (see the module doc)."""
    return LDDMMShootSSD.apply(v0, I0, I1, problem, ws)
