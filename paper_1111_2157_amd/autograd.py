"""torch.autograd.Function over the Dyson / Matsubara-sum step.

forward  -> density_matrix (N(k) of every k, concatenated, and G_loc)
backward -> density_matrix_vjp (the library's hand-written adjoint)

Gradients follow PyTorch's complex convention (dL/dRe + i dL/dIm) with the
positive-frequency Sigma(i w_n) as the independent variable and Sigma_inf and
V_DC held fixed; mu is a real scalar tensor.
"""
from __future__ import annotations

import torch

from .dyson import Context, Lattice, SelfEnergy


class DysonDensity(torch.autograd.Function):
    @staticmethod
    def forward(fctx, sigma, mu, context: Context, lat: Lattice, base: SelfEnergy, tail_order: int):
        sig = SelfEnergy(base.nw, base.beta, sigma.detach().contiguous(), base.sigma_inf, base.e_dc)
        nk, gl, _ = context.density_matrix(lat, sig, float(mu), tail_order, nk=True, gloc=True, scalars=False)
        fctx.context, fctx.lat, fctx.sig, fctx.tail = context, lat, sig, tail_order
        fctx.mu = float(mu)
        return nk, gl

    @staticmethod
    def backward(fctx, nk_bar, gl_bar):
        sb, mb = fctx.context.density_matrix_vjp(fctx.lat, fctx.sig, fctx.mu, nk_bar, gl_bar, fctx.tail)
        return sb, mb.reshape(()), None, None, None, None


def dyson_density(sigma: torch.Tensor, mu: torch.Tensor, context: Context, lat: Lattice, base: SelfEnergy,
                  tail_order: int = 2):
    """(N(k) of all k concatenated, G_loc) as differentiable functions of
    sigma [nw, nc, nc] (complex128) and mu (float64 scalar)."""
    return DysonDensity.apply(sigma, mu, context, lat, base, tail_order)
