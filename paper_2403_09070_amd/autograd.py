"""torch.autograd Functions over the C ABI (argument marshalling only; every step runs in the
HIP library).

* ``Density``      xyz -> rho (place3d_density); backward: the exact adjoint place3d_density_vjp.
* ``Field``        rho -> phi (place3d_field); the map rho -> phi of the spectral solve is
                   symmetric (forward coefficients and inverse sum share the cosine basis, the
                   weights sit on the diagonal), so backward is the same solve applied to the
                   incoming gradient.
* ``WAWirelength`` xyz -> the smoothed bistratal wirelength plus the alpha-weighted z term
                   (place3d_wl_grad); backward returns the library's gradient, whose z part is the
                   paper's normalised FDA surrogate (Eqs. fda-grad, fda-normalize) plus the z term's
                   derivative, not the derivative of the smoothed wirelength in z.

``density_energy(prob, xyz)`` composes the first two into U = 1/2 sum_b rho_b phi_b vol(b), whose
gradient through these Functions is the autograd form of the density penalty's gradient.
"""
from __future__ import annotations

import torch

from . import place3d


class Density(torch.autograd.Function):
    @staticmethod
    def forward(ctx, prob, xyz):
        xyz = prob.xyz(xyz.detach())
        ctx.prob = prob
        ctx.save_for_backward(xyz)
        return prob.density(xyz)

    @staticmethod
    def backward(ctx, g_rho):
        (xyz,) = ctx.saved_tensors
        return None, ctx.prob.density_vjp(xyz, g_rho.contiguous())


class Field(torch.autograd.Function):
    @staticmethod
    def forward(ctx, prob, rho):
        ctx.prob = prob
        return prob.field(rho.detach(), want=("phi",))["phi"]

    @staticmethod
    def backward(ctx, g_phi):
        return None, ctx.prob.field(g_phi.contiguous(), want=("phi",))["phi"]


class WAWirelength(torch.autograd.Function):
    @staticmethod
    def forward(ctx, prob, xyz):
        g, met = prob.wl_grad(xyz.detach())
        ctx.save_for_backward(g)
        total = met[place3d.M["wa_bi"]] + met[place3d.M["wa_z"]]
        return total.to(torch.float32)

    @staticmethod
    def backward(ctx, g_out):
        (g,) = ctx.saved_tensors
        return None, g * g_out.to(g.dtype)


def density_energy(prob, xyz):
    """U = 1/2 sum_b rho_b phi_b vol(b) through Density and Field."""
    rho = Density.apply(prob, xyz)
    phi = Field.apply(prob, rho)
    vol = (prob.die_x / prob.nx) * (prob.die_y / prob.ny) * 0.5 * (prob.die_x / prob.nx + prob.die_y / prob.ny)
    return 0.5 * vol * (rho * phi).sum()
