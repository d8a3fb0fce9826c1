"""torch.autograd Functions over the C ABI (argument marshalling only; every step runs in the
HIP library).

* ``Density``        xyz -> rho (place3d_density); backward: the exact adjoint place3d_density_vjp.
* ``Field``          rho -> phi (place3d_field); the map rho -> phi of the spectral solve is
                     symmetric (forward coefficients and inverse sum share the cosine basis, the
                     weights sit on the diagonal), so backward is the same solve applied to the
                     incoming gradient.
* ``DensityEnergy``  xyz -> U = 1/2 sum_b rho_b phi_b vol(b), reduced in float64 by the library
                     (place3d_density, then place3d_field with its energy output); backward:
                     dU/drho = phi vol(b) by the symmetry of the solve, taken through the exact
                     adjoint (place3d_density_vjp with the incoming gradient as its device factor).
* ``WAWirelength``   xyz -> W = sum_e (W^_e(x) + W^_e(y) + alpha p^_e(z)) (place3d_wl_value: net
                     totals only, nothing kept per pin); backward: place3d_wl_vjp recomputes every
                     net's extremes and shifted exponential sums from xyz.  With ``fda=True`` (the
                     placer's choice) the z part of the gradient is the paper's surrogate, the
                     normalised FDA of Eqs. fda-grad and fda-normalize plus alpha dp^(z)/dz; with
                     ``fda=False`` it is the derivative of W itself, alpha dp^(z)/dz (the bistratal
                     part changes with z only by steps).

``density_energy(prob, xyz)`` is ``DensityEnergy``; composing ``Density`` and ``Field`` gives the
same gradient and leaves the reduction to the caller.
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


class DensityEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, prob, xyz):
        xyz = prob.xyz(xyz.detach())
        rho = prob.density(xyz)
        out = prob.field(rho, want=("phi",), energy=True)
        ctx.prob = prob
        ctx.save_for_backward(xyz, out["phi"])
        return out["energy"].reshape(())

    @staticmethod
    def backward(ctx, g_u):
        xyz, phi = ctx.saved_tensors
        prob = ctx.prob
        vol = (prob.die_x / prob.nx) * (prob.die_y / prob.ny) * 0.5 * (prob.die_x / prob.nx + prob.die_y / prob.ny)
        return None, prob.density_vjp(xyz, phi, scale=vol, d_scale=g_u.reshape(1))


class WAWirelength(torch.autograd.Function):
    @staticmethod
    def forward(ctx, prob, xyz, fda=True):
        xyz = prob.xyz(xyz.detach())
        met = prob.wl_value(xyz)
        ctx.prob = prob
        ctx.fda = bool(fda)
        ctx.save_for_backward(xyz)
        return met[place3d.M["wa_bi"]] + met[place3d.M["wa_z"]]

    @staticmethod
    def backward(ctx, g_w):
        (xyz,) = ctx.saved_tensors
        mode = place3d.WLZ_FDA if ctx.fda else place3d.WLZ_VALUE
        return None, ctx.prob.wl_vjp(xyz, d_scale=g_w.reshape(1), z_mode=mode), None


def density_energy(prob, xyz):
    """U = 1/2 sum_b rho_b phi_b vol(b) (float64) with its gradient through the exact adjoint."""
    return DensityEnergy.apply(prob, xyz)


def wirelength(prob, xyz, fda=True):
    """W = sum_e (W^_e(x) + W^_e(y) + alpha p^_e(z)) (float64); see WAWirelength for the z part."""
    return WAWirelength.apply(prob, xyz, fda)
