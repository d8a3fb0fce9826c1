"""Objective gradient, 3D mixed-size preconditioner, Nesterov step and GP metrics.

* Objective: sum of the wirelength model plus lambda times the density penalty
  (Eq. analytical-placement), with the z-part of the wirelength gradient from ``wirelength``.
* Preconditioner (Eq. improved-precond): H_ii = max{1, |E_i| + lambda q_i} for movable macros,
  max{1, lambda q_i} otherwise; |E_i| is the pin count and q_i the volume.  The ePlace
  (|E_i| + lambda q_i) and ePlace3D (lambda q_i) forms of Eq. general-precond are kept as
  variants.  Reading: the same H_ii divides the x, y and z components.
* Optimiser: the paper does not describe it; it inherits the Nesterov method with a Lipschitz
  step estimate of ePlace/DREAMPlace.  Readings: a_0 = 1, a_{k+1} = (1 + sqrt(4 a_k^2 + 1))/2;
  step = |v_k - v_{k-1}|_2 / |g_k - g_{k-1}|_2 over movable coordinates (0 if the gradient did
  not change); u_{k+1} = clamp(v_k - step g_k); v_{k+1} = clamp(u_{k+1} + (a_k - 1)/a_{k+1}
  (u_{k+1} - u_k)); no backtracking; lambda_0 = |grad W|_1 / |grad U|_1 at the start, then
  lambda grows by a fixed ratio each step; the bootstrap point is
  v_{-1} = clamp(v_0 - 0.01 w_b g_0 / |g_0|_inf).  Parity unpinned beyond the convex-quadratic
  convergence test.
* Clamp: z to [d_z/4, 3 d_z/4] (the movable range of Sec. III-A), then x, y so that the
  instance, at the size its clamped z gives, stays inside the die.  Fixed instances never move.
* Overflow per die (reading; the paper prints overflow without defining it): the ePlace form
  sum_{b in die} max(rho_b - rho_t, 0) vol(b) / sum_{movable i on die} q_i, the bottom die being
  the lower half of the z-bins.  Fillers (Sec. III-A) are left out of both: the excess is taken
  on the map of the other instances and the charge sums over movable non-fillers.
* z-held instances (the z-fixed fillers of Sec. III-A): their z-gradient is set to zero in both
  objective parts before anything else uses them (lambda_0, preconditioning, the step).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import poisson
from .attributes import charge, instance_size, is_filler, is_fixed, is_macro, is_zfixed, partition
from .density import density_map
from .density_grad import density_vjp, field_gather
from .geometry import Geometry, geometry_of, hbt_alpha
from .wirelength import wirelength


@dataclass
class Problem:
    size: np.ndarray
    kind: np.ndarray
    net_start: np.ndarray
    pin2node: np.ndarray
    pin_off: np.ndarray
    geo: Geometry
    gamma: float
    alpha: float
    ramp: float
    target: float

    @property
    def npins(self):
        return np.bincount(np.asarray(self.pin2node), minlength=self.kind.shape[0]).astype(np.float64)

    @property
    def movable(self):
        return ~is_fixed(self.kind)


def problem_of(case) -> Problem:
    geo = geometry_of(case)
    cfg = case.config
    alpha = hbt_alpha(geo.die_x, geo.dz, cfg.hbt_pitch, cfg.row_top, cfg.row_bot, cfg.beta, cfg.alpha0)
    return Problem(case.size, case.kind, case.net_start, case.pin2node, case.pin_off, geo,
                   cfg.gamma_bins * geo.wb, alpha, cfg.lambda_ramp, cfg.target_density)


def preconditioner(pb: Problem, xyz, lam, mode="mixed"):
    w, h = instance_size(pb.size, pb.kind, np.asarray(xyz, dtype=np.float64)[2], pb.geo.dz)
    lq = lam * charge(w, h, pb.geo.dz)
    if mode == "mixed":
        mac = is_macro(pb.kind) & pb.movable
        return np.where(mac, np.maximum(1.0, pb.npins + lq), np.maximum(1.0, lq))
    if mode == "eplace":
        return pb.npins + lq
    if mode == "eplace3d":
        return lq
    raise ValueError(mode)


def clamp(pb: Problem, xyz):
    xyz = np.array(xyz, dtype=np.float64)
    out = xyz.copy()
    dz = pb.geo.dz
    out[2] = np.clip(xyz[2], 0.25 * dz, 0.75 * dz)
    w, h = instance_size(pb.size, pb.kind, out[2], dz)
    out[0] = np.minimum(np.maximum(xyz[0], 0.5 * w), pb.geo.die_x - 0.5 * w)
    out[1] = np.minimum(np.maximum(xyz[1], 0.5 * h), pb.geo.die_y - 0.5 * h)
    fixed = is_fixed(pb.kind)
    out[:, fixed] = xyz[:, fixed]
    return out


def density_gradient(pb: Problem, xyz, dgrad="field"):
    """Density map, potential/field and the penalty gradient (field gather or exact adjoint)."""
    rho = density_map(pb.size, pb.kind, xyz, pb.geo)
    if dgrad == "field":
        sol = poisson.solve(rho, pb.geo, want=("phi", "ex", "ey", "ez"))
        g = field_gather(pb.size, pb.kind, xyz, sol["ex"], sol["ey"], sol["ez"], pb.geo)
    elif dgrad == "adjoint":
        sol = poisson.solve(rho, pb.geo, want=("phi",))
        g = density_vjp(pb.size, pb.kind, xyz, sol["phi"] * pb.geo.vol_bin, pb.geo)
    else:
        raise ValueError(dgrad)
    return rho, sol, g


def overflow(pb: Problem, rho, xyz):
    """Per-die overflow (bottom, top); with fillers, of the map without them."""
    geo = pb.geo
    fill = is_filler(pb.kind)
    if fill.any():
        real = ~fill
        rho = density_map(pb.size[:, real], pb.kind[real], np.asarray(xyz)[:, real], geo)
    excess = np.maximum(np.asarray(rho) - pb.target, 0.0) * geo.vol_bin
    half = geo.nz // 2
    w, h = instance_size(pb.size, pb.kind, np.asarray(xyz, dtype=np.float64)[2], geo.dz)
    q = charge(w, h, geo.dz)
    top = partition(np.asarray(xyz, dtype=np.float64)[2], geo.dz)
    mov = pb.movable & ~fill
    q_bot = float(q[mov & ~top].sum())
    q_top = float(q[mov & top].sum())
    o_bot = float(excess[:half].sum()) / q_bot if q_bot > 0 else 0.0
    o_top = float(excess[half:].sum()) / q_top if q_top > 0 else 0.0
    return o_bot, o_top


def evaluate(pb: Problem, xyz, dgrad="field"):
    """Wirelength and density parts of the objective gradient at xyz (unscaled by lambda), with
    the z components of z-held instances set to zero."""
    wl = wirelength(pb.size, pb.kind, xyz, pb.net_start, pb.pin2node, pb.pin_off, pb.geo,
                    pb.gamma, pb.alpha)
    rho, sol, gd = density_gradient(pb, xyz, dgrad)
    held = is_zfixed(pb.kind)
    if held.any():
        wl = dict(wl)
        wl["grad"] = np.array(wl["grad"], dtype=np.float64)
        wl["grad"][2, held] = 0.0
        gd = np.array(gd, dtype=np.float64)
        gd[2, held] = 0.0
    return wl, rho, sol, gd


@dataclass
class GPState:
    u: np.ndarray
    v: np.ndarray
    v_prev: np.ndarray
    g_prev: np.ndarray
    a: float
    lam: float
    it: int = 0


def gp_init(pb: Problem, xyz0, dgrad="field", precond="mixed") -> GPState:
    v0 = clamp(pb, xyz0)
    wl, _, _, gd = evaluate(pb, v0, dgrad)
    mov = pb.movable
    gw = wl["grad"]
    lam = float(np.abs(gw[:, mov]).sum() / np.abs(gd[:, mov]).sum())
    g0 = (gw + lam * gd) / preconditioner(pb, v0, lam, precond)[None, :]
    gmax = float(np.abs(g0[:, mov]).max())
    v_prev = clamp(pb, v0 - 0.01 * pb.geo.wb * g0 / gmax)
    wl_p, _, _, gd_p = evaluate(pb, v_prev, dgrad)
    g_prev = (wl_p["grad"] + lam * gd_p) / preconditioner(pb, v_prev, lam, precond)[None, :]
    return GPState(u=v0.copy(), v=v0.copy(), v_prev=v_prev, g_prev=g_prev, a=1.0, lam=lam)


def nesterov_update(st: GPState, g, clamp_fn, movable):
    """Lipschitz step estimate and the Nesterov move; returns (u_new, v_new, a_new, step)."""
    dv = float(np.sqrt(np.sum((st.v - st.v_prev)[:, movable] ** 2)))
    dg = float(np.sqrt(np.sum((g - st.g_prev)[:, movable] ** 2)))
    step = dv / dg if dg > 0.0 else 0.0
    u_new = clamp_fn(st.v - step * g)
    a_new = 0.5 * (1.0 + math.sqrt(4.0 * st.a * st.a + 1.0))
    v_new = clamp_fn(u_new + (st.a - 1.0) / a_new * (u_new - st.u))
    return u_new, v_new, a_new, step


def gp_step(pb: Problem, st: GPState, dgrad="field", precond="mixed"):
    """One Nesterov iteration in place; returns the metrics measured at the evaluation point."""
    wl, rho, sol, gd = evaluate(pb, st.v, dgrad)
    g = (wl["grad"] + st.lam * gd) / preconditioner(pb, st.v, st.lam, precond)[None, :]
    u_new, v_new, a_new, step = nesterov_update(st, g, lambda p: clamp(pb, p), pb.movable)
    ob, ot = overflow(pb, rho, st.v)
    metrics = dict(it=st.it, lam=st.lam, step=step, hpwl_d2d=wl["hpwl_d2d"], wa_bi=wl["wa_bi"],
                   wa_z=wl["wa_z"], ncut=wl["ncut"], ovfl_bot=ob, ovfl_top=ot,
                   energy=poisson.energy(rho, sol["phi"], pb.geo))
    st.v_prev, st.g_prev = st.v, g
    st.u, st.v, st.a = u_new, v_new, a_new
    st.lam *= pb.ramp
    st.it += 1
    return metrics
