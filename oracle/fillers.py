"""Dummy fillers (Sec. III-A density model, Eqs. filler-vol and free-filler-vol).  Test infrastructure.

Two kinds of fillers join the instances:
* z-fixed fillers, one equal-sized set per die, of total volume vol_f^+ = 1/2 d_x d_y d_z (1 - u^+)
  on the top die and vol_f^- = 1/2 d_x d_y d_z (1 - u^-) on the bottom die (u^+- the maximum
  utilisation of each die), each of depth d_z/2, started at z = 3 d_z/4 (top) or d_z/4 (bottom);
  their z-gradient is zero, so their z never changes;
* free fillers, of total volume vol_fr = max{d_x d_y d_z - (vol_f^+ + vol_f^- + vol_a), 0}, with
  vol_a the volume of all instances at their initial position; they move in x, y and z.

Readings (the paper gives neither the filler footprint nor how a volume becomes a count):
* the footprint is a square; the z-fixed fillers of a die take the mean footprint area of the
  movable standard cells at that die's size, the free fillers the mean of the two dies' areas (so
  their volume does not depend on the die they sit on);
* the count is the volume over one filler's volume (footprint x d_z/2), rounded to the nearest
  integer, halves up;
* vol_a counts every instance (movable and fixed) at the size its initial z gives;
* a filler has no pins; the overflow is measured on the map of the real instances (fillers left
  out of the excess and of the charge it is divided by), as the fillers exist only to shape the
  density force.
"""
from __future__ import annotations

import math

import numpy as np

from .attributes import KIND_FILLER, KIND_FIXED, KIND_MACRO, charge, instance_size


def filler_volumes(die_x, die_y, dz, u_top, u_bot, vol_a):
    """(vol_f^+, vol_f^-, vol_fr) of Eqs. filler-vol and free-filler-vol."""
    total = die_x * die_y * dz
    vf_top = 0.5 * total * (1.0 - u_top)
    vf_bot = 0.5 * total * (1.0 - u_bot)
    vfr = max(total - (vf_top + vf_bot + vol_a), 0.0)
    return vf_top, vf_bot, vfr


def instance_volume(size, kind, z0, dz):
    """vol_a: total volume of the instances at their initial z."""
    w, h = instance_size(size, kind, z0, dz)
    return float(charge(w, h, dz).sum())


def filler_plan(size, kind, z0, die_x, die_y, dz, u_top, u_bot):
    """Counts and square sides of the top and bottom z-fixed fillers and of the free fillers."""
    size = np.asarray(size, dtype=np.float64)
    kind = np.asarray(kind)
    cells = (kind & (KIND_MACRO | KIND_FIXED | KIND_FILLER)) == 0
    if not cells.any():
        raise ValueError("fillers are sized from the movable standard cells; there are none")
    a_top = float(np.mean(size[2, cells] * size[3, cells]))
    a_bot = float(np.mean(size[0, cells] * size[1, cells]))
    a_free = 0.5 * (a_top + a_bot)
    vol_a = instance_volume(size, kind, z0, dz)
    vf_top, vf_bot, vfr = filler_volumes(die_x, die_y, dz, u_top, u_bot, vol_a)

    def count(vol, area):
        return int(math.floor(vol / (area * 0.5 * dz) + 0.5))

    return dict(n_top=count(vf_top, a_top), n_bot=count(vf_bot, a_bot), n_free=count(vfr, a_free),
                side_top=math.sqrt(a_top), side_bot=math.sqrt(a_bot), side_free=math.sqrt(a_free),
                vol_top=vf_top, vol_bot=vf_bot, vol_free=vfr, vol_a=vol_a)
