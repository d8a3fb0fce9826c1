"""Bin grid and stack geometry (Sec. II-A; experimental setup, Sec. V-A)."""
from __future__ import annotations

import math
from dataclasses import dataclass


@dataclass(frozen=True)
class Geometry:
    """The cuboid region [0, d_x] x [0, d_y] x [0, d_z] cut into N_x x N_y x N_z bins.

    Sec. V-A sets the z-bin size to the mean of the planar bin sizes and the region depth to
    N_z z-bins, so the depth is derived, not an input.
    """
    die_x: float
    die_y: float
    nx: int
    ny: int
    nz: int

    @property
    def wb(self) -> float:
        return self.die_x / self.nx

    @property
    def hb(self) -> float:
        return self.die_y / self.ny

    @property
    def db(self) -> float:
        return 0.5 * (self.wb + self.hb)

    @property
    def dz(self) -> float:
        return self.nz * self.db

    @property
    def vol_bin(self) -> float:
        return self.wb * self.hb * self.db


def geometry_of(case) -> Geometry:
    return Geometry(float(case.die_x), float(case.die_y), int(case.nx), int(case.ny), int(case.nz))


def hbt_alpha(die_x: float, dz: float, hbt_pitch: float, row_top: float, row_bot: float,
              beta: float, alpha0: float = 3.5e-3) -> float:
    """Weight of the cut-size term alpha * p_e(z) (Sec. V-A).

    eta is twice the HBT pitch over the sum of the two row heights, and
    alpha = alpha0 * (d_x eta^2 / d_z) * log(90 beta eta - 1).
    Reading: ``log`` is the natural logarithm.
    """
    eta = 2.0 * hbt_pitch / (row_top + row_bot)
    return alpha0 * (die_x * eta * eta / dz) * math.log(90.0 * beta * eta - 1.0)
