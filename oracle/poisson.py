"""Spectral solve of the Neumann Poisson problem (Sec. III-A, Eqs. 3d-poisson-equation,
density-coef, poisson-sol-potential, possion-sol-force).

Readings taken where the printed equations are silent or garbled:

* The density is sampled at bin centres x_i = (i + 1/2) w_b, with frequencies
  omega_j = j pi / d_x (and likewise in y and z).
* Normalisation: the printed coefficient (1/N) sum rho cos cos cos followed by the printed
  unweighted cosine sum does not reproduce rho, so the printed phi would not solve the printed
  Poisson equation.  The equation is taken as authoritative: per axis the coefficient carries
  (2 - [index = 0]) / N_axis, which makes the cosine series reproduce rho exactly.
* The (0,0,0) mode has 0/0 in the potential; it is dropped, which solves the equation for
  rho minus its mean with a potential of zero mean.

Dense transforms (matrix products with the sampled cosine and sine bases) are used throughout:
they are the definitions written out, not a fast algorithm.
"""
from __future__ import annotations

import numpy as np


def basis(n, length):
    """cos and sin of omega_j x_i on bin centres, as [sample i, frequency j] matrices, and omega."""
    i = np.arange(n)[:, None] + 0.5
    j = np.arange(n)[None, :]
    arg = np.pi * j * i / n
    omega = np.pi * np.arange(n) / length
    return np.cos(arg), np.sin(arg), omega


def _axis_weight(n):
    c = np.full(n, 2.0 / n)
    c[0] = 1.0 / n
    return c


def _apply(m, mat, axis):
    """Contract axis ``axis`` of map ``m`` (layout [z, y, x]) with mat[sample, out]."""
    return np.moveaxis(np.tensordot(m, mat, axes=([axis], [0])), -1, axis)


def coefficients(rho, geo):
    """a_jkl: cosine-series coefficients of rho (layout [l, k, j] = [z, y, x] frequencies)."""
    cx, _, _ = basis(geo.nx, geo.die_x)
    cy, _, _ = basis(geo.ny, geo.die_y)
    cz, _, _ = basis(geo.nz, geo.dz)
    a = _apply(np.asarray(rho, dtype=np.float64), cx * _axis_weight(geo.nx)[None, :], 2)
    a = _apply(a, cy * _axis_weight(geo.ny)[None, :], 1)
    a = _apply(a, cz * _axis_weight(geo.nz)[None, :], 0)
    return a


def synthesize(a, geo, kind=("c", "c", "c")):
    """sum_{jkl} a_jkl f_x(omega_j x) f_y(omega_k y) f_z(omega_l z) at bin centres, f = cos or sin.

    ``kind`` gives the function per axis in (x, y, z) order.
    """
    m = np.asarray(a, dtype=np.float64)
    for axis, n, length, f in ((2, geo.nx, geo.die_x, kind[0]), (1, geo.ny, geo.die_y, kind[1]),
                               (0, geo.nz, geo.dz, kind[2])):
        c, s, _ = basis(n, length)
        m = _apply(m, (c if f == "c" else s).T, axis)
    return m


def omega_squared(geo):
    _, _, wx = basis(geo.nx, geo.die_x)
    _, _, wy = basis(geo.ny, geo.die_y)
    _, _, wz = basis(geo.nz, geo.dz)
    return wz[:, None, None] ** 2 + wy[None, :, None] ** 2 + wx[None, None, :] ** 2, (wx, wy, wz)


def potential_coefficients(a, geo):
    """b_jkl = a_jkl / |omega|^2, with the (0,0,0) mode set to zero."""
    w2, _ = omega_squared(geo)
    b = np.zeros_like(np.asarray(a, dtype=np.float64))
    nz = w2 > 0
    b[nz] = a[nz] / w2[nz]
    return b


def solve(rho, geo, want=("phi", "ex", "ey", "ez")):
    """Potential phi and field E = -grad phi at bin centres (Eqs. poisson-sol-potential and
    possion-sol-force).  Returns a dict with the requested maps."""
    a = coefficients(rho, geo)
    b = potential_coefficients(a, geo)
    _, (wx, wy, wz) = omega_squared(geo)
    out = {}
    if "phi" in want:
        out["phi"] = synthesize(b, geo, ("c", "c", "c"))
    if "ex" in want:
        out["ex"] = synthesize(b * wx[None, None, :], geo, ("s", "c", "c"))
    if "ey" in want:
        out["ey"] = synthesize(b * wy[None, :, None], geo, ("c", "s", "c"))
    if "ez" in want:
        out["ez"] = synthesize(b * wz[:, None, None], geo, ("c", "c", "s"))
    return out


def energy(rho, phi, geo):
    """U = 1/2 sum_b rho_b phi_b vol(b).

    Reading: the paper writes the energy as sum_i q_i phi_i, which counts every pair of charges
    twice; the factor 1/2 makes its derivative the charge times the potential gradient.
    """
    return 0.5 * float(np.sum(np.asarray(rho) * np.asarray(phi))) * geo.vol_bin
