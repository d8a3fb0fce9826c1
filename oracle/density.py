"""Bin density map (Sec. IV-A, Eq. density-map-accum) and the prefix-sum route of Theorem 1.

``box_density`` is the plain definition: every instance adds omega * vol(D ∩ b) / vol(b) to
every bin b its cuboid D overlaps.  ``box_density_prefix`` builds the signed 8-corner map of
Eq. 3d-density-accum-cuboid and takes one 3D prefix sum (Eq. def-prefix-sum-3d); it exists only
so that the tests can check Theorem 1 against the plain definition.
"""
from __future__ import annotations

import numpy as np

from .attributes import instance_size, smoothing

_SMALL_SPAN = 4   # instances spanning at most this many bins per axis take the vectorised loop


def footprints(size, kind, xyz, geo):
    """Stretched cuboid of every instance, clipped to the region, and its weight omega.

    D_i = [x - w~/2, x + w~/2] x [y - h~/2, y + h~/2] x [z - d_z/4, z + d_z/4] (Sec. IV-A) with
    the local-smoothness stretch of ``attributes.smoothing``.  Reading: the cuboid is clipped to
    the region, so the part of a stretched footprint outside the die carries no charge.
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    w, h = instance_size(size, kind, xyz[2], geo.dz)
    wt, ht, omega = smoothing(w, h, geo.wb, geo.hb)
    x0 = np.clip(xyz[0] - 0.5 * wt, 0.0, geo.die_x)
    x1 = np.clip(xyz[0] + 0.5 * wt, 0.0, geo.die_x)
    y0 = np.clip(xyz[1] - 0.5 * ht, 0.0, geo.die_y)
    y1 = np.clip(xyz[1] + 0.5 * ht, 0.0, geo.die_y)
    z0 = np.clip(xyz[2] - 0.25 * geo.dz, 0.0, geo.dz)
    z1 = np.clip(xyz[2] + 0.25 * geo.dz, 0.0, geo.dz)
    return np.stack([x0, x1, y0, y1, z0, z1]), omega


def axis_overlap(lo, hi, b, step):
    """Length of [lo, hi] ∩ [b*step, (b+1)*step]."""
    return np.maximum(0.0, np.minimum(hi, (b + 1) * step) - np.maximum(lo, b * step))


def _bin_range(lo, hi, step, n):
    b0 = np.clip(np.floor(lo / step).astype(np.int64), 0, n - 1)
    b1 = np.clip(np.ceil(hi / step).astype(np.int64) - 1, 0, n - 1)
    return b0, np.maximum(b1, b0)


def box_density(boxes, weight, geo):
    """rho_b = sum_i weight_i * vol(box_i ∩ b) / vol(b), looping over the bins each box overlaps."""
    boxes = np.asarray(boxes, dtype=np.float64)
    weight = np.asarray(weight, dtype=np.float64)
    rho = np.zeros((geo.nz, geo.ny, geo.nx))
    steps = (geo.wb, geo.hb, geo.db)
    ns = (geo.nx, geo.ny, geo.nz)
    rng = [_bin_range(boxes[2 * a], boxes[2 * a + 1], steps[a], ns[a]) for a in range(3)]
    span = np.stack([r[1] - r[0] + 1 for r in rng])
    small = (span <= _SMALL_SPAN).all(axis=0)
    idx = np.nonzero(small)[0]
    for ox in range(_SMALL_SPAN):
        bx = rng[0][0][idx] + ox
        lx = np.where(bx <= rng[0][1][idx], axis_overlap(boxes[0, idx], boxes[1, idx], bx, geo.wb), 0.0)
        for oy in range(_SMALL_SPAN):
            by = rng[1][0][idx] + oy
            ly = np.where(by <= rng[1][1][idx], axis_overlap(boxes[2, idx], boxes[3, idx], by, geo.hb), 0.0)
            for oz in range(_SMALL_SPAN):
                bz = rng[2][0][idx] + oz
                lz = np.where(bz <= rng[2][1][idx],
                              axis_overlap(boxes[4, idx], boxes[5, idx], bz, geo.db), 0.0)
                val = weight[idx] * lx * ly * lz / geo.vol_bin
                hit = val != 0.0
                np.add.at(rho, (bz[hit], by[hit], bx[hit]), val[hit])
    for i in np.nonzero(~small)[0]:
        bx = np.arange(rng[0][0][i], rng[0][1][i] + 1)
        by = np.arange(rng[1][0][i], rng[1][1][i] + 1)
        bz = np.arange(rng[2][0][i], rng[2][1][i] + 1)
        lx = axis_overlap(boxes[0, i], boxes[1, i], bx, geo.wb)
        ly = axis_overlap(boxes[2, i], boxes[3, i], by, geo.hb)
        lz = axis_overlap(boxes[4, i], boxes[5, i], bz, geo.db)
        rho[bz[0]:bz[-1] + 1, by[0]:by[-1] + 1, bx[0]:bx[-1] + 1] += (
            weight[i] * lz[:, None, None] * ly[None, :, None] * lx[None, None, :] / geo.vol_bin)
    return rho


def density_map(size, kind, xyz, geo):
    """The density map of every instance (cells, macros, fixed macros) on the grid."""
    boxes, omega = footprints(size, kind, xyz, geo)
    return box_density(boxes, omega, geo)


# ---------------------------------------------------------------- Theorem 1 (test-only route)

def corner_value(a):
    """g(a) = max(1 - |a|, 0) (Eq. 3d-density-accum-corner)."""
    return np.maximum(1.0 - np.abs(a), 0.0)


def corner_map(xh, yh, zh, shape):
    """A^{(x,y,z)} with entries g(i - x^) g(j - y^) g(k - z^) on 0-based bin indices.

    Reading of the index convention: the printed corner formula is 1-based, g(i - 1 - x^); the
    Lemma's proof is 0-based, g(i' - x^).  Both put the corner's mass on bins floor(x^) and
    floor(x^) + 1.  Entries that fall past the last bin are dropped: they would only feed bins
    outside the grid.  ``shape`` is (nz, ny, nx).
    """
    A = np.zeros(shape)
    nz, ny, nx = shape
    ix = [i for i in (int(np.floor(xh)), int(np.floor(xh)) + 1) if 0 <= i < nx]
    iy = [j for j in (int(np.floor(yh)), int(np.floor(yh)) + 1) if 0 <= j < ny]
    iz = [k for k in (int(np.floor(zh)), int(np.floor(zh)) + 1) if 0 <= k < nz]
    for k in iz:
        for j in iy:
            for i in ix:
                A[k, j, i] += corner_value(i - xh) * corner_value(j - yh) * corner_value(k - zh)
    return A


def prefix_sum_3d(A):
    """Inclusive prefix sum over all three axes (Eq. def-prefix-sum-3d)."""
    return np.cumsum(np.cumsum(np.cumsum(A, axis=0), axis=1), axis=2)


def box_corner_map(box, geo):
    """A_v of Eq. 3d-density-accum-cuboid: the 8 corner maps, each signed -sigma_x sigma_y sigma_z."""
    x0, x1, y0, y1, z0, z1 = (float(v) for v in box)
    A = np.zeros((geo.nz, geo.ny, geo.nx))
    for sx, xc in ((-1, x0), (1, x1)):
        for sy, yc in ((-1, y0), (1, y1)):
            for sz, zc in ((-1, z0), (1, z1)):
                A += -sx * sy * sz * corner_map(xc / geo.wb, yc / geo.hb, zc / geo.db, A.shape)
    return A


def box_density_prefix(boxes, weight, geo):
    """Density of a set of boxes by Theorem 1: one prefix sum of the summed corner maps."""
    boxes = np.asarray(boxes, dtype=np.float64)
    A = np.zeros((geo.nz, geo.ny, geo.nx))
    for i in range(boxes.shape[1]):
        A += float(weight[i]) * box_corner_map(boxes[:, i], geo)
    return prefix_sum_3d(A)
