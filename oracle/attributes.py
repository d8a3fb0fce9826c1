"""Instance attributes that follow the z coordinate (Sec. II-B and Sec. III-A).

Partition, per-die cell size (Eq. std-size-tech), the linear macro size transition
(Eq. macro-size-tech), charge, the local-smoothness stretch of Sec. IV-A, and pin positions
whose offsets follow the partition like the cell sizes (bistratal model paragraph).
"""
from __future__ import annotations

import numpy as np

KIND_MACRO = 1
KIND_FIXED = 2
KIND_FILLER = 4     # dummy filler: no pins, left out of the overflow (Sec. III-A)
KIND_ZFIXED = 8     # z held: the z-gradient is zero (z-fixed fillers, Sec. III-A)


def partition(z, dz):
    """delta_i = 1 iff z_i - d_z/2 is strictly positive (top die); a tie is the bottom die."""
    return np.asarray(z, dtype=np.float64) > 0.5 * dz


def is_macro(kind):
    return (np.asarray(kind) & KIND_MACRO) != 0


def is_fixed(kind):
    return (np.asarray(kind) & KIND_FIXED) != 0


def is_filler(kind):
    return (np.asarray(kind) & KIND_FILLER) != 0


def is_zfixed(kind):
    return (np.asarray(kind) & KIND_ZFIXED) != 0


def instance_size(size, kind, z, dz):
    """Current width and height of every instance.

    Cells take the size of the die they sit on (Eq. std-size-tech).  Macros scale linearly with
    z between the bottom size at z = d_z/4 and the top size at z = 3 d_z/4 (Eq. macro-size-tech);
    reading: z is clamped to that range first, the movable range of Sec. III-A.
    """
    size = np.asarray(size, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    top = partition(z, dz)
    w = np.where(top, size[2], size[0])
    h = np.where(top, size[3], size[1])
    mac = is_macro(kind)
    zc = np.clip(z, 0.25 * dz, 0.75 * dz)
    t_top = 2.0 * zc / dz - 0.5
    t_bot = 1.5 - 2.0 * zc / dz
    w = np.where(mac, t_top * size[2] + t_bot * size[0], w)
    h = np.where(mac, t_top * size[3] + t_bot * size[1], h)
    return w, h


def macro_size_slope(size, kind, dz):
    """dw/dz and dh/dz of the macro size transition (zero for cells)."""
    size = np.asarray(size, dtype=np.float64)
    mac = is_macro(kind)
    dw = np.where(mac, 2.0 / dz * (size[2] - size[0]), 0.0)
    dh = np.where(mac, 2.0 / dz * (size[3] - size[1]), 0.0)
    return dw, dh


def charge(w, h, dz):
    """Electric quantity q_i: the physical volume, every instance having depth d_z/2."""
    return np.asarray(w) * np.asarray(h) * (0.5 * dz)


def smoothing(w, h, wb, hb):
    """Local smoothness (Sec. IV-A): weight omega and the stretched footprint.

    omega = min(1, w/(sqrt2 w_b)) * min(1, h/(sqrt2 h_b)).  Reading: as in ePlace, an instance
    smaller than sqrt2 bins is stretched to sqrt2 bins along that axis, so that omega times the
    stretched area equals the true area.  Depth is never stretched.
    """
    r2 = np.sqrt(2.0)
    wt = np.maximum(w, r2 * wb)
    ht = np.maximum(h, r2 * hb)
    omega = np.minimum(1.0, w / (r2 * wb)) * np.minimum(1.0, h / (r2 * hb))
    return wt, ht, omega


def pin_xy(xyz, pin2node, pin_off, dz, flip=False):
    """Pin x, y: the owner's centre plus the offset of the die the owner sits on.

    With ``flip`` the offset of the other die is used, i.e. the pin position after moving its
    owner across the bonding interface.  Reading: the offsets switch with delta for macros too.
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    node = np.asarray(pin2node)
    off = np.asarray(pin_off, dtype=np.float64)
    top = partition(xyz[2, node], dz)
    if flip:
        top = ~top
    px = xyz[0, node] + np.where(top, off[2], off[0])
    py = xyz[1, node] + np.where(top, off[3], off[1])
    return px, py, top
