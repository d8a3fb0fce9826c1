"""The multi-die 2D problem of a 3D placement (Sec. III-C, Eq. 2d-place), built on the host.

After 3D global placement fixes each instance's die, the multi-die 2D placement works on three
layers: the bottom die's instances, the top die's instances (each at its own die's size and pin
offsets), and one hybrid bonding terminal (HBT) per net that crosses the dies.  A crossing net is
cut into its top partial net (its top pins and the HBT) and its bottom partial net (its bottom pins
and the HBT); the HBT, a square of side ``hbt_side`` with its pin at its centre, starts in the
middle of the net's optimal region (Eq. optimal-region), so that the two partial nets' HPWL equals
the net's minimal D2D wirelength at the split.  Nets on one die stay as they are.

This is one-time preprocessing before ``place3d.MultiDie2D``: vectorised NumPy over the netlist.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .place3d import KIND_FIXED, KIND_MACRO, LAYER_BOTTOM, LAYER_HBT, LAYER_TOP


@dataclass(frozen=True)
class Grid:
    die_x: float
    die_y: float
    nx: int
    ny: int


@dataclass
class Layers:
    """Nodes [0, n_inst) are the placement's instances, then the HBTs, in crossing-net order."""
    w: np.ndarray             # [n] width on its layer
    h: np.ndarray             # [n] height
    kind: np.ndarray          # [n] uint8 (MACRO, FIXED bits of the instances; 0 for HBTs)
    layer: np.ndarray         # [n] LAYER_BOTTOM, LAYER_TOP or LAYER_HBT
    net_start: np.ndarray     # [m' + 1] partial nets (CSR)
    pin2node: np.ndarray      # [P']
    pin_off: np.ndarray       # [2][P'] pin offset on the owner's layer (0 for an HBT's pin)
    grid: Grid
    gamma: float
    ramp: float
    target: float
    n_inst: int
    n_hbt: int


def _segment_extremes(values, seg, nseg, take):
    """Per segment, the max and min of values[take] (-inf / +inf where a segment takes nothing)."""
    hi = np.full(nseg, -np.inf)
    lo = np.full(nseg, np.inf)
    np.maximum.at(hi, seg[take], values[take])
    np.minimum.at(lo, seg[take], values[take])
    return hi, lo


def split(size, kind, xyz, net_start, pin2node, pin_off, dz, grid: Grid, gamma, hbt_side, ramp=1.05, target=1.0):
    """Layers and start positions xy [2][n_inst + n_hbt] of the placement xyz ([3][n], centres).

    size [4][n] (bottom w, h, top w, h), pin_off [4][P] (bottom x, y, top x, y); an instance is on
    the top die when z > d_z/2."""
    size = np.asarray(size, dtype=np.float64)
    xyz = np.asarray(xyz, dtype=np.float64)
    ns = np.asarray(net_start, dtype=np.int64)
    p2n = np.asarray(pin2node, dtype=np.int64)
    off = np.asarray(pin_off, dtype=np.float64)
    n, m, P = xyz.shape[1], ns.shape[0] - 1, p2n.shape[0]
    top = xyz[2] > 0.5 * dz
    w = np.where(top, size[2], size[0])
    h = np.where(top, size[3], size[1])
    pin_top = top[p2n]
    ox = np.where(pin_top, off[2], off[0])
    oy = np.where(pin_top, off[3], off[1])
    px = xyz[0, p2n] + ox
    py = xyz[1, p2n] + oy
    net_of = np.repeat(np.arange(m), np.diff(ns))
    n_top = np.bincount(net_of, weights=pin_top, minlength=m)
    n_bot = np.diff(ns) - n_top
    crossing = (n_top > 0) & (n_bot > 0)
    k = int(crossing.sum())
    cross_nets = np.nonzero(crossing)[0]
    hbt_of_net = np.full(m, -1, dtype=np.int64)
    hbt_of_net[cross_nets] = n + np.arange(k)
    # the HBT's start: per axis, the middle of the interval between the facing sides of the top and
    # bottom pin ranges (or of their overlap)
    hxy = np.zeros((2, k))
    for a, pu in enumerate((px, py)):
        thi, tlo = _segment_extremes(pu, net_of, m, pin_top)
        bhi, blo = _segment_extremes(pu, net_of, m, ~pin_top)
        s = np.minimum(thi, bhi)[cross_nets]
        t = np.maximum(tlo, blo)[cross_nets]
        lo, hi = np.minimum(s, t), np.maximum(s, t)
        hxy[a] = 0.5 * (lo + hi)
    # partial nets: a crossing net gives its top part (its top pins in order, then the HBT) and
    # its bottom part; every other net its pins in order
    part = np.where(crossing[net_of] & ~pin_top, 1, 0)
    pos = np.arange(P)
    h_net = np.repeat(cross_nets, 2)
    h_part = np.tile(np.array([0, 1]), k)
    keys_net = np.concatenate([net_of, h_net])
    keys_part = np.concatenate([part, h_part])
    keys_pos = np.concatenate([pos, np.full(2 * k, P)])          # the HBT's pin ends its part
    order = np.lexsort((keys_pos, keys_part, keys_net))
    nodes = np.concatenate([p2n, hbt_of_net[h_net]])[order]
    pox = np.concatenate([ox, np.zeros(2 * k)])[order]
    poy = np.concatenate([oy, np.zeros(2 * k)])[order]
    deg = np.diff(ns) + np.where(crossing, 2, 0)                 # each part gains the HBT's pin
    seg_net = np.concatenate([np.arange(m), cross_nets])        # one part per net, two when crossing
    seg_part = np.concatenate([np.zeros(m, dtype=np.int64), np.ones(k, dtype=np.int64)])
    seg_order = np.lexsort((seg_part, seg_net))
    top_sizes = np.where(crossing, n_top + 1, np.diff(ns))      # first part: top pins + HBT, or all pins
    bot_sizes = n_bot[cross_nets] + 1
    seg_size = np.concatenate([top_sizes, bot_sizes])[seg_order]
    assert int(seg_size.sum()) == int(deg.sum()) == nodes.shape[0]
    new_start = np.concatenate([[0], np.cumsum(seg_size)])
    lay = Layers(w=np.concatenate([w, np.full(k, float(hbt_side))]),
                 h=np.concatenate([h, np.full(k, float(hbt_side))]),
                 kind=np.concatenate([np.asarray(kind, dtype=np.uint8) & (KIND_MACRO | KIND_FIXED),
                                      np.zeros(k, dtype=np.uint8)]),
                 layer=np.concatenate([np.where(top, LAYER_TOP, LAYER_BOTTOM).astype(np.uint8),
                                       np.full(k, LAYER_HBT, dtype=np.uint8)]),
                 net_start=new_start.astype(np.int64), pin2node=nodes.astype(np.int64),
                 pin_off=np.stack([pox, poy]), grid=grid, gamma=float(gamma), ramp=float(ramp),
                 target=float(target), n_inst=n, n_hbt=k)
    return lay, np.concatenate([xyz[:2], hxy], axis=1)
