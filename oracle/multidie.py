"""Multi-die 2D global placement (Sec. III-C, Eq. 2d-place): plain FP64 definitions (test
infrastructure, like the rest of this package).

With the partition fixed by a 3D placement, the z axis is dropped: the top die, the bottom die and
the layer of hybrid bonding terminals (HBTs) are three independent 2D electrostatic systems with
weights lambda = (lambda+, lambda-, lambda'), and the objective is

    sum_e W^_e(x, y) + lambda+ U+ + lambda- U- + lambda' U'.

Every net with pins on both dies gets one HBT, a movable node on the HBT layer that joins its top
partial net (the net's top pins and the HBT) and its bottom partial net (bottom pins and the HBT);
other nets are unchanged.  W^_e is the WA model (Eq. wa-model-approx) of each partial net in x and
y.  Readings (the paper states the formulation only):

* Node sizes: every instance takes the size of its die (macros included); an HBT is a square of
  side w', the HBT pitch of the technology; pins on an instance take that die's offsets, an HBT's
  pin sits at its centre.
* HBT start: the middle of the optimal region of Eq. optimal-region along each axis, the interval
  between the two boxes' facing sides (or their overlap), so that the start's partial-net HPWL
  equals the 3D bistratal wirelength of the net (Eq. wl-obj).
* Density of a layer: Eq. density-map-accum in 2D, rho_b = sum_i omega_i area(D_i ∩ b)/area(b),
  with the local-smoothness stretch to sqrt2 bins (reading 3 of the 3D model); energy
  U = 1/2 sum_b rho_b phi_b area(b) with phi from the 2D cosine solve (the 3D solve with one z
  layer: only l = 0 modes).  Gradient by the field gather, -omega sum_b area(D ∩ b) E_b.
* Fillers (the paper inserts fillers whose total area is the die area minus the instance area):
  per die, squares of the mean area of that die's movable standard cells; on the HBT layer,
  squares of one bin's area; a count is the free area over one filler's area, rounded to nearest.
* Preconditioner per node: Eq. improved-precond with the node's layer weight and q = w h;
  an HBT has |E| = 2 and is treated as a cell.
* lambda_0 per layer: |grad W|_1 over that layer's nodes / |grad U_L|_1; all three grow by the
  same ratio each iteration.  Optimiser and clamp as in the 3D oracle, in x and y only.
* Overflow per layer: sum_b max(rho_b - rho_t, 0) area(b) over the map without fillers, divided
  by the area of the layer's movable non-filler nodes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import poisson
from .attributes import KIND_FILLER, KIND_FIXED, KIND_MACRO, partition
from .density import box_density
from .geometry import Geometry
from .wirelength import degree_classes, exact_extent, wa_extent

BOTTOM, TOP, HBT = 0, 1, 2


@dataclass(frozen=True)
class Grid2D:
    die_x: float
    die_y: float
    nx: int
    ny: int

    @property
    def wb(self):
        return self.die_x / self.nx

    @property
    def hb(self):
        return self.die_y / self.ny

    @property
    def area_bin(self):
        return self.wb * self.hb

    def one_layer(self):
        """The 3D geometry with a single z layer: its cosine solve keeps only the l = 0 modes."""
        return Geometry(self.die_x, self.die_y, self.nx, self.ny, 1)


@dataclass
class Layered:
    """Nodes (instances, HBTs, fillers) and partial nets of a multi-die 2D problem."""
    w: np.ndarray            # [n] width on its layer
    h: np.ndarray            # [n] height
    kind: np.ndarray         # [n] uint8 KIND_* bits (MACRO, FIXED, FILLER)
    layer: np.ndarray        # [n] BOTTOM, TOP or HBT
    net_start: np.ndarray    # partial nets
    pin2node: np.ndarray
    pin_off: np.ndarray      # [2][P] pin offset on the owner's layer
    grid: Grid2D
    gamma: float
    ramp: float
    target: float
    n_inst: int              # nodes [0, n_inst) are the placement's instances, then HBTs, then fillers
    n_hbt: int

    @property
    def n(self):
        return self.w.shape[0]

    @property
    def movable(self):
        return (self.kind & KIND_FIXED) == 0

    @property
    def npins(self):
        return np.bincount(np.asarray(self.pin2node), minlength=self.n).astype(np.float64)


def optimal_hbt_interval(top_u, bot_u):
    """Along one axis, the interval of HBT positions that minimises p(top + HBT) + p(bottom + HBT)
    (Eq. optimal-region): between the facing sides of the two pin ranges, or their overlap."""
    a = min(max(top_u), max(bot_u))
    b = max(min(top_u), min(bot_u))
    return min(a, b), max(a, b)


def split(size, kind, xyz, net_start, pin2node, pin_off, dz, grid, gamma, hbt_side, ramp=1.05, target=1.0):
    """The multi-die 2D problem of a 3D placement: the partition by z, node sizes and pin offsets of
    each instance's die, one HBT per crossing net started in its optimal region, the partial nets.
    Returns (Layered, xy0 [2][n])."""
    size = np.asarray(size, dtype=np.float64)
    xyz = np.asarray(xyz, dtype=np.float64)
    ns = np.asarray(net_start, dtype=np.int64)
    p2n = np.asarray(pin2node, dtype=np.int64)
    off = np.asarray(pin_off, dtype=np.float64)
    n = xyz.shape[1]
    top = partition(xyz[2], dz)
    w = np.where(top, size[2], size[0])
    h = np.where(top, size[3], size[1])
    layer = np.where(top, TOP, BOTTOM)
    pins_top = top[p2n]
    px = xyz[0, p2n] + np.where(pins_top, off[2], off[0])
    py = xyz[1, p2n] + np.where(pins_top, off[3], off[1])
    ox = np.where(pins_top, off[2], off[0])
    oy = np.where(pins_top, off[3], off[1])
    new_start, new_pins, new_ox, new_oy, hbt_xy = [0], [], [], [], []
    for e in range(len(ns) - 1):
        q = np.arange(ns[e], ns[e + 1])
        t, b = q[pins_top[q]], q[~pins_top[q]]
        if len(t) and len(b):
            hid = n + len(hbt_xy)
            lo_x, hi_x = optimal_hbt_interval(px[t], px[b])
            lo_y, hi_y = optimal_hbt_interval(py[t], py[b])
            hbt_xy.append((0.5 * (lo_x + hi_x), 0.5 * (lo_y + hi_y)))
            for part in (t, b):
                new_pins += list(p2n[part]) + [hid]
                new_ox += list(ox[part]) + [0.0]
                new_oy += list(oy[part]) + [0.0]
                new_start.append(len(new_pins))
        else:
            new_pins += list(p2n[q])
            new_ox += list(ox[q])
            new_oy += list(oy[q])
            new_start.append(len(new_pins))
    k = len(hbt_xy)
    hxy = np.array(hbt_xy, dtype=np.float64).reshape(k, 2).T
    lay = Layered(w=np.concatenate([w, np.full(k, hbt_side)]), h=np.concatenate([h, np.full(k, hbt_side)]),
                  kind=np.concatenate([np.asarray(kind, dtype=np.uint8) & (KIND_MACRO | KIND_FIXED),
                                       np.zeros(k, dtype=np.uint8)]),
                  layer=np.concatenate([layer, np.full(k, HBT)]), net_start=np.array(new_start, dtype=np.int64),
                  pin2node=np.array(new_pins, dtype=np.int64), pin_off=np.array([new_ox, new_oy], dtype=np.float64),
                  grid=grid, gamma=gamma, ramp=ramp, target=target, n_inst=n, n_hbt=k)
    xy0 = np.concatenate([xyz[:2], hxy], axis=1)
    return lay, xy0


def filler_plan(lay: Layered):
    """Per layer (bottom, top, HBT): (count, side) of the fillers that take up the free area."""
    g = lay.grid
    out = []
    for L in (BOTTOM, TOP, HBT):
        on = (lay.layer == L) & ((lay.kind & KIND_FILLER) == 0)
        free = g.die_x * g.die_y - float(np.sum(lay.w[on] * lay.h[on]))
        if L == HBT:
            side = math.sqrt(g.area_bin)
        else:
            cells = on & ((lay.kind & (KIND_MACRO | KIND_FIXED)) == 0) & (np.arange(lay.n) < lay.n_inst)
            side = math.sqrt(float(np.mean(lay.w[cells] * lay.h[cells]))) if cells.any() else math.sqrt(g.area_bin)
        count = int(math.floor(max(free, 0.0) / (side * side) + 0.5))
        out.append((count, side))
    return out


def with_fillers(lay: Layered, xy, plan, seed=0):
    """The problem with the planned fillers appended (no pins), x and y uniform inside the die."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w, h, kind, layer, pts = [lay.w], [lay.h], [lay.kind], [lay.layer], [np.asarray(xy, dtype=np.float64)]
    g = lay.grid
    for L, (count, side) in zip((BOTTOM, TOP, HBT), plan):
        w.append(np.full(count, side))
        h.append(np.full(count, side))
        kind.append(np.full(count, KIND_FILLER, dtype=np.uint8))
        layer.append(np.full(count, L))
        pts.append(np.stack([side / 2 + rng.random(count) * (g.die_x - side),
                             side / 2 + rng.random(count) * (g.die_y - side)]))
    out = Layered(w=np.concatenate(w), h=np.concatenate(h), kind=np.concatenate(kind), layer=np.concatenate(layer),
                  net_start=lay.net_start, pin2node=lay.pin2node, pin_off=lay.pin_off, grid=lay.grid,
                  gamma=lay.gamma, ramp=lay.ramp, target=lay.target, n_inst=lay.n_inst, n_hbt=lay.n_hbt)
    return out, np.concatenate(pts, axis=1)


# ------------------------------------------------------------------ density, field, gradient

def _boxes(w, h, xy, grid):
    """Stretched footprints clipped to the die (as 3D boxes spanning the one z layer) and omega."""
    r2 = math.sqrt(2.0)
    wt = np.maximum(w, r2 * grid.wb)
    ht = np.maximum(h, r2 * grid.hb)
    omega = np.minimum(1.0, w / (r2 * grid.wb)) * np.minimum(1.0, h / (r2 * grid.hb))
    x, y = np.asarray(xy[0], dtype=np.float64), np.asarray(xy[1], dtype=np.float64)
    g1 = grid.one_layer()
    boxes = np.stack([np.clip(x - wt / 2, 0, grid.die_x), np.clip(x + wt / 2, 0, grid.die_x),
                      np.clip(y - ht / 2, 0, grid.die_y), np.clip(y + ht / 2, 0, grid.die_y),
                      np.zeros_like(x), np.full_like(x, g1.dz)])
    return boxes, omega


def density_2d(w, h, xy, grid):
    """rho_b = sum_i omega_i area(D_i ∩ b) / area(b) on the ny x nx grid (the 3D definition with
    one z layer that every footprint spans)."""
    boxes, omega = _boxes(w, h, xy, grid)
    return box_density(boxes, omega, grid.one_layer())[0]


def solve_2d(rho, grid, want=("phi", "ex", "ey")):
    """Potential and field of a 2D map (the cosine solve of Sec. III-A with one z layer)."""
    sol = poisson.solve(np.asarray(rho, dtype=np.float64)[None], grid.one_layer(),
                        want=tuple(k for k in want if k != "ez"))
    return {k: v[0] for k, v in sol.items()}


def energy_2d(rho, phi, grid):
    return 0.5 * float(np.sum(rho * phi)) * grid.area_bin


def field_gather_2d(w, h, kind, xy, ex, ey, grid):
    """-omega sum_b area(D ∩ b) E_b per node ([2][n]); fixed nodes get zero.  Footprints spanning
    at most four bins per axis go through a loop over their bin offsets, larger ones one by one."""
    boxes, omega = _boxes(w, h, xy, grid)
    wb, hb = grid.wb, grid.hb
    n = boxes.shape[1]
    bx0 = np.clip(np.floor(boxes[0] / wb).astype(np.int64), 0, grid.nx - 1)
    bx1 = np.maximum(np.clip(np.ceil(boxes[1] / wb).astype(np.int64) - 1, 0, grid.nx - 1), bx0)
    by0 = np.clip(np.floor(boxes[2] / hb).astype(np.int64), 0, grid.ny - 1)
    by1 = np.maximum(np.clip(np.ceil(boxes[3] / hb).astype(np.int64) - 1, 0, grid.ny - 1), by0)
    small = (bx1 - bx0 < 4) & (by1 - by0 < 4)
    out = np.zeros((2, n))
    idx = np.nonzero(small)[0]
    for ox in range(4):
        bx = bx0[idx] + ox
        lx = np.where(bx <= bx1[idx], np.maximum(0.0, np.minimum(boxes[1, idx], (bx + 1) * wb)
                                                 - np.maximum(boxes[0, idx], bx * wb)), 0.0)
        bxc = np.minimum(bx, grid.nx - 1)
        for oy in range(4):
            by = by0[idx] + oy
            ly = np.where(by <= by1[idx], np.maximum(0.0, np.minimum(boxes[3, idx], (by + 1) * hb)
                                                     - np.maximum(boxes[2, idx], by * hb)), 0.0)
            byc = np.minimum(by, grid.ny - 1)
            a = lx * ly
            out[0, idx] += a * ex[byc, bxc]
            out[1, idx] += a * ey[byc, bxc]
    for i in np.nonzero(~small)[0]:
        bx = np.arange(bx0[i], bx1[i] + 1)
        by = np.arange(by0[i], by1[i] + 1)
        lx = np.maximum(0.0, np.minimum(boxes[1, i], (bx + 1) * wb) - np.maximum(boxes[0, i], bx * wb))
        ly = np.maximum(0.0, np.minimum(boxes[3, i], (by + 1) * hb) - np.maximum(boxes[2, i], by * hb))
        a = ly[:, None] * lx[None, :]
        out[0, i] = float(np.sum(a * ex[by0[i]:by1[i] + 1, bx0[i]:bx1[i] + 1]))
        out[1, i] = float(np.sum(a * ey[by0[i]:by1[i] + 1, bx0[i]:bx1[i] + 1]))
    out *= -omega[None, :]
    out[:, (np.asarray(kind) & KIND_FIXED) != 0] = 0.0
    return out


def layer_parts(lay: Layered, xy):
    """Per layer: its density map, potential, field, energy and field-gather gradient of its nodes."""
    g = lay.grid
    parts = []
    for L in (BOTTOM, TOP, HBT):
        on = np.nonzero(lay.layer == L)[0]
        rho = density_2d(lay.w[on], lay.h[on], xy[:, on], g)
        sol = solve_2d(rho, g)
        grad = np.zeros((2, lay.n))
        grad[:, on] = field_gather_2d(lay.w[on], lay.h[on], lay.kind[on], xy[:, on], sol["ex"], sol["ey"], g)
        parts.append(dict(nodes=on, rho=rho, sol=sol, energy=energy_2d(rho, sol["phi"], g), grad=grad))
    return parts


# ------------------------------------------------------------------ wirelength of the partial nets

def wirelength_2d(lay: Layered, xy):
    """WA (Eq. wa-model-approx) of every partial net in x and y, its per-node gradient, and the exact
    HPWL of the partial nets (the D2D wirelength with the HBTs where they are)."""
    xy = np.asarray(xy, dtype=np.float64)
    node = np.asarray(lay.pin2node, dtype=np.int64)
    off = np.asarray(lay.pin_off, dtype=np.float64)
    grad = np.zeros((2, lay.n))
    wa = hpwl = 0.0
    for d, nets, pins in degree_classes(lay.net_start):
        nd = node[pins]
        everyone = np.ones(pins.shape, dtype=bool)
        for a in range(2):
            u = xy[a, nd] + off[a, pins]
            p, gp = wa_extent(u, everyone, lay.gamma)
            wa += float(np.sum(p))
            hpwl += float(np.sum(exact_extent(u, everyone)))
            np.add.at(grad[a], nd.ravel(), gp.ravel())
    grad[:, (lay.kind & KIND_FIXED) != 0] = 0.0
    return dict(wa=wa, hpwl=hpwl, grad=grad)


# ------------------------------------------------------------------ optimiser

def preconditioner_2d(lay: Layered, lam3):
    lam = np.asarray(lam3, dtype=np.float64)[lay.layer]
    lq = lam * lay.w * lay.h
    mac = ((lay.kind & KIND_MACRO) != 0) & lay.movable
    return np.where(mac, np.maximum(1.0, lay.npins + lq), np.maximum(1.0, lq))


def clamp_2d(lay: Layered, xy):
    out = np.array(xy, dtype=np.float64)
    g = lay.grid
    mov = lay.movable
    out[0, mov] = np.minimum(np.maximum(out[0, mov], 0.5 * lay.w[mov]), g.die_x - 0.5 * lay.w[mov])
    out[1, mov] = np.minimum(np.maximum(out[1, mov], 0.5 * lay.h[mov]), g.die_y - 0.5 * lay.h[mov])
    return out


def overflow_2d(lay: Layered, xy):
    """(bottom, top, HBT layer) overflow of the maps without fillers."""
    g = lay.grid
    out = []
    for L in (BOTTOM, TOP, HBT):
        on = np.nonzero((lay.layer == L) & ((lay.kind & KIND_FILLER) == 0))[0]
        rho = density_2d(lay.w[on], lay.h[on], xy[:, on], g)
        excess = float(np.sum(np.maximum(rho - lay.target, 0.0))) * g.area_bin
        mov = on[lay.movable[on]]
        area = float(np.sum(lay.w[mov] * lay.h[mov]))
        out.append(excess / area if area > 0 else 0.0)
    return tuple(out)


def evaluate_2d(lay: Layered, xy):
    """Wirelength gradient and the per-layer density gradient (unscaled by lambda) at xy."""
    wl = wirelength_2d(lay, xy)
    parts = layer_parts(lay, xy)
    gd = sum(p["grad"] for p in parts)
    return wl, parts, gd


@dataclass
class GPState2D:
    u: np.ndarray
    v: np.ndarray
    v_prev: np.ndarray
    g_prev: np.ndarray
    a: float
    lam: np.ndarray          # (lambda-, lambda+, lambda') in layer order (bottom, top, HBT)
    it: int = 0


def _combined(lay, wl, gd, lam):
    lamn = np.asarray(lam)[lay.layer]
    return (wl["grad"] + lamn[None, :] * gd) / preconditioner_2d(lay, lam)[None, :]


def gp_init_2d(lay: Layered, xy0):
    v0 = clamp_2d(lay, xy0)
    wl, parts, gd = evaluate_2d(lay, v0)
    mov = lay.movable
    lam = np.zeros(3)
    for L in (BOTTOM, TOP, HBT):
        on = mov & (lay.layer == L)
        den = float(np.abs(gd[:, on]).sum())
        lam[L] = float(np.abs(wl["grad"][:, on]).sum()) / den if den > 0 else 0.0
    g0 = _combined(lay, wl, gd, lam)
    gmax = float(np.abs(g0[:, mov]).max())
    v_prev = clamp_2d(lay, v0 - 0.01 * lay.grid.wb * g0 / gmax)
    wl_p, _, gd_p = evaluate_2d(lay, v_prev)
    g_prev = _combined(lay, wl_p, gd_p, lam)
    return GPState2D(u=v0.copy(), v=v0.copy(), v_prev=v_prev, g_prev=g_prev, a=1.0, lam=lam)


def gp_step_2d(lay: Layered, st: GPState2D):
    """One Nesterov iteration in place (the 3D oracle's optimiser in x, y); returns the metrics at
    the evaluation point."""
    from .optimizer import nesterov_update
    wl, parts, gd = evaluate_2d(lay, st.v)
    g = _combined(lay, wl, gd, st.lam)
    u_new, v_new, a_new, step = nesterov_update(st, g, lambda p: clamp_2d(lay, p), lay.movable)
    ob, ot, oh = overflow_2d(lay, st.v)
    metrics = dict(it=st.it, step=step, wa=wl["wa"], hpwl=wl["hpwl"], ovfl_bot=ob, ovfl_top=ot, ovfl_hbt=oh,
                   lam=st.lam.copy(), energy=[p["energy"] for p in parts])
    st.v_prev, st.g_prev = st.v, g
    st.u, st.v, st.a = u_new, v_new, a_new
    st.lam = st.lam * lay.ramp
    st.it += 1
    return metrics
