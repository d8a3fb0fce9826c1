"""Seeded synthetic netlists shaped like the paper's 3D mixed-size placement workloads.

This module only draws inputs: instance sizes on both dies, nets and their pins, pin offsets and
the initial placement.  It holds none of the placement method's arithmetic, so the oracle and the
HIP path can both read its output.  Every array uses the layouts the C ABI takes:

* ``size``    float32 [4][n]  (w_bot, h_bot, w_top, h_top), instance extents on each die
* ``kind``    uint8   [n]     bit 0 = macro, bit 1 = fixed, bit 2 = filler, bit 3 = z held
* ``net_start`` int32 [m+1]   net -> pin CSR, pins sorted by net
* ``pin2node``  int32 [P]     owning instance of each pin
* ``pin_off``   float32 [4][P] (ox_bot, oy_bot, ox_top, oy_top), pin offset from the instance centre
* ``xyz0``      float32 [3][n] initial instance centres

Units: one bottom-die site and row are one length unit.  The top die scales every width, height
and pin offset by 0.7 (a heterogeneous stack, Sec. II-B).  The ICCAD-2023 contest cases and the
RISC-V designs the paper measures on are not available; these netlists stand in for them, with the
instance counts, net-degree laws, macro mixes and grid sizes of the five workload configurations.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

KIND_CELL = 0
KIND_MACRO = 1
KIND_FIXED = 2
KIND_FIXED_MACRO = KIND_MACRO | KIND_FIXED
KIND_FILLER = 4          # dummy filler (no pins)
KIND_ZFIXED = 8          # z held at its start

TOP_SCALE = 0.7          # top-die size and pin-offset scale
WINDOW = 256             # index half-window of a local net
MACRO_PIN_PROB = 0.02    # chance that a net swaps one member for a macro


@dataclass(frozen=True)
class Config:
    name: str
    n_cells: int
    n_nets: int
    die: float
    nx: int
    ny: int
    nz: int
    degree: tuple            # ("geo", q, dmax) or ("mix", tail_weight, dmax)
    macros: tuple            # ("fixed4", frac) | ("uniform", n, lo, hi) | ("zipf", n, a1, expo)
    gamma_bins: float = 2.0  # WA smoothing in bin widths
    lambda_ramp: float = 1.05
    target_density: float = 1.0
    # technology constants of the synthetic stack (HBT pitch, row heights, HBT cost, alpha_0)
    hbt_pitch: float = 1.0
    row_bot: float = 1.0
    row_top: float = 0.7
    beta: float = 10.0
    alpha0: float = 3.5e-3
    local_fraction: float = 0.9  # share of nets drawn from an index window (0: every net uniform)


CONFIGS = {
    "c1": Config("c1", 2_000, 2_200, 200.0, 64, 64, 2, ("geo", 0.7733, 6), ("fixed4", 0.03)),
    "c2": Config("c2", 200_000, 220_000, 2000.0, 512, 512, 4, ("geo", 0.621, 20),
                 ("uniform", 40, 0.005, 0.02)),
    "c4": Config("c4", 1_200_000, 1_300_000, 4000.0, 1024, 1024, 4, ("mix", 0.0455, 50),
                 ("zipf", 150, 0.01, 0.6327)),
    "c5": Config("c5", 4_000_000, 4_400_000, 8000.0, 2048, 2048, 4, ("mix", 0.0346, 100),
                 ("zipf", 200, 0.05, 1.3528)),
}
# the 1.2M-cell netlist with every net drawn uniformly: no index locality, the worst case for the
# position gathers
CONFIGS["c4u"] = dataclasses.replace(CONFIGS["c4"], name="c4u", local_fraction=0.0)


@dataclass
class Case:
    config: Config
    seed: int
    die_x: float
    die_y: float
    nx: int
    ny: int
    nz: int
    size: np.ndarray
    kind: np.ndarray
    net_start: np.ndarray
    pin2node: np.ndarray
    pin_off: np.ndarray
    xyz0: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_inst(self) -> int:
        return int(self.kind.shape[0])

    @property
    def n_pins(self) -> int:
        return int(self.pin2node.shape[0])

    @property
    def n_nets(self) -> int:
        return int(self.net_start.shape[0] - 1)

    @property
    def gamma(self) -> float:
        return self.config.gamma_bins * self.die_x / self.nx


def _degree_law(rng, spec, m):
    kind = spec[0]
    if kind == "geo":
        q, dmax = spec[1], spec[2]
        d = np.arange(2, dmax + 1)
        p = q ** (d - 2.0)
        return rng.choice(d, size=m, p=p / p.sum())
    if kind == "mix":
        tail_w, dmax = spec[1], spec[2]
        d = np.arange(2, dmax + 1)
        p = 0.5 ** (d - 2.0)
        body = rng.choice(d, size=m, p=p / p.sum())
        t = np.arange(7, dmax + 1)
        pt = t ** -2.5
        tail = rng.choice(t, size=m, p=pt / pt.sum())
        return np.where(rng.random(m) < tail_w, tail, body)
    raise ValueError(spec)


def _macro_areas(rng, spec, die_area):
    kind = spec[0]
    if kind == "fixed4":
        return np.full(4, spec[1] * die_area)
    if kind == "uniform":
        return rng.uniform(spec[2], spec[3], size=spec[1]) * die_area
    if kind == "zipf":
        k = np.arange(1, spec[1] + 1, dtype=np.float64)
        return spec[2] * k ** -spec[3] * die_area
    raise ValueError(spec)


def _draw_members(rng, anchors, local, d, n_cells):
    """Distinct cell members for nets of one degree d (rows), by redrawing rows with repeats."""
    ne = anchors.shape[0]
    width = min(2 * WINDOW + 1, n_cells)
    lo = np.clip(anchors - WINDOW, 0, n_cells - width)
    out = np.empty((ne, d), dtype=np.int64)
    todo = np.arange(ne)
    while todo.size:
        loc = local[todo]
        draw = np.where(loc[:, None],
                        lo[todo, None] + rng.integers(0, width, size=(todo.size, d)),
                        rng.integers(0, n_cells, size=(todo.size, d)))
        out[todo] = draw
        srt = np.sort(draw, axis=1)
        dup = (srt[:, 1:] == srt[:, :-1]).any(axis=1)
        todo = todo[dup]
    return out


def make_case(name: str = "c1", seed: int = 2403, config: Config | None = None) -> Case:
    """Draw one synthetic placement instance.  Same (config, seed) -> same bytes."""
    cfg = config if config is not None else CONFIGS[name]
    rng = np.random.Generator(np.random.PCG64(seed))
    die_x = die_y = float(cfg.die)
    wb = die_x / cfg.nx
    hb = die_y / cfg.ny
    dz = cfg.nz * 0.5 * (wb + hb)

    # ---- instances: movable cells, then macros (movable, or fixed for the small case) ----
    nc = cfg.n_cells
    w_cell = rng.integers(1, 5, size=nc).astype(np.float64)
    h_cell = np.ones(nc)
    areas = _macro_areas(rng, cfg.macros, die_x * die_y)
    nm = areas.shape[0]
    aspect = rng.uniform(0.5, 2.0, size=nm)
    w_mac = np.sqrt(areas * aspect)
    h_mac = np.sqrt(areas / aspect)
    fixed_macros = cfg.macros[0] == "fixed4"
    n = nc + nm
    size = np.empty((4, n), dtype=np.float64)
    size[0, :nc], size[1, :nc] = w_cell, h_cell
    size[0, nc:], size[1, nc:] = w_mac, h_mac
    size[2] = TOP_SCALE * size[0]
    size[3] = TOP_SCALE * size[1]
    kind = np.zeros(n, dtype=np.uint8)
    kind[nc:] = KIND_FIXED_MACRO if fixed_macros else KIND_MACRO

    # ---- initial placement: x, y uniform with the (bottom-die) extent inside; z uniform ----
    xyz0 = np.empty((3, n), dtype=np.float64)
    xyz0[0] = size[0] / 2 + rng.random(n) * (die_x - size[0])
    xyz0[1] = size[1] / 2 + rng.random(n) * (die_y - size[1])
    xyz0[2] = dz / 4 + rng.random(n) * (dz / 2)
    if fixed_macros:
        # two fixed macros per die, on opposite diagonals (bottom, bottom, top, top)
        cx = np.array([0.25, 0.75, 0.75, 0.25]) * die_x
        cy = np.array([0.25, 0.75, 0.25, 0.75]) * die_y
        top = np.array([0, 0, 1, 1], dtype=bool)
        xyz0[0, nc:] = cx
        xyz0[1, nc:] = cy
        xyz0[2, nc:] = np.where(top, 0.75 * dz, 0.25 * dz)

    # ---- nets: degree law, index-local or uniform members, a few macro pins ----
    m = cfg.n_nets
    deg = _degree_law(rng, cfg.degree, m).astype(np.int64)
    anchors = rng.integers(0, nc, size=m)
    local = rng.random(m) < cfg.local_fraction
    members = [None] * m
    by_deg = {}
    for d in np.unique(deg):
        idx = np.nonzero(deg == d)[0]
        by_deg[int(d)] = (idx, _draw_members(rng, anchors[idx], local[idx], int(d), nc))
    swap = rng.random(m) < MACRO_PIN_PROB
    perim = w_mac + h_mac
    macro_pick = nc + rng.choice(nm, size=m, p=perim / perim.sum())
    swap_slot = rng.random(m)
    # nets are laid out in anchor order, the natural locality of a synthesised netlist
    order = np.argsort(anchors, kind="stable")
    rank = np.empty(m, dtype=np.int64)
    rank[order] = np.arange(m)
    deg_sorted = deg[order]
    net_start = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(deg_sorted, out=net_start[1:])
    P = int(net_start[-1])
    pin2node = np.empty(P, dtype=np.int64)
    for d, (idx, mem) in by_deg.items():
        mem = mem.copy()
        s = swap[idx]
        slot = np.minimum((swap_slot[idx] * d).astype(np.int64), d - 1)
        mem[s, slot[s]] = macro_pick[idx][s]
        starts = net_start[rank[idx]]
        pin2node[(starts[:, None] + np.arange(d)[None, :]).ravel()] = mem.ravel()

    # ---- pin offsets: uniform inside the bottom-die extent, scaled on the top die ----
    wn = size[0, pin2node]
    hn = size[1, pin2node]
    pin_off = np.empty((4, P), dtype=np.float64)
    pin_off[0] = (rng.random(P) - 0.5) * wn
    pin_off[1] = (rng.random(P) - 0.5) * hn
    pin_off[2] = TOP_SCALE * pin_off[0]
    pin_off[3] = TOP_SCALE * pin_off[1]

    return Case(
        config=cfg, seed=seed, die_x=die_x, die_y=die_y, nx=cfg.nx, ny=cfg.ny, nz=cfg.nz,
        size=size.astype(np.float32), kind=kind,
        net_start=net_start.astype(np.int32), pin2node=pin2node.astype(np.int32),
        pin_off=pin_off.astype(np.float32), xyz0=xyz0.astype(np.float32),
        meta={"n_cells": nc, "n_macros": nm},
    )


def small_config(n_cells=300, n_nets=330, die=100.0, nx=16, ny=16, nz=2, macros=("uniform", 3, 0.01, 0.03),
                 degree=("geo", 0.6, 8), name="tiny") -> Config:
    """A tiny configuration for brute-force and finite-difference tests."""
    return Config(name, n_cells, n_nets, die, nx, ny, nz, degree, macros)


def centre_start(case: Case, sigma: float = 0.02, seed: int = 1) -> Case:
    """The case with its movable instances re-drawn around the centre of the region: x and y
    normal with standard deviation sigma times the die side, z normal around the mid-plane with
    standard deviation 0.05 d_z (the usual start of a global placement from scratch)."""
    import dataclasses
    rng = np.random.Generator(np.random.PCG64(seed))
    dz = case.nz * 0.5 * (case.die_x / case.nx + case.die_y / case.ny)
    xyz = case.xyz0.astype(np.float64).copy()
    mov = (case.kind & KIND_FIXED) == 0
    k = int(mov.sum())
    xyz[0, mov] = case.die_x * (0.5 + sigma * rng.standard_normal(k))
    xyz[1, mov] = case.die_y * (0.5 + sigma * rng.standard_normal(k))
    xyz[2, mov] = dz * (0.5 + 0.05 * rng.standard_normal(k))
    return dataclasses.replace(case, xyz0=xyz.astype(np.float32))


def with_fillers(case: Case, plan: dict, sigma: float = 0.02, seed: int = 2) -> Case:
    """The case with fillers appended after its instances, as a filler plan describes them
    (counts n_top, n_bot, n_free and square sides side_top, side_bot, side_free): z-fixed top
    fillers at z = 3 d_z/4, z-fixed bottom fillers at z = d_z/4, free fillers around the
    mid-plane; x and y of all of them normal around the centre (sigma times the die side).
    Fillers have no pins; the netlist is unchanged."""
    import dataclasses
    rng = np.random.Generator(np.random.PCG64(seed))
    dz = case.nz * 0.5 * (case.die_x / case.nx + case.die_y / case.ny)
    groups = [(int(plan["n_top"]), float(plan["side_top"]), KIND_FILLER | KIND_ZFIXED, 0.75),
              (int(plan["n_bot"]), float(plan["side_bot"]), KIND_FILLER | KIND_ZFIXED, 0.25),
              (int(plan["n_free"]), float(plan["side_free"]), KIND_FILLER, None)]
    sizes, kinds, xyzs = [case.size.astype(np.float64)], [case.kind], [case.xyz0.astype(np.float64)]
    for k, side, kd, zf in groups:
        if k <= 0:
            continue
        sizes.append(np.full((4, k), side))
        kinds.append(np.full(k, kd, dtype=np.uint8))
        xyz = np.empty((3, k))
        xyz[0] = case.die_x * (0.5 + sigma * rng.standard_normal(k))
        xyz[1] = case.die_y * (0.5 + sigma * rng.standard_normal(k))
        xyz[2] = zf * dz if zf is not None else dz * (0.5 + 0.05 * rng.standard_normal(k))
        xyzs.append(xyz)
    meta = dict(case.meta)
    meta.update(n_fillers=sum(max(g[0], 0) for g in groups), filler_plan=dict(plan))
    return dataclasses.replace(case, size=np.concatenate(sizes, axis=1).astype(np.float32),
                               kind=np.concatenate(kinds), xyz0=np.concatenate(xyzs, axis=1).astype(np.float32),
                               meta=meta)
