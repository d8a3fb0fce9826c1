"""Pins of the multi-die 2D oracle (Sec. III-C, Eq. 2d-place): 2D density, 2D cosine solve,
partial-net wirelength with HBT nodes, fillers, the 2D optimiser."""
import math
import os

import numpy as np
import pytest

from oracle import multidie as md
from oracle import optimizer as opt
from oracle import wirelength as owl
from paper_2403_09070_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _grid(n=16, die=100.0):
    return md.Grid2D(die, die, n, n)


@pytest.mark.parametrize("jk", [(1, 0), (0, 3), (2, 5), (7, 7)])
def test_single_cosine_mode_closed_form_2d(jk):
    """rho = cos(w_j x) cos(w_k y) at bin centres: phi = rho / (w_j^2 + w_k^2) and
    E_x = w_j/|w|^2 sin(w_j x) cos(w_k y), E_y likewise, exactly."""
    g = md.Grid2D(80.0, 60.0, 16, 12)
    j, k = jk
    x = (np.arange(g.nx) + 0.5) * g.wb
    y = (np.arange(g.ny) + 0.5) * g.hb
    wj, wk = j * math.pi / g.die_x, k * math.pi / g.die_y
    rho = np.cos(wk * y)[:, None] * np.cos(wj * x)[None, :]
    sol = md.solve_2d(rho, g)
    w2 = wj * wj + wk * wk
    np.testing.assert_allclose(sol["phi"], rho / w2, atol=1e-12 / w2)
    np.testing.assert_allclose(sol["ex"], wj / w2 * np.cos(wk * y)[:, None] * np.sin(wj * x)[None, :], atol=1e-12)
    np.testing.assert_allclose(sol["ey"], wk / w2 * np.sin(wk * y)[:, None] * np.cos(wj * x)[None, :], atol=1e-12)


def test_density_2d_matches_brute_force_and_conserves_area():
    g = md.Grid2D(40.0, 30.0, 8, 6)
    rng = np.random.default_rng(1)
    n = 60
    w = rng.uniform(0.5, 12.0, n)
    h = rng.uniform(0.5, 9.0, n)
    xy = np.stack([rng.uniform(0, g.die_x, n), rng.uniform(0, g.die_y, n)])
    rho = md.density_2d(w, h, xy, g)
    ref = np.zeros((g.ny, g.nx))
    r2 = math.sqrt(2.0)
    for i in range(n):
        wt, ht = max(w[i], r2 * g.wb), max(h[i], r2 * g.hb)
        om = min(1.0, w[i] / (r2 * g.wb)) * min(1.0, h[i] / (r2 * g.hb))
        x0, x1 = max(xy[0, i] - wt / 2, 0.0), min(xy[0, i] + wt / 2, g.die_x)
        y0, y1 = max(xy[1, i] - ht / 2, 0.0), min(xy[1, i] + ht / 2, g.die_y)
        for by in range(g.ny):
            for bx in range(g.nx):
                lx = max(0.0, min(x1, (bx + 1) * g.wb) - max(x0, bx * g.wb))
                ly = max(0.0, min(y1, (by + 1) * g.hb) - max(y0, by * g.hb))
                ref[by, bx] += om * lx * ly / g.area_bin
    np.testing.assert_allclose(rho, ref, atol=1e-12)
    inside = ((xy[0] - np.maximum(w, r2 * g.wb) / 2 >= 0) & (xy[0] + np.maximum(w, r2 * g.wb) / 2 <= g.die_x)
              & (xy[1] - np.maximum(h, r2 * g.hb) / 2 >= 0) & (xy[1] + np.maximum(h, r2 * g.hb) / 2 <= g.die_y))
    rho_in = md.density_2d(w[inside], h[inside], xy[:, inside], g)
    assert abs(rho_in.sum() * g.area_bin - float(np.sum(w[inside] * h[inside]))) < 1e-9 * float(np.sum(w * h))


def _read_figures():
    cases = {}
    for line in open(os.path.join(GOLD, "bistratal_figures.txt")):
        if not line.startswith("case"):
            continue
        head, top, bot, vals = [s.strip() for s in line.split(";")]
        pts = lambda s: [tuple(float(v) for v in p.split(",")) for p in s.split()]  # noqa: E731
        exp = dict(kv.split("=") for kv in vals.split())
        cases[head.split()[1]] = (pts(top), pts(bot), exp)
    return cases


@pytest.mark.parametrize("name", ["hpwl_a", "hpwl_b", "region_a", "region_b"])
def test_hbt_in_its_optimal_region_gives_the_bistratal_wirelength(name):
    """Eqs. optimal-region and wl-obj: with the HBT started in its optimal region, the two partial
    nets' HPWL equals the bistratal wirelength the figures give (W_x; W_y where printed)."""
    top, bot, exp = _read_figures()[name]
    pts = top + bot
    n = len(pts)
    dz = 4.0
    xyz = np.array([[p[0] for p in pts], [p[1] for p in pts],
                    [0.75 * dz] * len(top) + [0.25 * dz] * len(bot)])
    size = np.ones((4, n))
    lay, xy0 = md.split(size, np.zeros(n, np.uint8), xyz, np.array([0, n]), np.arange(n), np.zeros((4, n)), dz,
                        _grid(), gamma=1.0, hbt_side=1.0)
    assert lay.n_hbt == 1 and len(lay.net_start) == 3
    lo, hi = md.optimal_hbt_interval([p[0] for p in top], [p[0] for p in bot])
    if "hbt_x_lo" in exp:
        assert (lo, hi) == (float(exp["hbt_x_lo"]), float(exp["hbt_x_hi"]))
    ns = lay.net_start
    p2n = lay.pin2node
    wx = sum(np.ptp(xy0[0, p2n[ns[k]:ns[k + 1]]]) for k in range(2))
    assert wx == float(exp["wx"])
    if "wy" in exp:
        wy = sum(np.ptp(xy0[1, p2n[ns[k]:ns[k + 1]]]) for k in range(2))
        assert wy == float(exp["wy"])


def test_start_partial_net_hpwl_equals_the_3d_bistratal_wirelength():
    """On a whole netlist (C1): the 2D start's exact partial-net HPWL equals the 3D oracle's D2D
    HPWL of the same placement, net by net summed (every HBT in its optimal region)."""
    case = synth.make_case("c1", 2403)
    pb = opt.problem_of(case)
    v = case.xyz0.astype(np.float64)
    lay, xy0 = md.split(case.size, case.kind, v, case.net_start, case.pin2node, case.pin_off, pb.geo.dz,
                        md.Grid2D(case.die_x, case.die_y, case.nx, case.ny), pb.gamma, hbt_side=1.0)
    w3 = owl.wirelength(pb.size, pb.kind, v, pb.net_start, pb.pin2node, pb.pin_off, pb.geo, pb.gamma, pb.alpha)
    w2 = md.wirelength_2d(lay, xy0)
    assert abs(w2["hpwl"] - w3["hpwl_d2d"]) <= 1e-12 * w3["hpwl_d2d"]
    assert lay.n_hbt == w3["ncut"]


def test_partial_net_wa_gradient_matches_central_differences():
    case = synth.make_case(config=synth.small_config(n_cells=120, n_nets=140), seed=3)
    pb = opt.problem_of(case)
    lay, xy0 = md.split(case.size, case.kind, case.xyz0, case.net_start, case.pin2node, case.pin_off, pb.geo.dz,
                        md.Grid2D(case.die_x, case.die_y, case.nx, case.ny), pb.gamma, hbt_side=1.0)
    g = md.wirelength_2d(lay, xy0)["grad"]
    rng = np.random.default_rng(0)
    h = 1e-5
    movable = np.nonzero(lay.movable)[0]
    for i in rng.choice(movable, size=40, replace=False):
        for a in range(2):
            p, m = xy0.copy(), xy0.copy()
            p[a, i] += h
            m[a, i] -= h
            fd = (md.wirelength_2d(lay, p)["wa"] - md.wirelength_2d(lay, m)["wa"]) / (2 * h)
            assert abs(g[a, i] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, a, g[a, i], fd)
    # translation invariance: every partial net's gradient sums to zero
    assert abs(g[0].sum()) < 1e-9 * np.abs(g[0]).sum() and abs(g[1].sum()) < 1e-9 * np.abs(g[1]).sum()


def test_fillers_take_up_the_free_area_of_each_layer():
    case = synth.make_case("c1", 2403)
    pb = opt.problem_of(case)
    grid = md.Grid2D(case.die_x, case.die_y, case.nx, case.ny)
    lay, xy0 = md.split(case.size, case.kind, case.xyz0, case.net_start, case.pin2node, case.pin_off, pb.geo.dz,
                        grid, pb.gamma, hbt_side=1.0)
    plan = md.filler_plan(lay)
    full, xy = md.with_fillers(lay, xy0, plan, seed=1)
    for L, (count, side) in zip((md.BOTTOM, md.TOP, md.HBT), plan):
        on = full.layer == L
        area = float(np.sum(full.w[on] * full.h[on]))
        assert abs(area - grid.die_x * grid.die_y) <= 0.5 * side * side
    assert np.all(xy[0] >= 0) and np.all(xy[0] <= grid.die_x)


def test_field_gather_2d_agrees_with_the_energy_gradient_under_refinement():
    """The 2D field gather approaches the gradient of the 2D energy (central differences) as the
    grid refines, and points the same way."""
    rng = np.random.default_rng(2)
    n = 40                                  # instances of several bins: a smooth field to resolve
    w = rng.uniform(6, 14, n)
    h = rng.uniform(6, 14, n)
    xy = np.stack([rng.uniform(15, 85, n), rng.uniform(15, 85, n)])
    kind = np.zeros(n, np.uint8)
    errs = []
    for k in (16, 32, 64):
        g = _grid(k)
        rho = md.density_2d(w, h, xy, g)
        sol = md.solve_2d(rho, g)
        gf = md.field_gather_2d(w, h, kind, xy, sol["ex"], sol["ey"], g)
        fd = np.zeros((2, 20))
        for t in range(20):
            for a in range(2):
                p, m = xy.copy(), xy.copy()
                p[a, t] += 1e-4
                m[a, t] -= 1e-4
                ep = md.energy_2d(md.density_2d(w, h, p, g), md.solve_2d(md.density_2d(w, h, p, g), g)["phi"], g)
                em = md.energy_2d(md.density_2d(w, h, m, g), md.solve_2d(md.density_2d(w, h, m, g), g)["phi"], g)
                fd[a, t] = (ep - em) / 2e-4
        assert float(np.sum(gf[:, :20] * fd)) > 0
        errs.append(np.linalg.norm(gf[:, :20] - fd) / np.linalg.norm(fd))
    assert errs[2] < errs[0], errs


def test_2d_overflow_of_a_hand_worked_layer():
    """Bottom layer: two 2 x 2 squares stacked on a 4 x 4 grid of unit bins: 4 bins at rho = 2 ->
    excess 4 over area 8 -> 0.5; the top layer one square, 0; the HBT layer is empty, 0."""
    g = md.Grid2D(4.0, 4.0, 4, 4)
    lay = md.Layered(w=np.array([2.0, 2.0, 2.0]), h=np.array([2.0, 2.0, 2.0]), kind=np.zeros(3, np.uint8),
                     layer=np.array([md.BOTTOM, md.BOTTOM, md.TOP]), net_start=np.array([0]),
                     pin2node=np.zeros(0, np.int64), pin_off=np.zeros((2, 0)), grid=g, gamma=1.0, ramp=1.05,
                     target=1.0, n_inst=3, n_hbt=0)
    xy = np.array([[1.0, 1.0, 3.0], [1.0, 1.0, 3.0]])
    assert md.overflow_2d(lay, xy) == (0.5, 0.0, 0.0)


def test_2d_gp_reduces_overflow_and_keeps_hbt_partial_nets_finite():
    case = synth.make_case("c1", 2403)
    pb = opt.problem_of(case)
    grid = md.Grid2D(case.die_x, case.die_y, case.nx, case.ny)
    lay, xy0 = md.split(case.size, case.kind, case.xyz0, case.net_start, case.pin2node, case.pin_off, pb.geo.dz,
                        grid, pb.gamma, hbt_side=1.0)
    st = md.gp_init_2d(lay, xy0)
    assert np.all(st.lam > 0)
    ms = [md.gp_step_2d(lay, st) for _ in range(8)]
    assert ms[-1]["ovfl_bot"] < ms[0]["ovfl_bot"] and ms[-1]["ovfl_top"] < ms[0]["ovfl_top"]
    assert all(np.isfinite(m["hpwl"]) for m in ms)
    np.testing.assert_allclose(st.lam, ms[0]["lam"] * lay.ramp ** 8)
