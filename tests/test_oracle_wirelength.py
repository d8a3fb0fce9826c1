"""Pins of the oracle's WA model, bistratal wirelength and FDA z-gradient."""
import os

import numpy as np
import pytest

from oracle import wirelength as wl
from oracle.geometry import Geometry, geometry_of
from oracle.optimizer import problem_of
from paper_2403_09070_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- WA model

@pytest.mark.parametrize("delta,gamma", [(1.0, 0.5), (3.0, 2.0), (40.0, 1.0), (0.01, 3.0)])
def test_wa_two_pin_closed_form(delta, gamma):
    u = np.array([[5.0, 5.0 + delta]])
    p, _ = wl.wa_extent(u, np.ones_like(u, dtype=bool), gamma)
    assert abs(p[0] - delta * np.tanh(delta / (2 * gamma))) < 1e-12 * max(1.0, delta)


def test_wa_is_between_zero_and_hpwl_and_within_derived_bound():
    # each non-extreme pin adds at most max_t t e^{-t/gamma} = gamma/e to each side
    rng = np.random.default_rng(0)
    for d in (2, 3, 5, 9, 20):
        u = rng.uniform(0, 100, size=(4000, d))
        mask = np.ones_like(u, dtype=bool)
        for gamma in (8.0, 1.0, 0.1):
            p, _ = wl.wa_extent(u, mask, gamma)
            hp = u.max(1) - u.min(1)
            assert np.all(p >= -1e-12) and np.all(p <= hp + 1e-12)
            assert np.all(hp - p <= 2 * (d - 1) * gamma / np.e + 1e-9)


def test_wa_tends_to_hpwl_as_gamma_goes_to_zero():
    rng = np.random.default_rng(1)
    u = rng.uniform(0, 50, size=(200, 6))
    mask = np.ones_like(u, dtype=bool)
    hp = u.max(1) - u.min(1)
    prev = None
    for k in range(0, 15):
        gamma = 2.0 ** -k * 4.0
        err = np.abs(wl.wa_extent(u, mask, gamma)[0] - hp).max()
        assert err <= 2 * 5 * gamma / np.e + 1e-9
        if prev is not None:
            assert err <= prev + 1e-12
        prev = err
    assert prev < 1e-3


def test_wa_gradient_matches_central_differences_and_sums_to_zero():
    rng = np.random.default_rng(2)
    u = rng.uniform(0, 20, size=(50, 5))
    mask = rng.random((50, 5)) < 0.8
    mask[:, 0] = True
    gamma = 1.7
    p, g = wl.wa_extent(u, mask, gamma)
    np.testing.assert_allclose(g.sum(axis=1), 0.0, atol=1e-12)     # translation invariance
    h = 1e-6
    for k in range(5):
        e = np.zeros_like(u)
        e[:, k] = h
        fd = (wl.wa_extent(u + e, mask, gamma)[0] - wl.wa_extent(u - e, mask, gamma)[0]) / (2 * h)
        np.testing.assert_allclose(g[:, k], np.where(mask[:, k], fd, 0.0), atol=1e-7)


def test_wa_empty_and_single_pin_sets_are_zero():
    u = np.array([[3.0, 7.0], [1.0, 2.0]])
    mask = np.array([[False, False], [True, False]])
    p, g = wl.wa_extent(u, mask, 1.0)
    assert list(p) == [0.0, 0.0] and np.all(g == 0.0)


# ----------------------------------------------------------------------------- bistratal model

def _hbt_brute_force(u, top):
    """min over HBT positions t of the x-extents of the top and bottom nets with t added."""
    best = np.inf
    cand = np.concatenate([u, 0.5 * (u[:, None] + u[None, :]).ravel()])
    for t in cand:
        ut = np.append(u[top], t)
        ub = np.append(u[~top], t)
        best = min(best, ut.max() - ut.min() + ub.max() - ub.min())
    return best


def test_bistratal_equals_optimal_hbt_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(400):
        d = rng.integers(2, 9)
        u = rng.uniform(0, 10, size=d).round(1)
        top = rng.random(d) < 0.5
        if top.all() or (~top).all():
            top[0] = not top[0]
        got = wl.bistratal_exact(u[None], top[None])[0]
        assert abs(got - _hbt_brute_force(u, top)) < 1e-12


def test_one_die_net_reduces_to_planar_hpwl():
    rng = np.random.default_rng(4)
    u = rng.uniform(0, 10, size=(100, 6))
    for top in (np.ones_like(u, dtype=bool), np.zeros_like(u, dtype=bool)):
        np.testing.assert_allclose(wl.bistratal_exact(u, top), u.max(1) - u.min(1), atol=0)


def _read_figures():
    cases = {}
    for line in open(os.path.join(GOLD, "bistratal_figures.txt")):
        if not line.startswith("case"):
            continue
        head, top, bot, vals = [s.strip() for s in line.split(";")]
        pts = lambda s: np.array([[float(v) for v in p.split(",")] for p in s.split()])  # noqa: E731
        exp = {}
        for kv in vals.split():
            k, v = kv.split("=")
            exp[k] = [float(t) for t in v.split(",")] if "," in v else float(v)
        cases[head.split()[1]] = (pts(top), pts(bot), exp)
    return cases


def _axis(top_pts, bot_pts, a):
    u = np.concatenate([top_pts[:, a], bot_pts[:, a]])[None]
    top = np.concatenate([np.ones(len(top_pts), bool), np.zeros(len(bot_pts), bool)])[None]
    return u, top


@pytest.mark.parametrize("name", ["hpwl_a", "hpwl_b", "region_a", "region_b"])
def test_figure_wirelengths(name):
    tp, bp, exp = _read_figures()[name]
    ux, tx = _axis(tp, bp, 0)
    uy, _ = _axis(tp, bp, 1)
    assert wl.bistratal_exact(ux, tx)[0] == exp["wx"]
    if "wy" in exp:
        assert wl.bistratal_exact(uy, tx)[0] == exp["wy"]
        assert wl.bistratal_exact(ux, tx)[0] + wl.bistratal_exact(uy, tx)[0] == exp["wbi"]
    if "pe_x" in exp:
        assert wl.exact_extent(ux, np.ones_like(tx))[0] == exp["pe_x"]
    if "hbt_x_lo" in exp:
        # Eq. optimal-region: the HBT range bounded by the medians of the two boxes
        lo = min(max(tp[:, 0].min(), bp[:, 0].min()), min(tp[:, 0].max(), bp[:, 0].max()))
        hi = max(max(tp[:, 0].min(), bp[:, 0].min()), min(tp[:, 0].max(), bp[:, 0].max()))
        assert (lo, hi) == (exp["hbt_x_lo"], exp["hbt_x_hi"])
        for t in np.linspace(lo, hi, 5):       # any HBT position in the region attains W_x
            ut, ub = np.append(tp[:, 0], t), np.append(bp[:, 0], t)
            assert ut.max() - ut.min() + ub.max() - ub.min() == exp["wx"]


def _net_case(top_pts, bot_pts, dz=4.0):
    """One net whose pins are instance centres (zero offsets); top/bottom set by z."""
    pts = np.concatenate([top_pts, bot_pts])
    n = len(pts)
    z = np.concatenate([np.full(len(top_pts), 0.75 * dz), np.full(len(bot_pts), 0.25 * dz)])
    xyz = np.stack([pts[:, 0], pts[:, 1], z])
    size = np.ones((4, n))
    kind = np.zeros(n, dtype=np.uint8)
    return xyz, size, kind, np.array([0, n]), np.arange(n), np.zeros((4, n))


def test_incremental_figure_flip_and_fda_gradient():
    tp, bp, exp = _read_figures()["incre"]
    xyz, size, kind, ns, p2n, off = _net_case(tp, bp)
    geo = Geometry(100.0, 100.0, 10, 10, 2)   # d_z = 20
    xyz[2] = np.where(xyz[2] > 2.0, 0.75 * geo.dz, 0.25 * geo.dz)
    k = int(exp["move"])
    top = xyz[2] > geo.dz / 2
    moved = top.copy()
    moved[k] = False
    ux, uy = xyz[0][None], xyz[1][None]
    dwx = wl.bistratal_exact(ux, moved[None])[0] - wl.bistratal_exact(ux, top[None])[0]
    dwy = wl.bistratal_exact(uy, moved[None])[0] - wl.bistratal_exact(uy, top[None])[0]
    assert (dwx, dwy, dwx + dwy) == (exp["dwx"], exp["dwy"], exp["dwbi"])
    # the second-extreme box of the top net
    tx = np.sort(tp[:, 0])
    ty = np.sort(tp[:, 1])
    assert [tx[1], tx[-2]] == exp["b2_x"] and [ty[1], ty[-2]] == exp["b2_y"]
    # FDA for the moved pin's instance: (4/d_z) (W_top - W_bot), p4 sits on the top die
    out = wl.wirelength(size, kind, xyz, ns, p2n, off, geo, gamma=1.0, alpha=0.0)
    assert abs(out["fda"][k] - 4.0 / geo.dz * (-exp["dwbi"])) < 1e-12


def test_hpwl_figure_fda_gradient():
    tp, bp, _ = _read_figures()["hpwl_a"]
    xyz, size, kind, ns, p2n, off = _net_case(tp, bp)
    geo = Geometry(100.0, 100.0, 10, 10, 2)
    xyz[2] = np.where(xyz[2] > 2.0, 0.75 * geo.dz, 0.25 * geo.dz)
    out = wl.wirelength(size, kind, xyz, ns, p2n, off, geo, gamma=1.0, alpha=0.0)
    # p3 (index 1 here) on top: W with it on top 6.5, on the bottom 5 (Fig. hpwl-analysis)
    assert abs(out["fda"][1] - 4.0 / geo.dz * 1.5) < 1e-12


def _total_exact(c, xyz, geo):
    pb = problem_of(c)
    return wl.wirelength(pb.size, pb.kind, xyz, pb.net_start, pb.pin2node, pb.pin_off, geo,
                         pb.gamma, pb.alpha)["hpwl_d2d"]


def test_fda_equals_full_reevaluation_with_instance_on_each_die():
    """The step-function argument of Eqs. fda-deriv-*: FDA = (4/d_z)(W(3d_z/4) - W(d_z/4)) for
    any z in range, checked by recomputing the whole design's exact wirelength twice."""
    c = synth.make_case(config=synth.small_config(n_cells=120, n_nets=150), seed=3)
    geo = geometry_of(c)
    pb = problem_of(c)
    out = wl.wirelength(pb.size, pb.kind, c.xyz0, pb.net_start, pb.pin2node, pb.pin_off, geo,
                        pb.gamma, pb.alpha)
    rng = np.random.default_rng(0)
    for i in rng.choice(c.n_inst, size=25, replace=False):
        if c.kind[i] & 2:
            continue
        hi = c.xyz0.astype(np.float64).copy()
        lo = hi.copy()
        hi[2, i] = 0.75 * geo.dz
        lo[2, i] = 0.25 * geo.dz
        ref = 4.0 / geo.dz * (_total_exact(c, hi, geo) - _total_exact(c, lo, geo))
        assert abs(out["fda"][i] - ref) < 1e-9 * max(1.0, abs(ref))


def test_fda_moves_every_pin_of_an_instance_and_counts_it_once():
    """An instance with two pins on a net (Eq. fda-grad takes instances, not pins): A owns the
    pins at x = 0 and x = 10, B and C one pin each at x = 2 and x = 8, all on the bottom die, zero
    offsets.  With A on top the net splits into {0, 10} and {2, 8}: 10 + 6 = 16 > 10; with A on
    the bottom W = 10, so A's FDA is (4/d_z) 6 by hand.  Moving one of A's pins at a time would
    give 0 for each (W stays 10), so a per-pin reading fails here; B and C change nothing."""
    geo = Geometry(100.0, 100.0, 10, 10, 2)
    xyz = np.array([[50.0, 52.0, 58.0], [50.0, 50.0, 50.0], [0.25 * geo.dz] * 3])
    xyz[0] -= 50.0
    xyz[0] += 20.0                       # A at 20, B at 22, C at 28; A's pins at offsets 0 and 10
    size = np.ones((4, 3))
    kind = np.zeros(3, dtype=np.uint8)
    p2n = np.array([0, 0, 1, 2])
    off = np.zeros((4, 4))
    off[0, 1] = off[2, 1] = 10.0         # A's second pin 10 to the right on either die
    out = wl.wirelength(size, kind, xyz, np.array([0, 4]), p2n, off, geo, gamma=1.0, alpha=0.0)
    assert abs(out["fda"][0] - 4.0 / geo.dz * 6.0) < 1e-12
    assert out["fda"][1] == 0.0 and out["fda"][2] == 0.0
    assert out["hpwl_d2d"] == 10.0


def test_fda_with_shared_instances_equals_full_reevaluation():
    """The full re-evaluation of the design with each instance on either die, on a netlist where a
    third of the nets hold one instance twice (on different pins)."""
    c = synth.make_case(config=synth.small_config(n_cells=120, n_nets=150), seed=4)
    rng = np.random.default_rng(1)
    p2n = c.pin2node.copy()
    ns = c.net_start
    for e in range(len(ns) - 1):
        if ns[e + 1] - ns[e] >= 3 and rng.random() < 0.33:
            p2n[ns[e + 1] - 1] = p2n[ns[e]]          # the last pin goes to the first pin's owner
    import dataclasses
    c = dataclasses.replace(c, pin2node=p2n)
    geo = geometry_of(c)
    pb = problem_of(c)
    out = wl.wirelength(pb.size, pb.kind, c.xyz0, pb.net_start, pb.pin2node, pb.pin_off, geo,
                        pb.gamma, pb.alpha)
    shared = set()
    for e in range(len(ns) - 1):
        m = p2n[ns[e]:ns[e + 1]]
        if len(set(m.tolist())) < len(m):
            shared.update(m.tolist())
    assert len(shared) > 10
    for i in sorted(shared)[:20]:
        if c.kind[i] & 2:
            continue
        hi = c.xyz0.astype(np.float64).copy()
        lo = hi.copy()
        hi[2, i] = 0.75 * geo.dz
        lo[2, i] = 0.25 * geo.dz
        ref = 4.0 / geo.dz * (_total_exact(c, hi, geo) - _total_exact(c, lo, geo))
        assert abs(out["fda"][i] - ref) < 1e-9 * max(1.0, abs(ref))


def test_smoothed_bistratal_gradient_matches_central_differences():
    c = synth.make_case(config=synth.small_config(n_cells=150, n_nets=160), seed=8)
    geo = geometry_of(c)
    pb = problem_of(c)
    args = (pb.size, pb.kind)
    base = c.xyz0.astype(np.float64)
    out = wl.wirelength(*args, base, pb.net_start, pb.pin2node, pb.pin_off, geo, pb.gamma, pb.alpha)
    rng = np.random.default_rng(1)
    h = 1e-5
    checked = 0
    for i in rng.choice(c.meta["n_cells"], size=40, replace=False):
        for a, key in ((0, "grad_x"), (1, "grad_y")):
            up, dn = base.copy(), base.copy()
            up[a, i] += h
            dn[a, i] -= h
            f = lambda p: wl.wirelength(*args, p, pb.net_start, pb.pin2node, pb.pin_off, geo,  # noqa
                                        pb.gamma, pb.alpha)["wa_bi"]
            fd = (f(up) - f(dn)) / (2 * h)
            assert abs(out[key][i] - fd) < 1e-6 * max(1.0, abs(fd))
            checked += 1
        # z part of the WA cut model
        up, dn = base.copy(), base.copy()
        up[2, i] += h
        dn[2, i] -= h
        fz = lambda p: wl.wirelength(*args, p, pb.net_start, pb.pin2node, pb.pin_off, geo,  # noqa
                                     pb.gamma, pb.alpha)["wa_z"]
        if abs(base[2, i] - geo.dz / 2) > 10 * h:
            assert abs(out["grad_zwa"][i] - (fz(up) - fz(dn)) / (2 * h)) < 1e-6
    assert checked == 80


def test_fda_normalisation_scales_to_planar_l1_norm():
    c = synth.make_case(config=synth.small_config(), seed=4)
    pb = problem_of(c)
    out = wl.wirelength(pb.size, pb.kind, c.xyz0, pb.net_start, pb.pin2node, pb.pin_off,
                        geometry_of(c), pb.gamma, pb.alpha)
    g = out["fda_scale"] * out["fda"]
    np.testing.assert_allclose(np.abs(g).sum(), 0.5 * (np.abs(out["grad_x"]).sum()
                                                       + np.abs(out["grad_y"]).sum()), rtol=1e-12)
