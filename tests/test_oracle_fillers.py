"""Pins of the oracle's fillers (Sec. III-A density model, Eqs. filler-vol and free-filler-vol)."""
import math

import numpy as np
import pytest

from oracle import attributes as at
from oracle import density as den
from oracle import fillers as fl
from oracle import optimizer as opt
from oracle.geometry import geometry_of
from paper_2403_09070_amd import synth


def _tiny_two_cells():
    """Die 10 x 10, grid 10 x 10 x 2 (bin 1 x 1 x 1, d_z = 2); two cells of bottom size 1 x 1 and
    top size 0.5 x 0.5, one on each die."""
    size = np.array([[1.0, 1.0], [1.0, 1.0], [0.5, 0.5], [0.5, 0.5]])
    kind = np.zeros(2, np.uint8)
    z0 = np.array([0.5, 1.5])
    return size, kind, z0


def test_plan_of_a_hand_worked_case():
    """By hand: vol_f^+ = 1/2 * 200 * (1 - 0.5) = 50, vol_f^- = 1/2 * 200 * (1 - 0.8) = 20,
    vol_a = 1 * 1 * 1 + 0.25 * 1 = 1.25, vol_fr = 200 - 71.25 = 128.75; filler areas 0.25 (top),
    1 (bottom), 0.625 (free), depth 1: counts 200, 20, 206."""
    size, kind, z0 = _tiny_two_cells()
    p = fl.filler_plan(size, kind, z0, 10.0, 10.0, 2.0, u_top=0.5, u_bot=0.8)
    assert (p["n_top"], p["n_bot"], p["n_free"]) == (200, 20, 206)
    for key, val in (("vol_top", 50.0), ("vol_bot", 20.0), ("vol_a", 1.25), ("vol_free", 128.75),
                     ("side_top", 0.5), ("side_bot", 1.0), ("side_free", math.sqrt(0.625))):
        assert abs(p[key] - val) <= 1e-14 * val, key


def test_volumes_fill_the_region():
    """With no clipping, z-fixed, free and instance volumes add up to the region's volume; when
    the instances alone exceed the region left by the z-fixed fillers there are no free fillers."""
    c = synth.make_case("c1", 2403)
    geo = geometry_of(c)
    for u_top, u_bot in ((0.8, 0.8), (0.6, 0.9), (1.0, 1.0)):
        p = fl.filler_plan(c.size, c.kind, c.xyz0[2], geo.die_x, geo.die_y, geo.dz, u_top, u_bot)
        total = geo.die_x * geo.die_y * geo.dz
        assert abs(p["vol_top"] + p["vol_bot"] + p["vol_free"] + p["vol_a"] - total) < 1e-9 * total
        for key, side in (("top", "side_top"), ("bot", "side_bot"), ("free", "side_free")):
            one = p[side] ** 2 * 0.5 * geo.dz
            assert abs(p["n_" + key] * one - p["vol_" + key]) <= 0.5 * one + 1e-9
    p = fl.filler_plan(c.size, c.kind, c.xyz0[2], geo.die_x, geo.die_y, geo.dz, 0.0, 0.0)
    assert p["vol_free"] == 0.0 and p["n_free"] == 0


def _with_fillers(case, u=0.8, seed=3):
    geo = geometry_of(case)
    p = fl.filler_plan(case.size, case.kind, case.xyz0[2], geo.die_x, geo.die_y, geo.dz, u, u)
    return synth.with_fillers(case, p, seed=seed), p


def test_fillers_add_their_volume_to_the_map():
    """The fillers (started near the centre, so none is clipped by the region) add exactly their
    volume to the map."""
    c = synth.make_case(config=synth.small_config(n_cells=200, n_nets=220), seed=4)
    cf, p = _with_fillers(c)
    geo = geometry_of(cf)
    fill = at.is_filler(cf.kind)
    assert int(fill.sum()) == p["n_top"] + p["n_bot"] + p["n_free"]
    added = (den.density_map(cf.size, cf.kind, cf.xyz0, geo) - den.density_map(c.size, c.kind, c.xyz0, geo)).sum()
    w, h = at.instance_size(cf.size[:, fill], cf.kind[fill], cf.xyz0[2, fill].astype(np.float64), geo.dz)
    q = at.charge(w, h, geo.dz)
    assert abs(added * geo.vol_bin - q.sum()) < 1e-9 * q.sum()


def test_overflow_ignores_fillers():
    """Adding fillers changes the density map but not the overflow measured on the real instances
    at the same positions."""
    c = synth.make_case(config=synth.small_config(n_cells=200, n_nets=220), seed=4)
    cf, _ = _with_fillers(c)
    pb, pbf = opt.problem_of(c), opt.problem_of(cf)
    v, vf = opt.clamp(pb, c.xyz0), opt.clamp(pbf, cf.xyz0)
    rho = den.density_map(c.size, c.kind, v, pb.geo)
    rhof = den.density_map(cf.size, cf.kind, vf, pbf.geo)
    assert np.abs(rhof - rho).max() > 0.1
    assert opt.overflow(pbf, rhof, vf) == pytest.approx(opt.overflow(pb, rho, v), rel=1e-12, abs=1e-15)


def test_z_fixed_fillers_keep_their_z():
    c = synth.make_case(config=synth.small_config(n_cells=200, n_nets=220), seed=4)
    cf, _ = _with_fillers(c)
    pb = opt.problem_of(cf)
    held = at.is_zfixed(cf.kind)
    free = at.is_filler(cf.kind) & ~held
    assert held.any() and free.any()
    st = opt.gp_init(pb, cf.xyz0)
    z0 = st.v[2, held].copy()
    assert np.all(st.g_prev[2, held] == 0.0)
    xy0 = st.v[:2, held].copy()
    zf0 = st.v[2, free].copy()
    for _ in range(3):
        opt.gp_step(pb, st)
    assert np.array_equal(st.v[2, held], z0) and np.array_equal(st.u[2, held], z0)
    assert np.abs(st.v[:2, held] - xy0).max() > 0.0
    assert np.abs(st.v[2, free] - zf0).max() > 0.0
