"""Pins of the oracle's density map and attribute model against what the paper fixes."""
import os

import numpy as np
import pytest

from oracle import attributes as at
from oracle import density as den
from oracle.geometry import Geometry, geometry_of, hbt_alpha
from paper_2403_09070_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_prefix_example():
    rho, corner = {}, {}
    for line in open(os.path.join(GOLD, "prefix_example_2d.txt")):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "macro":
            macro = tuple(float(v) for v in f[1:])
        elif f[0] == "grid":
            grid = (int(f[1]), int(f[2]))
        elif f[0] == "rho":
            rho[(int(f[1]), int(f[2]))] = float(f[3])
        elif f[0] == "corner":
            corner[(int(f[1]), int(f[2]))] = float(f[3])
    return macro, grid, rho, corner


def _dense(vals, grid):
    m = np.zeros((grid[1], grid[0]))
    for (ix, iy), v in vals.items():
        m[iy, ix] = v
    return m


def _example_geometry_and_box():
    macro, grid, rho, corner = _read_prefix_example()
    x0, y0, w, h = macro
    geo = Geometry(float(grid[0]), float(grid[1]), grid[0], grid[1], 1)   # unit bins, one layer
    box = np.array([[x0], [x0 + w], [y0], [y0 + h], [0.0], [1.0]])
    return geo, box, _dense(rho, grid), _dense(corner, grid)


def test_prefix_example_direct_overlap_matches_printed_density():
    geo, box, rho_printed, _ = _example_geometry_and_box()
    rho = den.box_density(box, np.ones(1), geo)
    np.testing.assert_allclose(rho[0], rho_printed, atol=1e-12)


def test_prefix_example_corner_map_matches_printed_map():
    geo, box, _, corner_printed = _example_geometry_and_box()
    A = den.box_corner_map(box[:, 0], geo)
    np.testing.assert_allclose(A[0], corner_printed, atol=1e-12)


def test_prefix_example_theorem1_reproduces_printed_density():
    geo, box, rho_printed, corner_printed = _example_geometry_and_box()
    np.testing.assert_allclose(den.prefix_sum_3d(corner_printed[None]), rho_printed[None], atol=1e-12)
    np.testing.assert_allclose(den.box_density_prefix(box, np.ones(1), geo)[0], rho_printed, atol=1e-12)


def _brute_force_density(boxes, weight, geo):
    """Per-bin loop: intersect every box with every bin (independent of the oracle's loops)."""
    rho = np.zeros((geo.nz, geo.ny, geo.nx))
    for k in range(geo.nz):
        for j in range(geo.ny):
            for i in range(geo.nx):
                bx = (i * geo.wb, (i + 1) * geo.wb)
                by = (j * geo.hb, (j + 1) * geo.hb)
                bz = (k * geo.db, (k + 1) * geo.db)
                for n in range(boxes.shape[1]):
                    lx = min(boxes[1, n], bx[1]) - max(boxes[0, n], bx[0])
                    ly = min(boxes[3, n], by[1]) - max(boxes[2, n], by[0])
                    lz = min(boxes[5, n], bz[1]) - max(boxes[4, n], bz[0])
                    if lx > 0 and ly > 0 and lz > 0:
                        rho[k, j, i] += weight[n] * lx * ly * lz / geo.vol_bin
    return rho


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_density_matches_brute_force_and_theorem1_on_random_boxes(seed):
    rng = np.random.default_rng(seed)
    geo = Geometry(12.0, 9.0, 6, 5, 3)
    n = 12
    lo = rng.uniform(0, 1, size=(3, n)) * np.array([[12.0], [9.0], [geo.dz]])
    ext = rng.uniform(0.1, 7.0, size=(3, n))
    hi = np.minimum(lo + ext, np.array([[12.0], [9.0], [geo.dz]]))
    boxes = np.stack([lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]])
    weight = rng.uniform(0.2, 1.0, size=n)
    ref = _brute_force_density(boxes, weight, geo)
    np.testing.assert_allclose(den.box_density(boxes, weight, geo), ref, atol=1e-12)
    np.testing.assert_allclose(den.box_density_prefix(boxes, weight, geo), ref, atol=1e-12)


def _tiny_case(seed=5):
    cfg = synth.small_config()
    return synth.make_case(config=cfg, seed=seed)


def test_total_density_equals_total_volume_for_interior_instances():
    c = _tiny_case()
    geo = geometry_of(c)
    xyz = c.xyz0.astype(np.float64).copy()
    # keep every stretched footprint inside the die so that no charge is clipped away
    w, h = at.instance_size(c.size, c.kind, xyz[2], geo.dz)
    wt, ht, _ = at.smoothing(w, h, geo.wb, geo.hb)
    xyz[0] = np.clip(xyz[0], wt / 2 + 1e-3, geo.die_x - wt / 2 - 1e-3)
    xyz[1] = np.clip(xyz[1], ht / 2 + 1e-3, geo.die_y - ht / 2 - 1e-3)
    rho = den.density_map(c.size, c.kind, xyz, geo)
    w, h = at.instance_size(c.size, c.kind, xyz[2], geo.dz)
    total_q = at.charge(w, h, geo.dz).sum()
    assert abs(rho.sum() * geo.vol_bin - total_q) <= 1e-12 * total_q


def test_total_density_equals_clipped_weighted_volume_everywhere():
    c = _tiny_case(7)
    geo = geometry_of(c)
    boxes, omega = den.footprints(c.size, c.kind, c.xyz0, geo)
    vol = np.prod(boxes[1::2] - boxes[0::2], axis=0)
    rho = den.density_map(c.size, c.kind, c.xyz0, geo)
    assert abs(rho.sum() * geo.vol_bin - (omega * vol).sum()) <= 1e-12 * (omega * vol).sum()


def test_local_smoothness_weight_times_stretched_area_is_true_area():
    w = np.array([0.5, 1.0, 4.0, 10.0])
    h = np.array([1.0, 7.0, 0.3, 12.0])
    wt, ht, om = at.smoothing(w, h, 3.0, 2.0)
    np.testing.assert_allclose(om * wt * ht, w * h, rtol=1e-15)
    assert np.all(wt >= np.sqrt(2) * 3.0) and np.all(ht >= np.sqrt(2) * 2.0)


def test_macro_size_transition_endpoints_and_linearity():
    dz = 8.0
    size = np.array([[10.0], [6.0], [7.0], [4.2]])
    kind = np.array([at.KIND_MACRO], dtype=np.uint8)
    w_lo, h_lo = at.instance_size(size, kind, np.array([dz / 4]), dz)
    w_hi, h_hi = at.instance_size(size, kind, np.array([3 * dz / 4]), dz)
    w_mid, _ = at.instance_size(size, kind, np.array([dz / 2]), dz)
    assert (w_lo[0], h_lo[0]) == (10.0, 6.0)
    assert np.isclose(w_hi[0], 7.0) and np.isclose(h_hi[0], 4.2)
    assert np.isclose(w_mid[0], 8.5)


def test_cell_size_and_pin_offset_follow_partition_with_strict_midplane():
    dz = 8.0
    size = np.array([[3.0, 3.0], [1.0, 1.0], [2.1, 2.1], [0.7, 0.7]])
    kind = np.zeros(2, dtype=np.uint8)
    z = np.array([dz / 2, dz / 2 + 1e-9])
    w, h = at.instance_size(size, kind, z, dz)
    assert list(w) == [3.0, 2.1] and list(h) == [1.0, 0.7]
    xyz = np.array([[10.0, 20.0], [5.0, 5.0], z])
    off = np.array([[1.0, 1.0], [0.5, 0.5], [0.7, 0.7], [0.35, 0.35]])
    px, py, top = at.pin_xy(xyz, np.array([0, 1]), off, dz)
    assert list(top) == [False, True]
    assert list(px) == [11.0, 20.7] and list(py) == [5.5, 5.35]


def test_hbt_alpha_worked_value():
    # 200 x 200 die on 64 x 64 bins, two z-bins: d_z = 6.25; eta = 2/(0.7 + 1)
    geo = Geometry(200.0, 200.0, 64, 64, 2)
    eta = 2.0 / 1.7
    expected = 3.5e-3 * 200.0 * eta ** 2 / 6.25 * np.log(90 * 10 * eta - 1)
    assert abs(geo.dz - 6.25) < 1e-15
    assert abs(hbt_alpha(200.0, geo.dz, 1.0, 0.7, 1.0, 10.0) - expected) < 1e-15
    assert abs(expected - 1.0795) < 1e-4
