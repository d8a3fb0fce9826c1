"""Pins of the oracle's GP metrics and start-up: per-die overflow, crossing-net count, 3D-HPWL and
D2D HPWL totals, the initial density weight lambda_0 and the bootstrap point v_-1.

Each expected value comes from a hand-worked case (tests/golden/) or from a route that shares no
code with the function under test: the closed-form WA gradient of a two-pin net and central
differences of the oracle's energy, which the Poisson tests pin separately.
"""
import os

import numpy as np

from oracle import attributes as at
from oracle import density as den
from oracle import optimizer as opt
from oracle import poisson
from oracle import wirelength as wl
from oracle.geometry import Geometry

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_overflow_toy():
    insts, expect = [], {}
    for line in open(os.path.join(GOLD, "overflow_toy.txt")):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "inst":
            insts.append((int(f[2]),) + tuple(float(v) for v in f[3:8]))
        elif f[0] == "expect":
            expect = {k: float(v) for k, v in (kv.split("=") for kv in f[1:])}
    return insts, expect


def _toy_problem(insts, geo):
    n = len(insts)
    kind = np.array([k for k, *_ in insts], dtype=np.uint8)
    w = np.array([r[1] for r in insts])
    h = np.array([r[2] for r in insts])
    xyz = np.array([[r[3] for r in insts], [r[4] for r in insts], [r[5] for r in insts]])
    size = np.stack([w, h, w, h])                # the given size on either die
    pb = opt.Problem(size=size, kind=kind, net_start=np.zeros(1, dtype=np.int64),
                     pin2node=np.zeros(0, dtype=np.int64), pin_off=np.zeros((4, 0)), geo=geo,
                     gamma=1.0, alpha=0.0, ramp=1.0, target=1.0)
    return pb, xyz, n


def test_per_die_overflow_of_a_hand_worked_stack():
    insts, exp = _read_overflow_toy()
    geo = Geometry(4.0, 4.0, 4, 4, 4)
    assert (geo.wb, geo.db, geo.dz, geo.vol_bin) == (1.0, 1.0, 4.0, 1.0)
    pb, xyz, _ = _toy_problem(insts, geo)
    rho = den.density_map(pb.size, pb.kind, xyz, geo)
    excess = np.maximum(rho - 1.0, 0.0) * geo.vol_bin
    assert excess[:2].sum() == exp["excess_bot"] and excess[2:].sum() == exp["excess_top"]
    w, h = at.instance_size(pb.size, pb.kind, xyz[2], geo.dz)
    q = at.charge(w, h, geo.dz)
    top = at.partition(xyz[2], geo.dz)
    mov = ~at.is_fixed(pb.kind)
    assert q[mov & ~top].sum() == exp["q_bot"] and q[mov & top].sum() == exp["q_top"]
    ob, ot = opt.overflow(pb, rho, xyz)
    assert abs(ob - exp["ovfl_bot"]) < 1e-15 and abs(ot - exp["ovfl_top"]) < 1e-15


def test_overflow_splits_the_dies_at_the_mid_plane_of_the_bins():
    """Moving the top die's excess into the bottom die's z-bins moves it to the bottom's overflow:
    the split is between z-bins N_z/2 - 1 and N_z/2, not elsewhere."""
    insts, exp = _read_overflow_toy()
    geo = Geometry(4.0, 4.0, 4, 4, 4)
    pb, xyz, _ = _toy_problem(insts, geo)
    rho = den.density_map(pb.size, pb.kind, xyz, geo)
    for k in range(4):                 # an excess of 1 in one bin of z-layer k only
        r = np.ones_like(rho)
        r[k, 0, 0] = 2.0
        ob, ot = opt.overflow(pb, r, xyz)
        assert (ob, ot) == ((1.0 / exp["q_bot"], 0.0) if k < 2 else (0.0, 1.0 / exp["q_top"]))


def _netlist(nets, dz):
    """Instances at the pins (zero offsets) of nets given as (top points, bottom points)."""
    pts, zs, p2n, starts = [], [], [], [0]
    for top, bot in nets:
        for p in top:
            p2n.append(len(pts)); pts.append(p); zs.append(0.75 * dz)
        for p in bot:
            p2n.append(len(pts)); pts.append(p); zs.append(0.25 * dz)
        starts.append(len(p2n))
    pts = np.array(pts, dtype=np.float64)
    n = len(pts)
    xyz = np.stack([pts[:, 0], pts[:, 1], np.array(zs)])
    return (xyz, np.ones((4, n)), np.zeros(n, dtype=np.uint8), np.array(starts), np.array(p2n),
            np.zeros((4, len(p2n))))


def test_crossing_count_and_hpwl_totals_of_the_figure_nets():
    """Nets of Fig. hpwl-analysis (a) and (b) plus a bottom-only net and a one-pin net.  By hand
    (Def. 3d-hpwl, Eq. wl-obj): net (a) whole box 3 x 2, W_x = 4, W_y = 2.5; net (b) whole box
    3 x 2, W_x = 3, W_y = 2; the bottom-only net (0,0)-(4,3) has box 4 x 3 and W = 7; a one-pin net
    contributes nothing.  Two nets cross the dies.  With the dies at z = d_z/4 and 3 d_z/4 a
    crossing net spans d_z/2 in z, the bottom-only net 0."""
    fig_a = ([(0, 1), (2, 0)], [(1, -1), (3, 0.5)])
    fig_b = ([(0, 1)], [(1, -1), (2, 0), (3, 0.5)])
    bottom = ([], [(0, 0), (4, 3)])
    single = ([(5, 5)], [])
    geo = Geometry(100.0, 100.0, 10, 10, 2)          # d_z = 20
    alpha = 0.3
    xyz, size, kind, ns, p2n, off = _netlist([fig_a, fig_b, bottom, single], geo.dz)
    out = wl.wirelength(size, kind, xyz, ns, p2n, off, geo, gamma=1.0, alpha=alpha)
    assert out["ncut"] == 2
    assert out["hpwl_d2d"] == 6.5 + 5.0 + 7.0 + 0.0
    half = 0.5 * geo.dz
    expect_3d = (3 + 2 + alpha * half) + (3 + 2 + alpha * half) + (4 + 3 + 0.0) + 0.0
    assert abs(out["hpwl_3d"] - expect_3d) < 1e-12
    # all on one die: no crossing net, and the D2D HPWL is the planar HPWL of the whole boxes
    xyz1 = xyz.copy()
    xyz1[2] = 0.25 * geo.dz
    out1 = wl.wirelength(size, kind, xyz1, ns, p2n, off, geo, gamma=1.0, alpha=alpha)
    assert out1["ncut"] == 0
    assert out1["hpwl_d2d"] == (3 + 2) + (3 + 2) + (4 + 3) + 0.0
    assert out1["hpwl_3d"] == out1["hpwl_d2d"]


def _two_cell_problem():
    """Two equal cells on the bottom die, mirror images about the region's centre in x, joined by
    one two-pin net (pins at the centres)."""
    geo = Geometry(32.0, 32.0, 16, 16, 2)              # w_b = 2, d_z = 4
    size = np.full((4, 2), 3.0)                        # 3 x 3 on either die (no stretch)
    kind = np.zeros(2, dtype=np.uint8)
    pb = opt.Problem(size=size, kind=kind, net_start=np.array([0, 2]), pin2node=np.array([0, 1]),
                     pin_off=np.zeros((4, 2)), geo=geo, gamma=2.0, alpha=0.0, ramp=1.05, target=1.0)
    xyz = np.array([[11.3, 32.0 - 11.3], [14.1, 14.1], [0.25 * geo.dz, 0.25 * geo.dz]])
    return pb, xyz


def _energy(pb, xyz):
    rho = den.density_map(pb.size, pb.kind, xyz, pb.geo)
    return poisson.energy(rho, poisson.solve(rho, pb.geo, want=("phi",))["phi"], pb.geo)


def _fd_energy_gradient(pb, xyz, h=1e-5):
    g = np.zeros_like(xyz)
    for i in range(xyz.shape[1]):
        for a in range(3):
            up, dn = xyz.copy(), xyz.copy()
            up[a, i] += h
            dn[a, i] -= h
            if a == 2:    # on the lower bound only the upward side exists; U is quadratic there
                up2 = xyz.copy()
                up2[a, i] += 2 * h
                g[a, i] = (-3 * _energy(pb, xyz) + 4 * _energy(pb, up) - _energy(pb, up2)) / (2 * h)
            else:
                g[a, i] = (_energy(pb, up) - _energy(pb, dn)) / (2 * h)
    return g


def test_lambda0_is_the_l1_ratio_of_independent_gradients():
    """lambda_0 = |grad W|_1 / |grad U|_1 at v_0 (reading of the optimiser's start).  grad W of the
    two-pin net is the closed form d/dD [D tanh(D/(2 gamma))] = tanh(t) + t sech^2(t), t = D/(2 gamma),
    on x only (equal y, equal z, no crossing); grad U by differences of the oracle energy."""
    pb, xyz = _two_cell_problem()
    D = xyz[0, 1] - xyz[0, 0]
    t = D / (2 * pb.gamma)
    gw = np.tanh(t) + t / np.cosh(t) ** 2
    gu = _fd_energy_gradient(pb, xyz)
    lam_hand = 2 * gw / np.abs(gu).sum()
    st = opt.gp_init(pb, xyz, dgrad="adjoint")
    assert abs(st.lam - lam_hand) <= 1e-6 * lam_hand, (st.lam, lam_hand)


def test_bootstrap_point_moves_the_largest_component_by_a_hundredth_of_a_bin():
    """v_-1 = clamp(v_0 - 0.01 w_b g_0 / |g_0|_inf): the coordinate with the largest preconditioned
    gradient moves by exactly 0.01 w_b against it, every move is against its gradient component and
    proportional to it.  g_0 is rebuilt from the independent gradients of the lambda_0 pin."""
    pb, xyz = _two_cell_problem()
    D = xyz[0, 1] - xyz[0, 0]
    t = D / (2 * pb.gamma)
    gw = np.tanh(t) + t / np.cosh(t) ** 2
    gW = np.array([[-gw, gw], [0.0, 0.0], [0.0, 0.0]])
    gu = _fd_energy_gradient(pb, xyz)
    st = opt.gp_init(pb, xyz, dgrad="adjoint")
    lq = st.lam * 3.0 * 3.0 * 0.5 * pb.geo.dz            # lambda q of each cell
    g0 = (gW + st.lam * gu) / max(1.0, lq)
    move = st.v_prev - st.v
    k = np.unravel_index(np.argmax(np.abs(g0)), g0.shape)
    assert abs(abs(move[k]) - 0.01 * pb.geo.wb) < 1e-9 * pb.geo.wb
    free = (np.abs(g0) > 1e-3 * np.abs(g0).max())
    free[2] &= g0[2] < 0                                  # z on its lower bound only moves up
    np.testing.assert_allclose(move[free], -0.01 * pb.geo.wb * g0[free] / np.abs(g0).max(), rtol=1e-4)
