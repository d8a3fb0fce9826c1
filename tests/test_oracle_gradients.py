"""Pins of the oracle's density gradients and optimiser."""
import numpy as np

from oracle import attributes as at
from oracle import density as den
from oracle import density_grad as dg
from oracle import optimizer as opt
from oracle import poisson
from oracle.geometry import geometry_of
from paper_2403_09070_amd import synth


def _case(seed=5, **kw):
    return synth.make_case(config=synth.small_config(**kw), seed=seed)


def _energy(c, xyz, geo):
    rho = den.density_map(c.size, c.kind, xyz, geo)
    return poisson.energy(rho, poisson.solve(rho, geo, want=("phi",))["phi"], geo)


def test_density_adjoint_identity():
    """<J u, w> = <u, J^T w> with J = d rho / d v taken by central differences."""
    c = _case(9)
    geo = geometry_of(c)
    rng = np.random.default_rng(0)
    v = c.xyz0.astype(np.float64)
    u = rng.normal(size=v.shape)
    u[:, (c.kind & 2) != 0] = 0.0
    u[2, np.abs(v[2] - geo.dz / 2) < 1e-3] = 0.0      # keep cells off the size switch
    w = rng.normal(size=(geo.nz, geo.ny, geo.nx))
    h = 1e-6
    ju = (den.density_map(c.size, c.kind, v + h * u, geo)
          - den.density_map(c.size, c.kind, v - h * u, geo)) / (2 * h)
    lhs = float(np.sum(ju * w))
    rhs = float(np.sum(u * dg.density_vjp(c.size, c.kind, v, w, geo)))
    assert abs(lhs - rhs) < 1e-6 * max(1.0, abs(lhs))


def test_adjoint_gradient_of_energy_matches_central_differences():
    c = _case(11)
    geo = geometry_of(c)
    v = c.xyz0.astype(np.float64)
    rho = den.density_map(c.size, c.kind, v, geo)
    phi = poisson.solve(rho, geo, want=("phi",))["phi"]
    g = dg.density_vjp(c.size, c.kind, v, phi * geo.vol_bin, geo)
    rng = np.random.default_rng(3)
    h = 1e-4 * geo.wb
    ok = total = 0
    idx = list(rng.choice(c.meta["n_cells"], size=25, replace=False)) + list(range(c.meta["n_cells"], c.n_inst))
    for i in idx:
        for a in range(3):
            if a == 2 and abs(v[2, i] - geo.dz / 2) < 2 * h:
                continue
            up, dn = v.copy(), v.copy()
            up[a, i] += h
            dn[a, i] -= h
            eu, e0, ed = _energy(c, up, geo), _energy(c, v, geo), _energy(c, dn, geo)
            fd = (eu - ed) / (2 * h)
            one_sided_gap = abs((eu - e0) / h - (e0 - ed) / h)
            total += 1
            if one_sided_gap > 1e-3 * max(1.0, abs(fd)):   # a kink inside the stencil
                continue
            assert abs(g[a, i] - fd) < 1e-5 * max(1.0, abs(fd)), (i, a, g[a, i], fd)
            ok += 1
    assert ok >= 0.9 * total


def test_field_gather_agrees_with_adjoint_and_converges_under_refinement():
    """The paper's field gather approaches the exact adjoint gradient as bins shrink."""
    errs = []
    for n in (16, 32, 64):
        cfg = synth.small_config(n_cells=200, n_nets=10, die=100.0, nx=n, ny=n, nz=2,
                                 macros=("uniform", 2, 0.02, 0.04))
        c = synth.make_case(config=cfg, seed=1)
        geo = geometry_of(c)
        v = c.xyz0.astype(np.float64)
        rho = den.density_map(c.size, c.kind, v, geo)
        sol = poisson.solve(rho, geo)
        g_f = dg.field_gather(c.size, c.kind, v, sol["ex"], sol["ey"], sol["ez"], geo)
        g_a = dg.density_vjp(c.size, c.kind, v, sol["phi"] * geo.vol_bin, geo)
        assert float(np.sum(g_f[:2] * g_a[:2])) > 0.0
        errs.append(np.linalg.norm(g_f[:2] - g_a[:2]) / np.linalg.norm(g_a[:2]))
    assert errs[2] < errs[0]


def test_field_gather_mirror_symmetry():
    """Mirroring the placement in x mirrors the x-gradient and keeps y and z."""
    c = _case(13)
    geo = geometry_of(c)
    v = c.xyz0.astype(np.float64)
    m = v.copy()
    m[0] = geo.die_x - v[0]
    out = []
    for p in (v, m):
        rho = den.density_map(c.size, c.kind, p, geo)
        sol = poisson.solve(rho, geo)
        out.append(dg.field_gather(c.size, c.kind, p, sol["ex"], sol["ey"], sol["ez"], geo))
    np.testing.assert_allclose(out[1][0], -out[0][0], atol=1e-9 * np.abs(out[0]).max())
    np.testing.assert_allclose(out[1][1:], out[0][1:], atol=1e-9 * np.abs(out[0]).max())


def _cell_die_size(c, i, z, dz):
    """A standard cell's (w, h) on the die its z puts it on (top above the mid-plane)."""
    top = z > 0.5 * dz
    return (float(c.size[2, i]), float(c.size[3, i])) if top else (float(c.size[0, i]), float(c.size[1, i]))


def test_field_gather_of_a_constant_field_is_the_charge_times_the_field():
    """Closed form of -omega sum_b vol(D ∩ b) E_b under a uniform field E = (c_x, c_y, c_z): for an
    instance whose stretched footprint lies inside the die, omega times the stretched volume is the
    true volume w h d_z/2, so the gather is -(w h d_z / 2) c per axis.  A lost omega, a dropped
    depth factor, an overlap that does not sum to the box, or swapped field axes fails it."""
    c = _case(31, nz=4)
    geo = geometry_of(c)
    shape = (geo.nz, geo.ny, geo.nx)
    cx, cy, cz = 0.7, -1.9, 2.6
    v = c.xyz0.astype(np.float64)
    g = dg.field_gather(c.size, c.kind, v, np.full(shape, cx), np.full(shape, cy), np.full(shape, cz), geo)
    r2 = np.sqrt(2.0)
    checked = 0
    for i in range(c.meta["n_cells"]):
        if c.kind[i] & 2:
            continue
        w, h = _cell_die_size(c, i, v[2, i], geo.dz)
        hw, hh = 0.5 * max(w, r2 * geo.wb), 0.5 * max(h, r2 * geo.hb)
        if not (hw <= v[0, i] <= geo.die_x - hw and hh <= v[1, i] <= geo.die_y - hh):
            continue
        q = w * h * 0.5 * geo.dz
        np.testing.assert_allclose(g[:, i], [-q * cx, -q * cy, -q * cz], rtol=1e-12)
        checked += 1
    assert checked >= 100


def test_field_gather_of_a_bin_centred_cell_weights_its_bins_by_hand():
    """A cell smaller than sqrt2 bins, centred in bin (b_x, b_y) at z = d_z/4 (or 3 d_z/4), has the
    stretched footprint [centre -+ bin/sqrt2] per planar axis: the whole centre bin and
    (sqrt2 - 1)/2 of each neighbour, and the full depth of z-bins 0 and 1 (2 and 3), N_z = 4.  With
    a random field the gather is -omega sum of those overlap volumes times E, omega =
    w h / (2 w_b h_b).  A transposed map index, a wrong z-bin or stretch fails it."""
    c = _case(32, nz=4)
    geo = geometry_of(c)
    rng = np.random.default_rng(8)
    shape = (geo.nz, geo.ny, geo.nx)
    fields = [rng.normal(size=shape) for _ in range(3)]
    v = c.xyz0.astype(np.float64)
    cells = [i for i in range(c.meta["n_cells"]) if not c.kind[i] & 2][:40]
    place = {}
    for k, i in enumerate(cells):
        bx, by = 1 + rng.integers(geo.nx - 2), 1 + rng.integers(geo.ny - 2)
        top = k % 2 == 1
        v[0, i], v[1, i] = (bx + 0.5) * geo.wb, (by + 0.5) * geo.hb
        v[2, i] = (0.75 if top else 0.25) * geo.dz
        place[i] = (bx, by, (2, 3) if top else (0, 1))
    g = dg.field_gather(c.size, c.kind, v, *fields, geo)
    side = 0.5 * (np.sqrt(2.0) - 1.0)
    wx = {-1: side * geo.wb, 0: geo.wb, 1: side * geo.wb}
    wy = {-1: side * geo.hb, 0: geo.hb, 1: side * geo.hb}
    for i, (bx, by, zbins) in place.items():
        w, h = _cell_die_size(c, i, v[2, i], geo.dz)
        assert w < np.sqrt(2.0) * geo.wb and h < np.sqrt(2.0) * geo.hb
        omega = (w / (np.sqrt(2.0) * geo.wb)) * (h / (np.sqrt(2.0) * geo.hb))
        for a in range(3):
            want = 0.0
            for ox in (-1, 0, 1):
                for oy in (-1, 0, 1):
                    for zb in zbins:
                        want += wx[ox] * wy[oy] * geo.db * fields[a][zb, by + oy, bx + ox]
            assert abs(g[a, i] - (-omega * want)) <= 1e-12 * max(1.0, abs(omega * want)), (i, a, g[a, i], -omega * want)


def test_preconditioner_follows_mixed_size_rule():
    c = _case(2)
    pb = opt.problem_of(c)
    v = c.xyz0.astype(np.float64)
    w, h = at.instance_size(c.size, c.kind, v[2], pb.geo.dz)
    q = at.charge(w, h, pb.geo.dz)
    for lam in (1e-6, 1e-2, 10.0):
        H = opt.preconditioner(pb, v, lam)
        mac = (c.kind & 1) != 0
        np.testing.assert_allclose(H[mac], np.maximum(1.0, pb.npins[mac] + lam * q[mac]))
        np.testing.assert_allclose(H[~mac], np.maximum(1.0, lam * q[~mac]))


def test_preconditioner_forms_against_net_counts():
    """Eq. general-precond and its two approximations: the ePlace form minus the ePlace3D form is
    |E_i|, the number of nets incident to instance i (counted here by a plain loop over the nets);
    the mixed form is max{1, ePlace} on macros and max{1, ePlace3D} elsewhere."""
    c = _case(2)
    pb = opt.problem_of(c)
    v = c.xyz0.astype(np.float64)
    count = np.zeros(c.n_inst)
    for e in range(c.n_nets):
        for i in set(int(x) for x in c.pin2node[c.net_start[e]:c.net_start[e + 1]]):
            count[i] += 1
    mac = (c.kind & 1) != 0
    for lam in (1e-6, 0.3, 10.0):
        he = opt.preconditioner(pb, v, lam, "eplace")
        h3 = opt.preconditioner(pb, v, lam, "eplace3d")
        hm = opt.preconditioner(pb, v, lam, "mixed")
        np.testing.assert_allclose(he - h3, count, atol=1e-9 * max(1.0, np.abs(he).max()))
        np.testing.assert_allclose(h3 / lam, opt.preconditioner(pb, v, 1.0, "eplace3d"), rtol=1e-12)
        np.testing.assert_allclose(hm[mac], np.maximum(1.0, he[mac]))
        np.testing.assert_allclose(hm[~mac], np.maximum(1.0, h3[~mac]))


def test_nesterov_converges_on_a_convex_quadratic():
    """With the objective replaced by 1/2 |v - v*|^2 the iterates converge to v*."""
    rng = np.random.default_rng(0)
    target = rng.uniform(10, 90, size=(3, 50))
    v0 = rng.uniform(10, 90, size=(3, 50))
    movable = np.ones(50, dtype=bool)
    grad = lambda v: v - target  # noqa: E731
    st = opt.GPState(u=v0.copy(), v=v0.copy(), v_prev=v0 - 0.01 * grad(v0), g_prev=None, a=1.0, lam=0.0)
    st.g_prev = grad(st.v_prev)
    err0 = np.abs(v0 - target).max()
    for _ in range(60):
        g = grad(st.v)
        u, v, a, _ = opt.nesterov_update(st, g, lambda p: p, movable)
        st.v_prev, st.g_prev, st.u, st.v, st.a = st.v, g, u, v, a
    assert np.abs(st.u - target).max() < 1e-8 * err0


def test_lipschitz_step_is_exact_on_a_uniform_quadratic():
    """Closed form: for the gradient c (v - v*) the estimate |dv| / |dg| is 1/c whatever the two
    points, so the first move lands on v* exactly; with a_0 = 1 the momentum coefficient
    (a_0 - 1)/a_1 is zero, so v_1 = u_1, and a_1 = (1 + sqrt(5))/2."""
    rng = np.random.default_rng(1)
    c = 2.5
    target = rng.uniform(10, 90, size=(3, 40))
    v0 = rng.uniform(10, 90, size=(3, 40))
    grad = lambda v: c * (v - target)  # noqa: E731
    vp = v0 + rng.normal(scale=3.0, size=v0.shape)
    st = opt.GPState(u=v0.copy(), v=v0.copy(), v_prev=vp, g_prev=grad(vp), a=1.0, lam=0.0)
    u, v, a, step = opt.nesterov_update(st, grad(v0), lambda p: p, np.ones(40, dtype=bool))
    assert abs(step - 1.0 / c) < 1e-14
    np.testing.assert_allclose(u, target, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(v, u)
    assert abs(a - (1.0 + 5.0 ** 0.5) / 2.0) < 1e-15


def test_clamp_keeps_instances_inside_region():
    c = _case(3)
    pb = opt.problem_of(c)
    rng = np.random.default_rng(0)
    v = c.xyz0.astype(np.float64) + rng.normal(scale=60.0, size=c.xyz0.shape)
    out = opt.clamp(pb, v)
    w, h = at.instance_size(c.size, c.kind, out[2], pb.geo.dz)
    mov = pb.movable
    assert np.all(out[2, mov] >= pb.geo.dz / 4) and np.all(out[2, mov] <= 3 * pb.geo.dz / 4)
    assert np.all(out[0, mov] - w[mov] / 2 >= -1e-12) and np.all(out[0, mov] + w[mov] / 2 <= pb.geo.die_x + 1e-12)
    assert np.all(out[1, mov] - h[mov] / 2 >= -1e-12) and np.all(out[1, mov] + h[mov] / 2 <= pb.geo.die_y + 1e-12)


def test_gp_reduces_overflow_and_keeps_wirelength_finite():
    c = synth.make_case("c1")
    pb = opt.problem_of(c)
    st = opt.gp_init(pb, c.xyz0)
    ms = [opt.gp_step(pb, st) for _ in range(8)]
    assert ms[-1]["ovfl_bot"] < ms[0]["ovfl_bot"] and ms[-1]["ovfl_top"] < ms[0]["ovfl_top"]
    assert all(np.isfinite(m["hpwl_d2d"]) for m in ms)


def _one_sided(c, v, w, geo, a, i, h, up):
    """(f(v + h e) - f(v)) / h from above, (f(v) - f(v - h e)) / h from below, f = <rho(v), w>."""
    f0 = float(np.sum(den.density_map(c.size, c.kind, v, geo) * w))
    p = v.copy()
    p[a, i] += h if up else -h
    f1 = float(np.sum(den.density_map(c.size, c.kind, p, geo) * w))
    return (f1 - f0) / h if up else (f0 - f1) / h


def test_adjoint_z_at_the_clamp_bounds_is_the_inward_one_sided_derivative():
    """At z = d_z/4 and z = 3d_z/4 (the bounds of the movable range, where every z-edge of a
    cuboid sits on a bin face or on the region's floor or ceiling when N_z is even) the adjoint's
    z component is the one-sided derivative into the range: from above at d_z/4, from below at
    3d_z/4.  The other one-sided derivative differs there, so a dropped or misplaced face fails."""
    c = _case(21, nz=4)
    geo = geometry_of(c)
    rng = np.random.default_rng(4)
    w = rng.normal(size=(geo.nz, geo.ny, geo.nx))
    v = c.xyz0.astype(np.float64)
    mov = np.nonzero((c.kind & 2) == 0)[0]
    pick = list(rng.choice(mov[mov < c.meta["n_cells"]], size=12, replace=False)) + \
        [i for i in mov if i >= c.meta["n_cells"]]
    v[2, pick[::2]] = 0.25 * geo.dz
    v[2, pick[1::2]] = 0.75 * geo.dz
    g = dg.density_vjp(c.size, c.kind, v, w, geo)
    h = 1e-7 * geo.db
    differs = 0
    for i in pick:
        up = v[2, i] < 0.5 * geo.dz
        inward = _one_sided(c, v, w, geo, 2, i, h, up)
        outward = _one_sided(c, v, w, geo, 2, i, h, not up)
        assert abs(g[2, i] - inward) <= 1e-5 * max(1.0, abs(inward)), (i, up, g[2, i], inward, outward)
        differs += abs(inward - outward) > 1e-3 * max(1.0, abs(inward))
    assert differs >= len(pick) // 2


def test_adjoint_planar_at_the_die_sides_is_the_inward_one_sided_derivative():
    """A macro that is not stretched (wider than sqrt2 bins), clamped against a die side, has an
    x (y) edge exactly on the region's face: the adjoint takes the derivative into the die."""
    c = _case(22, nz=4, macros=("uniform", 3, 0.04, 0.06))
    geo = geometry_of(c)
    rng = np.random.default_rng(5)
    w = rng.normal(size=(geo.nz, geo.ny, geo.nx))
    v = c.xyz0.astype(np.float64)
    macros = [i for i in range(c.meta["n_cells"], c.n_inst) if (c.kind[i] & 2) == 0]
    assert len(macros) >= 2
    v[2, macros] = 0.25 * geo.dz                 # bottom-die size exactly
    wd, hd = c.size[0].astype(np.float64), c.size[1].astype(np.float64)
    assert np.all(wd[macros] > np.sqrt(2.0) * geo.wb) and np.all(hd[macros] > np.sqrt(2.0) * geo.hb)
    i, j = macros[0], macros[1]
    v[0, i] = 0.5 * wd[i]                        # against the left side
    v[1, j] = geo.die_y - 0.5 * hd[j]            # against the far side in y
    g = dg.density_vjp(c.size, c.kind, v, w, geo)
    h = 1e-7 * geo.wb
    for (a, k, up) in ((0, i, True), (1, j, False)):
        inward = _one_sided(c, v, w, geo, a, k, h, up)
        outward = _one_sided(c, v, w, geo, a, k, h, not up)
        assert abs(g[a, k] - inward) <= 1e-5 * max(1.0, abs(inward)), (a, k, g[a, k], inward, outward)
        assert abs(inward - outward) > 1e-3 * max(1.0, abs(inward))


def test_field_gather_z_agrees_with_adjoint_at_the_clamp_bounds():
    """Where a placement ends, every instance clamped at z = d_z/4 or 3 d_z/4 (N_z = 4), the z
    component of the paper's field gather points the way of the exact adjoint's (cosine >= 0.85 on
    2,000 cells).  A clamp-bound derivative that drops a face, or takes the outward side, leaves
    the two near-orthogonal (cosine 0.6-0.7)."""
    for n in (16, 32):
        cfg = synth.small_config(n_cells=2000, n_nets=10, die=100.0, nx=n, ny=n, nz=4,
                                 macros=("uniform", 2, 0.02, 0.04))
        c = synth.make_case(config=cfg, seed=1)
        geo = geometry_of(c)
        v = c.xyz0.astype(np.float64)
        v[2] = np.where(v[2] > 0.5 * geo.dz, 0.75 * geo.dz, 0.25 * geo.dz)
        rho = den.density_map(c.size, c.kind, v, geo)
        sol = poisson.solve(rho, geo)
        g_f = dg.field_gather(c.size, c.kind, v, sol["ex"], sol["ey"], sol["ez"], geo)[2]
        g_a = dg.density_vjp(c.size, c.kind, v, sol["phi"] * geo.vol_bin, geo)[2]
        cos = float(np.sum(g_f * g_a) / (np.linalg.norm(g_f) * np.linalg.norm(g_a)))
        assert cos >= 0.85, (n, cos)


def test_adjoint_at_a_die_side_does_not_depend_on_the_rounding_of_the_clamp():
    """A macro at the upper z bound held against the far x and y sides grows as z moves into the
    range (down), pushing its far edges outward, where the region holds them.  At the exact
    position the adjoint's z component is the inward one-sided difference; with the position
    rounded to float32 (the clamp's arithmetic), the far edges sit a rounding inside or outside the
    faces, and the adjoint must take them as on the faces all the same: a rule that decided by the
    rounding would count or drop whole face terms."""
    c = _case(23, nz=4, macros=("uniform", 3, 0.04, 0.06))
    geo = geometry_of(c)
    rng = np.random.default_rng(6)
    w = rng.normal(size=(geo.nz, geo.ny, geo.nx))
    v = c.xyz0.astype(np.float64)
    macros = [i for i in range(c.meta["n_cells"], c.n_inst) if (c.kind[i] & 2) == 0]
    i = macros[0]
    v[2, i] = 0.75 * geo.dz                      # top-die size exactly; moving down grows it
    wt, ht = float(c.size[2, i]), float(c.size[3, i])
    assert c.size[0, i] > c.size[2, i] and c.size[1, i] > c.size[3, i]
    v[0, i] = geo.die_x - 0.5 * wt
    v[1, i] = geo.die_y - 0.5 * ht
    g = dg.density_vjp(c.size, c.kind, v, w, geo)
    h = 1e-7 * geo.db
    inward = _one_sided(c, v, w, geo, 2, i, h, False)
    outward = _one_sided(c, v, w, geo, 2, i, h, True)
    assert abs(g[2, i] - inward) <= 1e-5 * max(1.0, abs(inward)), (g[2, i], inward, outward)
    assert abs(inward - outward) > 1e-3 * max(1.0, abs(inward))
    for step in (-np.inf, np.inf):               # the float32 neighbours of the exact position
        r = v.copy()
        for a in (0, 1):
            r[a, i] = float(np.nextafter(np.float32(v[a, i]), np.float32(step)))
        r[2, i] = float(np.float32(v[2, i]))
        gr = dg.density_vjp(c.size, c.kind, r, w, geo)
        assert abs(gr[2, i] - g[2, i]) <= 1e-5 * max(1.0, abs(g[2, i])), (step, gr[2, i], g[2, i])
