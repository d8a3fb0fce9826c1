"""Density-penalty gradients: the paper's field gather and the exact adjoint of the density map.

Field gather (Sec. III-A: the gradient of the penalty is the charge times the field, gathered
from the overlapped bins in the backward phase of Sec. IV-A):

    dU/dv_i = - omega_i * sum_b vol(D_i ∩ b) * E_b          (per axis)

Reading of the sign: the paper names q_i E_i both the force and the gradient; the force is
+q_i E_i, so the gradient is its negative, and gradient descent spreads the charges.  For macros
the change of size with z is ignored here (force = charge x field).  This is not the derivative
of any discrete objective; its tests pin it by closed forms (a uniform field gives the charge
times the field; a bin-centred cell gathers its bins with overlaps worked by hand) and by its
properties (mirror symmetry, convergence to the exact adjoint under refinement).

Exact adjoint (the differentiation form): sum_b g_b d rho_b / d v_i for a map g, including the
z-dependence of the macro size transition and of the local-smoothness weight.  With
g = phi vol(b) it is the exact gradient of U = 1/2 sum rho phi vol(b).

One-sided derivatives (reading; the paper gives no adjoint).  The map is piecewise linear in each
coordinate, with kinks where an edge of the cuboid meets a bin face or a face of the region.  Per
axis the adjoint takes the derivative from above (the coordinate growing), except when the
cuboid's unclipped upper edge along that axis lies on or beyond the region's upper face, where it
takes the derivative from below.  At the bounds of the movable range this is the direction the
clamp allows: z = d_z/4 puts the lower z-edge on the region's floor (derivative from above, into
the region) and z = 3 d_z/4 puts the upper z-edge on its ceiling (derivative from below); an
unstretched instance clamped against a die side is treated alike.  Moving in the chosen
direction, an edge at e changes the overlap of exactly one bin, by +1 (upper edge) or -1 (lower
edge) per unit length: from above the bin floor(e/s), provided 0 <= e < L; from below the bin
ceil(e/s) - 1, provided 0 < e <= L (s the bin size, L the region's extent); an edge outside these
ranges is held by the region and changes nothing.  A z within 2^-20 d_z of a bound counts as on
it (the bounds are rounded when the coordinates are float32), and its z-edges are taken exactly
on the faces they then sit on: the floor and the mid-plane at d_z/4, the mid-plane and the ceiling
at 3 d_z/4 (N_z is even).  Likewise a planar edge within 2^-20 of the region's extent of a region
face is on that face when the derivative's direction and bin are decided: the clamp holds an
instance against a die side at a float32 position, which leaves its edge a rounding away from
the face on either side, and the derivative must not depend on which (the overlap lengths
themselves are taken from the edges as they are).
"""
from __future__ import annotations

import numpy as np

from .attributes import instance_size, is_fixed, macro_size_slope, smoothing
from .density import _bin_range, _SMALL_SPAN, axis_overlap

CLAMP_BAND = 2.0 ** -20      # a z this close to a bound of the movable range (times d_z) is on it


def z_bands(z, dz):
    """Instances at the lower and at the upper bound of the movable range [d_z/4, 3 d_z/4]."""
    z = np.asarray(z, dtype=np.float64)
    tol = CLAMP_BAND * dz
    return np.abs(z - 0.25 * dz) <= tol, np.abs(z - 0.75 * dz) <= tol


def _edges(size, kind, xyz, geo):
    """Raw (unclipped) cuboid edges, clipped edges, weight and stretch data per instance, and per
    axis whether the one-sided derivative is taken from below."""
    xyz = np.asarray(xyz, dtype=np.float64)
    w, h = instance_size(size, kind, xyz[2], geo.dz)
    wt, ht, omega = smoothing(w, h, geo.wb, geo.hb)
    raw = np.stack([xyz[0] - 0.5 * wt, xyz[0] + 0.5 * wt, xyz[1] - 0.5 * ht, xyz[1] + 0.5 * ht,
                    xyz[2] - 0.25 * geo.dz, xyz[2] + 0.25 * geo.dz])
    lim = np.array([geo.die_x, geo.die_x, geo.die_y, geo.die_y, geo.dz, geo.dz])[:, None]
    box = np.clip(raw, 0.0, lim)
    # planar edges a rounding away from a region face are on it (for the one-sided decisions only)
    for k in range(4):
        band = CLAMP_BAND * lim[k, 0]
        raw[k] = np.where(np.abs(raw[k]) <= band, 0.0, np.where(np.abs(raw[k] - lim[k, 0]) <= band, lim[k, 0], raw[k]))
    below = raw[1::2] >= lim[1::2]          # [3][n]: upper edge on or past the region's upper face
    at_lo, at_hi = z_bands(xyz[2], geo.dz)
    below[2] = at_hi | (~at_lo & below[2])
    return raw, box, below, w, h, wt, ht, omega


def _edge_bin(a, e, down, raw, geo, sel):
    """Bin whose overlap edge e (0 lower, 1 upper) of axis a changes when the edge moves down
    (``down``) or up, and whether it changes any (False while the region holds the edge)."""
    step = (geo.wb, geo.hb, geo.db)[a]
    n = (geo.nx, geo.ny, geo.nz)[a]
    L = (geo.die_x, geo.die_y, geo.dz)[a]
    edge = raw[2 * a + e, sel]
    dn = down[sel]
    moves = np.where(dn, (edge > 0.0) & (edge <= L), (edge >= 0.0) & (edge < L))
    eb = np.where(dn, np.ceil(edge / step) - 1.0, np.floor(edge / step))
    if a == 2:
        # at a bound the z-edges sit exactly on faces: lower bound (moving up) edges on bins 0 and
        # N_z/2, upper bound (moving down) on bins N_z/2 - 1 and N_z - 1
        z = 0.5 * (raw[4, sel] + raw[5, sel])
        at_lo, at_hi = z_bands(z, geo.dz)
        eb = np.where(at_lo, (0, n // 2)[e], np.where(at_hi, (n // 2 - 1, n - 1)[e], eb))
        moves = moves | at_lo | at_hi
    return np.clip(eb, 0, n - 1).astype(np.int64), moves


def _factor(mode, a, b, raw, box, geo, sel):
    """Per-bin factor along axis a for bins b of the selected instances.

    "len": the overlap length; (e, down): 1 on the bin whose overlap edge e changes under the
    one-sided motion (the derivative of the overlap length with respect to that edge), else 0.
    """
    step = (geo.wb, geo.hb, geo.db)[a]
    if mode == "len":
        return axis_overlap(box[2 * a, sel], box[2 * a + 1, sel], b, step)
    eb, moves = _edge_bin(a, mode[0], mode[1], raw, geo, sel)
    return np.where((b == eb) & moves, 1.0, 0.0)


def _box_sum(m, raw, box, geo, modes):
    """sum_b m[b] * Fx(bx) Fy(by) Fz(bz) for every instance, F chosen by ``modes`` (x, y, z).

    Along an axis with an edge mode the sum runs over that edge's bin alone, which may lie just
    outside the clipped cuboid (an upper edge on a bin face, moving up)."""
    m = np.asarray(m, dtype=np.float64)
    n_inst = box.shape[1]
    steps = (geo.wb, geo.hb, geo.db)
    ns = (geo.nx, geo.ny, geo.nz)
    everyone = np.arange(n_inst)
    rng = []
    for a in range(3):
        if modes[a] == "len":
            rng.append(_bin_range(box[2 * a], box[2 * a + 1], steps[a], ns[a]))
        else:
            eb, _ = _edge_bin(a, modes[a][0], modes[a][1], raw, geo, everyone)
            rng.append((eb, eb))
    span = np.stack([r[1] - r[0] + 1 for r in rng])
    small = (span <= _SMALL_SPAN).all(axis=0)
    out = np.zeros(n_inst)
    idx = np.nonzero(small)[0]
    for ox in range(_SMALL_SPAN):
        bx = rng[0][0][idx] + ox
        fx = np.where(bx <= rng[0][1][idx], _factor(modes[0], 0, bx, raw, box, geo, idx), 0.0)
        for oy in range(_SMALL_SPAN):
            by = rng[1][0][idx] + oy
            fy = np.where(by <= rng[1][1][idx], _factor(modes[1], 1, by, raw, box, geo, idx), 0.0)
            for oz in range(_SMALL_SPAN):
                bz = rng[2][0][idx] + oz
                fz = np.where(bz <= rng[2][1][idx], _factor(modes[2], 2, bz, raw, box, geo, idx), 0.0)
                f = fx * fy * fz
                hit = f != 0.0
                out[idx[hit]] += f[hit] * m[bz[hit], by[hit], bx[hit]]
    for i in np.nonzero(~small)[0]:
        fs = []
        for a in range(3):
            b = np.arange(rng[a][0][i], rng[a][1][i] + 1)
            fs.append(_factor(modes[a], a, b, raw, box, geo, np.full(b.shape, i)))
        sub = m[rng[2][0][i]:rng[2][1][i] + 1, rng[1][0][i]:rng[1][1][i] + 1, rng[0][0][i]:rng[0][1][i] + 1]
        out[i] = np.einsum("zyx,z,y,x->", sub, fs[2], fs[1], fs[0])
    return out


def field_gather(size, kind, xyz, ex, ey, ez, geo):
    """Gradient of the density penalty by the field gather: -omega sum_b vol(D ∩ b) E_b.

    Returns float64 [3][n]; fixed instances get zero.
    """
    raw, box, *_, omega = _edges(size, kind, xyz, geo)
    g = np.stack([-omega * _box_sum(e, raw, box, geo, ("len", "len", "len")) for e in (ex, ey, ez)])
    g[:, is_fixed(kind)] = 0.0
    return g


def density_vjp(size, kind, xyz, gmap, geo):
    """sum_b gmap[b] * d rho_b / d v_i for every instance (exact adjoint of ``density_map``).

    rho_b vol(b) = omega * Lx * Ly * Lz with L the overlap lengths of the stretched, clipped
    cuboid.  Planar derivatives move both edges of one axis; the z derivative moves both z
    edges and, for macros, the width and height through the linear size transition (and the
    weight omega when an extent is below the stretch threshold).  Cell sizes switch by a step in
    z and contribute no derivative.  Each derivative is one-sided, per the rule of the module
    docstring; the size-transition terms move the planar edges in the direction the z motion
    drives them (an upper edge with the sign of dw/dz, a lower edge against it).  Returns float64
    [3][n]; fixed instances get zero.
    """
    raw, box, below, w, h, wt, ht, omega = _edges(size, kind, xyz, geo)
    m = np.asarray(gmap, dtype=np.float64) / geo.vol_bin
    s = lambda modes: _box_sum(m, raw, box, geo, modes)  # noqa: E731
    L = "len"
    face = lambda a: (s(tuple((1, below[a]) if k == a else L for k in range(3)))      # noqa: E731
                      - s(tuple((0, below[a]) if k == a else L for k in range(3))))
    gx, gy, gz = omega * face(0), omega * face(1), omega * face(2)
    dw, dh = macro_size_slope(size, kind, geo.dz)
    z = np.asarray(xyz, dtype=np.float64)[2]
    zdown = below[2]
    # domain of the size transition: inside the movable range, its bounds included (the derivative
    # there is taken into the range)
    at_lo, at_hi = z_bands(z, geo.dz)
    inside = at_lo | at_hi | ((z > 0.25 * geo.dz) & (z < 0.75 * geo.dz))
    dw = np.where(inside, dw, 0.0)
    dh = np.where(inside, dh, 0.0)
    if np.any(dw != 0.0) or np.any(dh != 0.0):
        r2 = np.sqrt(2.0)
        stretched_w = w < r2 * geo.wb          # w~ fixed at sqrt2 w_b, omega grows with w
        stretched_h = h < r2 * geo.hb
        fw = np.minimum(1.0, w / (r2 * geo.wb))
        fh = np.minimum(1.0, h / (r2 * geo.hb))
        domega = (np.where(stretched_w, dw / (r2 * geo.wb), 0.0) * fh
                  + fw * np.where(stretched_h, dh / (r2 * geo.hb), 0.0))
        dwt = np.where(stretched_w, 0.0, dw)
        dht = np.where(stretched_h, 0.0, dh)
        gz = gz + domega * s((L, L, L))
        # the z motion moves an upper planar edge the way of dw/dz and the lower edge the other way
        up_w = zdown != (dwt < 0.0)            # upper x edge moving down
        up_h = zdown != (dht < 0.0)
        gz = gz + omega * 0.5 * dwt * (s(((1, up_w), L, L)) + s(((0, ~up_w), L, L)))
        gz = gz + omega * 0.5 * dht * (s((L, (1, up_h), L)) + s((L, (0, ~up_h), L)))
    g = np.stack([gx, gy, gz])
    g[:, is_fixed(kind)] = 0.0
    return g
