"""Density-penalty gradients: the paper's field gather and the exact adjoint of the density map.

Field gather (Sec. III-A: the gradient of the penalty is the charge times the field, gathered
from the overlapped bins in the backward phase of Sec. IV-A):

    dU/dv_i = - omega_i * sum_b vol(D_i ∩ b) * E_b          (per axis)

Reading of the sign: the paper names q_i E_i both the force and the gradient; the force is
+q_i E_i, so the gradient is its negative, and gradient descent spreads the charges.  For macros
the change of size with z is ignored here (force = charge x field).  This is not the derivative
of any discrete objective: parity unpinned beyond the properties its tests check.

Exact adjoint (the differentiation form): sum_b g_b d rho_b / d v_i for a map g, including the
z-dependence of the macro size transition and of the local-smoothness weight.  With
g = phi vol(b) it is the exact gradient of U = 1/2 sum rho phi vol(b).
"""
from __future__ import annotations

import numpy as np

from .attributes import instance_size, is_fixed, macro_size_slope, smoothing
from .density import _bin_range, _SMALL_SPAN, axis_overlap


def _edges(size, kind, xyz, geo):
    """Raw (unclipped) cuboid edges, clipped edges, weight and stretch data per instance."""
    xyz = np.asarray(xyz, dtype=np.float64)
    w, h = instance_size(size, kind, xyz[2], geo.dz)
    wt, ht, omega = smoothing(w, h, geo.wb, geo.hb)
    raw = np.stack([xyz[0] - 0.5 * wt, xyz[0] + 0.5 * wt, xyz[1] - 0.5 * ht, xyz[1] + 0.5 * ht,
                    xyz[2] - 0.25 * geo.dz, xyz[2] + 0.25 * geo.dz])
    lim = np.array([geo.die_x, geo.die_x, geo.die_y, geo.die_y, geo.dz, geo.dz])[:, None]
    box = np.clip(raw, 0.0, lim)
    free = (raw > 0.0) & (raw < lim)
    return raw, box, free, w, h, wt, ht, omega


def _factor(mode, a, b, raw, box, free, step, n, sel):
    """Per-bin factor along one axis for bins b of the selected instances.

    'len': overlap length; 'lo'/'hi': 1 on the bin holding the lower/upper edge, if that edge is
    not clipped by the region (the derivative of the overlap length with respect to the edge).
    """
    lo, hi = box[2 * a, sel], box[2 * a + 1, sel]
    if mode == "len":
        return axis_overlap(lo, hi, b, step)
    e = 0 if mode == "lo" else 1
    edge = raw[2 * a + e, sel]
    eb = np.clip(np.floor(edge / step).astype(np.int64), 0, n - 1)
    return np.where((b == eb) & free[2 * a + e, sel], 1.0, 0.0)


def _box_sum(m, raw, box, free, geo, modes):
    """sum_b m[b] * Fx(bx) Fy(by) Fz(bz) for every instance, F chosen by ``modes`` (x, y, z)."""
    m = np.asarray(m, dtype=np.float64)
    n_inst = box.shape[1]
    steps = (geo.wb, geo.hb, geo.db)
    ns = (geo.nx, geo.ny, geo.nz)
    rng = [_bin_range(box[2 * a], box[2 * a + 1], steps[a], ns[a]) for a in range(3)]
    span = np.stack([r[1] - r[0] + 1 for r in rng])
    small = (span <= _SMALL_SPAN).all(axis=0)
    out = np.zeros(n_inst)
    idx = np.nonzero(small)[0]
    for ox in range(_SMALL_SPAN):
        bx = rng[0][0][idx] + ox
        fx = np.where(bx <= rng[0][1][idx],
                      _factor(modes[0], 0, bx, raw, box, free, geo.wb, geo.nx, idx), 0.0)
        for oy in range(_SMALL_SPAN):
            by = rng[1][0][idx] + oy
            fy = np.where(by <= rng[1][1][idx],
                          _factor(modes[1], 1, by, raw, box, free, geo.hb, geo.ny, idx), 0.0)
            for oz in range(_SMALL_SPAN):
                bz = rng[2][0][idx] + oz
                fz = np.where(bz <= rng[2][1][idx],
                              _factor(modes[2], 2, bz, raw, box, free, geo.db, geo.nz, idx), 0.0)
                f = fx * fy * fz
                hit = f != 0.0
                out[idx[hit]] += f[hit] * m[bz[hit], by[hit], bx[hit]]
    for i in np.nonzero(~small)[0]:
        fs = []
        for a in range(3):
            b = np.arange(rng[a][0][i], rng[a][1][i] + 1)
            fs.append(_factor(modes[a], a, b, raw, box, free, steps[a], ns[a], np.full(b.shape, i)))
        sub = m[rng[2][0][i]:rng[2][1][i] + 1, rng[1][0][i]:rng[1][1][i] + 1, rng[0][0][i]:rng[0][1][i] + 1]
        out[i] = np.einsum("zyx,z,y,x->", sub, fs[2], fs[1], fs[0])
    return out


def field_gather(size, kind, xyz, ex, ey, ez, geo):
    """Gradient of the density penalty by the field gather: -omega sum_b vol(D ∩ b) E_b.

    Returns float64 [3][n]; fixed instances get zero.
    """
    raw, box, free, *_, omega = _edges(size, kind, xyz, geo)
    g = np.stack([-omega * _box_sum(e, raw, box, free, geo, ("len", "len", "len"))
                  for e in (ex, ey, ez)])
    g[:, is_fixed(kind)] = 0.0
    return g


def density_vjp(size, kind, xyz, gmap, geo):
    """sum_b gmap[b] * d rho_b / d v_i for every instance (exact adjoint of ``density_map``).

    rho_b vol(b) = omega * Lx * Ly * Lz with L the overlap lengths of the stretched, clipped
    cuboid.  Planar derivatives move both edges of one axis; the z derivative moves both z
    edges and, for macros, the width and height through the linear size transition (and the
    weight omega when an extent is below the stretch threshold).  Cell sizes switch by a step in
    z and contribute no derivative.  Returns float64 [3][n]; fixed instances get zero.
    """
    raw, box, free, w, h, wt, ht, omega = _edges(size, kind, xyz, geo)
    m = np.asarray(gmap, dtype=np.float64) / geo.vol_bin
    s = lambda modes: _box_sum(m, raw, box, free, geo, modes)  # noqa: E731
    gx = omega * (s(("hi", "len", "len")) - s(("lo", "len", "len")))
    gy = omega * (s(("len", "hi", "len")) - s(("len", "lo", "len")))
    gz = omega * (s(("len", "len", "hi")) - s(("len", "len", "lo")))
    dw, dh = macro_size_slope(size, kind, geo.dz)
    z = np.asarray(xyz, dtype=np.float64)[2]
    inside = (z >= 0.25 * geo.dz) & (z <= 0.75 * geo.dz)   # domain of the size transition
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
        gz = gz + domega * s(("len", "len", "len"))
        gz = gz + omega * 0.5 * dwt * (s(("hi", "len", "len")) + s(("lo", "len", "len")))
        gz = gz + omega * 0.5 * dht * (s(("len", "hi", "len")) + s(("len", "lo", "len")))
    g = np.stack([gx, gy, gz])
    g[:, is_fixed(kind)] = 0.0
    return g
