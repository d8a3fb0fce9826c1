"""Wirelength: WA model, bistratal D2D wirelength and its finite-difference z-gradient.

* WA extent of a pin set along one axis (Eq. wa-model-approx), with its per-pin derivative.
* Minimal D2D wirelength of a net per axis, max{p_e, p_e+ + p_e-} (Eqs. optimal-region and
  wl-obj); the bistratal wirelength is its x plus y part and the full model adds alpha p_e(z)
  (Eq. wl-model).  The smoothed model applies WA to each p inside the max.
* The z-gradient of the bistratal wirelength by finite differences (Eq. fda-grad): for every
  instance, the exact bistratal wirelength with the instance on the top die minus that with it
  on the bottom die, times 4/d_z, here computed the vanilla way (every flipped net re-scanned,
  Sec. IV-B), then normalised to the planar gradient's scale (Eq. fda-normalize).  An instance
  with several pins on one net moves all of them when it changes die, and that net's difference
  counts once for it.

Readings: the WA sums are shifted by the set's max (min) before exponentiation, which leaves the
model unchanged and keeps exp finite; an empty set or a single pin has extent 0.  The smoothed
max compares the smoothed branch values and takes the whole-net branch on an exact tie or when
the net does not cross the dies.  The finite difference uses the exact (unsmoothed) wirelength.
The normalising L1 norms run over movable instances; if the FDA gradient is zero everywhere,
the normalised gradient is zero.  Fixed instances get no gradient.
"""
from __future__ import annotations

import numpy as np

from .attributes import is_fixed, partition


def degree_classes(net_start):
    """Yield (d, net indices, pin index matrix [n_nets_of_degree_d, d]) for every degree d."""
    net_start = np.asarray(net_start, dtype=np.int64)
    deg = np.diff(net_start)
    for d in np.unique(deg):
        nets = np.nonzero(deg == d)[0]
        yield int(d), nets, net_start[nets][:, None] + np.arange(int(d))[None, :]


def wa_extent(u, mask, gamma):
    """Weighted-average extent over the masked members of each row, and d extent / d u."""
    u = np.asarray(u, dtype=np.float64)
    nonempty = mask.any(axis=1)
    hi = np.where(nonempty, np.max(np.where(mask, u, -np.inf), axis=1), 0.0)
    lo = np.where(nonempty, np.min(np.where(mask, u, np.inf), axis=1), 0.0)
    ep = np.where(mask, np.exp((u - hi[:, None]) / gamma), 0.0)
    em = np.where(mask, np.exp(-(u - lo[:, None]) / gamma), 0.0)
    sp = np.where(nonempty, ep.sum(axis=1), 1.0)
    sm = np.where(nonempty, em.sum(axis=1), 1.0)
    ap = (np.where(mask, u, 0.0) * ep).sum(axis=1) / sp
    am = (np.where(mask, u, 0.0) * em).sum(axis=1) / sm
    p = np.where(nonempty, ap - am, 0.0)
    grad = (ep / sp[:, None]) * (1.0 + (u - ap[:, None]) / gamma) \
        - (em / sm[:, None]) * (1.0 - (u - am[:, None]) / gamma)
    return p, np.where(mask, grad, 0.0)


def exact_extent(u, mask):
    """max - min over the masked members of each row (0 for an empty row)."""
    nonempty = mask.any(axis=1)
    hi = np.max(np.where(mask, u, -np.inf), axis=1)
    lo = np.min(np.where(mask, u, np.inf), axis=1)
    return np.where(nonempty, hi - lo, 0.0)


def bistratal_exact(u, top):
    """Minimal D2D wirelength along one axis: max{p_e, p_e+ + p_e-} (Eq. wl-obj)."""
    whole = exact_extent(u, np.ones_like(top))
    return np.maximum(whole, exact_extent(u, top) + exact_extent(u, ~top))


def bistratal_smoothed(u, top, gamma):
    """Smoothed bistratal wirelength along one axis and its per-pin derivative."""
    p_e, g_e = wa_extent(u, np.ones_like(top), gamma)
    p_t, g_t = wa_extent(u, top, gamma)
    p_b, g_b = wa_extent(u, ~top, gamma)
    crossing = top.any(axis=1) & (~top).any(axis=1)
    split = p_t + p_b
    use_split = crossing & (split > p_e)
    w = np.where(use_split, split, p_e)
    grad = np.where(use_split[:, None], np.where(top, g_t, g_b), g_e)
    return w, grad


def wirelength(size, kind, xyz, net_start, pin2node, pin_off, geo, gamma, alpha):
    """Wirelength values and gradients of every net, summed per instance.

    Returns a dict with
      wa_bi     sum of smoothed bistratal wirelength (x + y)
      wa_z      alpha * sum of WA p_e(z)
      hpwl_d2d  sum of exact bistratal (= minimal D2D) wirelength
      hpwl_3d   sum of p_e(x) + p_e(y) + alpha p_e(z) over the whole-net boxes (Def. 3d-hpwl)
      ncut      number of nets with pins on both dies
      grad_x, grad_y   smoothed bistratal gradient per instance
      fda       (4/d_z) (W_top - W_bot) per instance, summed over its nets (Eq. fda-grad)
      grad_zwa  alpha * d p^_e(z) / d z per instance
      fda_scale (|grad_x|_1 + |grad_y|_1) / (2 |fda|_1)     (Eq. fda-normalize)
      grad      [3][n]: grad_x, grad_y, fda_scale * fda + grad_zwa
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    node = np.asarray(pin2node, dtype=np.int64)
    off = np.asarray(pin_off, dtype=np.float64)
    n = xyz.shape[1]
    dz = geo.dz
    fixed = is_fixed(kind)
    top_node = partition(xyz[2], dz)

    gx = np.zeros(n)
    gy = np.zeros(n)
    gzwa = np.zeros(n)
    fda = np.zeros(n)
    tot = dict(wa_bi=0.0, wa_z=0.0, hpwl_d2d=0.0, hpwl_3d=0.0, ncut=0)
    for d, nets, pins in degree_classes(net_start):
        nd = node[pins]
        top = top_node[nd]
        ux = xyz[0, nd] + np.where(top, off[2, pins], off[0, pins])
        uy = xyz[1, nd] + np.where(top, off[3, pins], off[1, pins])
        uz = xyz[2, nd]
        # pin positions after flipping the owner to the other die
        fx = xyz[0, nd] + np.where(top, off[0, pins], off[2, pins])
        fy = xyz[1, nd] + np.where(top, off[1, pins], off[3, pins])

        wxs, gpx = bistratal_smoothed(ux, top, gamma)
        wys, gpy = bistratal_smoothed(uy, top, gamma)
        pz, gpz = wa_extent(uz, np.ones_like(top), gamma)
        np.add.at(gx, nd.ravel(), gpx.ravel())
        np.add.at(gy, nd.ravel(), gpy.ravel())
        np.add.at(gzwa, nd.ravel(), alpha * gpz.ravel())

        w_now = bistratal_exact(ux, top) + bistratal_exact(uy, top)
        everyone = np.ones_like(top)
        tot["wa_bi"] += float(np.sum(wxs + wys))
        tot["wa_z"] += alpha * float(np.sum(pz))
        tot["hpwl_d2d"] += float(np.sum(w_now))
        tot["hpwl_3d"] += float(np.sum(exact_extent(ux, everyone) + exact_extent(uy, everyone)
                                       + alpha * exact_extent(uz, everyone)))
        tot["ncut"] += int(np.sum(top.any(axis=1) & (~top).any(axis=1)))

        # vanilla FDA: re-evaluate the whole net with member k's instance on the other die (all
        # of that instance's pins on the net move with it); an instance with several pins on the
        # net counts once, at its first member
        for k in range(d):
            same = nd == nd[:, k:k + 1]                       # members owned by k's instance
            first = ~same[:, :k].any(axis=1)
            t2 = np.where(same, ~top, top)
            ux2 = np.where(same, fx, ux)
            uy2 = np.where(same, fy, uy)
            w_flip = bistratal_exact(ux2, t2) + bistratal_exact(uy2, t2)
            w_top = np.where(top[:, k], w_now, w_flip)
            w_bot = np.where(top[:, k], w_flip, w_now)
            np.add.at(fda, nd[:, k], np.where(first, (4.0 / dz) * (w_top - w_bot), 0.0))

    for g in (gx, gy, gzwa, fda):
        g[fixed] = 0.0
    nrm_xy = float(np.abs(gx).sum() + np.abs(gy).sum())
    nrm_f = float(np.abs(fda).sum())
    scale = nrm_xy / (2.0 * nrm_f) if nrm_f > 0.0 else 0.0
    out = dict(tot)
    out.update(grad_x=gx, grad_y=gy, fda=fda, grad_zwa=gzwa, fda_scale=scale,
               norm_x=float(np.abs(gx).sum()), norm_y=float(np.abs(gy).sum()), norm_fda=nrm_f,
               grad=np.stack([gx, gy, scale * fda + gzwa]))
    return out
