"""Central differences of the FP64 oracle's objective parts, evaluated locally (test helper).

A probe moves one coordinate a of one instance i by +-h.  Only what depends on that instance is
re-evaluated, which makes thousands of probes affordable on the 200k-instance netlist:

* Energy U = 1/2 sum_b rho_b phi_b vol(b) (quadratic in rho, rho(v) the oracle's density map):
  U(v + d) - U(v) = <phi, D> vol(b) + 1/2 <D, K D> vol(b), D = rho(v + d) - rho(v), K the solve.
  Between kinks an instance's density share is linear in its planar coordinates (D(-h) = -D(h)),
  so the second-order terms cancel in the central difference, which is then exactly
  <phi, rho_i(v + h e) - rho_i(v - h e)> vol(b) / (2h).  <phi, rho_i> vol(b) is minus the oracle's
  field gather of the map phi.  A macro's z enters quadratically (its size moves with z): there the
  identity holds to O(h^2).  tests/test_fd_local.py checks it against full evaluations of U.
* Wirelength W = sum_e (W^_e(x) + W^_e(y) + alpha p^_e(z)): only the nets of instance i change;
  they are re-evaluated by the oracle on a netlist holding just those nets.

Each probe also reports its two one-sided differences; where they disagree (an edge crossing a
bin face, the die switch at d_z/2, a bistratal branch switch inside the stencil) the probe sits on
a kink and is reported rather than assessed.
"""
from __future__ import annotations

import numpy as np

from oracle import density_grad as odg
from oracle import wirelength as owl


def _share(case, geo, phi, idx, xyz):
    """<phi, rho_i> vol(b) for the instances idx at positions xyz[:, k] (k-th probe)."""
    g = odg.field_gather(case.size[:, idx], case.kind[idx], xyz, phi, phi, phi, geo)
    return -g[0]


def energy_differences(case, geo, phi, v, probes, h):
    """(central, up, down) differences of U for probes [(i, a), ...] at the placement v."""
    idx = np.array([i for i, _ in probes])
    ax = np.array([a for _, a in probes])
    base = v[:, idx].copy()
    up, dn = base.copy(), base.copy()
    k = np.arange(len(probes))
    up[ax, k] += h
    dn[ax, k] -= h
    s0 = _share(case, geo, phi, idx, base)
    sp = _share(case, geo, phi, idx, up)
    sm = _share(case, geo, phi, idx, dn)
    return (sp - sm) / (2 * h), (sp - s0) / h, (s0 - sm) / h


def wirelength_differences(pb, v, probes, h):
    """(central, up, down) differences of W (x, y smoothed bistratal plus alpha p^(z)) per probe.
    The oracle evaluates the probed instance's nets on a sub-problem holding just their instances."""
    ns = np.asarray(pb.net_start, dtype=np.int64)
    p2n = np.asarray(pb.pin2node, dtype=np.int64)
    off = np.asarray(pb.pin_off, dtype=np.float64)
    size = np.asarray(pb.size, dtype=np.float64)
    net_of_pin = np.repeat(np.arange(len(ns) - 1), np.diff(ns))
    order = np.argsort(p2n, kind="stable")
    first = np.searchsorted(p2n[order], np.arange(v.shape[1] + 1))
    c, u, d = [], [], []
    for i, a in probes:
        nets = np.unique(net_of_pin[order[first[i]:first[i + 1]]])
        if len(nets) == 0:                      # on no net: W does not depend on it
            c.append(0.0); u.append(0.0); d.append(0.0)
            continue
        pins = np.concatenate([np.arange(ns[e], ns[e + 1]) for e in nets]) if len(nets) else np.zeros(0, np.int64)
        sns = np.zeros(len(nets) + 1, dtype=np.int64)
        np.cumsum(ns[nets + 1] - ns[nets], out=sns[1:])
        members, local = np.unique(p2n[pins], return_inverse=True)
        me = int(np.searchsorted(members, i))
        sub_v = v[:, members].copy()

        def total(x):
            sub_v[a, me] = x
            out = owl.wirelength(size[:, members], pb.kind[members], sub_v, sns, local, off[:, pins], pb.geo,
                                 pb.gamma, pb.alpha)
            return out["wa_bi"] + out["wa_z"]

        x0 = v[a, i]
        w0, wp, wm = total(x0), total(x0 + h), total(x0 - h)
        c.append((wp - wm) / (2 * h))
        u.append((wp - w0) / h)
        d.append((w0 - wm) / h)
    return np.array(c), np.array(u), np.array(d)


def jacobian_l1(case, geo, v, probes):
    """sum_b |d rho_b / d v_a,i| vol(b) per probe (i, a): the l1 norm of the density-Jacobian
    column, from the stretched, clipped cuboid of the oracle's attributes.  Moving a planar
    coordinate moves its two edges, each changing the overlap of one layer of bins by the cross
    extent (omega L_y L_z per edge along x); z likewise, and a macro's z also moves the planar
    edges (half the size slope each) and, for an extent below the stretch threshold, omega."""
    from oracle.attributes import instance_size, macro_size_slope, smoothing
    idx = np.array([i for i, _ in probes])
    ax = np.array([a for _, a in probes])
    xyz = np.asarray(v, dtype=np.float64)[:, idx]
    size, kind = case.size[:, idx], case.kind[idx]
    w, h = instance_size(size, kind, xyz[2], geo.dz)
    wt, ht, omega = smoothing(w, h, geo.wb, geo.hb)
    lx = np.clip(xyz[0] + 0.5 * wt, 0, geo.die_x) - np.clip(xyz[0] - 0.5 * wt, 0, geo.die_x)
    ly = np.clip(xyz[1] + 0.5 * ht, 0, geo.die_y) - np.clip(xyz[1] - 0.5 * ht, 0, geo.die_y)
    lz = np.clip(xyz[2] + 0.25 * geo.dz, 0, geo.dz) - np.clip(xyz[2] - 0.25 * geo.dz, 0, geo.dz)
    dw, dh = macro_size_slope(size, kind, geo.dz)
    r2 = np.sqrt(2.0)
    domega = np.abs(dw) / (r2 * geo.wb) + np.abs(dh) / (r2 * geo.hb)
    out = np.where(ax == 0, 2 * omega * ly * lz, np.where(ax == 1, 2 * omega * lx * lz, 2 * omega * lx * ly))
    zsize = domega * lx * ly * lz + omega * (np.abs(dw) * ly * lz + np.abs(dh) * lx * lz)
    return out + np.where(ax == 2, zsize, 0.0)


def assess(g, central, up, down, kink_tol=1e-2, extra=0.0):
    """Bound |g - g_FD| <= 1e-4 |g_FD| + 1e-5 median|g| (+ extra, per probe) on the probes off
    kinks.  A kink turns the derivative by an amount of the order of the gradient inside the
    stencil, so the one-sided differences then disagree by more than kink_tol (|g_FD| +
    median|g|); smooth curvature moves them apart by h |f''| only.  Returns (n_ok, n_assessed,
    n_kinks, worst ratio of error to bound)."""
    g = np.asarray(g, dtype=np.float64)
    med = float(np.median(np.abs(g))) if g.size else 0.0
    kink = np.abs(up - down) > kink_tol * (np.abs(central) + med)
    bound = 1e-4 * np.abs(central) + 1e-5 * med + extra
    err = np.abs(g - central)
    assessed = ~kink
    ok = assessed & (err <= bound)
    worst = float(np.max(err[assessed] / np.maximum(bound[assessed], 1e-300))) if assessed.any() else 0.0
    return int(ok.sum()), int(assessed.sum()), int(kink.sum()), worst
