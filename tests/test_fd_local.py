"""The local central differences of tests/fd_local.py against full evaluations of the FP64
oracle's U and W (so that the 200k-netlist check built on them measures the real objective)."""
import numpy as np

import fd_local
from oracle import density as oden
from oracle import optimizer as opt
from oracle import poisson as opois
from oracle import wirelength as owl
from oracle.geometry import geometry_of
from paper_2403_09070_amd import synth


def _energy(case, geo, v):
    rho = oden.density_map(case.size, case.kind, v, geo)
    return opois.energy(rho, opois.solve(rho, geo, want=("phi",))["phi"], geo)


def _probes(case, rng, k):
    mov = np.nonzero((case.kind & 2) == 0)[0]
    return [(int(rng.choice(mov)), int(rng.integers(0, 3))) for _ in range(k)]


def test_local_energy_difference_equals_the_full_one():
    case = synth.make_case("c1", 2403)
    geo = geometry_of(case)
    v = case.xyz0.astype(np.float64)
    rho = oden.density_map(case.size, case.kind, v, geo)
    phi = opois.solve(rho, geo, want=("phi",))["phi"]
    probes = _probes(case, np.random.default_rng(3), 40)
    h = 1e-3 * geo.wb
    c, up, dn = fd_local.energy_differences(case, geo, phi, v, probes, h)
    checked = 0
    u0 = _energy(case, geo, v)
    for k, (i, a) in enumerate(probes):
        if abs(up[k] - dn[k]) > 1e-3 * max(abs(c[k]), 1e-12):
            continue                                   # a kink in the stencil: not an identity there
        vp, vm = v.copy(), v.copy()
        vp[a, i] += h
        vm[a, i] -= h
        full = (_energy(case, geo, vp) - _energy(case, geo, vm)) / (2 * h)
        # the full difference carries the float64 rounding of U itself, ~1e-16 |U| / h
        assert abs(c[k] - full) <= 1e-7 * abs(full) + 1e-13 * abs(u0) / h, (i, a, c[k], full)
        checked += 1
    assert checked >= 30


def test_local_wirelength_difference_equals_the_full_one():
    case = synth.make_case("c1", 2403)
    pb = opt.problem_of(case)
    v = case.xyz0.astype(np.float64)
    probes = _probes(case, np.random.default_rng(4), 30)
    h = 1e-3 * pb.geo.wb
    c, _, _ = fd_local.wirelength_differences(pb, v, probes, h)

    def full(p):
        out = owl.wirelength(pb.size, pb.kind, p, pb.net_start, pb.pin2node, pb.pin_off, pb.geo, pb.gamma, pb.alpha)
        return out["wa_bi"] + out["wa_z"]

    for k, (i, a) in enumerate(probes):
        vp, vm = v.copy(), v.copy()
        vp[a, i] += h
        vm[a, i] -= h
        f = (full(vp) - full(vm)) / (2 * h)
        assert abs(c[k] - f) <= 1e-6 * max(1.0, abs(f)), (i, a, c[k], f)
