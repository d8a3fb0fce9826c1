"""The torch.autograd Functions over the C ABI (paper_2403_09070_amd.autograd) against the oracle.

* Field: the GPU solve is symmetric, <phi(a), b> = <a, phi(b)> (the property its backward uses).
* DensityEnergy: U = 1/2 sum rho phi vol(b) reduced in float64 by the library equals the oracle's,
  and its gradient equals the oracle's exact adjoint of the density map applied to phi vol(b)
  (Sec. III-A energy, reading 6).
* WAWirelength: forward value = the oracle's smoothed bistratal wirelength plus its z term (no
  gradient computed, nothing stored per pin); the backward recomputes the sums and returns the
  paper's gradient (FDA z part) or the value's own derivative, scaled by the incoming gradient.
* The autograd gradients against central differences of the FP64 oracle's U and W: C1 with full
  evaluations, and the 200k-instance netlist on 1,000 instances x {x, y, z} (3,000 coordinates)
  with the local differences of tests/fd_local.py.
"""
import numpy as np
import pytest
import torch

from gpu_common import gpu_problem, log, need_gpu, oracle_problem, rel_l2, tiny_case
from oracle import density as oden
from oracle import density_grad as odg
from oracle import poisson as opois
from oracle import wirelength as owl
from oracle.geometry import geometry_of
from paper_2403_09070_amd import place3d, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [place3d.FP32, place3d.BF16X3])
def test_field_is_symmetric(precision):
    need_gpu()
    from paper_2403_09070_amd import autograd as ag
    case = synth.make_case("c1", 2403)
    prob = gpu_problem(case, precision=precision)
    g = torch.Generator().manual_seed(5)
    a = torch.randn((case.nz, case.ny, case.nx), generator=g).cuda()
    b = torch.randn((case.nz, case.ny, case.nx), generator=g).cuda()
    pa = ag.Field.apply(prob, a)
    pb = ag.Field.apply(prob, b)
    lhs, rhs = float((pa.double() * b.double()).sum()), float((a.double() * pb.double()).sum())
    scale = float(pa.double().norm() * b.double().norm())
    log(f"[autograd] field symmetry precision={precision} |lhs-rhs|/scale={abs(lhs - rhs) / scale:.3e}")
    assert abs(lhs - rhs) <= 1e-5 * scale


@pytest.mark.parametrize("which", ["tiny", "c1"])
def test_density_energy_gradient_matches_the_oracle_adjoint(which):
    need_gpu()
    from paper_2403_09070_amd import autograd as ag
    case = tiny_case(5) if which == "tiny" else synth.make_case("c1", 2403)
    geo = geometry_of(case)
    prob = gpu_problem(case)
    xyz = torch.from_numpy(case.xyz0).cuda().requires_grad_(True)
    u = ag.density_energy(prob, xyz)
    u.backward()
    rho = oden.density_map(case.size, case.kind, case.xyz0, geo)
    phi = opois.solve(rho, geo, want=("phi",))["phi"]
    ref = odg.density_vjp(case.size, case.kind, case.xyz0, phi * geo.vol_bin, geo)
    e_ref = opois.energy(rho, phi, geo)
    e_gpu = float(u.detach())
    err = rel_l2(xyz.grad.cpu().numpy(), ref)
    log(f"[autograd] {which} energy gpu={e_gpu:.9g} ref={e_ref:.9g} grad rel_l2={err:.3e}")
    assert abs(e_gpu - e_ref) <= 1e-4 * abs(e_ref)
    assert err <= 1e-4


@pytest.mark.parametrize("precision", [place3d.FP32, place3d.BF16X3])
def test_wirelength_function(precision):
    need_gpu()
    from paper_2403_09070_amd import autograd as ag
    case = synth.make_case("c1", 2403)
    geo = geometry_of(case)
    pb = oracle_problem(case)
    prob = gpu_problem(case, precision=precision)
    ref = owl.wirelength(pb.size, pb.kind, case.xyz0, pb.net_start, pb.pin2node, pb.pin_off, geo, pb.gamma, pb.alpha)
    want = ref["wa_bi"] + ref["wa_z"]
    g_lib, met = prob.wl_grad(case.xyz0)
    for fda in (True, False):
        xyz = torch.from_numpy(case.xyz0).cuda().requires_grad_(True)
        w = ag.wirelength(prob, xyz, fda=fda)
        (2.0 * w).backward()
        w_gpu = float(w.detach())
        g = xyz.grad.cpu().numpy()
        e_xy = rel_l2(g[:2], 2.0 * ref["grad"][:2])
        e_z = rel_l2(g[2], 2.0 * (ref["grad"][2] if fda else ref["grad_zwa"]))
        log(f"[autograd] wirelength precision={precision} fda={fda} gpu={w_gpu:.12g} ref={want:.12g} "
            f"grad xy rel_l2={e_xy:.3e} z rel_l2={e_z:.3e}")
        assert abs(w_gpu - want) <= 1e-5 * abs(want)
        assert e_xy <= 1e-5
        if fda:     # the paper's z-gradient, the same kernels as place3d_wl_grad
            assert torch.equal(xyz.grad, 2.0 * g_lib)
        else:       # the derivative of the value: alpha dp^(z)/dz
            assert e_z <= 1e-5
    # the value call writes the net totals only; it is a separately compiled instance of the net
    # kernel (no per-pin phase), whose float32 contractions may round differently: 1e-6 relative
    m = prob.wl_value(case.xyz0).cpu().numpy()
    mg = met.cpu().numpy()[:5]
    assert np.all(np.abs(m[:5] - mg) <= 1e-6 * np.abs(mg))
    assert np.all(m[5:] == 0.0)


def test_energy_gradient_matches_fp64_finite_differences():
    """The GPU autograd gradient of U (exact adjoint through Density and Field) against central
    differences of the FP64 oracle's U, h = 1e-3 bin widths, on 300 sampled movable coordinates of
    C1: |g - g_FD| <= 1e-4 |g_FD| + 1e-5 median|g| for at least 99 % of them (a difference can
    straddle a kink of the overlap lengths, where an edge crosses a bin boundary)."""
    need_gpu()
    from paper_2403_09070_amd import autograd as ag
    case = synth.make_case("c1", 2403)
    geo = geometry_of(case)
    prob = gpu_problem(case)
    xyz = torch.from_numpy(case.xyz0).cuda().requires_grad_(True)
    ag.density_energy(prob, xyz).backward()
    g = xyz.grad.cpu().numpy().astype(np.float64)

    def energy(v):
        rho = oden.density_map(case.size, case.kind, v, geo)
        return opois.energy(rho, opois.solve(rho, geo, want=("phi",))["phi"], geo)

    rng = np.random.default_rng(7)
    movable = np.nonzero((case.kind & place3d.KIND_FIXED) == 0)[0]
    v0 = case.xyz0.astype(np.float64)
    h = 1e-3 * geo.wb
    med = float(np.median(np.abs(g[:, movable])))
    ok = total = 0
    for _ in range(300):
        i = int(rng.choice(movable))
        a = int(rng.integers(0, 3))
        if a == 2 and abs(v0[2, i] - 0.5 * geo.dz) < 2 * h:      # the per-die size switch
            continue
        vp, vm = v0.copy(), v0.copy()
        vp[a, i] += h
        vm[a, i] -= h
        fd = (energy(vp) - energy(vm)) / (2 * h)
        total += 1
        ok += abs(g[a, i] - fd) <= 1e-4 * abs(fd) + 1e-5 * med
    log(f"[autograd] FD check: {ok}/{total} within the bound")
    assert ok >= 0.99 * total


def test_c3_gradients_match_fp64_finite_differences_on_the_200k_netlist():
    """The differentiation form at the 200k-instance netlist (C3: 200k cells + 40 macros, 220k nets,
    512 x 512 x 4 bins; float32 spectral solve): the autograd gradients of U (DensityEnergy) and W
    (WAWirelength, its value's own z-derivative) on 1,000 random movable instances x {x, y, z},
    3,000 coordinates each, against central differences (h = 1e-3 bin widths) of the FP64 oracle's U
    and W: |g - g_FD| <= 1e-4 |g_FD| + 1e-5 median|g| on at least 99 % of the coordinates off
    kinks; kinks (one-sided differences that disagree) are counted and reported.  The U gradient
    also matches the oracle's exact adjoint over all instances (1e-4 rel L2).  The U bound adds
    what the float32 potential can move a gradient: the largest error of the GPU's float32 phi
    against the oracle's times the l1 norm of the instance's density-Jacobian column."""
    need_gpu()
    import fd_local
    from paper_2403_09070_amd import autograd as ag
    case = synth.make_case("c2", 2403)
    geo = geometry_of(case)
    pb = oracle_problem(case)
    prob = gpu_problem(case, precision=place3d.FP32, dgrad=place3d.DGRAD_ADJOINT)
    xyz = torch.from_numpy(case.xyz0).cuda().requires_grad_(True)
    u = ag.density_energy(prob, xyz)
    (g_u,) = torch.autograd.grad(u, xyz)
    w = ag.wirelength(prob, xyz, fda=False)
    (g_w,) = torch.autograd.grad(w, xyz)
    g_u = g_u.cpu().numpy().astype(np.float64)
    g_w = g_w.cpu().numpy().astype(np.float64)
    log("[autograd] c3: GPU gradients done, oracle density and potential")
    v = case.xyz0.astype(np.float64)
    rho = oden.density_map(case.size, case.kind, v, geo)
    phi = opois.solve(rho, geo, want=("phi",))["phi"]
    e_ref = opois.energy(rho, phi, geo)
    log(f"[autograd] c3 energy gpu={float(u):.9g} ref={e_ref:.9g}")
    assert abs(float(u) - e_ref) <= 1e-5 * abs(e_ref)
    ref_adj = odg.density_vjp(case.size, case.kind, v, phi * geo.vol_bin, geo)
    err_adj = rel_l2(g_u, ref_adj)
    log(f"[autograd] c3 dU/dxyz vs oracle adjoint rel_l2={err_adj:.3e}")
    assert err_adj <= 1e-4
    rng = np.random.default_rng(2403)
    movable = np.nonzero((case.kind & place3d.KIND_FIXED) == 0)[0]
    inst = rng.choice(movable, size=1000, replace=False)
    probes = [(int(i), a) for i in inst for a in range(3)]
    h = 1e-3 * geo.wb
    c, up, dn = fd_local.energy_differences(case, geo, phi, v, probes, h)
    gu = np.array([g_u[a, i] for i, a in probes])
    # the GPU gradient is <phi_32, d rho / d v> vol(b) with the float32 potential of the float32
    # solve: its error is at most max|phi_32 - phi| times the l1 norm of the density Jacobian
    # column (plus the float32 accumulation), which at this grid exceeds 1e-4 |g| for many cells
    # (phi ~ 2e4 against face differences ~ 1e2; phi rounded to float32 alone fails the bare bound
    # on 2.5 % of these coordinates)
    phi32 = prob.field(prob.density(xyz.detach()), want=("phi",))["phi"].cpu().numpy().astype(np.float64)
    dphi = float(np.max(np.abs(phi32 - phi))) + 4.0 * 2.0 ** -24 * float(np.max(np.abs(phi)))
    l1 = fd_local.jacobian_l1(case, geo, v, probes)
    log(f"[autograd] c3 max|phi_32 - phi| = {dphi:.3e} (max|phi| {np.max(np.abs(phi)):.3e})")
    ok, assessed, kinks, worst = fd_local.assess(gu, c, up, dn, extra=dphi * l1)
    log(f"[autograd] c3 U: {ok}/{assessed} coordinates within the bound, {kinks} on kinks, worst error/bound {worst:.3f}")
    assert assessed >= 0.9 * len(probes) and ok >= 0.99 * assessed
    # W: skip z probes whose stencil crosses the die switch at d_z/2 (a step of the bistratal part)
    wprobes = [(i, a) for i, a in probes if not (a == 2 and abs(v[2, i] - 0.5 * geo.dz) < 2 * h)]
    c, up, dn = fd_local.wirelength_differences(pb, v, wprobes, h)
    gw = np.array([g_w[a, i] for i, a in wprobes])
    ok, assessed, kinks, worst = fd_local.assess(gw, c, up, dn)
    log(f"[autograd] c3 W: {ok}/{assessed} coordinates within the bound, {kinks} on kinks, worst error/bound {worst:.3f}")
    assert assessed >= 0.9 * len(wprobes) and ok >= 0.99 * assessed
