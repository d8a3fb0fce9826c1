"""The torch.autograd Functions over the C ABI (paper_2403_09070_amd.autograd) against the oracle.

* Field: the GPU solve is symmetric, <phi(a), b> = <a, phi(b)> (the property its backward uses).
* Density + Field: the gradient of U = 1/2 sum rho phi vol(b) through autograd equals the oracle's
  exact adjoint of the density map applied to phi vol(b) (Sec. III-A energy, reading 6).
* WAWirelength: forward value = the oracle's smoothed bistratal wirelength plus its z term; the
  backward returns the library's gradient scaled by the upstream gradient.
* The autograd gradient of U against central differences of the FP64 oracle's U (C1).
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


def test_wirelength_function():
    need_gpu()
    from paper_2403_09070_amd import autograd as ag
    case = synth.make_case("c1", 2403)
    geo = geometry_of(case)
    pb = oracle_problem(case)
    prob = gpu_problem(case)
    xyz = torch.from_numpy(case.xyz0).cuda().requires_grad_(True)
    w = ag.WAWirelength.apply(prob, xyz)
    (2.0 * w).backward()
    ref = owl.wirelength(pb.size, pb.kind, case.xyz0, pb.net_start, pb.pin2node, pb.pin_off, geo, pb.gamma, pb.alpha)
    want = ref["wa_bi"] + ref["wa_z"]
    w_gpu = float(w.detach())
    log(f"[autograd] wirelength gpu={w_gpu:.9g} ref={want:.9g}")
    assert abs(w_gpu - want) <= 1e-5 * abs(want)
    g, _ = prob.wl_grad(case.xyz0)
    assert torch.equal(xyz.grad, 2.0 * g)
    assert rel_l2(xyz.grad[:2].cpu().numpy(), 2.0 * ref["grad"][:2]) <= 1e-5


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
