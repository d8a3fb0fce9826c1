"""GPU-vs-oracle parity of every hot-path call through the C ABI.

Inputs are the seeded synthetic cases; where a stage is compared in isolation, both sides take the
same input produced by the oracle and rounded to float32 (e.g. the oracle's density map for the
field), so the comparison measures that stage's arithmetic only.  Tolerances:
  density map        rel L2 <= 1e-6, total volume rel <= 1e-6   (float32 sums of <= 27 terms)
  field phi, E       rel L2 <= 1e-4                            (float32 and split-bf16 MFMA; for the
                     split form each E component's error relative to |(Ex, Ey, Ez)|)
  wirelength totals  rel <= 1e-5
  WA x/y gradient    rel L2 <= 1e-5
  FDA z-gradient     per instance |diff| <= (4/d_z) * npins_i * 8 ulp(d_x)
  density gradients  rel L2 <= 1e-5 given the same maps
"""
import numpy as np
import pytest

from gpu_common import (filler_case, gpu_problem, log, need_gpu, no_net_case, one_die_case, oracle_problem,
                        pair_case, ragged_case, rel_l2, shared_pin_case, tiny_case, wide_net_case)
from oracle import density as oden
from oracle import density_grad as odg
from oracle import poisson as opois
from oracle import wirelength as owl
from oracle.geometry import geometry_of
from paper_2403_09070_amd import synth

pytestmark = pytest.mark.gpu

CASES = {
    "tiny": lambda: tiny_case(5),
    "ragged": lambda: ragged_case(6),
    "ragged_even": lambda: ragged_case(7, nx=38, ny=30),
    "multi_tile": lambda: ragged_case(13, nx=280, ny=264, nz=4),
    # more than four layers: 16 x 16 bin tiles, and the float32 contractions in both forms
    "layers6": lambda: ragged_case(16, nx=40, ny=34, nz=6),
    "layers16": lambda: ragged_case(17, nx=24, ny=20, nz=16),
    "wide_nets": lambda: wide_net_case(8),
    "one_die": lambda: one_die_case(9),
    "no_nets": lambda: no_net_case(10),
    "shared_pins": lambda: shared_pin_case(14),
    "pairs": lambda: pair_case(15),
    "fillers": lambda: filler_case(11),
    "c1": lambda: synth.make_case("c1", 2403),
    "c2": lambda: synth.make_case("c2", 2403),
}


@pytest.fixture(scope="module", params=list(CASES))
def setup(request):
    need_gpu()
    import torch
    log(f"[parity] case {request.param}")
    case = CASES[request.param]()
    prob = gpu_problem(case)
    torch.cuda.synchronize()
    return request.param, case, prob


def test_density_map(setup):
    name, case, prob = setup
    geo = geometry_of(case)
    rho = prob.density(case.xyz0).cpu().numpy()
    ref = oden.density_map(case.size, case.kind, case.xyz0, geo)
    err = rel_l2(rho, ref)
    log(f"[parity] {name} density rel_l2={err:.3e}")
    assert err <= 1e-6
    assert abs(rho.astype(np.float64).sum() - ref.sum()) <= 1e-6 * ref.sum()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_field(setup, precision):
    name, case, prob = setup
    from paper_2403_09070_amd import place3d
    import torch
    if precision == "bf16x3":
        prob = gpu_problem(case, precision=place3d.BF16X3)
    geo = geometry_of(case)
    # both sides take the oracle's density map, rounded to float32
    rho32 = oden.density_map(case.size, case.kind, case.xyz0, geo).astype(np.float32)
    out = prob.field(torch.from_numpy(rho32).cuda(), energy=True)
    rho64 = rho32.astype(np.float64)
    ref = opois.solve(rho64, geo)
    # The split-bf16 operands carry 16 significant bits, so that form's error in each field
    # component scales with the whole field, not with the component: a component that cancels
    # (Ez when both dies hold nearly the same charge, as with fillers) is measured against |E|.
    enorm = float(np.sqrt(sum(np.linalg.norm(ref[k]) ** 2 for k in ("ex", "ey", "ez"))))
    for k in ("phi", "ex", "ey", "ez"):
        got = out[k].cpu().numpy()
        err = rel_l2(got, ref[k])
        if precision == "bf16x3" and k != "phi":
            err = float(np.linalg.norm(got.astype(np.float64) - ref[k]) / enorm)
        log(f"[parity] {name} {precision} {k} rel_l2={err:.3e}")
        assert err <= 1e-4, k
    e_ref = opois.energy(rho64, ref["phi"], geo)
    assert abs(float(out["energy"].cpu()[0]) - e_ref) <= 1e-4 * abs(e_ref)


def test_wirelength(setup, options=0):
    name, case, prob = setup
    if options:
        prob = gpu_problem(case, options=options)
    geo = geometry_of(case)
    pb = oracle_problem(case)
    g, met = prob.wl_grad(case.xyz0)
    g = g.cpu().numpy()
    met = met.cpu().numpy()
    ref = owl.wirelength(pb.size, pb.kind, case.xyz0, pb.net_start, pb.pin2node, pb.pin_off, geo, pb.gamma, pb.alpha)
    for key, slot in (("wa_bi", 0), ("wa_z", 1), ("hpwl_d2d", 2), ("hpwl_3d", 3)):
        err = abs(met[slot] - ref[key]) / max(abs(ref[key]), 1e-30)
        log(f"[parity] {name} {key} gpu={met[slot]:.9g} ref={ref[key]:.9g} rel={err:.2e}")
        assert err <= 1e-5, key
    assert int(round(met[4])) == ref["ncut"]
    ex, ey = rel_l2(g[0], ref["grad_x"]), rel_l2(g[1], ref["grad_y"])
    log(f"[parity] {name} wa grad rel_l2 x={ex:.3e} y={ey:.3e}")
    assert ex <= 1e-5 and ey <= 1e-5
    # z: normalised FDA plus the WA cut term.  The FDA differences are exact up to the rounding
    # of pin coordinates: a few ulp of the die size per net of the instance.
    scale = met[8]
    assert abs(scale - ref["fda_scale"]) <= 1e-5 * ref["fda_scale"]
    ulp = float(np.spacing(np.float32(geo.die_x)))
    npins = np.bincount(case.pin2node, minlength=case.n_inst)
    want = scale * ref["fda"] + ref["grad_zwa"]
    bound = scale * 4.0 / geo.dz * npins * 8 * ulp + 1e-5 * np.abs(ref["grad_zwa"]).max() + 1e-6 * np.abs(want)
    diff = np.abs(g[2] - want)
    log(f"[parity] {name} z-grad max|diff|/bound={np.max(diff / np.maximum(bound, 1e-30)):.3e} "
        f"rel_l2={rel_l2(g[2], ref['grad'][2]):.3e}")
    assert np.all(diff <= bound)


def test_field_gather(setup):
    name, case, prob = setup
    import torch
    geo = geometry_of(case)
    # field maps from the oracle's solve of the oracle's density, rounded to float32 for both sides
    rho = oden.density_map(case.size, case.kind, case.xyz0, geo)
    sol = opois.solve(rho, geo, want=("ex", "ey", "ez"))
    maps = [sol[k].astype(np.float32) for k in ("ex", "ey", "ez")]
    g = prob.field_force(case.xyz0, *(torch.from_numpy(m).cuda() for m in maps), lam=1.0).cpu().numpy()
    ref = odg.field_gather(case.size, case.kind, case.xyz0, *(m.astype(np.float64) for m in maps), geo)
    err = rel_l2(g, ref)
    log(f"[parity] {name} field-gather rel_l2={err:.3e}")
    assert err <= 1e-5


def test_density_vjp(setup):
    name, case, prob = setup
    import torch
    geo = geometry_of(case)
    rng = np.random.default_rng(0)
    gmap = rng.normal(size=(case.nz, case.ny, case.nx)).astype(np.float32)
    g = prob.density_vjp(case.xyz0, torch.from_numpy(gmap).cuda()).cpu().numpy()
    ref = odg.density_vjp(case.size, case.kind, case.xyz0, gmap.astype(np.float64), geo)
    err = rel_l2(g, ref)
    log(f"[parity] {name} density-vjp rel_l2={err:.3e}")
    assert err <= 1e-5


def _clamped(case, seed):
    """The case's start with a third of the movable instances on the lower z bound, a third on the
    upper (the float32 bounds the step's clamp produces) and every movable macro against a die side
    in x (even index) or y (odd index), at the size its z gives."""
    geo = geometry_of(case)
    f32 = np.float32
    dz = f32(geo.dz)
    xyz = case.xyz0.astype(np.float32).copy()
    mov = np.nonzero((case.kind & 2) == 0)[0]
    rng = np.random.default_rng(seed)
    pick = rng.permutation(mov)
    lo, hi = pick[: len(pick) // 3], pick[len(pick) // 3: 2 * len(pick) // 3]
    xyz[2, lo] = f32(0.25) * dz
    xyz[2, hi] = f32(0.75) * dz
    macros = [i for i in mov if case.kind[i] & 1]
    for k, i in enumerate(macros):
        top = xyz[2, i] > f32(0.5) * dz
        xyz[2, i] = f32(0.75) * dz if top else f32(0.25) * dz
        w, h = (case.size[2, i], case.size[3, i]) if top else (case.size[0, i], case.size[1, i])
        if k % 2 == 0:
            xyz[0, i] = f32(0.5) * f32(w) if k % 4 == 0 else f32(geo.die_x) - f32(0.5) * f32(w)
        else:
            xyz[1, i] = f32(0.5) * f32(h) if k % 4 == 1 else f32(geo.die_y) - f32(0.5) * f32(h)
    return xyz, np.concatenate([lo, hi])


def test_density_vjp_at_the_clamp_bounds(setup):
    """The exact adjoint where GP leaves most instances: on the bounds of the movable z range (every
    z-edge on a bin face or the region's floor or ceiling) and macros against the die sides.  The
    one-sided derivative into the range must match the oracle's, instance by instance."""
    name, case, prob = setup
    import torch
    geo = geometry_of(case)
    xyz, on_bound = _clamped(case, 1)
    rng = np.random.default_rng(2)
    gmap = rng.normal(size=(case.nz, case.ny, case.nx)).astype(np.float32)
    g = prob.density_vjp(xyz, torch.from_numpy(gmap).cuda()).cpu().numpy()
    ref = odg.density_vjp(case.size, case.kind, xyz.astype(np.float64), gmap.astype(np.float64), geo)
    err = rel_l2(g, ref)
    zerr = rel_l2(g[2, on_bound], ref[2, on_bound])
    log(f"[parity] {name} density-vjp at the clamp bounds rel_l2={err:.3e} z on the bounds {zerr:.3e}")
    assert err <= 1e-5 and zerr <= 1e-5


def test_baseline_algorithms(setup):
    """The paper's baselines (Sec. IV) behind the option bits: the instance-parallel scatter of
    large instances gives the same map as the tile-resident sweep (atomic order aside), and the
    O(|P_e|^2) FDA the same z-gradient as the incremental one, both to the default bars."""
    name, case, _ = setup
    from paper_2403_09070_amd import place3d
    geo = geometry_of(case)
    if (case.kind & place3d.KIND_FILLER).any():
        with pytest.raises(place3d.Place3dError):
            gpu_problem(case, options=place3d.OPT_MACRO_INSTANCE)
        opts = place3d.OPT_FDA_VANILLA
    else:
        opts = place3d.OPT_MACRO_INSTANCE | place3d.OPT_FDA_VANILLA
        prob = gpu_problem(case, options=opts)
        rho = prob.density(case.xyz0).cpu().numpy()
        ref = oden.density_map(case.size, case.kind, case.xyz0, geo)
        err = rel_l2(rho, ref)
        log(f"[parity] {name} instance-parallel density rel_l2={err:.3e}")
        assert err <= 1e-6
    test_wirelength(setup, options=opts)
