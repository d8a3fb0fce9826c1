"""Parity at the full 1.2M-cell workload (1.3M nets, 4.5M pins, grid 1024 x 1024 x 4) in every
form the benchmark times -- split-bf16 and float32 contractions, compensated and plain
exponential sums, field-gather and exact-adjoint density gradients -- launched exactly as
place3d_step launches them (folded contractions, the net schedule and the tile bucketing of that
size), the wirelength sweep also on the no-locality netlist of that size, and one whole step of each
form the benchmark times from the same state on both sides; and at the largest workload (4M cells, 15M pins, grid 2048 x 2048 x 4, clustered start) the
density map, the split-bf16 spectral solve and the wirelength sweep.  Every output is compared in full against the oracle on the
same seeded inputs, with the tolerances of the small-case parity tests:
  density map rel L2 <= 1e-6 (at the generated placement and at a clustered one, where bins hold
  many overlapping cells), field rel L2 <= 1e-4, wirelength totals rel <= 1e-5, WA x/y gradient
  rel L2 <= 1e-5, FDA z-gradient within (4/d_z) npins 8 ulp(d_x) per instance, field gather and
  exact adjoint rel L2 <= 1e-5.  Inputs of a stage come from the oracle (rounded to float32 for
  both sides).
"""
import numpy as np
import pytest

from gpu_common import gpu_problem, load_state, log, need_gpu, oracle_problem, rel_l2, round_state
from oracle import density as oden
from oracle import density_grad as odg
from oracle import poisson as opois
from oracle import wirelength as owl
from oracle.geometry import geometry_of
from paper_2403_09070_amd import synth

pytestmark = pytest.mark.gpu


PRECISIONS = ["bf16x3", "fp32"]


@pytest.fixture(scope="module")
def full():
    need_gpu()
    from paper_2403_09070_amd import place3d
    log("[full] generating the 1.2M-cell workload")
    case = synth.make_case("c4", 2403)
    probs = {"bf16x3": gpu_problem(case, precision=place3d.BF16X3, dgrad=place3d.DGRAD_FIELD),
             "fp32": gpu_problem(case, precision=place3d.FP32, dgrad=place3d.DGRAD_FIELD)}
    geo = geometry_of(case)
    log("[full] oracle density map")
    rho = oden.density_map(case.size, case.kind, case.xyz0, geo)
    return case, probs, geo, rho


def _clustered(case, seed=11):
    """Movable instances pulled to a quarter of the die around its centre (seeded jitter kept),
    so that many cells overlap in each bin."""
    rng = np.random.default_rng(seed)
    xyz = case.xyz0.astype(np.float64).copy()
    mov = (case.kind & 2) == 0
    for a, d in ((0, case.die_x), (1, case.die_y)):
        xyz[a, mov] = 0.5 * d + 0.25 * (xyz[a, mov] - 0.5 * d) + rng.normal(0.0, 0.01 * d, mov.sum())
        xyz[a, mov] = np.clip(xyz[a, mov], 0.0, d)
    return xyz.astype(np.float32)


@pytest.mark.parametrize("where", ["generated", "clustered"])
def test_density_full(full, where):
    case, probs, geo, rho_gen = full
    prob = probs["bf16x3"]
    xyz = case.xyz0 if where == "generated" else _clustered(case)
    ref = rho_gen if where == "generated" else oden.density_map(case.size, case.kind, xyz, geo)
    got = prob.density(xyz).cpu().numpy()
    err = rel_l2(got, ref)
    log(f"[full] density {where} rel_l2={err:.3e} max bin {ref.max():.2f}")
    assert err <= 1e-6
    assert abs(got.astype(np.float64).sum() - ref.sum()) <= 1e-6 * ref.sum()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_field_full(full, precision):
    import torch
    case, probs, geo, rho = full
    rho32 = rho.astype(np.float32)
    out = probs[precision].field(torch.from_numpy(rho32).cuda(), want=("phi", "ex", "ey", "ez"))
    ref = opois.solve(rho32.astype(np.float64), geo)
    for k in ("phi", "ex", "ey", "ez"):
        err = rel_l2(out[k].cpu().numpy(), ref[k])
        log(f"[full] {precision} field {k} rel_l2={err:.3e}")
        assert err <= 1e-4, k


def test_field_gather_full(full):
    import torch
    case, probs, geo, rho = full
    prob = probs["bf16x3"]
    sol = opois.solve(rho.astype(np.float32).astype(np.float64), geo, want=("ex", "ey", "ez"))
    maps = [sol[k].astype(np.float32) for k in ("ex", "ey", "ez")]
    g = prob.field_force(case.xyz0, *(torch.from_numpy(m).cuda() for m in maps), lam=1.0).cpu().numpy()
    log("[full] oracle field gather")
    ref = odg.field_gather(case.size, case.kind, case.xyz0, *(m.astype(np.float64) for m in maps), geo)
    err = rel_l2(g, ref)
    log(f"[full] field-gather rel_l2={err:.3e}")
    assert err <= 1e-5


@pytest.fixture(scope="module")
def wl_ref(full):
    case, probs, geo, rho = full
    pb = oracle_problem(case)
    log("[full] oracle wirelength")
    return owl.wirelength(pb.size, pb.kind, case.xyz0, pb.net_start, pb.pin2node, pb.pin_off, geo, pb.gamma, pb.alpha)


def _check_wirelength(case, geo, prob, ref, tag):
    """The sweep's totals, #cut, WA x/y gradient and FDA z-gradient against the oracle's."""
    g, met = prob.wl_grad(case.xyz0)
    g = g.cpu().numpy()
    met = met.cpu().numpy()
    for key, slot in (("wa_bi", 0), ("wa_z", 1), ("hpwl_d2d", 2), ("hpwl_3d", 3)):
        err = abs(met[slot] - ref[key]) / abs(ref[key])
        log(f"[full] {tag} {key} gpu={met[slot]:.10g} ref={ref[key]:.10g} rel={err:.2e}")
        assert err <= 1e-5, key
    assert int(round(met[4])) == ref["ncut"]
    ex, ey = rel_l2(g[0], ref["grad_x"]), rel_l2(g[1], ref["grad_y"])
    log(f"[full] {tag} wa grad rel_l2 x={ex:.3e} y={ey:.3e}")
    assert ex <= 1e-5 and ey <= 1e-5
    scale = met[8]
    assert abs(scale - ref["fda_scale"]) <= 1e-5 * ref["fda_scale"]
    ulp = float(np.spacing(np.float32(geo.die_x)))
    npins = np.bincount(case.pin2node, minlength=case.n_inst)
    want = scale * ref["fda"] + ref["grad_zwa"]
    bound = scale * 4.0 / geo.dz * npins * 8 * ulp + 1e-5 * np.abs(ref["grad_zwa"]).max() + 1e-6 * np.abs(want)
    diff = np.abs(g[2] - want)
    log(f"[full] {tag} z-grad max|diff|/bound={np.max(diff / np.maximum(bound, 1e-30)):.3e}")
    assert np.all(diff <= bound)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_wirelength_full(full, wl_ref, precision):
    case, probs, geo, rho = full
    _check_wirelength(case, geo, probs[precision], wl_ref, precision)


@pytest.fixture(scope="module")
def no_locality():
    need_gpu()
    log("[full] generating the no-locality 1.2M-cell netlist; oracle wirelength")
    case = synth.make_case("c4u", 2403)
    geo = geometry_of(case)
    pb = oracle_problem(case)
    ref = owl.wirelength(pb.size, pb.kind, case.xyz0, pb.net_start, pb.pin2node, pb.pin_off, geo, pb.gamma, pb.alpha)
    return case, geo, ref


@pytest.mark.parametrize("precision", PRECISIONS)
def test_wirelength_no_locality_netlist(no_locality, precision):
    """The 1.2M-cell workload with every net drawing its members uniformly over the instances (no
    index window): the sweep's owner gathers touch a different cache line per pin."""
    from paper_2403_09070_amd import place3d
    case, geo, ref = no_locality
    prob = gpu_problem(case, precision=place3d.BF16X3 if precision == "bf16x3" else place3d.FP32,
                       dgrad=place3d.DGRAD_FIELD)
    _check_wirelength(case, geo, prob, ref, "c4u " + precision)


# forms of the full-size step: (problem key or None for a context of its own, oracle density
# gradient, displacement bar before the float32 floor -- the small workload's one-step bars)
STEP_FORMS = {"field-bf16x3": ("bf16x3", "field", 5e-5), "field-fp32": ("fp32", "field", 2e-5),
              "adjoint-bf16x3": (None, "adjoint", 3e-4)}


@pytest.mark.parametrize("form", list(STEP_FORMS))
def test_one_step_at_full_size(full, form):
    """One step of each form the benchmark times (split-bf16 or float32 contractions, compensated or
    plain exp-sums, field gather or exact adjoint, Eq. improved-precond) at the 1.2M-cell
    workload, from the same state on both sides:
    v the clamped start, u and v_prev seeded perturbations of it (half a bin in x and y, 2 % of
    the die depth in z), g_prev zero, a = 2.5 (the momentum term active), lambda the ratio of the
    gradients' L1 norms at v.  The metrics at v, the step size and the new iterate against the
    oracle's gp_step, at the bars of the one-step test of the small workload (the displacement's
    plus twice the floor that rounding the new positions to float32 sets), and the new
    preconditioned gradient within 1e-4."""
    from oracle import optimizer as opt
    from paper_2403_09070_amd import place3d
    case, probs, geo, rho = full
    key, dgrad, bar = STEP_FORMS[form]
    prob = probs[key] if key else gpu_problem(case, precision=place3d.BF16X3, dgrad=place3d.DGRAD_ADJOINT)
    pb = oracle_problem(case)
    mov = pb.movable
    rng = np.random.default_rng(17)
    v = opt.clamp(pb, case.xyz0)

    def near(p):
        q = p.copy()
        for a, sd in ((0, 0.5 * geo.wb), (1, 0.5 * geo.hb), (2, 0.02 * geo.dz)):
            q[a, mov] += rng.normal(0.0, sd, int(mov.sum()))
        return opt.clamp(pb, q)

    u, v_prev = near(v), near(v)
    log(f"[full] {form}: oracle evaluation at v (lambda)")
    wl, _, _, gd = opt.evaluate(pb, v, dgrad)
    lam = float(np.abs(wl["grad"][:, mov]).sum() / np.abs(gd[:, mov]).sum())
    ref = round_state(opt.GPState(u=u, v=v, v_prev=v_prev, g_prev=np.zeros_like(v), a=2.5, lam=lam))
    st = load_state(prob, ref)
    v0 = ref.v.copy()
    prob.step(st)
    log(f"[full] {form}: oracle step")
    m = opt.gp_step(pb, ref, dgrad=dgrad, precond="mixed")
    s = st.read()
    for name, rkey in (("hpwl", "hpwl_d2d"), ("wa_bi", "wa_bi"), ("wa_z", "wa_z")):
        assert abs(s[name] - m[rkey]) <= 1e-5 * abs(m[rkey]), name
    assert s["ncut"] == m["ncut"]
    assert abs(s["ovfl_bot"] - m["ovfl_bot"]) <= 1e-6 and abs(s["ovfl_top"] - m["ovfl_top"]) <= 1e-6
    assert abs(s["lam"] - ref.lam) <= 1e-12 * ref.lam
    step_err = abs(s["step"] - m["step"]) / m["step"]
    disp = rel_l2(st.v.cpu().numpy() - v0, ref.v - v0)
    gerr = rel_l2(st.g_prev.cpu().numpy(), ref.g_prev)
    # the new positions are float32 (coordinates up to 4000, ulp 2.4e-4 to 4.9e-4): half an ulp of
    # each, against the move, is a floor the displacement error cannot go below
    floor = float(np.linalg.norm(0.5 * np.spacing(ref.v.astype(np.float32)).astype(np.float64)) /
                  np.linalg.norm(ref.v - v0))
    log(f"[full] {form} one step: gradient rel_l2={gerr:.3e} step rel={step_err:.3e} displacement rel_l2={disp:.3e} "
        f"(float32 floor {floor:.2e}) ovfl {s['ovfl_bot']:.6f}/{s['ovfl_top']:.6f} "
        f"ref {m['ovfl_bot']:.6f}/{m['ovfl_top']:.6f}")
    assert gerr <= 1e-4
    assert step_err <= 1e-5 and disp <= bar + 2.0 * floor
    if dgrad == "adjoint":
        assert abs(s["energy"] - m["energy"]) <= 1e-4 * abs(m["energy"])


def test_density_vjp_full(full):
    """The exact adjoint (the differentiation form's density backward) at full size, applied to the
    oracle's potential times the bin volume (rounded to float32 on both sides): the gradient of
    the energy, against the oracle's adjoint."""
    import torch
    case, probs, geo, rho = full
    phi = opois.solve(rho.astype(np.float32).astype(np.float64), geo, want=("phi",))["phi"]
    gmap = (phi * geo.vol_bin).astype(np.float32)
    g = probs["bf16x3"].density_vjp(case.xyz0, torch.from_numpy(gmap).cuda()).cpu().numpy()
    log("[full] oracle exact adjoint")
    ref = odg.density_vjp(case.size, case.kind, case.xyz0, gmap.astype(np.float64), geo)
    err = rel_l2(g, ref)
    log(f"[full] density-vjp rel_l2={err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("where", ["generated", "clustered"])
def test_density_many_bucket_blocks(where):
    """1.7M instances on a 512 x 512 x 2 grid: 831 bucketing blocks, more than the tile scan holds
    in registers per range (16 ranges of 48), so its long-range path runs; clustered, the tiles
    are split into chunks as well.  Density map and total volume against the oracle."""
    need_gpu()
    from paper_2403_09070_amd import place3d
    cfg = synth.small_config(n_cells=1_700_000, n_nets=1000, die=2000.0, nx=512, ny=512, nz=2,
                             macros=("uniform", 8, 0.002, 0.01))
    case = synth.make_case(config=cfg, seed=31)
    if where == "clustered":
        case = synth.centre_start(case, sigma=0.05, seed=32)
    geo = geometry_of(case)
    ref = oden.density_map(case.size, case.kind, case.xyz0, geo)
    got = gpu_problem(case, precision=place3d.BF16X3).density(case.xyz0).cpu().numpy()
    err = rel_l2(got, ref)
    log(f"[full] density, {case.n_inst} instances, {where}: rel_l2={err:.3e} max bin {ref.max():.2f}")
    assert err <= 1e-6
    assert abs(got.astype(np.float64).sum() - ref.sum()) <= 1e-6 * ref.sum()


def test_largest_workload_density_and_wirelength():
    """The largest workload (4M cells, 200 macros up to 5 % of the die, 4.4M nets of up to 100
    pins, 15M pins, grid 2048 x 2048 x 4) at the clustered start its run to overflow takes (x, y
    normal around the centre with sigma 0.02 of the die: most cells in a few dozen of the 4096
    tiles, which are split into many chunks): the density map and its total volume, the split-bf16
    spectral solve of that map, and the precision form's wirelength sweep (totals, x/y gradient,
    FDA z-gradient), against the oracle with the bars above."""
    need_gpu()
    from paper_2403_09070_amd import place3d
    log("[full] generating the 4M-cell workload")
    case = synth.centre_start(synth.make_case("c5", 2403), sigma=0.02, seed=2404)
    geo = geometry_of(case)
    prob = gpu_problem(case, precision=place3d.BF16X3, dgrad=place3d.DGRAD_FIELD)
    log("[full] 4M: oracle density map")
    ref = oden.density_map(case.size, case.kind, case.xyz0, geo)
    got = prob.density(case.xyz0).cpu().numpy()
    err = rel_l2(got, ref)
    log(f"[full] 4M density rel_l2={err:.3e} max bin {ref.max():.2f}")
    assert err <= 1e-6
    assert abs(got.astype(np.float64).sum() - ref.sum()) <= 1e-6 * ref.sum()
    # the split-bf16 solve of the oracle's map (rounded to float32 on both sides); the split form's
    # E components against |(Ex, Ey, Ez)|, as in the small cases
    import torch
    rho32 = ref.astype(np.float32)
    log("[full] 4M: oracle spectral solve")
    sol = opois.solve(rho32.astype(np.float64), geo)
    out = prob.field(torch.from_numpy(rho32).cuda())
    enorm = float(np.sqrt(sum(np.linalg.norm(sol[k]) ** 2 for k in ("ex", "ey", "ez"))))
    for k in ("phi", "ex", "ey", "ez"):
        got_k = out[k].cpu().numpy().astype(np.float64)
        e = rel_l2(got_k, sol[k]) if k == "phi" else float(np.linalg.norm(got_k - sol[k]) / enorm)
        log(f"[full] 4M bf16x3 {k} rel_l2={e:.3e}")
        assert e <= 1e-4, k
    del sol, out
    pb = oracle_problem(case)
    log("[full] 4M: oracle wirelength")
    with np.errstate(over="ignore"):        # exponentials of padded slots, masked out
        wl = owl.wirelength(pb.size, pb.kind, case.xyz0, pb.net_start, pb.pin2node, pb.pin_off, geo, pb.gamma,
                            pb.alpha)
    g, met = prob.wl_grad(case.xyz0)
    g = g.cpu().numpy()
    met = met.cpu().numpy()
    for key, slot in (("wa_bi", 0), ("wa_z", 1), ("hpwl_d2d", 2), ("hpwl_3d", 3)):
        e = abs(met[slot] - wl[key]) / abs(wl[key])
        log(f"[full] 4M {key} gpu={met[slot]:.10g} ref={wl[key]:.10g} rel={e:.2e}")
        assert e <= 1e-5, key
    assert int(round(met[4])) == wl["ncut"]
    ex, ey = rel_l2(g[0], wl["grad_x"]), rel_l2(g[1], wl["grad_y"])
    log(f"[full] 4M wa grad rel_l2 x={ex:.3e} y={ey:.3e}")
    assert ex <= 1e-5 and ey <= 1e-5
    scale = met[8]
    assert abs(scale - wl["fda_scale"]) <= 1e-5 * wl["fda_scale"]
    ulp = float(np.spacing(np.float32(geo.die_x)))
    npins = np.bincount(case.pin2node, minlength=case.n_inst)
    want = scale * wl["fda"] + wl["grad_zwa"]
    bound = scale * 4.0 / geo.dz * npins * 8 * ulp + 1e-5 * np.abs(wl["grad_zwa"]).max() + 1e-6 * np.abs(want)
    diff = np.abs(g[2] - want)
    log(f"[full] 4M z-grad max|diff|/bound={np.max(diff / np.maximum(bound, 1e-30)):.3e}")
    assert np.all(diff <= bound)
