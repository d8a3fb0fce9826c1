"""Multi-die 2D global placement (Sec. III-C, Eq. 2d-place) through the C ABI against the multi-die
oracle: the three layer maps, the partial nets' wirelength and gradient, each layer's field-gather
gradient, overflow and energy at one placement; lambda_0 of each layer, the bootstrap point and its
gradient; one step from the oracle's state; and a 20-step trajectory.

The problems come from 3D placements of the synthetic workloads split as the oracle splits them
(every crossing net's HBT started in its optimal region), with and without fillers.  Bars: maps
1e-6 rel L2, wirelength totals and gradient 1e-5, overflow 1e-6 absolute, the density gradient
(through the float32 or split-bf16 solve) 1e-4 rel L2, energies 1e-4 rel."""
import numpy as np
import pytest
import torch

from gpu_common import log, need_gpu, rel_l2, tiny_case
from oracle import multidie as md
from oracle import optimizer as opt
from paper_2403_09070_amd import place3d, synth

pytestmark = pytest.mark.gpu


def _split(case, fillers):
    pb = opt.problem_of(case)
    grid = md.Grid2D(case.die_x, case.die_y, case.nx, case.ny)
    lay, xy0 = md.split(case.size, case.kind, case.xyz0, case.net_start, case.pin2node, case.pin_off, pb.geo.dz,
                        grid, pb.gamma, hbt_side=1.0)
    if fillers:
        lay, xy0 = md.with_fillers(lay, xy0, md.filler_plan(lay), seed=1)
    return lay, xy0


CASES = {
    "tiny": lambda: _split(tiny_case(5), False),
    "c1": lambda: _split(synth.make_case("c1", 2403), False),
    "c1_fillers": lambda: _split(synth.make_case("c1", 2403), True),
}
PRECISIONS = {"fp32": place3d.FP32, "bf16x3": place3d.BF16X3}


def _gpu(lay, xy0, precision):
    return place3d.MultiDie2D.from_layered(lay, fixed_xy=np.asarray(xy0, np.float32), precision=precision)


@pytest.fixture(scope="module", params=list(CASES))
def problem(request):
    need_gpu()
    log(f"[md2d] case {request.param}")
    lay, xy0 = CASES[request.param]()
    return request.param, lay, np.asarray(xy0, np.float32).astype(np.float64)


@pytest.mark.parametrize("precision", list(PRECISIONS))
def test_md2d_evaluation(problem, precision):
    name, lay, xy = problem
    prob = _gpu(lay, xy, PRECISIONS[precision])
    gw, gd, rho, met = prob.eval(xy)
    gw, gd, rho, met = gw.cpu().numpy(), gd.cpu().numpy(), rho.cpu().numpy(), met.cpu().numpy()
    wl = md.wirelength_2d(lay, xy)
    parts = md.layer_parts(lay, xy)
    ov = md.overflow_2d(lay, xy)
    err_rho = max(rel_l2(rho[L], parts[L]["rho"]) for L in range(3))
    err_gw = rel_l2(gw, wl["grad"])
    ref_gd = sum(p["grad"] for p in parts)
    err_gd = rel_l2(gd, ref_gd)
    err_wa = abs(met[place3d.MD["wa"]] - wl["wa"]) / wl["wa"]
    err_hp = abs(met[place3d.MD["hpwl"]] - wl["hpwl"]) / wl["hpwl"]
    err_ov = max(abs(met[place3d.MD["ovfl_bot"] + L] - ov[L]) for L in range(3))
    err_en = max(abs(met[place3d.MD["energy_bot"] + L] - parts[L]["energy"]) / abs(parts[L]["energy"])
                 for L in range(3))
    log(f"[md2d] {name} {precision}: rho {err_rho:.2e} grad_wl {err_gw:.2e} grad_den {err_gd:.2e} wa {err_wa:.2e} "
        f"hpwl {err_hp:.2e} ovfl {err_ov:.2e} (ref {ov[0]:.4f}/{ov[1]:.4f}/{ov[2]:.4f}) energy {err_en:.2e}")
    assert err_rho <= 1e-6
    assert err_gw <= 1e-5 and err_wa <= 1e-5 and err_hp <= 1e-5
    assert err_ov <= 1e-6
    assert err_gd <= 1e-4 and err_en <= 1e-4
    fixed = (lay.kind & place3d.KIND_FIXED) != 0
    assert np.all(gw[:, fixed] == 0.0) and np.all(gd[:, fixed] == 0.0)


def _load(prob, ref):
    st = prob.new_state()
    for k in ("u", "v", "v_prev", "g_prev"):
        getattr(st, k).copy_(torch.from_numpy(np.asarray(getattr(ref, k), dtype=np.float32)))
    sc = np.zeros(place3d.NSCALARS)
    sc[place3d.MS["a"]] = ref.a
    sc[place3d.MS["lam_bot"]:place3d.MS["lam_bot"] + 3] = ref.lam
    st.scalars.copy_(torch.from_numpy(sc))
    return st


def _round(ref):
    for k in ("u", "v", "v_prev", "g_prev"):
        setattr(ref, k, np.asarray(getattr(ref, k), dtype=np.float32).astype(np.float64))
    return ref


@pytest.mark.parametrize("precision", list(PRECISIONS))
def test_md2d_init_and_one_step(problem, precision):
    name, lay, xy = problem
    prob = _gpu(lay, xy, PRECISIONS[precision])
    st = prob.gp_init(xy)
    ref = md.gp_init_2d(lay, xy)
    s = st.read()
    lam = np.array([s["lam_bot"], s["lam_top"], s["lam_hbt"]])
    err_lam = float(np.max(np.abs(lam - ref.lam) / ref.lam))
    err_g = rel_l2(st.g_prev.cpu().numpy(), ref.g_prev)
    err_vp = rel_l2(st.v_prev.cpu().numpy(), ref.v_prev)
    log(f"[md2d] {name} {precision} init: lambda {lam} ref {ref.lam} rel {err_lam:.2e} g_prev {err_g:.2e} "
        f"v_prev {err_vp:.2e}")
    assert err_lam <= 1e-5 and err_g <= 1e-4 and err_vp <= 1e-6
    assert rel_l2(st.v.cpu().numpy(), ref.v) <= 1e-7
    # one step from the oracle's state after three steps (rounded to float32 on both sides)
    for _ in range(3):
        md.gp_step_2d(lay, ref)
    ref = _round(ref)
    st = _load(prob, ref)
    v0 = ref.v.copy()
    prob.step(st)
    m = md.gp_step_2d(lay, ref)
    s = st.read()
    step_err = abs(s["step"] - m["step"]) / m["step"]
    disp = rel_l2(st.v.cpu().numpy() - v0, ref.v - v0)
    log(f"[md2d] {name} {precision} step: size rel {step_err:.2e} displacement rel_l2 {disp:.2e} hpwl "
        f"{s['hpwl']:.8g} ref {m['hpwl']:.8g}")
    assert abs(s["wa"] - m["wa"]) <= 1e-5 * m["wa"] and abs(s["hpwl"] - m["hpwl"]) <= 1e-5 * m["hpwl"]
    for L, k in enumerate(("ovfl_bot", "ovfl_top", "ovfl_hbt")):
        assert abs(s[k] - (m["ovfl_bot"], m["ovfl_top"], m["ovfl_hbt"])[L]) <= 1e-6
    assert np.allclose([s["lam_bot"], s["lam_top"], s["lam_hbt"]], ref.lam, rtol=1e-12)
    assert step_err <= 1e-3 and disp <= 1e-3


def test_md2d_trajectory_tracks_the_oracle():
    need_gpu()
    lay, xy = _split(synth.make_case("c1", 2403), True)
    xy = np.asarray(xy, np.float32).astype(np.float64)
    prob = _gpu(lay, xy, place3d.BF16X3)
    st = prob.gp_init(xy)
    ref = md.gp_init_2d(lay, xy)
    worst_h = worst_o = 0.0
    for k in range(20):
        prob.step(st)
        m = md.gp_step_2d(lay, ref)
        s = st.read()
        dh = abs(s["hpwl"] - m["hpwl"]) / m["hpwl"]
        do = max(abs(s["ovfl_bot"] - m["ovfl_bot"]), abs(s["ovfl_top"] - m["ovfl_top"]),
                 abs(s["ovfl_hbt"] - m["ovfl_hbt"]))
        worst_h, worst_o = max(worst_h, dh), max(worst_o, do)
        log(f"[md2d] it {k} hpwl rel {dh:.2e} ovfl diff {do:.2e} ovfl {m['ovfl_bot']:.4f}/{m['ovfl_top']:.4f}/"
            f"{m['ovfl_hbt']:.4f}")
    assert worst_h <= 1e-3 and worst_o <= 1e-3
