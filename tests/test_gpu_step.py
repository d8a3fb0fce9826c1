"""GP initialisation and Nesterov steps: GPU (C ABI) against the oracle's GP loop.

* gp_init: lambda_0 and the bootstrap point agree with the oracle's.
* One step from the same state (the oracle's state rounded to float32 on both sides): the
  metrics at the evaluation point and the new iterate agree.  The step size divides by
  |g_k - g_{k-1}|, which amplifies the float32 rounding of the gradient by |g| / |g_k - g_{k-1}|;
  the bars are about ten times the measured errors of each form (DISP_BAR).
* A short trajectory: the D2D HPWL of GPU and oracle stay within 2e-6 of each other (measured
  1.9e-7 over 20 steps).
* The ePlace and ePlace3D preconditioners of Eq. general-precond: init and one step, as above.
* Fillers (z-fixed and free): init, one step and a 20-step trajectory with the overflow measured
  without them; z-fixed fillers keep their z exactly.
"""
import numpy as np
import pytest
import torch

from gpu_common import (gpu_problem, load_state, log, need_gpu, oracle_problem, ragged_case, rel_l2, round_state,
                        tiny_case)
from oracle import optimizer as opt
from paper_2403_09070_amd import place3d, synth

pytestmark = pytest.mark.gpu

FORMS = {
    "field-fp32": dict(dgrad=place3d.DGRAD_FIELD, precision=place3d.FP32),
    "field-bf16x3": dict(dgrad=place3d.DGRAD_FIELD, precision=place3d.BF16X3),
    "adjoint-bf16x3": dict(dgrad=place3d.DGRAD_ADJOINT, precision=place3d.BF16X3),
    # the two earlier preconditioners of Eq. general-precond (ePlace and ePlace3D forms)
    "field-bf16x3-eplace": dict(dgrad=place3d.DGRAD_FIELD, precision=place3d.BF16X3,
                                precond=place3d.PRECOND_EPLACE),
    "field-bf16x3-eplace3d": dict(dgrad=place3d.DGRAD_FIELD, precision=place3d.BF16X3,
                                  precond=place3d.PRECOND_EPLACE3D),
}
# one-step displacement bars, about ten times the measured rel L2 (float32 field gather 1.3e-6,
# split-bf16 3.7e-6, split-bf16 with the exact adjoint 2.4e-5, ePlace 5.1e-6, ePlace3D 3.1e-6)
DISP_BAR = {"field-fp32": 2e-5, "field-bf16x3": 5e-5, "adjoint-bf16x3": 3e-4, "field-bf16x3-eplace": 1e-4,
            "field-bf16x3-eplace3d": 5e-5}
STEP_BAR = 1e-5      # the Lipschitz step size (measured <= 9.1e-7)
PRECOND_NAMES = {place3d.PRECOND_MIXED: "mixed", place3d.PRECOND_EPLACE: "eplace",
                 place3d.PRECOND_EPLACE3D: "eplace3d"}


def _oracle_form(form):
    return "field" if FORMS[form]["dgrad"] == place3d.DGRAD_FIELD else "adjoint"


def _oracle_precond(form):
    return PRECOND_NAMES[FORMS[form].get("precond", place3d.PRECOND_MIXED)]


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("which", ["tiny", "c1"])
def test_gp_init(which, form):
    need_gpu()
    log(f"[step] init {which} {form}")
    case = tiny_case(5) if which == "tiny" else synth.make_case("c1", 2403)
    prob = gpu_problem(case, **FORMS[form])
    pb = oracle_problem(case)
    st = prob.gp_init(case.xyz0)
    ref = opt.gp_init(pb, case.xyz0, dgrad=_oracle_form(form), precond=_oracle_precond(form))
    s = st.read()
    log(f"[step] lambda0 gpu={s['lam']:.9g} ref={ref.lam:.9g}")
    assert abs(s["lam"] - ref.lam) <= 1e-5 * ref.lam
    assert rel_l2(st.v.cpu().numpy(), ref.v) <= 1e-7
    assert rel_l2(st.v_prev.cpu().numpy(), ref.v_prev) <= 1e-6
    err = rel_l2(st.g_prev.cpu().numpy(), ref.g_prev)
    log(f"[step] g_prev rel_l2={err:.3e}")
    assert err <= 1e-4


@pytest.mark.parametrize("form", list(FORMS))
def test_one_step_from_the_same_state(form):
    need_gpu()
    log(f"[step] one step c1 {form}")
    case = synth.make_case("c1", 2403)
    prob = gpu_problem(case, **FORMS[form])
    pb = oracle_problem(case)
    ref = opt.gp_init(pb, case.xyz0, dgrad=_oracle_form(form), precond=_oracle_precond(form))
    for _ in range(3):                                   # move away from the bootstrap point
        opt.gp_step(pb, ref, dgrad=_oracle_form(form), precond=_oracle_precond(form))
    ref = round_state(ref)
    st = load_state(prob, ref)
    v0 = ref.v.copy()
    prob.step(st)
    m = opt.gp_step(pb, ref, dgrad=_oracle_form(form), precond=_oracle_precond(form))
    s = st.read()
    for key, rkey in (("hpwl", "hpwl_d2d"), ("wa_bi", "wa_bi"), ("wa_z", "wa_z")):
        assert abs(s[key] - m[rkey]) <= 1e-5 * abs(m[rkey]), key
    assert s["ncut"] == m["ncut"]
    assert abs(s["ovfl_bot"] - m["ovfl_bot"]) <= 1e-6 and abs(s["ovfl_top"] - m["ovfl_top"]) <= 1e-6
    assert abs(s["lam"] - ref.lam) <= 1e-12 * ref.lam
    step_err = abs(s["step"] - m["step"]) / m["step"]
    disp = rel_l2(st.v.cpu().numpy() - v0, ref.v - v0)
    log(f"[step] {form} step rel={step_err:.3e} displacement rel_l2={disp:.3e}")
    assert step_err <= STEP_BAR and disp <= DISP_BAR[form]
    if FORMS[form]["dgrad"] == place3d.DGRAD_ADJOINT:
        assert abs(s["energy"] - m["energy"]) <= 1e-4 * abs(m["energy"])


def test_short_trajectory_tracks_the_oracle():
    need_gpu()
    log("[step] 20-step trajectory c1")
    case = synth.make_case("c1", 2403)
    prob = gpu_problem(case)
    pb = oracle_problem(case)
    st = prob.gp_init(case.xyz0)
    ref = opt.gp_init(pb, case.xyz0)
    worst = 0.0
    for k in range(20):
        prob.step(st)
        m = opt.gp_step(pb, ref)
        s = st.read()
        d = abs(s["hpwl"] - m["hpwl_d2d"]) / m["hpwl_d2d"]
        worst = max(worst, d)
        log(f"[step] it {k} hpwl gpu={s['hpwl']:.7g} ref={m['hpwl_d2d']:.7g} rel={d:.2e} "
            f"ovfl gpu={s['ovfl_bot']:.4f}/{s['ovfl_top']:.4f} ref={m['ovfl_bot']:.4f}/{m['ovfl_top']:.4f}")
    assert worst <= 2e-6


def test_fillers_init_step_and_trajectory():
    """z-fixed and free fillers (density model, Sec. III-A) on a centre start: lambda_0 and the
    bootstrap agree with the oracle, the per-die overflow (fillers left out) and the D2D HPWL track
    it for 20 steps, z-fixed fillers keep their z bit for bit and free fillers move in z."""
    from gpu_common import filler_case
    need_gpu()
    log("[step] fillers: init + 20 steps")
    case = filler_case(11)
    held = (case.kind & place3d.KIND_ZFIXED) != 0
    free = ((case.kind & place3d.KIND_FILLER) != 0) & ~held
    assert held.any() and free.any()
    prob = gpu_problem(case, precision=place3d.BF16X3)
    pb = oracle_problem(case)
    st = prob.gp_init(case.xyz0)
    ref = opt.gp_init(pb, case.xyz0)
    s = st.read()
    assert abs(s["lam"] - ref.lam) <= 1e-5 * ref.lam
    assert rel_l2(st.g_prev.cpu().numpy(), ref.g_prev) <= 1e-4
    assert np.all(st.g_prev.cpu().numpy()[2, held] == 0.0)
    z_held = case.xyz0[2, held].copy()
    z_free = st.v.cpu().numpy()[2, free].copy()
    worst_h = worst_o = 0.0
    saw_overflow = False
    for k in range(20):
        prob.step(st)
        m = opt.gp_step(pb, ref)
        s = st.read()
        dh = abs(s["hpwl"] - m["hpwl_d2d"]) / m["hpwl_d2d"]
        do = max(abs(s["ovfl_bot"] - m["ovfl_bot"]), abs(s["ovfl_top"] - m["ovfl_top"]))
        worst_h, worst_o = max(worst_h, dh), max(worst_o, do)
        saw_overflow |= max(m["ovfl_bot"], m["ovfl_top"]) > 0.05
        log(f"[step] fillers it {k} hpwl rel={dh:.2e} ovfl gpu={s['ovfl_bot']:.4f}/{s['ovfl_top']:.4f} "
            f"ref={m['ovfl_bot']:.4f}/{m['ovfl_top']:.4f} diff={do:.2e}")
    v = st.v.cpu().numpy()
    assert np.array_equal(v[2, held], z_held) and np.array_equal(st.u.cpu().numpy()[2, held], z_held)
    assert np.abs(v[2, free] - z_free).max() > 0.0
    assert saw_overflow
    # measured: HPWL 3.1e-6 after 20 steps, overflow equal to the fourth decimal every step
    assert worst_h <= 3e-5 and worst_o <= 1e-5


def test_fillers_one_step_from_the_same_state():
    from gpu_common import filler_case
    need_gpu()
    log("[step] fillers: one step c1-sized")
    case = filler_case(12, config=synth.CONFIGS["c1"], u=0.9, sigma=0.08)
    prob = gpu_problem(case, precision=place3d.BF16X3)
    pb = oracle_problem(case)
    ref = opt.gp_init(pb, case.xyz0)
    for _ in range(3):
        opt.gp_step(pb, ref)
    ref = round_state(ref)
    st = load_state(prob, ref)
    v0 = ref.v.copy()
    prob.step(st)
    m = opt.gp_step(pb, ref)
    s = st.read()
    assert abs(s["hpwl"] - m["hpwl_d2d"]) <= 1e-5 * m["hpwl_d2d"]
    assert abs(s["ovfl_bot"] - m["ovfl_bot"]) <= 1e-6 and abs(s["ovfl_top"] - m["ovfl_top"]) <= 1e-6
    step_err = abs(s["step"] - m["step"]) / m["step"]
    disp = rel_l2(st.v.cpu().numpy() - v0, ref.v - v0)
    log(f"[step] fillers step rel={step_err:.3e} displacement rel_l2={disp:.3e} "
        f"ovfl={m['ovfl_bot']:.4f}/{m['ovfl_top']:.4f}")
    assert step_err <= STEP_BAR and disp <= 3e-4        # measured 1.5e-8, 2.6e-5


def test_baseline_algorithms_in_the_step():
    """The option bits of the paper's baselines (instance-parallel macro scatter, vanilla FDA)
    leave a 10-step trajectory where the default algorithms take it (atomic order aside)."""
    need_gpu()
    log("[step] baseline algorithm options: 10 steps")
    case = tiny_case(5)
    assert ((case.kind & place3d.KIND_MACRO) != 0).any()
    a = gpu_problem(case, precision=place3d.BF16X3)
    b = gpu_problem(case, precision=place3d.BF16X3, options=place3d.OPT_MACRO_INSTANCE | place3d.OPT_FDA_VANILLA)
    sa, sb = a.gp_init(case.xyz0), b.gp_init(case.xyz0)
    for k in range(10):
        a.step(sa)
        b.step(sb)
        ra, rb = sa.read(), sb.read()
        dh = abs(ra["hpwl"] - rb["hpwl"]) / ra["hpwl"]
        do = max(abs(ra["ovfl_bot"] - rb["ovfl_bot"]), abs(ra["ovfl_top"] - rb["ovfl_top"]))
        log(f"[step] options it {k} hpwl rel={dh:.2e} ovfl diff={do:.2e}")
        assert dh <= 1e-5 and do <= 1e-5                   # measured 1.3e-6, 0


def test_nonfinite_iteration_is_flagged_and_reported():
    """A NaN density weight (set from the host) makes the step's float64 gradient-change norm NaN:
    the step records the iteration and place3d_read_scalars returns PLACE3D_ERR_NONFINITE.  The
    positions stay finite (the clamp takes a NaN move to the region's bound), so no kernel sees a
    NaN index.  A clean run reads back without error."""
    need_gpu()
    log("[step] non-finite flag")
    case = tiny_case(5)
    prob = gpu_problem(case)
    st = prob.gp_init(case.xyz0)
    prob.step(st)
    sc = prob.read_scalars(st)
    assert sc[place3d.S["nonfinite"]] == 0.0 and sc[place3d.S["it"]] == 1.0
    st.scalars[place3d.S["lam"]] = float("nan")
    prob.step(st)
    with pytest.raises(place3d.Place3dError) as e:
        prob.read_scalars(st)
    assert e.value.code == -4 and "iteration 1" in str(e.value)
    assert torch.isfinite(st.v).all()


@pytest.mark.parametrize("form", ["field-bf16x3", "adjoint-bf16x3"])
def test_init_and_one_step_with_eight_layers(form):
    """Eight layers (16 x 16 bin tiles, float32 contractions in the split form, four layers per
    die in the overflow): gp_init and one step from the oracle's state three steps on, to the bars
    of the two-layer-per-die tests."""
    need_gpu()
    log(f"[step] eight layers {form}")
    case = ragged_case(18, nx=48, ny=40, nz=8)
    prob = gpu_problem(case, **FORMS[form])
    pb = oracle_problem(case)
    st = prob.gp_init(case.xyz0)
    ref = opt.gp_init(pb, case.xyz0, dgrad=_oracle_form(form), precond=_oracle_precond(form))
    s = st.read()
    assert abs(s["lam"] - ref.lam) <= 1e-5 * ref.lam
    assert rel_l2(st.g_prev.cpu().numpy(), ref.g_prev) <= 1e-4
    for _ in range(3):
        opt.gp_step(pb, ref, dgrad=_oracle_form(form), precond=_oracle_precond(form))
    ref = round_state(ref)
    st = load_state(prob, ref)
    v0 = ref.v.copy()
    prob.step(st)
    m = opt.gp_step(pb, ref, dgrad=_oracle_form(form), precond=_oracle_precond(form))
    s = st.read()
    for key, rkey in (("hpwl", "hpwl_d2d"), ("wa_bi", "wa_bi"), ("wa_z", "wa_z")):
        assert abs(s[key] - m[rkey]) <= 1e-5 * abs(m[rkey]), key
    assert abs(s["ovfl_bot"] - m["ovfl_bot"]) <= 1e-6 and abs(s["ovfl_top"] - m["ovfl_top"]) <= 1e-6
    step_err = abs(s["step"] - m["step"]) / m["step"]
    disp = rel_l2(st.v.cpu().numpy() - v0, ref.v - v0)
    log(f"[step] eight layers {form} step rel={step_err:.3e} displacement rel_l2={disp:.3e}")
    assert step_err <= STEP_BAR and disp <= DISP_BAR[form]


def test_captured_step_replays_match_eager_steps():
    """place3d_step under stream capture (it allocates, fills and synchronises nothing; its side
    stream forks from and joins the captured stream): one captured step replayed five times, with
    eager steps, an eager density call and host synchronisations between the replays, gives the
    eager steps' iterates and scalars bit for bit after every replay."""
    need_gpu()
    log("[step] captured step, c1")
    case = synth.make_case("c1", 2403)
    prob = gpu_problem(case, precision=place3d.BF16X3)
    work = torch.cuda.Stream()
    with torch.cuda.stream(work):
        sa = prob.gp_init(case.xyz0)
        sb = prob.new_state()
        for k in ("u", "v", "v_prev", "g_prev", "scalars"):
            getattr(sb, k).copy_(getattr(sa, k))
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(work)
        with torch.cuda.stream(cap):
            with torch.cuda.graph(graph, stream=cap):
                prob.step(sb)
        torch.cuda.synchronize()
        for r in range(5):
            prob.step(sa)
            graph.replay()
            prob.density(case.xyz0)
            torch.cuda.synchronize()
            for k in ("u", "v", "v_prev", "g_prev", "scalars"):
                assert torch.equal(getattr(sa, k), getattr(sb, k)), (r, k)
    log(f"[step] captured step: 5 replays equal to the eager steps, hpwl {sb.read()['hpwl']:.6g}")
