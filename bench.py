"""Benchmark: global-placement iterations per second on one MI355X.

Workload: the 1.2M-cell synthetic netlist (150 macros, 1.3M nets, ~4.5M pins, grid
1024 x 1024 x 4, seed 2403).  Two forms run from the same seed:
  plain  -- float32 DCT contractions, the paper's field-gather density gradient
  mixed  -- split-bf16 (hi/lo, three products, float32 accumulation) DCT contractions, same
            field-gather gradient (the precision form of this workload)
  autograd (optional, --forms) -- split-bf16 contractions with the exact-adjoint density gradient
A step is one full GP iteration (place3d_step): density map, spectral solve, density gradient,
bistratal WA wirelength with the FDA z-gradient, preconditioned Nesterov move.  `value` is the
mixed form's iterations/s over exactly --steps timed steps after --warmup warm-up and
--profile-steps untimed ones, with the metrics read back to the host every --readback-every
steps inside the timed loop (a placer's convergence check); the plain form's rate, both final
D2D HPWLs and their relative difference are reported beside it, the HPWLs taken after
--hpwl-iters iterations (untimed steps follow the timed ones when fewer were run).  With --repeats R the forms
alternate R times, each repeat from the same start, and the median rate is reported.

The roofline entry is for the stage with the largest GPU time in the mixed step (found in an
untimed block of steps with every stage's launches bracketed by HIP events); its average launch
time comes from HIP events on the launch stream around that stage's launches only, during the
timed steps.  The CPU baseline is one full FP64 oracle iteration of the same workload, stage by
stage.

``--ablation precond`` runs the preconditioner ablation instead (one JSON line, curves to
``--ablation-csv``): the mixed-size preconditioner against the ePlace and ePlace3D forms on the
macro-heavy 200k-cell workload from a clustered start.  ``--ablation algo`` times the density map
and the wirelength call with the paper's baseline algorithms (instance-parallel macro scatter,
O(|P_e|^2) FDA) against the default ones on the 1.2M-cell workload.  ``--ablation converge`` runs
global placement on the 4M-cell workload from a clustered start until the overflow is below 0.1,
for the plain, mixed and autograd forms.  ``--ablation divergence`` records the per-iteration
HPWL of plain, mixed, and plain from a start moved by one ulp (default workload c1).
``--ablation md2d`` times multi-die 2D global placement (Sec. III-C) on the die split of a 3D
placement of the 1.2M-cell workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GP iterations/s at 1.2M cells: BF16-split vs FP32, HPWL within 0.1%"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0}


def gemm_flops_per_step(nx, ny, nz, dgrad_field, bf16x3):
    """Executed MFMA flops of the DCT contractions in one step (3 products per contraction in the
    split form).  Dense: x passes M = nz ny, N = K = nx; y passes nz batches of M = ny, N = nx,
    K = ny.  With even nx and ny every pass is folded into an even and an odd half of half the
    size each, which halves its flops."""
    x_pass = 2.0 * nz * ny * nx * nx
    y_pass = 2.0 * nz * ny * nx * ny
    if dgrad_field:          # forward x, y; inverse y (cos, sin); inverse x (Ex, Ey, Ez)
        total = x_pass + y_pass + 2 * y_pass + 3 * x_pass
    else:                    # forward x, y; inverse y (cos); inverse x (phi)
        total = x_pass + y_pass + y_pass + x_pass
    if nx % 2 == 0 and ny % 2 == 0:
        total *= 0.5
    return total * (3.0 if bf16x3 else 1.0)


def wl_bytes(n, P, m):
    """Algorithmic bytes of the wirelength sweep: per pin the owner index and four offsets (20 B),
    per instance the xyz read and the gradient write (24 B), per net its CSR entry (4 B)."""
    return 20.0 * P + 24.0 * n + 4.0 * m


def density_bytes(n, bins):
    """Algorithmic bytes of the density map: per instance xyz and four sizes (28 B), per bin the
    fixed-instance map read and the map write (8 B)."""
    return 28.0 * n + 8.0 * bins


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.txt")


def recorded_traffic(stage, form, workload):
    """HBM bytes per launch of a stage, from the rocprofv3 FETCH_SIZE / WRITE_SIZE counts recorded in
    profiles/hbm_traffic.txt (already scaled by the copy-kernel factors noted there), or None when
    nothing is recorded for this stage, form and workload or the stage's kernel source has changed
    since."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    for line in open(TRAFFIC_FILE):
        if not line.startswith("stage="):
            continue
        rec = dict(kv.split("=", 1) for kv in line.split())
        if rec.get("stage") != stage or rec.get("form") != form or rec.get("workload") != workload:
            continue
        src = os.path.join(ROOT, rec["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["sha256"]:
            return None
        return float(rec["bytes_per_launch"])
    return None


def run_forms(case, names, forms, args, log):
    """Time the forms in alternation, args.repeats times each, every repeat from a fresh
    gp_init at the same start: warm-up steps, args.profile_steps untimed steps, then args.steps
    timed steps with the host reading the metrics back every args.readback_every steps (a placer's
    convergence check, through pinned memory, one period late, so the GPU never waits for it).  In the first repeat the reported form's untimed steps carry HIP events
    around every stage's launches, which give the per-stage breakdown and the dominant stage; its
    timed steps then carry events around that stage's launches only (one pair per step for the
    four back-to-back contractions), which give its average launch time under the timed
    conditions.  The other forms run without events.  Rates are medians over the repeats."""
    import statistics
    import torch
    from paper_2403_09070_amd import place3d
    head = "mixed" if "mixed" in names else names[0]
    probs = {nm: place3d.Problem.from_case(case, precision=forms[nm][0], dgrad=forms[nm][1]) for nm in names}
    out = {nm: dict(runs=[], state=None, prof=None, timed=None) for nm in names}
    dominant, ev_ms, ev_n = None, 0.0, 0
    for r in range(args.repeats):
        for nm in names:
            prob = probs[nm]
            st = prob.gp_init(case.xyz0)
            for _ in range(args.warmup):
                prob.step(st)
            events = nm == head
            if events and r == 0 and args.profile_steps > 0:
                prob.profile(True)
                for _ in range(args.profile_steps):
                    prob.step(st)
                torch.cuda.synchronize()
                prof = prob.profile_read(reset=True)
                prob.profile(False)
                out[nm]["prof"] = prof
                dominant = max(prof, key=lambda k: prof[k][0])
            else:
                for _ in range(args.profile_steps):
                    prob.step(st)
            if events and dominant is not None:
                prob.profile(True, stages=(dominant,))
            # the convergence check copies the metrics into pinned host memory without waiting and
            # reads each copy at the next check, when it has long completed (a check one period late)
            host = torch.empty(st.scalars.shape, dtype=st.scalars.dtype, pin_memory=True)
            pending = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(args.steps):
                prob.step(st)
                if args.readback_every and (k + 1) % args.readback_every == 0:
                    if pending is not None:
                        pending.synchronize()
                        float(host[place3d.S["ovfl_bot"]])
                    host.copy_(st.scalars, non_blocking=True)
                    pending = torch.cuda.Event()
                    pending.record()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if events and dominant is not None:
                ms, cnt = prob.profile_read(reset=True)[dominant]
                prob.profile(False)
                ev_ms, ev_n = ev_ms + ms, ev_n + cnt
            out[nm]["runs"].append(args.steps / dt)
            # untimed steps after the timed ones, so that the final HPWLs compared between the
            # forms are taken at --hpwl-iters iterations whatever --steps is
            for _ in range(max(0, args.hpwl_iters - (args.warmup + args.profile_steps + args.steps))):
                prob.step(st)
            out[nm]["state"] = st.read()
            log(f"[bench] repeat {r} form {nm}: {args.steps / dt:.1f} it/s, hpwl {out[nm]['state']['hpwl']:.6e}")
    for nm in names:
        ips = statistics.median(out[nm]["runs"])
        out[nm].update(ips=ips, ms=1e3 / ips)
    if dominant is not None:
        out[head]["timed"] = (dominant, (ev_ms, ev_n))
    del probs
    torch.cuda.empty_cache()
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case):
    """One full FP64 oracle GP iteration of the same workload, stage by stage and unsampled: the
    wirelength with the vanilla FDA, the density map, the dense spectral solve, the field gather,
    the preconditioned gradient, the Nesterov move and the overflow (the steps of
    oracle.optimizer.gp_step, called one by one to time them), from the start placement.  The
    spectral solve's contractions run on the BLAS thread pool and are timed again on one thread;
    every other stage is single-threaded NumPy."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import density as den
    from oracle import density_grad as dg
    from oracle import optimizer as opt
    from oracle import poisson
    from oracle import wirelength as wl
    pb = opt.problem_of(case)
    geo = pb.geo
    pool = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    t = {}
    v = opt.clamp(pb, case.xyz0)
    t0 = time.perf_counter()
    w = wl.wirelength(pb.size, pb.kind, v, pb.net_start, pb.pin2node, pb.pin_off, geo, pb.gamma, pb.alpha)
    t["wirelength"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    rho = den.density_map(pb.size, pb.kind, v, geo)
    t["density"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    sol = poisson.solve(rho, geo, want=("phi", "ex", "ey", "ez"))
    t["field"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    gd = dg.field_gather(pb.size, pb.kind, v, sol["ex"], sol["ey"], sol["ez"], geo)
    t["gather"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    lam = 1.0
    g = (w["grad"] + lam * gd) / opt.preconditioner(pb, v, lam)[None, :]
    st = opt.GPState(u=v.copy(), v=v.copy(), v_prev=v.copy(), g_prev=np.zeros_like(g), a=1.0, lam=lam)
    opt.nesterov_update(st, g, lambda p: opt.clamp(pb, p), pb.movable)
    opt.overflow(pb, rho, v)
    t["update"] = time.perf_counter() - t0
    per_iter = sum(t.values())
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        poisson.solve(rho, geo, want=("phi", "ex", "ey", "ez"))
        field_1 = time.perf_counter() - t0
    per_iter_1 = per_iter - t["field"] + field_1
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": 1.0 / per_iter, "unit": "iterations/s", "cores": int(pool), "kind": "oracle",
            "sample": (f"one full FP64 oracle GP iteration of the same {case.n_inst}-instance workload at its "
                       f"start placement, every instance and net (no sampling, no extrapolation): the stages of "
                       f"oracle.optimizer.gp_step timed one by one"),
            "seconds_per_iteration": per_iter,
            "stage_seconds": {k: round(x, 3) for k, x in t.items()},
            "threads_per_stage": {"wirelength": 1, "density": 1, "field": int(pool), "gather": 1, "update": 1},
            "one_thread": {"value": 1.0 / per_iter_1, "seconds_per_iteration": per_iter_1,
                           "field_seconds": round(field_1, 3)},
            "host": {"nproc": os.cpu_count(), "affinity": affinity, "cpu_model": _cpu_model(),
                     "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}}


def precond_ablation(args, log):
    """Eq. improved-precond against the ePlace (|E_i| + lambda q_i) and ePlace3D (lambda q_i) forms of
    Eq. general-precond (Sec. III-A, and the preconditioner ablation of Sec. V): the same macro-heavy
    netlist is placed from the same clustered start with each form, recording per iteration the D2D
    HPWL and per-die overflow (fillers left out), and every --ablation-every iterations the macro
    density overflow, i.e. the overflow of the map of the macros alone against the target density.
    Fillers (z-fixed and free, Eqs. filler-vol and free-filler-vol) fill the region unless
    --ablation-util is 0."""
    import numpy as np
    import torch
    from paper_2403_09070_amd import place3d, synth
    case = synth.centre_start(synth.make_case(args.config, args.seed), sigma=args.ablation_spread, seed=args.seed + 1)
    nc = case.meta["n_cells"]
    plan = None
    if args.ablation_util > 0:
        plan = place3d.plan_fillers(case.size, case.kind, case.xyz0[2], case.die_x, case.die_y, case.nx, case.ny,
                                    case.nz, args.ablation_util, args.ablation_util)
        case = synth.with_fillers(case, plan, sigma=args.ablation_spread, seed=args.seed + 2)
        log(f"[ablation] fillers: {plan['n_top']} + {plan['n_bot']} z-fixed, {plan['n_free']} free")
    start = case.xyz0
    sig = args.ablation_spread
    mac = np.nonzero((case.kind & place3d.KIND_MACRO) != 0)[0]
    params = place3d.Problem.case_params(case)
    mprob = place3d.Problem(size=case.size[:, mac], kind=case.kind[mac], net_start=np.zeros(1, np.int32),
                            pin2node=np.zeros(0, np.int32), pin_off=np.zeros((4, 0), np.float32),
                            fixed_xyz=case.xyz0[:, mac], die_x=case.die_x, die_y=case.die_y,
                            nx=case.nx, ny=case.ny, nz=case.nz, gamma=params["gamma"], alpha=params["alpha"],
                            target_density=params["target_density"])
    mac_t = torch.as_tensor(mac, device="cuda", dtype=torch.long)
    target = mprob.params["target_density"]
    half = case.nz // 2

    def macro_overflow(v):
        rho = mprob.density(v.index_select(1, mac_t))
        ex = (rho - target).clamp(min=0.0)
        return [float(x) for x in torch.stack([ex[:half].sum() / rho[:half].sum().clamp(min=1e-30),
                                               ex[half:].sum() / rho[half:].sum().clamp(min=1e-30),
                                               ex.sum() / rho.sum()]).cpu()]

    forms = {"mixed": place3d.PRECOND_MIXED, "eplace": place3d.PRECOND_EPLACE,
             "eplace3d": place3d.PRECOND_EPLACE3D}
    rows, summary = [], {}
    for name, code in forms.items():
        prob = place3d.Problem.from_case(case, precision=place3d.BF16X3, precond=code)
        st = prob.gp_init(start)
        h0 = None
        stop_at, diverged, mo_after = None, False, []
        t0 = time.perf_counter()
        for k in range(args.ablation_iters):
            prob.step(st)
            s = st.read()
            mo = macro_overflow(st.v) if (k % args.ablation_every == 0 or k == args.ablation_iters - 1) else None
            h0 = s["hpwl"] if h0 is None else h0
            ov = max(s["ovfl_bot"], s["ovfl_top"])
            rows.append((name, k, s["hpwl"], s["ovfl_bot"], s["ovfl_top"], s["lam"], s["step"], s["ncut"],
                         *(mo if mo else (float("nan"),) * 3)))
            if mo and k >= args.ablation_iters // 4:
                mo_after.append(mo[2])
            if stop_at is None and ov < args.ablation_stop:
                stop_at = dict(iteration=k, hpwl=s["hpwl"], ovfl=ov, ncut=s["ncut"],
                               macro_ovfl=macro_overflow(st.v)[2])
            if not np.isfinite(s["hpwl"]) or s["hpwl"] > 20.0 * h0:
                diverged = True
                break
            if (k + 1) % 200 == 0:
                log(f"  {name} it {k + 1}: hpwl {s['hpwl']:.5e} ovfl {s['ovfl_bot']:.3f}/{s['ovfl_top']:.3f} "
                    f"macro {mo_after[-1] if mo_after else float('nan'):.4f}")
        torch.cuda.synchronize()
        s = st.read()
        mo = macro_overflow(st.v)
        summary[name] = dict(iterations=k + 1, diverged=diverged, final_hpwl=s["hpwl"],
                             final_ovfl=[s["ovfl_bot"], s["ovfl_top"]], final_macro_ovfl=mo[2],
                             reached=stop_at, macro_ovfl_late_max=max(mo_after) if mo_after else None,
                             macro_ovfl_late_mean=float(np.mean(mo_after)) if mo_after else None,
                             seconds=round(time.perf_counter() - t0, 2))
        log(f"[ablation] {name}: {summary[name]}")
        del prob
        torch.cuda.empty_cache()
    if args.ablation_csv:
        os.makedirs(os.path.dirname(os.path.abspath(args.ablation_csv)), exist_ok=True)
        with open(args.ablation_csv, "w") as f:
            f.write("precond,iteration,hpwl,ovfl_bot,ovfl_top,lambda,step,ncut,macro_ovfl_bot,macro_ovfl_top,"
                    "macro_ovfl\n")
            for r in rows:
                f.write(",".join(str(x) for x in r) + "\n")
    ref = summary["mixed"]
    for name in ("eplace", "eplace3d"):
        a, b = summary[name].get("reached"), ref.get("reached")
        summary[name]["hpwl_vs_mixed_at_stop"] = (a["hpwl"] / b["hpwl"]) if a and b else None
    fill = (f", fillers for utilisation {args.ablation_util}: {plan['n_top']} + {plan['n_bot']} z-fixed, "
            f"{plan['n_free']} free") if plan else ", no fillers"
    print(json.dumps({"ablation": "preconditioner", "workload": f"{args.config} seed {args.seed}, "
                      f"{nc} cells + {len(mac)} macros, clustered start (sigma {sig} of the die){fill}",
                      "stop_overflow": args.ablation_stop, "forms": summary}), flush=True)


def algo_ablation(args, log):
    """The paper's algorithm ablation (Sec. IV; its Fig. acc-density) on this hardware: the density
    map with large instances scattered instance-parallel (one thread per instance, global atomics)
    against the tile-resident bin-parallel sweep, and the wirelength call with the O(|P_e|^2)
    vanilla FDA against the incremental one.  Each call is timed alone (HIP events on the launch
    stream, mean over --ablation-iters calls after 5 warm-up calls) at the workload's start."""
    import torch
    from paper_2403_09070_amd import place3d, synth
    case = synth.make_case(args.config, args.seed)
    forms = {"default": 0, "macro_instance": place3d.OPT_MACRO_INSTANCE, "fda_vanilla": place3d.OPT_FDA_VANILLA}
    out = {}
    for name, opt in forms.items():
        prob = place3d.Problem.from_case(case, precision=place3d.BF16X3, options=opt)
        xyz = prob.xyz(case.xyz0)
        rho = prob.new_map()
        g = torch.empty((3, prob.n), dtype=torch.float32, device="cuda")
        res = {}
        for call, fn in (("density", lambda: prob.density(xyz, out=rho)), ("wl_grad", lambda: prob.wl_grad(xyz, out=g))):
            for _ in range(5):
                fn()
            torch.cuda.synchronize()
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(args.ablation_iters):
                fn()
            t1.record()
            torch.cuda.synchronize()
            res[call + "_ms"] = t0.elapsed_time(t1) / args.ablation_iters
        out[name] = res
        log(f"[ablation] {name}: {res}")
        del prob
        torch.cuda.empty_cache()
    d, m, v = out["default"], out["macro_instance"], out["fda_vanilla"]
    print(json.dumps({"ablation": "algorithms", "workload": f"{args.config} seed {args.seed}: {case.meta['n_cells']} "
                      f"cells + {case.meta['n_macros']} macros, {case.n_nets} nets, {case.n_pins} pins, grid "
                      f"{case.nx}x{case.ny}x{case.nz}", "calls": args.ablation_iters, "forms": out,
                      "density_speedup_tiles_over_instance": m["density_ms"] / d["density_ms"],
                      "wl_speedup_incremental_over_vanilla": v["wl_grad_ms"] / d["wl_grad_ms"],
                      "paper_context": {"density": 4.7, "fda": 1.7}}), flush=True)


def divergence_run(args, log):
    """Per-iteration D2D HPWL of three runs from the workload's start: plain (float32 contractions),
    mixed (split-bf16) and plain again from the start with one coordinate (the first movable
    instance's x) moved by one float32 ulp.  The relative HPWL difference of mixed against plain,
    beside that of the one-ulp run against plain, separates what the split form changes from the
    trajectory's own sensitivity to rounding.  --ablation-iters iterations (default: 525, 1025 for
    c2); the full curves go to --ablation-csv."""
    import numpy as np
    import torch
    from paper_2403_09070_amd import place3d, synth
    case = synth.make_case(args.config, args.seed)
    iters = args.ablation_iters
    mov = np.nonzero((case.kind & synth.KIND_FIXED) == 0)[0]
    xyz_ulp = case.xyz0.copy()
    i0 = int(mov[0])
    xyz_ulp[0, i0] = np.nextafter(xyz_ulp[0, i0], np.float32(np.inf))
    runs = {"plain": (place3d.FP32, case.xyz0), "mixed": (place3d.BF16X3, case.xyz0),
            "plain_1ulp": (place3d.FP32, xyz_ulp)}
    curves = {}
    for name, (precision, xyz0) in runs.items():
        prob = place3d.Problem.from_case(case, precision=precision)
        st = prob.gp_init(xyz0)
        h = np.empty(iters)
        for k in range(iters):
            prob.step(st)
            h[k] = st.read()["hpwl"]
        curves[name] = h
        log(f"[divergence] {name}: hpwl at {iters} = {h[-1]:.6e}")
        del prob
        torch.cuda.empty_cache()
    d_mixed = np.abs(curves["mixed"] - curves["plain"]) / curves["plain"]
    d_ulp = np.abs(curves["plain_1ulp"] - curves["plain"]) / curves["plain"]
    marks = [k for k in (1, 2, 5, 10, 20, 50, 100, 200, 300, 400, 500, 700, 1000) if k <= iters]
    if iters not in marks:
        marks.append(iters)
    if args.ablation_csv:
        with open(args.ablation_csv, "w") as f:
            f.write("iteration,hpwl_plain,hpwl_mixed,hpwl_plain_1ulp,rel_mixed,rel_1ulp\n")
            for k in range(iters):
                f.write(f"{k + 1},{curves['plain'][k]:.9e},{curves['mixed'][k]:.9e},{curves['plain_1ulp'][k]:.9e},"
                        f"{d_mixed[k]:.3e},{d_ulp[k]:.3e}\n")
    print(json.dumps({"run": "divergence", "workload": f"{args.config} seed {args.seed}: {case.meta['n_cells']} "
                      f"cells + {case.meta['n_macros']} macros, {case.n_nets} nets, {case.n_pins} pins, grid "
                      f"{case.nx}x{case.ny}x{case.nz}", "iterations": iters, "perturbed": f"x of instance {i0}, +1 ulp",
                      "rel_hpwl_mixed_vs_plain": {str(k): float(d_mixed[k - 1]) for k in marks},
                      "rel_hpwl_1ulp_vs_plain": {str(k): float(d_ulp[k - 1]) for k in marks},
                      "max_rel_mixed": float(d_mixed.max()), "max_rel_1ulp": float(d_ulp.max())}), flush=True)


def md2d_run(args, log):
    """Multi-die 2D global placement (Sec. III-C, Eq. 2d-place) after 3D global placement: the
    workload placed by --md-3d-iters mixed 3D steps from its start, split by die with the
    package's ``layers.split`` (one HBT per crossing net, started in its optimal region; the split
    is timed on the host), then --warmup and --steps multi-die 2D steps in float32 and in
    split-bf16 form from the same split: iterations/s, the partial nets' HPWL and the per-layer
    overflow (bottom, top, HBT layer) after the timed steps.  Inputs are resident on the GPU before
    timing; no host readback inside the timed loop."""
    import numpy as np
    import torch
    from paper_2403_09070_amd import layers, place3d, synth
    case = synth.make_case(args.config, args.seed)
    params = place3d.Problem.case_params(case)
    prob3 = place3d.Problem.from_case(case, precision=place3d.BF16X3)
    st3 = prob3.gp_init(case.xyz0)
    for _ in range(args.md_3d_iters):
        prob3.step(st3)
    torch.cuda.synchronize()
    xyz = st3.v.cpu().numpy().astype(np.float64)
    s3 = st3.read()
    del prob3, st3
    torch.cuda.empty_cache()
    wb = case.die_x / case.nx
    dz = case.nz * 0.5 * (wb + case.die_y / case.ny)
    t0 = time.perf_counter()
    lay, xy0 = layers.split(case.size, case.kind, xyz, case.net_start, case.pin2node, case.pin_off, dz,
                            layers.Grid(case.die_x, case.die_y, case.nx, case.ny), params["gamma"],
                            hbt_side=case.config.hbt_pitch, ramp=params["lambda_ramp"],
                            target=params["target_density"])
    t_split = time.perf_counter() - t0
    xy0 = xy0.astype(np.float32)
    log(f"[md2d] split after {args.md_3d_iters} 3D steps: {lay.n_hbt} HBTs, {len(lay.net_start) - 1} partial nets, "
        f"{t_split:.2f} s")
    out = {}
    for name, precision in (("plain", place3d.FP32), ("mixed", place3d.BF16X3)):
        prob = place3d.MultiDie2D.from_layered(lay, fixed_xy=xy0, precision=precision)
        st = prob.gp_init(xy0)
        for _ in range(args.warmup):
            prob.step(st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            prob.step(st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s = st.read()
        out[name] = dict(iters_per_s=round(args.steps / dt, 1), ms_per_step=round(1e3 * dt / args.steps, 4),
                         hpwl=s["hpwl"], ovfl=[s["ovfl_bot"], s["ovfl_top"], s["ovfl_hbt"]])
        log(f"[md2d] {name}: {out[name]}")
        del prob, st
        torch.cuda.empty_cache()
    print(json.dumps({"run": "multi-die 2D", "workload": f"{args.config} seed {args.seed}: {case.meta['n_cells']} "
                      f"cells + {case.meta['n_macros']} macros, {case.n_nets} nets, {case.n_pins} pins, grid "
                      f"{case.nx}x{case.ny}", "iterations_3d": args.md_3d_iters, "hpwl_3d_d2d": s3["hpwl"],
                      "n_hbt": int(lay.n_hbt), "partial_nets": int(len(lay.net_start) - 1),
                      "nodes": int(lay.w.shape[0]), "pins": int(lay.pin2node.shape[0]), "split_seconds": round(t_split, 3),
                      "steps": args.steps, "warmup": args.warmup, "forms": out,
                      "mixed_over_plain": round(out["mixed"]["iters_per_s"] / out["plain"]["iters_per_s"], 3),
                      "hpwl_rel_diff": abs(out["mixed"]["hpwl"] - out["plain"]["hpwl"]) / out["plain"]["hpwl"]}),
          flush=True)


def converge_run(args, log):
    """Global placement from a clustered start until the larger per-die overflow falls below
    --converge-overflow (or --converge-max iterations), for the plain (float32, field gather),
    mixed (split-bf16, field gather) and autograd (split-bf16, exact adjoint) forms from the same
    start; the host reads the overflow and HPWL back every 10 iterations, inside the timed loop,
    as a placer's convergence check does."""
    import torch
    from paper_2403_09070_amd import place3d, synth
    case = synth.centre_start(synth.make_case(args.config, args.seed), sigma=args.ablation_spread, seed=args.seed + 1)
    forms = {"plain": (place3d.FP32, place3d.DGRAD_FIELD), "mixed": (place3d.BF16X3, place3d.DGRAD_FIELD),
             "autograd": (place3d.BF16X3, place3d.DGRAD_ADJOINT)}
    out = {}
    for name in args.forms.split(","):
        precision, dgrad = forms[name]
        prob = place3d.Problem.from_case(case, precision=precision, dgrad=dgrad)
        st = prob.gp_init(case.xyz0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, s = 0, None
        while it < args.converge_max:
            for _ in range(10):
                prob.step(st)
            it += 10
            s = st.read()
            if max(s["ovfl_bot"], s["ovfl_top"]) < args.converge_overflow:
                break
            if it % 200 == 0:
                log(f"  {name} it {it}: hpwl {s['hpwl']:.5e} ovfl {s['ovfl_bot']:.3f}/{s['ovfl_top']:.3f}")
        dt = time.perf_counter() - t0
        out[name] = dict(iterations=it, seconds=round(dt, 3), iters_per_s=round(it / dt, 1), hpwl=s["hpwl"],
                         ovfl=[s["ovfl_bot"], s["ovfl_top"]], ncut=s["ncut"],
                         reached=max(s["ovfl_bot"], s["ovfl_top"]) < args.converge_overflow)
        log(f"[converge] {name}: {out[name]}")
        del prob
        torch.cuda.empty_cache()
    if "plain" in out:
        for name in out:
            out[name]["hpwl_vs_plain"] = out[name]["hpwl"] / out["plain"]["hpwl"]
            out[name]["time_vs_plain"] = out["plain"]["seconds"] / out[name]["seconds"]
    print(json.dumps({"run": "to overflow", "workload": f"{args.config} seed {args.seed}: {case.meta['n_cells']} "
                      f"cells + {case.meta['n_macros']} macros, {case.n_nets} nets, {case.n_pins} pins, grid "
                      f"{case.nx}x{case.ny}x{case.nz}, clustered start (sigma {args.ablation_spread} of the die), "
                      f"no fillers", "target_overflow": args.converge_overflow, "forms": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default=None, help="workload (default c4; c2 for --ablation)")
    ap.add_argument("--seed", type=int, default=2403)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=1, help="timed repeats per form (median reported)")
    ap.add_argument("--readback-every", type=int, default=10,
                    help="read the metrics back to the host every this many timed steps (0: never)")
    ap.add_argument("--hpwl-iters", type=int, default=525,
                    help="iterations after gp_init at which the forms' final HPWLs are compared (untimed steps "
                         "follow the timed ones when --warmup + --profile-steps + --steps is fewer)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="plain,mixed,autograd")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first copy a float32 buffer of this many MiB three times (a plain copy kernel of "
                         "known traffic, to scale hardware byte counters)")
    ap.add_argument("--ablation", choices=["precond", "algo", "converge", "divergence", "md2d"], default=None,
                    help="run an ablation or study instead of the timing benchmark")
    ap.add_argument("--ablation-iters", type=int, default=1000)
    ap.add_argument("--ablation-every", type=int, default=5)
    ap.add_argument("--ablation-spread", type=float, default=0.02)
    ap.add_argument("--ablation-stop", type=float, default=0.1)
    ap.add_argument("--md-3d-iters", type=int, default=200, help="3D steps before the multi-die split (md2d)")
    ap.add_argument("--converge-overflow", type=float, default=0.1)
    ap.add_argument("--converge-max", type=int, default=3000)
    ap.add_argument("--ablation-util", type=float, default=0.8,
                    help="maximum utilisation u of both dies for the fillers (0: no fillers)")
    ap.add_argument("--ablation-csv", default=None)
    args = ap.parse_args()
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (this path has no "
              f"multi-GPU form).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2403_09070_amd import place3d, synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    place3d.lib()
    if args.ablation == "precond":
        args.config = args.config or "c2"
        precond_ablation(args, log)
        return
    if args.ablation == "algo":
        args.config = args.config or "c4"
        algo_ablation(args, log)
        return
    if args.ablation == "converge":
        args.config = args.config or "c5"
        converge_run(args, log)
        return
    if args.ablation == "md2d":
        args.config = args.config or "c4"
        md2d_run(args, log)
        return
    if args.ablation == "divergence":
        args.config = args.config or "c1"
        if "--ablation-iters" not in sys.argv:
            args.ablation_iters = 1025 if args.config == "c2" else 525
        divergence_run(args, log)
        return
    args.config = args.config or "c4"
    if args.copy_mb > 0:
        src = torch.ones(args.copy_mb * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] copied {args.copy_mb} MiB x3")
    log(f"[bench] generating {args.config} seed {args.seed}")
    case = synth.make_case(args.config, args.seed)
    forms = {"plain": (place3d.FP32, place3d.DGRAD_FIELD), "mixed": (place3d.BF16X3, place3d.DGRAD_FIELD),
             "autograd": (place3d.BF16X3, place3d.DGRAD_ADJOINT)}
    names = args.forms.split(",")
    log(f"[bench] forms {names}: {args.repeats} repeats of warmup {args.warmup} + {args.profile_steps} untimed + "
        f"{args.steps} timed steps")
    res = run_forms(case, names, forms, args, log)
    head = res.get("mixed") or res[list(res)[0]]
    head_name = "mixed" if "mixed" in res else list(res)[0]
    bf16x3 = head_name in ("mixed", "autograd")
    n, P, m = case.n_inst, case.n_pins, case.n_nets
    bins = case.nx * case.ny * case.nz

    roof = None
    if head["prof"]:
        prof = head["prof"]
        ps = args.profile_steps
        field_form = head_name != "autograd"
        cands = {
            "gemm": ("mfma", gemm_flops_per_step(case.nx, case.ny, case.nz, field_form, bf16x3) / 1e12,
                     PEAK_TFLOPS["bf16" if bf16x3 else "f32"], "TFLOP/s"),
            "wl_nets": ("hbm", wl_bytes(n, P, m) / 1e9, HBM_PEAK_GBS, "GB/s"),
            "density": ("hbm", density_bytes(n, bins) / 1e9, HBM_PEAK_GBS, "GB/s"),
        }
        per_step_ms = {k: v[0] / ps for k, v in prof.items()}
        key, (ms, launches) = head["timed"]
        if key not in cands:
            key, (ms, launches) = "gemm", prof["gemm"]
        bound, work, peak, unit = cands[key]
        lps = launches / (args.steps * args.repeats if key == head["timed"][0] else ps)
        avg_ms = ms / launches
        achieved = (work / lps) / (avg_ms / 1e3)        # per launch / average launch duration
        traffic = recorded_traffic(key, head_name, args.config)
        roof = {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": key,
                "avg_launch_ms": round(avg_ms, 4), "launches_per_step": lps,
                "timing": "HIP events around this stage's launches during the timed steps",
                "stage_ms_per_step_all_events": {k: round(v, 4) for k, v in per_step_ms.items()},
                # HBM bytes per launch of each stage from the recorded FETCH_SIZE / WRITE_SIZE counters
                # (null where none is recorded for the current source), beside its algorithmic bytes
                "stage_traffic_bytes": {k: recorded_traffic(k, head_name, args.config)
                                        for k in ("bucket", "density", "gemm", "wl_nets")},
                "stage_algorithmic_bytes": {"bucket+density": density_bytes(n, bins),
                                            "wl_nets": wl_bytes(n, P, m)}}

    line = {
        "metric": METRIC, "value": round(head["ips"], 2), "unit": "iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms"], 4),
        "repeats": args.repeats, "readback_every": args.readback_every,
        "runs_iters_per_s": [round(v, 1) for v in head["runs"]],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3/f32" if bf16x3 else "f32", "data": "synthetic",
        "config": {"workload": f"{args.config}: {n - case.meta['n_macros']} cells + {case.meta['n_macros']} macros, "
                               f"{m} nets, {P} pins, grid {case.nx}x{case.ny}x{case.nz}, seed {args.seed}",
                   "form": head_name, "parallelism": "single GPU"},
    }
    if "plain" in res and "mixed" in res:
        hp, hm = res["plain"]["state"]["hpwl"], res["mixed"]["state"]["hpwl"]
        line["config"].update({"plain_iters_per_s": round(res["plain"]["ips"], 2),
                               "mixed_over_plain": round(res["mixed"]["ips"] / res["plain"]["ips"], 3),
                               "hpwl_plain": hp, "hpwl_mixed": hm, "hpwl_rel_diff": abs(hm - hp) / hp,
                               "iterations": max(args.hpwl_iters, args.warmup + args.profile_steps + args.steps)})
    if "plain" in res and "autograd" in res:
        hp, ha = res["plain"]["state"]["hpwl"], res["autograd"]["state"]["hpwl"]
        line["config"].update({"autograd_iters_per_s": round(res["autograd"]["ips"], 2),
                               "autograd_over_plain": round(res["autograd"]["ips"] / res["plain"]["ips"], 3),
                               "hpwl_autograd": ha, "hpwl_autograd_rel_diff": abs(ha - hp) / hp})
    if roof:
        line["roofline"] = roof
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle sample)")
        line["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
