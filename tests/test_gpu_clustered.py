"""Clustered placements, where a few density tiles hold most cells: a tile with more (cell, tile)
entries than one workgroup takes at a time (16384) is split into chunks over several workgroups,
and the chunks' density sums meet in a fixed-point accumulator that the last chunk reads back.

Against the oracle, with the bars of the small-case parity tests: density map rel L2 <= 1e-6 and
its total volume, field gather and exact adjoint rel L2 <= 1e-5 (same float32 maps on both
sides), and one GP step from the oracle's state (metrics 1e-5, overflow 1e-6, preconditioned
gradient 1e-4, step size 1e-5, displacement as for the uniform cases plus twice the floor that
rounding the new positions to float32 sets).  Every case is checked first to hold tiles of several
chunks.  Repeated calls must give the same map bit for bit (the accumulators are left at zero),
and a uniform placement after a clustered one the same map as on a fresh problem.
"""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_common import filler_case, gpu_problem, log, need_gpu, oracle_problem, rel_l2
from oracle import density as oden
from oracle import density_grad as odg
from oracle import optimizer as opt
from oracle import poisson as opois
from oracle.geometry import geometry_of
from paper_2403_09070_amd import place3d, synth

pytestmark = pytest.mark.gpu

CHUNK = 16384      # entries per chunk of a tile (the library's constant)
TILE = 32          # bins per tile side at these grids


def _half_clustered(case, seed=5):
    """Every other movable instance pulled to a patch of 0.05 of the die around (0.3, 0.6) of it,
    the rest left where the generator put them: heavy and light tiles in one map."""
    rng = np.random.default_rng(seed)
    xyz = case.xyz0.astype(np.float64).copy()
    mov = np.nonzero((case.kind & 2) == 0)[0][::2]
    for a, (d, c) in enumerate(((case.die_x, 0.3), (case.die_y, 0.6))):
        xyz[a, mov] = np.clip(c * d + 0.05 * d * rng.standard_normal(mov.size), 0.0, d)
    return dataclasses.replace(case, xyz0=xyz.astype(np.float32))


CASES = {
    "c2_clustered": lambda: synth.centre_start(synth.make_case("c2", 2403), sigma=0.02, seed=2404),
    "c2_half_clustered": lambda: _half_clustered(synth.make_case("c2", 2403)),
    "c1_fillers_clustered": lambda: filler_case(12, config=synth.CONFIGS["c1"], u=0.9, sigma=0.02),
}


def tile_entries(case):
    """(cell, tile) entries per tile at the case's start, from the oracle's footprints: every
    movable cell smaller than a tile is bucketed in each tile its stretched box meets."""
    geo = geometry_of(case)
    box, _ = oden.footprints(case.size, case.kind, case.xyz0, geo)
    cell = ((case.kind & (1 | 2)) == 0)
    tw, th = TILE * geo.wb, TILE * geo.hb
    ntx, nty = -(-case.nx // TILE), -(-case.ny // TILE)
    tx0 = np.clip((box[0] / tw).astype(int), 0, ntx - 1)
    tx1 = np.clip((box[1] / tw).astype(int), 0, ntx - 1)
    ty0 = np.clip((box[2] / th).astype(int), 0, nty - 1)
    ty1 = np.clip((box[3] / th).astype(int), 0, nty - 1)
    count = np.zeros((nty, ntx), dtype=np.int64)
    for i in np.nonzero(cell)[0]:
        count[ty0[i]:ty1[i] + 1, tx0[i]:tx1[i] + 1] += 1
    return count


@pytest.fixture(scope="module", params=list(CASES))
def clustered(request):
    need_gpu()
    log(f"[clustered] case {request.param}")
    case = CASES[request.param]()
    count = tile_entries(case)
    heavy = int((count > CHUNK).sum())
    log(f"[clustered] {request.param}: {case.n_inst} instances, max entries per tile {count.max()}, "
        f"{heavy} tiles of several chunks, {int((count <= CHUNK).sum())} of one")
    assert count.max() > 1.2 * CHUNK, "the case must hold tiles of several chunks"
    return request.param, case, gpu_problem(case, precision=place3d.BF16X3)


def test_density_of_split_tiles(clustered):
    name, case, prob = clustered
    geo = geometry_of(case)
    ref = oden.density_map(case.size, case.kind, case.xyz0, geo)
    got = prob.density(case.xyz0).cpu().numpy()
    again = prob.density(case.xyz0).cpu().numpy()
    err = rel_l2(got, ref)
    log(f"[clustered] {name} density rel_l2={err:.3e} max bin {ref.max():.2f}")
    assert err <= 1e-6
    assert abs(got.astype(np.float64).sum() - ref.sum()) <= 1e-6 * ref.sum()
    assert np.array_equal(got, again), "a second call must find the accumulators cleared"


def test_uniform_map_after_a_clustered_one(clustered):
    name, case, prob = clustered
    uniform = case.xyz0.copy()
    mov = (case.kind & 2) == 0
    rng = np.random.default_rng(3)
    uniform[0, mov] = rng.uniform(0.05, 0.95, mov.sum()) * case.die_x
    uniform[1, mov] = rng.uniform(0.05, 0.95, mov.sum()) * case.die_y
    prob.density(case.xyz0)
    after = prob.density(uniform).cpu().numpy()
    fresh = gpu_problem(case, precision=place3d.BF16X3).density(uniform).cpu().numpy()
    assert np.array_equal(after, fresh)


def test_field_gather_of_split_tiles(clustered):
    name, case, prob = clustered
    geo = geometry_of(case)
    rho = oden.density_map(case.size, case.kind, case.xyz0, geo)
    sol = opois.solve(rho, geo, want=("ex", "ey", "ez"))
    maps = [sol[k].astype(np.float32) for k in ("ex", "ey", "ez")]
    g = prob.field_force(case.xyz0, *(torch.from_numpy(m).cuda() for m in maps), lam=1.0).cpu().numpy()
    ref = odg.field_gather(case.size, case.kind, case.xyz0, *(m.astype(np.float64) for m in maps), geo)
    err = rel_l2(g, ref)
    log(f"[clustered] {name} field-gather rel_l2={err:.3e}")
    assert err <= 1e-5


def test_adjoint_of_split_tiles(clustered):
    name, case, prob = clustered
    geo = geometry_of(case)
    rng = np.random.default_rng(0)
    gmap = rng.normal(size=(case.nz, case.ny, case.nx)).astype(np.float32)
    g = prob.density_vjp(case.xyz0, torch.from_numpy(gmap).cuda()).cpu().numpy()
    ref = odg.density_vjp(case.size, case.kind, case.xyz0, gmap.astype(np.float64), geo)
    err = rel_l2(g, ref)
    log(f"[clustered] {name} density-vjp rel_l2={err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("dgrad", ["field", "adjoint"])
def test_one_step_at_a_clustered_start(clustered, dgrad):
    """One fused GP step (the cells' density-gradient shares summed in the combine) from the
    oracle's state three steps after gp_init at the clustered start (the first moves from the
    bootstrap point are a few hundredths of a length unit, below what float32 positions near the
    die centre resolve to the displacement bar): the new preconditioned gradient and the move."""
    name, case, _ = clustered
    prob = gpu_problem(case, precision=place3d.BF16X3,
                       dgrad=place3d.DGRAD_FIELD if dgrad == "field" else place3d.DGRAD_ADJOINT)
    pb = oracle_problem(case)
    ref = opt.gp_init(pb, case.xyz0, dgrad=dgrad)
    for _ in range(3):
        opt.gp_step(pb, ref, dgrad=dgrad)
    for k in ("u", "v", "v_prev", "g_prev"):
        setattr(ref, k, np.asarray(getattr(ref, k), dtype=np.float32).astype(np.float64))
    st = prob.new_state()
    for k in ("u", "v", "v_prev", "g_prev"):
        getattr(st, k).copy_(torch.from_numpy(np.asarray(getattr(ref, k), dtype=np.float32)))
    sc = np.zeros(place3d.NSCALARS)
    sc[place3d.S["a"]] = ref.a
    sc[place3d.S["lam"]] = ref.lam
    st.scalars.copy_(torch.from_numpy(sc))
    v0 = ref.v.copy()
    prob.step(st)
    m = opt.gp_step(pb, ref, dgrad=dgrad)
    s = st.read()
    step_err = abs(s["step"] - m["step"]) / m["step"]
    disp = rel_l2(st.v.cpu().numpy() - v0, ref.v - v0)
    gerr = rel_l2(st.g_prev.cpu().numpy(), ref.g_prev)
    # the new positions are float32: half an ulp of each, against the move, is a floor the
    # displacement error cannot go below (the moves are small next to the cluster's coordinates)
    floor = float(np.linalg.norm(0.5 * np.spacing(ref.v.astype(np.float32)).astype(np.float64)) /
                  np.linalg.norm(ref.v - v0))
    log(f"[clustered] {name} {dgrad} gradient rel_l2={gerr:.3e} step rel={step_err:.3e} displacement "
        f"rel_l2={disp:.3e} (float32 floor {floor:.2e}) ovfl={m['ovfl_bot']:.4f}/{m['ovfl_top']:.4f}")
    assert gerr <= 1e-4
    assert abs(s["hpwl"] - m["hpwl_d2d"]) <= 1e-5 * m["hpwl_d2d"]
    assert abs(s["ovfl_bot"] - m["ovfl_bot"]) <= 1e-6 and abs(s["ovfl_top"] - m["ovfl_top"]) <= 1e-6
    assert step_err <= 1e-5 and disp <= (5e-5 if dgrad == "field" else 3e-4) + 2.0 * floor
