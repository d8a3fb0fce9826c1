"""place3d_wl_value_static (the value call whose scratch is the library's static device array)
against place3d_wl_value (the same kernels, scratch in the context's workspace), through the C
ABI: two calls in a row, the second on a smaller netlist, so the second reuses the array the first
left filled.  Both reduce the same per-workgroup partials in the same fixed order, so the totals
agree bit for bit (the floating-point bar, 1e-5 relative, is met a fortiori); the unused slots are
zero.  Sizes beyond the static array are refused with PLACE3D_ERR_SIZE before anything runs."""
import numpy as np
import pytest
import torch

from gpu_common import gpu_problem, log, need_gpu, tiny_case
from paper_2403_09070_amd import place3d, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [place3d.FP32, place3d.BF16X3])
def test_static_value_matches_the_workspace_call(precision):
    need_gpu()
    big = synth.make_case("c2", 2403)          # 200k instances, 220k nets
    small = tiny_case(5)
    for name, case in (("c2", big), ("tiny", small)):
        prob = gpu_problem(case, precision=precision)
        xyz = prob.xyz(case.xyz0)
        ref = prob.wl_value(xyz).cpu().numpy()
        got = prob.wl_value_static(xyz).cpu().numpy()
        torch.cuda.synchronize()
        rel = np.abs(got[:5] - ref[:5]) / np.maximum(np.abs(ref[:5]), 1e-300)
        log(f"[no-alloc] {name} precision={precision} totals {got[:5]} max rel diff {rel.max():.3e}")
        assert np.all(rel <= 1e-5)
        assert np.array_equal(got, ref)
        assert np.all(got[5:] == 0.0)
        del prob


def test_static_value_refuses_what_the_array_cannot_hold():
    need_gpu()
    cfg = synth.small_config(n_cells=(1 << 21) + 16, n_nets=64)
    case = synth.make_case(config=cfg, seed=3)
    prob = gpu_problem(case)
    with pytest.raises(place3d.Place3dError) as e:
        prob.wl_value_static(prob.xyz(case.xyz0))
    assert e.value.code == -2          # PLACE3D_ERR_SIZE
    # the workspace call still takes it
    assert np.isfinite(prob.wl_value(prob.xyz(case.xyz0)).cpu().numpy()[:5]).all()
