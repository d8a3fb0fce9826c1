"""place3d_create refuses a malformed netlist with PLACE3D_ERR_NETLIST (and a filler that is
also a macro with PLACE3D_ERR_ARG).

The library reads the netlist back once at creation and checks it on the host before any kernel
uses it: net_start must start at 0, end at n_pins and never decrease; every pin's owner must be
an instance; a filler must hold no pin.  Each case below is a tiny valid problem with one of these
broken (the device arrays keep their sizes, only values change), so nothing out of range reaches
the GPU; a valid problem created afterwards must work as before.
"""
import dataclasses

import numpy as np
import pytest

from gpu_common import gpu_problem, log, need_gpu, tiny_case

pytestmark = pytest.mark.gpu


def _broken(case, what):
    c = dataclasses.replace(case, net_start=case.net_start.copy(), pin2node=case.pin2node.copy(),
                            kind=case.kind.copy())
    ns, p2n = c.net_start, c.pin2node
    if what == "owner_past_end":
        p2n[len(p2n) // 2] = case.n_inst
    elif what == "owner_negative":
        p2n[0] = -1
    elif what == "net_start_decreasing":
        k = int(np.nonzero(np.diff(ns) >= 2)[0][1])        # a net of two or more pins, not the first
        ns[k + 1] = ns[k] - 1 if ns[k] > 0 else ns[k + 2] + 1
        assert np.any(np.diff(ns) < 0)
    elif what == "net_start_short":
        ns[-1] = len(p2n) - 1
    elif what == "filler_with_pin":
        from paper_2403_09070_amd import place3d
        owner = int(p2n[0])
        assert owner < case.meta["n_cells"]                  # a standard cell: not macro, not fixed
        c.kind[owner] = place3d.KIND_FILLER | place3d.KIND_ZFIXED
    elif what == "filler_also_macro":
        from paper_2403_09070_amd import place3d
        pinless = np.setdiff1d(np.arange(case.meta["n_cells"]), p2n)
        i = int(pinless[0]) if len(pinless) else 0
        c.kind[i] = place3d.KIND_FILLER | place3d.KIND_MACRO
    return c


# the status each case must return (the kind rule is an argument error, the others netlist errors)
EXPECT = {"owner_past_end": "ERR_NETLIST", "owner_negative": "ERR_NETLIST", "net_start_decreasing": "ERR_NETLIST",
          "net_start_short": "ERR_NETLIST", "filler_with_pin": "ERR_NETLIST", "filler_also_macro": "ERR_ARG"}


@pytest.mark.parametrize("what", list(EXPECT))
def test_malformed_netlist_is_refused_at_create(what):
    need_gpu()
    from paper_2403_09070_amd import place3d
    log(f"[netlist] {what}")
    case = tiny_case(5)
    with pytest.raises(place3d.Place3dError) as e:
        gpu_problem(_broken(case, what))
    assert place3d.STATUS.get(e.value.code) == EXPECT[what], str(e.value)
    # the library is left usable: the valid problem creates and evaluates
    import torch
    prob = gpu_problem(case)
    _, met = prob.wl_grad(case.xyz0)
    torch.cuda.synchronize()
    assert np.isfinite(met.cpu().numpy()[:4]).all()
