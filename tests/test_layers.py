"""The package's multi-die split (host preprocessing before place3d.MultiDie2D) against the
multi-die oracle's split of the same 3D placements: the same nodes, layers, sizes, partial nets,
pin offsets and HBT start positions, bit for bit."""
import dataclasses

import numpy as np
import pytest

from gpu_common import shared_pin_case, tiny_case, with_nets
from oracle import multidie as md
from oracle import optimizer as opt
from paper_2403_09070_amd import layers, synth


def _both(case):
    pb = opt.problem_of(case)
    grid_o = md.Grid2D(case.die_x, case.die_y, case.nx, case.ny)
    grid_p = layers.Grid(case.die_x, case.die_y, case.nx, case.ny)
    args = (case.size, case.kind, case.xyz0, case.net_start, case.pin2node, case.pin_off, pb.geo.dz)
    ref, xy_ref = md.split(*args, grid_o, pb.gamma, hbt_side=1.0)
    got, xy_got = layers.split(*args, grid_p, pb.gamma, hbt_side=1.0)
    return ref, xy_ref, got, xy_got


def _one_die_nets(case):
    """Some nets kept on one die, one empty net and a single-pin net."""
    nets = [case.pin2node[case.net_start[e]:case.net_start[e + 1]] for e in range(len(case.net_start) - 1)]
    nets = nets[:40] + [np.array([], dtype=np.int64), np.array([3])] + nets[40:]
    c = with_nets(case, nets, 2)
    xyz = c.xyz0.copy()
    dz = c.nz * 0.5 * (c.die_x / c.nx + c.die_y / c.ny)
    xyz[2, :100] = 0.25 * dz                  # a block of instances on the bottom die
    return dataclasses.replace(c, xyz0=xyz)


@pytest.mark.parametrize("name", ["tiny", "c1", "one_die_nets", "shared_pins"])
def test_split_matches_the_oracle(name):
    case = {"tiny": lambda: tiny_case(5), "c1": lambda: synth.make_case("c1", 2403),
            "one_die_nets": lambda: _one_die_nets(tiny_case(6)), "shared_pins": lambda: shared_pin_case(14)}[name]()
    ref, xy_ref, got, xy_got = _both(case)
    assert (got.n_inst, got.n_hbt) == (ref.n_inst, ref.n_hbt) and got.n_hbt > 0
    for a in ("w", "h", "kind", "layer", "net_start", "pin2node", "pin_off"):
        assert np.array_equal(np.asarray(getattr(got, a)), np.asarray(getattr(ref, a))), a
    assert np.array_equal(xy_got, xy_ref)
