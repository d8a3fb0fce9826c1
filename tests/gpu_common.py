"""Shared helpers of the GPU parity tests (imported by tests only)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import optimizer as opt  # noqa: E402
from paper_2403_09070_amd import synth  # noqa: E402


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def tiny_case(seed=5, **kw):
    return synth.make_case(config=synth.small_config(**kw), seed=seed)


def ragged_case(seed=6, nx=37, ny=29):
    """A grid that is not a multiple of any tile size, with macros and a ragged netlist.  Odd
    sides take the dense spectral contractions; even sides (e.g. 38 x 30, halves 19 x 15) the
    folded ones with ragged halves."""
    cfg = synth.small_config(n_cells=700, n_nets=800, die=150.0, nx=nx, ny=ny, nz=4,
                             macros=("uniform", 4, 0.01, 0.04), degree=("geo", 0.75, 70))
    return synth.make_case(config=cfg, seed=seed)


def gpu_problem(case, **kw):
    from paper_2403_09070_amd import place3d
    return place3d.Problem.from_case(case, **kw)


def oracle_problem(case):
    return opt.problem_of(case)


def log(msg):
    print(msg, flush=True)
