"""GPU parity of every step of the optimisation ladder (gpp_ladder_fwd,
the paper's Sec. III v0-v8 replayed as gfx950 kernels) against the oracle,
at the same 1e-12 per-entry bar as the production forward."""
import numpy as np
import pytest

import oracle
from paper_2008_11326_amd import inputs as I
from tests.gpu_helpers import assert_parity, mixed_pole_problem, say, to_device

pytestmark = pytest.mark.gpu

STEPS = list(range(12))
SHAPES = [(6, 2, 100, 5, 3), (5, 0, 65, 3, 2), (7, 7, 130, 4, 1), (9, 2, 200, 6, 4),
          (17, 3, 777, 13, 3), (1, 1, 1, 1, 3), (3, 1, 64, 1, 2)]


@pytest.fixture(scope="module")
def ladder():
    from paper_2008_11326_amd import _lib, ladder
    _lib.load()
    return ladder


def run(ladder, step, prob):
    import torch
    d = to_device(prob)
    ach, asx = ladder.ladder_fwd(step, **d, nvband=prob.dims.nvband)
    torch.cuda.synchronize()
    return ach.cpu().numpy(), asx.cpu().numpy()


@pytest.fixture(scope="module")
def cases():
    out = []
    for k, shape in enumerate(SHAPES):
        prob = I.make_problem(I.Dims(*shape), 100 + k, 0.1 if k % 2 else 0.0)
        out.append((f"shape {shape}", prob, oracle.sigma_fwd(prob, nthreads=1)))
    prob = mixed_pole_problem(61, I.Dims(12, 2, 150, 6, 3), 0.5)
    out.append(("tiny-Im lanes and exact poles", prob, oracle.sigma_fwd(prob, nthreads=1)))
    return out


@pytest.mark.parametrize("step", STEPS)
def test_step_against_oracle(ladder, cases, step):
    say(f"[ladder] step {step}: {ladder.ladder_name(step)}")
    for what, prob, ref in cases:
        ach, asx = run(ladder, step, prob)
        assert_parity(ach, ref[0], ref[2], f"step {step} {what} achtemp")
        assert_parity(asx, ref[1], ref[3], f"step {step} {what} asxtemp")


@pytest.mark.parametrize("step", STEPS)
def test_step_empty_dimensions(ladder, step):
    for dims in (I.Dims(0, 0, 64, 4, 3), I.Dims(4, 1, 64, 0, 2)):
        ach, asx = run(ladder, step, I.make_problem(dims, 1))
        assert np.all(ach == 0) and np.all(asx == 0)


def test_steps_at_the_adjoint_workload_size(ladder):
    """The workload the ladder is timed on, against the oracle's stored
    outputs (only the fast steps; the collapsed steps 0-3 re-read the
    G'-column arrays once per band and take seconds)."""
    import json
    import os
    from tests.gpu_helpers import load_golden
    gold = load_golden("adjoint")
    if gold is None:
        pytest.skip("tests/golden/fwd_adjoint.json not generated")
    wl = I.WORKLOADS["adjoint"]
    prob = I.make_problem(wl.dims, wl.seed)
    for step in range(4, 12):
        ach, asx = run(ladder, step, prob)
        e1 = assert_parity(ach, gold["ach"], gold["ach_abs_sum"], f"step {step} achtemp")
        e2 = assert_parity(asx, gold["asx"], gold["asx_abs_sum"], f"step {step} asxtemp")
        say(f"[ladder] step {step} adjoint workload max rel err {max(e1, e2):.2e}")
