"""GPU: classification pipelining of prescribed-motion solves
(IBM_OPT_PIPELINE).  The next step's classification runs on a side stream
into a second set of buffers while the current step's stages run; the
states must be bit-identical to classifying each step before its stages,
across calls of ibm_advance, with explicit classifications and time resets
in between; and a non-finite state is reported whichever buffer is
current."""
import numpy as np
import pytest
import torch

import workloads as w
from gpu_common import smooth_prim

pytestmark = pytest.mark.gpu

CASES = {
    "moving-cylinder": lambda: w.small_case("moving-cylinder", 64, steps=5),
    "tube-moving": lambda: w.small_case("tube", 32, steps=5, nz=8, ntheta=64, nzt=4),
    "supersonic-moving": lambda: w.small_case("supersonic-moving-cylinder", 40, steps=5),
    "moving-cylinder-dual": lambda: _dual_moving(),
}


def _dual_moving():
    import dataclasses
    from workloads.cases import dual_dt
    c = w.small_case("moving-cylinder", 48, steps=3)
    return dataclasses.replace(c, mach=0.05, scheme="dual", ib_family="quadratic", n_inner=3,
                               dt=dual_dt([c.xf, c.yf]))


def _solver(case, precision, pipeline):
    from paper_1912_11908_amd import Solver
    s = Solver(case, precision, "cuda:0")
    s.init_prim(smooth_prim(case))
    s.L.ibm_set_option(s.h, 4, 1 if pipeline else 0)
    return s


@pytest.mark.parametrize("kind", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pipelined_classification_is_bit_identical(kind, precision):
    case = CASES[kind]()
    a, b = _solver(case, precision, True), _solver(case, precision, False)
    for s in (a, b):
        s.advance(3)          # pipelined within the call
        s.advance(1)          # a call of one step: nothing to prefetch
        s.classify()          # an explicit classification at the current time
        s.advance(2)
        t = s.info().time
        s.set_time(t)         # a time reset drops any prefetched classification
        s.advance(2)
    torch.cuda.synchronize()
    a.check_status()
    b.check_status()
    assert np.array_equal(a.interior().cpu().numpy(), b.interior().cpu().numpy())
    assert np.array_equal(a.classes(), b.classes())
    ra, rb = a.records(), b.records()
    assert np.array_equal(ra[0], rb[0]) and np.array_equal(ra[1], rb[1])


def test_nonfinite_reported_from_either_buffer():
    case = CASES["tube-moving"]()
    for nsteps in (1, 2, 3, 4):
        s = _solver(case, "mixed", True)
        idx = (0, case.nk // 4, case.nj // 4, case.ni // 4)
        s.interior()[idx] = float("nan")
        s.advance(nsteps)
        torch.cuda.synchronize()
        assert s.status() == -4, nsteps
        # the status word the serving loop reads from the current buffer
        assert s.counts()[5] & 1, nsteps
