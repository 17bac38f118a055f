"""GPU: the two timing calls of the C ABI leave the solve untouched.

ibm_time_update_kernel reads the state and the dual-time history and writes
scratch buffers only, so a solve advanced after it is bit-identical to one
that never called it; the stage timer (IBM_OPT_STAGE_TIMING) counts every
stage launch of ibm_advance and changes nothing but the launch path (eager
instead of graph replay, bit-identical)."""
import numpy as np
import pytest
import torch

import workloads as w
from gpu_common import smooth_prim

pytestmark = pytest.mark.gpu


def _solver(case, precision="fp64"):
    from paper_1912_11908_amd import Solver
    s = Solver(case, precision, "cuda:0")
    s.init_prim(smooth_prim(case))
    return s


def _tube_dual():
    import dataclasses
    from workloads.cases import dual_dt
    c = w.small_case("tube", 24, steps=3, nz=8, ntheta=48, nzt=4)
    return dataclasses.replace(c, mach=0.05, scheme="dual", ib_family="quadratic", n_inner=3,
                               dt=dual_dt([c.xf, c.yf, c.zf]))


@pytest.mark.parametrize("kind,stage", [("naca", 0), ("cylinder", 2), ("moving-cylinder", 3),
                                        ("tube-moving", 1), ("tube-static", 3), ("tube-dual", 0)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_kernel_timing_leaves_the_solve_unchanged(kind, stage, precision):
    make = {"naca": lambda: w.small_case("naca", 48, steps=3, n_inner=3),
            "cylinder": lambda: w.small_case("cylinder", 64, steps=3),
            "moving-cylinder": lambda: w.small_case("moving-cylinder", 64, steps=3),
            "tube-moving": lambda: w.small_case("tube", 32, steps=3, nz=8, ntheta=64, nzt=4),
            "tube-static": lambda: w.small_case("tube", 30, steps=3, nz=10, ntheta=48, nzt=5, moving=False),
            "tube-dual": _tube_dual}[kind]
    case = make()
    a, b = _solver(case, precision), _solver(case, precision)
    a.advance(1)
    b.advance(1)
    before = a.state.clone()
    ms = a.time_update_kernel(stage, 3)
    assert ms > 0.0
    assert bool((a.state == before).all())   # the input is only read
    a.advance(2)
    b.advance(2)
    torch.cuda.synchronize()
    a.check_status()
    b.check_status()
    assert np.array_equal(a.interior().cpu().numpy(), b.interior().cpu().numpy())


def test_kernel_timing_dual_needs_a_step():
    from paper_1912_11908_amd._lib import IbmError
    case = w.small_case("naca", 48, steps=1, n_inner=3)
    s = _solver(case)
    s.classify()
    with pytest.raises(IbmError):
        s.time_update_kernel(0, 1)


@pytest.mark.parametrize("kind,precision", [("cylinder", "mixed"), ("naca", "mixed"), ("tube-moving", "mixed"),
                                            ("wedge", "mixed"), ("tube-moving", "fp64"), ("tube-static", "fp64"),
                                            ("tube-dual", "fp64")])
def test_stage_timer_counts_launches_and_changes_nothing(kind, precision):
    """One timing per stage (3D FP64 with a body: from the start of its fill
    launches to the end of the stage kernel)."""
    make = {"naca": lambda: w.small_case("naca", 48, steps=3, n_inner=3),
            "cylinder": lambda: w.small_case("cylinder", 64, steps=3),
            "wedge": lambda: w.small_case("wedge", 48, steps=3),
            "tube-moving": lambda: w.small_case("tube", 32, steps=3, nz=8, ntheta=64, nzt=4),
            "tube-static": lambda: w.small_case("tube", 30, steps=3, nz=10, ntheta=48, nzt=5, moving=False),
            "tube-dual": _tube_dual}[kind]
    case = make()
    a, b = _solver(case, precision), _solver(case, precision)
    nsteps = 10 if case.scheme == "rk3" else 3
    per = case.evals_per_step
    a.set_stage_timing(1000)
    a.advance(nsteps)
    b.advance(nsteps)
    tot, n, lo, hi = a.stage_timing()
    assert n == nsteps * per, (n, nsteps, per)
    assert 0.0 < lo <= hi and tot >= n * lo * 0.999
    # counting starts again; a pool smaller than the launches times the first ones
    a.set_stage_timing(2)
    a.advance(1)
    b.advance(1)
    tot2, n2, _, _ = a.stage_timing()
    assert n2 == 2
    a.set_stage_timing(0)
    a.advance(1)
    b.advance(1)
    assert a.stage_timing()[1] == 0
    torch.cuda.synchronize()
    a.check_status()
    assert np.array_equal(a.interior().cpu().numpy(), b.interior().cpu().numpy())
