"""GPU: the allocation-free force entry point (ibm_forces_static) against
ibm_forces, through the C ABI.

Both run the same kernels in the same order on the same filled state, so
force, per-facet rows and the count of facets without a valid centre must be
bit-identical.  Two calls in a row share the device's scratch array: a large
body first, then a smaller one (fewer blocks of partial sums), so stale
partials of the first call must not leak into the second.  Bodies over the
stated limit are refused."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as w
from gpu_common import smooth_prim

pytestmark = pytest.mark.gpu


def _filled(case, precision="fp64"):
    from paper_1912_11908_amd import Solver
    s = Solver(case, precision, "cuda:0")
    s.init_prim(smooth_prim(case))
    s.advance(1)
    t = s.info().time
    s.set_time(t)
    s.classify()
    s.fill(t)
    torch.cuda.synchronize()
    return s


def _call(s, static, with_missed=True):
    """One force evaluation through the C ABI; returns (force, rows, missed)."""
    nf = int(s.case.facet.shape[0])
    F = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda:0")
    rows = torch.full((nf, 5), float("nan"), dtype=torch.float64, device="cuda:0")
    missed = torch.full((1,), -7, dtype=torch.int32, device="cuda:0")
    fn = s.L.ibm_forces_static if static else s.L.ibm_forces
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(s.h, ctypes.c_void_p(s.state.data_ptr()), ctypes.c_void_p(F.data_ptr()),
            ctypes.c_void_p(rows.data_ptr()), ctypes.c_void_p(missed.data_ptr()) if with_missed else None, st)
    assert rc == 0, (rc, s.L.ibm_last_error(s.h))
    torch.cuda.synchronize()
    return F.cpu().numpy(), rows.cpu().numpy(), int(missed.item())


def test_static_forces_match_workspace_forces_two_calls():
    big = w.small_case("tube", 32, steps=1, nz=8, ntheta=512, nzt=64)      # 65,536 facets
    small = w.small_case("cylinder", 64, steps=1, nseg=256)               # 256 facets
    assert big.facet.shape[0] == 65536 and small.facet.shape[0] == 256
    sb, ss = _filled(big), _filled(small)
    for s in (sb, ss):          # the large body first, then the smaller one
        ref = _call(s, static=False)
        got = _call(s, static=True)
        assert np.array_equal(got[0], ref[0]), (got[0], ref[0])
        assert np.array_equal(got[1], ref[1])
        assert got[2] == ref[2]
        assert np.all(np.isfinite(got[0])) and abs(got[0]).max() > 0.0
        # the counter kept in the scratch array (d_missed NULL) is cleared
        # by each call: a second call gives the same force
        again = _call(s, static=True, with_missed=False)
        assert np.array_equal(again[0], ref[0]) and np.array_equal(again[1], ref[1])


def test_static_forces_mixed_precision_state():
    case = w.small_case("moving-cylinder", 64, steps=1)
    s = _filled(case, "mixed")
    ref = _call(s, static=False)
    got = _call(s, static=True)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]) and got[2] == ref[2]


def test_static_forces_refuse_bodies_over_the_limit():
    from paper_1912_11908_amd import _lib
    case = w.small_case("tube", 24, steps=1, nz=6, ntheta=2048, nzt=66)
    assert case.facet.shape[0] > _lib.FORCES_STATIC_MAX_FACETS
    from paper_1912_11908_amd import Solver
    s = Solver(case, "fp64", "cuda:0")
    s.init_prim(smooth_prim(case))
    F = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    rc = s.L.ibm_forces_static(s.h, ctypes.c_void_p(s.state.data_ptr()), ctypes.c_void_p(F.data_ptr()), None,
                               None, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1
    assert b"IBM_FORCES_STATIC_MAX_FACETS" in s.L.ibm_last_error(s.h)
