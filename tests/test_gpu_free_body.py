"""GPU parity of the free rigid body (section 6, eq.10; motion 2): a
shock-driven cylinder advanced by ibm_advance against the oracle's coupled
driver on the same initial state -- body displacement, velocity and
acceleration within 1e-10 relative, flow fields within the FP64 tolerance,
classification exact at the final pose."""
import numpy as np
import pytest

import workloads as w
from workloads.cases import shock_prim
from gpu_common import make_pair, compare_fields

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,steps", [(64, 5), (96, 3)])
def test_free_body_matches_oracle(n, steps):
    case = w.small_case("shock-cylinder", n, steps=steps)
    prim = shock_prim(case, 1.2)
    s, o = make_pair(case, prim, "fp64")
    s.advance(steps)
    s.check_status()
    got = s.body_state()
    q = o.prim_to_state(prim)
    o.run_free(q, steps)
    ref = np.array(o.body)
    assert np.all(np.abs(got[:3] - ref) <= 1e-10 * np.abs(ref)), (got, ref)
    assert abs(got[3] - o.last_force[0]) <= 1e-10 * abs(o.last_force[0])
    errs = compare_fields(s.interior().cpu().numpy(), o.interior(q))
    assert errs.max() < 1e-12, errs
    assert np.array_equal(s.classes(), o.classes())


def test_free_body_mixed_precision_tracks_fp64():
    import torch
    case = w.small_case("shock-cylinder", 64, steps=5)
    prim = shock_prim(case, 1.2)
    out = []
    for prec in ("fp64", "mixed"):
        s, _ = make_pair(case, prim, prec)
        s.advance(case.steps)
        torch.cuda.synchronize()
        s.check_status()
        out.append(s.body_state())
    assert np.all(np.abs(out[1][:3] - out[0][:3]) <= 1e-4 * np.abs(out[0][:3])), out
