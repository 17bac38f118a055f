"""GPU parity of the surface force integral (section 6, eq.9; ibm_forces)
against the oracle on the same filled state: per-facet rows within 1e-11 of
each column's scale, the total within 1e-11 of the sum of the facets'
absolute contributions (the two sides add in different orders), the same
count of facets without a valid centre, and bit-identical repeated calls.
P - p_inf also carries the double oracle's fill floor: it forms a filled
node's pressure in absolute terms and then less p_inf, which leaves an
absolute error of a few ulps of p_inf (16 eps p_inf allowed; the low-Mach
case is compared with the oracle's __float128 build, where it vanishes)."""
import numpy as np
import pytest

from gpu_common import make_pair, smooth_prim
from test_gpu_parity import SMALL

pytestmark = pytest.mark.gpu

CASES = [("cylinder", "fp64", 0.0), ("cylinder-quad", "mixed", 0.0), ("wedge", "mixed", 0.0),
         ("naca", "fp64", 0.0), ("tube-moving", "fp64", 1.3), ("tube-static", "mixed", 0.0),
         ("octahedron", "fp64", 0.0)]


@pytest.mark.parametrize("kind,precision,t", CASES)
def test_forces_match_oracle(kind, precision, t):
    import torch
    case = SMALL[kind]()
    prim = smooth_prim(case)
    s, o = make_pair(case, prim, precision)
    s.set_time(t)
    s.classify()
    s.fill(t)
    F, rows, missed = s.forces(facets=True)
    F2 = s.forces()
    torch.cuda.synchronize()
    s.check_status()
    o.classify(t)
    q = o.prim_to_state(prim)
    o.fill(q, t)
    o.bc(q)
    Fo, per, mo = o.forces(q)
    F, F2, rows = F.cpu().numpy(), F2.cpu().numpy(), rows.cpu().numpy()
    assert int(missed.cpu()[0]) == mo
    assert np.array_equal(F, F2)
    floor = 16 * np.finfo(float).eps * o.param("pinf")
    for col in range(5):
        scale = max(np.abs(per[:, col]).max(), 1e-300)
        tol = 1e-11 * scale + (floor if col == 0 else 0.0)
        assert np.abs(rows[:, col] - per[:, col]).max() <= tol, col
    nd = case.ndim
    terms = per[:, 4:5] * (np.abs(per[:, 0:1]) + np.abs(per[:, 1:4]))
    bound = 1e-11 * terms.sum(axis=0) + floor * per[:, 4].sum() + 1e-300
    assert np.all(np.abs(F - Fo)[:nd] <= bound[:nd]), (F, Fo)
    assert F[2] == 0.0 or nd == 3


def test_symmetric_airfoil_has_no_lift():
    """NACA 00xx at zero incidence on a grid symmetric about its chord, in a
    uniform stream: the solution stays mirror-symmetric, so the lift is zero
    up to rounding (a property that holds at any size)."""
    import torch
    import workloads as w
    case = SMALL["naca"]()
    prim = w.freestream_prim(2, case.ni, case.nj, 1, case.p_inf)
    for precision in ("fp64", "mixed"):
        s, _ = make_pair(case, prim, precision)
        s.advance(case.steps)
        t = s.info().time
        s.fill(t)
        F = s.forces().cpu().numpy()
        torch.cuda.synchronize()
        s.check_status()
        assert F[0] > 0.0
        assert abs(F[1]) <= 1e-7 * abs(F[0]), (precision, F)
