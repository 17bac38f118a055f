"""Oblique-shock pin of the oracle: a 15 degree wedge at M = 2 (Re = 1e4,
the boundary layer resolved at h = 1/256: the no-slip immersed wall deflects
the stream only where its boundary layer is resolved, see the GPU test of
the impulsive start), started from the exact attached solution -- the
theta-beta-M shock angle beta = 45.34 degrees through the apex and the
Rankine-Hugoniot state behind it, p2/p1 = 2.195 -- holds that solution: after
200 RK3 steps (0.1 convective times, the shock travels no more than a cell)
the shock stays within one cell of the exact line and the plateau within 5 %
of the exact pressure ratio, near the apex and downstream.  A wrong sign or
scale anywhere in the inviscid flux, the wall fill or the update moves the
shock or the plateau."""
import math

import numpy as np

import oracle
import workloads as w
from workloads.cases import Case, rk3_dt
from gasdyn import beta_weak, oblique_jumps, wedge_shock_prim, shock_offsets

MACH, THETA = 2.0, math.radians(15.0)
APEX = (-0.5, 0.0)


def apex_case(h=1.0 / 256, re=1.0e4):
    """The wedge's nose in a box [-0.55, -0.25] x [-0.1, 0.28]: both surfaces
    leave through the outflow side (zero-gradient), the inflow side is the
    free stream."""
    x0, x1, y0, y1 = -0.55, -0.25, -0.1, 0.28
    xf = w.uniform_faces(int(round((x1 - x0) / h)), x0, x1)
    yf = w.uniform_faces(int(round((y1 - y0) / h)), y0, y1)
    v, s = w.wedge_polygon(15.0, 1.0, APEX)
    bc = ("farfield", "extrap", "extrap", "extrap", "periodic", "periodic")
    return Case("oblique-apex", 2, xf, yf, np.array([-0.5, 0.5]), bc, v, s, MACH, re,
                dt=rk3_dt(MACH, re, [xf, yf]), steps=200)


def test_theta_beta_mach_values():
    """The weak root is 45.34 degrees at M = 2, 15 degrees, with
    p2/p1 = 2.195 (the tabulated oblique-shock values)."""
    b = beta_weak(MACH, THETA)
    r21, p21, _ = oblique_jumps(MACH, b)
    assert math.degrees(b) == pytest_approx(45.3436, 1e-4)
    assert p21 == pytest_approx(2.1946, 1e-4)
    assert r21 == pytest_approx(1.7289, 1e-4)


def pytest_approx(v, tol):
    import pytest
    return pytest.approx(v, abs=tol)


def test_oracle_holds_the_exact_oblique_shock():
    case = apex_case()
    beta = beta_weak(MACH, THETA)
    _, p21, _ = oblique_jumps(MACH, beta)
    o = oracle.Oracle(case)
    o.classify()
    q = o.prim_to_state(wedge_shock_prim(case, APEX, THETA, MACH, beta, case.p_inf))
    o.run(q, case.steps)
    p = o.state_to_prim(q)[3, 0] / case.p_inf
    for e in shock_offsets(case, p, APEX, THETA, beta, p21, (0.1, 0.15, 0.2)):
        assert abs(e["offset_cells"]) <= 1.0, e
        assert abs(e["p21"] / p21 - 1.0) <= 0.05, e
