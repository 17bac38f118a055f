"""Pins of the free rigid body (section 6, eq.10) in the oracle's driver and
of the shock-driven workload's initial states.

1. Verlet with the 1/2 of its standard form: under a constant force the
   driver must reproduce x_n = a (n dt)^2 / 2 and u_n = a n dt exactly (up to
   rounding) -- the force is replaced by a constant for this check only.
2. A body in uniform quiescent gas feels no force and stays at rest.
3. The Rankine-Hugoniot states of the workload match the paper's printed
   pressure ratio and post-shock speed (tests/golden; the printed densities
   are not self-consistent and are not used).
4. The shock over the body's front pushes it along +x with no lift (the box
   and body are mirror-symmetric about y = 2): the lift starts at rounding
   level and stays below 1e-4 of the drag over a few steps (mirrored cells'
   stencils are evaluated in different operation orders, and the shock
   amplifies those rounding differences)."""
import json
import os

import numpy as np

import oracle
import workloads as w
from workloads.cases import shock_prim, shock_states

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_verlet_closed_form_under_constant_force():
    case = w.small_case("shock-cylinder", 48, steps=6)
    o = oracle.Oracle(case)
    q = o.prim_to_state(w.freestream_prim(2, case.ni, case.nj, 1, case.p_inf, velocity=(0.0, 0.0, 0.0)))
    F = np.array([0.37, 0.0, 0.0])
    o.forces = lambda q: (F, None, 0)
    o.run_free(q, case.steps)
    a, T = F[0] / case.motion["mass"], case.steps * case.dt
    x, u, acc = o.body
    assert abs(x - 0.5 * a * T * T) <= 1e-13 * abs(0.5 * a * T * T)
    assert abs(u - a * T) <= 1e-13 * abs(a * T)
    assert acc == a


def test_body_at_rest_in_quiescent_gas():
    case = w.small_case("shock-cylinder", 48, steps=3)
    o = oracle.Oracle(case)
    q = o.prim_to_state(w.freestream_prim(2, case.ni, case.nj, 1, case.p_inf, velocity=(0.0, 0.0, 0.0)))
    o.run_free(q, case.steps)
    x, u, a = o.body
    scale = case.p_inf / case.motion["mass"]
    assert abs(a) <= 1e-12 * scale and abs(u) <= 1e-12 * scale and abs(x) <= 1e-12 * scale


def test_shock_states_match_printed_ratios():
    g = json.load(open(os.path.join(GOLDEN, "rh_shock_driven_cylinder.json")))["printed"]
    (r0, u0, p0), (r1, u1, p1) = shock_states(g["mach_shock"], g["gamma"])
    assert abs(p1 / p0 - g["p1_Pa"] / g["p0_Pa"]) <= 2e-6 * p1 / p0
    assert abs(u1 - g["u1_m_s"] / g["shock_speed_m_s"]) <= 2e-6 * u1
    assert (r0, u0) == (1.0, 0.0) and abs(p0 - 1.0 / (g["gamma"] * g["mach_shock"] ** 2)) < 1e-15


def test_shock_pushes_the_body_forward_without_lift():
    case = w.small_case("shock-cylinder", 64, steps=4)
    o = oracle.Oracle(case)
    q = o.prim_to_state(shock_prim(case, 1.2))
    o.run_free(q, case.steps)
    x, u, a = o.body
    F = o.last_force
    assert a > 0 and u > 0 and x > 0
    assert abs(F[1]) <= 1e-4 * F[0]
