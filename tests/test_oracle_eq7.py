"""Pins of the eq.7 wall-pressure condition in the oracle's fill (supersonic
moving bodies; read as the normal momentum balance at the wall,
dp/dn = rho u_t^2 kappa - rho a_n with n into the fluid and u_t relative to
the wall).

1. An isothermal potential vortex around a circle, u_theta = C / r, T = 1,
   p = p_inf exp(-C^2 / (2 R r^2)), is in exact radial equilibrium
   (dp/dr = rho u_theta^2 / r): eq.7 is the exact wall gradient.  Filled
   with the quadratic family from the exact field, the FORCING nodes' p
   errs at second order in h under eq.7 and at first order under eq.6
   (whose zero gradient is wrong by O(1)); eq.7 is the smaller at every
   size.  A curvature term of the wrong sign would double eq.6's error.
2. With no tangential motion relative to the wall (still fluid, body
   velocity zero at t = 0 of an oscillation, acceleration not), eq.7
   reduces to eq.6 exactly: the fills are bit-identical.
3. The polygon curvature is 1/r on a regular polygon inscribed in a circle
   of radius r (records of the faces): exact for the polygon itself, here
   within 1e-3 because the vertices sit on the 2^-24 lattice (a vertex moves
   by up to 3e-8, and the curvature divides differences of normals by
   segment lengths down to 0.007)."""
import numpy as np
import pytest

import oracle
import workloads as w
from workloads.cases import Case

C = 0.5


def vortex_case(n, wall, nseg=512):
    f = w.uniform_faces(n, -1.5, 1.5)
    v, s = w.circle_polygon(nseg, 1.0)
    return Case(f"vortex{n}", 2, f, f.copy(), np.array([0.0, 1.0]), ("farfield",) * 4 + ("periodic",) * 2,
                v, s, 0.3, 100.0, dt=1e-3, ib_family="quadratic", wall_pressure=wall)


def vortex_errors(n, wall):
    c = vortex_case(n, wall)
    o = oracle.Oracle(c)
    Rg, pinf = o.param("R"), o.param("pinf")
    xc = 0.5 * (c.xf[1:] + c.xf[:-1])
    Y, X = np.meshgrid(xc, xc, indexing="ij")
    r2 = X ** 2 + Y ** 2
    p = pinf * np.exp(-C ** 2 / (2 * Rg * r2))
    prim = np.zeros((4, 1, n, n))
    prim[0, 0] = p / Rg
    prim[1, 0] = -C * Y / r2
    prim[2, 0] = C * X / r2
    prim[3, 0] = p
    o.classify()
    q = o.prim_to_state(prim)
    o.fill(q)
    got = o.state_to_prim(q)[3, 0]
    lf, lg, _ = o.lists()
    drop = pinf - pinf * np.exp(-C ** 2 / (2 * Rg * 0.25))
    err = np.abs(got[lf // n, lf % n] - p[lf // n, lf % n]) / drop
    return err.max()


def test_vortex_equilibrium_orders():
    e6 = [vortex_errors(n, "eq6") for n in (96, 192)]
    e7 = [vortex_errors(n, "eq7") for n in (96, 192)]
    assert e6[0] / e6[1] < 2.2, e6            # first order
    assert e7[0] / e7[1] > 2.8, e7            # second order
    assert all(a < b / 5 for a, b in zip(e7, e6)), (e7, e6)


def test_eq7_reduces_to_eq6_without_tangential_motion():
    f = w.uniform_faces(64, -2.0, 2.0)
    v, s = w.circle_polygon(128, 1.0)
    out = []
    for wall in ("eq6", "eq7"):
        c = Case("osc", 2, f, f.copy(), np.array([0.0, 1.0]), ("farfield",) * 4 + ("periodic",) * 2, v, s,
                 1.2, 300.0, dt=1e-3, u_inf=(0.0, 0.0, 0.0), wall_pressure=wall,
                 motion=dict(axis=1, amplitude=0.2, frequency=0.5, phase=0.0))
        o = oracle.Oracle(c)
        prim = w.freestream_prim(2, c.ni, c.nj, 1, c.p_inf, velocity=(0.0, 0.0, 0.0))
        prim[3] *= 1.0 + 0.01 * np.cos(np.linspace(0, 3, c.ni))[None, None, :]
        o.classify(0.0)
        q = o.prim_to_state(prim)
        o.fill(q, 0.0)
        out.append(q)
    assert np.array_equal(out[0], out[1])


def test_polygon_curvature_is_inverse_radius():
    for nseg, diameter in ((64, 1.0), (256, 0.6)):
        f = w.uniform_faces(48, -1.0, 1.0)
        v, s = w.circle_polygon(nseg, diameter)
        c = Case("k", 2, f, f.copy(), np.array([0.0, 1.0]), ("farfield",) * 4 + ("periodic",) * 2, v, s,
                 0.3, 100.0, dt=1e-3, wall_pressure="eq7")
        o = oracle.Oracle(c)
        o.classify()
        ir, dr = o.records()
        faces = ir[:, 1] == 0
        assert faces.any()
        assert np.abs(dr[faces, 26] * 0.5 * diameter - 1.0).max() < 1e-3
