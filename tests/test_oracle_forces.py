"""Pins of the oracle's surface force integral (section 6, eq.9) against the
divergence theorem, independent of the oracle's own sampling formulas.

Fields are set analytically on every cell (no fill).  For a closed surface,
integral of -p' n = -integral of grad p' over the body's volume, and integral of
tau n = integral of div tau over it; with p' = a x, u = (y^2, 0), u = (x^2, 0)
these are -a V, 2 mu V and (8/3) mu V along x (the last one needs the
-2/3 div u term of tau).  The one-point-per-facet quadrature is exact for
these linear integrands, so the only error is the inverse-distance sampling,
which is first order in h: the tests require the error to shrink by the
expected factor on a refined grid and to be small on the fine one.  A
constant p' and a constant-gradient shear must give zero (the facets' area
vectors sum to zero).  V comes from the polygon's shoelace area and the
octahedron's closed form."""
import numpy as np
import pytest

import oracle
import workloads as w
from workloads.cases import Case

A = 0.37


def cylinder(n, nseg=256):
    f = w.uniform_faces(n, -2.0, 2.0)
    v, s = w.circle_polygon(nseg, 1.0)
    return Case(f"cyl{n}", 2, f, f.copy(), np.array([0.0, 1.0]), ("farfield",) * 4 + ("periodic",) * 2,
                v, s, 0.3, 100.0, dt=1e-3)


def octahedron(n, r=1.1):
    v = w.snap(np.array([[r, 0, 0], [-r, 0, 0], [0, r, 0], [0, -r, 0], [0, 0, r], [0, 0, -r]], float))
    t = []
    for a, b in ((0, 2), (2, 1), (1, 3), (3, 0)):
        t.append([a, b, 4])
        t.append([b, a, 5])
    f = w.uniform_faces(n, -1.53, 1.47)
    return Case(f"oct{n}", 3, f, f.copy() + 0.011, f.copy() - 0.007, ("farfield",) * 6, v,
                np.array(t, np.int32), 0.3, 100.0, dt=1e-3)


def volume(case):
    if case.ndim == 2:
        v = case.vert
        return 0.5 * sum(v[i, 0] * v[j, 1] - v[j, 0] * v[i, 1] for i, j in case.facet)
    r = case.vert[0, 0]
    return 4.0 / 3.0 * r ** 3


def forces(case, kind):
    nd = case.ndim
    c = [0.5 * (a[1:] + a[:-1]) for a in (case.xf, case.yf, case.zf if nd == 3 else np.array([-0.5, 0.5]))]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    o = oracle.Oracle(case)
    pinf = o.param("pinf")
    prim = np.zeros((nd + 2, case.nk, case.nj, case.ni))
    prim[0] = 1.0
    prim[-1] = pinf
    along = X if nd == 2 else Z       # the field's axis: x in 2D, z in 3D
    cross = Y if nd == 2 else Z
    if kind == "pconst":
        prim[-1] = pinf + A
    elif kind == "plin":
        prim[-1] = pinf + A * along
    elif kind == "shear":             # u = (y^2, 0) / (z^2, 0, 0): constant-free shear
        prim[1] = cross ** 2
    elif kind == "uniform-shear":     # u = (y, 0) / (z, 0, 0): constant tau
        prim[1] = cross
    elif kind == "dil":               # u = (x^2, 0) / w = z^2: dilatation
        prim[1 if nd == 2 else 3] = along ** 2
    o.classify()
    q = o.prim_to_state(prim)
    F, per, missed = o.forces(q)
    assert missed == 0
    return F, per, o


def expected(case, kind, o):
    V, mu = volume(case), o.param("mu")
    ax = 0 if case.ndim == 2 else 2
    e = np.zeros(3)
    if kind == "plin":
        e[ax] = -A * V
    elif kind == "shear":
        e[0] = 2.0 * mu * V
    elif kind == "dil":
        e[ax] = 8.0 / 3.0 * mu * V
    return e


@pytest.mark.parametrize("make,n", [(cylinder, 64), (octahedron, 24)])
@pytest.mark.parametrize("kind", ["pconst", "uniform-shear"])
def test_zero_force_fields(make, n, kind):
    case = make(n)
    F, per, o = forces(case, kind)
    scale = A * per[:, 4].sum() + o.param("mu") * per[:, 4].sum()
    assert np.abs(F).max() <= 1e-13 * scale, F


@pytest.mark.parametrize("make,ns,ratio,fine_tol", [(cylinder, (64, 128), 1.7, 0.04),
                                                    (octahedron, (24, 48), 2.5, 0.03)])
@pytest.mark.parametrize("kind", ["plin", "shear", "dil"])
def test_divergence_theorem_first_order(make, ns, ratio, fine_tol, kind):
    errs = []
    for n in ns:
        case = make(n)
        F, _, o = forces(case, kind)
        e = expected(case, kind, o)
        scale = np.abs(e).max()
        errs.append(np.abs(F - e).max() / scale)
        # the other components vanish to the same order
        other = [d for d in range(case.ndim) if e[d] == 0.0]
        assert np.abs(F[other]).max() <= 0.05 * scale
    assert errs[1] < fine_tol, errs
    assert errs[0] / errs[1] > ratio, errs


def test_per_facet_rows():
    """Facet rows: the areas add up to the polygon's perimeter and the
    sampled p' of a linear field lies between its values at the corners of
    the facet's cell box (inverse-distance weights are convex)."""
    case = cylinder(64)
    F, per, o = forces(case, "plin")
    v, s = case.vert, case.facet
    perim = np.linalg.norm(v[s[:, 1]] - v[s[:, 0]], axis=1).sum()
    assert abs(per[:, 4].sum() - perim) <= 1e-12 * perim
    xm = 0.5 * (v[s[:, 0], 0] + v[s[:, 1], 0])
    h = 4.0 / 64
    assert np.all(np.abs(per[:, 0] / A - xm) <= h)
