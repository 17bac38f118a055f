"""Pins for the oracle's 3D geometry: ray-parity classification against
exact inside tests of simple solids, closest points against an independent
brute force, and the pseudo-normal sign theorem on a closed mesh."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from oracle import exact
import workloads as w
from workloads.cases import Case


def _case3d(vert, tri, n=(20, 20, 12), lo=(-1.5, -1.5, -1.0), hi=(1.5, 1.5, 1.0), bcz="farfield"):
    xf = w.uniform_faces(n[0], lo[0], hi[0])
    yf = w.uniform_faces(n[1], lo[1], hi[1])
    zf = w.uniform_faces(n[2], lo[2], hi[2])
    bc = ("farfield",) * 4 + (bcz, bcz)
    return Case("solid3d", 3, xf, yf, zf, bc, np.asarray(vert, float), np.asarray(tri, np.int32),
                0.3, 100.0, dt=1e-3)


def _box(lo, hi):
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = [[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
         [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]]
    # outward counter-clockwise triangles
    t = [[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7], [0, 1, 5], [0, 5, 4],
         [1, 2, 6], [1, 6, 5], [2, 3, 7], [2, 7, 6], [3, 0, 4], [3, 4, 7]]
    return w.snap(np.array(v)), np.array(t, np.int32)


def _octahedron(r):
    v = [[r, 0, 0], [-r, 0, 0], [0, r, 0], [0, -r, 0], [0, 0, r], [0, 0, -r]]
    t = []
    for a, b in ((0, 2), (2, 1), (1, 3), (3, 0)):
        t.append([a, b, 4])
        t.append([b, a, 5])
    return w.snap(np.array(v, float)), np.array(t, np.int32)


def _centres(c):
    return [0.5 * (f[:-1] + f[1:]) for f in (c.xf, c.yf, c.zf)]


def test_box_classification_exact_including_shared_diagonals():
    """Axis-aligned box whose faces' shared diagonals pass through cell
    centres: inside iff strictly within the bounds (top-left rule counts a
    ray through a shared edge exactly once)."""
    c0 = _case3d(np.zeros((1, 3)), np.zeros((0, 3)), n=(16, 16, 16), lo=(-1, -1, -1), hi=(1, 1, 1))
    xc, yc, zc = _centres(c0)
    lo = (xc[3] - 0.0625 / 2, yc[3], zc[3])
    hi = (xc[12] + 0.0625 / 2, yc[12], zc[12])
    v, t = _box(lo, hi)
    c = _case3d(v, t, n=(16, 16, 16), lo=(-1, -1, -1), hi=(1, 1, 1))
    o = oracle.Oracle(c)
    o.classify()
    inside = o.classes() >= oracle.G1
    X, Y, Z = np.meshgrid(xc, yc, zc, indexing="ij")
    exp = (X > v[:, 0].min()) & (X < v[:, 0].max()) & (Y > v[:, 1].min()) & (Y < v[:, 1].max()) & \
          (Z > v[:, 2].min()) & (Z < v[:, 2].max())
    on_yz_boundary = (np.isin(Y, [v[:, 1].min(), v[:, 1].max()]) | np.isin(Z, [v[:, 2].min(), v[:, 2].max()]))
    exp = exp.transpose(2, 1, 0)
    mask = ~on_yz_boundary.transpose(2, 1, 0)
    assert np.array_equal(inside[mask], exp[mask])
    assert inside.sum() > 100


def test_octahedron_classification_exact():
    v, t = _octahedron(1.1)
    c = _case3d(v, t, n=(18, 18, 18), lo=(-1.4, -1.4, -1.4), hi=(1.4, 1.4, 1.4))
    o = oracle.Oracle(c)
    o.classify()
    inside = o.classes() >= oracle.G1
    xc, yc, zc = _centres(c)
    R = Fr(float(v[0, 0]))
    for k in range(c.nk):
        for j in range(c.nj):
            for i in range(c.ni):
                s = abs(Fr(float(xc[i]))) + abs(Fr(float(yc[j]))) + abs(Fr(float(zc[k])))
                if s == R:
                    continue
                assert bool(inside[k, j, i]) == (s < R), (i, j, k)


@pytest.mark.parametrize("disp", [0.0, 0.13])
def test_tube_classification_matches_cross_section_polygon(disp):
    """An open tube spanning the periodic z range classifies exactly like its
    polygonal cross-section (exact rational winding number) at every z."""
    v, t = w.tube_mesh(0.5, 32, 4, -0.5, 0.5)
    xf = w.uniform_faces(24, -1.0, 1.0)
    zf = w.uniform_faces(6, -0.5, 0.5)
    motion = dict(axis=1, amplitude=0.2, frequency=0.25, phase=0.0)
    c = Case("tube", 3, xf, xf.copy(), zf, ("farfield",) * 4 + ("periodic",) * 2, v, t, 0.2, 185.0,
             dt=1e-3, motion=motion)
    o = oracle.Oracle(c)
    # t chosen so that the displacement is 0.2 cos(2 pi 0.25 t) = disp
    tt = np.arccos(disp / 0.2) / (2 * np.pi * 0.25)
    o.classify(tt)
    inside = o.classes() >= oracle.G1
    dy = o.param("disp")
    ring = v[:32, :2]
    poly = [(exact.fr(x), exact.fr(y) + exact.fr(dy)) for x, y in ring]
    xc = 0.5 * (xf[:-1] + xf[1:])
    for j in range(24):
        for i in range(24):
            p = (exact.fr(xc[i]), exact.fr(xc[j]))
            if exact.on_boundary(poly, p):
                continue
            exp = exact.winding_number(poly, p) != 0
            assert np.all(inside[:, j, i] == exp), (i, j)


def _closest_bruteforce(p, v, t):
    """Independent closest point: project onto each triangle's plane, keep it
    if its barycentrics are inside, else take the best point on the three
    edges; minimum over triangles."""
    best = np.inf
    for tri in t:
        a, b, c = v[tri[0]], v[tri[1]], v[tri[2]]
        n = np.cross(b - a, c - a)
        n = n / np.linalg.norm(n)
        q = p - np.dot(p - a, n) * n
        # barycentric by areas
        def area(u, w_, x):
            return np.dot(np.cross(w_ - u, x - u), n)
        A = area(a, b, c)
        l0, l1, l2 = area(q, b, c) / A, area(a, q, c) / A, area(a, b, q) / A
        if min(l0, l1, l2) >= 0:
            d2 = float(np.dot(p - q, p - q))
        else:
            d2 = np.inf
            for u, x in ((a, b), (b, c), (c, a)):
                e = x - u
                s = np.clip(np.dot(p - u, e) / np.dot(e, e), 0, 1)
                r = p - (u + s * e)
                d2 = min(d2, float(np.dot(r, r)))
        best = min(best, d2)
    return best


def test_closest_points_3d_against_bruteforce_and_sign_theorem():
    """Closest distance (eq.1) matches an independent projection brute force;
    for the closed octahedron the sign of (X - C) . n_feature (facet, edge or
    vertex pseudo-normal of the closest feature) agrees with ray parity."""
    v, t = _octahedron(1.1)
    # an asymmetric grid so that some nodes fall in edge regions
    c = _case3d(v, t, n=(23, 21, 19), lo=(-1.37, -1.41, -1.33), hi=(1.45, 1.39, 1.42))
    o = oracle.Oracle(c)
    o.classify()
    ir, dr = o.records()
    nF = o.lists()[2][0]
    xc, yc, zc = _centres(c)
    kinds = set()
    for r in range(len(ir)):
        cell = ir[r, 0]
        i, j, k = cell % c.ni, (cell // c.ni) % c.nj, cell // (c.ni * c.nj)
        X = np.array([xc[i], yc[j], zc[k]])
        d2 = _closest_bruteforce(X, v, t)
        assert abs(dr[r, 25] - np.sqrt(d2)) < 1e-12
        kinds.add(int(ir[r, 1]))
        # P' lies on the surface: |x|+|y|+|z| = R
        P = dr[r, 3:6]
        assert abs(np.abs(P).sum() - v[0, 0]) < 1e-12
    assert kinds >= {0, 2}          # faces and edges both occur
    assert o.stats()["fallback_none"] == 0
    # sign theorem on the closest point recomputed from P' when the feature
    # is a face, and from the record normal otherwise
    for r in range(len(ir)):
        cell = ir[r, 0]
        i, j, k = cell % c.ni, (cell // c.ni) % c.nj, cell // (c.ni * c.nj)
        X = np.array([xc[i], yc[j], zc[k]])
        n = dr[r, 0:3]
        s = float(np.dot(X - dr[r, 3:6], n))
        if abs(s) < 1e-12:
            continue
        assert (s > 0) == (r < nF), r


def test_probe_stencils_wrap_across_periodic_axis():
    """A body spanning a periodic axis (the tube) has valid probe stencils at
    every node; nodes in the last layer take their enclosing pair across the
    periodic boundary (cells n-1 and 0) rather than falling back."""
    c = w.small_case("tube", 30, steps=1, nz=10, ntheta=48, nzt=5, moving=False)
    o = oracle.Oracle(c)
    o.classify()
    st = o.stats()
    assert st["fallback_probe"] == 0 and st["fallback_none"] == 0
    ir, dr = o.records()
    top = [r for r in range(len(ir)) if ir[r, 0] // (c.ni * c.nj) == c.nk - 1]
    assert top
    straddle = 0
    for r in top:
        ks = {int(cid) // (c.ni * c.nj) for cid in ir[r, 7:15] if cid >= 0}
        assert ks in ({c.nk - 2, c.nk - 1}, {c.nk - 1, 0}), ks
        straddle += ks == {c.nk - 1, 0}
        assert abs(dr[r, 9:17].sum() - 1.0) < 1e-14
    assert straddle > 0
