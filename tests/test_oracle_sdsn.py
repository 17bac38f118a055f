"""Pins of the oracle's signed-distance classification and surface-normal
reconstruction (the standard HCIB/GC framework that section 7 compares the
ray-tracing / local-normal one with; 2D).  Signed distance: a node inside the
body's bounding box is solid iff (X - P0) . n_f < 0, with P0 its closest
surface point and n_f the outward normal of the closest segment (lowest id
among equals); nodes outside the box are fluid (section 7).

1. Convex bodies.  Where the closest point of an outside node is a vertex V,
   X - V lies in V's normal cone.  The sign test can only fail there, and
   only at an acute vertex (outward normals n_a . n_b < 0).  Such a cone
   opens wider than 90 degrees, so it holds an axis direction, and on a
   convex body V is then the extreme vertex along that axis.  A short case
   analysis shows that the whole cone lies beyond the bounding box.  Nodes
   inside a convex body project onto a segment interior they lie behind.
   So on the cylinder, the wedge (three acute corners) and the NACA section,
   signed distance plus the box gives exactly the ray-parity classes.  A
   flipped sign, or a normal of the wrong segment, breaks this.
2. The non-convex star (five 36-degree tips, inner vertices at 0.38 of the
   tip radius).  The tip at 306 degrees is extreme only in -y, and part of
   its normal cone points back into the box.  Take the direction
   d = (1, 0.15) from that tip, between its two segment normals.  The
   closest point is the tip, and the lower-id adjacent segment has the
   outward normal at 234 degrees, so (X - V) . n5 = d . n5 < 0.  A cell
   centred on that ray is therefore solid by signed distance and fluid by
   ray parity.  Every cell where the two differ is fluid by ray parity, lies
   in the box, and lies in the normal cone of a tip.  The classes differ on
   this body and on no convex one.  With the angle-weighted vertex normal
   the test would be exact, so a normal taken from the wrong feature fails
   here too.
3. Surface-normal records: the normal is the closest segment's unit normal
   (perpendicular to that segment); P' is the closest point, at the record's
   distance.  A node whose closest feature is a segment interior gets the
   same record in both frameworks.  On a regular n-gon the surface normal stays
   within half a vertex's turning angle (pi / n) of the local normal."""
import numpy as np
import pytest

import oracle
import workloads as w
from workloads.cases import Case, rk3_dt

SOLID_MIN = 2  # G1 and beyond are inside the body
FEAT_FACE, FEAT_VERTEX = 0, 1


def classes(case):
    o = oracle.Oracle(case)
    o.classify()
    cl = o.classes()
    return (cl[0] if case.ndim == 2 else cl), o


@pytest.mark.parametrize("kind,n", [("cylinder", 64), ("wedge", 48), ("naca", 48), ("cylinder", 61)])
def test_convex_signed_distance_equals_ray_parity(kind, n):
    rt, _ = classes(w.small_case(kind, n))
    sd, _ = classes(w.small_case(kind, n, ib_framework="sdsn"))
    assert (rt >= SOLID_MIN).sum() > 20
    np.testing.assert_array_equal(sd, rt)


def test_star_signed_distance_marks_outside_cells_solid():
    case = w.small_case("star", 64)
    rt, _ = classes(case)
    sd, _ = classes(w.small_case("star", 64, ib_framework="sdsn"))
    diff = np.argwhere((sd >= SOLID_MIN) != (rt >= SOLID_MIN))
    assert len(diff) > 0
    xc = 0.5 * (case.xf[1:] + case.xf[:-1])
    yc = 0.5 * (case.yf[1:] + case.yf[:-1])
    v = case.vert
    lo, hi = v.min(axis=0), v.max(axis=0)
    for j, i in diff:
        x = np.array([xc[i], yc[j]])
        assert rt[j, i] < SOLID_MIN <= sd[j, i]
        assert lo[0] <= x[0] <= hi[0] and lo[1] <= x[1] <= hi[1]
        # x lies in the normal cone of some tip (its closest point there)
        in_cone = [(x - v[t]) @ (v[t] - v[t - 1]) >= 0 and (x - v[t]) @ (v[(t + 1) % len(v)] - v[t]) <= 0
                   for t in range(0, len(v), 2)]
        assert any(in_cone)


def test_star_hand_point():
    v, s = w.star_polygon(5, 1.0, 0.38)
    tip = v[6]
    assert np.allclose(tip, [np.cos(np.radians(306)), np.sin(np.radians(306))], atol=1e-7)
    d = np.array([1.0, 0.15]) / np.hypot(1.0, 0.15)
    target = tip + 0.05 * d
    h = 3.0 / 64
    # faces with one cell centred (up to the face lattice) on the target
    k = np.arange(-40, 41)
    xf = w.snap(target[0] - 0.5 * h + h * k, 23)
    yf = w.snap(target[1] - 0.5 * h + h * k, 23)
    kw = dict(dt=rk3_dt(0.3, 100.0, [xf, yf]), steps=1)
    bc = ("farfield",) * 4 + ("periodic",) * 2
    rt, _ = classes(Case("star-point", 2, xf, yf, np.array([0.0, 1.0]), bc, v, s, 0.3, 100.0, **kw))
    sd, _ = classes(Case("star-point", 2, xf, yf, np.array([0.0, 1.0]), bc, v, s, 0.3, 100.0,
                         ib_framework="sdsn", **kw))
    assert rt[40, 40] < SOLID_MIN
    assert sd[40, 40] >= SOLID_MIN
    # the mirror ray along the other segment's side stays fluid in both
    n5 = np.array([np.cos(np.radians(234)), np.sin(np.radians(234))])
    assert d @ n5 < 0


def _seg_normals(case):
    a, b = case.vert[case.facet[:, 0]], case.vert[case.facet[:, 1]]
    e = b - a
    nrm = np.stack([e[:, 1], -e[:, 0]], axis=1)
    return a, b, nrm / np.hypot(*nrm.T)[:, None]


@pytest.mark.parametrize("kind,n", [("star", 64), ("wedge", 96)])
def test_surface_normal_records(kind, n):
    case = w.small_case(kind, n, ib_framework="sdsn")
    _, o = classes(case)
    ir, dr = o.records()
    a, b, nrm = _seg_normals(case)
    xc = 0.5 * (case.xf[1:] + case.xf[:-1])
    yc = 0.5 * (case.yf[1:] + case.yf[:-1])
    f = ir[:, 3]
    np.testing.assert_allclose(dr[:, :2], nrm[f], atol=1e-12)
    e = b[f] - a[f]
    P = dr[:, 3:5]
    cross = (P[:, 0] - a[f, 0]) * e[:, 1] - (P[:, 1] - a[f, 1]) * e[:, 0]
    assert np.abs(cross).max() < 1e-12
    t = ((P - a[f]) * e).sum(1) / (e * e).sum(1)
    assert t.min() >= -1e-12 and t.max() <= 1 + 1e-12
    X = np.stack([xc[ir[:, 0] % case.ni], yc[ir[:, 0] // case.ni]], axis=1)
    np.testing.assert_allclose(np.hypot(*(X - P).T), dr[:, 25], rtol=0, atol=1e-13)
    if kind == "star":
        assert (ir[:, 1] == FEAT_VERTEX).sum() > 0


@pytest.mark.parametrize("kind,n", [("cylinder", 64), ("wedge", 48), ("star", 64)])
def test_face_feature_records_agree(kind, n):
    """n, P' and the signed node distance of a node closest to a segment
    interior do not depend on the framework (the probes may, through the
    classes they land on)."""
    _, o_rt = classes(w.small_case(kind, n))
    _, o_sd = classes(w.small_case(kind, n, ib_framework="sdsn"))
    ir_rt, dr_rt = o_rt.records()
    ir_sd, dr_sd = o_sd.records()
    row_sd = {(c, r < o_sd.lists()[2][0]): r for r, c in enumerate(ir_sd[:, 0])}
    nF_rt = o_rt.lists()[2][0]
    nface = 0
    for r, c in enumerate(ir_rt[:, 0]):
        s = row_sd.get((c, r < nF_rt))
        if ir_rt[r, 1] != FEAT_FACE or s is None:
            continue
        np.testing.assert_array_equal(ir_rt[r, 1:4], ir_sd[s, 1:4])
        np.testing.assert_array_equal(dr_rt[r, :7], dr_sd[s, :7])
        nface += 1
    assert nface > 10


@pytest.mark.parametrize("n,nseg", [(160, 32), (200, 32)])
def test_surface_normal_turning_bound_on_polygon_circle(n, nseg):
    c_rt = w.small_case("cylinder", n, nseg=nseg)
    c_sd = w.small_case("cylinder", n, nseg=nseg, ib_framework="sdsn")
    _, o_rt = classes(c_rt)
    _, o_sd = classes(c_sd)
    ir_rt, dr_rt = o_rt.records()
    ir_sd, dr_sd = o_sd.records()
    np.testing.assert_array_equal(ir_rt[:, :4], ir_sd[:, :4])
    cosang = np.clip((dr_rt[:, :3] * dr_sd[:, :3]).sum(1), -1, 1)
    ang = np.arccos(cosang)
    vert = ir_rt[:, 1] == FEAT_VERTEX
    assert vert.sum() > 0
    assert ang.max() <= np.pi / nseg + 1e-6
    assert ang.max() > 0.1 * np.pi / nseg
    assert ang[~vert].max() < 1e-12


def _octahedron(framework):
    r = 1.1
    v = w.snap(np.array([[r, 0, 0], [-r, 0, 0], [0, r, 0], [0, -r, 0], [0, 0, r], [0, 0, -r]], float))
    t = []
    for a, b in ((0, 2), (2, 1), (1, 3), (3, 0)):
        t.append([a, b, 4])
        t.append([b, a, 5])
    xf = w.uniform_faces(23, -1.37, 1.45)
    yf = w.uniform_faces(21, -1.41, 1.39)
    zf = w.uniform_faces(19, -1.33, 1.42)
    return Case("octahedron", 3, xf, yf, zf, ("farfield",) * 6, v, np.array(t, np.int32), 0.3, 100.0,
                dt=rk3_dt(0.3, 100.0, [xf, yf, zf]), ib_framework=framework)


def _sphere(framework):
    return w.cases.case_sphere_preprocessing(24, framework)


def _tube(framework):
    return w.small_case("tube", 32, nz=8, ntheta=64, nzt=4, ib_framework=framework)


@pytest.mark.parametrize("make", [_sphere, _octahedron, _tube])
def test_convex_3d_signed_distance_equals_ray_parity(make):
    """3D: on the UV sphere and the open tube all dihedral angles are
    obtuse, and every vertex normal cone of the octahedron points out of
    its box, so the classes agree with ray parity exactly."""
    rt, _ = classes(make("rtln"))
    sd, o = classes(make("sdsn"))
    assert (rt >= SOLID_MIN).sum() > 20
    np.testing.assert_array_equal(sd, rt)


@pytest.mark.parametrize("make", [_sphere, _octahedron])
def test_surface_normal_records_3d(make):
    case = make("sdsn")
    _, o = classes(case)
    ir, dr = o.records()
    tri = case.vert[case.facet[ir[:, 3]]]
    nrm = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    np.testing.assert_allclose(dr[:, :3], nrm, atol=1e-12)
    P = dr[:, 3:6]
    assert np.abs(((P - tri[:, 0]) * nrm).sum(1)).max() < 1e-12
    xc = [0.5 * (f[1:] + f[:-1]) for f in (case.xf, case.yf, case.zf)]
    c = ir[:, 0]
    X = np.stack([xc[0][c % case.ni], xc[1][(c // case.ni) % case.nj], xc[2][c // (case.ni * case.nj)]], axis=1)
    np.testing.assert_allclose(np.linalg.norm(X - P, axis=1), dr[:, 25], rtol=0, atol=1e-13)
