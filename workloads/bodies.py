"""Synthetic immersed bodies.

2D bodies are closed polygons listed counter-clockwise (interior on the left);
facets are segments (v[k], v[k+1]).  The 3D body is a triangulated open tube
whose triangles are counter-clockwise seen from outside.  All vertex
coordinates are snapped to multiples of 2**-24.
"""
import numpy as np

from .grids import snap


def _polygon(v):
    v = snap(np.asarray(v, dtype=np.float64))
    n = len(v)
    seg = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1).astype(np.int32)
    return v, seg


def circle_polygon(n=256, diameter=1.0, center=(0.0, 0.0)):
    """Regular n-gon inscribed in the circle, vertices at angles 2 pi k / n."""
    t = 2.0 * np.pi * np.arange(n) / n
    r = 0.5 * diameter
    v = np.stack([center[0] + r * np.cos(t), center[1] + r * np.sin(t)], axis=1)
    return _polygon(v)


def wedge_polygon(half_angle_deg=15.0, length=1.0, apex=(-0.5, 0.0)):
    """Triangle with its apex pointing upstream (-x) and a vertical base."""
    t = length * np.tan(np.radians(half_angle_deg))
    ax, ay = apex
    v = [[ax, ay], [ax + length, ay - t], [ax + length, ay + t]]
    return _polygon(v)


def star_polygon(n_tips=5, r_out=1.0, r_in=0.38, center=(0.0, 0.0), rot_deg=90.0):
    """Regular star: n_tips outer vertices on radius r_out alternating with
    inner vertices on r_in (a non-convex body with acute tips)."""
    k = np.arange(2 * n_tips)
    t = np.radians(rot_deg) + np.pi * k / n_tips
    r = np.where(k % 2 == 0, r_out, r_in)
    v = np.stack([center[0] + r * np.cos(t), center[1] + r * np.sin(t)], axis=1)
    return _polygon(v)


def naca00_polygon(thickness=0.12, n_vert=1024, x0=0.0, chord=1.0):
    """Symmetric NACA 4-digit section with a closed, sharp trailing edge
    (last coefficient -0.1036), cosine-spaced; n_vert unique vertices."""
    if n_vert % 2:
        raise ValueError("n_vert must be even")
    m = n_vert // 2
    k = np.arange(m + 1)
    x = 0.5 * (1.0 - np.cos(np.pi * k / m))
    yt = 5.0 * thickness * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x ** 2
                            + 0.2843 * x ** 3 - 0.1036 * x ** 4)
    yt[0] = 0.0
    yt[-1] = 0.0
    upper = [[x[i], yt[i]] for i in range(m, 0, -1)]    # TE, upper ... (x>0)
    lower = [[x[i], -yt[i]] for i in range(0, m)]       # LE, lower ...
    v = np.array(upper + lower, dtype=np.float64)
    v[:, 0] = x0 + chord * v[:, 0]
    v[:, 1] = chord * v[:, 1]
    return _polygon(v)


def tube_mesh(radius=0.5, n_theta=512, n_z=64, z_lo=-2.0, z_hi=2.0,
              center=(0.0, 0.0)):
    """Open circular tube along z (no caps): (n_z+1)*n_theta vertices and
    2*n_theta*n_z triangles with outward orientation."""
    t = 2.0 * np.pi * np.arange(n_theta) / n_theta
    z = z_lo + (z_hi - z_lo) * np.arange(n_z + 1) / n_z
    zz, tt = np.meshgrid(z, t, indexing="ij")
    v = np.stack([center[0] + radius * np.cos(tt), center[1] + radius * np.sin(tt), zz],
                 axis=-1).reshape(-1, 3)
    v = snap(v)

    def vid(a, b):
        return b * n_theta + (a % n_theta)

    tri = []
    for b in range(n_z):
        for a in range(n_theta):
            p00, p10 = vid(a, b), vid(a + 1, b)
            p11, p01 = vid(a + 1, b + 1), vid(a, b + 1)
            tri.append((p00, p10, p11))
            tri.append((p00, p11, p01))
    return v, np.asarray(tri, dtype=np.int32)


def sphere_mesh(n_theta=30, n_phi=21, diameter=1.0, center=(0.0, 0.0, 0.0)):
    """Closed UV sphere: n_phi - 1 latitude rings of n_theta vertices plus
    the two poles, 2 n_theta (n_phi - 1) triangles (1200 for 30 x 21),
    counter-clockwise seen from outside."""
    r = 0.5 * diameter
    phis = np.pi * np.arange(1, n_phi) / n_phi            # interior latitudes
    t = 2.0 * np.pi * np.arange(n_theta) / n_theta
    verts = [(center[0], center[1], center[2] + r)]          # north pole
    for ph in phis:
        for a in t:
            verts.append((center[0] + r * np.sin(ph) * np.cos(a), center[1] + r * np.sin(ph) * np.sin(a),
                          center[2] + r * np.cos(ph)))
    verts.append((center[0], center[1], center[2] - r))      # south pole
    v = snap(np.asarray(verts))
    south = len(verts) - 1

    def ring(k, a):
        return 1 + k * n_theta + (a % n_theta)

    tri = []
    for a in range(n_theta):
        tri.append((0, ring(0, a), ring(0, a + 1)))
    for k in range(n_phi - 2):
        for a in range(n_theta):
            p00, p01 = ring(k, a), ring(k, a + 1)
            p10, p11 = ring(k + 1, a), ring(k + 1, a + 1)
            tri.append((p00, p10, p11))
            tri.append((p00, p11, p01))
    for a in range(n_theta):
        tri.append((south, ring(n_phi - 2, a + 1), ring(n_phi - 2, a)))
    return v, np.asarray(tri, dtype=np.int32)
