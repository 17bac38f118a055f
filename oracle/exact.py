"""Exact-rational brute-force geometry used to pin the oracle.

TEST INFRASTRUCTURE ONLY.  Everything here works on ``fractions.Fraction``
values built exactly from the (dyadic) float coordinates, so no rounding
enters any decision.
"""
from fractions import Fraction as Fr


def fr(x):
    return Fr(float(x))


def winding_number(poly, p):
    """Winding number of a closed polygon (list of (x, y) Fractions) around p,
    by signed upward/downward crossings of the horizontal line through p.
    Non-zero means inside for a simple polygon; p must not lie on an edge."""
    wn = 0
    n = len(poly)
    px, py = p
    for k in range(n):
        ax, ay = poly[k]
        bx, by = poly[(k + 1) % n]
        cross = (bx - ax) * (py - ay) - (by - ay) * (px - ax)
        if ay <= py:
            if by > py and cross > 0:
                wn += 1
        else:
            if by <= py and cross < 0:
                wn -= 1
    return wn


def on_boundary(poly, p):
    px, py = p
    n = len(poly)
    for k in range(n):
        ax, ay = poly[k]
        bx, by = poly[(k + 1) % n]
        cross = (bx - ax) * (py - ay) - (by - ay) * (px - ax)
        if cross == 0 and min(ax, bx) <= px <= max(ax, bx) and min(ay, by) <= py <= max(ay, by):
            return True
    return False


def parity_minus_x(poly, p):
    """Crossing parity of a ray cast toward -x (half-open rule in y, crossing
    strictly to the left of p)."""
    px, py = p
    cnt = 0
    n = len(poly)
    for k in range(n):
        ax, ay = poly[k]
        bx, by = poly[(k + 1) % n]
        if (ay > py) == (by > py):
            continue
        xs = ax + (py - ay) * (bx - ax) / (by - ay)
        if xs < px:
            cnt += 1
    return cnt & 1


def closest_on_segment(p, a, b):
    """Exact closest point on segment [a, b] to p: (squared distance, t)."""
    ex, ey = b[0] - a[0], b[1] - a[1]
    t = ((p[0] - a[0]) * ex + (p[1] - a[1]) * ey) / (ex * ex + ey * ey)
    t = min(max(t, Fr(0)), Fr(1))
    cx, cy = a[0] + t * ex, a[1] + t * ey
    return (p[0] - cx) ** 2 + (p[1] - cy) ** 2, t
