"""Closed-form gas dynamics for the shock pins (ideal gas): the weak root
of the theta-beta-M relation of an attached oblique shock, the
Rankine-Hugoniot jumps across it, and the shock position measured from a
pressure field.  Test helpers only; independent of both solvers."""
import math

import numpy as np


def beta_weak(mach, theta, gamma=1.4):
    """Weak-shock angle beta of a wedge of half-angle theta (radians) at Mach
    mach: tan(theta) = 2 cot(beta) (M^2 sin^2 beta - 1) / (M^2 (gamma +
    cos 2 beta) + 2), solved by bisection between the Mach angle and the
    angle of maximum deflection (64 degrees bounds it for M <= 3)."""
    def f(b):
        return math.tan(theta) - 2.0 / math.tan(b) * (mach ** 2 * math.sin(b) ** 2 - 1.0) / (
            mach ** 2 * (gamma + math.cos(2.0 * b)) + 2.0)
    lo, hi = math.asin(1.0 / mach) + 1e-12, math.radians(64.0)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(lo) * f(mid) <= 0.0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def oblique_jumps(mach, beta, gamma=1.4):
    """Density and pressure ratios across an oblique shock of angle beta and
    the speed behind it, for a unit upstream speed."""
    mn = mach * math.sin(beta)
    r21 = (gamma + 1.0) * mn ** 2 / ((gamma - 1.0) * mn ** 2 + 2.0)
    p21 = 1.0 + 2.0 * gamma / (gamma + 1.0) * (mn ** 2 - 1.0)
    v2 = math.hypot(math.cos(beta), math.sin(beta) / r21)
    return r21, p21, v2


def wedge_shock_prim(case, apex, theta, mach, beta, p_inf):
    """Primitive field (rho, u, v, p) of the exact attached solution of a
    symmetric wedge with its apex at `apex`: free stream ahead of the two
    shocks, the uniform post-shock state, flowing parallel to the surfaces,
    between them."""
    r21, p21, v2 = oblique_jumps(mach, beta)
    xc = 0.5 * (case.xf[1:] + case.xf[:-1])
    yc = 0.5 * (case.yf[1:] + case.yf[:-1])
    X, Y = np.meshgrid(xc, yc)
    d, yy = X - apex[0], Y - apex[1]
    post = (d > 0) & (np.abs(yy) < math.tan(beta) * d)
    prim = np.zeros((4, 1, case.nj, case.ni))
    prim[0, 0] = np.where(post, r21, 1.0)
    prim[1, 0] = np.where(post, v2 * math.cos(theta), 1.0)
    prim[2, 0] = np.where(post, v2 * math.sin(theta) * np.sign(yy), 0.0)
    prim[3, 0] = np.where(post, p21 * p_inf, p_inf)
    return prim


def shock_offsets(case, p_ratio, apex, theta, beta, p21, stations):
    """At each distance d from the apex (columns nearest to the stations):
    the shock's height, taken where the pressure, scanned downward from the
    free stream above, first reaches the mean of the two plateaus (linear
    interpolation between the bracketing cells), its offset from the exact
    line through the apex in cells, and the median pressure ratio between
    30 % and 70 % of the way from the wall to the shock."""
    xc = 0.5 * (case.xf[1:] + case.xf[:-1])
    yc = 0.5 * (case.yf[1:] + case.yf[:-1])
    h = float(yc[1] - yc[0])
    mid = 0.5 * (p21 + 1.0)
    out = []
    for st in stations:
        i = int(np.argmin(np.abs(xc - (apex[0] + st))))
        d = float(xc[i] - apex[0])
        col = p_ratio[:, i]
        ywall = apex[1] + math.tan(theta) * d
        top = int(np.searchsorted(yc, apex[1] + 2.0 * math.tan(beta) * d))
        top = min(top, case.nj - 1)
        k = top
        while k > 0 and col[k] < mid and yc[k] > ywall:
            k -= 1
        # crossing between k (>= mid) and k + 1 (< mid)
        ysh = yc[k] + (col[k] - mid) / (col[k] - col[k + 1]) * (yc[k + 1] - yc[k])
        sel = (yc > ywall + 0.3 * (ysh - ywall)) & (yc < ywall + 0.7 * (ysh - ywall))
        out.append({"d": d, "beta_deg": math.degrees(math.atan2(ysh - apex[1], d)),
                    "offset_cells": (ysh - apex[1] - d * math.tan(beta)) / h,
                    "p21": float(np.median(col[sel]))})
    return out
