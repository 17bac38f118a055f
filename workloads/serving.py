"""Seeded serving request stream: independent 2D solves with Poisson arrivals.

Grid side uniform in {64, 128, 256, 512} on [-8, 8]^2; body uniform over
{256-gon cylinder, 15 degree wedge, NACA 00tt with tt ~ U[6, 18] %} (chord
centred on the origin); Mach log-uniform in [0.01, 2]; Reynolds log-uniform in
[40, 1000]; exponential inter-arrival gaps.  Solves with M < 0.1 use dual time
stepping with the quadratic IB family.  Every request costs the same number
of residual evaluations: `steps` RK3 steps (3 each), or 3 steps / n_inner
physical dual-time steps of n_inner pseudo-iterations.
"""
import numpy as np

from .grids import uniform_faces
from .bodies import circle_polygon, wedge_polygon, naca00_polygon
from .cases import Case, rk3_dt, dual_dt

SEED = 191211908


def request_stream(n=2000, rate=50.0, steps=500, seed=SEED, sides=(64, 128, 256, 512)):
    """Return a list of (arrival_time_s, Case) in arrival order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for r in range(n):
        t += rng.exponential(1.0 / rate)
        side = int(rng.choice(sides))
        body = int(rng.integers(0, 3))
        mach = float(np.exp(rng.uniform(np.log(0.01), np.log(2.0))))
        re = float(np.exp(rng.uniform(np.log(40.0), np.log(1000.0))))
        tt = float(rng.uniform(0.06, 0.18))
        f = uniform_faces(side, -8.0, 8.0)
        if body == 0:
            v, s = circle_polygon(256, 1.0)
        elif body == 1:
            v, s = wedge_polygon(15.0, 1.0, (-0.5, 0.0))
        else:
            v, s = naca00_polygon(tt, 256, -0.5, 1.0)
        bc = ["farfield"] * 4 + ["periodic"] * 2
        if mach > 1.0:
            bc[1] = "extrap"
        if mach < 0.1:
            n_inner = 20
            case = Case(f"req{r}", 2, f, f.copy(), np.array([-0.5, 0.5]), tuple(bc), v, s,
                        mach, re, scheme="dual", ib_family="quadratic", dt=dual_dt([f, f]),
                        n_inner=n_inner, steps=max(1, 3 * steps // n_inner))
        else:
            case = Case(f"req{r}", 2, f, f.copy(), np.array([-0.5, 0.5]), tuple(bc), v, s,
                        mach, re, dt=rk3_dt(mach, re, [f, f]), steps=steps)
        out.append((t, case))
    return out
