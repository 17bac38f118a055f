"""Pins of the oracle's second-order TVD reconstruction (section 2 names the
scheme; reading: MUSCL with the minmod limiter), independent of its formula:

1. linear data are reconstructed exactly (the limited slope is the slope);
2. no new extrema: the face value seen from b lies between b and c, and at a
   local extremum of (a, b, c) it is b itself (the slope is limited to 0);
3. face values from exact cell averages of a smooth function converge at
   second order in the mean (first order only at the isolated extrema,
   where TVD schemes clip).
4. A step is captured without overshoot, with the upwind plateau value."""
import math

import numpy as np
import pytest

import oracle


def test_linear_data_exact():
    for a0, s in [(0.0, 1.0), (3.25, -0.5), (-7.0, 2.0)]:
        assert oracle.tvd2(a0, a0 + s, a0 + 2 * s) == a0 + 1.5 * s
        assert oracle.tvd2(a0 + 2 * s, a0 + s, a0) == a0 + 0.5 * s


def test_no_new_extrema():
    rng = np.random.Generator(np.random.PCG64(7))
    for _ in range(2000):
        a, b, c = rng.normal(size=3)
        r = oracle.tvd2(a, b, c)
        assert min(b, c) <= r <= max(b, c)
        if (b - a) * (c - b) <= 0.0:
            assert r == b


def test_second_order_on_smooth_data():
    errs = []
    for n in (40, 80, 160, 320):
        h = 1.0 / n
        xf = np.arange(-2, n + 3) * h
        f = lambda x: np.exp(np.sin(2 * np.pi * x) * 0.3) - x * x  # noqa: E731
        g, gw = np.polynomial.legendre.leggauss(8)
        avg = np.array([np.sum(gw * f(0.5 * (xf[i] + xf[i + 1]) + 0.5 * h * g)) / 2 for i in range(len(xf) - 1)])
        e = [abs(oracle.tvd2(*avg[i - 1:i + 2]) - f(xf[i + 1])) for i in range(2, n + 2)]
        errs.append(np.mean(e))
    slopes = [math.log(errs[k] / errs[k + 1], 2) for k in range(len(errs) - 1)]
    assert slopes[-1] > 1.8, (errs, slopes)


@pytest.mark.parametrize("jump", [1.0, 100.0, -3.0])
def test_step_without_overshoot(jump):
    assert oracle.tvd2(0.0, 0.0, jump) == 0.0
    assert oracle.tvd2(0.0, jump, jump) == jump


# ---------------------------------------------- the solver with TVD-2 faces
def _tvd_box(ndim, n, **kw):
    from test_oracle_flow import _box
    c = _box(ndim, n, **kw)
    c.reconstruction = "tvd2"
    return c


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("scheme", ["rk3", "dual"])
def test_tvd_freestream_preservation(ndim, scheme):
    import workloads as w
    c = _tvd_box(ndim, 16, scheme=scheme, stretched=True, nz=6)
    o = oracle.Oracle(c)
    o.classify()
    q = o.prim_to_state(w.freestream_prim(ndim, c.ni, c.nj, c.nk, c.p_inf))
    o.bc(q)
    assert np.all(o.residual(q) == 0.0)


def test_tvd_conservation_periodic_box():
    import workloads as w
    c = _tvd_box(2, 32, re=50.0)
    o = oracle.Oracle(c)
    o.classify()
    prim = w.random_periodic_prim(2, c.xf, c.yf, c.zf, c.p_inf, seed=0)
    q = o.prim_to_state(prim)
    vol = np.diff(c.yf)[None, :, None] * np.diff(c.xf)[None, None, :]
    tot = lambda q: [math.fsum((o.interior(q)[v] * vol).ravel()) for v in range(4)]  # noqa: E731
    t0 = tot(q)
    o.run(q, 5)
    t1 = tot(q)
    for v in range(4):
        scale = math.fsum(np.abs(o.interior(q)[v] * vol).ravel())
        assert abs(t1[v] - t0[v]) <= 150 * np.finfo(float).eps * scale


def test_tvd_entropy_wave_order():
    """Smooth advection, rho = 1 + 0.2 sin(2 pi x): the mass residual
    converges at about second order in the mean (first order at the two
    extrema, where minmod clips), against fifth order for WENO5."""
    import workloads as w
    errs = []
    for n in (32, 64, 128, 256):
        c = _tvd_box(2, n, re=1e15)
        c.yf = w.uniform_faces(4, 0.0, 4.0 / n)
        o = oracle.Oracle(c)
        o.classify()
        q = o.prim_to_state(w.entropy_wave_prim(2, c.xf, 4, 1, c.p_inf, amp=0.2, u=1.0))
        o.bc(q)
        r = o.residual(q)
        xf = c.xf
        exact = (0.2 * np.sin(2 * np.pi * xf[1:]) - 0.2 * np.sin(2 * np.pi * xf[:-1])) / np.diff(xf)
        errs.append(np.mean(np.abs(r[0, 0, 1, :] - exact)))
    slopes = [math.log(errs[k] / errs[k + 1], 2) for k in range(len(errs) - 1)]
    assert 1.5 < slopes[-1] < 2.6, (errs, slopes)
