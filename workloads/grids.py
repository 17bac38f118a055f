"""Rectilinear grid face coordinates (per axis), snapped to a dyadic lattice.

Face coordinates are multiples of 2**-(LATTICE_BITS-1), so cell centres
(face midpoints) are exact multiples of 2**-LATTICE_BITS.
"""
import numpy as np

LATTICE_BITS = 24


def snap(x, bits=LATTICE_BITS):
    """Round to the nearest multiple of 2**-bits (ties to even)."""
    s = float(2 ** bits)
    return np.rint(np.asarray(x, dtype=np.float64) * s) / s


def _faces(x):
    f = snap(x, LATTICE_BITS - 1)
    if np.any(np.diff(f) <= 0):
        raise ValueError("face coordinates must be strictly increasing")
    return f


def uniform_faces(n, lo, hi):
    """n cells of equal width on [lo, hi]."""
    return _faces(lo + (hi - lo) * np.arange(n + 1) / n)


def _tanh_half(m, length, delta):
    # m cells on [0, length], finest at 0: y = L (1 - tanh(d (1 - s)) / tanh d)
    s = np.arange(m + 1) / m
    return length * (1.0 - np.tanh(delta * (1.0 - s)) / np.tanh(delta))


def tanh_center_faces(n, lo, hi, ratio=1.02):
    """n (even) cells on [lo, hi], mirror-symmetric about the midpoint and
    clustered toward it with tanh stretching; the largest ratio of adjacent
    cell widths equals ``ratio`` (found by bisection on the stretching
    parameter)."""
    if n % 2:
        raise ValueError("n must be even")
    m, half = n // 2, 0.5 * (hi - lo)

    def max_ratio(d):
        y = _tanh_half(m, half, d)
        h = np.diff(y)
        return float(np.max(h[1:] / h[:-1]))

    a, b = 1e-6, 20.0
    for _ in range(200):
        c = 0.5 * (a + b)
        if max_ratio(c) > ratio:
            b = c
        else:
            a = c
    y = _tanh_half(m, half, a)
    mid = 0.5 * (lo + hi)
    full = np.concatenate([mid - y[::-1], mid + y[1:]])
    return _faces(full)


def _geometric_side(h, n, length):
    """n cells growing geometrically from width h*r so that they span length."""
    def span(r):
        return h * np.sum(r ** np.arange(1, n + 1))
    a, b = 1.0, 2.0
    if span(a) > length:
        raise ValueError("core spacing too coarse for the side length")
    for _ in range(200):
        c = 0.5 * (a + b)
        if span(c) > length:
            b = c
        else:
            a = c
    w = h * a ** np.arange(1, n + 1)
    w *= length / np.sum(w)
    return np.concatenate([[0.0], np.cumsum(w)])


def core_stretched_faces(n, lo, hi, core_lo, core_hi, h):
    """Uniform core [core_lo, core_hi] of width-h cells, then geometric
    stretching outward to [lo, hi]; the cells outside the core are split
    evenly between the two sides."""
    nc = int(round((core_hi - core_lo) / h))
    rest = n - nc
    if rest < 2 or rest % 2:
        raise ValueError("bad cell split")
    nl = nr = rest // 2
    core = core_lo + h * np.arange(nc + 1)
    left = core_lo - _geometric_side(h, nl, core_lo - lo)[::-1]
    right = core_hi + _geometric_side(h, nr, hi - core_hi)
    full = np.concatenate([left[:-1], core, right[1:]])
    full[0], full[-1] = lo, hi
    return _faces(full)
