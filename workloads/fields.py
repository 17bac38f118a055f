"""Seeded primitive initial fields on the interior cells of a rectilinear grid.

Every field is returned as an array of shape (ndim + 2, nk, nj, ni) holding
the primitive variables (rho, u, v[, w], p); the caller supplies the reference
pressure.  Cell centres are the midpoints of the given face coordinates.
"""
import numpy as np


def _centres(f):
    f = np.asarray(f, dtype=np.float64)
    return 0.5 * (f[:-1] + f[1:])


def freestream_prim(ndim, ni, nj, nk, p_ref, velocity=(1.0, 0.0, 0.0), rho=1.0):
    nv = ndim + 2
    out = np.empty((nv, nk, nj, ni))
    out[0] = rho
    for d in range(ndim):
        out[1 + d] = velocity[d]
    out[nv - 1] = p_ref
    return out


def random_periodic_prim(ndim, xf, yf, zf, p_ref, seed=0, modes=3, amp=0.05,
                         u_amp=0.3, p_amp=None, u_base=(1.0, 0.0, 0.0)):
    """Smooth periodic random field: a few Fourier modes per variable with
    seeded amplitudes and phases (numpy PCG64).  The box must be periodic in
    every direction for the field to be smooth across the boundaries.
    Relative amplitudes: amp for density, p_amp (default amp) for pressure,
    u_amp absolute for velocity (about u_base)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = [_centres(xf), _centres(yf)] + ([_centres(zf)] if ndim == 3 else [np.zeros(1)])
    lens = [xf[-1] - xf[0], yf[-1] - yf[0], (zf[-1] - zf[0]) if ndim == 3 else 1.0]
    z, y, x = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    coords = [x, y, z]

    def smooth():
        f = np.zeros_like(x)
        for _ in range(modes):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi, size=3)
            a = rng.uniform(-1, 1)
            term = np.ones_like(x)
            for d in range(ndim):
                term = term * np.cos(2 * np.pi * k[d] * coords[d] / lens[d] + ph[d])
            f += a * term
        return f / modes

    nv = ndim + 2
    out = np.empty((nv,) + x.shape)
    out[0] = 1.0 + amp * smooth()
    for d in range(ndim):
        out[1 + d] = u_base[d] + u_amp * smooth()
    out[nv - 1] = p_ref * (1.0 + (amp if p_amp is None else p_amp) * smooth())
    return out


def entropy_wave_prim(ndim, xf, ny, nz, p_ref, amp=0.2, u=1.0):
    """rho = 1 + amp sin(2 pi x) as exact cell averages over [xf[i], xf[i+1]],
    constant velocity (u, 0, 0) and pressure; x-periodic on [0, 1]."""
    xf = np.asarray(xf, dtype=np.float64)
    dx = np.diff(xf)
    avg = 1.0 + amp * (np.cos(2 * np.pi * xf[:-1]) - np.cos(2 * np.pi * xf[1:])) / (2 * np.pi * dx)
    ni = len(dx)
    nv = ndim + 2
    out = np.empty((nv, nz, ny, ni))
    out[0] = avg[None, None, :]
    out[1] = u
    for d in range(1, ndim):
        out[1 + d] = 0.0
    out[nv - 1] = p_ref
    return out
