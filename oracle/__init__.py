"""CPU oracle: plain FP64 implementation of the immersed-boundary step.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  The product path
(the HIP library and its binding) never imports, links or calls it.

The arithmetic lives in ``oracle.c`` (built by :func:`build`); this module only
marshals numpy arrays through ctypes.  ``exact.py`` holds exact-rational
brute-force checks used as pins.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None
# builds of the flow half in a wider scalar type (same arithmetic, loops and
# order): long double and __float128, for parity at low Mach, where the
# double oracle's absolute-variable rounding (about eps * p_inf per unit
# dynamic pressure) is above the tolerance of the FP64 GPU path
WIDE = {"long": ("liboracle_ld.so", 1, []), "quad": ("liboracle_q.so", 2, ["-lquadmath"])}
_wide = {}

BC = {"farfield": 0, "extrap": 1, "periodic": 2}
FLUID, FORCING, G1, G2, G3, SOLID = range(6)
IREC, DREC = 24, 32


CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-D_GNU_SOURCE",
          "-fPIC", "-shared", "-Wall", "-Wno-unused-function"]


def build(openmp=True):
    """Compile oracle.c (gcc, -O2, no FP contraction, no fast-math): the
    double oracle, and its flow half in long double and in __float128."""
    for so, kind, libs in [("liboracle.so", 0, [])] + list(WIDE.values()):
        path = os.path.join(_HERE, so)
        cmd = ["gcc"] + CFLAGS + [f"-DORC_REAL_KIND={kind}"]
        if openmp:
            cmd.append("-fopenmp")
        cmd += ["-o", path + ".tmp", os.path.join(_HERE, "oracle.c"), "-lm"] + libs
        subprocess.check_call(cmd)
        os.replace(path + ".tmp", path)


def lib(precision="double"):
    """The oracle library: precision "double" (the oracle), or "long" /
    "quad" for the builds whose flow half computes in long double /
    __float128."""
    global _lib
    if precision != "double":
        if precision not in _wide:
            path = os.path.join(_HERE, WIDE[precision][0])
            if not os.path.exists(path):
                build()
            _wide[precision] = _bind(ctypes.CDLL(path))
        return _wide[precision]
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = _bind(ctypes.CDLL(_SO))
    return _lib


def _bind(L):
    if True:
        P = ctypes.c_void_p
        d, i = ctypes.c_double, ctypes.c_int
        L.orc_create.restype = P
        L.orc_create.argtypes = [i, i, i, i, P, P, P, P, i, i, P, P, d, d, d, d, i, i, d, d, i, i, P, P, i, i, i]
        L.orc_destroy.argtypes = [P]
        L.orc_set_pose.argtypes = [P, d]
        L.orc_set_body.argtypes = [P, d, d, d]
        L.orc_classify.argtypes = [P]
        L.orc_geometry.argtypes = [P]
        L.orc_bc.argtypes = [P, P]
        L.orc_fill.argtypes = [P, P, d]
        L.orc_residual.argtypes = [P, P, P]
        L.orc_rk3_step.argtypes = [P, P, P, P, d]
        L.orc_dual_step.argtypes = [P, P, P, P, P, i, d]
        L.orc_dual_begin.argtypes = [P, P, P, P, i, d]
        L.orc_dual_iterate.argtypes = [P, P, P, P, P, i, d, i]
        L.orc_prim_to_state.argtypes = [P, P, P]
        L.orc_state_to_prim.argtypes = [P, P, P]
        L.orc_forces.argtypes = [P, P, P, P]
        L.orc_forces.restype = i
        L.orc_get_class.argtypes = [P, P]
        L.orc_get_lists.argtypes = [P, P, P, P]
        L.orc_get_lists.restype = i
        L.orc_get_records.argtypes = [P, i, P, P]
        L.orc_get_stats.argtypes = [P, P]
        L.orc_get_param.argtypes = [P, i]
        L.orc_get_param.restype = d
        L.orc_weno5.argtypes = [d] * 5
        L.orc_weno5.restype = d
        L.orc_tvd2.argtypes = [d] * 3
        L.orc_tvd2.restype = d
        L.orc_ldfss.argtypes = [i, P, P, P, d, i, d, P]
        L.orc_set_threads.argtypes = [i]
        L.orc_set_threads.restype = None
        L.orc_get_threads.restype = i
        L.orc_real_bytes.restype = ctypes.c_size_t
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n):
    """OpenMP threads of the oracle's cell loops (timing only)."""
    lib().orc_set_threads(int(n))


def threads():
    return int(lib().orc_get_threads())


def compiler():
    """gcc version line and the flags the oracle is built with."""
    try:
        ver = subprocess.run(["gcc", "--version"], capture_output=True, text=True).stdout.splitlines()[0]
    except (OSError, IndexError):
        ver = "gcc (version unavailable)"
    return {"compiler": ver, "flags": " ".join(CFLAGS + ["-fopenmp"])}


def weno5(a, b, c, d, e):
    return lib().orc_weno5(a, b, c, d, e)


def tvd2(a, b, c):
    return lib().orc_tvd2(a, b, c)


def ldfss(ndim, wl, wr, nrm, gamma=1.4, precond=False, uc2=1.0):
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    n = np.ascontiguousarray(nrm, dtype=np.float64)
    f = np.zeros(ndim + 2)
    lib().orc_ldfss(ndim, _p(wl), _p(wr), _p(n), gamma, int(bool(precond)), uc2, _p(f))
    return f


class Oracle:
    """One solve on the CPU.  State arrays use the halo layout
    [nv][nk + 2 hz][nj + 6][ni + 6]; see ``new_state``."""

    def __init__(self, case, precision="double"):
        """precision: "double" (the oracle), or "long" / "quad" for its flow
        half in long double / __float128 (states stay double)."""
        self.L = lib(precision)
        self.precision = precision
        self.case = case
        c = case
        self.ndim, self.ni, self.nj, self.nk = c.ndim, c.ni, c.nj, c.nk
        self.nv = c.ndim + 2
        self.hz = 3 if c.ndim == 3 else 0
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        xf, yf = arr(c.xf, np.float64), arr(c.yf, np.float64)
        zf = arr(c.zf if c.ndim == 3 else [0.0, 1.0], np.float64)
        bc = arr([BC[b] for b in c.bc], np.int32)
        vert = arr(c.vert.reshape(-1) if len(c.vert) else np.zeros(1), np.float64)
        facet = arr(c.facet.reshape(-1) if len(c.facet) else np.zeros(1, np.int32), np.int32)
        mo = c.motion or {}
        mpar = arr([mo.get("axis", 0), mo.get("mass", 0.0) if mo.get("free") else mo.get("amplitude", 0.0),
                    mo.get("frequency", 0.0), mo.get("phase", 0.0), mo.get("velocity", 0.0)], np.float64)
        # free body (section 6): displacement, velocity, acceleration along the axis
        self.body = [0.0, float(mo.get("velocity", 0.0)), 0.0]
        uinf = arr(list(c.u_inf) + [0.0] * (3 - len(c.u_inf)), np.float64)
        self.h = self.L.orc_create(
            c.ndim, c.ni, c.nj, c.nk, _p(xf), _p(yf), _p(zf), _p(bc), len(c.vert), len(c.facet),
            _p(vert), _p(facet), c.mach, c.reynolds, c.prandtl, c.gamma,
            0 if c.scheme == "rk3" else 1, 0 if c.ib_family == "linear" else 1, c.dt,
            c.cfl_tau, c.n_inner, (2 if mo.get("free") else 1) if mo else 0, _p(mpar), _p(uinf),
            {"eq6": 0, "eq7": 1}[c.wall_pressure], {"weno5": 0, "tvd2": 1}[c.reconstruction],
            {"rtln": 0, "sdsn": 1}[c.ib_framework])
        self.t = 0.0
        self.step_index = 0

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None

    @property
    def state_shape(self):
        return (self.nv, self.nk + 2 * self.hz, self.nj + 6, self.ni + 6)

    def new_state(self):
        return np.zeros(self.state_shape)

    def interior(self, q):
        h = self.hz
        return q[:, h:h + self.nk, 3:3 + self.nj, 3:3 + self.ni]

    def param(self, which):
        return self.L.orc_get_param(self.h, {"pinf": 0, "R": 1, "cp": 2, "mu": 3, "k": 4,
                                            "uc2": 5, "disp": 6}[which])

    def prim_to_state(self, prim):
        prim = np.ascontiguousarray(prim, dtype=np.float64)
        q = self.new_state()
        self.L.orc_prim_to_state(self.h, _p(prim), _p(q))
        return q

    def dual_begin(self, q):
        """Start a physical dual-time step (history rotation); returns the
        'first step' flag to pass to dual_iterate."""
        c = self.case
        self._history()
        first = 1 if self.step_index == 0 else 0
        self.t += c.dt
        self.L.orc_dual_begin(self.h, _p(q), _p(self._qn), _p(self._qnm1), first, self.t)
        self.step_index += 1
        return first

    def dual_iterate(self, q, first, n_iter):
        wt = q.copy()
        self.L.orc_dual_iterate(self.h, _p(q), _p(wt), _p(self._qn), _p(self._qnm1), first,
                               self.t, n_iter)
        return q

    def _history(self):
        """Dual-time history Q^n, Q^{n-1} (conserved, interior layout), in the
        flow half's scalar type: opaque buffers of orc_real_bytes() per value."""
        if not hasattr(self, "_qn"):
            n = self.nv * self.ni * self.nj * self.nk * int(self.L.orc_real_bytes())
            self._qn = np.zeros(n, dtype=np.uint8)
            self._qnm1 = np.zeros(n, dtype=np.uint8)

    def state_to_prim(self, q):
        prim = np.zeros((self.nv, self.nk, self.nj, self.ni))
        self.L.orc_state_to_prim(self.h, _p(q), _p(prim))
        return prim

    def set_pose(self, t):
        self.L.orc_set_pose(self.h, t)

    def classify(self, t=0.0):
        self.set_pose(t)
        self.L.orc_classify(self.h)
        self.L.orc_geometry(self.h)

    def classes(self):
        out = np.zeros((self.nk, self.nj, self.ni), dtype=np.uint8)
        self.L.orc_get_class(self.h, _p(out))
        return out

    def lists(self):
        counts = np.zeros(5, dtype=np.int32)
        n = (self.ni * self.nj * self.nk) + 1
        lf = np.zeros(n, dtype=np.int32)
        lg = np.zeros(n, dtype=np.int32)
        self.L.orc_get_lists(self.h, _p(lf), _p(lg), _p(counts))
        return lf[:counts[0]].copy(), lg[:counts[4]].copy(), counts

    def records(self):
        _, _, counts = self.lists()
        nrec = int(counts[0] + counts[4])
        ir = np.zeros((max(nrec, 1), IREC), dtype=np.int32)
        dr = np.zeros((max(nrec, 1), DREC))
        self.L.orc_get_records(self.h, 0, _p(ir), _p(dr))
        return ir[:nrec], dr[:nrec]

    def stats(self):
        s = np.zeros(6, dtype=np.int64)
        self.L.orc_get_stats(self.h, _p(s))
        return dict(zip(["fallback_pprime", "fallback_probe", "fallback_none",
                         "stencil_violation", "fresh_cleared", "fresh_violation"], s.tolist()))

    def bc(self, q):
        self.L.orc_bc(self.h, _p(q))

    def fill(self, q, t=0.0):
        self.L.orc_fill(self.h, _p(q), t)

    def residual(self, q):
        r = np.zeros((self.nv, self.nk, self.nj, self.ni))
        self.L.orc_residual(self.h, _p(q), _p(r))
        return r

    def run(self, q, nsteps):
        """Advance nsteps RK3 steps or physical dual-time steps in place."""
        c = self.case
        if c.scheme == "rk3":
            q1, q2 = q.copy(), q.copy()
            for _ in range(nsteps):
                self.L.orc_rk3_step(self.h, _p(q), _p(q1), _p(q2), self.t)
                self.t += c.dt
                self.step_index += 1
        else:
            self._history()
            wt = q.copy()
            for _ in range(nsteps):
                self.t += c.dt
                self.L.orc_dual_step(self.h, _p(q), _p(wt), _p(self._qn), _p(self._qnm1),
                                    1 if self.step_index == 0 else 0, self.t)
                self.step_index += 1
        return q

    def forces(self, q):
        """Section 6, eq.9 on a filled state q: (F[3], per-facet rows
        [p - p_inf, (tau n)_x, (tau n)_y, (tau n)_z, area], facets missed)."""
        F = np.zeros(3)
        per = np.zeros((max(len(self.case.facet), 1), 5))
        missed = self.L.orc_forces(self.h, _p(q), _p(F), _p(per))
        return F, per[:len(self.case.facet)], missed

    def run_free(self, q, nsteps):
        """Section 6, eq.10: a free rigid body translating along the motion
        axis, RK3.  Per step: the body posed at x^n; the force F^n on the
        state at t^n, filled with the body's velocity u^n and its last
        acceleration; a^n = F^n / M; one RK3 step with the body at x^n
        moving at u^n and accelerating at a^n; then (Verlet, with the 1/2 of
        the standard form) x^{n+1} = x^n + u^n dt + dt^2 a^n / 2,
        u^{n+1} = u^n + dt a^n."""
        c = self.case
        ax, mass, dt = c.motion["axis"], c.motion["mass"], c.dt
        q1, q2 = q.copy(), q.copy()
        for _ in range(nsteps):
            x, u, a_prev = self.body
            self.L.orc_set_body(self.h, x, u, a_prev)
            self.classify(self.t)
            self.fill(q, self.t)
            self.bc(q)
            F, _, _ = self.forces(q)
            a = F[ax] / mass
            self.L.orc_set_body(self.h, x, u, a)
            self.L.orc_rk3_step(self.h, _p(q), _p(q1), _p(q2), self.t)
            self.t += dt
            self.step_index += 1
            self.body = [x + u * dt + 0.5 * dt * dt * a, u + dt * a, a]
            self.last_force = F
        return q
