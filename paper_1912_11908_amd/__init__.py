"""MI355X (gfx950) implementation of the per-step residual and immersed
boundary step of the all-speed sharp-interface IB finite-volume solver of
Seshadri & De (arXiv 1912.11908).

The compute lives in libibm.so (hand-written HIP kernels behind the C ABI of
include/ibm.h).  This package only marshals arguments: torch provides device
memory and the stream; ``Solver`` wraps one context.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import IbmError, FLUID, FORCING, G1, G2, G3, SOLID, REC_INT, REC_DBL

__all__ = ["Solver", "IbmError", "FLUID", "FORCING", "G1", "G2", "G3", "SOLID",
           "case_struct", "workspace_bytes", "batch_advance", "BATCH_MAX"]

BATCH_MAX = _lib.BATCH_MAX


def _torch():
    import torch
    return torch


def case_struct(case, precision="fp64"):
    """ctypes descriptor for a workloads.Case; returns (struct, keepalive)."""
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(ctypes.c_void_p)

    c = _lib.IbmCase()
    c.ndim = case.ndim
    c.ni, c.nj = case.ni, case.nj
    c.nk = case.nk if case.ndim == 3 else 1
    c.xf = arr(case.xf, np.float64)
    c.yf = arr(case.yf, np.float64)
    c.zf = arr(case.zf, np.float64) if case.ndim == 3 else None
    for s, b in enumerate(case.bc):
        c.bc[s] = _lib.BC[b]
    c.nvert = len(case.vert)
    c.nfacet = len(case.facet)
    c.vert = arr(np.asarray(case.vert).reshape(-1), np.float64) if c.nvert else None
    c.facet = arr(np.asarray(case.facet).reshape(-1), np.int32) if c.nfacet else None
    mo = case.motion or {}
    c.motion = (2 if mo.get("free") else 1) if mo else 0
    keys = ["axis", "mass", "frequency", "phase"] if mo.get("free") else ["axis", "amplitude", "frequency", "phase"]
    for m, key in enumerate(keys):
        c.motion_par[m] = float(mo.get(key, 0.0))
    c.mach, c.reynolds, c.prandtl, c.gamma = case.mach, case.reynolds, case.prandtl, case.gamma
    c.scheme = 0 if case.scheme == "rk3" else 1
    c.ib_family = 0 if case.ib_family == "linear" else 1
    c.precision = {"fp64": 0, "mixed": 1}[precision]
    c.dt, c.cfl_tau, c.n_inner = case.dt, case.cfl_tau, case.n_inner
    u = list(getattr(case, "u_inf", (1.0, 0.0, 0.0)))
    for d in range(3):
        c.u_inf[d] = float(u[d]) if d < len(u) else 0.0
    c.motion_vel = float(mo.get("velocity", 0.0))
    c.wall_pressure = {"eq6": 0, "eq7": 1}[getattr(case, "wall_pressure", "eq6")]
    c.reconstruction = {"weno5": 0, "tvd2": 1}[getattr(case, "reconstruction", "weno5")]
    c.ib_framework = {"rtln": 0, "sdsn": 1}[getattr(case, "ib_framework", "rtln")]
    return c, keep


def workspace_bytes(case, precision="fp64"):
    L = _lib.load()
    c, keep = case_struct(case, precision)
    n = ctypes.c_size_t(0)
    _lib.check(L.ibm_workspace_bytes(ctypes.byref(c), ctypes.byref(n)), "ibm_workspace_bytes")
    return n.value


class Solver:
    """One solve on one GPU.  ``state`` is the device state array
    [nv][nk + 2 hz][nj + 6][ni + 6] (float64) in the scheme's variables."""

    def __init__(self, case, precision="fp64", device="cuda:0", stream=None):
        torch = _torch()
        self.L = _lib.load()
        self.case = case
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream
        c, self._keep = case_struct(case, precision)
        self._desc = c
        nbytes = ctypes.c_size_t(0)
        _lib.check(self.L.ibm_workspace_bytes(ctypes.byref(c), ctypes.byref(nbytes)),
                   "ibm_workspace_bytes")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.L.ibm_create(ctypes.byref(c), ctypes.c_void_p(self.workspace.data_ptr()),
                                         nbytes.value, ctypes.byref(h)), "ibm_create")
        self.h = h
        info = self.info()
        self.ndim, self.ni, self.nj, self.nk, self.nv = info.ndim, info.ni, info.nj, info.nk, info.nv
        self.hz = 3 if self.ndim == 3 else 0
        self.state = torch.zeros(self.state_shape, dtype=torch.float64, device=self.device)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                self.L.ibm_destroy(h)
            except Exception:
                pass
            self.h = None

    # -------------------------------------------------------------- helpers
    @property
    def state_shape(self):
        return (self.nv, self.nk + 2 * self.hz, self.nj + 6, self.ni + 6)

    def _s(self):
        torch = _torch()
        st = self.stream if self.stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(st.cuda_stream)

    @staticmethod
    def _p(t):
        return ctypes.c_void_p(t.data_ptr())

    def info(self):
        inf = _lib.IbmInfo()
        _lib.check(self.L.ibm_info_get(self.h, ctypes.byref(inf)), "ibm_info_get")
        return inf

    def interior(self, q=None):
        q = self.state if q is None else q
        h = self.hz
        return q[:, h:h + self.nk, 3:3 + self.nj, 3:3 + self.ni]

    # ------------------------------------------------------------------ ABI
    def set_time(self, t):
        _lib.check(self.L.ibm_set_time(self.h, float(t)), "ibm_set_time", self.h)

    def init_prim(self, prim):
        """prim: (nv, nk, nj, ni) primitive (rho, u, v[, w], p), any device."""
        torch = _torch()
        p = torch.as_tensor(prim, dtype=torch.float64).to(self.device).contiguous()
        _lib.check(self.L.ibm_init_state(self.h, self._p(p), self._p(self.state), self._s()),
                   "ibm_init_state", self.h)
        self._prim_keep = p

    def to_prim(self, q=None):
        torch = _torch()
        q = self.state if q is None else q
        out = torch.empty((self.nv, self.nk, self.nj, self.ni), dtype=torch.float64, device=self.device)
        _lib.check(self.L.ibm_state_to_prim(self.h, self._p(q), self._p(out), self._s()),
                   "ibm_state_to_prim", self.h)
        return out

    def classify(self):
        _lib.check(self.L.ibm_classify(self.h, self._s()), "ibm_classify", self.h)

    def fill(self, t=0.0, q=None):
        q = self.state if q is None else q
        _lib.check(self.L.ibm_fill(self.h, self._p(q), float(t), self._s()), "ibm_fill", self.h)

    def forces(self, q=None, facets=False):
        """Section 6, eq.9 on a filled state (call fill first): the force on
        the body as a float64 device tensor [3]; with facets, also the
        per-facet rows [P - p_inf, (tau n)_x, (tau n)_y, (tau n)_z, area] and
        the count of facets without a valid centre (device tensors)."""
        torch = _torch()
        q = self.state if q is None else q
        F = torch.zeros(3, dtype=torch.float64, device=self.device)
        rows = torch.zeros((max(self.case.facet.shape[0], 1), 5), dtype=torch.float64,
                           device=self.device) if facets else None
        missed = torch.zeros(1, dtype=torch.int32, device=self.device)
        _lib.check(self.L.ibm_forces(self.h, self._p(q), self._p(F), self._p(rows) if facets else None,
                                     self._p(missed), self._s()), "ibm_forces", self.h)
        if facets:
            return F, rows[:self.case.facet.shape[0]], missed
        return F

    def residual(self, q=None):
        torch = _torch()
        q = self.state if q is None else q
        r = torch.empty((self.nv, self.nk, self.nj, self.ni), dtype=torch.float64, device=self.device)
        _lib.check(self.L.ibm_residual(self.h, self._p(q), self._p(r), self._s()),
                   "ibm_residual", self.h)
        return r

    def advance(self, nsteps, q=None):
        q = self.state if q is None else q
        _lib.check(self.L.ibm_advance(self.h, self._p(q), int(nsteps), self._s()),
                   "ibm_advance", self.h)

    def set_graphs(self, on):
        """Replay whole steps as HIP graphs (stationary bodies; default on)."""
        _lib.check(self.L.ibm_set_option(self.h, 1, 1 if on else 0), "ibm_set_option", self.h)

    def body_state(self):
        """Free body: (displacement, velocity, acceleration, axial force) of
        the last step along the motion axis."""
        out = np.zeros(4)
        _lib.check(self.L.ibm_body_state(self.h, out.ctypes.data_as(ctypes.c_void_p)), "ibm_body_state", self.h)
        return out

    def set_corner_lists(self, on):
        """Fill the FORCING probe corners of ghost nodes per tile from lists
        built at classification (default), or per ghost node."""
        _lib.check(self.L.ibm_set_option(self.h, 2, 1 if on else 0), "ibm_set_option", self.h)

    def status(self):
        return self.L.ibm_status(self.h, self._s())

    def check_status(self):
        _lib.check(self.status(), "ibm_status", self.h)

    def counts(self):
        out = np.zeros(8, dtype=np.int32)
        _lib.check(self.L.ibm_read_counts(self.h, out.ctypes.data_as(ctypes.c_void_p), self._s()),
                   "ibm_read_counts", self.h)
        return out

    def set_pipeline(self, on):
        """Classify a prescribed-motion solve's next step on a side stream
        during the current step's stages (default), or each step before its
        stages."""
        _lib.check(self.L.ibm_set_option(self.h, 4, 1 if on else 0), "ibm_set_option", self.h)

    def set_stage_timing(self, launches):
        """Time the next `launches` stage launches of advance() with HIP
        events (0: off; steps then replay as graphs again)."""
        _lib.check(self.L.ibm_set_option(self.h, 3, int(launches)), "ibm_set_option", self.h)

    def stage_timing(self):
        """(total_ms, launches, min_ms, max_ms) of the stage launches timed
        since the last call; synchronises."""
        tot, mn, mx = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        n = ctypes.c_int()
        _lib.check(self.L.ibm_stage_timing(self.h, ctypes.byref(tot), ctypes.byref(n), ctypes.byref(mn),
                                           ctypes.byref(mx)), "ibm_stage_timing", self.h)
        return tot.value, n.value, mn.value, mx.value

    def time_update_kernel(self, stage, nrep, q=None):
        q = self.state if q is None else q
        ms = ctypes.c_float(0.0)
        _lib.check(self.L.ibm_time_update_kernel(self.h, self._p(q), int(stage), int(nrep), self._s(),
                                                 ctypes.byref(ms)), "ibm_time_update_kernel", self.h)
        return ms.value

    # --------------------------------------------- device views for tests
    def _view(self, ptr, n, dtype):
        """Copy n elements of a device array owned by the context to host."""
        torch = _torch()
        nbytes = n * np.dtype(dtype).itemsize
        out = np.empty(n, dtype=dtype)
        if n == 0:
            return out
        base = self.workspace.data_ptr()
        off = ptr - base
        if off < 0 or off + nbytes > self.workspace.numel():
            raise ValueError("pointer outside the workspace")
        torch.cuda.current_stream(self.device).synchronize()
        raw = self.workspace[off:off + nbytes].cpu().numpy()
        out[:] = np.frombuffer(raw.tobytes(), dtype=dtype)
        return out

    def classes(self):
        inf = self.info()
        return self._view(inf.cls, self.ni * self.nj * self.nk, np.uint8).reshape(self.nk, self.nj, self.ni)

    def lists(self):
        inf = self.info()
        cnt = self.counts()
        lf = self._view(inf.list_forcing, int(cnt[0]), np.int32)
        lg = self._view(inf.list_ghost, int(cnt[4]), np.int32)
        return lf, lg, cnt

    def records(self):
        inf = self.info()
        cnt = self.counts()
        n = int(cnt[0] + cnt[4])
        ir = self._view(inf.rec_int, n * REC_INT, np.int32).reshape(n, REC_INT)
        dr = self._view(inf.rec_dbl, n * REC_DBL, np.float64).reshape(n, REC_DBL)
        return ir, dr


def batch_advance(solvers, nsteps, stream=None):
    """Advance several solvers by nsteps steps each through ibm_batch_advance
    (stationary-body solves of one kind share each stage's launch).  The
    solvers must be distinct and on one device; at most BATCH_MAX."""
    solvers = list(solvers)
    if not solvers:
        return
    if len(solvers) > BATCH_MAX:
        raise ValueError(f"at most {BATCH_MAX} solvers per batch")
    torch = _torch()
    L = solvers[0].L
    n = len(solvers)
    ctxs = (ctypes.c_void_p * n)(*[s.h.value for s in solvers])
    qs = (ctypes.c_void_p * n)(*[s.state.data_ptr() for s in solvers])
    st = stream if stream is not None else torch.cuda.current_stream(solvers[0].device)
    rc = L.ibm_batch_advance(ctypes.cast(ctxs, ctypes.c_void_p), ctypes.cast(qs, ctypes.c_void_p), n,
                             int(nsteps), ctypes.c_void_p(st.cuda_stream))
    if rc != 0:
        msgs = "; ".join(L.ibm_last_error(s.h).decode(errors="replace") for s in solvers)
        raise IbmError(rc, "ibm_batch_advance", msgs)
