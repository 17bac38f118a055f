"""Shared helpers for the GPU parity tests: build the same case and seeded
initial field on the HIP path and on the CPU oracle, and compare."""
import numpy as np

import oracle
import workloads as w


def smooth_prim(case, seed=0, amp=0.03, u_amp=0.1):
    """Free stream plus a smooth seeded perturbation (non-trivial residual
    everywhere)."""
    # pressure perturbations on the dynamic-pressure scale (rho U^2 = 1, so
    # relative amplitude amp * gamma M^2), never an acoustic wave far larger
    # than the flow itself at low Mach
    p_amp = amp * min(1.0, case.gamma * case.mach ** 2)
    prim = w.random_periodic_prim(case.ndim, case.xf, case.yf, case.zf, case.p_inf, seed=seed,
                                  amp=amp, u_amp=u_amp, p_amp=p_amp, u_base=case.u_inf)
    return prim


# achieved errors of the parity tests, printed at the end of the session
ACHIEVED = []


def record(name, errs):
    """Keep a test's achieved error(s) for the end-of-session summary."""
    errs = np.atleast_1d(np.asarray(errs, dtype=float))
    ACHIEVED.append((name, float(errs.max()), errs.tolist()))


def oracle_precision(case):
    """Scalar type of the oracle's flow half for a case.  The double oracle
    forms fluxes in absolute variables, whose largest terms are p_inf and
    rho H_inf, so at low Mach its own rounding is about eps (p_inf + H_inf)
    per unit dynamic pressure (7e-9 at M = 0.001, a few 1e-13 per
    pseudo-iteration at M = 0.1): the dual-time (low-Mach) cases use its
    __float128 build, whose floor is far below the FP64 tolerance."""
    return "quad" if case.mach <= 0.01 or case.scheme == "dual" else "double"


def make_pair(case, prim, precision="fp64", oracle_prec=None):
    from paper_1912_11908_amd import Solver
    s = Solver(case, precision, "cuda:0")
    s.init_prim(prim)
    o = oracle.Oracle(case, oracle_prec or oracle_precision(case))
    return s, o


def tol64(case):
    """FP64 parity tolerance: 1e-12 relative L2 per variable (with the
    scales of compare_state), at every Mach number: the low-Mach cases are
    compared with the oracle's wide build (oracle_precision)."""
    return 1e-12


def resid_tol_abs(case, var):
    """Absolute residual floor of the oracle (units rho_inf U_inf^2 / L per
    conserved variable).  Its face fluxes are formed in absolute variables:
    the pressure difference of the mass flux's pressure diffusion carries
    eps p_inf, momentum and energy fluxes carry eps times p_inf and rho H_inf;
    the energy flux also multiplies the mass-flux error by H_inf.  Divided by
    the smallest cell width, times 10 for the handful of roundings."""
    h = min(float(np.min(np.diff(a))) for a in ([case.xf, case.yf] + ([case.zf] if case.ndim == 3 else [])))
    p_inf = case.p_inf
    h_inf = case.gamma / (case.gamma - 1.0) * p_inf + 0.5
    base = 10 * np.finfo(float).eps * (p_inf + h_inf) / h
    return base * (1.0 + h_inf) if var == case.ndim + 1 else base


def rel_l2(a, b):
    num = np.sqrt(np.sum((a - b) ** 2))
    den = np.sqrt(np.sum(b ** 2))
    return num / den if den > 0 else num


def compare_fields(got, ref, mask=None):
    """Per-variable relative L2 error over the interior (optionally masked).
    Velocity and momentum components are measured against the free-stream
    scale (|U_inf| = rho_inf |U_inf| = 1 per cell) when their own norm is
    smaller: a component that is ~0 everywhere has no scale of its own."""
    out = []
    nd = ref.shape[0] - 2
    for v in range(ref.shape[0]):
        a, b = got[v], ref[v]
        if mask is not None:
            a, b = a[mask], b[mask]
        num = np.sqrt(np.sum((a - b) ** 2))
        den = np.sqrt(np.sum(b ** 2))
        if 1 <= v <= nd:
            den = max(den, np.sqrt(b.size))   # |U_inf| = 1 per cell
        out.append(num / den if den > 0 else num)
    return np.array(out)


def conserved_from_prim(prim, gamma=1.4):
    nd = prim.shape[0] - 2
    rho = prim[0]
    u = prim[1:1 + nd]
    p = prim[nd + 1]
    out = np.empty_like(prim)
    out[0] = rho
    for d in range(nd):
        out[1 + d] = rho * u[d]
    out[nd + 1] = p / (gamma - 1) + 0.5 * rho * np.sum(u * u, axis=0)
    return out


def compare_state(got, ref, case, mask=None):
    """Per-variable relative L2 error of solver states (interior).  RK3
    states (conserved) as compare_fields.  Dual-time states (p - p_inf, u..,
    T - 1): velocities against the free-stream speed and p' against the
    dynamic pressure rho_inf U_inf^2 (both 1 per cell) when their own norm
    is smaller, T' against T_inf (1 per cell) likewise: the perturbations
    at low Mach are O(M^2) of their absolute values, and these are the
    scales on which the flow is measured."""
    if case.scheme != "dual":
        return compare_fields(got, ref, mask)
    out = []
    for v in range(ref.shape[0]):
        a, b = got[v], ref[v]
        if mask is not None:
            a, b = a[mask], b[mask]
        num = np.sqrt(np.sum((a - b) ** 2))
        den = max(np.sqrt(np.sum(b ** 2)), np.sqrt(b.size))
        out.append(num / den)
    return np.array(out)
