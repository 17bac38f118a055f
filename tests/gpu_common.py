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


def make_pair(case, prim, precision="fp64"):
    from paper_1912_11908_amd import Solver
    s = Solver(case, precision, "cuda:0")
    s.init_prim(prim)
    o = oracle.Oracle(case)
    return s, o


def tol64(case):
    """FP64 parity tolerance.  1e-12 relative L2, unless the oracle's own
    rounding floor is higher: it forms fluxes in absolute variables, whose
    largest terms are p_inf and rho H_inf, so its residual carries an
    absolute error of about eps * (p_inf + H_inf) per unit dynamic pressure
    (rho_inf U_inf^2 = 1); a factor 10 covers accumulation over a step."""
    p_inf = case.p_inf
    h_inf = case.gamma / (case.gamma - 1.0) * p_inf + 0.5
    return max(1e-12, 10 * np.finfo(float).eps * (p_inf + h_inf))


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
