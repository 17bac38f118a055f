"""Case descriptions: grid, body, flow conditions and numerics parameters.

The four fixed workloads mirror the paper's case shapes (circular cylinder,
supersonic wedge, low-Mach NACA section, transversely oscillating cylinder)
and ``small_case`` builds scaled-down versions for parity tests.  Time steps
are fixed per case and computed here once, so every implementation advances
with the same step.
"""
from dataclasses import dataclass, field
import numpy as np

from .grids import uniform_faces, tanh_center_faces, core_stretched_faces
from .bodies import circle_polygon, wedge_polygon, naca00_polygon, star_polygon, tube_mesh, sphere_mesh

BC_NAMES = ("farfield", "extrap", "periodic")


@dataclass
class Case:
    name: str
    ndim: int
    xf: np.ndarray
    yf: np.ndarray
    zf: np.ndarray
    bc: tuple                      # (x-, x+, y-, y+, z-, z+), names from BC_NAMES
    vert: np.ndarray               # (nvert, ndim) float64
    facet: np.ndarray              # (nfacet, ndim) int32
    mach: float
    reynolds: float
    prandtl: float = 0.72
    gamma: float = 1.4
    scheme: str = "rk3"            # "rk3" | "dual"
    ib_family: str = "linear"      # "linear" (IDW + image point) | "quadratic"
    dt: float = 0.0
    cfl_tau: float = 0.5
    n_inner: int = 20
    # {} or {axis, amplitude, frequency, phase[, velocity]}:
    # x_axis(t) = amplitude cos(2 pi frequency t + phase) + velocity t
    motion: dict = field(default_factory=dict)
    steps: int = 1                 # RK3 steps, or physical steps for dual time
    # free-stream velocity (unit speed, or zero for a body moving through still fluid)
    u_inf: tuple = (1.0, 0.0, 0.0)
    wall_pressure: str = "eq6"     # "eq6" | "eq7" (supersonic moving body, 2D)
    reconstruction: str = "weno5"  # "weno5" | "tvd2" (section 2)
    # "rtln": ray tracing + local normals (the paper's framework); "sdsn":
    # signed distance + surface normals (the standard HCIB/GC, 2D)
    ib_framework: str = "rtln"

    @property
    def ni(self):
        return len(self.xf) - 1

    @property
    def nj(self):
        return len(self.yf) - 1

    @property
    def nk(self):
        return len(self.zf) - 1 if self.ndim == 3 else 1

    @property
    def ncells(self):
        return self.ni * self.nj * self.nk

    @property
    def evals_per_step(self):
        return 3 if self.scheme == "rk3" else self.n_inner

    @property
    def p_inf(self):
        return 1.0 / (self.gamma * self.mach ** 2)


def _hmin(axes):
    return [float(np.min(np.diff(a))) for a in axes]


def rk3_dt(mach, reynolds, axes, cfl=None, prandtl=0.72, gamma=1.4):
    """Explicit step: CFL / sum_d (|U_inf,d| + a_inf) / h_min,d (U_inf = 1
    along x, a_inf = 1 / M), capped by the explicit diffusion limit
    0.5 / (4 nu_max sum_d 1 / h_min,d^2) with the thermal diffusivity
    nu_max = (gamma / Pr) mu / rho_floor; rho_floor = 0.1 for supersonic free
    streams (deep expansions behind bases), 0.5 otherwise."""
    if cfl is None:
        cfl = 0.4 if mach > 1.0 else 0.5
    h = _hmin(axes)
    a = 1.0 / mach
    s = sum(((1.0 if d == 0 else 0.0) + a) / h[d] for d in range(len(h)))
    rho_floor = 0.1 if mach > 1.0 else 0.5
    nu = gamma / prandtl / reynolds / rho_floor
    dt_visc = 0.5 / (4.0 * nu * sum(1.0 / hd ** 2 for hd in h))
    return min(cfl / s, dt_visc)


def dual_dt(axes):
    """Physical step of dual time stepping: h_min / U_inf (unit CFL on U_inf)."""
    return min(_hmin(axes))


def _z_dummy():
    return np.array([-0.5, 0.5])


def case_c1(steps=200):
    f = uniform_faces(128, -8.0, 8.0)
    v, s = circle_polygon(256, 1.0)
    return Case("C1-cylinder-M0.3", 2, f, f.copy(), _z_dummy(), ("farfield",) * 4 + ("periodic",) * 2,
                v, s, 0.3, 40.0, dt=rk3_dt(0.3, 40.0, [f, f]), steps=steps)


def case_c2(steps=2000):
    xf = uniform_faces(1024, -1.0, 3.0)
    yf = tanh_center_faces(512, -2.0, 2.0, 1.02)
    v, s = wedge_polygon(15.0, 1.0, (-0.5, 0.0))
    bc = ("farfield", "extrap", "extrap", "extrap", "periodic", "periodic")
    return Case("C2-wedge-M2", 2, xf, yf, _z_dummy(), bc, v, s, 2.0, 1.0e4,
                dt=rk3_dt(2.0, 1.0e4, [xf, yf]), steps=steps)


def case_c3(physical_steps=250, n_inner=20):
    h = 1.0 / 512
    xf = core_stretched_faces(2048, -20.0, 20.0, -0.5, 1.5, h)
    yf = core_stretched_faces(1024, -15.0, 15.0, -0.25, 0.25, h)
    v, s = naca00_polygon(0.12, 1024, 0.0, 1.0)
    return Case("C3-naca0012-M0.001", 2, xf, yf, _z_dummy(), ("farfield",) * 4 + ("periodic",) * 2,
                v, s, 0.001, 1000.0, scheme="dual", ib_family="quadratic",
                dt=dual_dt([xf, yf]), n_inner=n_inner, steps=physical_steps)


def case_c4(steps=1000):
    xf = uniform_faces(384, -8.0, 16.0)
    yf = uniform_faces(256, -8.0, 8.0)
    zf = uniform_faces(64, -2.0, 2.0)
    v, t = tube_mesh(0.5, 512, 64, -2.0, 2.0)
    bc = ("farfield",) * 4 + ("periodic",) * 2
    motion = dict(axis=1, amplitude=0.2, frequency=0.2, phase=0.0)
    return Case("C4-oscillating-tube-M0.2", 3, xf, yf, zf, bc, v, t, 0.2, 185.0,
                dt=rk3_dt(0.2, 185.0, [xf, yf, zf]), motion=motion, steps=steps)


def case_supersonic_cylinder(mach=1.2, moving=True, t_end=60.0, nx=5740, ny=242):
    """Section 8.2.3: a cylinder (D = 1, 256-segment polygon) at supersonic
    speed, Re_D = 300 (M and Re on the body speed), on an 80 D x 16 D box of
    nx x ny cells: x uniform (the body's whole path), y uniform at D/80 over
    the band [7, 9] and stretched outside.  moving: the body starts at
    (1.5, 8) and moves at unit speed along +x through still fluid for
    t_end (it reaches x = 61.5 at t* = 60).  Otherwise the same body is held
    at (61.5, 8) in a stream of unit speed along -x: in the body's frame the
    two problems are the same, so their steady surface pressures agree
    (Galilean invariance).  Both use the eq.7 wall pressure."""
    xf = uniform_faces(nx, 0.0, 80.0)
    yf = core_stretched_faces(ny, 0.0, 16.0, 7.0, 9.0, 1.0 / 80.0)
    x0 = 1.5 if moving else 61.5
    v, s = circle_polygon(256, 1.0, (x0, 8.0))
    re = 300.0
    dt = rk3_dt(mach, re, [xf, yf])
    steps = int(round(t_end / dt))
    dt = t_end / steps
    bc = ("farfield",) * 4 + ("periodic",) * 2
    if moving:
        return Case(f"supersonic-moving-cylinder-M{mach:g}", 2, xf, yf, _z_dummy(), bc, v, s, mach, re,
                    dt=dt, steps=steps, u_inf=(0.0, 0.0, 0.0), wall_pressure="eq7",
                    motion=dict(axis=0, amplitude=0.0, frequency=0.0, phase=0.0, velocity=1.0))
    return Case(f"supersonic-stationary-cylinder-M{mach:g}", 2, xf, yf, _z_dummy(), bc, v, s, mach, re,
                dt=dt, steps=steps, u_inf=(-1.0, 0.0, 0.0), wall_pressure="eq7")


def shock_states(mach_s=1.5, gamma=1.4):
    """Quiescent gas ahead of a planar shock of Mach mach_s and the
    Rankine-Hugoniot state behind it, in units of the gas ahead (rho0 = 1)
    and the shock speed (U_S = 1): p0 = 1 / (gamma M_s^2)."""
    m2 = mach_s * mach_s
    p0 = 1.0 / (gamma * m2)
    r1 = (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p1 = p0 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    u1 = 1.0 - 1.0 / r1
    return (1.0, 0.0, p0), (r1, u1, p1)


def shock_prim(case, x_shock, mach_s=1.5):
    """Primitive field of a planar shock at x = x_shock moving along +x into
    gas at rest (the state behind it on the left)."""
    (r0, u0, p0), (r1, u1, p1) = shock_states(mach_s, case.gamma)
    xc = 0.5 * (case.xf[1:] + case.xf[:-1])
    behind = (xc < x_shock)[None, None, :]
    prim = np.zeros((case.ndim + 2, case.nk, case.nj, case.ni))
    prim[0] = np.where(behind, r1, r0)
    prim[1] = np.where(behind, u1, u0)
    prim[case.ndim + 1] = np.where(behind, p1, p0)
    return prim


def case_shock_cylinder(n=656, t_end=2.0, density_ratio=1.0):
    """Section 8.2.6 in units of D, the gas ahead of the shock and the shock
    speed (t* = t U_S / D): a free cylinder (D = 1, 256-segment polygon,
    centre (1.5, 2)) in a 4 x 4 box of n x n cells (D / 164 at n = 656),
    driven along x by a Mach 1.5 shock; zero-gradient sides, Re = 3.5e6
    (air at the printed speeds: nearly inviscid), linear (IDW / image point)
    family.  The body's mass per unit span is density_ratio times the mass
    of the gas it displaces (pi / 4)."""
    xf = uniform_faces(n, 0.0, 4.0)
    yf = uniform_faces(n, 0.0, 4.0)
    v, s = circle_polygon(256, 1.0, (1.5, 2.0))
    m, re = 1.5, 3.5e6
    dt = rk3_dt(m, re, [xf, yf])
    steps = int(round(t_end / dt))
    dt = t_end / steps
    mass = density_ratio * np.pi / 4.0
    return Case(f"shock-driven-cylinder-{n}", 2, xf, yf, _z_dummy(), ("extrap",) * 4 + ("periodic",) * 2, v, s,
                m, re, dt=dt, steps=steps, u_inf=(0.0, 0.0, 0.0),
                motion=dict(axis=0, mass=mass, free=True, velocity=0.0))


def case_sphere_preprocessing(n=40, ib_framework="rtln"):
    """Appendix A: a sphere of 1200 triangles (D = 1, centre at the origin)
    in a cube [-1, 1]^3 of n^3 cells, for timing the IB preprocessing
    (classification, tagging, closest features, stencils) of either
    framework."""
    f = uniform_faces(n, -1.0, 1.0)
    v, t = sphere_mesh(30, 21, 1.0)
    return Case(f"sphere-preprocessing-{n}", 3, f, f.copy(), f.copy(), ("farfield",) * 6, v, t, 0.3, 100.0,
                dt=rk3_dt(0.3, 100.0, [f, f, f]), ib_framework=ib_framework)


def small_case(kind, n=64, steps=2, **kw):
    """Scaled-down parity cases: kind in cylinder | wedge | naca | tube |
    moving-cylinder | box (no body, periodic)."""
    if kind == "cylinder":
        f = uniform_faces(n, -4.0, 4.0)
        v, s = circle_polygon(kw.get("nseg", 64), 1.0)
        m = kw.get("mach", 0.3)
        return Case(f"small-cylinder-{n}", 2, f, f.copy(), _z_dummy(),
                    ("farfield",) * 4 + ("periodic",) * 2, v, s, m, 40.0,
                    dt=rk3_dt(m, 40.0, [f, f]), steps=steps,
                    ib_family=kw.get("ib_family", "linear"),
                    reconstruction=kw.get("reconstruction", "weno5"),
                    ib_framework=kw.get("ib_framework", "rtln"))
    if kind == "star":
        # a non-convex body with acute tips (the signed-distance failure case)
        f = uniform_faces(n, -1.5, 1.5)
        v, s = star_polygon(5, 1.0, 0.38)
        return Case(f"small-star-{n}", 2, f, f.copy(), _z_dummy(),
                    ("farfield",) * 4 + ("periodic",) * 2, v, s, 0.3, 100.0,
                    dt=rk3_dt(0.3, 100.0, [f, f]), steps=steps,
                    ib_framework=kw.get("ib_framework", "rtln"))
    if kind == "moving-cylinder":
        f = uniform_faces(n, -4.0, 4.0)
        v, s = circle_polygon(kw.get("nseg", 64), 1.0)
        motion = dict(axis=1, amplitude=0.2, frequency=0.2, phase=0.0)
        return Case(f"small-moving-cylinder-{n}", 2, f, f.copy(), _z_dummy(),
                    ("farfield",) * 4 + ("periodic",) * 2, v, s, 0.2, 185.0,
                    dt=rk3_dt(0.2, 185.0, [f, f]), motion=motion, steps=steps,
                    ib_framework=kw.get("ib_framework", "rtln"))
    if kind == "shock-cylinder":
        # section 8.2.6 in miniature: a free cylinder, the shock already over
        # its front half
        c = case_shock_cylinder(n, t_end=1.0, density_ratio=kw.get("density_ratio", 1.0))
        return Case(f"small-shock-cylinder-{n}", 2, c.xf, c.yf, c.zf, c.bc, c.vert, c.facet, c.mach,
                    c.reynolds, dt=c.dt, steps=steps, u_inf=c.u_inf, motion=c.motion)
    if kind == "supersonic-moving-cylinder":
        # section 8.2.3 in miniature: the body moves at unit speed (M, Re on
        # that speed) through still fluid
        xf = uniform_faces(2 * n, -6.0, 2.0)
        yf = uniform_faces(n, -2.0, 2.0)
        v, s = circle_polygon(kw.get("nseg", 64), 1.0)
        m = kw.get("mach", 1.2)
        motion = dict(axis=0, amplitude=0.0, frequency=0.0, phase=0.0, velocity=-1.0)
        return Case(f"small-supersonic-moving-cylinder-{2*n}x{n}", 2, xf, yf, _z_dummy(),
                    ("farfield",) * 4 + ("periodic",) * 2, v, s, m, 300.0,
                    dt=rk3_dt(m, 300.0, [xf, yf]), motion=motion, steps=steps,
                    u_inf=(0.0, 0.0, 0.0), wall_pressure=kw.get("wall_pressure", "eq6"))
    if kind == "wedge":
        xf = uniform_faces(2 * n, -1.0, 3.0)
        yf = tanh_center_faces(n, -2.0, 2.0, 1.02)
        v, s = wedge_polygon(15.0, 1.0, (-0.5, 0.0))
        bc = ("farfield", "extrap", "extrap", "extrap", "periodic", "periodic")
        return Case(f"small-wedge-{2*n}x{n}", 2, xf, yf, _z_dummy(), bc, v, s, 2.0, 1.0e4,
                    dt=rk3_dt(2.0, 1.0e4, [xf, yf]), steps=steps,
                    ib_framework=kw.get("ib_framework", "rtln"))
    if kind == "naca":
        h = kw.get("h", 1.0 / 32)
        xf = core_stretched_faces(2 * n, -4.0, 5.0, -0.5, 1.5, h)
        yf = core_stretched_faces(n, -4.0, 4.0, -0.25, 0.25, h)
        v, s = naca00_polygon(kw.get("thickness", 0.12), kw.get("nvert", 256), 0.0, 1.0)
        m = kw.get("mach", 0.001)
        return Case(f"small-naca-{2*n}x{n}", 2, xf, yf, _z_dummy(), ("farfield",) * 4 + ("periodic",) * 2,
                    v, s, m, 1000.0, scheme="dual", ib_family="quadratic",
                    dt=dual_dt([xf, yf]), n_inner=kw.get("n_inner", 4), steps=steps,
                    ib_framework=kw.get("ib_framework", "rtln"))
    if kind == "tube":
        xf = uniform_faces(n, -2.0, 4.0)
        yf = uniform_faces(n, -3.0, 3.0)
        zf = uniform_faces(kw.get("nz", 8), -0.5, 0.5)
        v, t = tube_mesh(0.5, kw.get("ntheta", 64), kw.get("nzt", 4), -0.5, 0.5)
        bc = ("farfield",) * 4 + ("periodic",) * 2
        motion = dict(axis=1, amplitude=0.2, frequency=0.2, phase=0.0) if kw.get("moving", True) else {}
        return Case(f"small-tube-{n}", 3, xf, yf, zf, bc, v, t, 0.2, 185.0,
                    dt=rk3_dt(0.2, 185.0, [xf, yf, zf]), motion=motion, steps=steps,
                    ib_framework=kw.get("ib_framework", "rtln"))
    if kind == "box":
        ndim = kw.get("ndim", 2)
        f = uniform_faces(n, 0.0, 1.0)
        zf = uniform_faces(kw.get("nz", 8), 0.0, 1.0) if ndim == 3 else _z_dummy()
        m = kw.get("mach", 0.5)
        empty_v = np.zeros((0, ndim))
        empty_f = np.zeros((0, ndim), dtype=np.int32)
        axes = [f, f] + ([zf] if ndim == 3 else [])
        return Case(f"box-{ndim}d-{n}", ndim, f, f.copy(), zf, ("periodic",) * 6,
                    empty_v, empty_f, m, kw.get("reynolds", 100.0),
                    scheme=kw.get("scheme", "rk3"),
                    dt=kw.get("dt", rk3_dt(m, kw.get("reynolds", 100.0), axes)),
                    n_inner=kw.get("n_inner", 4), steps=steps)
    raise ValueError(kind)


CASES = {"C1": case_c1, "C2": case_c2, "C3": case_c3, "C4": case_c4}
