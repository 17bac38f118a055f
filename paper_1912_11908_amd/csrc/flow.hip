// Flow kernels for gfx950: domain ghost layers, immersed-boundary fill, and
// the fused residual + update (WENO5, low-diffusion flux splitting with
// low-Mach preconditioning, central viscous fluxes; SSP-RK3 or
// preconditioned dual time stepping) of Seshadri & De, sections 2 and 4.4-5.
//
// The residual works on perturbation variables rho' = rho - 1,
// p' = p - p_inf, T' = T - 1 in a template precision Real (double for the
// FP64 path, float for the mixed path): the mean pressure's contribution
// cancels exactly over a closed cell, and the energy residual is split as
// R_E = H_inf R_rho + R_E' (H_inf the free-stream total enthalpy), so no
// O(p_inf) quantity is ever rounded to Real.  Conserved updates and the
// recovery of (rho', p', T') from the state are FP64.
#include <cstring>

#include <hip/hip_ext.h>

#include "common.h"

namespace ibm {
namespace {

constexpr int kBlock = 256;

inline int blocks_for(long long n, int bs) { return (int)((n + bs - 1) / bs); }

template <typename R> __device__ inline R rcp_fast(R x);
// FP64: the hardware reciprocal refined by two Newton steps (within an ulp
// or so; the arguments are densities, sound speeds and WENO weight sums,
// positive and normal)
template <> __device__ inline double rcp_fast<double>(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}
template <> __device__ inline float rcp_fast<float>(float x) { return __builtin_amdgcn_rcpf(x); }
// square root without the denormal scaling and final rounding fix-up of the
// library (the arguments are squared sound speeds and Mach numbers: zero or
// positive and normal).  FP64: the hardware reciprocal square root, one
// Goldschmidt step and one Newton correction (within an ulp or two); FP32:
// the hardware instruction (about 1 ulp)
template <typename R> __device__ inline R sqrt_fast(R x);
template <> __device__ inline double sqrt_fast<double>(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    double g = x * r, h = 0.5 * r;
    double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    g = fma(fma(-g, g, x), h, g);
    return x > 0.0 ? g : x;
}
template <> __device__ inline float sqrt_fast<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ inline long long sidx(const Grid &g, int i, int j, int k)
{
    return ((long long)(k + g.hz) * g.sy + (j + 3)) * g.sx + (i + 3);
}

// State -> primitive (FP64).  RK3: conserved; dual time: (p', u, v[, w], T').
struct PrimD {
    double rho, u[3], p, T;
};

__device__ inline PrimD load_prim(const Grid &g, const Flow &f, const double *q, long long s)
{
    PrimD w;
    int nd = g.ndim;
    w.u[0] = w.u[1] = w.u[2] = 0.0;
    if (f.scheme == IBM_RK3) {
        w.rho = q[s];
        double ke = 0.0;
        for (int d = 0; d < nd; ++d) {
            w.u[d] = q[s + (1 + d) * g.vs] / w.rho;
            ke += w.u[d] * w.u[d];
        }
        w.p = (f.gamma - 1.0) * (q[s + (nd + 1) * g.vs] - 0.5 * w.rho * ke);
        w.T = w.p / (w.rho * f.R);
    } else {
        w.p = f.pinf + q[s];
        for (int d = 0; d < nd; ++d)
            w.u[d] = q[s + (1 + d) * g.vs];
        w.T = 1.0 + q[s + (nd + 1) * g.vs];
        w.rho = w.p / (f.R * w.T);
    }
    return w;
}

__device__ inline void store_prim(const Grid &g, const Flow &f, const PrimD &w, double *q,
                                  long long s)
{
    int nd = g.ndim;
    if (f.scheme == IBM_RK3) {
        double ke = 0.0;
        for (int d = 0; d < nd; ++d)
            ke += w.u[d] * w.u[d];
        q[s] = w.rho;
        for (int d = 0; d < nd; ++d)
            q[s + (1 + d) * g.vs] = w.rho * w.u[d];
        q[s + (nd + 1) * g.vs] = w.p / (f.gamma - 1.0) + 0.5 * w.rho * ke;
    } else {
        q[s] = w.p - f.pinf;
        for (int d = 0; d < nd; ++d)
            q[s + (1 + d) * g.vs] = w.u[d];
        q[s + (nd + 1) * g.vs] = w.T - 1.0;
    }
}

// ------------------------------------------------------ domain ghosts
// Three ghost layers per side: FARFIELD = free stream, EXTRAP = nearest
// interior cell, PERIODIC = wrap; corner ghosts resolve the later axis
// first (the x, then y, then z sweep order).
struct FreeStream {
    double v[5];
};

__device__ inline void halo_cell(const Grid &g, int t, int &i, int &j, int &k)
{
    if (g.ndim == 2) {
        int band = 3 * g.sx;
        k = 0;
        if (t < 2 * band) {
            int top = t >= band;
            int r = t - top * band;
            j = r / g.sx + (top ? g.nj : -3);
            i = r % g.sx - 3;
            return;
        }
        t -= 2 * band;
        j = t / 6;
        int c = t % 6;
        i = c < 3 ? c - 3 : g.ni + (c - 3);
        return;
    }
    int plane = g.sx * g.sy;
    int zb = 3 * plane;
    if (t < 2 * zb) {
        int top = t >= zb;
        int r = t - top * zb;
        k = r / plane + (top ? g.nk : -3);
        r %= plane;
        j = r / g.sx - 3;
        i = r % g.sx - 3;
        return;
    }
    t -= 2 * zb;
    int yb = 6 * g.sx;
    if (t < yb * g.nk) {
        k = t / yb;
        int r = t % yb;
        int top = r >= 3 * g.sx;
        r -= top * 3 * g.sx;
        j = r / g.sx + (top ? g.nj : -3);
        i = r % g.sx - 3;
        return;
    }
    t -= yb * g.nk;
    k = t / (6 * g.nj);
    int r = t % (6 * g.nj);
    j = r / 6;
    int c = r % 6;
    i = c < 3 ? c - 3 : g.ni + (c - 3);
}

__device__ inline void bc_cell(const Grid &g, const FreeStream &fs, double *q, int t)
{
    int i, j, k;
    halo_cell(g, t, i, j, k);
    int c[3] = {i, j, k}, n[3] = {g.ni, g.nj, g.nk};
    bool farfield = false;
    for (int ax = g.ndim - 1; ax >= 0; --ax) {
        if (c[ax] >= 0 && c[ax] < n[ax])
            continue;
        int type = g.bc[2 * ax + (c[ax] < 0 ? 0 : 1)];
        if (type == IBM_BC_FARFIELD) {
            farfield = true;
            break;
        }
        if (type == IBM_BC_EXTRAP)
            c[ax] = c[ax] < 0 ? 0 : n[ax] - 1;
        else
            c[ax] = c[ax] < 0 ? c[ax] + n[ax] : c[ax] - n[ax];
    }
    long long dst = sidx(g, i, j, k);
    long long src = sidx(g, c[0], c[1], c[2]);
    for (int v = 0; v < g.nv; ++v)
        q[dst + v * g.vs] = farfield ? fs.v[v] : q[src + v * g.vs];
}

__global__ void bc_kernel(Grid g, FreeStream fs, double *q, int nhalo)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nhalo)
        bc_cell(g, fs, q, t);
}

// ------------------------------------------------------------ IB fill
// Boundary conditions along the local-normal line (section 4.4): velocity
// Dirichlet = body velocity (eq.4); dp/dn = -rho n . a_body (eqs 5-6);
// dT/dn = 0 (eq.8).  Linear family: linear profile through the wall value
// (Dirichlet) or slope (Neumann) and the probe; quadratic family: profile
// through two probes (sections 4.5-4.6 and 5).  s = 0 at P', s > 0 in the
// fluid; the node sits at s_X.
// (rho, u.., p, T) of state values qv (the cell's NV state variables).  For
// dual time p and T are the perturbations p - p_inf and T - 1: the fill's
// profiles are affine in p and T (the weights of a probe sum to one), so
// they run on the perturbations and no O(p_inf) value is ever rounded.
template <int DIM>
__device__ inline void prim_of_state(const Flow &f, const double *qv, double &rho, double *u, double &p,
                                     double &T)
{
    if (f.scheme == IBM_RK3) {
        rho = qv[0];
        double ri = rcp_fast<double>(rho);
        double ke = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            u[d] = qv[1 + d] * ri;
            ke += u[d] * u[d];
        }
        p = (f.gamma - 1.0) * (qv[DIM + 1] - 0.5 * rho * ke);
        T = p * ri * f.rR;
    } else {
        p = qv[0];
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            u[d] = qv[1 + d];
        T = qv[DIM + 1];
        rho = (f.pinf + p) * f.rR * rcp_fast<double>(1.0 + T);
    }
}

template <int DIM, bool NEST>
__device__ __forceinline__ void node_fill(const Grid &g, const Flow &f, const IB &ib, const double *q, int r,
                                          int c, double ub, double ab, int axis, double *qs);

// Records are filled by groups of 2^DIM consecutive lanes: lane c of the
// group takes probe corner c, so that the corners' loads are in flight
// together.  Value at probe `p` (0 or 1) of record r: the weighted sum of
// (p, u.., T) over the plan's corners (unused corners carry zero weight),
// added by butterfly shuffles, so that every lane of the group holds the
// same sums.  With NEST, a weighted corner that is a FORCING node takes its
// filled value from ib.fval (stored there by forcing_corners), not from q.
template <int DIM, bool NEST>
__device__ __forceinline__ void plan_probe(const Grid &g, const Flow &f, const IB &ib, const double *q, int r,
                                           int p, int c, double *phi)
{
    constexpr int NC = 1 << DIM;
    constexpr int NV = DIM + 2;
    int idx = (8 * p + c) * ib.cap + r;
    int off = ib.plan_off[idx];
    double w = ib.plan_w[idx];
    int fr = NEST ? ib.plan_frec[idx] : -1;
    double qv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        qv[v] = fr >= 0 ? ib.fval[(long long)v * ib.cap + fr] : q[off + v * g.vs];
    double rho, u[DIM], pr, T;
    prim_of_state<DIM>(f, qv, rho, u, pr, T);
    bool on = w != 0.0;
    phi[0] = on ? w * pr : 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d)
        phi[1 + d] = on ? w * u[d] : 0.0;
    phi[NV - 1] = on ? w * T : 0.0;
#pragma unroll
    for (int o = 1; o < NC; o <<= 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
            phi[v] += __shfl_xor(phi[v], o);
    }
}

// State value qs of IB record r (its plan and the node's boundary
// conditions) from the cells of q; NEST as for plan_probe.
template <int DIM, bool NEST>
__device__ __forceinline__ void node_fill(const Grid &g, const Flow &f, const IB &ib, const double *q, int r,
                                          int c, double ub, double ab, int axis, double *qs)
{
    constexpr int NV = DIM + 2;
    int cap = ib.cap;
    bool quad = f.family == IBM_IB_QUADRATIC;
    int mode = ib.plan_mode[r];
    int mode1 = mode & 15, mode2 = mode >> 4;
    double n[DIM], ubv[DIM], abv[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        n[d] = ib.plan_geo[d * cap + r];
        ubv[d] = d == axis ? ub : 0.0;
        abv[d] = d == axis ? ab : 0.0;
    }
    double sx = ib.plan_geo[3 * cap + r], s1 = ib.plan_geo[4 * cap + r], s2 = ib.plan_geo[5 * cap + r];
    // p and T as prim_of_state gives them: absolute (RK3) or the
    // perturbations (dual time)
    const bool pert = f.scheme != IBM_RK3;
    const double p0 = pert ? f.pinf : 0.0, T0 = pert ? 1.0 : 0.0;
    double rp, ru[DIM], rT;
    if (mode1 == 2) {  // no valid probe corner at all: counted fallback
        rp = f.pinf - p0;
        rT = 1.0 - T0;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            ru[d] = ubv[d];
    } else {
        double phi1[NV];
        plan_probe<DIM, NEST>(g, f, ib, q, r, 0, c, phi1);
        double rho1 = (p0 + phi1[0]) * f.rR * rcp_fast<double>(T0 + phi1[NV - 1]);
        double an = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            an += n[d] * abv[d];
        double gp = -rho1 * an, gT = 0.0;
        if (DIM == 2 && f.wallp == IBM_WALL_EQ7) {
            // eq.7, read as the normal momentum balance at the wall (n into
            // the fluid): dp/dn = rho u_t^2 kappa - rho a_n, u_t the
            // tangential velocity relative to the wall at probe 1
            double ut = -(phi1[1] - ubv[0]) * n[1] + (phi1[2] - ubv[1]) * n[0];
            gp = rho1 * ut * ut * ib.plan_kappa[r] - rho1 * an;
        }
        if (!quad || mode2 == 2) {
            double ratio = sx * rcp_fast<double>(s1);
#pragma unroll
            for (int d = 0; d < DIM; ++d)
                ru[d] = ubv[d] + (phi1[1 + d] - ubv[d]) * ratio;
            rp = phi1[0] + gp * (sx - s1);
            rT = phi1[NV - 1] + gT * (sx - s1);
        } else {
            double phi2[NV];
            plan_probe<DIM, NEST>(g, f, ib, q, r, 1, c, phi2);
            double L0 = (sx - s1) * (sx - s2) * rcp_fast<double>(s1 * s2);
            double L1 = sx * (sx - s2) * rcp_fast<double>(s1 * (s1 - s2));
            double L2 = sx * (sx - s1) * rcp_fast<double>(s2 * (s2 - s1));
            double rq = rcp_fast<double>(s2 * s2 - s1 * s1);
#pragma unroll
            for (int d = 0; d < DIM; ++d)
                ru[d] = ubv[d] * L0 + phi1[1 + d] * L1 + phi2[1 + d] * L2;
            double c2p = (phi2[0] - phi1[0] - gp * (s2 - s1)) * rq;
            double c0p = phi1[0] - gp * s1 - c2p * s1 * s1;
            rp = c0p + gp * sx + c2p * sx * sx;
            double c2T = (phi2[NV - 1] - phi1[NV - 1] - gT * (s2 - s1)) * rq;
            double c0T = phi1[NV - 1] - gT * s1 - c2T * s1 * s1;
            rT = c0T + gT * sx + c2T * sx * sx;
        }
    }
    if (f.scheme == IBM_RK3) {
        double rrho = rp * f.rR * rcp_fast<double>(rT);
        double ke = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            ke += ru[d] * ru[d];
        qs[0] = rrho;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            qs[1 + d] = rrho * ru[d];
        qs[DIM + 1] = rp * f.gm1inv + 0.5 * rrho * ke;
    } else {
        qs[0] = rp;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            qs[1 + d] = ru[d];
        qs[DIM + 1] = rT;
    }
}

// The FORCING corners of ghost record r: each one's filled value, from the
// FLUID cells of q, stored at ib.fval for node_fill<DIM, true>.  Called by
// the record's lane group; every lane stores every corner (the same value),
// so that each lane reads back its own store.
template <int DIM>
__device__ __forceinline__ void forcing_corners(const Grid &g, const Flow &f, const IB &ib, const double *q,
                                                int r, int c, double ub, double ab, int axis)
{
    constexpr int NC = 1 << DIM;
#pragma nounroll
    for (int k = 0; k < 2 * NC; ++k) {
        int p = k / NC, m = k % NC;
        int fr = ib.plan_frec[(8 * p + m) * ib.cap + r];
        if (fr < 0)
            continue;
        double qv[DIM + 2];
        node_fill<DIM, false>(g, f, ib, q, fr, c, ub, ab, axis, qv);
#pragma unroll
        for (int v = 0; v < DIM + 2; ++v)
            ib.fval[(long long)v * ib.cap + fr] = qv[v];
    }
}

// fill record r of q in place from the values stored in q (lane group;
// lane 0 stores)
template <int DIM>
__device__ __forceinline__ void fill_one(const Grid &g, const Flow &f, const IB &ib, double *q, int r, int c,
                                         double ub, double ab, int axis)
{
    double qs[DIM + 2];
    node_fill<DIM, false>(g, f, ib, q, r, c, ub, ab, axis, qs);
    int node = ib.plan_node[r];
    if (c == 0) {
#pragma unroll
        for (int v = 0; v < DIM + 2; ++v)
            q[node + v * g.vs] = qs[v];
    }
}

// FORCING nodes (they read interior FLUID cells only), one lane group per
// record, grid-stride.
template <int DIM>
__global__ void forcing_fill_kernel(Grid g, Flow f, IB ib, double *q, double ub, double ab, int axis)
{
    constexpr int G = 1 << DIM;
    int nF = min(ib.counts[CNT_F], ib.cap);
    int stride = gridDim.x * blockDim.x / G;
    int c = threadIdx.x % G;
    for (int r = (blockIdx.x * blockDim.x + threadIdx.x) / G; r < nF; r += stride)
        fill_one<DIM>(g, f, ib, q, r, c, ub, ab, axis);
}

// Ghost layers G1-G3 (they read FLUID and FORCING cells), one lane group
// per record, grid-stride.
template <int DIM>
__global__ void ghost_fill_kernel(Grid g, Flow f, IB ib, double *q, double ub, double ab, int axis)
{
    constexpr int G = 1 << DIM;
    int nF = min(ib.counts[CNT_F], ib.cap);
    int nG = min(ib.counts[CNT_G], ib.cap - nF);
    int stride = gridDim.x * blockDim.x / G;
    int c = threadIdx.x % G;
    for (int t = (blockIdx.x * blockDim.x + threadIdx.x) / G; t < nG; t += stride)
        fill_one<DIM>(g, f, ib, q, nF + t, c, ub, ab, axis);
}

// ------------------------------------------------ fused residual / update
template <int DIM> struct TileCfg;
template <> struct TileCfg<2> {
    static constexpr int TX = kTile2[0], TY = kTile2[1], TZ = kTile2[2], HZ = 0, NT = kThreads2;
};
template <> struct TileCfg<3> {
    static constexpr int TX = kTile3[0], TY = kTile3[1], TZ = kTile3[2], HZ = 3, NT = kThreads3;
};

enum { MODE_RESID = 0, MODE_RK3 = 1, MODE_DUAL = 2 };

struct StepArgs {
    Grid g;
    Flow f;
    const uint8_t *cls;
    int32_t *counts;
    const double *qin;   // state read by the stencils (its IB nodes are filled on the fly)
    const double *qn;    // RK3: Q^n (state layout); dual: Q'^n (interior layout)
    const double *qnm1;  // dual: Q'^{n-1} (interior layout)
    double *out;         // RK3/dual: next state; residual mode: R (interior)
    double a, b;         // RK3 stage coefficients / dual b0, b2
    int ntx, nty, ntz;
    const int32_t *tiles;  // tile ids to run (null: every tile, in order)
    int ntiles;
    IB ib;
    double ub, ab;       // body velocity / acceleration along `axis`
    int axis;
    FreeStream fs;       // conserved or perturbation free-stream state
};


// Domain ghost cell -> source cell, by the rules of the ghost-layer fill:
// EXTRAP copies the nearest interior cell, PERIODIC wraps; a cell outside
// a FARFIELD side takes the free stream (returns true).
template <int DIM> __device__ inline bool ghost_source(const Grid &g, int *c)
{
    const int n[3] = {g.ni, g.nj, g.nk};
    bool ff = false;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        if (c[ax] >= 0 && c[ax] < n[ax])
            continue;
        int type = g.bc[2 * ax + (c[ax] < 0 ? 0 : 1)];
        if (type == IBM_BC_FARFIELD)
            ff = true;
        else if (type == IBM_BC_EXTRAP)
            c[ax] = c[ax] < 0 ? 0 : n[ax] - 1;
        else {
            // periodic: the stencils reach at most three cells beyond the
            // grid, so a shift by n (repeated for grids narrower than the
            // halo) wraps without an integer division
            while (c[ax] < 0)
                c[ax] += n[ax];
            while (c[ax] >= n[ax])
                c[ax] -= n[ax];
        }
    }
    return ff;
}

// WENO5 (Jiang-Shu, eps 1e-6, linear weights 0.1, 0.6, 0.3).  For the face
// between cells v2 and v3 of the six cells v0..v5: wl from v0..v4 (left
// state), wr from v5..v1 (right state).  Written on first differences
// D_k = v_{k+1} - v_k, which the two states share (the right state's are
// the left state's mirrored and negated), as are two of the three second
// differences.  Per state, with d1..d4 its first differences and c its
// central cell:
//   4 (eps + beta_k) = 4 eps + (13/3) t_k^2 + u_k^2,
//   t = (d2 - d1, d3 - d2, d4 - d3), u = (3 d2 - d1, d2 + d3, d4 - 3 d3);
// the candidate values are c + r_k / 6 with r = (5 d2 - 2 d1, d2 + 2 d3,
// 4 d3 - d4), and the state is c + sum_k w_k r_k / 6 with
// w_k ~ gamma_k / (4 (eps + beta_k))^2, formed with a single reciprocal
// (the common factor 4 cancels in the normalised weights).
template <typename R>
__device__ inline R weno5_state(R c, R d1, R d2, R d3, R d4, R t0, R t1, R t2, R k0, R k1, R k2)
{
    // k = (13/3) t (shared with the other state of the face)
    const R e4 = R(4.0e-6);
    R u0 = R(3) * d2 - d1, u1 = d2 + d3, u2 = d4 - R(3) * d3;
    R s0 = fma(t0, k0, fma(u0, u0, e4));
    R s1 = fma(t1, k1, fma(u1, u1, e4));
    R s2 = fma(t2, k2, fma(u2, u2, e4));
    s0 *= s0;
    s1 *= s1;
    s2 *= s2;
    R a0 = s1 * s2, a1 = s0 * s2, a2 = s0 * s1;
    // gamma_k r_k / 6
    R r0 = R(0.5 / 6.0) * d2 - R(0.2 / 6.0) * d1;
    R r1 = R(0.6 / 6.0) * d2 + R(1.2 / 6.0) * d3;
    R r2 = R(1.2 / 6.0) * d3 - R(0.3 / 6.0) * d4;
    R num = a0 * r0 + a1 * r1 + a2 * r2;
    R den = R(0.1) * a0 + R(0.6) * a1 + R(0.3) * a2;
    return c + num * rcp_fast<R>(den);
}

template <typename R>
__device__ inline void weno5_pair(R v0, R v1, R v2, R v3, R v4, R v5, R &wl, R &wr)
{
    R D0 = v1 - v0, D1 = v2 - v1, D2 = v3 - v2, D3 = v4 - v3, D4 = v5 - v4;
    R T1 = D1 - D0, T2 = D2 - D1, T3 = D3 - D2, T4 = D4 - D3;
    R K1 = R(13.0 / 3.0) * T1, K2 = R(13.0 / 3.0) * T2, K3 = R(13.0 / 3.0) * T3, K4 = R(13.0 / 3.0) * T4;
    // left: d = (D0, D1, D2, D3), t = (T1, T2, T3)
    wl = weno5_state<R>(v2, D0, D1, D2, D3, T1, T2, T3, K1, K2, K3);
    // right (v5, v4, v3, v2, v1): d = (-D4, -D3, -D2, -D1), t = (T4, T3, T2)
    wr = weno5_state<R>(v3, -D4, -D3, -D2, -D1, T4, T3, T2, K4, K3, K2);
}

template <typename R> struct FlowR {
    R gamma, gm1inv, pinf, mu, kc, uc2, uinf2;
    R rR;  // 1 / R (R = p_inf)
    bool precond;
    bool tvd;  // second-order TVD faces instead of WENO5
};

// Second-order TVD face states (section 2 names the scheme, not its limiter;
// MUSCL with the minmod limiter): from cell v1 | v2 | v3 | v4 the left and
// right states at the face between v2 and v3.
template <typename R> __device__ inline R minmod(R x, R y)
{
    if (x > R(0) && y > R(0))
        return x < y ? x : y;
    if (x < R(0) && y < R(0))
        return x > y ? x : y;
    return R(0);
}

template <typename R>
__device__ inline void tvd2_pair(R v1, R v2, R v3, R v4, R &wl, R &wr)
{
    wl = v2 + R(0.5) * minmod<R>(v2 - v1, v3 - v2);
    wr = v3 + R(0.5) * minmod<R>(v3 - v4, v2 - v3);
}

__device__ inline double sgn1(double m) { return m >= 0.0 ? 1.0 : -1.0; }
__device__ inline float sgn1(float m) { return m >= 0.0f ? 1.0f : -1.0f; }

// split-pressure coefficient D of Edwards' LDFSS(0) for Mach number m on the
// left (+) or right (-) side
template <typename R>
__device__ inline R dsplit(R m, bool plus, bool &sub)
{
    R am = fabs(m);
    sub = am < R(1);
    if (!sub)
        return plus ? (m >= R(0) ? R(1) : R(0)) : (m >= R(0) ? R(0) : R(1));
    return plus ? R(0.25) * (m + R(1)) * (m + R(1)) * (R(2) - m)
                : R(0.25) * (m - R(1)) * (m - R(1)) * (R(2) + m);
}

// D+ + D- - 1 without cancellation when both sides are subsonic
template <typename R>
__device__ inline R dsum_minus1(R mL, R mR, R dp, R dm, bool subL, bool subR)
{
    if (subL && subR)
        return R(0.25) * (mL - mR) * (R(3) - (mL * mL + mL * mR + mR * mR));
    return (dp + dm) - R(1);
}

// Section 2 inviscid flux, perturbation form; w = (rho', u.., p').  Reading:
// LDFSS(0) with the Weiss-Smith preconditioned interface sound speed a~ in
// the mass flux; the pressure split of the preconditioned flux uses the
// unpreconditioned Mach numbers with its velocity-diffusion part scaled by
// a~ / a_half.  Momentum flux excludes the constant p_inf; the energy slot
// holds the H' part (total flux = H_inf * mass flux + this).
template <typename R, int NV, int d>
__device__ inline void ldfss_pert(const R *wl, const R *wr, const FlowR<R> &fp, R *fl_out)
{
    constexpr int ND = NV - 2;
    R rl = R(1) + wl[0], rr = R(1) + wr[0];
    R plp = wl[NV - 1], prp = wr[NV - 1];
    R pl = fp.pinf + plp, pr = fp.pinf + prp;
    R UL = wl[1 + d], UR = wr[1 + d];
    R ql2 = R(0), qr2 = R(0);
#pragma unroll
    for (int e = 0; e < ND; ++e) {
        ql2 += wl[1 + e] * wl[1 + e];
        qr2 += wr[1 + e] * wr[1 + e];
    }
    R al = sqrt_fast<R>(fp.gamma * pl * rcp_fast<R>(rl)), ar = sqrt_fast<R>(fp.gamma * pr * rcp_fast<R>(rr));
    R ah = R(0.5) * (al + ar);
    R at = ah, eps = R(1);
    if (fp.precond) {
        R ah2 = ah * ah;
        eps = fmin(R(1), fmax(R(0.5) * ql2 + R(0.5) * qr2, fp.uc2) * rcp_fast<R>(ah2));
        if (eps < R(1)) {
            R ub = R(0.5) * (UL + UR);
            at = R(0.5) * sqrt_fast<R>((R(1) - eps) * (R(1) - eps) * ub * ub + R(4) * eps * ah2);
        }
    }
    R rat = rcp_fast<R>(at);
    R ML = UL * rat, MR = UR * rat;
    R apl = R(0.5) * (R(1) + sgn1(ML)), amr = R(0.5) * (R(1) - sgn1(MR));
    R bl = fabs(ML) < R(1) ? R(-1) : R(0), br = fabs(MR) < R(1) ? R(-1) : R(0);
    R mpl = R(0.25) * (ML + R(1)) * (ML + R(1)), mmr = R(-0.25) * (MR - R(1)) * (MR - R(1));
    R cp = apl * (R(1) + bl) * ML - bl * mpl;
    R cm = amr * (R(1) + br) * MR - br * mmr;
    R sq = sqrt_fast<R>(R(0.5) * (ML * ML + MR * MR)) - R(1);
    R mh = R(0.25) * bl * br * sq * sq;
    R dpp = plp - prp;
    R ri = rcp_fast<R>(at * at);
    R mhp = mh * (R(1) - (dpp + fabs(dpp)) * R(0.5) * rcp_fast<R>(rl) * ri);
    R mhm = mh * (R(1) + (dpp - fabs(dpp)) * R(0.5) * rcp_fast<R>(rr) * ri);
    R fl = at * rl * (cp - mhp), fr = at * rr * (cm + mhm);
    R pf;
    if (eps >= R(1)) {
        bool sl, sr;
        R dp = dsplit(ML, true, sl), dm = dsplit(MR, false, sr);
        pf = dp * plp + dm * prp + fp.pinf * dsum_minus1(ML, MR, dp, dm, sl, sr);
    } else {
        R rah = rcp_fast<R>(ah);
        R mL = UL * rah, mR = UR * rah;
        bool sl, sr;
        R eL = dsplit(mL, true, sl), eR = dsplit(mR, false, sr);
        R pbp = R(0.5) * (plp + prp);
        pf = pbp + R(0.5) * (eL - eR) * dpp + at * rah * (fp.pinf + pbp) * dsum_minus1(mL, mR, eL, eR, sl, sr);
    }
    fl_out[0] = fl + fr;
#pragma unroll
    for (int e = 0; e < ND; ++e)
        fl_out[1 + e] = fl * wl[1 + e] + fr * wr[1 + e] + (e == d ? pf : R(0));
    R g1 = fp.gamma * fp.gm1inv;
    R hl = g1 * (plp - fp.pinf * wl[0]) * rcp_fast<R>(rl) + R(0.5) * (ql2 - fp.uinf2);
    R hr = g1 * (prp - fp.pinf * wr[0]) * rcp_fast<R>(rr) + R(0.5) * (qr2 - fp.uinf2);
    fl_out[NV - 1] = fl * hl + fr * hr;
}

template <typename Real> __device__ inline Real metric(const double *d64, const float *d32, int idx)
{
    if constexpr (sizeof(Real) == 4)
        return d32[idx];
    else
        return d64[idx];
}

// Flux through the face between tile-local cells L (LDS index `base`) and
// L + e_D: WENO5 face states, LDFSS, minus the central viscous flux.
// rdn = 1 / (distance of the two cell centres); rt3[e] (e != D) =
// 1 / (distance of the centres of L's neighbours along e).
// TDER: the staging holds (rho', u.., p') only and T' = (p' - R rho') /
// (R (1 + rho')) is formed at the two cells of the face (p_inf = R).
template <int DIM, int D, typename Real, int LX, int LY, int LCELLS, bool TDER = false>
__device__ inline void face_flux(const Real *__restrict__ S, int base, Real rdn, const Real *rt3,
                                 const FlowR<Real> &fp, Real *flux)
{
    constexpr int NV = DIM + 2;
    constexpr int SD = D == 0 ? 1 : (D == 1 ? LX : LX * LY);
    Real wl[NV], wr[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        const Real *s = S + m * LCELLS + base;
        if (fp.tvd) {
            tvd2_pair<Real>(s[-SD], s[0], s[SD], s[2 * SD], wl[m], wr[m]);
        } else {
            Real v0 = s[-2 * SD], v1 = s[-SD], v2 = s[0], v3 = s[SD], v4 = s[2 * SD], v5 = s[3 * SD];
            weno5_pair<Real>(v0, v1, v2, v3, v4, v5, wl[m], wr[m]);
        }
    }
    ldfss_pert<Real, NV, D>(wl, wr, fp, flux);

    // viscous flux: tau = mu (grad u + grad u^T - 2/3 div u I), q = -k grad T;
    // normal derivatives from the two cells, tangential ones the mean of the
    // two cells' central differences, face velocity the mean of the cells
    const Real *SU = S + LCELLS;
    const Real *ST = S + (TDER ? 0 : (DIM + 2) * LCELLS);
    Real dudn[DIM], uf[DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
        Real uL = SU[m * LCELLS + base], uR = SU[m * LCELLS + base + SD];
        dudn[m] = (uR - uL) * rdn;
        uf[m] = Real(0.5) * (uL + uR);
    }
    Real dTdn;
    if constexpr (TDER) {
        const Real *SR = S, *SP = S + (DIM + 1) * LCELLS;
        Real tL = (SP[base] - fp.pinf * SR[base]) * fp.rR * rcp_fast<Real>(Real(1) + SR[base]);
        Real tR = (SP[base + SD] - fp.pinf * SR[base + SD]) * fp.rR * rcp_fast<Real>(Real(1) + SR[base + SD]);
        dTdn = (tR - tL) * rdn;
    } else {
        dTdn = (ST[base + SD] - ST[base]) * rdn;
    }
    Real div = dudn[D];
    Real tau[DIM];
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
        if (e == D)
            continue;
        const int SE = e == 0 ? 1 : (e == 1 ? LX : LX * LY);
        Real rt = rt3[e];
        const Real *UD = SU + D * LCELLS, *UE = SU + e * LCELLS;
        Real dUD = Real(0.5) * ((UD[base + SE] - UD[base - SE]) + (UD[base + SD + SE] - UD[base + SD - SE])) * rt;
        Real dUE = Real(0.5) * ((UE[base + SE] - UE[base - SE]) + (UE[base + SD + SE] - UE[base + SD - SE])) * rt;
        div += dUE;
        tau[e] = fp.mu * (dudn[e] + dUD);
    }
    tau[D] = fp.mu * (Real(2) * dudn[D] - Real(2.0 / 3.0) * div);
    Real work = Real(0);
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
        flux[1 + m] -= tau[m];
        work += uf[m] * tau[m];
    }
    flux[NV - 1] -= work + fp.kc * dTdn;
}

// Metrics of a tile, staged in LDS once per block so that the face loops
// read no global memory for them: mn[d][l + 1] = 1 / (x_{c+1} - x_c) for the
// tile-local cell l in [-1, T_d) along axis d (the normal derivative across
// the face after it), mt[d][l] = 1 / (x_{c+1} - x_{c-1}) for l in [0, T_d)
// (its tangential central difference); c = o_d + l.  Entries past the grid
// repeat the last halo entry (their faces are skipped).
template <typename Real, int TMAX> struct TileMetrics {
    Real mn[3][TMAX + 1];
    Real mt[3][TMAX];
};

template <int DIM, typename Real, int TMAX>
__device__ inline void stage_metrics(TileMetrics<Real, TMAX> &M, const Grid &g, const int *T, const int *o, int tid)
{
    const int n[3] = {g.ni, g.nj, g.nk};
    int e = tid;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        if (e >= 0 && e < T[d] + 1) {
            int c = o[d] + e - 1;
            c = c > n[d] + 2 ? n[d] + 2 : c;
            M.mn[d][e] = metric<Real>(g.rdxc[d], g.rdxc_f[d], c + 3);
        }
        e -= T[d] + 1;
        if (e >= 0 && e < T[d]) {
            int c = o[d] + e;
            c = c > n[d] + 2 ? n[d] + 2 : c;
            M.mt[d][e] = metric<Real>(g.rdtc[d], g.rdtc_f[d], c + 3);
        }
        e -= T[d];
    }
}

// All faces of direction D in a tile, written to F at offset `off`.
template <int DIM, int D, typename Real, int TX, int TY, int TZ, int HZ, int TMAX>
__device__ inline void face_pass(const Real *__restrict__ S, Real *__restrict__ F, int NFACE, int off,
                                 const int *lim, const TileMetrics<Real, TMAX> &M, const FlowR<Real> &fp, int tid)
{
    constexpr int LX = TX + 6, LY = TY + 6, LZ = TZ + 2 * HZ;
    constexpr int LCELLS = LX * LY * LZ;
    constexpr int NV = DIM + 2;
    constexpr int FX = TX + (D == 0), FY = TY + (D == 1), FZ = TZ + (D == 2);
    constexpr int NF = FX * FY * FZ;
    constexpr int NT = TileCfg<DIM>::NT;
    for (int fi = tid; fi < NF; fi += NT) {
        int fx = fi % FX, fy = (fi / FX) % FY, fz = fi / (FX * FY);
        int lc[3] = {fx - (D == 0), fy - (D == 1), fz - (D == 2)};
        // the face is needed if its left cell lies in [-1, n) along D and
        // the transverse coordinates are interior (lim: the tile's cells
        // inside the grid along each axis)
        bool need = lc[0] < lim[0] && lc[1] < lim[1] && (DIM == 2 || lc[2] < lim[2]);
        if (!need)
            continue;
        int base = (lc[0] + 3) + (lc[1] + 3) * LX + (DIM == 3 ? (lc[2] + HZ) * LX * LY : 0);
        Real rt3[3];
#pragma unroll
        for (int e = 0; e < DIM; ++e)
            rt3[e] = e == D ? Real(0) : M.mt[e][lc[e]];
        Real flux[NV];
        face_flux<DIM, D, Real, LX, LY, LCELLS>(S, base, M.mn[D][lc[D] + 1], rt3, fp, flux);
#pragma unroll
        for (int m = 0; m < NV; ++m)
            F[m * NFACE + off + fi] = flux[m];
    }
}

// 3. per-cell residual and update, one thread per tile cell: FLUID cells
// take the RK3 stage or the dual-time pseudo step (FP64), IB nodes keep
// their filled value (written by the inline fill, or copied), SOLID cells
// their state; residual mode writes R.
template <int DIM, typename Real, int MODE, bool INLINE_GHOSTS>
__device__ __forceinline__ void update_cell(const StepArgs &__restrict__ A, bool own, uint8_t cls, const double *qc,
                                            const Real *racc, long long cell, long long s_own, int i, int j, int k,
                                            const double *qn_pre = nullptr)
{
    constexpr int NV = DIM + 2;
    const Grid &g = A.g;
    const Flow &f = A.f;
    if (!own)
        return;
    long long s = s_own;
    if (MODE != MODE_RESID) {
        if (cls != IBM_FLUID) {  // IB nodes carry their filled value, solid cells their state
            if (INLINE_GHOSTS && cls >= IBM_FORCING && cls <= IBM_G3)
                return;  // written by the inline fill
#pragma unroll
            for (int m = 0; m < NV; ++m)
                A.out[s + m * g.vs] = qc[m];
            return;
        }
    } else if (cls != IBM_FLUID) {
#pragma unroll
        for (int m = 0; m < NV; ++m)
            A.out[m * g.ncell + cell] = 0.0;
        return;
    }
    double R[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m)
        R[m] = (double)racc[m];
    R[NV - 1] += f.Hinf * R[0];

    if (MODE == MODE_RESID) {
#pragma unroll
        for (int m = 0; m < NV; ++m)
            A.out[m * g.ncell + cell] = R[m];
        return;
    }
    if (MODE == MODE_RK3) {
        bool bad = false;
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            double qv = A.b * (qc[m] - f.dt * R[m]);
            if (A.a != 0.0)
                qv += A.a * (qn_pre ? qn_pre[m] : A.qn[s + m * g.vs]);
            A.out[s + m * g.vs] = qv;
            bad |= !isfinite(qv);
            if (m == 0)
                bad |= !(qv > 0.0);
        }
        if (bad)
            raise_status(A.ib, A.counts, ST_NONFINITE);
        return;
    }
    // MODE_DUAL: point-implicit preconditioned pseudo-time step, FP64
    {
        constexpr int N = NV;
        double pp = qc[0], tp = qc[DIM + 1];
        double u[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            u[d] = qc[1 + d];
        double p = f.pinf + pp, T = 1.0 + tp;
        // reciprocals instead of divides (within an ulp or so)
        double rTi = rcp_fast<double>(T);
        double rho = p * f.rR * rTi;
        double rhop = (pp - f.R * tp) * f.rR * rTi;  // rho - 1
        double rrho = rcp_fast<double>(rho);
        double q2 = 0.0;
        for (int d = 0; d < DIM; ++d)
            q2 += u[d] * u[d];
        double a2 = f.gamma * p * rrho;
        double ur2 = fmin(a2, fmax(q2, f.uc2));
        double eps = ur2 * rcp_fast<double>(a2);
        double nuv = f.mu * rrho * fmax(4.0 / 3.0, f.gamma / f.pr);
        double lam = 0.0;
        for (int d = 0; d < DIM; ++d) {
            double rdx = g.rdx[d][(d == 0 ? i : d == 1 ? j : k) + 3];
            double ud = u[d];
            double up = 0.5 * (1.0 + eps) * fabs(ud);
            double cpr = 0.5 * sqrt_fast<double>((1.0 - eps) * (1.0 - eps) * ud * ud + 4.0 * eps * a2);
            lam += (up + cpr) * rdx + 2.0 * nuv * rdx * rdx;
        }
        double rdt = rcp_fast<double>(f.dt);
        double b0 = A.a, b2 = A.b;
        double cdt = b0 * rdt, ctau = lam * rcp_fast<double>(f.cfl_tau);
        double rp = f.rR * rTi, rT = -rho * rTi;
        double th = rcp_fast<double>(ur2) + rcp_fast<double>(f.cp * T);
        // perturbation conserved vector of the current state
        double Qp[N];
        Qp[0] = rhop;
        for (int d = 0; d < DIM; ++d)
            Qp[1 + d] = rhop * u[d] + (u[d] - f.uinf[d]);
        Qp[N - 1] = pp * f.gm1inv + 0.5 * (rhop * q2 + q2 - f.uinf2);
        double rhs[N];
#pragma unroll
        for (int m = 0; m < N; ++m) {
            double qn = A.qn[m * g.ncell + cell], qm = A.qnm1[m * g.ncell + cell];
            rhs[m] = -((b0 * (Qp[m] - qn) - b2 * (qn - qm)) * rdt + R[m]);
        }
        // energy row minus H times the mass row: exact row operation that
        // removes the O(H) terms (H' = c_p T' + (|u|^2 - 1) / 2)
        double H = f.cp * T + 0.5 * q2;
        double Hp = f.cp * tp + 0.5 * (q2 - f.uinf2);
        {
            double qn0 = A.qn[cell], qm0 = A.qnm1[cell];
            double qnE = A.qn[(N - 1) * g.ncell + cell], qmE = A.qnm1[(N - 1) * g.ncell + cell];
            double bdf0 = b0 * (Qp[0] - qn0) - b2 * (qn0 - qm0);
            double bdfE = b0 * (Qp[N - 1] - qnE) - b2 * (qnE - qmE);
            double Rrho = R[0], REp = R[N - 1] - f.Hinf * R[0];
            rhs[N - 1] = -((bdfE - H * bdf0) * rdt + (REp - Hp * Rrho));
        }
        double M[N][N];
        for (int r = 0; r < N; ++r)
            for (int c = 0; c < N; ++c)
                M[r][c] = 0.0;
        double cc = ctau + cdt;
        M[0][0] = th * ctau + rp * cdt;
        M[0][N - 1] = rT * cc;
        for (int d = 0; d < DIM; ++d) {
            M[1 + d][0] = u[d] * (th * ctau + rp * cdt);
            M[1 + d][1 + d] = rho * cc;
            M[1 + d][N - 1] = u[d] * rT * cc;
            M[N - 1][1 + d] = rho * u[d] * cc;
        }
        M[N - 1][0] = -cc;
        M[N - 1][N - 1] = rho * f.cp * cc;
        (void)H;
        // Gaussian elimination with partial pivoting; every index is fixed
        // at compile time (row swaps by selects), so that the matrix stays
        // in registers, and each pivot is inverted once
        double dinv[N];
#pragma unroll
        for (int c = 0; c < N; ++c) {
            int piv = c;
            double big = fabs(M[c][c]);
#pragma unroll
            for (int r = c + 1; r < N; ++r)
                if (fabs(M[r][c]) > big) {
                    big = fabs(M[r][c]);
                    piv = r;
                }
#pragma unroll
            for (int r = c + 1; r < N; ++r) {
                if (r == piv) {
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        double t = M[c][m];
                        M[c][m] = M[r][m];
                        M[r][m] = t;
                    }
                    double t = rhs[c];
                    rhs[c] = rhs[r];
                    rhs[r] = t;
                }
            }
            dinv[c] = rcp_fast<double>(M[c][c]);
#pragma unroll
            for (int r = c + 1; r < N; ++r) {
                double fct = M[r][c] * dinv[c];
#pragma unroll
                for (int m = c; m < N; ++m)
                    M[r][m] -= fct * M[c][m];
                rhs[r] -= fct * rhs[c];
            }
        }
#pragma unroll
        for (int r = N - 1; r >= 0; --r) {
            double sum = rhs[r];
#pragma unroll
            for (int m = r + 1; m < N; ++m)
                sum -= M[r][m] * rhs[m];
            rhs[r] = sum * dinv[r];
        }
        bool bad = false;
        for (int m = 0; m < N; ++m) {
            double v = qc[m] + rhs[m];
            A.out[s + m * g.vs] = v;
            bad |= !isfinite(v);
        }
        if (bad)
            raise_status(A.ib, A.counts, ST_NONFINITE);
    }
}

template <int DIM, typename Real, int MODE, bool INLINE_GHOSTS>
__device__ __forceinline__ void step_body(const StepArgs &__restrict__ A, int bid)
{
    using C = TileCfg<DIM>;
    constexpr int TX = C::TX, TY = C::TY, TZ = C::TZ, HZ = C::HZ, NT = C::NT;
    constexpr int LX = TX + 6, LY = TY + 6, LZ = TZ + 2 * HZ;
    constexpr int NV = DIM + 2;          // conserved variables
    constexpr int NS = DIM + 3;          // rho', u.., p', T'
    constexpr int LCELLS = LX * LY * LZ;
    constexpr int NF0 = (TX + 1) * TY * TZ;
    constexpr int NF1 = TX * (TY + 1) * TZ;
    constexpr int NF2 = DIM == 3 ? TX * TY * (TZ + 1) : 0;
    // 3D and FP64 keep the fluxes of one direction at a time (the residual
    // accumulates per cell in registers; for FP64 2D that halves the flux
    // LDS, five blocks per CU instead of four), mixed 2D all of them
    constexpr bool SPLIT = DIM == 3 || sizeof(Real) == 8;
    constexpr int NFMAX = NF0 > NF1 ? (NF0 > NF2 ? NF0 : NF2) : (NF1 > NF2 ? NF1 : NF2);
    constexpr int NFACE = SPLIT ? NFMAX : NF0 + NF1 + NF2;
    __shared__ Real S[NS * LCELLS];
    __shared__ Real F[NV * NFACE];
    constexpr int TMAX = TX > TY ? (TX > TZ ? TX : TZ) : (TY > TZ ? TY : TZ);
    __shared__ TileMetrics<Real, TMAX> M;

    const Grid &g = A.g;
    const Flow &f = A.f;
    // tile id: the blocks b with the same b mod 8 (dispatched to the same
    // XCD) take a contiguous run of the tile list, so neighbouring tiles
    // share that XCD's L2
    const int32_t *list = A.tiles;
    int nt = list ? A.ntiles : A.ntx * A.nty * A.ntz;
    int b = bid;
    int per = (nt + 7) / 8;
    int pos = (b % 8) * per + b / 8;
    if (pos >= nt)
        return;
    int tile = list ? list[pos] : pos;
    if (tile < 0)  // padding of a tile list
        return;
    int tx0 = tile % A.ntx, ty0 = (tile / A.ntx) % A.nty, tz0 = tile / (A.ntx * A.nty);
    int i0 = tx0 * TX, j0 = ty0 * TY, k0 = tz0 * TZ;
    int tid = threadIdx.x;
    constexpr int NCELL = TX * TY * TZ;
    static_assert(NCELL <= NT, "one thread per tile cell");
    const int T3[3] = {TX, TY, TZ}, o3[3] = {i0, j0, k0};
    static_assert(2 * (TX + TY + TZ) + 3 <= NT, "one thread per staged metric");
    stage_metrics<DIM, Real, TMAX>(M, g, T3, o3, tid);
    const int lim[3] = {g.ni - i0, g.nj - j0, DIM == 3 ? g.nk - k0 : 1};


    // perturbation primitives of state values qv into LDS cell t
    const double rinv = f.rR;
    auto put = [&](int t, const double *qv) {
        double v[NS];
        if (f.scheme == IBM_RK3) {
            double rho = qv[0];
            double ri = rcp_fast<double>(rho);  // one reciprocal per cell
            double ke = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                v[1 + d] = qv[1 + d] * ri;
                ke += v[1 + d] * v[1 + d];
            }
            double p = (f.gamma - 1.0) * (qv[DIM + 1] - 0.5 * rho * ke);
            v[0] = rho - 1.0;
            v[DIM + 1] = p - f.pinf;
            v[DIM + 2] = p * ri * rinv - 1.0;
        } else {
            double pp = qv[0], tp = qv[DIM + 1];
#pragma unroll
            for (int d = 0; d < DIM; ++d)
                v[1 + d] = qv[1 + d];
            v[0] = (pp - f.R * tp) * f.rR * rcp_fast<double>(1.0 + tp);
            v[DIM + 1] = pp;
            v[DIM + 2] = tp;
        }
#pragma unroll
        for (int m = 0; m < NS; ++m)
            S[m * LCELLS + t] = (Real)v[m];
    };

    // 1. load the tile and its 3-cell halo, recovering (rho', u.., p', T');
    //    domain ghost cells are resolved on the fly.  Several rounds of
    //    loads are issued before any is converted.
    constexpr int NR = (LCELLS + NT - 1) / NT;
    // (3D: every round in flight at once, 2548 cells over 512 threads;
    // C4 stage 0.473 -> 0.453 ms against two rounds at a time)
    constexpr int NB = DIM == 3 ? NR : (NR < 2 ? NR : 2);
    for (int r0 = 0; r0 < NR; r0 += NB) {
        double qv[NB][NV];
#pragma unroll
        for (int rr = 0; rr < NB; ++rr) {
            int t = tid + (r0 + rr) * NT;
            if (r0 + rr >= NR || t >= LCELLS)
                continue;
            int lx = t % LX, ly = (t / LX) % LY, lz = t / (LX * LY);
            int c[3] = {i0 + lx - 3, j0 + ly - 3, k0 + lz - HZ};
            bool ff = ghost_source<DIM>(g, c);
            if (ff) {
#pragma unroll
                for (int m = 0; m < NV; ++m)
                    qv[rr][m] = A.fs.v[m];
            } else {
                long long s = sidx(g, c[0], c[1], c[2]);
#pragma unroll
                for (int m = 0; m < NV; ++m)
                    qv[rr][m] = A.qin[s + m * g.vs];
            }
        }
#pragma unroll
        for (int rr = 0; rr < NB; ++rr) {
            int t = tid + (r0 + rr) * NT;
            if (r0 + rr >= NR || t >= LCELLS)
                continue;
            put(t, qv[rr]);
        }
    }

    // 1b. inline IB fill (tiles whose stencils reach the IB region): the IB
    //     nodes among the loaded cells (the tile's list, built after
    //     classification) take their filled values, computed from the stage
    //     input in two sweeps, one node per lane group: FORCING nodes from FLUID
    //     cells, then ghost nodes G1-G3 from FLUID cells and the filled
    //     values of their FORCING corners.  A node inside the tile also
    //     stores its value as its stage output.
    if constexpr (INLINE_GHOSTS) {
        const IB &ib = A.ib;
        int slot = ib.cap > 0 ? ib.tile_slot[tile] : -1;
        int n = slot >= 0 ? ib.tg_cnt[slot] : 0;
        if (n > 0) {
            int nF = min(ib.counts[CNT_F], ib.cap);
            int nj = ib.tj_cnt[slot];
            bool own_corners = nj < 0;  // the corner list did not fit
            nj = max(nj, 0);
            const int32_t *lt = ib.tg_t + (long long)slot * ib.tg_stride;
            const int32_t *lr = ib.tg_rec + (long long)slot * ib.tg_stride;
            const int32_t *lj = ib.tj_rec + (long long)slot * ib.tg_stride;
            // list entry e: its LDS cell, its state offset, whether it lies
            // in the tile (then its value is also the stage output)
            auto where = [&](int e, int &t, long long &so, bool &inside) {
                t = lt[e];
                int lx = t % LX, ly = (t / LX) % LY, lz = t / (LX * LY);
                int c[3] = {i0 + lx - 3, j0 + ly - 3, k0 + lz - HZ};
                inside = lx >= 3 && lx < 3 + TX && ly >= 3 && ly < 3 + TY && lz >= HZ && lz < HZ + TZ &&
                         c[0] < g.ni && c[1] < g.nj && (DIM == 2 || c[2] < g.nk);
                ghost_source<DIM>(g, c);
                so = sidx(g, c[0], c[1], c[2]);
            };
            auto place = [&](int t, long long so, bool inside, const double *qs) {
                put(t, qs);
                if (inside) {
#pragma unroll
                    for (int m = 0; m < NV; ++m)
                        A.out[so + m * g.vs] = qs[m];
                }
            };
            __syncthreads();  // the loaded values are in LDS before IB values replace them
            // one lane group (2^DIM lanes) per list entry; lane 0 stores
            constexpr int G = 1 << DIM, NG = NT / G;
            const int gc = tid % G;
            // sweep 1: the listed FORCING nodes and the FORCING corners the
            // listed ghosts read outside the loaded cells, each filled from
            // FLUID cells and kept in fval; entries without a record keep
            // their stored value
            for (int e = tid / G; e < n + nj; e += NG) {
                double qs[NV];
                if (e < n) {
                    int rec = lr[e];
                    if (rec >= nF)
                        continue;  // ghost node: sweep 2
                    int t;
                    long long so;
                    bool inside;
                    where(e, t, so, inside);
                    if (rec < 0) {  // no record (capacity exceeded, flagged)
#pragma unroll
                        for (int m = 0; m < NV; ++m)
                            qs[m] = A.qin[so + m * g.vs];
                    } else {
                        node_fill<DIM, false>(g, f, ib, A.qin, rec, gc, A.ub, A.ab, A.axis, qs);
                        if (gc == 0) {
#pragma unroll
                            for (int m = 0; m < NV; ++m)
                                ib.fval[(long long)m * ib.cap + rec] = qs[m];
                        }
                    }
                    if (gc == 0)
                        place(t, so, inside, qs);
                } else {
                    int rec = lj[e - n];
                    node_fill<DIM, false>(g, f, ib, A.qin, rec, gc, A.ub, A.ab, A.axis, qs);
                    if (gc == 0) {
#pragma unroll
                        for (int m = 0; m < NV; ++m)
                            ib.fval[(long long)m * ib.cap + rec] = qs[m];
                    }
                }
            }
            __syncthreads();  // sweep 1's fval stores are seen by the whole block
            // sweep 2: ghost nodes G1-G3, their FORCING corners from fval
            for (int e = tid / G; e < n; e += NG) {
                int rec = lr[e];
                if (rec < nF)
                    continue;
                int t;
                long long so;
                bool inside;
                where(e, t, so, inside);
                double qs[NV];
                if (own_corners)
                    forcing_corners<DIM>(g, f, ib, A.qin, rec, gc, A.ub, A.ab, A.axis);
                node_fill<DIM, true>(g, f, ib, A.qin, rec, gc, A.ub, A.ab, A.axis, qs);
                if (gc == 0)
                    place(t, so, inside, qs);
            }
        }
    }

    // own cell of the update: its class and state are fetched before the
    // stencil work so that their latency overlaps it
    int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / (TX * TY);
    int i = i0 + tx, j = j0 + ty, k = k0 + tz;
    bool own = tid < NCELL && i < g.ni && j < g.nj && (DIM == 2 || k < g.nk);
    long long cell = ((long long)k * g.nj + j) * g.ni + i;
    long long s_own = sidx(g, i, j, k);
    uint8_t cls = IBM_SOLID;
    double qc[NV];
    // RK3 stages 2 and 3 also fetch Q^n here, so that its latency is
    // covered by the face passes rather than exposed at the update (3D:
    // stages 2-3 of the C4 tube 0.48 -> 0.45 ms; the 2D FP64 kernel would
    // lose a wave per SIMD to the registers, and does not)
    constexpr bool PRE_QN = MODE == MODE_RK3 && (DIM == 3 || sizeof(Real) == 4);
    double qn_pre[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m)
        qc[m] = qn_pre[m] = 0.0;
    if (own) {
        cls = A.cls[cell];
        if (MODE != MODE_RESID) {
#pragma unroll
            for (int m = 0; m < NV; ++m)
                qc[m] = A.qin[s_own + m * g.vs];
        }
        if (PRE_QN && A.a != 0.0) {
#pragma unroll
            for (int m = 0; m < NV; ++m)
                qn_pre[m] = A.qn[s_own + m * g.vs];
        }
    }
    __syncthreads();

    FlowR<Real> fp;
    fp.gamma = (Real)f.gamma;
    fp.gm1inv = (Real)f.gm1inv;
    fp.pinf = (Real)f.pinf;
    fp.mu = (Real)f.mu;
    fp.kc = (Real)f.kc;
    fp.uc2 = (Real)f.uc2;
    fp.uinf2 = (Real)f.uinf2;
    fp.rR = (Real)f.rR;
    fp.precond = f.scheme == IBM_DUAL;
    fp.tvd = f.recon == IBM_RECON_TVD2;
    // 2. face fluxes, one pass per direction (compile-time direction)
    int fl0 = (tz * TY + ty) * (TX + 1) + tx;  // x-face at i - 1/2
    int fl1 = (tz * (TY + 1) + ty) * TX + tx;  // y-face at j - 1/2
    int fl2 = (tz * TY + ty) * TX + tx;        // z-face at k - 1/2
    // threads without a cell of their own (past the tile's cells or the
    // grid) touch neither metrics nor fluxes
    Real rd[3] = {Real(0), Real(0), Real(0)};
    if (own) {
        rd[0] = metric<Real>(g.rdx[0], g.rdx_f[0], i + 3);
        rd[1] = metric<Real>(g.rdx[1], g.rdx_f[1], j + 3);
        if (DIM == 3)
            rd[2] = metric<Real>(g.rdx[2], g.rdx_f[2], k + 3);
    }
    Real racc[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m)
        racc[m] = Real(0);
    if constexpr (SPLIT) {
        face_pass<DIM, 0, Real, TX, TY, TZ, HZ, TMAX>(S, F, NFACE, 0, lim, M, fp, tid);
        __syncthreads();
        if (own) {
#pragma unroll
            for (int m = 0; m < NV; ++m)
                racc[m] = (F[m * NFACE + fl0 + 1] - F[m * NFACE + fl0]) * rd[0];
        }
        __syncthreads();
        face_pass<DIM, 1, Real, TX, TY, TZ, HZ, TMAX>(S, F, NFACE, 0, lim, M, fp, tid);
        __syncthreads();
        if (own) {
#pragma unroll
            for (int m = 0; m < NV; ++m)
                racc[m] += (F[m * NFACE + fl1 + TX] - F[m * NFACE + fl1]) * rd[1];
        }
        if constexpr (DIM == 3) {
            __syncthreads();
            face_pass<DIM, 2, Real, TX, TY, TZ, HZ, TMAX>(S, F, NFACE, 0, lim, M, fp, tid);
            __syncthreads();
            if (own) {
#pragma unroll
                for (int m = 0; m < NV; ++m)
                    racc[m] += (F[m * NFACE + fl2 + TX * TY] - F[m * NFACE + fl2]) * rd[2];
            }
        }
    } else {
        face_pass<DIM, 0, Real, TX, TY, TZ, HZ, TMAX>(S, F, NFACE, 0, lim, M, fp, tid);
        face_pass<DIM, 1, Real, TX, TY, TZ, HZ, TMAX>(S, F, NFACE, NF0, lim, M, fp, tid);
        __syncthreads();
        if (own) {
#pragma unroll
            for (int m = 0; m < NV; ++m) {
                const Real *Fm = F + m * NFACE;
                racc[m] = (Fm[fl0 + 1] - Fm[fl0]) * rd[0] + (Fm[NF0 + fl1 + TX] - Fm[NF0 + fl1]) * rd[1];
            }
        }
    }

    update_cell<DIM, Real, MODE, INLINE_GHOSTS>(A, own, cls, qc, racc, cell, s_own, i, j, k,
                                                PRE_QN ? qn_pre : nullptr);
}

// ----------------------------- 3D FP64 stages staged one direction at a time
// For tiles whose stencils never reach an IB node (the far tiles of a
// launch with a body, every tile without one): the tile's cells are staged
// in LDS one face direction at a time -- along it the three-cell WENO5 halo,
// across it the one cell the tangential derivatives read -- with
// (rho', u, v, w, p') only (T' follows from rho' and p').  That is about
// half the cells of the full halo'd tile and five of its six variables, so
// two 512-thread FP64 blocks share a CU (72 KB of LDS each) instead of one.
template <int D> struct DirBox {
    static constexpr int OX = D == 0 ? 3 : 1, OY = D == 1 ? 3 : 1, OZ = D == 2 ? 3 : 1;
    static constexpr int LX = kTile3[0] + 2 * OX, LY = kTile3[1] + 2 * OY, LZ = kTile3[2] + 2 * OZ;
    static constexpr int LCELLS = LX * LY * LZ;
};
constexpr int dir_cells_max()
{
    int a = DirBox<0>::LCELLS, b = DirBox<1>::LCELLS, c = DirBox<2>::LCELLS;
    return a > b ? (a > c ? a : c) : (b > c ? b : c);
}
constexpr int kDirCells = dir_cells_max();
constexpr int kDirFaces = 512;  // the most faces of a direction of the 8x7x8 tile
static_assert((kTile3[0] + 1) * kTile3[1] * kTile3[2] <= kDirFaces && kTile3[0] * (kTile3[1] + 1) * kTile3[2] <= kDirFaces &&
                  kTile3[0] * kTile3[1] * (kTile3[2] + 1) <= kDirFaces,
              "face buffer");

// Stage the box of direction D: state -> (rho', u, v, w, p') in FP64, domain
// ghost cells resolved on the fly, all rounds of loads in flight.
template <int D>
__device__ __forceinline__ void load_dir(const StepArgs &__restrict__ A, double *__restrict__ S, int i0, int j0,
                                         int k0, int tid)
{
    using B = DirBox<D>;
    constexpr int NV = 5, NT = kThreads3;
    constexpr int NR = (B::LCELLS + NT - 1) / NT;
    const Grid &g = A.g;
    const Flow &f = A.f;
    // every round of the box in flight at once (three for each box)
    for (int r0 = 0; r0 < NR; r0 += NR) {
        double qv[NR][NV];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            int t = tid + (r0 + rr) * NT;
            if (r0 + rr >= NR || t >= B::LCELLS)
                continue;
            int lx = t % B::LX, ly = (t / B::LX) % B::LY, lz = t / (B::LX * B::LY);
            int c[3] = {i0 + lx - B::OX, j0 + ly - B::OY, k0 + lz - B::OZ};
            bool ff = ghost_source<3>(g, c);
            if (ff) {
#pragma unroll
                for (int m = 0; m < NV; ++m)
                    qv[rr][m] = A.fs.v[m];
            } else {
                long long s = sidx(g, c[0], c[1], c[2]);
#pragma unroll
                for (int m = 0; m < NV; ++m)
                    qv[rr][m] = A.qin[s + m * g.vs];
            }
        }
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            int t = tid + (r0 + rr) * NT;
            if (r0 + rr >= NR || t >= B::LCELLS)
                continue;
            const double *v = qv[rr];
            double w[NV];
            if (f.scheme == IBM_RK3) {
                double rho = v[0];
                double ri = rcp_fast<double>(rho);
                double ke = 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    w[1 + d] = v[1 + d] * ri;
                    ke += w[1 + d] * w[1 + d];
                }
                w[0] = rho - 1.0;
                w[4] = (f.gamma - 1.0) * (v[4] - 0.5 * rho * ke) - f.pinf;
            } else {
                double pp = v[0], tp = v[4];
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    w[1 + d] = v[1 + d];
                w[0] = (pp - f.R * tp) * f.rR * rcp_fast<double>(1.0 + tp);
                w[4] = pp;
            }
#pragma unroll
            for (int m = 0; m < NV; ++m)
                S[m * B::LCELLS + t] = w[m];
        }
    }
}

// All faces of direction D of the tile, from the staging box of D.
template <int D>
__device__ __forceinline__ void face_pass_dir(const double *__restrict__ S, double *__restrict__ F, const int *lim,
                                              const TileMetrics<double, 8> &M, const FlowR<double> &fp, int tid)
{
    using B = DirBox<D>;
    constexpr int TX = kTile3[0], TY = kTile3[1], TZ = kTile3[2];
    constexpr int NV = 5, NT = kThreads3;
    constexpr int FX = TX + (D == 0), FY = TY + (D == 1), FZ = TZ + (D == 2);
    constexpr int NF = FX * FY * FZ;
    for (int fi = tid; fi < NF; fi += NT) {
        int fx = fi % FX, fy = (fi / FX) % FY, fz = fi / (FX * FY);
        int lc[3] = {fx - (D == 0), fy - (D == 1), fz - (D == 2)};
        if (!(lc[0] < lim[0] && lc[1] < lim[1] && lc[2] < lim[2]))
            continue;
        int base = (lc[0] + B::OX) + (lc[1] + B::OY) * B::LX + (lc[2] + B::OZ) * B::LX * B::LY;
        double rt3[3];
#pragma unroll
        for (int e = 0; e < 3; ++e)
            rt3[e] = e == D ? 0.0 : M.mt[e][lc[e]];
        double flux[NV];
        face_flux<3, D, double, B::LX, B::LY, B::LCELLS, true>(S, base, M.mn[D][lc[D] + 1], rt3, fp, flux);
#pragma unroll
        for (int m = 0; m < NV; ++m)
            F[m * kDirFaces + fi] = flux[m];
    }
}

template <int MODE>
__device__ __forceinline__ void step_body_dir3(const StepArgs &__restrict__ A, int bid)
{
    constexpr int TX = kTile3[0], TY = kTile3[1], TZ = kTile3[2], NT = kThreads3;
    constexpr int NV = 5;
    __shared__ double S[NV * kDirCells];
    __shared__ double F[NV * kDirFaces];
    __shared__ TileMetrics<double, 8> M;
    const Grid &g = A.g;
    const Flow &f = A.f;
    const int32_t *list = A.tiles;
    int nt = list ? A.ntiles : A.ntx * A.nty * A.ntz;
    int b = bid;
    int per = (nt + 7) / 8;
    int pos = (b % 8) * per + b / 8;
    if (pos >= nt)
        return;
    int tile = list ? list[pos] : pos;
    if (tile < 0)
        return;
    int tx0 = tile % A.ntx, ty0 = (tile / A.ntx) % A.nty, tz0 = tile / (A.ntx * A.nty);
    int i0 = tx0 * TX, j0 = ty0 * TY, k0 = tz0 * TZ;
    int tid = threadIdx.x;
    {
        const int T3[3] = {TX, TY, TZ}, o3[3] = {i0, j0, k0};
        stage_metrics<3, double, 8>(M, g, T3, o3, tid);
    }
    const int lim[3] = {g.ni - i0, g.nj - j0, g.nk - k0};
    int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / (TX * TY);
    int i = i0 + tx, j = j0 + ty, k = k0 + tz;
    bool own = tid < TX * TY * TZ && i < g.ni && j < g.nj && k < g.nk;
    long long cell = ((long long)k * g.nj + j) * g.ni + i;
    long long s_own = sidx(g, i, j, k);
    uint8_t cls = IBM_SOLID;
    double qc[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m)
        qc[m] = 0.0;
    double qn_pre[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m)
        qn_pre[m] = 0.0;
    if (own) {
        cls = A.cls[cell];
        if (MODE != MODE_RESID) {
#pragma unroll
            for (int m = 0; m < NV; ++m)
                qc[m] = A.qin[s_own + m * g.vs];
        }
        if (MODE == MODE_RK3 && A.a != 0.0) {
#pragma unroll
            for (int m = 0; m < NV; ++m)
                qn_pre[m] = A.qn[s_own + m * g.vs];
        }
    }
    FlowR<double> fp;
    fp.gamma = f.gamma;
    fp.gm1inv = f.gm1inv;
    fp.pinf = f.pinf;
    fp.mu = f.mu;
    fp.kc = f.kc;
    fp.uc2 = f.uc2;
    fp.uinf2 = f.uinf2;
    fp.rR = f.rR;
    fp.precond = f.scheme == IBM_DUAL;
    fp.tvd = f.recon == IBM_RECON_TVD2;
    double rd[3] = {0.0, 0.0, 0.0};
    if (own) {
        rd[0] = g.rdx[0][i + 3];
        rd[1] = g.rdx[1][j + 3];
        rd[2] = g.rdx[2][k + 3];
    }
    int fl0 = (tz * TY + ty) * (TX + 1) + tx;  // x-face at i - 1/2
    int fl1 = (tz * (TY + 1) + ty) * TX + tx;  // y-face at j - 1/2
    int fl2 = (tz * TY + ty) * TX + tx;        // z-face at k - 1/2
    double racc[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m)
        racc[m] = 0.0;
    load_dir<0>(A, S, i0, j0, k0, tid);
    __syncthreads();
    face_pass_dir<0>(S, F, lim, M, fp, tid);
    __syncthreads();
    if (own) {
#pragma unroll
        for (int m = 0; m < NV; ++m)
            racc[m] = (F[m * kDirFaces + fl0 + 1] - F[m * kDirFaces + fl0]) * rd[0];
    }
    load_dir<1>(A, S, i0, j0, k0, tid);
    __syncthreads();
    face_pass_dir<1>(S, F, lim, M, fp, tid);
    __syncthreads();
    if (own) {
#pragma unroll
        for (int m = 0; m < NV; ++m)
            racc[m] += (F[m * kDirFaces + fl1 + TX] - F[m * kDirFaces + fl1]) * rd[1];
    }
    load_dir<2>(A, S, i0, j0, k0, tid);
    __syncthreads();
    face_pass_dir<2>(S, F, lim, M, fp, tid);
    __syncthreads();
    if (own) {
#pragma unroll
        for (int m = 0; m < NV; ++m)
            racc[m] += (F[m * kDirFaces + fl2 + TX * TY] - F[m * kDirFaces + fl2]) * rd[2];
    }
    update_cell<3, double, MODE, false>(A, own, cls, qc, racc, cell, s_own, i, j, k,
                                        MODE == MODE_RK3 ? qn_pre : nullptr);
}


template <int DIM, typename Real, int MODE>
__global__ __launch_bounds__(TileCfg<DIM>::NT) void step_kernel(StepArgs A)
{
    (void)A;
    step_body<DIM, Real, MODE, false>(kernarg_block<StepArgs>(), blockIdx.x);
}

template <int DIM, typename Real, int MODE>
__global__ __launch_bounds__(TileCfg<DIM>::NT) void step_ghost_kernel(StepArgs A)
{
    (void)A;
    step_body<DIM, Real, MODE, true>(kernarg_block<StepArgs>(), blockIdx.x);
}


// Several solves in one launch: the blocks [off[m], off[m + 1]) run the
// launch described by args[m] (prepared in device memory).
struct BatchArgs {
    int n;
    int off[IBM_BATCH_MAX + 1];
    const StepArgs *args[IBM_BATCH_MAX];
};

template <int DIM, typename Real, int MODE, bool GHOSTS, bool DIR = false>
__device__ __forceinline__ void batch_body(const BatchArgs &B)
{
    int b = blockIdx.x;
    int lo = 0, hi = B.n - 1;  // the m with off[m] <= b < off[m + 1]
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (B.off[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    // the solve, its argument block and its first block are the same for
    // every lane: keep them in scalar registers, and read the block (never
    // written during a launch) through the constant address space, so the
    // argument loads are scalar too
    lo = __builtin_amdgcn_readfirstlane(lo);
    unsigned long long pa = reinterpret_cast<unsigned long long>(B.args[lo]);
    unsigned plo = __builtin_amdgcn_readfirstlane((unsigned)pa);
    unsigned phi = __builtin_amdgcn_readfirstlane((unsigned)(pa >> 32));
    using ConstArgs = __attribute__((address_space(4))) const StepArgs;
    const ConstArgs *ap = (const ConstArgs *)(((unsigned long long)phi << 32) | plo);
    int first = __builtin_amdgcn_readfirstlane(B.off[lo]);
    if constexpr (DIR)
        step_body_dir3<MODE>(*(const StepArgs *)ap, b - first);
    else
        step_body<DIM, Real, MODE, GHOSTS>(*(const StepArgs *)ap, b - first);
}

template <int DIM, typename Real, int MODE, bool GHOSTS>
__global__ __launch_bounds__(TileCfg<DIM>::NT) void step_batch_kernel(BatchArgs B)
{
    batch_body<DIM, Real, MODE, GHOSTS>(B);
}

// 3D FP32: the tile fits two 512-thread blocks per CU in LDS (four waves
// per SIMD), which leaves 128 registers per lane; the budget is stated
// (left to itself the compiler takes more and halves the occupancy).
template <int MODE>
__global__ __launch_bounds__(kThreads3) __attribute__((amdgpu_num_vgpr(128))) void step_kernel_3f(StepArgs A)
{
    (void)A;
    step_body<3, float, MODE, false>(kernarg_block<StepArgs>(), blockIdx.x);
}

template <int MODE>
__global__ __launch_bounds__(kThreads3) __attribute__((amdgpu_num_vgpr(128))) void step_ghost_kernel_3f(StepArgs A)
{
    (void)A;
    step_body<3, float, MODE, true>(kernarg_block<StepArgs>(), blockIdx.x);
}

template <int MODE, bool GHOSTS>
__global__ __launch_bounds__(kThreads3) __attribute__((amdgpu_num_vgpr(128))) void step_batch_kernel_3f(BatchArgs B)
{
    batch_body<3, float, MODE, GHOSTS>(B);
}

// 3D FP64 staged one direction at a time (tiles without IB nodes in their
// stencils): two blocks per CU, 128 registers per lane.
template <int MODE>
__global__ __launch_bounds__(kThreads3) __attribute__((amdgpu_num_vgpr(128))) void step_dir_kernel_3d(StepArgs A)
{
    // (by value: measured faster for this kernel than kernarg_block())
    step_body_dir3<MODE>(A, blockIdx.x);
}

template <int MODE>
__global__ __launch_bounds__(kThreads3) __attribute__((amdgpu_num_vgpr(128))) void step_batch_dir_kernel_3d(BatchArgs B)
{
    batch_body<3, double, MODE, false, true>(B);
}

// 2D FP32: the tile fits eight 256-thread blocks per CU in LDS; the
// register budget for eight (RK3) or seven (dual time, whose FP64 update is
// larger) waves per SIMD is stated, which the kernels meet without spills
// (left to itself the compiler takes a few registers more and loses a wave).
template <int MODE> constexpr int waves2f() { return MODE == MODE_DUAL ? 7 : 8; }
template <int MODE>
__global__ __launch_bounds__(kThreads2) __attribute__((amdgpu_waves_per_eu(waves2f<MODE>(), waves2f<MODE>()))) void
step_kernel_2f(StepArgs A)
{
    (void)A;
    step_body<2, float, MODE, false>(kernarg_block<StepArgs>(), blockIdx.x);
}

template <int MODE>
__global__ __launch_bounds__(kThreads2) __attribute__((amdgpu_waves_per_eu(waves2f<MODE>(), waves2f<MODE>()))) void
step_ghost_kernel_2f(StepArgs A)
{
    (void)A;
    step_body<2, float, MODE, true>(kernarg_block<StepArgs>(), blockIdx.x);
}

template <int MODE, bool GHOSTS>
__global__ __launch_bounds__(kThreads2) __attribute__((amdgpu_waves_per_eu(waves2f<MODE>(), waves2f<MODE>()))) void
step_batch_kernel_2f(BatchArgs B)
{
    batch_body<2, float, MODE, GHOSTS>(B);
}

// the kernel of each launch kind for (DIM, Real, MODE)
template <int DIM, typename Real, int MODE> constexpr auto plain_kernel()
{
    if constexpr (DIM == 3 && sizeof(Real) == 4)
        return &step_kernel_3f<MODE>;
    else if constexpr (DIM == 3)
        return &step_dir_kernel_3d<MODE>;
    else if constexpr (DIM == 2 && sizeof(Real) == 4 && MODE != MODE_RESID)
        return &step_kernel_2f<MODE>;
    else
        return &step_kernel<DIM, Real, MODE>;
}
template <int DIM, typename Real, int MODE> constexpr auto ghost_kernel()
{
    if constexpr (DIM == 3 && sizeof(Real) == 4)
        return &step_ghost_kernel_3f<MODE>;
    else if constexpr (DIM == 2 && sizeof(Real) == 4)
        return &step_ghost_kernel_2f<MODE>;
    else
        return &step_ghost_kernel<DIM, Real, MODE>;
}
template <int DIM, typename Real, int MODE, bool GHOSTS> constexpr auto batch_kernel()
{
    if constexpr (DIM == 3 && sizeof(Real) == 4)
        return &step_batch_kernel_3f<MODE, GHOSTS>;
    else if constexpr (DIM == 3 && !GHOSTS)
        return &step_batch_dir_kernel_3d<MODE>;
    else if constexpr (DIM == 2 && sizeof(Real) == 4)
        return &step_batch_kernel_2f<MODE, GHOSTS>;
    else
        return &step_batch_kernel<DIM, Real, MODE, GHOSTS>;
}

// IB lists of the near tiles: block p scans the cells tile slot_tile[p]
// loads (tile plus halo, domain ghost cells resolved as the stencils do) and
// lists those that are IB nodes (FORCING, G1-G3), with their records; then
// the FORCING probe corners of the listed ghost nodes that lie outside the
// loaded cells (the ones inside are listed already).  Without corner lists
// (or when one does not fit) the count is -1: the tile's ghost nodes then
// fill their FORCING corners themselves, with the same results.
template <int DIM>
__global__ __launch_bounds__(kBlock) void ghost_lists_kernel(Grid g, IB ib, int ntx, int nty, int quad, int corner_lists)
{
    using C = TileCfg<DIM>;
    constexpr int TX = C::TX, TY = C::TY, TZ = C::TZ, HZ = C::HZ;
    constexpr int LX = TX + 6, LY = TY + 6, LZ = TZ + 2 * HZ;
    constexpr int LCELLS = LX * LY * LZ;
    __shared__ int n;
    if (threadIdx.x == 0)
        n = 0;
    __syncthreads();
    int slot = blockIdx.x;
    int tile = ib.slot_tile[slot];
    int i0 = (tile % ntx) * TX, j0 = ((tile / ntx) % nty) * TY, k0 = (tile / (ntx * nty)) * TZ;
    // every round's class loads in flight at once (cells outside the region
    // or the grid read cell 0 and are skipped)
    constexpr int NR = (LCELLS + kBlock - 1) / kBlock;
    int rcs[NR];
    uint8_t kcs[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        int t = threadIdx.x + r * kBlock;
        int rc = -1;
        long long cell = 0;
        if (t < LCELLS) {
            int lx = t % LX, ly = (t / LX) % LY, lz = t / (LX * LY);
            int c[3] = {i0 + lx - 3, j0 + ly - 3, k0 + lz - HZ};
            if (!ghost_source<DIM>(g, c)) {
                int li = c[0] - ib.region[0], lj = c[1] - ib.region[2], lk = c[2] - ib.region[4];
                if (li >= 0 && li < ib.rw && lj >= 0 && lj < ib.rh && lk >= 0 && lk < ib.rd) {
                    rc = (lk * ib.rh + lj) * ib.rw + li;
                    cell = ((long long)c[2] * g.nj + c[1]) * g.ni + c[0];
                }
            }
        }
        rcs[r] = rc;
        kcs[r] = ib.cls[cell];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        uint8_t kc = kcs[r];
        if (rcs[r] < 0 || kc < IBM_FORCING || kc > IBM_G3)
            continue;
        int e = atomicAdd(&n, 1);
        ib.tg_t[(long long)slot * ib.tg_stride + e] = threadIdx.x + r * kBlock;
        ib.tg_rec[(long long)slot * ib.tg_stride + e] = ib.rmap[rcs[r]];
    }
    __syncthreads();
    int nl = n;
    int nF = min(ib.counts[CNT_F], ib.cap);
    __shared__ int nj;
    if (threadIdx.x == 0)
        nj = 0;
    __syncthreads();
    constexpr int NC = 1 << DIM;
    int np = quad ? 2 : 1;  // probes per node
    for (int e = threadIdx.x; e < nl; e += kBlock) {
        int rec = ib.tg_rec[(long long)slot * ib.tg_stride + e];
        if (rec < nF)  // FORCING entry, or no record
            continue;
        int fr[2 * NC];
#pragma unroll
        for (int k = 0; k < 2 * NC; ++k)
            fr[k] = k < np * NC ? ib.plan_frec[(8 * (k / NC) + k % NC) * ib.cap + rec] : -1;
#pragma unroll
        for (int k = 0; k < 2 * NC; ++k) {
            if (fr[k] < 0)
                continue;
            int cc = ib.listF[fr[k]];
            int ci, cj, ck;
            split_cell(g, cc, ci, cj, ck);
            int lx = ci - i0 + 3, ly = cj - j0 + 3, lz = ck - k0 + HZ;
            if (lx >= 0 && lx < LX && ly >= 0 && ly < LY && lz >= 0 && lz < LZ)
                continue;
            int q = atomicAdd(&nj, 1);
            if (q < ib.tg_stride)
                ib.tj_rec[(long long)slot * ib.tg_stride + q] = fr[k];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ib.tg_cnt[slot] = nl;
        ib.tj_cnt[slot] = corner_lists && nj <= ib.tg_stride ? nj : -1;
    }
}

// Q'^{n-1} <- Q'^n (at the first step Q'^{n-1} <- Q(W) - Q_inf too); Q'^n <- Q(W) - Q_inf
__global__ void dual_begin_kernel(Grid g, Flow f, const double *w, double *qn, double *qnm1,
                                  int first)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell)
        return;
    int nd = g.ndim, N = g.nv;
    int i = (int)(c % g.ni), j = (int)((c / g.ni) % g.nj), k = (int)(c / ((long long)g.ni * g.nj));
    long long s = sidx(g, i, j, k);
    double pp = w[s], tp = w[s + (nd + 1) * g.vs];
    double u[3] = {0.0, 0.0, 0.0}, q2 = 0.0;
    for (int d = 0; d < nd; ++d) {
        u[d] = w[s + (1 + d) * g.vs];
        q2 += u[d] * u[d];
    }
    double T = 1.0 + tp;
    double rhop = (pp - f.R * tp) / (f.R * T);
    double Q[5];
    Q[0] = rhop;
    for (int d = 0; d < nd; ++d)
        Q[1 + d] = rhop * u[d] + (u[d] - f.uinf[d]);
    Q[N - 1] = pp / (f.gamma - 1.0) + 0.5 * (rhop * q2 + q2 - f.uinf2);
    // the first step (BDF1) weights Q'^{n-1} by zero; it is set to Q'^n so
    // that the term is an exact zero whatever the workspace held
    for (int m = 0; m < N; ++m) {
        qnm1[m * g.ncell + c] = first ? Q[m] : qn[m * g.ncell + c];
        qn[m * g.ncell + c] = Q[m];
    }
}

__global__ void prim_to_state_kernel(Grid g, Flow f, const double *prim, double *q)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell)
        return;
    int nd = g.ndim;
    int i = (int)(c % g.ni), j = (int)((c / g.ni) % g.nj), k = (int)(c / ((long long)g.ni * g.nj));
    PrimD w;
    w.u[0] = w.u[1] = w.u[2] = 0.0;
    w.rho = prim[c];
    for (int d = 0; d < nd; ++d)
        w.u[d] = prim[(1 + d) * g.ncell + c];
    w.p = prim[(nd + 1) * g.ncell + c];
    w.T = w.p / (w.rho * f.R);
    store_prim(g, f, w, q, sidx(g, i, j, k));
}

__global__ void state_to_prim_kernel(Grid g, Flow f, const double *q, double *prim)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell)
        return;
    int nd = g.ndim;
    int i = (int)(c % g.ni), j = (int)((c / g.ni) % g.nj), k = (int)(c / ((long long)g.ni * g.nj));
    PrimD w = load_prim(g, f, q, sidx(g, i, j, k));
    prim[c] = w.rho;
    for (int d = 0; d < nd; ++d)
        prim[(1 + d) * g.ncell + c] = w.u[d];
    prim[(nd + 1) * g.ncell + c] = w.p;
}

// interior cells of every variable (the halo is left as it is)
__global__ void copy_kernel(Grid g, const double *src, double *dst)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell)
        return;
    int i = (int)(c % g.ni), j = (int)((c / g.ni) % g.nj), k = (int)(c / ((long long)g.ni * g.nj));
    long long s = sidx(g, i, j, k);
    for (int m = 0; m < g.nv; ++m)
        dst[s + m * g.vs] = src[s + m * g.vs];
}

FreeStream freestream_of(const Grid &g, const Flow &f)
{
    FreeStream fs;
    for (int m = 0; m < 5; ++m)
        fs.v[m] = 0.0;
    if (f.scheme == IBM_RK3) {
        fs.v[0] = 1.0;
        for (int d = 0; d < g.ndim; ++d)
            fs.v[1 + d] = f.uinf[d];
        fs.v[g.nv - 1] = f.pinf / (f.gamma - 1.0) + 0.5 * f.uinf2;
    } else {
        for (int d = 0; d < g.ndim; ++d)
            fs.v[1 + d] = f.uinf[d];
    }
    return fs;
}

// Arguments of one stage launch, and its block count.
template <int DIM>
StepArgs make_args(const Grid &g, const Flow &f, const IB &ib, double *qin, const double *qn,
                   const double *qnm1, double *out, double a, double b, const StagePart *part,
                   int *nblk)
{
    const int *T = DIM == 2 ? kTile2 : kTile3;
    StepArgs A;
    A.g = g;
    A.f = f;
    A.cls = ib.cls;
    A.counts = ib.counts;
    A.qin = qin;
    A.qn = qn;
    A.qnm1 = qnm1;
    A.out = out;
    A.a = a;
    A.b = b;
    A.ntx = (g.ni + T[0] - 1) / T[0];
    A.nty = (g.nj + T[1] - 1) / T[1];
    A.ntz = DIM == 3 ? (g.nk + T[2] - 1) / T[2] : 1;
    A.tiles = part ? part->tiles : nullptr;
    A.ntiles = part ? part->ntiles : 0;
    A.ib = ib;
    A.ub = part ? part->ub : 0.0;
    A.ab = part ? part->ab : 0.0;
    A.axis = part ? part->axis : -1;
    A.fs = freestream_of(g, f);
    int nt = A.tiles ? A.ntiles : A.ntx * A.nty * A.ntz;
    *nblk = 8 * ((nt + 7) / 8);
    return A;
}

template <int DIM, typename Real, int MODE>
hipError_t run_step(const Grid &g, const Flow &f, const IB &ib, double *qin, const double *qn,
                    const double *qnm1, double *out, double a, double b, hipStream_t s,
                    const StagePart *part)
{
    int nblk = 0;
    StepArgs A = make_args<DIM>(g, f, ib, qin, qn, qnm1, out, a, b, part, &nblk);
    if (nblk == 0)
        return hipSuccess;
    hipEvent_t e0 = part ? part->ev_start : nullptr, e1 = part ? part->ev_stop : nullptr;
    if constexpr (MODE != MODE_RESID && DIM == 3 && sizeof(Real) == 8) {
        if (part && ib.cap > 0 && part->prefill) {
            // the IB nodes of the stage input filled in place, then every
            // tile with the kernel that stages one direction at a time
            StagePart pa = *part;
            pa.tiles = nullptr;
            pa.ntiles = 0;
            A = make_args<DIM>(g, f, ib, qin, qn, qnm1, out, a, b, &pa, &nblk);
            hipError_t e = launch_ib_fill(g, f, ib, qin, part->ub, part->ab, part->axis, s, e0);
            if (e != hipSuccess)
                return e;
            if (e1)
                hipExtLaunchKernelGGL((plain_kernel<DIM, Real, MODE>()), dim3(nblk), dim3(TileCfg<DIM>::NT), 0, s,
                                      nullptr, e1, 0, A);
            else
                hipLaunchKernelGGL((plain_kernel<DIM, Real, MODE>()), dim3(nblk), dim3(TileCfg<DIM>::NT), 0, s, A);
            return hipGetLastError();
        }
    }
    if constexpr (MODE != MODE_RESID) {
        if (part && ib.cap > 0) {
            if (e0)
                hipExtLaunchKernelGGL((ghost_kernel<DIM, Real, MODE>()), dim3(nblk), dim3(TileCfg<DIM>::NT), 0, s,
                                      e0, e1, 0, A);
            else
                hipLaunchKernelGGL((ghost_kernel<DIM, Real, MODE>()), dim3(nblk), dim3(TileCfg<DIM>::NT), 0, s, A);
            return hipGetLastError();
        }
    }
    if (e0)
        hipExtLaunchKernelGGL((plain_kernel<DIM, Real, MODE>()), dim3(nblk), dim3(TileCfg<DIM>::NT), 0, s, e0, e1, 0,
                              A);
    else
        hipLaunchKernelGGL((plain_kernel<DIM, Real, MODE>()), dim3(nblk), dim3(TileCfg<DIM>::NT), 0, s, A);
    return hipGetLastError();
}

template <int MODE>
hipError_t dispatch_step(const Grid &g, const Flow &f, const IB &ib, double *qin, const double *qn,
                         const double *qnm1, double *out, double a, double b, hipStream_t s,
                         const StagePart *part = nullptr)
{
    bool mixed = f.precision == IBM_MIXED;
    if (g.ndim == 2)
        return mixed ? run_step<2, float, MODE>(g, f, ib, qin, qn, qnm1, out, a, b, s, part)
                     : run_step<2, double, MODE>(g, f, ib, qin, qn, qnm1, out, a, b, s, part);
    return mixed ? run_step<3, float, MODE>(g, f, ib, qin, qn, qnm1, out, a, b, s, part)
                 : run_step<3, double, MODE>(g, f, ib, qin, qn, qnm1, out, a, b, s, part);
}

}  // namespace

hipError_t launch_domain_bc(const Grid &g, const Flow &f, double *q, hipStream_t s)
{
    int nhalo = (int)((long long)g.sx * g.sy * g.sz - g.ncell);
    hipLaunchKernelGGL(bc_kernel, dim3(blocks_for(nhalo, kBlock)), dim3(kBlock), 0, s, g,
                       freestream_of(g, f), q, nhalo);
    return hipGetLastError();
}

template <int DIM>
hipError_t ib_fill(const Grid &g, const Flow &f, const IB &ib, double *q, double ub_axis, double ab_axis, int axis,
                   hipStream_t s, hipEvent_t ev_start)
{
    int nbf = blocks_for((long long)ib.cap * (1 << DIM), kBlock);
    nbf = nbf < 256 ? nbf : 256;
    if (ev_start)
        hipExtLaunchKernelGGL(forcing_fill_kernel<DIM>, dim3(nbf), dim3(kBlock), 0, s, ev_start, nullptr, 0, g, f,
                              ib, q, ub_axis, ab_axis, axis);
    else
        hipLaunchKernelGGL(forcing_fill_kernel<DIM>, dim3(nbf), dim3(kBlock), 0, s, g, f, ib, q, ub_axis, ab_axis,
                           axis);
    hipLaunchKernelGGL(ghost_fill_kernel<DIM>, dim3(nbf), dim3(kBlock), 0, s, g, f, ib, q, ub_axis, ab_axis, axis);
    return hipGetLastError();
}

hipError_t launch_ib_fill(const Grid &g, const Flow &f, const IB &ib, double *q, double ub_axis, double ab_axis,
                          int axis, hipStream_t s, hipEvent_t ev_start)
{
    if (ib.cap <= 0)
        return hipSuccess;
    return g.ndim == 2 ? ib_fill<2>(g, f, ib, q, ub_axis, ab_axis, axis, s, ev_start)
                       : ib_fill<3>(g, f, ib, q, ub_axis, ab_axis, axis, s, ev_start);
}

// IB nodes (FORCING, then the ghost layers that read them), then the domain
// ghost layers as images of the filled interior.
hipError_t launch_bc_fill(const Grid &g, const Flow &f, const IB &ib, double *q, double ub_axis,
                          double ab_axis, int axis, hipStream_t s)
{
    hipError_t e = launch_ib_fill(g, f, ib, q, ub_axis, ab_axis, axis, s, nullptr);
    if (e != hipSuccess)
        return e;
    return launch_domain_bc(g, f, q, s);
}

hipError_t launch_residual(const Grid &g, const Flow &f, const IB &ib, const double *q, double *r,
                           hipStream_t s)
{
    // no fill part: the kernel only reads q
    return dispatch_step<MODE_RESID>(g, f, ib, const_cast<double *>(q), nullptr, nullptr, r, 0.0, 0.0,
                                     s);
}

hipError_t launch_rk_stage(const Grid &g, const Flow &f, const IB &ib, const double *qn, double *qin,
                           double *qout, double a, double b, hipStream_t s, const StagePart *part)
{
    return dispatch_step<MODE_RK3>(g, f, ib, qin, qn, nullptr, qout, a, b, s, part);
}

hipError_t launch_dual_iter(const Grid &g, const Flow &f, const IB &ib, double *w, double *wout,
                            const double *qn, const double *qnm1, double b0, double b2, hipStream_t s,
                            const StagePart *part)
{
    return dispatch_step<MODE_DUAL>(g, f, ib, w, qn, qnm1, wout, b0, b2, s, part);
}

hipError_t launch_dual_begin(const Grid &g, const Flow &f, const double *w, double *qn,
                             double *qnm1, int first, hipStream_t s)
{
    hipLaunchKernelGGL(dual_begin_kernel, dim3(blocks_for(g.ncell, kBlock)), dim3(kBlock), 0, s, g,
                       f, w, qn, qnm1, first);
    return hipGetLastError();
}

hipError_t launch_prim_to_state(const Grid &g, const Flow &f, const double *prim, double *q,
                                hipStream_t s)
{
    hipLaunchKernelGGL(prim_to_state_kernel, dim3(blocks_for(g.ncell, kBlock)), dim3(kBlock), 0, s,
                       g, f, prim, q);
    return hipGetLastError();
}

hipError_t launch_state_to_prim(const Grid &g, const Flow &f, const double *q, double *prim,
                                hipStream_t s)
{
    hipLaunchKernelGGL(state_to_prim_kernel, dim3(blocks_for(g.ncell, kBlock)), dim3(kBlock), 0, s,
                       g, f, q, prim);
    return hipGetLastError();
}

size_t stage_args_bytes() { return sizeof(StepArgs); }

int stage_args(const Grid &g, const Flow &f, const IB &ib, double *qin, const double *qn,
               const double *qnm1, double *out, double a, double b, const StagePart *part, void *dst)
{
    int nblk = 0;
    StepArgs A = g.ndim == 2 ? make_args<2>(g, f, ib, qin, qn, qnm1, out, a, b, part, &nblk)
                             : make_args<3>(g, f, ib, qin, qn, qnm1, out, a, b, part, &nblk);
    std::memcpy(dst, &A, sizeof A);
    return nblk;
}

template <int DIM, typename Real, int MODE>
hipError_t batch_launch(const BatchArgs &B, bool ghosts, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    int nblk = B.off[B.n];
    auto k = ghosts ? batch_kernel<DIM, Real, MODE, true>() : batch_kernel<DIM, Real, MODE, false>();
    if (e0 || e1)
        hipExtLaunchKernelGGL(k, dim3(nblk), dim3(TileCfg<DIM>::NT), 0, s, e0, e1, 0, B);
    else
        hipLaunchKernelGGL(k, dim3(nblk), dim3(TileCfg<DIM>::NT), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_stage_batch(int ndim, int precision, int scheme, bool ghosts, int n, const void *const *d_args,
                              const int *nblk, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    BatchArgs B;
    B.n = 0;
    B.off[0] = 0;
    for (int m = 0; m < n && m < IBM_BATCH_MAX; ++m) {
        if (nblk[m] <= 0)
            continue;
        B.args[B.n] = static_cast<const StepArgs *>(d_args[m]);
        B.off[B.n + 1] = B.off[B.n] + nblk[m];
        ++B.n;
    }
    if (B.n == 0)
        return hipSuccess;
    bool mixed = precision == IBM_MIXED, rk = scheme == IBM_RK3;
    if (ndim == 2) {
        if (rk)
            return mixed ? batch_launch<2, float, MODE_RK3>(B, ghosts, s, e0, e1)
                         : batch_launch<2, double, MODE_RK3>(B, ghosts, s, e0, e1);
        return mixed ? batch_launch<2, float, MODE_DUAL>(B, ghosts, s, e0, e1)
                     : batch_launch<2, double, MODE_DUAL>(B, ghosts, s, e0, e1);
    }
    if (rk)
        return mixed ? batch_launch<3, float, MODE_RK3>(B, ghosts, s, e0, e1)
                     : batch_launch<3, double, MODE_RK3>(B, ghosts, s, e0, e1);
    return mixed ? batch_launch<3, float, MODE_DUAL>(B, ghosts, s, e0, e1)
                 : batch_launch<3, double, MODE_DUAL>(B, ghosts, s, e0, e1);
}

int tile_load_cells(int ndim)
{
    const int *T = ndim == 2 ? kTile2 : kTile3;
    int hz = ndim == 2 ? 0 : 3;
    return (T[0] + 6) * (T[1] + 6) * (T[2] + 2 * hz);
}

hipError_t launch_ghost_lists(const Grid &g, const IB &ib, bool quad, bool corner_lists, hipStream_t s)
{
    if (ib.nslot == 0 || ib.cap == 0)
        return hipSuccess;
    const int *T = g.ndim == 2 ? kTile2 : kTile3;
    int ntx = (g.ni + T[0] - 1) / T[0], nty = (g.nj + T[1] - 1) / T[1];
    if (g.ndim == 2)
        hipLaunchKernelGGL(ghost_lists_kernel<2>, dim3(ib.nslot), dim3(kBlock), 0, s, g, ib, ntx, nty, (int)quad, (int)corner_lists);
    else
        hipLaunchKernelGGL(ghost_lists_kernel<3>, dim3(ib.nslot), dim3(kBlock), 0, s, g, ib, ntx, nty, (int)quad, (int)corner_lists);
    return hipGetLastError();
}

hipError_t launch_copy_state(const Grid &g, const double *src, double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(copy_kernel, dim3(blocks_for(g.ncell, kBlock)), dim3(kBlock), 0, s, g, src, dst);
    return hipGetLastError();
}

}  // namespace ibm
