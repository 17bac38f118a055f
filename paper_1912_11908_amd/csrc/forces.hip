// Surface force on the immersed body (Seshadri & De, section 6, eq.9) for
// gfx950: F_i = integral over the surface of (-P delta_ij + tau_ij) n_j.
//
// Quadrature and sampling (the paper names the integral and an
// inverse-distance sampling of the surface values, section 4.6): one point
// per facet, its centroid (2D: the segment midpoint), weighted by the facet's
// length (per unit span) or area, with the facet's outward unit normal.  P
// enters as P - p_inf (the constant's share, -p_inf times the sum of the
// area vectors, vanishes for a closed surface or a periodic prism).  P - p_inf
// and the velocity gradient at the point are weighted 1/r^2 over the centres
// of the enclosing cell box that are FLUID or FORCING (normalised; a centre at
// r = 0 takes the whole weight; no such centre: the facet adds nothing and is
// counted); the gradient at a cell is the central difference over its face
// neighbours; tau_ij = mu (d_j u_i + d_i u_j - 2/3 delta_ij div u) at the point.
//
// One thread per facet; the block sums its facets in a fixed tree order and a
// single block adds the block sums in a fixed order, so the result does not
// depend on scheduling.  Built with -ffp-contract=off, like the geometry.
#include <mutex>

#include "common.h"

namespace ibm {
namespace {

constexpr int kForceBlock = 256;

// Scratch of the allocation-free force entry point: the block sums of
// forces_kernel (3 doubles per block, at most kStaticForceBlocks blocks)
// followed by the facets-missed counter (one int32 in the next double slot).
// Each device holds its own copy until the process ends; host code reaches
// it only through the address hipGetSymbolAddress gives on that device.
constexpr int kStaticForceBlocks = IBM_FORCES_STATIC_MAX_FACETS / kForceBlock;
static __device__ __align__(256) double scratch[3 * kStaticForceBlocks + 32];
constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
double *scratch_ptr[kMaxDevices];  // per device, once resolved

__global__ void zero_i32_kernel(int32_t *p) { *p = 0; }

__device__ inline long long state_index(const Grid &g, int i, int j, int k)
{
    return ((long long)(k + g.hz) * g.sy + (j + 3)) * g.sx + (i + 3);
}

__device__ inline int wrap_cell(int i, int n) { return ((i % n) + n) % n; }

// enclosing centre pair along one axis: largest i0 with c[i0] <= y < c[i0 + 1]
// (interior pairs; on a periodic axis the pair may straddle the boundary)
__device__ inline bool bracket(const double *c, int n, bool periodic, double y, int &i0)
{
    int lo = periodic ? -1 : 0, hi = periodic ? n : n - 1;
    if (!(y >= c[lo + 3]) || !(y < c[hi + 3]))
        return false;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (c[mid + 3] <= y)
            lo = mid;
        else
            hi = mid;
    }
    i0 = lo;
    return true;
}

// velocity of the state at offset s
template <int DIM>
__device__ inline void velocity(const Grid &g, const Flow &f, const double *q, long long s, double *u)
{
    if (f.scheme == IBM_RK3) {
        double rho = q[s];
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            u[d] = q[s + (1 + d) * g.vs] / rho;
    } else {
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            u[d] = q[s + (1 + d) * g.vs];
    }
}

// P - p_inf of the state at offset s (dual time stores it directly)
template <int DIM>
__device__ inline double pressure_pert(const Grid &g, const Flow &f, const double *q, long long s)
{
    if (f.scheme != IBM_RK3)
        return q[s];
    double rho = q[s], ke = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        double u = q[s + (1 + d) * g.vs] / rho;
        ke += u * u;
    }
    double p = (f.gamma - 1.0) * (q[s + (DIM + 1) * g.vs] - 0.5 * rho * ke);
    return p - f.pinf;
}

template <int DIM>
__global__ __launch_bounds__(kForceBlock) void forces_kernel(Grid g, Body b, Flow f, IB ib, const double *q,
                                                             double *facet_out, double *part, int32_t *missed)
{
    constexpr int NC = 1 << DIM;
    __shared__ double red[3][kForceBlock];
    int fid = blockIdx.x * kForceBlock + threadIdx.x;
    double Fc[3] = {0.0, 0.0, 0.0};
    if (fid < b.nfacet) {
        const int *fv = b.facet + DIM * fid;
        double y[3] = {0.0, 0.0, 0.0}, area;
        for (int m = 0; m < DIM; ++m)
            for (int d = 0; d < DIM; ++d)
                y[d] += b.v[DIM * fv[m] + d] / DIM;
        if (DIM == 2) {
            double ex = b.v[2 * fv[1]] - b.v[2 * fv[0]], ey = b.v[2 * fv[1] + 1] - b.v[2 * fv[0] + 1];
            area = sqrt(ex * ex + ey * ey);
        } else {
            double e1[3], e2[3];
            for (int d = 0; d < 3; ++d) {
                e1[d] = b.v[3 * fv[1] + d] - b.v[3 * fv[0] + d];
                e2[d] = b.v[3 * fv[2] + d] - b.v[3 * fv[0] + d];
            }
            double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                            e1[0] * e2[1] - e1[1] * e2[0]};
            area = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        }
        const double *n = b.fnrm + 3 * fid;
        int nn[3] = {g.ni, g.nj, g.nk};
        int i0[3] = {0, 0, 0};
        bool ok = true;
        for (int d = 0; d < DIM && ok; ++d)
            ok = bracket(g.xc[d], nn[d], g.bc[2 * d] == IBM_BC_PERIODIC, y[d], i0[d]);
        double w[NC];
        int zero = -1, nvalid = 0;
        for (int m = 0; m < NC; ++m) {
            w[m] = 0.0;
            if (!ok)
                continue;
            int ci[3] = {0, 0, 0};
            double r2 = 0.0;
            for (int d = 0; d < DIM; ++d) {
                int bd = (m >> d) & 1;
                ci[d] = wrap_cell(i0[d] + bd, nn[d]);
                double dx = y[d] - g.xc[d][i0[d] + bd + 3];
                r2 += dx * dx;
            }
            uint8_t t = ib.cls[((long long)ci[2] * g.nj + ci[1]) * g.ni + ci[0]];
            if (t != IBM_FLUID && t != IBM_FORCING)
                continue;
            nvalid++;
            if (r2 == 0.0 && zero < 0)
                zero = m;
            w[m] = r2 > 0.0 ? 1.0 / r2 : 0.0;
        }
        double pp = 0.0, gr[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        if (!ok || nvalid == 0) {
            atomicAdd(missed, 1);
            area = 0.0;
        } else {
            if (zero >= 0)
                for (int m = 0; m < NC; ++m)
                    w[m] = m == zero ? 1.0 : 0.0;
            double wsum = 0.0;
            for (int m = 0; m < NC; ++m)
                wsum += w[m];
            for (int m = 0; m < NC; ++m) {
                if (w[m] == 0.0)
                    continue;
                double wm = w[m] / wsum;
                int ci[3] = {0, 0, 0};
                for (int d = 0; d < DIM; ++d)
                    ci[d] = wrap_cell(i0[d] + ((m >> d) & 1), nn[d]);
                pp += wm * pressure_pert<DIM>(g, f, q, state_index(g, ci[0], ci[1], ci[2]));
                for (int d = 0; d < DIM; ++d) {
                    int cp[3] = {ci[0], ci[1], ci[2]}, cm[3] = {ci[0], ci[1], ci[2]};
                    cp[d] += 1;
                    cm[d] -= 1;
                    double up[3], um[3];
                    velocity<DIM>(g, f, q, state_index(g, cp[0], cp[1], cp[2]), up);
                    velocity<DIM>(g, f, q, state_index(g, cm[0], cm[1], cm[2]), um);
                    double dxd = g.xc[d][ci[d] + 4] - g.xc[d][ci[d] + 2];
                    for (int i = 0; i < DIM; ++i)
                        gr[i][d] += wm * (up[i] - um[i]) / dxd;
                }
            }
        }
        double div = 0.0;
        for (int d = 0; d < DIM; ++d)
            div += gr[d][d];
        double tn[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < DIM; ++i)
            for (int j = 0; j < DIM; ++j) {
                double tau = f.mu * (gr[i][j] + gr[j][i] - (i == j ? 2.0 / 3.0 * div : 0.0));
                tn[i] += tau * n[j];
            }
        for (int i = 0; i < DIM; ++i)
            Fc[i] = area * (-pp * n[i] + tn[i]);
        if (facet_out) {
            double *fo = facet_out + 5 * (long long)fid;
            fo[0] = pp;
            fo[1] = tn[0];
            fo[2] = tn[1];
            fo[3] = tn[2];
            fo[4] = area;
        }
    }
    for (int i = 0; i < 3; ++i)
        red[i][threadIdx.x] = Fc[i];
    __syncthreads();
    for (int s = kForceBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int i = 0; i < 3; ++i)
                red[i][threadIdx.x] += red[i][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3)
        part[3 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// sum of the block sums, in a fixed order
__global__ __launch_bounds__(kForceBlock) void forces_sum_kernel(const double *part, int nblk, double *out)
{
    __shared__ double red[3][kForceBlock];
    double s[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nblk; k += kForceBlock)
        for (int i = 0; i < 3; ++i)
            s[i] += part[3 * k + i];
    for (int i = 0; i < 3; ++i)
        red[i][threadIdx.x] = s[i];
    __syncthreads();
    for (int st = kForceBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int i = 0; i < 3; ++i)
                red[i][threadIdx.x] += red[i][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 3)
        out[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace

int forces_blocks(int nfacet) { return (nfacet + kForceBlock - 1) / kForceBlock; }

hipError_t forces_static_scratch(int device, double **part, int32_t **missed)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[device]) {
        // resolved once per device, with that device current (the caller's)
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        scratch_ptr[device] = static_cast<double *>(p);
    }
    *part = scratch_ptr[device];
    *missed = reinterpret_cast<int32_t *>(scratch_ptr[device] + 3 * kStaticForceBlocks);
    return hipSuccess;
}

hipError_t launch_zero_i32(int32_t *p, hipStream_t s)
{
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_forces(const Grid &g, const Body &b, const Flow &f, const IB &ib, const double *q, double *force,
                         double *facet_out, double *part, int32_t *missed, hipStream_t s)
{
    int nblk = forces_blocks(b.nfacet);
    if (nblk == 0)
        return hipErrorInvalidValue;
    if (g.ndim == 2)
        hipLaunchKernelGGL(forces_kernel<2>, dim3(nblk), dim3(kForceBlock), 0, s, g, b, f, ib, q, facet_out, part,
                           missed);
    else
        hipLaunchKernelGGL(forces_kernel<3>, dim3(nblk), dim3(kForceBlock), 0, s, g, b, f, ib, q, facet_out, part,
                           missed);
    hipLaunchKernelGGL(forces_sum_kernel, dim3(1), dim3(kForceBlock), 0, s, part, nblk, force);
    return hipGetLastError();
}

}  // namespace ibm
