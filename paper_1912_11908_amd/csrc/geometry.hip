// Immersed-boundary geometry kernels for gfx950: body pose, ray-parity
// classification, forcing/ghost tagging, list compaction and the per-node
// reconstruction records (Seshadri & De, sections 3-4).
//
// Built with -ffp-contract=off: every floating-point decision taken here
// (closest feature, boundary point, probe validity) must be reproducible
// bit for bit, so no multiply-add is fused behind the source's back.
#include "common.h"

namespace ibm {
namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;

__device__ inline int cell_index(const Grid &g, int i, int j, int k)
{
    return (k * g.nj + j) * g.ni + i;
}

// ------------------------------------------------------------------ pose
// a1: translate the lattice body by an integer displacement along one axis;
// the floating coordinates are the exact lattice values.
__global__ void pose_kernel(int n, int ndim, const long long *V0, long long *V, double *v,
                            long long disp, int axis)
{
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n * ndim)
        return;
    long long x = V0[m] + ((m % ndim) == axis ? disp : 0);
    V[m] = x;
    v[m] = (double)x / kLatScale;
}

// ---------------------------------------------------------- classification
__global__ void clear_kernel(uint8_t *inside, int ncell, uint32_t *toggle, int nwords)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ncell)
        inside[t] = 0;
    if (t < nwords)
        toggle[t] = 0u;
}

// first index in [lo, hi) with X[idx] >= key (X increasing); hi if none
__device__ inline int lower_bound_ll(const long long *X, int lo, int hi, long long key)
{
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (X[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Section 3.2 ray casting, +x rays, exact lattice predicates.  A segment
// a->b crosses the ray of node p iff (a_y > p_y) != (b_y > p_y) and the
// crossing lies strictly right of p.  Rows crossed are those with
// min(a_y, b_y) <= Y_j < max(a_y, b_y); in each, the crossed nodes form a
// prefix of the row, found by binary search; one bit toggles at its end.
__global__ void cross2d_kernel(Grid g, Body b, IB ib)
{
    // one wavefront per facet, lanes over the crossed rows
    int f = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    int lane = threadIdx.x & (kWave - 1);
    if (f >= b.nfacet)
        return;
    const long long *A = b.V + 2 * b.facet[2 * f];
    const long long *B = b.V + 2 * b.facet[2 * f + 1];
    if (A[1] == B[1])
        return;  // horizontal: never satisfies the half-open rule
    long long ylo = A[1] < B[1] ? A[1] : B[1];
    long long yhi = A[1] < B[1] ? B[1] : A[1];
    const long long *Y = g.Xc[1];
    const long long *X = g.Xc[0];
    int j0 = lower_bound_ll(Y, ib.region[2], ib.region[3], ylo);
    int j1 = lower_bound_ll(Y, ib.region[2], ib.region[3], yhi);
    long long dxab = B[0] - A[0], dyab = B[1] - A[1];
    for (int j = j0 + lane; j < j1; j += kWave) {
        long long py = Y[j];
        // crossing strictly right of px <=> orient * sign(dy) > 0, which is
        // true on a prefix of the row
        int lo = ib.region[0], hi = ib.region[1];
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            long long o = dxab * (py - A[1]) - dyab * (X[mid] - A[0]);
            bool right = dyab > 0 ? o > 0 : o < 0;
            if (right)
                lo = mid + 1;
            else
                hi = mid;
        }
        int pos = lo - ib.region[0];
        int row = j - ib.region[2];
        atomicXor(&ib.toggle[row * ib.words_per_row + (pos >> 5)], 1u << (pos & 31));
    }
}

__device__ inline bool edge_owns(long long dy, long long dz) { return (dz == 0 && dy < 0) || dz > 0; }

// 3D: a triangle counts for node (py, pz) iff the point lies in its (y, z)
// projection (top-left tie rule; triangles parallel to the ray skipped) and
// the crossing lies strictly ahead in +x (exact 128-bit arithmetic).
__global__ void cross3d_kernel(Grid g, Body b, IB ib)
{
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= b.nfacet)
        return;
    const int *t = b.facet + 3 * f;
    const long long *P[3] = {b.V + 3 * t[0], b.V + 3 * t[1], b.V + 3 * t[2]};
    long long area = (P[1][1] - P[0][1]) * (P[2][2] - P[0][2]) - (P[1][2] - P[0][2]) * (P[2][1] - P[0][1]);
    if (area == 0)
        return;
    if (area < 0) {
        const long long *tmp = P[1];
        P[1] = P[2];
        P[2] = tmp;
    }
    long long ylo = P[0][1], yhi = P[0][1], zlo = P[0][2], zhi = P[0][2];
    for (int m = 1; m < 3; ++m) {
        ylo = P[m][1] < ylo ? P[m][1] : ylo;
        yhi = P[m][1] > yhi ? P[m][1] : yhi;
        zlo = P[m][2] < zlo ? P[m][2] : zlo;
        zhi = P[m][2] > zhi ? P[m][2] : zhi;
    }
    const long long *X = g.Xc[0], *Y = g.Xc[1], *Z = g.Xc[2];
    int j0 = lower_bound_ll(Y, ib.region[2], ib.region[3], ylo);
    int j1 = lower_bound_ll(Y, ib.region[2], ib.region[3], yhi + 1);
    int k0 = lower_bound_ll(Z, ib.region[4], ib.region[5], zlo);
    int k1 = lower_bound_ll(Z, ib.region[4], ib.region[5], zhi + 1);
    for (int k = k0; k < k1; ++k)
        for (int j = j0; j < j1; ++j) {
            long long py = Y[j], pz = Z[k];
            long long w[3];
            bool ok = true;
            for (int m = 0; m < 3; ++m) {
                const long long *p = P[m], *q = P[(m + 1) % 3];
                long long dy = q[1] - p[1], dz = q[2] - p[2];
                w[m] = dy * (pz - p[2]) - dz * (py - p[1]);
                if (w[m] < 0 || (w[m] == 0 && !edge_owns(dy, dz)))
                    ok = false;
            }
            if (!ok)
                continue;
            // crossing ahead of px <=> sum_m w[m] (x_opp(m) - px) > 0; the
            // sum decreases with px, so crossed nodes form a row prefix
            __int128 base = 0, wsum = 0;
            for (int m = 0; m < 3; ++m) {
                base += (__int128)w[m] * (__int128)P[(m + 2) % 3][0];
                wsum += (__int128)w[m];
            }
            int lo = ib.region[0], hi = ib.region[1];
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                __int128 s = base - wsum * (__int128)X[mid];
                if (s > 0)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            int pos = lo - ib.region[0];
            int row = (k - ib.region[4]) * ib.rh + (j - ib.region[2]);
            atomicXor(&ib.toggle[row * ib.words_per_row + (pos >> 5)], 1u << (pos & 31));
        }
}

// One wavefront per region row: a node is inside iff an odd number of
// toggles sit at positions above it.  Suffix parity over words with a
// wavefront ballot, processed from the high end in chunks of 64 words.
__global__ void parity_kernel(IB ib, int nrows)
{
    int lane = threadIdx.x & (kWave - 1);
    int row = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (row >= nrows)
        return;
    const uint32_t *T = ib.toggle + (long long)row * ib.words_per_row;
    uint8_t *out = ib.inside + (long long)row * ib.rw;
    int nw = ib.words_per_row;
    int carry = 0;
    for (int top = nw; top > 0; top -= kWave) {
        int w = top - kWave + lane;  // this lane's word
        uint32_t word = (w >= 0) ? T[w] : 0u;
        int pw = __popc(word) & 1;
        unsigned long long mask = __ballot(pw);
        // parity of the words strictly above w within this chunk
        unsigned long long above = lane == kWave - 1 ? 0ull : (mask >> (lane + 1));
        int suffix = (__popcll(above) + carry) & 1;
        if (w >= 0) {
            for (int bit = 0; bit < 32; ++bit) {
                int pos = 32 * w + bit;
                if (pos >= ib.rw)
                    break;
                unsigned long long higher = (unsigned long long)word >> (bit + 1);
                out[pos] = (uint8_t)((__popcll(higher) + suffix) & 1);
            }
        }
        carry = (carry + __popcll(mask)) & 1;
    }
}

// a3 tagging.  Outside the region every cell is fluid.  FORCING: a fluid
// cell with an inside face neighbour.  Inside cells take the face-graph
// distance to the nearest fluid cell: 1, 2, 3 -> G1, G2, G3, more -> SOLID
// (the BFS layers of successive face neighbours).  Periodic axes wrap;
// cells beyond other domain boundaries do not exist.
__device__ inline bool nb_coord(const Grid &g, int axis, int c, int &out)
{
    int n = axis == 0 ? g.ni : axis == 1 ? g.nj : g.nk;
    if (c >= 0 && c < n) {
        out = c;
        return true;
    }
    if (g.bc[2 * axis] != IBM_BC_PERIODIC)
        return false;
    out = ((c % n) + n) % n;
    return true;
}

__device__ inline int inside_at(const IB &ib, int i, int j, int k)
{
    if (i < ib.region[0] || i >= ib.region[1] || j < ib.region[2] || j >= ib.region[3] ||
        k < ib.region[4] || k >= ib.region[5])
        return 0;
    return ib.inside[((k - ib.region[4]) * ib.rh + (j - ib.region[2])) * ib.rw + (i - ib.region[0])];
}

// Is any cell at face-graph distance DIST (the offsets with |a|+|b|+|c| =
// DIST) a fluid cell?  Every axis has at least four cells (checked when a
// solve is created), so one shift by n wraps an offset of up to three.  The
// shell's indices are formed first (a cell beyond a non-periodic side, or
// outside the region, reads region cell 0 and is masked), then all its
// flags are loaded at once.
template <int ND, int DIST>
__device__ inline bool shell_has_fluid(const Grid &g, const IB &ib, int i, int j, int k)
{
    constexpr int RZ = ND == 3 ? DIST : 0;
    constexpr int N = ND == 3 ? 4 * DIST * DIST + 2 : 4 * DIST;
    const int n3[3] = {g.ni, g.nj, g.nk};
    const bool per[3] = {g.bc[0] == IBM_BC_PERIODIC, g.bc[2] == IBM_BC_PERIODIC, g.bc[4] == IBM_BC_PERIODIC};
    const int c0[3] = {i, j, k};
    int idx[N];
    unsigned long long valid = 0;
    int e = 0;
#pragma unroll
    for (int c = -RZ; c <= RZ; ++c) {
        const int rb = DIST - (c < 0 ? -c : c);
#pragma unroll
        for (int b2 = -rb; b2 <= rb; ++b2) {
            const int ra = rb - (b2 < 0 ? -b2 : b2);
#pragma unroll
            for (int sgn = 0; sgn < 2; ++sgn) {
                if (sgn == 1 && ra == 0)
                    continue;
                const int off[3] = {sgn == 0 ? -ra : ra, b2, c};
                bool ok = true;
                int l[3];
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    int x = c0[d] + off[d];
                    bool in = x >= 0 && x < n3[d];
                    ok = ok && (in || per[d]);
                    x += x < 0 ? n3[d] : 0;
                    x -= x >= n3[d] ? n3[d] : 0;
                    l[d] = x - ib.region[2 * d];
                }
                if (ND == 2)
                    l[2] = k - ib.region[4];
                bool inreg = (unsigned)l[0] < (unsigned)ib.rw && (unsigned)l[1] < (unsigned)ib.rh &&
                             (unsigned)l[2] < (unsigned)ib.rd;
                // valid bit: the cell exists; idx: its region cell, or 0 (a
                // cell outside the region is fluid: masked below)
                idx[e] = ok && inreg ? (l[2] * ib.rh + l[1]) * ib.rw + l[0] : -1;
                valid |= (unsigned long long)ok << e;
                ++e;
            }
        }
    }
    uint8_t fl[N];
#pragma unroll
    for (int m = 0; m < N; ++m)
        fl[m] = ib.inside[idx[m] >= 0 ? idx[m] : 0];
    bool hit = false;
#pragma unroll
    for (int m = 0; m < N; ++m)
        hit = hit | (((valid >> m) & 1ull) != 0 && (idx[m] < 0 || fl[m] == 0));
    return hit;
}

template <int ND> __device__ inline int fluid_distance(const Grid &g, const IB &ib, int i, int j, int k)
{
    if (shell_has_fluid<ND, 1>(g, ib, i, j, k))
        return 1;
    if (shell_has_fluid<ND, 2>(g, ib, i, j, k))
        return 2;
    if (shell_has_fluid<ND, 3>(g, ib, i, j, k))
        return 3;
    return 4;
}

__global__ void tag_kernel(Grid g, IB ib)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int n = ib.rw * ib.rh * ib.rd;
    if (t >= n)
        return;
    int li = t % ib.rw, lj = (t / ib.rw) % ib.rh, lk = t / (ib.rw * ib.rh);
    int i = li + ib.region[0], j = lj + ib.region[2], k = lk + ib.region[4];
    int nd = g.ndim;
    uint8_t cls;
    if (!ib.inside[t]) {
        cls = IBM_FLUID;
        for (int d = 0; d < nd; ++d)
            for (int s = -1; s <= 1; s += 2) {
                int c[3] = {i, j, k}, o;
                if (!nb_coord(g, d, c[d] + s, o))
                    continue;
                c[d] = o;
                if (inside_at(ib, c[0], c[1], c[2]))
                    cls = IBM_FORCING;
            }
    } else {
        // the shells of face-graph distance 1, then 2, then 3, stopping at
        // the first that holds a fluid cell
        int best = nd == 3 ? fluid_distance<3>(g, ib, i, j, k) : fluid_distance<2>(g, ib, i, j, k);
        cls = best == 1 ? IBM_G1 : best == 2 ? IBM_G2 : best == 3 ? IBM_G3 : IBM_SOLID;
    }
    ib.cls[cell_index(g, i, j, k)] = cls;
}

// --------------------------------------------------------- compaction
__device__ inline int region_cell(const Grid &g, const IB &ib, int t)
{
    int li = t % ib.rw, lj = (t / ib.rw) % ib.rh, lk = t / (ib.rw * ib.rh);
    return cell_index(g, li + ib.region[0], lj + ib.region[2], lk + ib.region[4]);
}

__global__ void zero_counts_kernel(int32_t *counts)
{
    if (threadIdx.x < CNT_WORDS && threadIdx.x != CNT_STATUS)
        counts[threadIdx.x] = 0;
}

// per-block counts of FORCING, ghost (G1-G3), G1, G2 and G3 cells
__global__ __launch_bounds__(kBlock) void count_kernel(Grid g, IB ib)
{
    __shared__ int sc[5][kBlock / kWave];
    int n = ib.rw * ib.rh * ib.rd;
    int t = blockIdx.x * kBlock + threadIdx.x;
    uint8_t c = t < n ? ib.cls[region_cell(g, ib, t)] : (uint8_t)IBM_SOLID;
    bool f = c == IBM_FORCING, gh = c >= IBM_G1 && c <= IBM_G3;
    int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    int cnt[5] = {(int)__popcll(__ballot(f)), (int)__popcll(__ballot(gh)), (int)__popcll(__ballot(c == IBM_G1)),
                  (int)__popcll(__ballot(c == IBM_G2)), (int)__popcll(__ballot(c == IBM_G3))};
    if (lane == 0)
        for (int l = 0; l < 5; ++l)
            sc[l][w] = cnt[l];
    __syncthreads();
    if (threadIdx.x < 5) {
        int a = 0;
        for (int m = 0; m < kBlock / kWave; ++m)
            a += sc[threadIdx.x][m];
        ib.blk[threadIdx.x * ib.nblk + blockIdx.x] = a;
    }
}

// single block: exclusive scan of the per-block counts of both lists (in
// place), the list sizes and the G1-G3 totals into the count words.  Thread
// t sums a run of `per` blocks; the 1024 run sums of a list are scanned
// across each wavefront (shuffles), then across the 16 wavefront totals.
__global__ __launch_bounds__(1024) void scan_kernel(IB ib)
{
    constexpr int NW = 1024 / kWave;
    __shared__ int wsum[5][NW];
    int nb = ib.nblk;
    int per = (nb + 1023) / 1024;
    int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    int run[2];  // exclusive scan of the run sums within the wavefront
    for (int l = 0; l < 5; ++l) {
        const int *a = ib.blk + l * nb;
        int s = 0;
        for (int m = 0; m < per; ++m) {
            int idx = t * per + m;
            if (idx < nb)
                s += a[idx];
        }
        int incl = s;
        for (int o = 1; o < kWave; o <<= 1) {
            int v = __shfl_up(incl, o, kWave);
            if (lane >= o)
                incl += v;
        }
        if (l < 2)
            run[l] = incl - s;
        if (lane == kWave - 1)
            wsum[l][w] = incl;
    }
    __syncthreads();
    int offs[2] = {0, 0};
    for (int l = 0; l < 2; ++l)
        for (int m = 0; m < w; ++m)
            offs[l] += wsum[l][m];
    if (t < 5) {
        int all = 0;
        for (int m = 0; m < NW; ++m)
            all += wsum[t][m];
        const int word[5] = {CNT_F, CNT_G, CNT_G1, CNT_G2, CNT_G3};
        ib.counts[word[t]] = all;
        if (t < 2 && all > ib.cap)
            raise_status(ib, ib.counts, ST_CAPACITY);
    }
    for (int l = 0; l < 2; ++l) {
        int *a = ib.blk + l * nb;
        int r = offs[l] + run[l];
        for (int m = 0; m < per; ++m) {
            int idx = t * per + m;
            if (idx < nb) {
                int v = a[idx];
                a[idx] = r;
                r += v;
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void write_lists_kernel(Grid g, IB ib)
{
    __shared__ int sF[kBlock / kWave], sG[kBlock / kWave];
    int n = ib.rw * ib.rh * ib.rd;
    int t = blockIdx.x * kBlock + threadIdx.x;
    int cell = t < n ? region_cell(g, ib, t) : 0;
    uint8_t c = t < n ? ib.cls[cell] : (uint8_t)IBM_SOLID;
    bool f = c == IBM_FORCING, gh = c >= IBM_G1 && c <= IBM_G3;
    unsigned long long bf = __ballot(f), bg = __ballot(gh);
    int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    unsigned long long lower = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    if (lane == 0) {
        sF[w] = __popcll(bf);
        sG[w] = __popcll(bg);
    }
    __syncthreads();
    int offF = ib.blk[blockIdx.x], offG = ib.blk[ib.nblk + blockIdx.x];
    for (int m = 0; m < w; ++m) {
        offF += sF[m];
        offG += sG[m];
    }
    // record index per IB node: forcing records first, then the ghosts
    // (-1 beyond the capacity, which the scan has flagged)
    int nF = min(ib.counts[CNT_F], ib.cap);
    if (f) {
        int pos = offF + __popcll(bf & lower);
        if (pos < ib.cap)
            ib.listF[pos] = cell;
        ib.rmap[t] = pos < ib.cap ? pos : -1;
    }
    if (gh) {
        int pos = offG + __popcll(bg & lower);
        if (pos < ib.cap)
            ib.listG[pos] = cell;
        ib.rmap[t] = nF + pos < ib.cap ? nF + pos : -1;
    }
}

// ------------------------------------------------------ records (a4)
struct Closest {
    int kind, id, facet;
    double c[3], d2;
};
enum { FEAT_FACE = 0, FEAT_VERTEX = 1, FEAT_EDGE = 2 };

__device__ inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__device__ inline void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Section 4.1: minimum of the squared distance of eq.1 over all facets;
// the lowest facet id wins exact ties.  2D: clamped segment parameter.
// Lexicographic minimum of (d2, facet) over the wavefront: every lane
// returns the winning lane's candidate.
__device__ inline Closest wave_min(const Closest &c)
{
    double d = c.d2;
    for (int o = kWave / 2; o >= 1; o >>= 1) {
        double t = __shfl_xor(d, o, kWave);
        d = t < d ? t : d;
    }
    int f = c.d2 == d ? c.facet : 0x7fffffff;
    for (int o = kWave / 2; o >= 1; o >>= 1) {
        int t = __shfl_xor(f, o, kWave);
        f = t < f ? t : f;
    }
    unsigned long long m = __ballot(c.d2 == d && c.facet == f);
    int src = __ffsll((long long)m) - 1;
    Closest r;
    r.kind = __shfl(c.kind, src, kWave);
    r.id = __shfl(c.id, src, kWave);
    r.facet = __shfl(c.facet, src, kWave);
    r.d2 = __shfl(c.d2, src, kWave);
    for (int k = 0; k < 3; ++k)
        r.c[k] = __shfl(c.c[k], src, kWave);
    return r;
}

// smallest non-negative value over the wavefront (-1 if none)
__device__ inline double wave_min_hit(double sig)
{
    double d = sig < 0.0 ? __builtin_inf() : sig;
    for (int o = kWave / 2; o >= 1; o >>= 1) {
        double t = __shfl_xor(d, o, kWave);
        d = t < d ? t : d;
    }
    return d == __builtin_inf() ? -1.0 : d;
}

__device__ inline void keep(Closest &best, const Closest &cur)
{
    if (cur.d2 < best.d2 || (cur.d2 == best.d2 && cur.facet < best.facet))
        best = cur;
}

// 2D: closest point of each segment (vertex or interior); the minimum over
// all segments, lowest segment id among equals.  Called by a whole
// wavefront for one node: lanes split the segments.
__device__ Closest closest2d(const Body &b, const double *p, int lane)
{
    Closest best;
    best.d2 = __builtin_inf();
    best.kind = best.id = best.facet = -1;
    best.c[0] = best.c[1] = best.c[2] = 0.0;
    for (int f = lane; f < b.nfacet; f += kWave) {
        int ia = b.facet[2 * f], ibv = b.facet[2 * f + 1];
        const double *a = b.v + 2 * ia, *q = b.v + 2 * ibv;
        double ex = q[0] - a[0], ey = q[1] - a[1];
        double t = ((p[0] - a[0]) * ex + (p[1] - a[1]) * ey) / (ex * ex + ey * ey);
        Closest cur;
        cur.c[2] = 0.0;
        if (t <= 0.0) {
            cur.c[0] = a[0]; cur.c[1] = a[1]; cur.kind = FEAT_VERTEX; cur.id = ia;
        } else if (t >= 1.0) {
            cur.c[0] = q[0]; cur.c[1] = q[1]; cur.kind = FEAT_VERTEX; cur.id = ibv;
        } else {
            cur.c[0] = a[0] + t * ex; cur.c[1] = a[1] + t * ey; cur.kind = FEAT_FACE; cur.id = f;
        }
        double dx = p[0] - cur.c[0], dy = p[1] - cur.c[1];
        cur.d2 = dx * dx + dy * dy;
        cur.facet = f;
        keep(best, cur);
    }
    return wave_min(best);
}

__device__ inline void seg_closest(const double *p, const double *a, const double *q, double &t,
                                   double *c, double &d2)
{
    double e[3] = {q[0] - a[0], q[1] - a[1], q[2] - a[2]};
    double w[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    t = dot3(w, e) / dot3(e, e);
    if (t <= 0.0) {
        t = 0.0;
        c[0] = a[0]; c[1] = a[1]; c[2] = a[2];
    } else if (t >= 1.0) {
        t = 1.0;
        c[0] = q[0]; c[1] = q[1]; c[2] = q[2];
    } else {
        c[0] = a[0] + t * e[0];
        c[1] = a[1] + t * e[1];
        c[2] = a[2] + t * e[2];
    }
    double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
    d2 = dx * dx + dy * dy + dz * dz;
}

// 3D: interior stationary point of eq.1 (face region) when feasible,
// otherwise the best of the three edge minimisers (edge or vertex regions).
__device__ inline Closest facet_closest(const Body &b, const double *p, int f)
{
    const int *tv = b.facet + 3 * f;
    const double *A = b.v + 3 * tv[0], *B = b.v + 3 * tv[1], *C = b.v + 3 * tv[2];
    double e0[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double e1[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    double dd[3] = {A[0] - p[0], A[1] - p[1], A[2] - p[2]};
    double a = dot3(e0, e0), bb = dot3(e0, e1), c = dot3(e1, e1);
    double d = dot3(e0, dd), e = dot3(e1, dd);
    double det = a * c - bb * bb;
    double s = bb * e - c * d, t = bb * d - a * e;
    Closest cur;
    cur.kind = cur.id = -1;
    cur.facet = f;
    if (s > 0.0 && t > 0.0 && s + t < det) {
        s /= det;
        t /= det;
        cur.kind = FEAT_FACE;
        cur.id = f;
        for (int m = 0; m < 3; ++m)
            cur.c[m] = A[m] + s * e0[m] + t * e1[m];
        double dx = p[0] - cur.c[0], dy = p[1] - cur.c[1], dz = p[2] - cur.c[2];
        cur.d2 = dx * dx + dy * dy + dz * dz;
    } else {
        cur.d2 = __builtin_inf();
        for (int m = 0; m < 3; ++m) {
            const double *pa = b.v + 3 * tv[m], *pb = b.v + 3 * tv[(m + 1) % 3];
            double tt, cc[3], d2;
            seg_closest(p, pa, pb, tt, cc, d2);
            if (d2 < cur.d2) {
                cur.d2 = d2;
                cur.c[0] = cc[0]; cur.c[1] = cc[1]; cur.c[2] = cc[2];
                if (tt == 0.0) {
                    cur.kind = FEAT_VERTEX;
                    cur.id = tv[m];
                } else if (tt == 1.0) {
                    cur.kind = FEAT_VERTEX;
                    cur.id = tv[(m + 1) % 3];
                } else {
                    cur.kind = FEAT_EDGE;
                    cur.id = b.edge_of[3 * f + m];
                }
            }
        }
    }
    return cur;
}

// bin index of rest-frame coordinate y along axis d (may lie outside the grid)
__device__ inline int bin_of(const Body &b, int d, double y) { return (int)floor((y - b.bin_o[d]) / b.bin_h); }

// Visits the facets listed in the bins of the box lo..lo+ext-1 (clipped to
// the bin grid; with shell >= 0 only the bins on the surface of the cube of
// half-width shell around lo + shell), spread over the whole wavefront:
// lane l reads the range of the box's bin l of each group of 64, a prefix
// sum over the lanes numbers the group's entries, and every lane takes
// every 64th entry, finding its bin in the sums in LDS by walking forward
// from the bin of its previous entry (the sums grow with the entry).  With
// PAIR the lane takes two entries 64 apart per round and hands their
// listing indices to visit(la, lb) (lb = -1 past the end), which can then
// issue the loads of both at once; otherwise visit(facet).  A facet listed
// in several bins is visited once per listing.
// With a finite cut2 (the same on every lane), a bin whose box lies farther
// from the point y than sqrt(cut2) (by more than a margin far above
// rounding) is skipped: a facet listed there that came closer than that
// would also be listed in a bin that does not lie that far.
// Wavefront-uniform control flow; `nb` (the sums) and `st` (the bin
// starts) are this wavefront's 64-entry LDS slices.
template <bool PAIR = false, typename Visit>
__device__ inline void visit_bins(const Body &b, const int *lo, const int *ext, int shell, int lane, int *nb,
                                  int *st, const double *y, double cut2, Visit &&visit)
{
    int nbox = ext[0] * ext[1] * ext[2];
    for (int base = 0; base < nbox; base += kWave) {
        int e = base + lane, s = 0, n = 0;
        if (e < nbox) {
            int ex = e % ext[0], ey = (e / ext[0]) % ext[1], ez = e / (ext[0] * ext[1]);
            bool on = shell < 0 || max(abs(ex - shell), max(abs(ey - shell), abs(ez - shell))) == shell;
            int kx = lo[0] + ex, ky = lo[1] + ey, kz = lo[2] + ez;
            if (on && kx >= 0 && kx < b.bin_n[0] && ky >= 0 && ky < b.bin_n[1] && kz >= 0 && kz < b.bin_n[2]) {
                int k3[3] = {kx, ky, kz};
                double bd2 = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double c0 = b.bin_o[d] + k3[d] * b.bin_h, c1 = c0 + b.bin_h;
                    double u = fmax(fmax(c0 - y[d], y[d] - c1), 0.0);
                    bd2 += u * u;
                }
                bool far = false;
                if (bd2 > cut2) {
                    double lb = sqrt(bd2) - 1e-9 * b.bin_h;
                    far = lb > 0.0 && lb * lb > cut2;
                }
                if (!far) {
                    int bin = (kz * b.bin_n[1] + ky) * b.bin_n[0] + kx;
                    s = b.bin_start[bin];
                    n = b.bin_start[bin + 1] - s;
                }
            }
        }
        int incl = n;
        for (int o = 1; o < kWave; o <<= 1) {
            int t = __shfl_up(incl, o, kWave);
            if (lane >= o)
                incl += t;
        }
        int total = __shfl(incl, kWave - 1, kWave);
        if (total == 0)
            continue;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        nb[lane] = incl;
        st[lane] = s - (incl - n);  // entry of item t of this bin: st + t
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // l0: the first lane whose sum exceeds the entry (nb[63] = total
        // bounds every walk)
        int l0 = 0;
        if constexpr (PAIR) {
            for (int t = lane; t < total; t += 2 * kWave) {
                while (nb[l0] <= t)
                    ++l0;
                int la = st[l0] + t, lb = -1;
                int t2 = t + kWave;
                if (t2 < total) {
                    while (nb[l0] <= t2)
                        ++l0;
                    lb = st[l0] + t2;
                }
                visit(la, lb);
            }
        } else {
            for (int t = lane; t < total; t += kWave) {
                while (nb[l0] <= t)
                    ++l0;
                visit(b.bin_facet[st[l0] + t]);
            }
        }
    }
}

// squared distance from rest-frame point y to the box bx = (lo, hi)
__device__ inline double box_dist2v(const float *bx, const double *y)
{
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        double u = fmax(fmax(bx[d] - y[d], y[d] - bx[3 + d]), 0.0);
        s += u * u;
    }
    return s;
}

// The brute-force minimum over all facets, smallest squared distance first
// and the lowest facet id among equals.  With bins, cubic shells of bins
// around the node's bin are searched outwards.  A facet not listed in any
// bin of the shells up to K lies outside their cube, so it is no closer
// than the node's distance r to the cube's surface: once the minimum so far
// is below r (less a margin far above rounding) the search stops with the
// brute-force result.  Within a shell a facet whose bounding box is farther
// than the lane's minimum so far (by the same margin) cannot win or tie and
// is skipped.  Called by a whole wavefront for one node: lanes split the
// facets of each shell, and every shell ends on the wavefront's minimum.
// A valid facet id `hint` (the previous search's answer from the same cell)
// is measured first: its distance bounds the minimum from above, so the
// bins and facets farther than it are skipped from the first shell on; the
// result is the same for any hint.
__device__ Closest closest3d(const Body &b, const double *p, int lane, int *nb, int *st, int hint)
{
    Closest best;
    best.d2 = __builtin_inf();
    best.kind = best.id = best.facet = -1;
    best.c[0] = best.c[1] = best.c[2] = 0.0;
    if (b.nbin == 0) {
        for (int f = lane; f < b.nfacet; f += kWave)
            keep(best, facet_closest(b, p, f));
        return wave_min(best);
    }
    if (hint >= 0 && hint < b.nfacet)
        keep(best, facet_closest(b, p, hint));
    double y[3];
    int ic[3], far = 0;
    for (int d = 0; d < 3; ++d) {
        y[d] = p[d] - b.disp[d];
        ic[d] = bin_of(b, d, y[d]);
        far = max(far, max(ic[d], b.bin_n[d] - 1 - ic[d]));
    }
    double margin = 1e-9 * b.bin_h;
    for (int K = 0; K <= far; ++K) {
        int lo[3] = {ic[0] - K, ic[1] - K, ic[2] - K}, ext[3] = {2 * K + 1, 2 * K + 1, 2 * K + 1};
        double cut2 = best.d2;  // the wavefront's minimum after the inner shells
        visit_bins<true>(b, lo, ext, K, lane, nb, st, y, cut2, [&](int la, int lb) {
            // both listings' facets and boxes in flight before either test
            bool two = lb >= 0;
            lb = two ? lb : la;
            int fa = b.bin_facet[la], fb = b.bin_facet[lb];
            const float *ba = b.bin_box + 6 * (long long)la, *bb = b.bin_box + 6 * (long long)lb;
            float xa[6], xb[6];
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                xa[m] = ba[m];
                xb[m] = bb[m];
            }
            auto test = [&](int f, const float *bx) {
                double bd2 = box_dist2v(bx, y);
                if (bd2 > best.d2) {
                    double lb = sqrt(bd2) - margin;
                    if (lb > 0.0 && lb * lb > best.d2)
                        return;
                }
                keep(best, facet_closest(b, p, f));
            };
            test(fa, xa);
            if (two)
                test(fb, xb);
        });
        best = wave_min(best);
        double r = __builtin_inf();
        for (int d = 0; d < 3; ++d) {
            double c0 = b.bin_o[d] + (ic[d] - K) * b.bin_h, c1 = b.bin_o[d] + (ic[d] + K + 1) * b.bin_h;
            r = fmin(r, fmin(y[d] - c0, c1 - y[d]));
        }
        r -= margin;
        if (r > 0.0 && best.d2 < r * r)
            break;
    }
    return best;
}

__device__ double line_hit2d(const Body &b, const double *x, const double *dir, double smax, int lane)
{
    double best = -1.0;
    for (int f = lane; f < b.nfacet; f += kWave) {
        const double *a = b.v + 2 * b.facet[2 * f], *q = b.v + 2 * b.facet[2 * f + 1];
        double ex = q[0] - a[0], ey = q[1] - a[1];
        double den = dir[0] * ey - dir[1] * ex;
        if (den == 0.0)
            continue;
        double ax = a[0] - x[0], ay = a[1] - x[1];
        double sig = (ax * ey - ay * ex) / den;
        double tau = (ax * dir[1] - ay * dir[0]) / den;
        if (tau < 0.0 || tau > 1.0 || sig < 0.0 || sig > smax)
            continue;
        if (best < 0.0 || sig < best)
            best = sig;
    }
    return wave_min_hit(best);
}

// Moller-Trumbore line/triangle intersection (section 3.2)
// Moller-Trumbore: parameter sig in [0, smax] where x + sig dir meets facet
// f, or -1
__device__ inline double facet_hit(const Body &b, const double *x, const double *dir, double smax, int f)
{
    const int *tv = b.facet + 3 * f;
    const double *A = b.v + 3 * tv[0], *B = b.v + 3 * tv[1], *C = b.v + 3 * tv[2];
    double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    double pv[3];
    cross3(dir, e2, pv);
    double det = dot3(e1, pv);
    if (det == 0.0)
        return -1.0;
    double tv_[3] = {x[0] - A[0], x[1] - A[1], x[2] - A[2]};
    double u = dot3(tv_, pv) / det;
    if (u < 0.0 || u > 1.0)
        return -1.0;
    double qv[3];
    cross3(tv_, e1, qv);
    double vv = dot3(dir, qv) / det;
    if (vv < 0.0 || u + vv > 1.0)
        return -1.0;
    double sig = dot3(e2, qv) / det;
    if (sig < 0.0 || sig > smax)
        return -1.0;
    return sig;
}

// First hit along the segment (smallest sig over all facets).  With bins,
// only the bins that meet the segment's bounding box (widened by a little
// for rounding) are searched: a facet the segment meets is listed in the bin
// of the meeting point.
__device__ double line_hit3d(const Body &b, const double *x, const double *dir, double smax, int lane, int *nb,
                             int *st)
{
    double best = -1.0;
    if (b.nbin == 0) {
        for (int f = lane; f < b.nfacet; f += kWave) {
            double sig = facet_hit(b, x, dir, smax, f);
            if (sig >= 0.0 && (best < 0.0 || sig < best))
                best = sig;
        }
        return wave_min_hit(best);
    }
    int lo[3], ext[3];
    for (int d = 0; d < 3; ++d) {
        double y0 = x[d] - b.disp[d], y1 = y0 + smax * dir[d];
        double slack = 1e-9 * b.bin_h;
        lo[d] = max(0, bin_of(b, d, fmin(y0, y1) - slack));
        ext[d] = max(0, min(b.bin_n[d] - 1, bin_of(b, d, fmax(y0, y1) + slack)) - lo[d] + 1);
    }
    visit_bins(b, lo, ext, -1, lane, nb, st, x, __builtin_inf(), [&](int f) {
        double sig = facet_hit(b, x, dir, smax, f);
        if (sig >= 0.0 && (best < 0.0 || sig < best))
            best = sig;
    });
    return wave_min_hit(best);
}

// enclosing cell along one axis: largest i0 with c[i0] <= y < c[i0 + 1];
// interior pairs only, except on a periodic axis where the pair may
// straddle the boundary (i0 = -1 or i0 + 1 = n, the extended centres being
// the periodic images)
__device__ inline bool locate(const double *c, int n, bool periodic, double y, int hint, int &i0, double &frac)
{
    // the unique lo with c[lo] <= y < c[lo + 1], walked to from the index
    // `hint` (probes lie a few cells from their node)
    int lo = periodic ? -1 : 0, hi = periodic ? n : n - 1;
    if (!(y >= c[lo + 3]) || !(y < c[hi + 3]))
        return false;
    int k = min(max(hint, lo), hi - 1);
    while (c[k + 3] > y)
        --k;
    while (c[k + 4] <= y)
        ++k;
    i0 = k;
    frac = (y - c[k + 3]) / (c[k + 4] - c[k + 3]);
    return true;
}

// i in [-1, n]: the enclosing pair of a probe may straddle a periodic side
__device__ inline int wrap_idx(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Probe stencil set-up: mode 0 multilinear (all corners valid), mode 1
// inverse-distance 1/r^2 over the valid corners (a corner at r = 0 takes all
// the weight).  Valid corners: FLUID, plus FORCING for ghost nodes.
__device__ bool probe_setup(const Grid &g, const uint8_t *cls, const double *y, const int *hint, int mode,
                            bool allow_forcing, int *ids, double *w)
{
    int nd = g.ndim, ncorner = 1 << nd;
    for (int m = 0; m < 8; ++m) {
        ids[m] = -1;
        w[m] = 0.0;
    }
    int i0[3] = {0, 0, 0};
    double fr[3] = {0.0, 0.0, 0.0};
    bool per[3] = {g.bc[0] == IBM_BC_PERIODIC, g.bc[2] == IBM_BC_PERIODIC, g.bc[4] == IBM_BC_PERIODIC};
    if (!locate(g.xc[0], g.ni, per[0], y[0], hint[0], i0[0], fr[0]) ||
        !locate(g.xc[1], g.nj, per[1], y[1], hint[1], i0[1], fr[1]))
        return false;
    if (nd == 3 && !locate(g.xc[2], g.nk, per[2], y[2], hint[2], i0[2], fr[2]))
        return false;
    int nvalid = 0, zero = -1;
    // the corners' classes, all loads in flight before any test
    uint8_t tc[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        if (m >= ncorner)
            break;
        int bx = m & 1, by = (m >> 1) & 1, bz = (m >> 2) & 1;
        int c = cell_index(g, wrap_idx(i0[0] + bx, g.ni), wrap_idx(i0[1] + by, g.nj),
                           nd == 3 ? wrap_idx(i0[2] + bz, g.nk) : 0);
        ids[m] = c;
        tc[m] = cls[c];
    }
    for (int m = 0; m < ncorner; ++m) {
        int bx = m & 1, by = (m >> 1) & 1, bz = (m >> 2) & 1;
        uint8_t t = tc[m];
        bool valid = t == IBM_FLUID || (allow_forcing && t == IBM_FORCING);
        if (mode == 0) {
            if (!valid)
                return false;
            double wt = 1.0;
            int bb[3] = {bx, by, bz};
            for (int d = 0; d < nd; ++d)
                wt *= bb[d] ? fr[d] : 1.0 - fr[d];
            w[m] = wt;
            nvalid++;
        } else {
            if (!valid) {
                w[m] = 0.0;
                continue;
            }
            double cc[3] = {g.xc[0][i0[0] + bx + 3], g.xc[1][i0[1] + by + 3],
                            nd == 3 ? g.xc[2][i0[2] + bz + 3] : 0.0};
            double r2 = 0.0;
            for (int d = 0; d < nd; ++d)
                r2 += (y[d] - cc[d]) * (y[d] - cc[d]);
            if (r2 == 0.0 && zero < 0)
                zero = m;
            w[m] = r2 > 0.0 ? 1.0 / r2 : 0.0;
            nvalid++;
        }
    }
    if (nvalid == 0)
        return false;
    if (mode == 1) {
        if (zero >= 0) {
            for (int m = 0; m < ncorner; ++m)
                w[m] = m == zero ? 1.0 : 0.0;
        } else {
            double s = 0.0;
            for (int m = 0; m < ncorner; ++m)
                s += w[m];
            for (int m = 0; m < ncorner; ++m)
                w[m] /= s;
        }
    }
    return true;
}

// Sections 4.1-4.3 in two launches.  records_kernel: closest feature,
// local normal (face normal or the pseudo-normals of eqs 2-3) and the
// boundary point P' where the line through the node parallel to the normal
// meets the surface; one wavefront per node (the facet searches are split
// across the lanes; lane 0 writes).  probes_kernel: the probes along that
// line and their stencils, one thread per record.
__device__ void node_geometry(const Grid &g, const Body &b, const Flow &fl, const IB &ib, int r, int nF, int lane,
                              int *nb, int *st);

struct GeoArgs {
    Grid g;
    Body b;
    Flow fl;
    IB ib;
};

// four wavefronts per SIMD (at most 128 VGPRs): the searches are latency
// bound, and the occupancy outweighs the few spills it costs
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void records_kernel(GeoArgs args)
{
    (void)args;
    const GeoArgs &A = kernarg_block<GeoArgs>();
    const Grid &g = A.g;
    const Body &b = A.b;
    const Flow &fl = A.fl;
    const IB &ib = A.ib;
    __shared__ int lds[kBlock / kWave][2][kWave];
    int nF = min(ib.counts[CNT_F], ib.cap);
    int nG = min(ib.counts[CNT_G], ib.cap - nF);
    int lane = threadIdx.x % kWave;
    int *nb = lds[threadIdx.x / kWave][0], *st = lds[threadIdx.x / kWave][1];
    int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
    int nwave = gridDim.x * blockDim.x / kWave;
    for (int r = wave; r < nF + nG; r += nwave)
        node_geometry(g, b, fl, ib, r, nF, lane, nb, st);
}

__device__ inline void node_coords(const Grid &g, int c, int &i, int &j, int &k, double *X, double &h)
{
    split_cell(g, c, i, j, k);
    X[0] = g.xc[0][i + 3];
    X[1] = g.xc[1][j + 3];
    X[2] = g.ndim == 3 ? g.xc[2][k + 3] : 0.0;
    h = fmin(g.xf[0][i + 4] - g.xf[0][i + 3], g.xf[1][j + 4] - g.xf[1][j + 3]);
    if (g.ndim == 3)
        h = fmin(h, g.xf[2][k + 4] - g.xf[2][k + 3]);
}

__device__ void node_geometry(const Grid &g, const Body &b, const Flow &fl, const IB &ib, int r, int nF, int lane,
                              int *nb, int *st)
{
    bool forcing = r < nF;
    int c = forcing ? ib.listF[r] : ib.listG[r - nF];
    int nd = g.ndim;
    int i, j, k;
    double X[3], h;
    node_coords(g, c, i, j, k, X, h);
    // region cell of the node (IB nodes lie in the region)
    int li = i - ib.region[0], lj = j - ib.region[2], lk = k - ib.region[4];
    int rc = li >= 0 && li < ib.rw && lj >= 0 && lj < ib.rh && lk >= 0 && lk < ib.rd ? (lk * ib.rh + lj) * ib.rw + li : -1;
    Closest cl;
    if (nd == 2) {
        cl = closest2d(b, X, lane);
    } else {
        cl = closest3d(b, X, lane, nb, st, rc >= 0 ? ib.hint[rc] : -1);
        if (lane == 0 && rc >= 0)
            ib.hint[rc] = cl.facet;
    }
    const double *src = cl.kind == FEAT_FACE ? b.fnrm + 3 * cl.id
                        : cl.kind == FEAT_VERTEX ? b.vnrm + 3 * cl.id
                                                 : b.enrm + 3 * cl.id;
    double n[3] = {src[0], src[1], src[2]};
    double P[3] = {cl.c[0], cl.c[1], cl.c[2]};
    int fb = 0;
    if (b.frame == IBM_FRAME_SDSN) {
        // surface normal: the closest facet's normal through the closest
        // point, whatever the feature
        for (int d = 0; d < 3; ++d)
            n[d] = b.fnrm[3 * cl.facet + d];
    } else if (cl.kind != FEAT_FACE) {
        double dir[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < nd; ++d)
            dir[d] = forcing ? -n[d] : n[d];
        double sig = nd == 2 ? line_hit2d(b, X, dir, 4.0 * h, lane) : line_hit3d(b, X, dir, 4.0 * h, lane, nb, st);
        if (sig >= 0.0) {
            for (int d = 0; d < nd; ++d)
                P[d] = X[d] + sig * dir[d];
        } else {
            fb |= 1;
            if (lane == 0)
                atomicAdd(&ib.counts[CNT_FB_PPRIME], 1);
        }
    }
    if (lane != 0)
        return;
    double dist2 = 0.0;
    for (int d = 0; d < nd; ++d)
        dist2 += (X[d] - P[d]) * (X[d] - P[d]);
    double sx = forcing ? sqrt(dist2) : -sqrt(dist2);
    int *ir = ib.rec_i + (long long)kRecI * r;
    double *dr = ib.rec_d + (long long)kRecD * r;
    ir[0] = c;
    ir[1] = cl.kind;
    ir[2] = cl.id;
    ir[3] = cl.facet;
    ir[6] = fb;
    for (int d = 0; d < 3; ++d) {
        dr[d] = n[d];
        dr[3 + d] = P[d];
    }
    dr[6] = sx;
    dr[25] = sqrt(cl.d2);
    // eq.7: curvature of the closest feature (2D)
    double kappa = nd == 2 ? (cl.kind == FEAT_FACE ? b.fcurv[cl.id] : b.vcurv[cl.id]) : 0.0;
    dr[26] = kappa;
    int cap = ib.cap;
    ib.plan_kappa[r] = kappa;
    ib.plan_node[r] = (int)(((long long)(k + g.hz) * g.sy + (j + 3)) * g.sx + (i + 3));
    for (int d = 0; d < 3; ++d)
        ib.plan_geo[d * cap + r] = n[d];
    ib.plan_geo[3 * cap + r] = sx;
}

// Probes of record r along its line (sections 4.3, 4.5-4.6): s1 = s_X + h
// (FORCING) or max(-s_X, h) (ghost), s2 = s1 + h; moved out by h/2 up to six
// times until the stencils are valid, else inverse-distance weights over the
// valid corners (flagged).  Fill plan: state offsets instead of cell ids,
// unused corners aimed at the node itself with zero weight, so that the fill
// loops are branch-free.
__global__ __launch_bounds__(kBlock) void probes_kernel(GeoArgs args)
{
    (void)args;
    const GeoArgs &A = kernarg_block<GeoArgs>();
    const Grid &g = A.g;
    const Flow &fl = A.fl;
    const IB &ib = A.ib;
    int nF = min(ib.counts[CNT_F], ib.cap);
    int nG = min(ib.counts[CNT_G], ib.cap - nF);
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nF + nG)
        return;
    bool forcing = r < nF;
    int nd = g.ndim;
    int *ir = ib.rec_i + (long long)kRecI * r;
    double *dr = ib.rec_d + (long long)kRecD * r;
    int c = ir[0];
    int i, j, k;
    double X[3], h;
    node_coords(g, c, i, j, k, X, h);
    double n[3] = {dr[0], dr[1], dr[2]}, P[3] = {dr[3], dr[4], dr[5]};
    double sx = dr[6];
    const int hint[3] = {i, j, k};
    int fb = ir[6];
    bool quad = fl.family == IBM_IB_QUADRATIC;
    int mode = (!quad && forcing) ? 1 : 0;
    bool allow_forcing = !forcing;
    double s1 = forcing ? sx + h : fmax(-sx, h);
    double s2 = s1 + h;
    int ids1[8], ids2[8];
    double w1[8], w2[8];
    bool ok = false;
    int mode1 = mode, mode2 = mode;
    for (int attempt = 0; attempt <= 6; ++attempt) {
        double y1[3] = {0.0, 0.0, 0.0}, y2[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < nd; ++d) {
            y1[d] = P[d] + s1 * n[d];
            y2[d] = P[d] + s2 * n[d];
        }
        bool v1 = probe_setup(g, ib.cls, y1, hint, mode, allow_forcing, ids1, w1);
        bool v2 = quad ? probe_setup(g, ib.cls, y2, hint, mode, allow_forcing, ids2, w2) : true;
        if (v1 && v2) {
            ok = true;
            break;
        }
        if (attempt < 6) {
            s1 += 0.5 * h;
            s2 += 0.5 * h;
        }
    }
    if (!ok) {
        double y1[3] = {0.0, 0.0, 0.0}, y2[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < nd; ++d) {
            y1[d] = P[d] + s1 * n[d];
            y2[d] = P[d] + s2 * n[d];
        }
        fb |= 2;
        atomicAdd(&ib.counts[CNT_FB_PROBE], 1);
        mode1 = mode2 = 1;
        bool v1 = probe_setup(g, ib.cls, y1, hint, 1, allow_forcing, ids1, w1);
        bool v2 = quad ? probe_setup(g, ib.cls, y2, hint, 1, allow_forcing, ids2, w2) : true;
        if (!v1)
            mode1 = 2;
        if (quad && !v2)
            mode2 = 2;
        if (!v1 || (quad && !v2))
            fb |= 4;
    }
    if (!quad) {
        for (int m = 0; m < 8; ++m) {
            ids2[m] = -1;
            w2[m] = 0.0;
        }
        mode2 = 3;
    }
    ir[4] = mode1;
    ir[5] = mode2;
    ir[6] = fb;
    for (int m = 0; m < 8; ++m) {
        ir[7 + m] = ids1[m];
        ir[15 + m] = ids2[m];
        dr[9 + m] = w1[m];
        dr[17 + m] = w2[m];
    }
    ir[23] = 0;
    dr[7] = s1;
    dr[8] = s2;
    for (int m = 27; m < kRecD; ++m)
        dr[m] = 0.0;
    int cap = ib.cap;
    int node_off = ib.plan_node[r];
    // per probe: the eight corners' offsets first, then their classes and
    // region-map entries, each round of loads in flight at once
    for (int p = 0; p < (quad ? 2 : 1); ++p) {
        int off8[8], rmi[8];
        double wt8[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            int cc = p ? ids2[m] : ids1[m];
            double ws = p ? w2[m] : w1[m];
            off8[m] = node_off;
            wt8[m] = 0.0;
            rmi[m] = -1;
            if (cc >= 0 && ws != 0.0) {
                int ci, cj, ck;
                split_cell(g, cc, ci, cj, ck);
                off8[m] = (int)(((long long)(ck + g.hz) * g.sy + (cj + 3)) * g.sx + (ci + 3));
                wt8[m] = ws;
                int li = ci - ib.region[0], lj = cj - ib.region[2], lk = ck - ib.region[4];
                if (li >= 0 && li < ib.rw && lj >= 0 && lj < ib.rh && lk >= 0 && lk < ib.rd)
                    rmi[m] = (lk * ib.rh + lj) * ib.rw + li;
            }
        }
        // a ghost's weighted FORCING corner: its record, so that a tile can
        // fill the corner before the ghost (a FORCING cell lies in the region)
        uint8_t c8[8];
        int fr8[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {  // unconditional loads (cell 0 when unused)
            int cc = p ? ids2[m] : ids1[m];
            uint8_t v = ib.cls[rmi[m] >= 0 ? cc : 0];
            c8[m] = !forcing && rmi[m] >= 0 ? v : (uint8_t)IBM_SOLID;
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            int v = ib.rmap[rmi[m] >= 0 ? rmi[m] : 0];
            fr8[m] = c8[m] == IBM_FORCING ? v : -1;
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            int pm = 8 * p + m;
            ib.plan_off[pm * cap + r] = off8[m];
            ib.plan_w[pm * cap + r] = wt8[m];
            ib.plan_frec[pm * cap + r] = fr8[m];
        }
    }
    if (!quad) {
        for (int m = 8; m < 16; ++m) {
            ib.plan_off[m * cap + r] = node_off;
            ib.plan_w[m * cap + r] = 0.0;
            ib.plan_frec[m * cap + r] = -1;
        }
    }
    ib.plan_geo[4 * cap + r] = s1;
    ib.plan_geo[5 * cap + r] = s2;
    ib.plan_mode[r] = mode1 | (mode2 << 4);
}

// Signed-distance classification (the standard HCIB/GC compared with in
// section 7): a region cell inside the posed lattice box of the body is
// inside iff (X - P0) . n_f < 0, with P0 its closest surface point and n_f
// the outward normal of the closest facet (lowest id among equals).  One
// wavefront per cell; overwrites the inside flags.
__global__ __launch_bounds__(kBlock) void sd_inside_kernel(Grid g, Body b, IB ib, int ncell)
{
    __shared__ int lds[kBlock / kWave][2][kWave];
    int lane = threadIdx.x % kWave;
    int *nb = lds[threadIdx.x / kWave][0], *st = lds[threadIdx.x / kWave][1];
    int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
    int nwave = gridDim.x * blockDim.x / kWave;
    int nd = g.ndim;
    for (int rc = wave; rc < ncell; rc += nwave) {
        int li = rc % ib.rw, lj = (rc / ib.rw) % ib.rh, lk = rc / (ib.rw * ib.rh);
        int c[3] = {li + ib.region[0], lj + ib.region[2], lk + ib.region[4]};
        bool inbox = true;
        for (int d = 0; d < nd; ++d) {
            long long p = g.Xc[d][c[d]];
            inbox = inbox && p >= b.lat_lo[d] && p <= b.lat_hi[d];
        }
        int in = 0;
        if (inbox) {
            double X[3] = {g.xc[0][c[0] + 3], g.xc[1][c[1] + 3], nd == 3 ? g.xc[2][c[2] + 3] : 0.0};
            Closest cl;
            if (nd == 2) {
                cl = closest2d(b, X, lane);
            } else {
                cl = closest3d(b, X, lane, nb, st, ib.hint[rc]);
                if (lane == 0)
                    ib.hint[rc] = cl.facet;
            }
            const double *n = b.fnrm + 3 * cl.facet;
            double sd = 0.0;
            for (int d = 0; d < nd; ++d)
                sd += (X[d] - cl.c[d]) * n[d];
            in = sd < 0.0;
        }
        if (lane == 0)
            ib.inside[rc] = (uint8_t)in;
    }
}

inline int blocks_for(long long n, int bs) { return (int)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_pose(const Grid &g, Body &b, long long disp, int axis, hipStream_t s)
{
    int n = b.nvert * g.ndim;
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(pose_kernel, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, b.nvert,
                       g.ndim, b.V0, b.V, b.v, disp, axis);
    return hipGetLastError();
}

hipError_t launch_classify(const Grid &g, const Body &b, IB &ib, hipStream_t s)
{
    int ncell = ib.rw * ib.rh * ib.rd;
    int nrows = ib.rh * ib.rd;
    int nwords = nrows * ib.words_per_row;
    int nmax = ncell > nwords ? ncell : nwords;
    hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(64), 0, s, ib.counts);
    if (ncell == 0)
        return hipGetLastError();
    hipLaunchKernelGGL(clear_kernel, dim3(blocks_for(nmax, kBlock)), dim3(kBlock), 0, s, ib.inside,
                       ncell, ib.toggle, nwords);
    if (b.nfacet > 0 && b.frame == IBM_FRAME_SDSN) {
        int nb = blocks_for(ncell, kBlock / kWave);
        nb = nb < 8192 ? nb : 8192;
        hipLaunchKernelGGL(sd_inside_kernel, dim3(nb), dim3(kBlock), 0, s, g, b, ib, ncell);
    } else if (b.nfacet > 0) {
        if (g.ndim == 2)
            hipLaunchKernelGGL(cross2d_kernel, dim3(blocks_for(b.nfacet, kBlock / kWave)), dim3(kBlock),
                               0, s, g, b, ib);
        else
            hipLaunchKernelGGL(cross3d_kernel, dim3(blocks_for(b.nfacet, 64)), dim3(64), 0, s, g, b,
                               ib);
        hipLaunchKernelGGL(parity_kernel, dim3(blocks_for(nrows, kBlock / kWave)), dim3(kBlock), 0,
                           s, ib, nrows);
    }
    hipLaunchKernelGGL(tag_kernel, dim3(blocks_for(ncell, kBlock)), dim3(kBlock), 0, s, g, ib);
    hipLaunchKernelGGL(count_kernel, dim3(ib.nblk), dim3(kBlock), 0, s, g, ib);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, ib);
    hipLaunchKernelGGL(write_lists_kernel, dim3(ib.nblk), dim3(kBlock), 0, s, g, ib);
    return hipGetLastError();
}

hipError_t launch_records(const Grid &g, const Body &b, const Flow &f, IB &ib, hipStream_t s)
{
    if (ib.cap == 0 || b.nfacet == 0)
        return hipSuccess;
    int nb = blocks_for(ib.cap, kBlock / kWave);  // one wavefront per node
    nb = nb < 4096 ? nb : 4096;
    GeoArgs a{g, b, f, ib};
    hipLaunchKernelGGL(records_kernel, dim3(nb), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(probes_kernel, dim3(blocks_for(ib.cap, kBlock)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace ibm
