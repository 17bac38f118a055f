// Host side of the C ABI declared in include/ibm.h: descriptor checks,
// workspace layout, host preprocessing of grid and body (lattice snapping,
// facet normals, angle-weighted pseudo-normals of eqs 2-3, edge adjacency),
// and the orchestration of the HIP kernels for classify / fill / residual /
// advance.  No device memory is allocated here: everything lives in the
// caller's workspace.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

using namespace ibm;

constexpr int kSlots = 9;  // 8 stage launches of a step + 1 for kernel timing

struct ibm_ctx {
    int device;
    Grid g;
    Body b;
    Flow f;
    IB ib;
    Motion mo;
    double *q1, *q2, *wtmp, *qn, *qnm1;
    double t;
    long long step;
    int n_inner;
    bool classified;
    // the stage launch's tile list (device, body present): eight XCD
    // chunks, near tiles spread over them first, padded with -1
    const int32_t *tiles;
    int ntiles;
    // 3D FP64 with a body: each stage fills the IB nodes of its input in
    // place (standalone fill kernels), then runs the kernel that stages one
    // face direction at a time over every tile
    bool prefill;
    double *slot_qin[kSlots];  // stage input of each batched launch slot (prefill)
    double *qfill;             // kernel timing of a prefill solve: filled copy of the input
    double *fpart;           // surface force block sums
    int32_t *fmissed;        // surface force: facets without a valid centre
    double *fforce;          // surface force of a free body's step (device, 3)
    // graph replay of whole steps (stationary bodies): slot 0 holds one
    // step, slot 1 a chunk of kChunk steps
    bool use_graphs;
    bool corner_lists;       // IBM_OPT_CORNER_LISTS
    hipStream_t cap_stream;
    hipGraph_t graph[2];
    hipGraphExec_t graph_exec[2];
    const double *graph_q[2];
    // batched serving: device argument blocks of every stage launch of a
    // step (RK3: 3 stages x 2 kernel kinds; dual time: first / later step x
    // iteration parity x 2 kernel kinds; one kind is empty per solve),
    // prepared for the state batch_q
    void *d_args;
    int slot_nblk[kSlots];
    const double *batch_q;
    std::vector<char> h_args;
    long long rest_box_lat[6];
    long long region_lat[6];  // lattice box of the IB region's node centres
    // classification buffers: ib is ibb[cur], the one the stages read.  With
    // two (prescribed motion), the next step's classification runs on a side
    // stream into the other while the current step's stages run
    IB ibb[2];
    int nbuf, cur;
    bool buf_ok[2], buf_side[2];
    double buf_t[2];
    bool pipeline;            // IBM_OPT_PIPELINE
    hipStream_t side;
    hipEvent_t ev_fork, ev_ready[2];
    // stage timing (IBM_OPT_STAGE_TIMING): event pairs recorded at the start
    // and end of each stage launch, tev_used of tev_cap taken since the last
    // ibm_stage_timing
    std::vector<hipEvent_t> tev;
    int tev_used;
    char err[256];
};

namespace {

constexpr size_t kAlign = 256;

struct Carve {
    char *base;
    size_t off;
    template <typename T> T *take(size_t n)
    {
        off = (off + kAlign - 1) / kAlign * kAlign;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

int set_err(ibm_ctx *c, int code, const char *msg)
{
    if (c)
        std::snprintf(c->err, sizeof c->err, "%s", msg);
    return code;
}

int check_desc(const ibm_case *c)
{
    if (!c || (c->ndim != 2 && c->ndim != 3))
        return IBM_EINVAL;
    if (c->ni < 4 || c->nj < 4 || (c->ndim == 3 && c->nk < 4))
        return IBM_EINVAL;
    if (c->ndim == 2 && c->nk != 1)
        return IBM_EINVAL;
    if (!c->xf || !c->yf || (c->ndim == 3 && !c->zf))
        return IBM_EINVAL;
    const double *f[3] = {c->xf, c->yf, c->zf};
    int n[3] = {c->ni, c->nj, c->nk};
    for (int d = 0; d < c->ndim; ++d)
        for (int i = 0; i < n[d]; ++i)
            if (!(f[d][i + 1] > f[d][i]))
                return IBM_EINVAL;
    for (int s = 0; s < 6; ++s)
        if (c->bc[s] < IBM_BC_FARFIELD || c->bc[s] > IBM_BC_PERIODIC)
            return IBM_EINVAL;
    for (int d = 0; d < c->ndim; ++d)
        if ((c->bc[2 * d] == IBM_BC_PERIODIC) != (c->bc[2 * d + 1] == IBM_BC_PERIODIC))
            return IBM_EINVAL;
    if (c->nfacet < 0 || c->nvert < 0 || (c->nfacet > 0 && (!c->vert || !c->facet)))
        return IBM_EINVAL;
    for (long long m = 0; m < (long long)c->nfacet * c->ndim; ++m)
        if (c->facet[m] < 0 || c->facet[m] >= c->nvert)
            return IBM_EINVAL;
    if (!(c->mach > 0) || !(c->reynolds > 0) || !(c->prandtl > 0) || !(c->gamma > 1) || !(c->dt > 0))
        return IBM_EINVAL;
    if (c->scheme != IBM_RK3 && c->scheme != IBM_DUAL)
        return IBM_EINVAL;
    if (c->ib_family != IBM_IB_LINEAR && c->ib_family != IBM_IB_QUADRATIC)
        return IBM_EINVAL;
    if (c->precision != IBM_FP64 && c->precision != IBM_MIXED)
        return IBM_EINVAL;
    if (c->scheme == IBM_DUAL && (c->n_inner < 1 || !(c->cfl_tau > 0)))
        return IBM_EINVAL;
    if (c->motion < 0 || c->motion > 2)
        return IBM_EINVAL;
    if (c->motion && (c->motion_par[0] < 0 || c->motion_par[0] >= c->ndim))
        return IBM_EINVAL;
    if (c->motion == 2 && (!(c->motion_par[1] > 0) || c->scheme != IBM_RK3 || c->nfacet == 0))
        return IBM_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(c->u_inf[d]) || (d >= c->ndim && c->u_inf[d] != 0.0))
            return IBM_EINVAL;
    if (!std::isfinite(c->motion_vel) || (c->motion_vel != 0.0 && !c->motion))
        return IBM_EINVAL;
    if (c->wall_pressure != IBM_WALL_EQ6 && c->wall_pressure != IBM_WALL_EQ7)
        return IBM_EINVAL;
    if (c->wall_pressure == IBM_WALL_EQ7 && c->ndim != 2)
        return IBM_EINVAL;
    if (c->reconstruction != IBM_RECON_WENO5 && c->reconstruction != IBM_RECON_TVD2)
        return IBM_EINVAL;
    if (c->ib_framework != IBM_FRAME_RTLN && c->ib_framework != IBM_FRAME_SDSN)
        return IBM_EINVAL;
    return IBM_OK;
}

// extended faces: periodic axes take the periodic images of the far end,
// the others mirror the first / last interior cells
std::vector<double> ext_faces(const double *f, int n, bool periodic)
{
    std::vector<double> e(n + 7);
    for (int i = 0; i <= n; ++i)
        e[i + 3] = f[i];
    for (int k = 1; k <= 3; ++k) {
        if (periodic) {
            e[3 - k] = f[0] - (f[n] - f[n - k]);
            e[n + 3 + k] = f[n] + (f[k] - f[0]);
        } else {
            e[3 - k] = 2.0 * f[0] - f[k];
            e[n + 3 + k] = 2.0 * f[n] - f[n - k];
        }
    }
    return e;
}

struct HostGeom {
    int nd, n[3], hz, sx, sy, sz;
    long long vs, ncell;
    std::vector<double> xf[3], xc[3], rdx[3], rdxc[3], rdtc[3];
    std::vector<float> rdx_f[3], rdxc_f[3], rdtc_f[3];
    std::vector<long long> Xc[3];
    // body
    std::vector<long long> V0;
    std::vector<double> v0;
    std::vector<int> facet;
    std::vector<double> fnrm, vnrm, enrm;
    std::vector<double> fcurv, vcurv;  // 2D: signed curvature per segment / vertex (eq.7)
    std::vector<int> edge_of;
    int nedge;
    int region[6];
    int cap, wpr, nblk;
    // tiles of the fused residual/update kernel: those whose stencils never
    // reach the IB region ("far") and the others ("near"), raster order
    std::vector<int32_t> tiles_far, tiles_near;
    // 3D facet bins (rest frame), see Body
    double bin_o[3], bin_h;
    int bin_n[3], nbin;
    std::vector<int32_t> bin_start, bin_facet;
    std::vector<float> fbox, bin_box;
};

// Uniform bins over the rest-pose body box for the 3D closest-feature and
// line searches: cubes of side 2 h_min (at least the box over 2^21 bins),
// one bin of margin; every facet is listed in each bin its bounding box
// (widened by 1e-9 of a side against rounding) meets.
void facet_bins(HostGeom &h, const std::vector<double> &v)
{
    h.nbin = 0;
    h.bin_h = 1.0;
    for (int d = 0; d < 3; ++d) {
        h.bin_o[d] = 0.0;
        h.bin_n[d] = 0;
    }
    h.bin_start.assign(1, 0);
    h.bin_facet.clear();
    h.fbox.clear();
    h.bin_box.clear();
    int nf = (int)(h.facet.size() / 3);
    if (h.nd != 3 || nf == 0)
        return;
    h.fbox.assign((size_t)6 * nf, 0.0f);
    for (int f = 0; f < nf; ++f)
        for (int d = 0; d < 3; ++d) {
            double fl = 1e300, fh = -1e300;
            for (int m = 0; m < 3; ++m) {
                fl = std::min(fl, v[3 * h.facet[3 * f + m] + d]);
                fh = std::max(fh, v[3 * h.facet[3 * f + m] + d]);
            }
            // rounded outward: the float box contains the exact one
            float flf = (float)fl, fhf = (float)fh;
            if ((double)flf > fl)
                flf = std::nextafter(flf, -HUGE_VALF);
            if ((double)fhf < fh)
                fhf = std::nextafter(fhf, HUGE_VALF);
            h.fbox[6 * f + d] = flf;
            h.fbox[6 * f + 3 + d] = fhf;
        }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (size_t m = 0; m < v.size() / 3; ++m)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], v[3 * m + d]);
            hi[d] = std::max(hi[d], v[3 * m + d]);
        }
    double hmin = 1e300;
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < h.n[d]; ++i)
            hmin = std::min(hmin, h.xf[d][i + 4] - h.xf[d][i + 3]);
    double bs = 2.0 * hmin;
    for (;;) {
        long long tot = 1;
        for (int d = 0; d < 3; ++d)
            tot *= (long long)std::floor((hi[d] - lo[d]) / bs) + 3;
        if (tot <= (1LL << 21))
            break;
        bs *= 2.0;
    }
    h.bin_h = bs;
    for (int d = 0; d < 3; ++d) {
        h.bin_o[d] = lo[d] - bs;
        h.bin_n[d] = (int)std::floor((hi[d] - h.bin_o[d]) / bs) + 2;
    }
    h.nbin = h.bin_n[0] * h.bin_n[1] * h.bin_n[2];
    auto range = [&](int f, int *a, int *b) {
        for (int d = 0; d < 3; ++d) {
            double fl = 1e300, fh = -1e300;
            for (int m = 0; m < 3; ++m) {
                fl = std::min(fl, v[3 * h.facet[3 * f + m] + d]);
                fh = std::max(fh, v[3 * h.facet[3 * f + m] + d]);
            }
            double slack = 1e-9 * bs;
            a[d] = std::max(0, (int)std::floor((fl - slack - h.bin_o[d]) / bs));
            b[d] = std::min(h.bin_n[d] - 1, (int)std::floor((fh + slack - h.bin_o[d]) / bs));
        }
    };
    std::vector<int32_t> cnt(h.nbin + 1, 0);
    for (int f = 0; f < nf; ++f) {
        int a[3], b[3];
        range(f, a, b);
        for (int kz = a[2]; kz <= b[2]; ++kz)
            for (int ky = a[1]; ky <= b[1]; ++ky)
                for (int kx = a[0]; kx <= b[0]; ++kx)
                    ++cnt[(kz * h.bin_n[1] + ky) * h.bin_n[0] + kx + 1];
    }
    for (int k = 0; k < h.nbin; ++k)
        cnt[k + 1] += cnt[k];
    h.bin_start = cnt;
    h.bin_facet.assign(cnt[h.nbin], 0);
    std::vector<int32_t> fillp(cnt.begin(), cnt.end() - 1);
    for (int f = 0; f < nf; ++f) {
        int a[3], b[3];
        range(f, a, b);
        for (int kz = a[2]; kz <= b[2]; ++kz)
            for (int ky = a[1]; ky <= b[1]; ++ky)
                for (int kx = a[0]; kx <= b[0]; ++kx)
                    h.bin_facet[fillp[(kz * h.bin_n[1] + ky) * h.bin_n[0] + kx]++] = f;
    }
    h.bin_box.resize(h.bin_facet.size() * 6);
    for (size_t m = 0; m < h.bin_facet.size(); ++m)
        for (int q = 0; q < 6; ++q)
            h.bin_box[6 * m + q] = h.fbox[6 * (size_t)h.bin_facet[m] + q];
}

// Does [lo, hi) meet [r0, r1), directly or through a periodic wrap of an
// axis of n cells?
bool meets(int lo, int hi, int r0, int r1, int n, bool periodic)
{
    if (r1 <= r0)
        return false;
    for (int sh = periodic ? -1 : 0; sh <= (periodic ? 1 : 0); ++sh)
        if (lo + sh * n < r1 && hi + sh * n > r0)
            return true;
    return false;
}

void tile_lists(const ibm_case *c, HostGeom &h)
{
    const int *T = h.nd == 2 ? kTile2 : kTile3;
    int nt[3];
    for (int d = 0; d < 3; ++d)
        nt[d] = d < h.nd ? (h.n[d] + T[d] - 1) / T[d] : 1;
    h.tiles_far.clear();
    h.tiles_near.clear();
    for (int tz = 0; tz < nt[2]; ++tz)
        for (int ty = 0; ty < nt[1]; ++ty)
            for (int tx = 0; tx < nt[0]; ++tx) {
                int t0[3] = {tx, ty, tz};
                bool near = h.cap > 0;
                for (int d = 0; d < h.nd && near; ++d) {
                    int lo = t0[d] * T[d] - 3, hi = t0[d] * T[d] + T[d] + 3;
                    near = meets(lo, hi, h.region[2 * d], h.region[2 * d + 1], h.n[d],
                                 c->bc[2 * d] == IBM_BC_PERIODIC);
                }
                int id = (tz * nt[1] + ty) * nt[0] + tx;
                (near ? h.tiles_near : h.tiles_far).push_back(id);
            }
}

double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
void unit3(double *a)
{
    double l = std::sqrt(dot3(a, a));
    if (l > 0.0) {
        a[0] /= l;
        a[1] /= l;
        a[2] /= l;
    }
}

// Facet normals and the pseudo-normals of section 4.2.  2D: a polygon
// vertex is the planar image of an extruded edge, so it takes eq.3 with both
// incident segments weighted equally (normalised).  3D: eq.2 weights the
// incident facet normals by their interior angles at the vertex; eq.3 weights
// the two facets of an edge equally (pi each), normalised; a boundary edge
// of an open mesh takes its single facet's normal.
void body_normals(HostGeom &h, const std::vector<double> &v)
{
    int nd = h.nd;
    int nf = (int)(h.facet.size() / nd), nv = (int)(v.size() / nd);
    h.fnrm.assign((size_t)std::max(nf, 1) * 3, 0.0);
    h.vnrm.assign((size_t)std::max(nv, 1) * 3, 0.0);
    if (nd == 2) {
        for (int f = 0; f < nf; ++f) {
            const double *a = &v[2 * h.facet[2 * f]], *b = &v[2 * h.facet[2 * f + 1]];
            double ex = b[0] - a[0], ey = b[1] - a[1], l = std::sqrt(ex * ex + ey * ey);
            h.fnrm[3 * f] = ey / l;
            h.fnrm[3 * f + 1] = -ex / l;
        }
        for (int f = 0; f < nf; ++f)
            for (int e = 0; e < 2; ++e) {
                int id = h.facet[2 * f + e];
                h.vnrm[3 * id] += h.fnrm[3 * f];
                h.vnrm[3 * id + 1] += h.fnrm[3 * f + 1];
            }
        for (int m = 0; m < nv; ++m)
            unit3(&h.vnrm[3 * m]);
        // eq.7 curvature: the turn of the unit vertex normals along a segment
        // over its length, (n_b - n_a).(b - a) / |b - a|^2 (1/r on a regular
        // polygon inscribed in a circle of radius r; positive where convex);
        // a vertex takes the mean of its two segments
        h.fcurv.assign((size_t)std::max(nf, 1), 0.0);
        h.vcurv.assign((size_t)std::max(nv, 1), 0.0);
        for (int f = 0; f < nf; ++f) {
            int ia = h.facet[2 * f], ib = h.facet[2 * f + 1];
            double ex = v[2 * ib] - v[2 * ia], ey = v[2 * ib + 1] - v[2 * ia + 1];
            double dn = (h.vnrm[3 * ib] - h.vnrm[3 * ia]) * ex + (h.vnrm[3 * ib + 1] - h.vnrm[3 * ia + 1]) * ey;
            h.fcurv[f] = dn / (ex * ex + ey * ey);
        }
        for (int f = 0; f < nf; ++f)
            for (int e = 0; e < 2; ++e)
                h.vcurv[h.facet[2 * f + e]] += 0.5 * h.fcurv[f];
        h.nedge = 0;
        h.enrm.assign(3, 0.0);
        h.edge_of.assign(3, 0);
        return;
    }
    for (int f = 0; f < nf; ++f) {
        const int *t = &h.facet[3 * f];
        const double *a = &v[3 * t[0]], *b = &v[3 * t[1]], *c = &v[3 * t[2]];
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double *n = &h.fnrm[3 * f];
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        unit3(n);
        for (int m = 0; m < 3; ++m) {
            const double *p = &v[3 * t[m]], *q = &v[3 * t[(m + 1) % 3]], *r = &v[3 * t[(m + 2) % 3]];
            double u[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
            double w[3] = {r[0] - p[0], r[1] - p[1], r[2] - p[2]};
            double cs = dot3(u, w) / (std::sqrt(dot3(u, u)) * std::sqrt(dot3(w, w)));
            cs = std::min(1.0, std::max(-1.0, cs));
            double ang = std::acos(cs);
            for (int d = 0; d < 3; ++d)
                h.vnrm[3 * t[m] + d] += ang * n[d];
        }
    }
    for (int m = 0; m < nv; ++m)
        unit3(&h.vnrm[3 * m]);
    // edge adjacency: half-edges keyed by (min vertex, max vertex), sorted
    struct HE {
        long long a, b;
        int f, m;
    };
    std::vector<HE> he((size_t)3 * nf);
    for (int f = 0; f < nf; ++f)
        for (int m = 0; m < 3; ++m) {
            int p = h.facet[3 * f + m], q = h.facet[3 * f + (m + 1) % 3];
            he[3 * f + m] = {std::min(p, q), std::max(p, q), f, m};
        }
    std::sort(he.begin(), he.end(), [](const HE &x, const HE &y) {
        if (x.a != y.a) return x.a < y.a;
        if (x.b != y.b) return x.b < y.b;
        if (x.f != y.f) return x.f < y.f;
        return x.m < y.m;
    });
    h.edge_of.assign((size_t)std::max(3 * nf, 1), 0);
    h.enrm.assign((size_t)std::max(3 * nf, 1) * 3, 0.0);
    int ne = 0;
    for (size_t s = 0; s < he.size();) {
        size_t e = s;
        while (e < he.size() && he[e].a == he[s].a && he[e].b == he[s].b)
            ++e;
        for (size_t m = s; m < e; ++m) {
            h.edge_of[3 * he[m].f + he[m].m] = ne;
            for (int d = 0; d < 3; ++d)
                h.enrm[3 * ne + d] += M_PI * h.fnrm[3 * he[m].f + d];
        }
        unit3(&h.enrm[3 * ne]);
        ++ne;
        s = e;
    }
    h.nedge = ne;
}

// Lattice box of the node centres of the IB region (empty: nhi < nlo).
void region_lattice(const HostGeom &h, long long *nlo, long long *nhi)
{
    for (int d = 0; d < 3; ++d) {
        int i0 = h.region[2 * d], i1 = h.region[2 * d + 1];
        if (d >= h.nd || i1 <= i0) {
            nlo[d] = 1;
            nhi[d] = 0;
            continue;
        }
        nlo[d] = h.Xc[d][i0];
        nhi[d] = h.Xc[d][i1 - 1];
    }
}

// The exact crossing predicates (section 3.2) multiply a facet's edge
// extent by a node-to-vertex distance in 64-bit integers on the 2^24
// lattice (the 3D crossing sum then uses 128 bits).  Both factors are bounded
// by the body's lattice box (vertices shifted by sh along each axis) and the
// lattice box of the node centres the classification visits (nlo, nhi; empty
// when nhi < nlo); the products, and the difference of two, must stay below
// 2^63.  Checked in floating point, which has ample range.
bool lattice_products_fit(int nd, const long long *vlo, const long long *vhi, const long long *sh,
                          const long long *nlo, const long long *nhi)
{
    double eb = 0.0, er = 0.0;
    for (int d = 0; d < nd; ++d) {
        double lo = (double)vlo[d] + (double)sh[d], hi = (double)vhi[d] + (double)sh[d];
        eb = std::max(eb, hi - lo);
        if (nhi[d] >= nlo[d])
            er = std::max(er, std::max(std::fabs((double)nhi[d] - lo), std::fabs(hi - (double)nlo[d])));
    }
    return 2.0 * eb * std::max(eb, er) < 0x1p62;
}

int host_geom(const ibm_case *c, HostGeom &h)
{
    h.nd = c->ndim;
    h.n[0] = c->ni;
    h.n[1] = c->nj;
    h.n[2] = c->ndim == 3 ? c->nk : 1;
    h.hz = c->ndim == 3 ? 3 : 0;
    h.sx = c->ni + 6;
    h.sy = c->nj + 6;
    h.sz = h.n[2] + 2 * h.hz;
    h.vs = (long long)h.sx * h.sy * h.sz;
    h.ncell = (long long)c->ni * c->nj * h.n[2];
    const double *fa[3] = {c->xf, c->yf, c->zf};
    static const double unit_z[2] = {-0.5, 0.5};
    for (int d = 0; d < 3; ++d) {
        int n = h.n[d];
        if (d < c->ndim)
            h.xf[d] = ext_faces(fa[d], n, c->bc[2 * d] == IBM_BC_PERIODIC);
        else
            h.xf[d] = ext_faces(unit_z, 1, false);
        h.xc[d].resize(n + 6);
        for (int i = 0; i < n + 6; ++i)
            h.xc[d][i] = 0.5 * (h.xf[d][i] + h.xf[d][i + 1]);
        h.rdx[d].resize(n + 6);
        h.rdxc[d].assign(n + 6, 0.0);
        h.rdtc[d].assign(n + 6, 0.0);
        for (int i = 0; i < n + 6; ++i) {
            h.rdx[d][i] = 1.0 / (h.xf[d][i + 1] - h.xf[d][i]);
            if (i + 1 < n + 6)
                h.rdxc[d][i] = 1.0 / (h.xc[d][i + 1] - h.xc[d][i]);
            if (i >= 1 && i + 1 < n + 6)
                h.rdtc[d][i] = 1.0 / (h.xc[d][i + 1] - h.xc[d][i - 1]);
        }
        h.rdx_f[d].assign(h.rdx[d].begin(), h.rdx[d].end());
        h.rdxc_f[d].assign(h.rdxc[d].begin(), h.rdxc[d].end());
        h.rdtc_f[d].assign(h.rdtc[d].begin(), h.rdtc[d].end());
        h.Xc[d].resize(n);
        for (int i = 0; i < n; ++i)
            h.Xc[d][i] = std::llrint(h.xc[d][i + 3] * kLatScale);
    }
    // body on the lattice
    int nv = c->nvert, nf = c->nfacet, nd = c->ndim;
    h.V0.resize((size_t)std::max(nv, 1) * nd);
    h.v0.resize((size_t)std::max(nv, 1) * nd);
    for (long long m = 0; m < (long long)nv * nd; ++m) {
        double x = c->vert[m];
        if (!(std::fabs(x) < 1.0e6))
            return IBM_EGEOM;
        h.V0[m] = std::llrint(x * kLatScale);
        h.v0[m] = (double)h.V0[m] / kLatScale;
    }
    h.facet.assign(c->facet, c->facet + (size_t)nf * nd);
    if (nf > 0) {
        for (int f = 0; f < nf; ++f) {
            bool same = h.facet[nd * f] == h.facet[nd * f + 1];
            if (nd == 3)
                same = same || h.facet[3 * f + 1] == h.facet[3 * f + 2] || h.facet[3 * f] == h.facet[3 * f + 2];
            if (same)
                return IBM_EGEOM;
        }
        body_normals(h, h.v0);
        facet_bins(h, h.v0);
    } else {
        facet_bins(h, h.v0);
        h.fnrm.assign(3, 0.0);
        h.vnrm.assign(3, 0.0);
        h.enrm.assign(3, 0.0);
        h.edge_of.assign(3, 0);
        h.nedge = 0;
    }
    // immersed-boundary region: body box over all poses, 4 cells of margin
    if (nf == 0) {
        for (int s = 0; s < 6; ++s)
            h.region[s] = 0;
        h.region[5] = h.region[4] = 0;
    } else {
        for (int d = 0; d < 3; ++d) {
            int n = h.n[d];
            if (d >= nd) {
                h.region[2 * d] = 0;
                h.region[2 * d + 1] = 1;
                continue;
            }
            double lo = 1e300, hi = -1e300;
            for (int m = 0; m < nv; ++m) {
                lo = std::min(lo, h.v0[(size_t)m * nd + d]);
                hi = std::max(hi, h.v0[(size_t)m * nd + d]);
            }
            if (c->motion && (int)c->motion_par[0] == d) {
                double a = std::fabs(c->motion_par[1]) + 1e-6;
                lo -= a;
                hi += a;
                if (c->motion_vel != 0.0 || c->motion == 2) {  // unbounded travel: the whole axis
                    lo = -1e300;
                    hi = 1e300;
                }
            }
            int i0 = 0, i1 = n;
            while (i0 < n && h.xc[d][i0 + 3] < lo)
                ++i0;
            while (i1 > 0 && h.xc[d][i1 + 2] > hi)
                --i1;
            i0 = std::max(0, i0 - 4);
            i1 = std::min(n, i1 + 4);
            if (i1 <= i0) {
                i0 = 0;
                i1 = 0;
            }
            h.region[2 * d] = i0;
            h.region[2 * d + 1] = i1;
        }
    }
    int rw = h.region[1] - h.region[0], rh = h.region[3] - h.region[2], rd = h.region[5] - h.region[4];
    if (rw <= 0 || rh <= 0 || rd <= 0)
        rw = rh = rd = 0;
    if (nf > 0) {
        long long vlo[3], vhi[3], nlo[3], nhi[3], zero[3] = {0, 0, 0};
        region_lattice(h, nlo, nhi);
        for (int d = 0; d < nd; ++d) {
            vlo[d] = vhi[d] = h.V0[d];
            for (int m = 1; m < nv; ++m) {
                vlo[d] = std::min(vlo[d], h.V0[(size_t)m * nd + d]);
                vhi[d] = std::max(vhi[d], h.V0[(size_t)m * nd + d]);
            }
        }
        if (!lattice_products_fit(nd, vlo, vhi, zero, nlo, nhi))
            return IBM_EGEOM;
    }
    h.cap = rw * rh * rd;
    h.wpr = (rw + 1 + 31) / 32;
    h.nblk = (h.cap + 255) / 256;
    tile_lists(c, h);
    return IBM_OK;
}

struct Layout {
    double *xc[3], *xf[3], *rdx[3], *rdxc[3], *rdtc[3];
    float *rdx_f[3], *rdxc_f[3], *rdtc_f[3];
    long long *Xc[3];
    long long *V0, *V;
    double *v;
    int *facet;
    double *fnrm, *vnrm, *enrm;
    double *fcurv, *vcurv;
    int *edge_of;
    int32_t *bin_start, *bin_facet;
    float *bin_box;
    uint8_t *cls, *inside;
    uint32_t *toggle;
    int32_t *counts, *blk, *listF, *listG, *rec_i;
    double *rec_d;
    int32_t *plan_node, *plan_off, *plan_mode, *plan_frec;
    double *plan_kappa;
    double *plan_w, *plan_geo, *fval;
    double *fpart;           // surface force block sums
    int32_t *fmissed;        // surface force: facets without a valid centre
    double *fforce;          // surface force of a free body's step
    int32_t *rmap;
    int32_t *hint;
    int32_t *tile_slot, *slot_tile, *tg_cnt, *tg_t, *tg_rec, *tj_cnt, *tj_rec;
    // a second set of the classification's outputs (prescribed motion: the
    // next step is classified while the current one's stages run)
    struct Out2 {
        uint8_t *cls;
        int32_t *counts, *listF, *listG, *rec_i, *plan_node, *plan_off, *plan_mode, *plan_frec, *rmap;
        double *rec_d, *plan_w, *plan_geo, *plan_kappa;
        int32_t *tg_cnt, *tg_t, *tg_rec, *tj_cnt, *tj_rec;
    } out2;
    bool has_out2;
    int32_t *tiles;
    char *args;
    double *q1, *q2, *wtmp, *qn, *qnm1, *qfill;
};

// 3D FP64 solves with a body fill the IB nodes of each stage input in place
// with the standalone fill launches, then run the kernel that stages one
// face direction at a time over every tile: its 72 KB of LDS leave room for
// two blocks per CU, the 122 KB FP64 tile of the inline fill for one.
bool prefill_solve(int nd, int precision, int nfacet, int cap)
{
    return nd == 3 && precision == IBM_FP64 && nfacet > 0 && cap > 0;
}

size_t carve(const ibm_case *c, const HostGeom &h, char *base, Layout &L)
{
    Carve cv{base, 0};
    int nd = c->ndim;
    for (int d = 0; d < 3; ++d) {
        int n = h.n[d];
        L.xc[d] = cv.take<double>(n + 6);
        L.xf[d] = cv.take<double>(n + 7);
        L.rdx[d] = cv.take<double>(n + 6);
        L.rdxc[d] = cv.take<double>(n + 6);
        L.rdtc[d] = cv.take<double>(n + 6);
        L.rdx_f[d] = cv.take<float>(n + 6);
        L.rdxc_f[d] = cv.take<float>(n + 6);
        L.rdtc_f[d] = cv.take<float>(n + 6);
        L.Xc[d] = cv.take<long long>(n);
    }
    size_t nvx = (size_t)std::max(c->nvert, 1) * nd;
    size_t nfx = (size_t)std::max(c->nfacet, 1);
    L.V0 = cv.take<long long>(nvx);
    L.V = cv.take<long long>(nvx);
    L.v = cv.take<double>(nvx);
    L.facet = cv.take<int>(nfx * nd);
    L.fnrm = cv.take<double>(nfx * 3);
    L.vnrm = cv.take<double>((size_t)std::max(c->nvert, 1) * 3);
    L.enrm = cv.take<double>(nfx * 3 * 3);
    L.edge_of = cv.take<int>(nfx * 3);
    L.fcurv = cv.take<double>(nfx);
    L.vcurv = cv.take<double>((size_t)std::max(c->nvert, 1));
    L.bin_start = cv.take<int32_t>(h.bin_start.size());
    L.bin_facet = cv.take<int32_t>(std::max<size_t>(h.bin_facet.size(), 1));
    L.bin_box = cv.take<float>(std::max<size_t>(h.bin_box.size(), 1));
    size_t cap = (size_t)std::max(h.cap, 1);
    int rows = (h.region[3] - h.region[2]) * (h.region[5] - h.region[4]);
    L.cls = cv.take<uint8_t>(h.ncell);
    L.inside = cv.take<uint8_t>(cap);
    L.toggle = cv.take<uint32_t>((size_t)std::max(rows * h.wpr, 1));
    L.counts = cv.take<int32_t>(CNT_WORDS);
    L.blk = cv.take<int32_t>((size_t)5 * std::max(h.nblk, 1));
    L.listF = cv.take<int32_t>(cap);
    L.listG = cv.take<int32_t>(cap);
    L.rec_i = cv.take<int32_t>(cap * kRecI);
    L.rec_d = cv.take<double>(cap * kRecD);
    L.plan_node = cv.take<int32_t>(cap);
    L.plan_off = cv.take<int32_t>(16 * cap);
    L.plan_w = cv.take<double>(16 * cap);
    L.plan_geo = cv.take<double>(6 * cap);
    L.plan_mode = cv.take<int32_t>(cap);
    L.plan_frec = cv.take<int32_t>(16 * cap);
    L.plan_kappa = cv.take<double>(cap);
    L.fval = cv.take<double>((size_t)(nd + 2) * cap);
    L.fpart = cv.take<double>((size_t)3 * std::max(forces_blocks(c->nfacet), 1));
    L.fforce = cv.take<double>(3);
    L.fmissed = cv.take<int32_t>(1);
    L.rmap = cv.take<int32_t>(cap);
    L.hint = cv.take<int32_t>(cap);
    {
        size_t ntile = h.tiles_far.size() + h.tiles_near.size(), nslot = h.tiles_near.size();
        size_t stride = (size_t)tile_load_cells(nd);
        L.tile_slot = cv.take<int32_t>(std::max<size_t>(ntile, 1));
        L.slot_tile = cv.take<int32_t>(std::max<size_t>(nslot, 1));
        L.tg_cnt = cv.take<int32_t>(std::max<size_t>(nslot, 1));
        L.tg_t = cv.take<int32_t>(std::max<size_t>(nslot * stride, 1));
        L.tg_rec = cv.take<int32_t>(std::max<size_t>(nslot * stride, 1));
        L.tj_cnt = cv.take<int32_t>(std::max<size_t>(nslot, 1));
        L.tj_rec = cv.take<int32_t>(std::max<size_t>(nslot * stride, 1));
    }
    L.tiles = cv.take<int32_t>(h.tiles_far.size() + h.tiles_near.size() + 16);
    L.args = cv.take<char>(kSlots * stage_args_bytes());
    size_t st = (size_t)h.vs * (nd + 2);
    L.q1 = L.q2 = L.wtmp = L.qn = L.qnm1 = L.qfill = nullptr;
    if (c->scheme == IBM_RK3) {
        L.q1 = cv.take<double>(st);
        L.q2 = cv.take<double>(st);
    } else {
        L.wtmp = cv.take<double>(st);
        L.qn = cv.take<double>((size_t)h.ncell * (nd + 2));
        L.qnm1 = cv.take<double>((size_t)h.ncell * (nd + 2));
        if (prefill_solve(nd, c->precision, c->nfacet, h.cap))
            L.qfill = cv.take<double>(st);
    }
    L.has_out2 = c->motion == 1 && c->nfacet > 0 && h.cap > 0;
    L.out2 = {};
    if (L.has_out2) {
        Layout::Out2 &o = L.out2;
        size_t nslot = h.tiles_near.size(), stride = (size_t)tile_load_cells(nd);
        o.cls = cv.take<uint8_t>(h.ncell);
        o.counts = cv.take<int32_t>(CNT_WORDS);
        o.listF = cv.take<int32_t>(cap);
        o.listG = cv.take<int32_t>(cap);
        o.rec_i = cv.take<int32_t>(cap * kRecI);
        o.rec_d = cv.take<double>(cap * kRecD);
        o.plan_node = cv.take<int32_t>(cap);
        o.plan_off = cv.take<int32_t>(16 * cap);
        o.plan_w = cv.take<double>(16 * cap);
        o.plan_geo = cv.take<double>(6 * cap);
        o.plan_mode = cv.take<int32_t>(cap);
        o.plan_frec = cv.take<int32_t>(16 * cap);
        o.plan_kappa = cv.take<double>(cap);
        o.rmap = cv.take<int32_t>(cap);
        o.tg_cnt = cv.take<int32_t>(std::max<size_t>(nslot, 1));
        o.tg_t = cv.take<int32_t>(std::max<size_t>(nslot * stride, 1));
        o.tg_rec = cv.take<int32_t>(std::max<size_t>(nslot * stride, 1));
        o.tj_cnt = cv.take<int32_t>(std::max<size_t>(nslot, 1));
        o.tj_rec = cv.take<int32_t>(std::max<size_t>(nslot * stride, 1));
    }
    return (cv.off + kAlign - 1) / kAlign * kAlign;
}

template <typename T> hipError_t up(T *dst, const std::vector<T> &src)
{
    if (src.empty())
        return hipSuccess;
    return hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

int dev_err(ibm_ctx *c, hipError_t e, const char *where)
{
    if (e == hipSuccess)
        return IBM_OK;
    if (c)
        std::snprintf(c->err, sizeof c->err, "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
    return IBM_EDEVICE;
}

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

void motion_kin(const ibm_ctx *c, double t, double &disp, double &vel, double &acc)
{
    if (c->mo.free) {
        disp = c->mo.x;
        vel = c->mo.u;
        acc = c->mo.a;
        return;
    }
    double w = 2.0 * M_PI * c->mo.freq;
    disp = c->mo.amp * std::cos(w * t + c->mo.phase) + c->mo.vel * t;
    vel = -w * c->mo.amp * std::sin(w * t + c->mo.phase) + c->mo.vel;
    acc = -w * w * c->mo.amp * std::cos(w * t + c->mo.phase);
}

// Pose the body at t and classify into buffer k on stream s (ray parity,
// tags, lists, records, near-tile lists).
int classify_buf(ibm_ctx *c, int k, double t, hipStream_t s)
{
    IB &ib = c->ibb[k];
    hipError_t e = hipSuccess;
    if (c->mo.on && c->b.nvert > 0) {
        double disp, vel, acc;
        motion_kin(c, t, disp, vel, acc);
        long long dl = std::llrint(disp * kLatScale);
        {
            long long vlo[3], vhi[3], nlo[3], nhi[3], sh[3];
            for (int d = 0; d < 3; ++d) {
                vlo[d] = c->rest_box_lat[2 * d];
                vhi[d] = c->rest_box_lat[2 * d + 1];
                nlo[d] = c->region_lat[2 * d];
                nhi[d] = c->region_lat[2 * d + 1];
                sh[d] = d == c->mo.axis ? dl : 0;
            }
            if (!std::isfinite(disp) || std::fabs(disp) > 1.0e6 ||
                !lattice_products_fit(c->g.ndim, vlo, vhi, sh, nlo, nhi))
                return set_err(c, IBM_EGEOM, "body pose beyond the range of the exact lattice predicates");
        }
        for (int d = 0; d < 3; ++d) {
            long long sh = d == c->mo.axis ? dl : 0;
            c->b.disp[d] = (double)sh / kLatScale;
            c->b.lat_lo[d] = c->rest_box_lat[2 * d] + sh;
            c->b.lat_hi[d] = c->rest_box_lat[2 * d + 1] + sh;
        }
        e = launch_pose(c->g, c->b, dl, c->mo.axis, s);
        if (e != hipSuccess)
            return dev_err(c, e, "pose");
    }
    c->buf_ok[k] = false;
    if (c->b.nfacet > 0) {
        e = launch_classify(c->g, c->b, ib, s);
        if (e != hipSuccess)
            return dev_err(c, e, "classify");
        e = launch_records(c->g, c->b, c->f, ib, s);
        if (e != hipSuccess)
            return dev_err(c, e, "records");
        e = launch_ghost_lists(c->g, ib, c->f.family == IBM_IB_QUADRATIC, c->corner_lists, s);
        if (e != hipSuccess)
            return dev_err(c, e, "ghost lists");
    }
    c->buf_ok[k] = true;
    c->buf_t[k] = t;
    c->buf_side[k] = false;
    return IBM_OK;
}

// Classify at t into the current buffer, on the caller's stream.
int do_classify(ibm_ctx *c, double t, hipStream_t s)
{
    int rc = classify_buf(c, c->cur, t, s);
    c->ib = c->ibb[c->cur];
    if (rc)
        return rc;
    c->classified = true;
    return IBM_OK;
}



int do_fill(ibm_ctx *c, double *q, double t, hipStream_t s)
{
    double disp = 0.0, vel = 0.0, acc = 0.0;
    int axis = -1;
    if (c->mo.on) {
        motion_kin(c, t, disp, vel, acc);
        axis = c->mo.axis;
    }
    hipError_t e = c->b.nfacet == 0 ? launch_domain_bc(c->g, c->f, q, s)
                                    : launch_bc_fill(c->g, c->f, c->ib, q, vel, acc, axis, s);
    return dev_err(c, e, "fill");
}

}  // namespace

extern "C" {

int ibm_workspace_bytes(const ibm_case *c, size_t *bytes)
{
    if (!bytes)
        return IBM_EINVAL;
    int rc = check_desc(c);
    if (rc)
        return rc;
    HostGeom h;
    rc = host_geom(c, h);
    if (rc)
        return rc;
    Layout L;
    *bytes = carve(c, h, nullptr, L);
    return IBM_OK;
}

int ibm_create(const ibm_case *c, void *d_workspace, size_t bytes, ibm_ctx **out)
{
    if (!out)
        return IBM_EINVAL;
    *out = nullptr;
    int rc = check_desc(c);
    if (rc)
        return rc;
    if (!d_workspace)
        return IBM_EINVAL;
    HostGeom h;
    rc = host_geom(c, h);
    if (rc)
        return rc;
    Layout L;
    size_t need = carve(c, h, nullptr, L);
    if (bytes < need)
        return IBM_ENOSPACE;
    carve(c, h, static_cast<char *>(d_workspace), L);
    ibm_ctx *x = new (std::nothrow) ibm_ctx();
    if (!x)
        return IBM_EINVAL;
    std::memset(x->err, 0, sizeof x->err);
    if (hipGetDevice(&x->device) != hipSuccess)
        x->device = -1;
    int nd = c->ndim;
    Grid &g = x->g;
    g.ndim = nd;
    g.ni = c->ni;
    g.nj = c->nj;
    g.nk = h.n[2];
    g.nv = nd + 2;
    g.hz = h.hz;
    g.sx = h.sx;
    g.sy = h.sy;
    g.sz = h.sz;
    g.vs = h.vs;
    g.ncell = h.ncell;
    for (int s = 0; s < 6; ++s)
        g.bc[s] = c->bc[s];
    hipError_t e = hipSuccess;
    for (int d = 0; d < 3; ++d) {
        g.xc[d] = L.xc[d];
        g.xf[d] = L.xf[d];
        g.rdx[d] = L.rdx[d];
        g.rdxc[d] = L.rdxc[d];
        g.rdtc[d] = L.rdtc[d];
        g.rdx_f[d] = L.rdx_f[d];
        g.rdxc_f[d] = L.rdxc_f[d];
        g.rdtc_f[d] = L.rdtc_f[d];
        g.Xc[d] = L.Xc[d];
        if (e == hipSuccess) e = up(L.xc[d], h.xc[d]);
        if (e == hipSuccess) e = up(L.xf[d], h.xf[d]);
        if (e == hipSuccess) e = up(L.rdx[d], h.rdx[d]);
        if (e == hipSuccess) e = up(L.rdxc[d], h.rdxc[d]);
        if (e == hipSuccess) e = up(L.rdtc[d], h.rdtc[d]);
        if (e == hipSuccess) e = up(L.rdx_f[d], h.rdx_f[d]);
        if (e == hipSuccess) e = up(L.rdxc_f[d], h.rdxc_f[d]);
        if (e == hipSuccess) e = up(L.rdtc_f[d], h.rdtc_f[d]);
        if (e == hipSuccess) e = up(L.Xc[d], h.Xc[d]);
    }
    Body &b = x->b;
    b.nvert = c->nvert;
    b.nfacet = c->nfacet;
    b.nedge = h.nedge;
    b.V0 = L.V0;
    b.V = L.V;
    b.v = L.v;
    b.facet = L.facet;
    b.fnrm = L.fnrm;
    b.vnrm = L.vnrm;
    b.enrm = L.enrm;
    b.edge_of = L.edge_of;
    b.fcurv = L.fcurv;
    b.vcurv = L.vcurv;
    for (int d = 0; d < 3; ++d) {
        b.bin_o[d] = h.bin_o[d];
        b.bin_n[d] = h.bin_n[d];
        b.disp[d] = 0.0;
    }
    b.bin_h = h.bin_h;
    b.nbin = h.nbin;
    b.bin_start = L.bin_start;
    b.bin_facet = L.bin_facet;
    b.bin_box = L.bin_box;
    b.frame = c->ib_framework;
    for (int d = 0; d < 3; ++d) {
        long long lo = 0, hi = 0;
        for (int m = 0; m < c->nvert && d < nd; ++m) {
            long long v = h.V0[(size_t)m * nd + d];
            lo = m == 0 ? v : std::min(lo, v);
            hi = m == 0 ? v : std::max(hi, v);
        }
        x->rest_box_lat[2 * d] = b.lat_lo[d] = lo;
        x->rest_box_lat[2 * d + 1] = b.lat_hi[d] = hi;
    }
    {
        long long nlo[3], nhi[3];
        region_lattice(h, nlo, nhi);
        for (int d = 0; d < 3; ++d) {
            x->region_lat[2 * d] = nlo[d];
            x->region_lat[2 * d + 1] = nhi[d];
        }
    }
    if (e == hipSuccess) e = up(L.bin_start, h.bin_start);
    if (e == hipSuccess) e = up(L.bin_facet, h.bin_facet);
    if (e == hipSuccess && !h.bin_box.empty()) e = up(L.bin_box, h.bin_box);
    if (e == hipSuccess) e = up(L.V0, h.V0);
    if (e == hipSuccess) e = up(L.V, h.V0);
    if (e == hipSuccess) e = up(L.v, h.v0);
    if (e == hipSuccess && c->nfacet > 0) e = up(L.facet, h.facet);
    if (e == hipSuccess) e = up(L.fnrm, h.fnrm);
    if (e == hipSuccess) e = up(L.vnrm, h.vnrm);
    if (e == hipSuccess && !h.enrm.empty()) e = up(L.enrm, h.enrm);
    if (e == hipSuccess && !h.edge_of.empty()) e = up(L.edge_of, h.edge_of);
    if (e == hipSuccess && !h.fcurv.empty()) e = up(L.fcurv, h.fcurv);
    if (e == hipSuccess && !h.vcurv.empty()) e = up(L.vcurv, h.vcurv);

    Flow &f = x->f;
    f.gamma = c->gamma;
    f.pinf = 1.0 / (c->gamma * c->mach * c->mach);
    f.R = f.pinf;
    f.rR = 1.0 / f.R;
    f.gm1inv = 1.0 / (c->gamma - 1.0);
    f.cp = c->gamma * f.R / (c->gamma - 1.0);
    f.mu = 1.0 / c->reynolds;
    f.kc = f.mu * f.cp / c->prandtl;
    f.pr = c->prandtl;
    f.uinf2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        f.uinf[d] = c->u_inf[d];
        f.uinf2 += c->u_inf[d] * c->u_inf[d];
    }
    f.wallp = c->wall_pressure;
    f.recon = c->reconstruction;
    f.Hinf = c->gamma / (c->gamma - 1.0) * f.pinf + 0.5 * f.uinf2;
    f.dt = c->dt;
    f.cfl_tau = c->cfl_tau;
    f.scheme = c->scheme;
    f.family = c->ib_family;
    f.precision = c->precision;
    {
        // preconditioning cut-off: U_c^2 = max(U_inf^2, (nu/h)^2, (h/(pi dt))^2)
        double hmin = 1e300;
        for (int d = 0; d < nd; ++d)
            for (int i = 0; i < h.n[d]; ++i)
                hmin = std::min(hmin, h.xf[d][i + 4] - h.xf[d][i + 3]);
        double bb = f.mu / hmin, cc = hmin / (M_PI * c->dt);
        f.uc2 = std::max(f.uinf2, std::max(bb * bb, cc * cc));
    }
    IB &ib = x->ib;
    ib.counts_other = nullptr;
    for (int s = 0; s < 6; ++s)
        ib.region[s] = h.region[s];
    ib.rw = h.region[1] - h.region[0];
    ib.rh = h.region[3] - h.region[2];
    ib.rd = h.region[5] - h.region[4];
    if (h.cap == 0)
        ib.rw = ib.rh = ib.rd = 0;
    ib.words_per_row = h.wpr;
    ib.cap = h.cap;
    ib.cls = L.cls;
    ib.inside = L.inside;
    ib.toggle = L.toggle;
    ib.counts = L.counts;
    ib.blk = L.blk;
    ib.nblk = h.nblk;
    ib.listF = L.listF;
    ib.listG = L.listG;
    ib.rec_i = L.rec_i;
    ib.rec_d = L.rec_d;
    ib.plan_node = L.plan_node;
    ib.plan_off = L.plan_off;
    ib.plan_w = L.plan_w;
    ib.plan_geo = L.plan_geo;
    ib.plan_mode = L.plan_mode;
    ib.plan_frec = L.plan_frec;
    ib.plan_kappa = L.plan_kappa;
    ib.fval = L.fval;
    ib.rmap = L.rmap;
    ib.hint = L.hint;
    ib.tile_slot = L.tile_slot;
    ib.slot_tile = L.slot_tile;
    ib.tg_cnt = L.tg_cnt;
    ib.tg_t = L.tg_t;
    ib.tg_rec = L.tg_rec;
    ib.tj_cnt = L.tj_cnt;
    ib.tj_rec = L.tj_rec;
    ib.nslot = (int)h.tiles_near.size();
    ib.tg_stride = tile_load_cells(nd);
    x->nbuf = 1;
    x->cur = 0;
    x->pipeline = true;
    x->side = nullptr;
    x->ev_fork = x->ev_ready[0] = x->ev_ready[1] = nullptr;
    for (int k = 0; k < 2; ++k) {
        x->buf_ok[k] = x->buf_side[k] = false;
        x->buf_t[k] = 0.0;
    }
    {
        std::vector<int32_t> ts(h.tiles_far.size() + h.tiles_near.size(), -1);
        for (size_t m = 0; m < h.tiles_near.size(); ++m)
            ts[h.tiles_near[m]] = (int32_t)m;
        if (e == hipSuccess) e = up(L.tile_slot, ts);
        if (e == hipSuccess) e = up(L.slot_tile, h.tiles_near);
    }
    // one launch per stage: the blocks of one XCD (same index mod 8) take a
    // contiguous chunk of the list; the near tiles, which also fill the IB
    // nodes they read, are spread evenly over the chunks and start first,
    // then the far tiles follow in raster order.  (Chunks of whole raster
    // runs, near tiles first, keep the cache lines neighbouring tiles share
    // in one L2 but load the XCDs unevenly: measured slower.)
    std::vector<int32_t> list;
    {
        int nfar = (int)h.tiles_far.size(), nnear = (int)h.tiles_near.size();
        std::vector<int32_t> chunk[8];
        size_t per = 0;
        for (int x = 0; x < 8; ++x) {
            for (long long m = (long long)x * nnear / 8; m < (long long)(x + 1) * nnear / 8; ++m)
                chunk[x].push_back(h.tiles_near[m]);
            for (long long m = (long long)x * nfar / 8; m < (long long)(x + 1) * nfar / 8; ++m)
                chunk[x].push_back(h.tiles_far[m]);
            per = std::max(per, chunk[x].size());
        }
        for (int x = 0; x < 8; ++x) {
            chunk[x].resize(per, -1);
            list.insert(list.end(), chunk[x].begin(), chunk[x].end());
        }
    }
    if (e == hipSuccess) e = up(L.tiles, list);
    if (e == hipSuccess) e = hipMemset(L.cls, IBM_FLUID, (size_t)h.ncell);
    if (e == hipSuccess) e = hipMemset(L.counts, 0, sizeof(int32_t) * CNT_WORDS);
    if (e == hipSuccess) e = hipMemset(L.hint, 0xff, sizeof(int32_t) * (size_t)std::max(h.cap, 1));  // no hints yet (-1)
    x->ibb[0] = x->ib;
    if (L.has_out2) {
        const Layout::Out2 &o = L.out2;
        IB b2 = x->ib;
        b2.cls = o.cls;
        b2.counts = o.counts;
        b2.listF = o.listF;
        b2.listG = o.listG;
        b2.rec_i = o.rec_i;
        b2.rec_d = o.rec_d;
        b2.plan_node = o.plan_node;
        b2.plan_off = o.plan_off;
        b2.plan_w = o.plan_w;
        b2.plan_geo = o.plan_geo;
        b2.plan_mode = o.plan_mode;
        b2.plan_frec = o.plan_frec;
        b2.plan_kappa = o.plan_kappa;
        b2.rmap = o.rmap;
        b2.tg_cnt = o.tg_cnt;
        b2.tg_t = o.tg_t;
        b2.tg_rec = o.tg_rec;
        b2.tj_cnt = o.tj_cnt;
        b2.tj_rec = o.tj_rec;
        b2.counts_other = x->ib.counts;
        x->ibb[1] = b2;
        x->ibb[0].counts_other = o.counts;
        x->ib = x->ibb[0];
        x->nbuf = 2;
        if (e == hipSuccess) e = hipMemset(o.cls, IBM_FLUID, (size_t)h.ncell);
        if (e == hipSuccess) e = hipMemset(o.counts, 0, sizeof(int32_t) * CNT_WORDS);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    x->mo.on = c->motion != 0;
    x->mo.axis = c->motion ? (int)c->motion_par[0] : 0;
    x->mo.amp = c->motion_par[1];
    x->mo.freq = c->motion_par[2];
    x->mo.phase = c->motion_par[3];
    x->mo.vel = c->motion_vel;
    x->mo.free = c->motion == 2;
    x->mo.mass = c->motion == 2 ? c->motion_par[1] : 0.0;
    x->mo.x = 0.0;
    x->mo.u = c->motion == 2 ? c->motion_vel : 0.0;
    x->mo.a = 0.0;
    x->mo.force = 0.0;
    if (x->mo.free) {
        x->mo.amp = x->mo.freq = x->mo.phase = x->mo.vel = 0.0;
    }
    x->q1 = L.q1;
    x->q2 = L.q2;
    x->wtmp = L.wtmp;
    x->qn = L.qn;
    x->qnm1 = L.qnm1;
    x->t = 0.0;
    x->step = 0;
    x->n_inner = c->n_inner;
    x->classified = false;
    x->use_graphs = true;
    x->corner_lists = true;
    x->cap_stream = nullptr;
    for (int k = 0; k < 2; ++k) {
        x->graph[k] = nullptr;
        x->graph_exec[k] = nullptr;
        x->graph_q[k] = nullptr;
    }
    x->d_args = L.args;
    x->fpart = L.fpart;
    x->fmissed = L.fmissed;
    x->fforce = L.fforce;
    x->batch_q = nullptr;
    for (int k = 0; k < kSlots; ++k)
        x->slot_nblk[k] = 0;
    x->tiles = L.tiles;
    x->ntiles = (int)list.size();
    x->prefill = prefill_solve(nd, x->f.precision, c->nfacet, h.cap);
    x->qfill = x->prefill ? (x->f.scheme == IBM_RK3 ? L.q2 : L.qfill) : nullptr;
    for (int k = 0; k < kSlots; ++k)
        x->slot_qin[k] = nullptr;
    x->tev_used = 0;
    if (e != hipSuccess) {
        delete x;
        return IBM_EDEVICE;
    }
    *out = x;
    return IBM_OK;
}

static void drop_graph(ibm_ctx *c)
{
    for (int k = 0; k < 2; ++k) {
        if (c->graph_exec[k])
            (void)hipGraphExecDestroy(c->graph_exec[k]);
        if (c->graph[k])
            (void)hipGraphDestroy(c->graph[k]);
        c->graph_exec[k] = nullptr;
        c->graph[k] = nullptr;
        c->graph_q[k] = nullptr;
    }
}

static void drop_timing(ibm_ctx *c)
{
    for (hipEvent_t e : c->tev)
        (void)hipEventDestroy(e);
    c->tev.clear();
    c->tev_used = 0;
}

void ibm_destroy(ibm_ctx *c)
{
    if (!c)
        return;
    drop_graph(c);
    drop_timing(c);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    if (c->ev_fork)
        (void)hipEventDestroy(c->ev_fork);
    for (int k = 0; k < 2; ++k)
        if (c->ev_ready[k])
            (void)hipEventDestroy(c->ev_ready[k]);
    if (c->cap_stream)
        (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

int ibm_set_option(ibm_ctx *c, int option, int value)
{
    if (!c)
        return IBM_EINVAL;
    if (option == IBM_OPT_GRAPHS) {
        c->use_graphs = value != 0;
        drop_graph(c);
        return IBM_OK;
    }
    if (option == IBM_OPT_CORNER_LISTS) {
        c->corner_lists = value != 0;
        c->classified = false;  // the lists are rebuilt by the next classification
        c->buf_ok[0] = c->buf_ok[1] = false;
        return IBM_OK;
    }
    if (option == IBM_OPT_PIPELINE) {
        c->pipeline = value != 0;
        return IBM_OK;
    }
    if (option == IBM_OPT_STAGE_TIMING) {
        if (value < 0 || value > IBM_STAGE_TIMING_MAX)
            return set_err(c, IBM_EINVAL, "stage timing: 0 to IBM_STAGE_TIMING_MAX launches");
        drop_timing(c);
        for (int k = 0; k < 2 * value; ++k) {
            hipEvent_t e = nullptr;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) {
                drop_timing(c);
                return dev_err(c, r, "stage timing events");
            }
            c->tev.push_back(e);
        }
        return IBM_OK;
    }
    return IBM_EINVAL;
}

int ibm_set_time(ibm_ctx *c, double t)
{
    if (!c || !std::isfinite(t))
        return IBM_EINVAL;
    c->t = t;
    c->buf_ok[0] = c->buf_ok[1] = false;
    return IBM_OK;
}

int ibm_classify(ibm_ctx *c, void *stream)
{
    if (!c)
        return IBM_EINVAL;
    return do_classify(c, c->t, S(stream));
}

int ibm_fill(ibm_ctx *c, double *q, double t, void *stream)
{
    if (!c || !q)
        return IBM_EINVAL;
    if (!c->classified) {
        int rc = do_classify(c, c->t, S(stream));
        if (rc)
            return rc;
    }
    return do_fill(c, q, t, S(stream));
}

int ibm_forces(ibm_ctx *c, const double *q, double *force, double *facet_out, int32_t *missed, void *stream)
{
    if (!c || !q || !force)
        return IBM_EINVAL;
    if (c->b.nfacet == 0)
        return IBM_EINVAL;
    if (!c->classified) {
        int rc = do_classify(c, c->t, S(stream));
        if (rc)
            return rc;
    }
    int32_t *m = missed ? missed : c->fmissed;
    hipError_t e = hipMemsetAsync(m, 0, sizeof(int32_t), S(stream));
    if (e == hipSuccess)
        e = launch_forces(c->g, c->b, c->f, c->ib, q, force, facet_out, c->fpart, m, S(stream));
    return dev_err(c, e, "forces");
}

int ibm_forces_static(ibm_ctx *c, const double *q, double *force, double *facet_out, int32_t *missed,
                      void *stream)
{
    if (!c || !q || !force)
        return IBM_EINVAL;
    if (c->b.nfacet == 0)
        return set_err(c, IBM_EINVAL, "ibm_forces_static: no body");
    if (c->b.nfacet > IBM_FORCES_STATIC_MAX_FACETS)
        return set_err(c, IBM_EINVAL, "ibm_forces_static: more facets than IBM_FORCES_STATIC_MAX_FACETS");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return dev_err(c, e, "ibm_forces_static: current device");
    if (dev != c->device)
        return set_err(c, IBM_EINVAL, "ibm_forces_static: the context's device must be current");
    if (!c->classified) {
        int rc = do_classify(c, c->t, S(stream));
        if (rc)
            return rc;
    }
    double *part = nullptr;
    int32_t *own_missed = nullptr;
    e = forces_static_scratch(dev, &part, &own_missed);
    if (e != hipSuccess)
        return dev_err(c, e, "ibm_forces_static: scratch address");
    int32_t *m = missed ? missed : own_missed;
    e = launch_zero_i32(m, S(stream));
    if (e == hipSuccess)
        e = launch_forces(c->g, c->b, c->f, c->ib, q, force, facet_out, part, m, S(stream));
    return dev_err(c, e, "ibm_forces_static");
}

int ibm_body_state(const ibm_ctx *c, double *out)
{
    if (!c || !out || !c->mo.free)
        return IBM_EINVAL;
    out[0] = c->mo.x;
    out[1] = c->mo.u;
    out[2] = c->mo.a;
    out[3] = c->mo.force;
    return IBM_OK;
}

int ibm_residual(ibm_ctx *c, const double *q, double *r, void *stream)
{
    if (!c || !q || !r)
        return IBM_EINVAL;
    if (!c->classified) {
        int rc = do_classify(c, c->t, S(stream));
        if (rc)
            return rc;
    }
    return dev_err(c, launch_residual(c->g, c->f, c->ib, q, r, S(stream)), "residual");
}

}  // extern "C"

namespace {

// Next free event pair of the stage timer (both null when timing is off or
// the pool is used up).
void take_timing_pair(ibm_ctx *c, hipEvent_t &e0, hipEvent_t &e1)
{
    e0 = e1 = nullptr;
    if (2 * (c->tev_used + 1) > (int)c->tev.size())
        return;
    e0 = c->tev[2 * c->tev_used];
    e1 = c->tev[2 * c->tev_used + 1];
    ++c->tev_used;
}

// The side stream and events of the classification pipeline (created on
// first use, on the context's device, default priority).
int ensure_side(ibm_ctx *c)
{
    if (c->side)
        return IBM_OK;
    hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&c->ev_ready[k], hipEventDisableTiming);
    return dev_err(c, e, "pipeline stream");
}

// The tile lists of a stage launch with a body (the body moving along
// `axis` at vel, acc; axis -1 when stationary).
StagePart stage_part(const ibm_ctx *c, double vel, double acc, int axis)
{
    StagePart p{c->tiles, c->ntiles, vel, acc, axis};
    p.prefill = c->prefill;
    return p;
}

// One stage is one launch on the stream.  With a body it runs the tile list,
// whose near tiles fill the IB nodes they read; without one, every tile.
// (3D FP64 with a body: the two standalone fill launches on the stage input,
// then every tile.)
template <typename Launch> int enqueue_stage(ibm_ctx *c, double t, hipStream_t s, Launch launch)
{
    if (c->b.nfacet == 0 || c->ib.cap == 0)
        return dev_err(c, launch(s, nullptr), "stage");
    double disp = 0.0, vel = 0.0, acc = 0.0;
    int axis = -1;
    if (c->mo.on) {
        motion_kin(c, t, disp, vel, acc);
        axis = c->mo.axis;
    }
    StagePart p = stage_part(c, vel, acc, axis);
    take_timing_pair(c, p.ev_start, p.ev_stop);
    return dev_err(c, launch(s, &p), "stage");
}

// One SSP-RK3 step (Shu-Osher) starting at time t; a fill at each stage time.
int enqueue_rk3_step(ibm_ctx *c, double *q, double t, hipStream_t s)
{
    int rc;
    double dt = c->f.dt;
    const Grid &g = c->g;
    const Flow &f = c->f;
    const IB &ib = c->ib;
    double *q1 = c->q1, *q2 = c->q2;
    if ((rc = enqueue_stage(c, t, s, [&](hipStream_t st, const StagePart *p) {
             return launch_rk_stage(g, f, ib, q, q, q1, 0.0, 1.0, st, p);
         })))
        return rc;
    if ((rc = enqueue_stage(c, t + dt, s, [&](hipStream_t st, const StagePart *p) {
             return launch_rk_stage(g, f, ib, q, q1, q2, 0.75, 0.25, st, p);
         })))
        return rc;
    return enqueue_stage(c, t + 0.5 * dt, s, [&](hipStream_t st, const StagePart *p) {
        return launch_rk_stage(g, f, ib, q, q2, q, 1.0 / 3.0, 2.0 / 3.0, st, p);
    });
}

// One physical dual-time step ending at tn: history rotation, then n_inner
// pseudo-iterations ping-ponging between q and the scratch state.
int enqueue_dual_step(ibm_ctx *c, double *q, double tn, int first, hipStream_t s)
{
    int rc;
    if ((rc = dev_err(c, launch_dual_begin(c->g, c->f, q, c->qn, c->qnm1, first, s), "dual begin")))
        return rc;
    double b0 = first ? 1.0 : 1.5, b2 = first ? 0.0 : 0.5;
    double *cur = q, *nxt = c->wtmp;
    const Grid &g = c->g;
    const Flow &f = c->f;
    const IB &ib = c->ib;
    for (int it = 0; it < c->n_inner; ++it) {
        double *in = cur, *out = nxt;
        if ((rc = enqueue_stage(c, tn, s, [&](hipStream_t st, const StagePart *p) {
                 return launch_dual_iter(g, f, ib, in, out, c->qn, c->qnm1, b0, b2, st, p);
             })))
            return rc;
        cur = out;
        nxt = in;
    }
    if (cur != q)
        return dev_err(c, launch_copy_state(c->g, cur, q, s), "copy");
    return IBM_OK;
}

// Write the device argument blocks of every stage launch of a step of a
// stationary-body solve on state q (see ibm_ctx::d_args).
int prepare_batch(ibm_ctx *c, double *q, hipStream_t s)
{
    size_t nb = stage_args_bytes();
    c->h_args.assign(kSlots * nb, 0);
    bool body = c->b.nfacet > 0 && c->ib.cap > 0;
    StagePart p = stage_part(c, 0.0, 0.0, -1);
    if (c->prefill) {
        p.tiles = nullptr;
        p.ntiles = 0;
    }
    // launch 0 of a stage is the plain kernel (solves without a body, and
    // 3D FP64 ones with a body after the fill of their input, c->slot_qin),
    // launch 1 the kernel with the inline IB fill (other solves with a body)
    auto put = [&](int slot, int launch, double *qin, const double *qn, const double *qnm1, double *out,
                   double a, double b) {
        const StagePart *part = body ? &p : nullptr;
        c->slot_qin[slot] = qin;
        if ((body && !c->prefill) != (launch == 1)) {
            c->slot_nblk[slot] = 0;
            return;
        }
        c->slot_nblk[slot] = stage_args(c->g, c->f, c->ib, qin, qn, qnm1, out, a, b, part, &c->h_args[slot * nb]);
    };
    for (int k = 0; k < kSlots; ++k)
        c->slot_nblk[k] = 0;
    if (c->f.scheme == IBM_RK3) {
        static const double A[3] = {0.0, 0.75, 1.0 / 3.0}, B[3] = {1.0, 0.25, 2.0 / 3.0};
        double *in[3] = {q, c->q1, c->q2}, *out[3] = {c->q1, c->q2, q};
        for (int st = 0; st < 3; ++st)
            for (int l = 0; l < 2; ++l)
                put(2 * st + l, l, in[st], q, nullptr, out[st], A[st], B[st]);
    } else {
        for (int first = 0; first < 2; ++first)
            for (int par = 0; par < 2; ++par)
                for (int l = 0; l < 2; ++l) {
                    double *in = par == 0 ? q : c->wtmp, *out = par == 0 ? c->wtmp : q;
                    put(4 * first + 2 * par + l, l, in, c->qn, c->qnm1, out, first ? 1.0 : 1.5, first ? 0.0 : 0.5);
                }
    }
    hipError_t e = hipMemcpyAsync(c->d_args, c->h_args.data(), c->h_args.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return dev_err(c, e, "batch arguments");
    c->batch_q = q;
    return IBM_OK;
}

// One step of a group of stationary-body solves that share ndim, precision
// and scheme (their launch arguments prepared by prepare_batch): each stage
// launch of all of them is one batched launch.  Every stationary advance
// path (eager, graph replay, batched serving) goes through here, so they
// run the same kernels on the same arguments.  Time and step counters are
// left to the caller.
int enqueue_group_step(ibm_ctx *const *ctx, double *const *q, const std::vector<int> &gp, hipStream_t s)
{
    const ibm_ctx *c0 = ctx[gp[0]];
    int nd = c0->g.ndim, prec = c0->f.precision, scheme = c0->f.scheme;
    size_t nb = stage_args_bytes();
    std::vector<const void *> args[2];
    std::vector<int> nblk[2];
    auto run = [&](auto slot_of) -> int {
        int tot[2] = {0, 0};
        for (int l = 0; l < 2; ++l) {
            args[l].clear();
            nblk[l].clear();
            for (int m : gp) {
                int slot = slot_of(ctx[m]);
                if (slot < 0)
                    continue;
                args[l].push_back(static_cast<char *>(ctx[m]->d_args) + (slot + l) * nb);
                nblk[l].push_back(ctx[m]->slot_nblk[slot + l]);
                tot[l] += std::max(ctx[m]->slot_nblk[slot + l], 0);
            }
        }
        // the stage timer of a single solve times each stage: from the start
        // of its first non-empty launch (a prefill solve's fill) to the end
        // of its last
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (gp.size() == 1 && tot[0] + tot[1] > 0)
            take_timing_pair(ctx[gp[0]], e0, e1);
        int first = tot[0] > 0 ? 0 : 1, last = tot[1] > 0 ? 1 : 0;
        for (int m : gp) {
            const ibm_ctx *c = ctx[m];
            int slot = slot_of(c);
            if (slot < 0 || !c->prefill || c->slot_nblk[slot] <= 0)
                continue;
            hipError_t e = launch_ib_fill(c->g, c->f, c->ib, c->slot_qin[slot], 0.0, 0.0, -1, s, e0);
            if (e != hipSuccess)
                return dev_err(ctx[gp[0]], e, "stage fill");
            e0 = nullptr;
        }
        for (int l = 0; l < 2; ++l) {
            hipError_t e = launch_stage_batch(nd, prec, scheme, l == 1, (int)args[l].size(), args[l].data(),
                                              nblk[l].data(), s, l == first ? e0 : nullptr, l == last ? e1 : nullptr);
            if (e != hipSuccess)
                return dev_err(ctx[gp[0]], e, "batched stage");
        }
        return IBM_OK;
    };
    int rc;
    if (scheme == IBM_RK3) {
        for (int st = 0; st < 3; ++st)
            if ((rc = run([&](const ibm_ctx *) { return 2 * st; })))
                return rc;
        return IBM_OK;
    }
    int most = 0;
    for (int m : gp) {
        ibm_ctx *c = ctx[m];
        most = std::max(most, c->n_inner);
        hipError_t e = launch_dual_begin(c->g, c->f, q[m], c->qn, c->qnm1, c->step == 0, s);
        if (e != hipSuccess)
            return dev_err(c, e, "dual begin");
    }
    for (int it = 0; it < most; ++it)
        if ((rc = run([&](const ibm_ctx *c) { return it < c->n_inner ? 4 * (c->step == 0) + 2 * (it % 2) : -1; })))
            return rc;
    for (int m : gp) {
        ibm_ctx *c = ctx[m];
        if (c->n_inner % 2 == 1) {
            hipError_t e = launch_copy_state(c->g, c->wtmp, q[m], s);
            if (e != hipSuccess)
                return dev_err(c, e, "copy");
        }
    }
    return IBM_OK;
}

// One step of a free body (section 6, eq.10): the force on the state at t^n
// (filled with the body's velocity and last acceleration), a = F / M, the
// RK3 stages with the body at x^n moving at u^n and accelerating at a, then
// the Verlet update with the 1/2 of its standard form.
int free_step(ibm_ctx *c, double *q, hipStream_t s)
{
    int rc;
    if ((rc = do_classify(c, c->t, s)))
        return rc;
    if ((rc = do_fill(c, q, c->t, s)))
        return rc;
    hipError_t e = hipMemsetAsync(c->fmissed, 0, sizeof(int32_t), s);
    if (e == hipSuccess)
        e = launch_forces(c->g, c->b, c->f, c->ib, q, c->fforce, nullptr, c->fpart, c->fmissed, s);
    double F[3] = {0.0, 0.0, 0.0};
    if (e == hipSuccess)
        e = hipMemcpyAsync(F, c->fforce, sizeof F, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if ((rc = dev_err(c, e, "free-body force")))
        return rc;
    double a = F[c->mo.axis] / c->mo.mass;
    if (!std::isfinite(a))
        return set_err(c, IBM_ENONFINITE, "free-body force is not finite");
    c->mo.a = a;
    c->mo.force = F[c->mo.axis];
    if ((rc = enqueue_rk3_step(c, q, c->t, s)))
        return rc;
    double dt = c->f.dt, x = c->mo.x, u = c->mo.u;
    {
#pragma clang fp contract(off)
        c->mo.x = x + u * dt + 0.5 * dt * dt * a;
        c->mo.u = u + dt * a;
    }
    return IBM_OK;
}

// Steps per chunk graph: RK3 steps are 9 launches, dual-time steps 3 n_inner + 1.
int chunk_steps(const ibm_ctx *c) { return c->f.scheme == IBM_RK3 ? 8 : 2; }

// Capture `slot` (0: one step, 1: a chunk of steps) of a stationary-body solve
// into a graph, on a private stream (the caller's stream may be the legacy
// default stream, which cannot be captured).  Returns false if capture is
// unavailable; the caller then enqueues eagerly.
bool build_graph(ibm_ctx *c, double *q, int slot)
{
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c->cap_stream = nullptr;
        return false;
    }
    if (c->graph_exec[slot])
        (void)hipGraphExecDestroy(c->graph_exec[slot]);
    if (c->graph[slot])
        (void)hipGraphDestroy(c->graph[slot]);
    c->graph_exec[slot] = nullptr;
    c->graph[slot] = nullptr;
    c->graph_q[slot] = nullptr;
    int nsteps = slot == 0 ? 1 : chunk_steps(c);
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return false;
    int rc = IBM_OK;
    ibm_ctx *one[1] = {c};
    double *qs[1] = {q};
    const std::vector<int> gp{0};
    for (int n = 0; n < nsteps && rc == IBM_OK; ++n)
        rc = enqueue_group_step(one, qs, gp, c->cap_stream);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &gr);
    if (rc != IBM_OK || e != hipSuccess || !gr) {
        if (gr)
            (void)hipGraphDestroy(gr);
        (void)hipGetLastError();
        return false;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(gr);
        (void)hipGetLastError();
        return false;
    }
    c->graph[slot] = gr;
    c->graph_exec[slot] = ex;
    c->graph_q[slot] = q;
    return true;
}

}  // namespace

extern "C" {

int ibm_advance(ibm_ctx *c, double *q, int nsteps, void *stream)
{
    if (!c || !q || nsteps < 0)
        return IBM_EINVAL;
    hipStream_t s = S(stream);
    int rc;
    double dt = c->f.dt;
    for (int n = 0; n < nsteps;) {
        if (c->mo.free) {
            if ((rc = free_step(c, q, s)))
                return rc;
            c->t += dt;
            c->step += 1;
            n += 1;
            continue;
        }
        bool rk = c->f.scheme == IBM_RK3;
        // moving bodies are posed at t^n (RK3) or t^{n+1} (dual time)
        double tpose = rk ? c->t : c->t + dt;
        int nxt = -1;
        if (c->mo.on) {
            // this step's classification: prefetched by the previous step on
            // the side stream (wait for it), or done now on the stream
            int k = c->cur;
            if (c->buf_ok[k] && c->buf_t[k] == tpose) {
                if (c->buf_side[k]) {
                    if ((rc = dev_err(c, hipStreamWaitEvent(s, c->ev_ready[k], 0), "pipeline join")))
                        return rc;
                    c->buf_side[k] = false;
                }
                c->ib = c->ibb[k];
                c->classified = true;
            } else if ((rc = do_classify(c, tpose, s))) {
                return rc;
            }
            // the next step's, into the other buffer, while this step's stages
            // run: the side stream starts once this step's classification
            // is ready (and with it the stages of the previous step, the last
            // readers of the other buffer, are done)
            if (c->nbuf == 2 && c->pipeline && n + 1 < nsteps) {
                if ((rc = ensure_side(c)))
                    return rc;
                nxt = k ^ 1;
                hipError_t e = hipEventRecord(c->ev_fork, s);
                if (e == hipSuccess)
                    e = hipStreamWaitEvent(c->side, c->ev_fork, 0);
                if ((rc = dev_err(c, e, "pipeline fork")))
                    return rc;
                if ((rc = classify_buf(c, nxt, tpose + dt, c->side)))
                    return rc;
                if ((rc = dev_err(c, hipEventRecord(c->ev_ready[nxt], c->side), "pipeline event")))
                    return rc;
                c->buf_side[nxt] = true;
            }
        } else if (!c->classified && (rc = do_classify(c, tpose, s))) {
            return rc;
        }
        int first = !rk && c->step == 0;
        int k = 1;
        // stationary bodies: the shared batched path on prepared arguments
        if (!c->mo.on && c->batch_q != q && (rc = prepare_batch(c, q, s)))
            return rc;
        // graph replay, unless the stage timer is on (its events go with
        // eager launches)
        bool graphable = c->use_graphs && !c->mo.on && !first && c->tev.empty();
        if (graphable) {
            int slot = nsteps - n >= chunk_steps(c) ? 1 : 0;
            if (c->graph_q[slot] != q && !build_graph(c, q, slot))
                graphable = false;
            else {
                if ((rc = dev_err(c, hipGraphLaunch(c->graph_exec[slot], s), "graph launch")))
                    return rc;
                k = slot == 1 ? chunk_steps(c) : 1;
            }
        }
        if (!graphable) {
            ibm_ctx *one[1] = {c};
            double *qs[1] = {q};
            if (!c->mo.on)
                rc = enqueue_group_step(one, qs, std::vector<int>{0}, s);
            else if (rk)
                rc = enqueue_rk3_step(c, q, c->t, s);
            else
                rc = enqueue_dual_step(c, q, c->t + dt, first, s);
            if (rc)
                return rc;
        }
        c->t += k * dt;
        c->step += k;
        n += k;
        if (nxt >= 0)
            c->cur = nxt;
    }
    return IBM_OK;
}

int ibm_batch_advance(ibm_ctx *const *ctx, double *const *q, int n, int nsteps, void *stream)
{
    if (!ctx || !q || n < 0 || n > IBM_BATCH_MAX || nsteps < 0)
        return IBM_EINVAL;
    hipStream_t s = S(stream);
    int dev = -1;
    for (int m = 0; m < n; ++m) {
        if (!ctx[m] || !q[m])
            return IBM_EINVAL;
        if (m == 0)
            dev = ctx[m]->device;
        else if (ctx[m]->device != dev)
            return set_err(ctx[m], IBM_EINVAL, "batched contexts must share one device");
        for (int k = 0; k < m; ++k)
            if (ctx[k] == ctx[m])
                return set_err(ctx[m], IBM_EINVAL, "a context appears twice in a batch");
    }
    // moving bodies are reclassified every step: they advance on their own
    std::vector<int> batched;
    for (int m = 0; m < n; ++m) {
        ibm_ctx *c = ctx[m];
        int rc;
        if (c->mo.on) {
            if ((rc = ibm_advance(c, q[m], nsteps, stream)))
                return rc;
            continue;
        }
        if (!c->classified && (rc = do_classify(c, c->t, s)))
            return rc;
        if (c->batch_q != q[m] && (rc = prepare_batch(c, q[m], s)))
            return rc;
        batched.push_back(m);
    }
    // groups sharing a kernel: (ndim, precision, scheme)
    std::vector<std::vector<int>> groups;
    for (int m : batched) {
        bool placed = false;
        for (auto &gp : groups) {
            const ibm_ctx *a = ctx[gp[0]], *b = ctx[m];
            if (a->g.ndim == b->g.ndim && a->f.precision == b->f.precision && a->f.scheme == b->f.scheme) {
                gp.push_back(m);
                placed = true;
                break;
            }
        }
        if (!placed)
            groups.push_back({m});
    }
    for (int step = 0; step < nsteps; ++step)
        for (auto &gp : groups) {
            int rc = enqueue_group_step(ctx, q, gp, s);
            if (rc)
                return rc;
            for (int m : gp) {
                ctx[m]->t += ctx[m]->f.dt;
                ctx[m]->step++;
            }
        }
    return IBM_OK;
}

int ibm_init_state(ibm_ctx *c, const double *prim, double *q, void *stream)
{
    if (!c || !prim || !q)
        return IBM_EINVAL;
    return dev_err(c, launch_prim_to_state(c->g, c->f, prim, q, S(stream)), "init state");
}

int ibm_state_to_prim(ibm_ctx *c, const double *q, double *prim, void *stream)
{
    if (!c || !prim || !q)
        return IBM_EINVAL;
    return dev_err(c, launch_state_to_prim(c->g, c->f, q, prim, S(stream)), "state to prim");
}

int ibm_read_counts(ibm_ctx *c, int32_t *host_counts, void *stream)
{
    if (!c || !host_counts)
        return IBM_EINVAL;
    hipError_t e = hipMemcpyAsync(host_counts, c->ib.counts, sizeof(int32_t) * CNT_WORDS,
                                  hipMemcpyDeviceToHost, S(stream));
    if (e == hipSuccess)
        e = hipStreamSynchronize(S(stream));
    return dev_err(c, e, "read counts");
}

int ibm_status(ibm_ctx *c, void *stream)
{
    if (!c)
        return IBM_EINVAL;
    int32_t cnt[CNT_WORDS];
    int rc = ibm_read_counts(c, cnt, stream);
    if (rc)
        return rc;
    if (cnt[CNT_STATUS] & ST_CAPACITY)
        return set_err(c, IBM_ECAPACITY, "more immersed-boundary nodes than the workspace holds");
    if (cnt[CNT_STATUS] & ST_NONFINITE)
        return set_err(c, IBM_ENONFINITE, "non-finite state or non-positive density in a fluid cell");
    return IBM_OK;
}

int ibm_info_get(const ibm_ctx *c, ibm_info *o)
{
    if (!c || !o)
        return IBM_EINVAL;
    o->ndim = c->g.ndim;
    o->ni = c->g.ni;
    o->nj = c->g.nj;
    o->nk = c->g.nk;
    o->nv = c->g.nv;
    o->state_elems = c->g.vs * c->g.nv;
    o->ncell = c->g.ncell;
    o->cap_nodes = c->ib.cap;
    for (int s = 0; s < 6; ++s)
        o->region[s] = c->ib.region[s];
    o->cls = c->ib.cls;
    o->counts = c->ib.counts;
    o->list_forcing = c->ib.listF;
    o->list_ghost = c->ib.listG;
    o->rec_int = c->ib.rec_i;
    o->rec_dbl = c->ib.rec_d;
    o->time = c->t;
    return IBM_OK;
}

const char *ibm_last_error(const ibm_ctx *c) { return c ? c->err : "null context"; }

int ibm_time_update_kernel(ibm_ctx *c, const double *q, int stage, int nrep, void *stream,
                           float *avg_ms)
{
    if (!c || !q || !avg_ms || nrep < 1)
        return IBM_EINVAL;
    hipStream_t s = S(stream);
    if (!c->classified) {
        int rc = do_classify(c, c->t, s);
        if (rc)
            return rc;
    }
    bool rk = c->f.scheme == IBM_RK3;
    if (rk && (stage < 1 || stage > 3))
        return IBM_EINVAL;
    // a pseudo-iteration reads the step history Q'^n, Q'^{n-1}, which the
    // solve's first step sets up; it is only read here
    if (!rk && c->step == 0)
        return set_err(c, IBM_EINVAL, "dual time: advance at least one step before timing a pseudo-iteration");
    static const double A[4] = {0.0, 0.0, 0.75, 1.0 / 3.0}, B[4] = {0.0, 1.0, 0.25, 2.0 / 3.0};
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    if (e != hipSuccess)
        return dev_err(c, e, "event create");
    // the kernel of the step's stage launches (batched form): with a body,
    // the tile list whose near tiles fill the IB nodes they read (the body
    // at the context time), else every tile.  d_q is only read; the output
    // goes to a scratch stage buffer (the filled FORCING corner values to
    // their scratch slots)
    // (3D FP64 with a body: the fill launches on a copy of d_q, c->qfill,
    // then the plain kernel over every tile, as in the step)
    size_t nb = stage_args_bytes();
    std::vector<char> h(nb);
    double *qm = const_cast<double *>(q);
    bool body = c->b.nfacet > 0 && c->ib.cap > 0;
    double disp = 0.0, vel = 0.0, acc = 0.0;
    if (c->mo.on)
        motion_kin(c, c->t, disp, vel, acc);
    int axis = c->mo.on ? c->mo.axis : -1;
    StagePart p = stage_part(c, vel, acc, axis);
    const StagePart *part = body ? &p : nullptr;
    if (c->prefill) {
        p.tiles = nullptr;
        p.ntiles = 0;
        qm = c->qfill;
        if (e == hipSuccess)
            e = hipMemcpyAsync(qm, q, sizeof(double) * (size_t)c->g.vs * c->g.nv, hipMemcpyDeviceToDevice, s);
    }
    int nblk = rk ? stage_args(c->g, c->f, c->ib, qm, q, nullptr, c->q1, A[stage], B[stage], part, h.data())
                  : stage_args(c->g, c->f, c->ib, qm, c->qn, c->qnm1, c->wtmp, 1.5, 0.5, part, h.data());
    const void *d = static_cast<char *>(c->d_args) + (kSlots - 1) * nb;
    bool ghosts = body && !c->prefill;
    if (e == hipSuccess)
        e = hipMemcpyAsync(const_cast<void *>(d), h.data(), nb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipEventRecord(e0, s);
    for (int r = 0; r < nrep && e == hipSuccess; ++r) {
        if (c->prefill)
            e = launch_ib_fill(c->g, c->f, c->ib, qm, vel, acc, axis, s, nullptr);
        if (e == hipSuccess)
            e = launch_stage_batch(c->g.ndim, c->f.precision, c->f.scheme, ghosts, 1, &d, &nblk, s);
    }
    if (e == hipSuccess)
        e = hipEventRecord(e1, s);
    if (e == hipSuccess)
        e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = ms / nrep;
    return dev_err(c, e, "time kernel");
}

int ibm_stage_timing(ibm_ctx *c, float *total_ms, int *launches, float *min_ms, float *max_ms)
{
    if (!c || !total_ms || !launches)
        return IBM_EINVAL;
    *total_ms = 0.0f;
    *launches = 0;
    float lo = 0.0f, hi = 0.0f;
    hipError_t e = hipSuccess;
    if (c->tev_used > 0)
        e = hipEventSynchronize(c->tev[2 * c->tev_used - 1]);
    for (int k = 0; k < c->tev_used && e == hipSuccess; ++k) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, c->tev[2 * k], c->tev[2 * k + 1]);
        if (e != hipSuccess)
            break;
        *total_ms += ms;
        lo = k == 0 ? ms : std::min(lo, ms);
        hi = k == 0 ? ms : std::max(hi, ms);
        ++*launches;
    }
    c->tev_used = 0;
    if (min_ms)
        *min_ms = lo;
    if (max_ms)
        *max_ms = hi;
    return dev_err(c, e, "stage timing");
}

}  // extern "C"
