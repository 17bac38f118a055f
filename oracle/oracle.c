/*
 * CPU oracle for the all-speed sharp-interface immersed-boundary step of
 * Seshadri & De (arXiv 1912.11908).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU baseline; never by the product path.  Plain scalar FP64,
 * built with -O2 -ffp-contract=off (no FMA contraction, no fast-math).  Every
 * loop over cells takes one cell per iteration; OpenMP (if enabled) only
 * splits those loops, so results do not depend on the thread count.
 *
 * Each function cites the paper passage it follows; where the paper names a
 * method without writing it out, the function states the reading it uses.
 */
/* Scalar type of the flow half (fills, residual, updates): ORC_REAL_KIND 0
 * double (the oracle), 1 long double, 2 __float128 (builds with less
 * rounding for low-Mach parity: same arithmetic, loops and order).  Arrays
 * that cross the interface (states, residuals, primitives, records) stay
 * double; the dual-time history arrays take the scalar type. */
#ifndef ORC_REAL_KIND
#define ORC_REAL_KIND 0
#endif
#if ORC_REAL_KIND == 2
#include <quadmath.h>
#define ORC_REAL __float128
#define RSQRT sqrtq
#define RFABS fabsq
#define RFLOOR floorq
#define RFMIN fminq
#define RFMAX fmaxq
#elif ORC_REAL_KIND == 1
#define ORC_REAL long double
#define RSQRT sqrtl
#define RFABS fabsl
#define RFLOOR floorl
#define RFMIN fminl
#define RFMAX fmaxl
#else
#define ORC_REAL double
#define RSQRT sqrt
#define RFABS fabs
#define RFLOOR floor
#define RFMIN fmin
#define RFMAX fmax
#endif

#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LAT_SCALE 16777216.0 /* 2^24: the integer lattice for exact predicates */
#define WENO_EPS 1.0e-6
#define MAXFEAT 32
#define IREC 24
#define DREC 32

typedef long long i64;
typedef orc_real real;

struct orc {
    int ndim, ni, nj, nk, nv, hz;
    int sx, sy, sz;     /* extended sizes */
    long vstride;       /* doubles per variable in a state array */
    double *xf, *yf, *zf; /* extended faces, index f + 3 (f = -3 .. n + 3) */
    double *xc, *yc, *zc; /* extended centres, index i + 3 */
    i64 *Xc, *Yc, *Zc;    /* lattice centres, interior */
    int bc[6];
    /* body */
    int nvert, nfacet;
    i64 *V0, *V;        /* lattice vertices at rest / posed */
    double *v;          /* posed vertices (exact V / 2^24) */
    int *facet;
    double *fnrm;       /* facet outward unit normals */
    double *vnrm;       /* vertex pseudo-normals */
    int *edge_of;       /* 3D: per facet edge, global edge id */
    double *enrm;       /* 3D: edge pseudo-normals per global edge */
    double *fcurv, *vcurv; /* 2D: signed curvature per segment / vertex (eq.7) */
    int nedge;
    /* flow */
    double gamma, mach, re, pr, R, cp, mu, kc, pinf, uc2;
    int scheme, family;
    double dt, cfl_tau;
    int n_inner;
    int motion, maxis;
    double mamp, mfreq, mphase, mvel;
    double bx, bu, ba;    /* free body (motion 2): displacement, velocity, acceleration */
    double uinf[3];       /* free-stream velocity */
    int wallp;            /* ORC_WALL_EQ6 / ORC_WALL_EQ7 */
    int recon;            /* ORC_RECON_WENO5 / ORC_RECON_TVD2 */
    int frame;            /* ORC_FRAME_RTLN / ORC_FRAME_SDSN */
    i64 disp;
    /* classification */
    uint8_t *cls, *cls_prev;
    int have_prev;
    int nF, nG, nG1, nG2, nG3;
    int32_t *listF, *listG;
    int32_t *irec;
    double *drec;
    /* statistics */
    i64 stat_fallback_pprime, stat_fallback_probe, stat_fallback_none;
    i64 stat_stencil_violation, stat_fresh_cleared, stat_fresh_violation;
    int dual_first_done;
};

/* ------------------------------------------------------------------ indexing */
static long sidx(const orc *o, int i, int j, int k)
{
    return ((long)(k + o->hz) * o->sy + (j + 3)) * o->sx + (i + 3);
}
static long cidx(const orc *o, int i, int j, int k)
{
    return ((long)k * o->nj + j) * o->ni + i;
}

/* -------------------------------------------------------------- set-up / grid */
/* Extended face coordinates: periodic axes use the periodic images of the
 * opposite end; the other axes mirror the first/last interior cells. */
static double *extend_faces(const double *f, int n, int periodic)
{
    double *e = (double *)malloc(sizeof(double) * (n + 7));
    for (int i = 0; i <= n; i++)
        e[i + 3] = f[i];
    for (int k = 1; k <= 3; k++) {
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

static double *centres(const double *e, int n)
{
    double *c = (double *)malloc(sizeof(double) * (n + 6));
    for (int i = 0; i < n + 6; i++)
        c[i] = 0.5 * (e[i] + e[i + 1]);
    return c;
}

static i64 *lattice_centres(const double *c, int n)
{
    i64 *L = (i64 *)malloc(sizeof(i64) * (n > 0 ? n : 1));
    for (int i = 0; i < n; i++)
        L[i] = llrint(c[i + 3] * LAT_SCALE);
    return L;
}

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void normalize3(double *a)
{
    double l = sqrt(dot3(a, a));
    if (l > 0.0) {
        a[0] /= l;
        a[1] /= l;
        a[2] /= l;
    }
}

/* Facet normals and pseudo-normals (section 4.2, eqs 2 and 3).
 * 2D: segment a->b of a counter-clockwise polygon has outward normal
 *     (b_y - a_y, -(b_x - a_x)) / |b - a|; a polygon vertex is the planar
 *     image of an extruded edge, so it takes the edge rule of eq.3, read as
 *     normalised: (n1 + n2) / |n1 + n2|.
 * 3D: triangle normal (b - a) x (c - a) normalised; vertex pseudo-normal is
 *     the incident-angle-weighted sum of incident facet normals (eq.2), the
 *     angle being acos of the clamped cosine between the two incident edges;
 *     edge pseudo-normal (eq.3) weights both incident facets by pi, i.e. the
 *     normalised sum; an edge with a single incident facet takes its normal. */
static int edge_cmp(const void *pa, const void *pb)
{
    const i64 *a = (const i64 *)pa, *b = (const i64 *)pb;
    if (a[0] != b[0])
        return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1])
        return a[1] < b[1] ? -1 : 1;
    return 0;
}

static void body_normals(orc *o)
{
    int nd = o->ndim;
    free(o->fnrm);
    free(o->vnrm);
    o->fnrm = (double *)calloc((size_t)(o->nfacet > 0 ? o->nfacet : 1) * 3, sizeof(double));
    o->vnrm = (double *)calloc((size_t)(o->nvert > 0 ? o->nvert : 1) * 3, sizeof(double));
    if (nd == 2) {
        for (int f = 0; f < o->nfacet; f++) {
            const double *a = o->v + 2 * o->facet[2 * f], *b = o->v + 2 * o->facet[2 * f + 1];
            double ex = b[0] - a[0], ey = b[1] - a[1], l = sqrt(ex * ex + ey * ey);
            o->fnrm[3 * f] = ey / l;
            o->fnrm[3 * f + 1] = -ex / l;
            o->fnrm[3 * f + 2] = 0.0;
        }
        for (int f = 0; f < o->nfacet; f++)
            for (int e = 0; e < 2; e++) {
                int vid = o->facet[2 * f + e];
                o->vnrm[3 * vid] += o->fnrm[3 * f];
                o->vnrm[3 * vid + 1] += o->fnrm[3 * f + 1];
            }
        for (int vtx = 0; vtx < o->nvert; vtx++)
            normalize3(o->vnrm + 3 * vtx);
        /* curvature for eq.7 (reading): the turn of the unit vertex normals
         * along a segment over its length, (n_b - n_a).(b - a) / |b - a|^2,
         * exactly 1/r on a regular polygon inscribed in a circle of radius r,
         * positive where the surface bends away from the fluid (convex); a
         * vertex takes the mean of its two segments */
        free(o->fcurv);
        free(o->vcurv);
        o->fcurv = (double *)calloc((size_t)(o->nfacet > 0 ? o->nfacet : 1), sizeof(double));
        o->vcurv = (double *)calloc((size_t)(o->nvert > 0 ? o->nvert : 1), sizeof(double));
        for (int f = 0; f < o->nfacet; f++) {
            int ia = o->facet[2 * f], ib = o->facet[2 * f + 1];
            const double *a = o->v + 2 * ia, *b = o->v + 2 * ib;
            double ex = b[0] - a[0], ey = b[1] - a[1];
            double dn = (o->vnrm[3 * ib] - o->vnrm[3 * ia]) * ex + (o->vnrm[3 * ib + 1] - o->vnrm[3 * ia + 1]) * ey;
            o->fcurv[f] = dn / (ex * ex + ey * ey);
        }
        for (int f = 0; f < o->nfacet; f++)
            for (int e = 0; e < 2; e++)
                o->vcurv[o->facet[2 * f + e]] += 0.5 * o->fcurv[f];
        return;
    }
    for (int f = 0; f < o->nfacet; f++) {
        const int *t = o->facet + 3 * f;
        const double *a = o->v + 3 * t[0], *b = o->v + 3 * t[1], *c = o->v + 3 * t[2];
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        cross3(e1, e2, o->fnrm + 3 * f);
        normalize3(o->fnrm + 3 * f);
        for (int m = 0; m < 3; m++) {
            const double *p = o->v + 3 * t[m], *q = o->v + 3 * t[(m + 1) % 3],
                         *r = o->v + 3 * t[(m + 2) % 3];
            double u[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
            double w[3] = {r[0] - p[0], r[1] - p[1], r[2] - p[2]};
            double cs = dot3(u, w) / (sqrt(dot3(u, u)) * sqrt(dot3(w, w)));
            if (cs > 1.0)
                cs = 1.0;
            if (cs < -1.0)
                cs = -1.0;
            double ang = acos(cs);
            for (int d = 0; d < 3; d++)
                o->vnrm[3 * t[m] + d] += ang * o->fnrm[3 * f + d];
        }
    }
    for (int vtx = 0; vtx < o->nvert; vtx++)
        normalize3(o->vnrm + 3 * vtx);
    /* edge adjacency: sort (min vid, max vid, facet, local edge) keys */
    int nh = 3 * o->nfacet;
    i64 *keys = (i64 *)malloc(sizeof(i64) * 4 * (nh > 0 ? nh : 1));
    for (int f = 0; f < o->nfacet; f++)
        for (int m = 0; m < 3; m++) {
            int p = o->facet[3 * f + m], q = o->facet[3 * f + (m + 1) % 3];
            i64 *k = keys + 4 * (3 * f + m);
            k[0] = p < q ? p : q;
            k[1] = p < q ? q : p;
            k[2] = f;
            k[3] = m;
        }
    qsort(keys, nh, sizeof(i64) * 4, edge_cmp);
    free(o->edge_of);
    free(o->enrm);
    o->edge_of = (int *)malloc(sizeof(int) * (nh > 0 ? nh : 1));
    o->enrm = (double *)calloc((size_t)(nh > 0 ? nh : 1) * 3, sizeof(double));
    int ne = 0;
    for (int s = 0; s < nh;) {
        int e = s;
        while (e < nh && keys[4 * e] == keys[4 * s] && keys[4 * e + 1] == keys[4 * s + 1])
            e++;
        for (int m = s; m < e; m++) {
            int f = (int)keys[4 * m + 2];
            o->edge_of[3 * f + keys[4 * m + 3]] = ne;
            for (int d = 0; d < 3; d++)
                o->enrm[3 * ne + d] += M_PI * o->fnrm[3 * f + d];
        }
        normalize3(o->enrm + 3 * ne);
        ne++;
        s = e;
    }
    o->nedge = ne;
    free(keys);
}

orc *orc_create(int ndim, int ni, int nj, int nk, const double *xf, const double *yf,
                const double *zf, const int *bc, int nvert, int nfacet, const double *vert,
                const int *facet, double mach, double re, double pr, double gamma, int scheme,
                int family, double dt, double cfl_tau, int n_inner, int motion,
                const double *mpar, const double *uinf, int wall_pressure, int reconstruction,
                int framework)
{
    orc *o = (orc *)calloc(1, sizeof(orc));
    o->ndim = ndim;
    o->ni = ni;
    o->nj = nj;
    o->nk = ndim == 3 ? nk : 1;
    o->nv = ndim + 2;
    o->hz = ndim == 3 ? 3 : 0;
    o->sx = ni + 6;
    o->sy = nj + 6;
    o->sz = o->nk + 2 * o->hz;
    o->vstride = (long)o->sx * o->sy * o->sz;
    memcpy(o->bc, bc, sizeof(int) * 6);
    o->xf = extend_faces(xf, ni, bc[0] == ORC_BC_PERIODIC);
    o->yf = extend_faces(yf, nj, bc[2] == ORC_BC_PERIODIC);
    if (ndim == 3)
        o->zf = extend_faces(zf, nk, bc[4] == ORC_BC_PERIODIC);
    else {
        o->zf = (double *)malloc(sizeof(double) * 8);
        for (int i = 0; i < 8; i++)
            o->zf[i] = (double)(i - 3) - 0.5; /* unit depth: dz = 1 */
    }
    o->xc = centres(o->xf, ni);
    o->yc = centres(o->yf, nj);
    o->zc = centres(o->zf, ndim == 3 ? nk : 1);
    o->Xc = lattice_centres(o->xc, ni);
    o->Yc = lattice_centres(o->yc, nj);
    o->Zc = lattice_centres(o->zc, ndim == 3 ? nk : 1);

    o->nvert = nvert;
    o->nfacet = nfacet;
    o->V0 = (i64 *)malloc(sizeof(i64) * (size_t)(nvert > 0 ? nvert : 1) * ndim);
    o->V = (i64 *)malloc(sizeof(i64) * (size_t)(nvert > 0 ? nvert : 1) * ndim);
    o->v = (double *)malloc(sizeof(double) * (size_t)(nvert > 0 ? nvert : 1) * ndim);
    for (long m = 0; m < (long)nvert * ndim; m++) {
        o->V0[m] = llrint(vert[m] * LAT_SCALE);
        o->V[m] = o->V0[m];
        o->v[m] = (double)o->V[m] / LAT_SCALE;
    }
    o->facet = (int *)malloc(sizeof(int) * (size_t)(nfacet > 0 ? nfacet : 1) * ndim);
    memcpy(o->facet, facet, sizeof(int) * (size_t)nfacet * ndim);

    /* c.0 reading: rho_inf = T_inf = L = 1 and unit reference speed (the
     * free stream's, or the body's in still fluid), so p_inf = R = 1/(gamma M^2);
     * constant mu = 1/Re, Pr fixed, Stokes hypothesis. */
    for (int d = 0; d < 3; d++)
        o->uinf[d] = uinf[d];
    o->wallp = wall_pressure;
    o->recon = reconstruction;
    o->frame = framework;
    o->gamma = gamma;
    o->mach = mach;
    o->re = re;
    o->pr = pr;
    o->pinf = 1.0 / (gamma * mach * mach);
    o->R = o->pinf;
    o->cp = gamma * o->R / (gamma - 1.0);
    o->mu = 1.0 / re;
    o->kc = o->mu * o->cp / pr;
    o->scheme = scheme;
    o->family = family;
    o->dt = dt;
    o->cfl_tau = cfl_tau;
    o->n_inner = n_inner;
    /* preconditioning cut-off velocity^2: max(U_inf^2, (nu/h)^2, (h/(pi dt))^2) */
    {
        double hmin = 1e300;
        for (int i = 0; i < ni; i++)
            hmin = fmin(hmin, xf[i + 1] - xf[i]);
        for (int j = 0; j < nj; j++)
            hmin = fmin(hmin, yf[j + 1] - yf[j]);
        if (ndim == 3)
            for (int k = 0; k < nk; k++)
                hmin = fmin(hmin, zf[k + 1] - zf[k]);
        double a2 = o->uinf[0] * o->uinf[0] + o->uinf[1] * o->uinf[1] + o->uinf[2] * o->uinf[2];
        double b = o->mu / hmin, c = hmin / (M_PI * dt);
        o->uc2 = fmax(a2, fmax(b * b, c * c));
    }
    o->motion = motion;
    if (motion) {
        o->maxis = (int)mpar[0];
        o->mamp = mpar[1];
        o->mfreq = mpar[2];
        o->mphase = mpar[3];
        o->mvel = mpar[4];
    }
    long ncell = (long)ni * nj * o->nk;
    o->cls = (uint8_t *)calloc(ncell, 1);
    o->cls_prev = (uint8_t *)calloc(ncell, 1);
    o->listF = (int32_t *)malloc(sizeof(int32_t) * (ncell + 1));
    o->listG = (int32_t *)malloc(sizeof(int32_t) * (ncell + 1));
    body_normals(o);
    return o;
}

void orc_destroy(orc *o)
{
    if (!o)
        return;
    free(o->xf); free(o->yf); free(o->zf);
    free(o->xc); free(o->yc); free(o->zc);
    free(o->Xc); free(o->Yc); free(o->Zc);
    free(o->V0); free(o->V); free(o->v); free(o->facet);
    free(o->fnrm); free(o->vnrm); free(o->edge_of); free(o->enrm); free(o->fcurv); free(o->vcurv);
    free(o->cls); free(o->cls_prev); free(o->listF); free(o->listG);
    free(o->irec); free(o->drec);
    free(o);
}

/* ------------------------------------------------------------------ a1 pose */
/* Prescribed translation along one axis, y(t) = A cos(2 pi f t + phase)
 * (section 8.2.2 motion law).  The displacement is snapped to the lattice and
 * added to the integer vertices, so posed coordinates stay exact. */
/* x_axis(t) = A cos(2 pi f t + phase) + V t: the oscillation of section 8.2.2
 * plus a constant speed (section 8.2.3).  A free body (motion 2, section 6)
 * has the displacement, velocity and acceleration its driver last set. */
static double pose_disp(const orc *o, double t)
{
    if (o->motion == 2)
        return o->bx;
    return o->mamp * cos(2.0 * M_PI * o->mfreq * t + o->mphase) + o->mvel * t;
}
static double pose_vel(const orc *o, double t)
{
    if (o->motion == 2)
        return o->bu;
    return -2.0 * M_PI * o->mfreq * o->mamp * sin(2.0 * M_PI * o->mfreq * t + o->mphase) + o->mvel;
}
static double pose_acc(const orc *o, double t)
{
    if (o->motion == 2)
        return o->ba;
    double w = 2.0 * M_PI * o->mfreq;
    return -w * w * o->mamp * cos(w * t + o->mphase);
}

void orc_set_body(orc *o, double x, double u, double a)
{
    o->bx = x;
    o->bu = u;
    o->ba = a;
}

void orc_set_pose(orc *o, double t)
{
    if (!o->motion)
        return;
    o->disp = llrint(pose_disp(o, t) * LAT_SCALE);
    for (int m = 0; m < o->nvert; m++)
        for (int d = 0; d < o->ndim; d++) {
            long q = (long)m * o->ndim + d;
            o->V[q] = o->V0[q] + (d == o->maxis ? o->disp : 0);
            o->v[q] = (double)o->V[q] / LAT_SCALE;
        }
    body_normals(o);
}

/* ------------------------------------------------------------ a2 classify */
/* Ray casting with crossing parity (section 3.2): a +x ray from the cell
 * centre; odd crossing count => inside (solid).  Readings: all decisions use
 * exact integer lattice coordinates; 2D: a segment counts iff
 * (a_y > p_y) != (b_y > p_y) and the crossing lies strictly to the right of
 * the node; 3D: a triangle counts iff (p_y, p_z) lies in its (y, z)
 * projection under the top-left tie rule and the crossing lies strictly
 * ahead in +x.  Nodes outside the body's axis-aligned box are fluid (the
 * parity there is always even, so the box is a pure shortcut). */
static int inside2d(const orc *o, i64 px, i64 py)
{
    int cnt = 0;
    for (int f = 0; f < o->nfacet; f++) {
        const i64 *a = o->V + 2 * o->facet[2 * f], *b = o->V + 2 * o->facet[2 * f + 1];
        if ((a[1] > py) == (b[1] > py))
            continue;
        i64 orient = (b[0] - a[0]) * (py - a[1]) - (b[1] - a[1]) * (px - a[0]);
        if (b[1] > a[1] ? orient > 0 : orient < 0)
            cnt++;
    }
    return cnt & 1;
}

/* top-left rule for a projected edge from P to Q of a triangle with positive
 * projected orientation: the edge owns its points iff it is a "top" edge
 * (horizontal, pointing in -y... in (y, z) coordinates: dz == 0 and dy < 0)
 * or a "left" edge (dz > 0). */
static int edge_owns(i64 dy, i64 dz) { return (dz == 0 && dy < 0) || dz > 0; }

static int inside3d(const orc *o, i64 px, i64 py, i64 pz)
{
    int cnt = 0;
    for (int f = 0; f < o->nfacet; f++) {
        const int *t = o->facet + 3 * f;
        const i64 *A = o->V + 3 * t[0], *B = o->V + 3 * t[1], *C = o->V + 3 * t[2];
        /* projected (y, z) orientation of the triangle */
        i64 area = (B[1] - A[1]) * (C[2] - A[2]) - (B[2] - A[2]) * (C[1] - A[1]);
        if (area == 0)
            continue; /* parallel to the ray */
        const i64 *P[3] = {A, B, C};
        if (area < 0) { /* make the projected orientation positive */
            P[1] = C;
            P[2] = B;
        }
        int ok = 1;
        i64 w[3];
        for (int m = 0; m < 3 && ok; m++) {
            const i64 *p = P[m], *q = P[(m + 1) % 3];
            i64 dy = q[1] - p[1], dz = q[2] - p[2];
            w[m] = dy * (pz - p[2]) - dz * (py - p[1]);
            if (w[m] < 0 || (w[m] == 0 && !edge_owns(dy, dz)))
                ok = 0;
        }
        if (!ok)
            continue;
        /* crossing x* > px  <=>  sum_m w[m] * (x_opp(m) - px) > 0, where
         * w[m] is the edge function of edge m and x_opp(m) the x of the
         * vertex opposite that edge (barycentric interpolation of x). */
        __int128 s = 0;
        for (int m = 0; m < 3; m++) {
            const i64 *opp = P[(m + 2) % 3];
            s += (__int128)w[m] * (__int128)(opp[0] - px);
        }
        if (s > 0)
            cnt++;
    }
    return cnt & 1;
}

static void body_box(const orc *o, i64 *lo, i64 *hi)
{
    for (int d = 0; d < 3; d++) {
        lo[d] = (i64)1 << 62;
        hi[d] = -((i64)1 << 62);
    }
    for (int m = 0; m < o->nvert; m++)
        for (int d = 0; d < o->ndim; d++) {
            i64 c = o->V[(long)m * o->ndim + d];
            if (c < lo[d]) lo[d] = c;
            if (c > hi[d]) hi[d] = c;
        }
}

/* a3 tagging (section 3.2, last paragraph; section 5).  Reading: FORCING =
 * fluid cell with a solid face neighbour; G1 = solid cell with a FORCING
 * face neighbour; G2 / G3 = further face-neighbour layers into the solid
 * (three ghost layers for WENO5); the remaining solid cells are SOLID.
 * Neighbours across a periodic boundary wrap; across any other domain
 * boundary they count as fluid. */
static int nbr(const orc *o, int i, int j, int k, int d, int s, long *out)
{
    int c[3] = {i, j, k}, n[3] = {o->ni, o->nj, o->nk};
    c[d] += s;
    if (c[d] < 0 || c[d] >= n[d]) {
        if (o->bc[2 * d] != ORC_BC_PERIODIC)
            return 0;
        c[d] = (c[d] + n[d]) % n[d];
    }
    *out = cidx(o, c[0], c[1], c[2]);
    return 1;
}

static int sd_inside(const orc *o, const double *X);

int orc_classify(orc *o)
{
    long ncell = (long)o->ni * o->nj * o->nk;
    memcpy(o->cls_prev, o->cls, ncell);
    int had_prev = o->have_prev;
    uint8_t *in = (uint8_t *)calloc(ncell, 1);
    i64 lo[3], hi[3];
    body_box(o, lo, hi);
    /* the predicates multiply lattice differences inside the body's box in
     * 64-bit integers: refuse a box too large for that */
    if (o->nfacet > 0) {
        double ext = 0.0;
        for (int d = 0; d < o->ndim; d++)
            ext = fmax(ext, (double)hi[d] - (double)lo[d]);
        if (2.0 * ext * ext >= 0x1p62) {
            free(in);
            return -2;
        }
    }
#pragma omp parallel for schedule(static)
    for (long c = 0; c < ncell; c++) {
        int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
        if (o->nfacet == 0)
            continue;
        i64 px = o->Xc[i], py = o->Yc[j];
        if (px < lo[0] || px > hi[0] || py < lo[1] || py > hi[1])
            continue;
        if (o->ndim == 3 && (o->Zc[k] < lo[2] || o->Zc[k] > hi[2]))
            continue;
        if (o->frame == ORC_FRAME_SDSN) {
            double X[3] = {o->xc[i + 3], o->yc[j + 3], o->ndim == 3 ? o->zc[k + 3] : 0.0};
            in[c] = (uint8_t)sd_inside(o, X);
        } else if (o->ndim == 2)
            in[c] = (uint8_t)inside2d(o, px, py);
        else
            in[c] = (uint8_t)inside3d(o, px, py, o->Zc[k]);
    }
    /* tagging */
    for (long c = 0; c < ncell; c++)
        o->cls[c] = in[c] ? ORC_SOLID : ORC_FLUID;
    for (long c = 0; c < ncell; c++) {
        if (in[c])
            continue;
        int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
        for (int d = 0; d < o->ndim; d++)
            for (int s = -1; s <= 1; s += 2) {
                long q;
                if (nbr(o, i, j, k, d, s, &q) && in[q])
                    o->cls[c] = ORC_FORCING;
            }
    }
    for (int layer = 0; layer < 3; layer++) {
        uint8_t src = layer == 0 ? ORC_FORCING : (uint8_t)(ORC_G1 + layer - 1);
        uint8_t dst = (uint8_t)(ORC_G1 + layer);
        uint8_t *next = (uint8_t *)malloc(ncell);
        memcpy(next, o->cls, ncell);
        for (long c = 0; c < ncell; c++) {
            if (o->cls[c] != ORC_SOLID)
                continue;
            int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
            for (int d = 0; d < o->ndim; d++)
                for (int s = -1; s <= 1; s += 2) {
                    long q;
                    if (nbr(o, i, j, k, d, s, &q) && o->cls[q] == src)
                        next[c] = dst;
                }
        }
        memcpy(o->cls, next, ncell);
        free(next);
    }
    free(in);
    /* list compaction in raster order */
    o->nF = o->nG = o->nG1 = o->nG2 = o->nG3 = 0;
    for (long c = 0; c < ncell; c++) {
        uint8_t t = o->cls[c];
        if (t == ORC_FORCING)
            o->listF[o->nF++] = (int32_t)c;
        else if (t >= ORC_G1 && t <= ORC_G3) {
            o->listG[o->nG++] = (int32_t)c;
            if (t == ORC_G1) o->nG1++;
            if (t == ORC_G2) o->nG2++;
            if (t == ORC_G3) o->nG3++;
        }
    }
    /* moving bodies (section 5): a cell solid before and fluid now keeps the
     * state stored at its last fill; that needs it to have been a ghost. */
    if (had_prev)
        for (long c = 0; c < ncell; c++) {
            int was_in = o->cls_prev[c] >= ORC_G1;
            int is_fluid = o->cls[c] <= ORC_FORCING;
            if (was_in && is_fluid) {
                o->stat_fresh_cleared++;
                if (o->cls_prev[c] == ORC_SOLID)
                    o->stat_fresh_violation++;
            }
        }
    o->have_prev = 1;
    return 0;
}

/* --------------------------------------------------------- a4 geometry */
/* Closest feature (section 4.1): minimise the squared distance of eq.1 over
 * every facet (brute force; the bounding-sphere step of the paper is only an
 * acceleration).  The minimum squared distance wins, ties go to the lowest
 * facet id.  2D: the segment parameter t is clamped to [0, 1]; t <= 0 or
 * t >= 1 is a vertex feature, otherwise the segment itself (a "face"). */
enum { FEAT_FACE = 0, FEAT_VERTEX = 1, FEAT_EDGE = 2 };

typedef struct {
    int kind, id, facet;
    double c[3], d2;
} closest_t;

static closest_t closest2d(const orc *o, const double *p)
{
    closest_t best;
    best.d2 = INFINITY;
    best.kind = -1;
    best.id = -1;
    best.facet = -1;
    for (int f = 0; f < o->nfacet; f++) {
        int ia = o->facet[2 * f], ib = o->facet[2 * f + 1];
        const double *a = o->v + 2 * ia, *b = o->v + 2 * ib;
        double ex = b[0] - a[0], ey = b[1] - a[1];
        double t = ((p[0] - a[0]) * ex + (p[1] - a[1]) * ey) / (ex * ex + ey * ey);
        double cx, cy;
        int kind, id;
        if (t <= 0.0) {
            cx = a[0]; cy = a[1]; kind = FEAT_VERTEX; id = ia;
        } else if (t >= 1.0) {
            cx = b[0]; cy = b[1]; kind = FEAT_VERTEX; id = ib;
        } else {
            cx = a[0] + t * ex; cy = a[1] + t * ey; kind = FEAT_FACE; id = f;
        }
        double dx = p[0] - cx, dy = p[1] - cy, d2 = dx * dx + dy * dy;
        if (d2 < best.d2) {
            best.d2 = d2;
            best.kind = kind;
            best.id = id;
            best.facet = f;
            best.c[0] = cx;
            best.c[1] = cy;
            best.c[2] = 0.0;
        }
    }
    return best;
}

/* 3D closest point on a triangle: the minimiser of eq.1 is either the
 * interior stationary point (region R1, a face feature) or lies on the
 * boundary, where it is the best of the three segment minimisers (edge
 * regions R2-R4 when the segment parameter is interior, vertex regions R5-R7
 * when it is clamped).  This partition is the seven-region one of the paper. */
static void seg_closest(const double *p, const double *a, const double *b, double *t_out,
                        double *c, double *d2)
{
    double e[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double w[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    double t = dot3(w, e) / dot3(e, e);
    if (t <= 0.0) {
        t = 0.0;
        c[0] = a[0]; c[1] = a[1]; c[2] = a[2];
    } else if (t >= 1.0) {
        t = 1.0;
        c[0] = b[0]; c[1] = b[1]; c[2] = b[2];
    } else {
        c[0] = a[0] + t * e[0];
        c[1] = a[1] + t * e[1];
        c[2] = a[2] + t * e[2];
    }
    double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
    *d2 = dx * dx + dy * dy + dz * dz;
    *t_out = t;
}

static closest_t closest3d(const orc *o, const double *p)
{
    closest_t best;
    best.d2 = INFINITY;
    best.kind = -1;
    best.id = -1;
    best.facet = -1;
    for (int f = 0; f < o->nfacet; f++) {
        const int *tv = o->facet + 3 * f;
        const double *A = o->v + 3 * tv[0], *B = o->v + 3 * tv[1], *C = o->v + 3 * tv[2];
        double e0[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        double e1[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
        double dd[3] = {A[0] - p[0], A[1] - p[1], A[2] - p[2]};
        double a = dot3(e0, e0), b = dot3(e0, e1), c = dot3(e1, e1);
        double d = dot3(e0, dd), e = dot3(e1, dd);
        double det = a * c - b * b;
        double s = b * e - c * d, t = b * d - a * e;
        closest_t cur;
        cur.kind = -1;
        cur.id = -1;
        if (s > 0.0 && t > 0.0 && s + t < det) {
            s /= det;
            t /= det;
            cur.kind = FEAT_FACE;
            cur.id = f;
            for (int m = 0; m < 3; m++)
                cur.c[m] = A[m] + s * e0[m] + t * e1[m];
            double dx = p[0] - cur.c[0], dy = p[1] - cur.c[1], dz = p[2] - cur.c[2];
            cur.d2 = dx * dx + dy * dy + dz * dz;
        } else {
            cur.d2 = INFINITY;
            for (int m = 0; m < 3; m++) {
                const double *pa = o->v + 3 * tv[m], *pb = o->v + 3 * tv[(m + 1) % 3];
                double tt, cc[3], d2;
                seg_closest(p, pa, pb, &tt, cc, &d2);
                if (d2 < cur.d2) {
                    cur.d2 = d2;
                    memcpy(cur.c, cc, sizeof cc);
                    if (tt == 0.0) {
                        cur.kind = FEAT_VERTEX;
                        cur.id = tv[m];
                    } else if (tt == 1.0) {
                        cur.kind = FEAT_VERTEX;
                        cur.id = tv[(m + 1) % 3];
                    } else {
                        cur.kind = FEAT_EDGE;
                        cur.id = o->edge_of[3 * f + m];
                    }
                }
            }
        }
        if (cur.d2 < best.d2) {
            best = cur;
            best.facet = f;
        }
    }
    return best;
}

/* The standard HCIB/GC classification the paper replaces (section 3.2; its
 * comparison in section 7): signed distance, inside where (X - P0) . n_f < 0
 * with P0 the closest surface point and n_f the outward normal of the
 * closest facet (the lowest facet id among equals).  Near a sharp edge or
 * corner the closest facet's normal need not separate inside from outside,
 * which is its known failure. */
static int sd_inside(const orc *o, const double *X)
{
    closest_t cl = o->ndim == 2 ? closest2d(o, X) : closest3d(o, X);
    const double *n = o->fnrm + 3 * cl.facet;
    double s = 0.0;
    for (int d = 0; d < o->ndim; d++)
        s += (X[d] - cl.c[d]) * n[d];
    return s < 0.0;
}

/* First intersection (smallest sigma >= 0, sigma <= smax) of the line
 * x + sigma * dir with the body surface; returns -1 if none. */
static double line_hit2d(const orc *o, const double *x, const double *dir, double smax)
{
    double best = -1.0;
    for (int f = 0; f < o->nfacet; f++) {
        const double *a = o->v + 2 * o->facet[2 * f], *b = o->v + 2 * o->facet[2 * f + 1];
        double ex = b[0] - a[0], ey = b[1] - a[1];
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
    return best;
}

/* Moller-Trumbore ray/triangle intersection (section 3.2) for the line
 * x + sigma * dir; barycentric criteria u, v >= 0, u + v <= 1. */
static double line_hit3d(const orc *o, const double *x, const double *dir, double smax)
{
    double best = -1.0;
    for (int f = 0; f < o->nfacet; f++) {
        const int *tv = o->facet + 3 * f;
        const double *A = o->v + 3 * tv[0], *B = o->v + 3 * tv[1], *C = o->v + 3 * tv[2];
        double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        double e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
        double pv[3];
        cross3(dir, e2, pv);
        double det = dot3(e1, pv);
        if (det == 0.0)
            continue;
        double tv_[3] = {x[0] - A[0], x[1] - A[1], x[2] - A[2]};
        double u = dot3(tv_, pv) / det;
        if (u < 0.0 || u > 1.0)
            continue;
        double qv[3];
        cross3(tv_, e1, qv);
        double vv = dot3(dir, qv) / det;
        if (vv < 0.0 || u + vv > 1.0)
            continue;
        double sig = dot3(e2, qv) / det;
        if (sig < 0.0 || sig > smax)
            continue;
        if (best < 0.0 || sig < best)
            best = sig;
    }
    return best;
}

/* Enclosing cell of a probe point: per axis the largest centre index i0 with
 * c[i0] <= y < c[i0 + 1].  On a non-periodic axis both cells must be
 * interior; on a periodic axis the pair may straddle the boundary
 * (i0 = -1 or i0 + 1 = n, their periodic images), so every point of the
 * period has an enclosing cell.  Extended centres hold those images. */
static int locate(const double *c, int n, int periodic, double y, int *i0, double *frac)
{
    int lo = periodic ? -1 : 0, hi = periodic ? n : n - 1; /* c[lo+3] <= y < c[hi+3] */
    if (!(y >= c[lo + 3]) || !(y < c[hi + 3]))
        return 0;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (c[mid + 3] <= y)
            lo = mid;
        else
            hi = mid;
    }
    *i0 = lo;
    *frac = (y - c[lo + 3]) / (c[lo + 4] - c[lo + 3]);
    return 1;
}

static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* Probe interpolation set-up.  Returns 1 when the probe passes its validity
 * rule; fills corner ids (-1 where unused) and weights.
 *   mode 0 (multilinear over the enclosing cell): all corners must be
 *     FLUID (quadratic family, forcing node) or FLUID/FORCING (ghost nodes);
 *   mode 1 (inverse distance, weight 1/r^2, over the valid corners): at least
 *     one corner valid; a corner at r = 0 takes the whole weight. */
static int probe_setup(const orc *o, const double *y, int mode, int allow_forcing,
                       int32_t *ids, double *w)
{
    int nd = o->ndim, ncorner = 1 << nd;
    for (int m = 0; m < 8; m++) {
        ids[m] = -1;
        w[m] = 0.0;
    }
    int i0[3] = {0, 0, 0};
    double fr[3] = {0, 0, 0};
    int per[3] = {o->bc[0] == ORC_BC_PERIODIC, o->bc[2] == ORC_BC_PERIODIC,
                  o->bc[4] == ORC_BC_PERIODIC};
    if (!locate(o->xc, o->ni, per[0], y[0], &i0[0], &fr[0]) ||
        !locate(o->yc, o->nj, per[1], y[1], &i0[1], &fr[1]))
        return 0;
    if (nd == 3 && !locate(o->zc, o->nk, per[2], y[2], &i0[2], &fr[2]))
        return 0;
    int nvalid = 0, zero = -1;
    for (int m = 0; m < ncorner; m++) {
        int b[3] = {m & 1, (m >> 1) & 1, (m >> 2) & 1};
        long c = cidx(o, wrap(i0[0] + b[0], o->ni), wrap(i0[1] + b[1], o->nj),
                      nd == 3 ? wrap(i0[2] + b[2], o->nk) : 0);
        uint8_t t = o->cls[c];
        int valid = t == ORC_FLUID || (allow_forcing && t == ORC_FORCING);
        ids[m] = (int32_t)c;
        if (mode == 0) {
            if (!valid)
                return 0;
            double wt = 1.0;
            for (int d = 0; d < nd; d++)
                wt *= b[d] ? fr[d] : 1.0 - fr[d];
            w[m] = wt;
            nvalid++;
        } else {
            if (!valid) {
                w[m] = 0.0;
                continue;
            }
            double cc[3] = {o->xc[i0[0] + b[0] + 3], o->yc[i0[1] + b[1] + 3],
                            nd == 3 ? o->zc[i0[2] + b[2] + 3] : 0.0};
            double r2 = 0.0;
            for (int d = 0; d < nd; d++)
                r2 += (y[d] - cc[d]) * (y[d] - cc[d]);
            if (r2 == 0.0 && zero < 0)
                zero = m;
            w[m] = r2 > 0.0 ? 1.0 / r2 : 0.0;
            nvalid++;
        }
    }
    if (nvalid == 0)
        return 0;
    if (mode == 1) {
        if (zero >= 0) {
            for (int m = 0; m < ncorner; m++)
                w[m] = m == zero ? 1.0 : 0.0;
        } else {
            double s = 0.0;
            for (int m = 0; m < ncorner; m++)
                s += w[m];
            for (int m = 0; m < ncorner; m++)
                w[m] /= s;
        }
    }
    return 1;
}

/* Local-normal reconstruction geometry per listed node (sections 4.1-4.3):
 *  1. closest feature (face / edge / vertex);
 *  2. its normal: facet normal, or the edge / vertex pseudo-normal (eqs 2-3);
 *  3. the line through the node parallel to that normal meets the surface at
 *     P'.  Reading: for a face feature P' is the closest point; otherwise the
 *     first hit of the line followed into the body (forcing node) or out of
 *     it (ghost node) within 4 h, else the closest point (counted fallback).
 * Along the line s = 0 at P', s > 0 on the fluid side; the node sits at
 * s_X = +|X - P'| (forcing) or -|X - P'| (ghost).  Probes: s1 = s_X + h
 * (forcing) or max(|s_X|, h) (ghost), s2 = s1 + h (quadratic family); a probe
 * failing its validity rule moves out by h/2, at most six times, then falls
 * back to inverse-distance weights over its valid corners (counted). */
static void node_geometry(orc *o, int r, long c, int is_forcing)
{
    int nd = o->ndim;
    int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
    double X[3] = {o->xc[i + 3], o->yc[j + 3], nd == 3 ? o->zc[k + 3] : 0.0};
    double h = fmin(o->xf[i + 4] - o->xf[i + 3], o->yf[j + 4] - o->yf[j + 3]);
    if (nd == 3)
        h = fmin(h, o->zf[k + 4] - o->zf[k + 3]);
    closest_t cl = nd == 2 ? closest2d(o, X) : closest3d(o, X);
    double n[3] = {0, 0, 0};
    const double *src = cl.kind == FEAT_FACE ? o->fnrm + 3 * cl.id
                        : cl.kind == FEAT_VERTEX ? o->vnrm + 3 * cl.id
                                                 : o->enrm + 3 * cl.id;
    for (int d = 0; d < 3; d++)
        n[d] = src[d];
    double P[3] = {cl.c[0], cl.c[1], cl.c[2]};
    int fb = 0;
    if (o->frame == ORC_FRAME_SDSN) {
        /* surface-normal reconstruction (the standard HCIB/GC): the closest
         * facet's normal through the closest point, whatever the feature */
        for (int d = 0; d < 3; d++)
            n[d] = o->fnrm[3 * cl.facet + d];
    } else if (cl.kind != FEAT_FACE) {
        double dir[3] = {0, 0, 0};
        for (int d = 0; d < nd; d++)
            dir[d] = is_forcing ? -n[d] : n[d];
        double sig = nd == 2 ? line_hit2d(o, X, dir, 4.0 * h) : line_hit3d(o, X, dir, 4.0 * h);
        if (sig >= 0.0) {
            for (int d = 0; d < nd; d++)
                P[d] = X[d] + sig * dir[d];
        } else {
            fb |= 1;
#pragma omp atomic
            o->stat_fallback_pprime++;
        }
    }
    double dist2 = 0.0;
    for (int d = 0; d < nd; d++)
        dist2 += (X[d] - P[d]) * (X[d] - P[d]);
    double sx = is_forcing ? sqrt(dist2) : -sqrt(dist2);
    int quad = o->family == ORC_IB_QUADRATIC;
    int mode = (!quad && is_forcing) ? 1 : 0;
    int allow_forcing = !is_forcing;
    double s1 = is_forcing ? sx + h : fmax(-sx, h);
    double s2 = s1 + h;
    int32_t ids1[8], ids2[8];
    double w1[8], w2[8];
    int ok = 0, mode1 = mode, mode2 = mode;
    for (int attempt = 0; attempt <= 6; attempt++) {
        double y1[3] = {0, 0, 0}, y2[3] = {0, 0, 0};
        for (int d = 0; d < nd; d++) {
            y1[d] = P[d] + s1 * n[d];
            y2[d] = P[d] + s2 * n[d];
        }
        int v1 = probe_setup(o, y1, mode, allow_forcing, ids1, w1);
        int v2 = quad ? probe_setup(o, y2, mode, allow_forcing, ids2, w2) : 1;
        if (v1 && v2) {
            ok = 1;
            break;
        }
        if (attempt < 6) {
            s1 += 0.5 * h;
            s2 += 0.5 * h;
        }
    }
    if (!ok) {
        double y1[3] = {0, 0, 0}, y2[3] = {0, 0, 0};
        for (int d = 0; d < nd; d++) {
            y1[d] = P[d] + s1 * n[d];
            y2[d] = P[d] + s2 * n[d];
        }
        fb |= 2;
#pragma omp atomic
        o->stat_fallback_probe++;
        mode1 = mode2 = 1;
        int v1 = probe_setup(o, y1, 1, allow_forcing, ids1, w1);
        int v2 = quad ? probe_setup(o, y2, 1, allow_forcing, ids2, w2) : 1;
        if (!v1)
            mode1 = 2;
        if (quad && !v2)
            mode2 = 2;
        if (!v1 || (quad && !v2)) {
            fb |= 4;
#pragma omp atomic
            o->stat_fallback_none++;
        }
    }
    if (!quad) {
        for (int m = 0; m < 8; m++) {
            ids2[m] = -1;
            w2[m] = 0.0;
        }
        mode2 = 3;
    }
    int32_t *ir = o->irec + (long)IREC * r;
    double *dr = o->drec + (long)DREC * r;
    memset(ir, 0, sizeof(int32_t) * IREC);
    memset(dr, 0, sizeof(double) * DREC);
    ir[0] = (int32_t)c;
    ir[1] = cl.kind;
    ir[2] = cl.id;
    ir[3] = cl.facet;
    ir[4] = mode1;
    ir[5] = mode2;
    ir[6] = fb;
    for (int m = 0; m < 8; m++) {
        ir[7 + m] = ids1[m];
        ir[15 + m] = ids2[m];
        dr[9 + m] = w1[m];
        dr[17 + m] = w2[m];
    }
    for (int d = 0; d < 3; d++) {
        dr[d] = n[d];
        dr[3 + d] = P[d];
    }
    dr[6] = sx;
    dr[7] = s1;
    dr[8] = s2;
    dr[25] = sqrt(cl.d2);
    /* eq.7: curvature of the closest feature (2D) */
    dr[26] = nd == 2 ? (cl.kind == FEAT_FACE ? o->fcurv[cl.id] : o->vcurv[cl.id]) : 0.0;
}

int orc_geometry(orc *o)
{
    int nrec = o->nF + o->nG;
    free(o->irec);
    free(o->drec);
    o->irec = (int32_t *)calloc((size_t)(nrec > 0 ? nrec : 1) * IREC, sizeof(int32_t));
    o->drec = (double *)calloc((size_t)(nrec > 0 ? nrec : 1) * DREC, sizeof(double));
    /* one node per iteration; each writes only its own record */
#pragma omp parallel for schedule(dynamic, 16)
    for (int r = 0; r < nrec; r++) {
        int forcing = r < o->nF;
        long c = forcing ? o->listF[r] : o->listG[r - o->nF];
        node_geometry(o, r, c, forcing);
    }
    return 0;
}

/* ------------------------------------------------------ state conversions */
/* Conserved Q = (rho, rho u, rho v[, rho w], rho E) for the explicit scheme;
 * for dual time the state is Q_p' = (p - p_inf, u, v[, w], T - T_inf), the
 * primitive unknowns of section 4.4 taken as perturbations. */
typedef struct {
    real rho, u[3], p, T;
} prim_t;

static prim_t state_prim(const orc *o, const double *q, long s)
{
    prim_t w;
    long vs = o->vstride;
    int nd = o->ndim;
    w.u[0] = w.u[1] = w.u[2] = 0.0;
    /* the sums below are taken in the scalar type (the state values and
     * constants are double) */
    if (o->scheme == ORC_RK3) {
        w.rho = q[s];
        real ke = 0.0;
        for (int d = 0; d < nd; d++) {
            w.u[d] = q[s + (1 + d) * vs] / w.rho;
            ke += w.u[d] * w.u[d];
        }
        w.p = (o->gamma - 1.0) * (q[s + (nd + 1) * vs] - 0.5 * w.rho * ke);
        w.T = w.p / (w.rho * o->R);
    } else {
        w.p = (real)o->pinf + q[s];
        for (int d = 0; d < nd; d++)
            w.u[d] = q[s + (1 + d) * vs];
        w.T = (real)1.0 + q[s + (nd + 1) * vs];
        w.rho = w.p / (o->R * w.T);
    }
    return w;
}

static void prim_state(const orc *o, prim_t w, double *q, long s)
{
    long vs = o->vstride;
    int nd = o->ndim;
    if (o->scheme == ORC_RK3) {
        real ke = 0.0;
        for (int d = 0; d < nd; d++)
            ke += w.u[d] * w.u[d];
        q[s] = w.rho;
        for (int d = 0; d < nd; d++)
            q[s + (1 + d) * vs] = w.rho * w.u[d];
        q[s + (nd + 1) * vs] = w.p / (o->gamma - 1.0) + 0.5 * w.rho * ke;
    } else {
        q[s] = w.p - o->pinf;
        for (int d = 0; d < nd; d++)
            q[s + (1 + d) * vs] = w.u[d];
        q[s + (nd + 1) * vs] = w.T - 1.0;
    }
}

/* conserved vector of a primitive state (always conserved, any scheme) */
static void prim_cons(const orc *o, prim_t w, real *Q)
{
    int nd = o->ndim;
    real ke = 0.0;
    for (int d = 0; d < nd; d++)
        ke += w.u[d] * w.u[d];
    Q[0] = w.rho;
    for (int d = 0; d < nd; d++)
        Q[1 + d] = w.rho * w.u[d];
    Q[nd + 1] = w.p / (o->gamma - 1.0) + 0.5 * w.rho * ke;
}

void orc_prim_to_state(orc *o, const double *prim, double *q)
{
    int nd = o->ndim;
    long n = (long)o->ni * o->nj * o->nk;
    for (long c = 0; c < n; c++) {
        int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
        prim_t w;
        w.rho = prim[c];
        w.u[0] = w.u[1] = w.u[2] = 0.0;
        for (int d = 0; d < nd; d++)
            w.u[d] = prim[(1 + d) * n + c];
        w.p = prim[(nd + 1) * n + c];
        w.T = w.p / (w.rho * o->R);
        prim_state(o, w, q, sidx(o, i, j, k));
    }
}

void orc_state_to_prim(orc *o, const double *q, double *prim)
{
    int nd = o->ndim;
    long n = (long)o->ni * o->nj * o->nk;
    for (long c = 0; c < n; c++) {
        int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
        prim_t w = state_prim(o, q, sidx(o, i, j, k));
        prim[c] = w.rho;
        for (int d = 0; d < nd; d++)
            prim[(1 + d) * n + c] = w.u[d];
        prim[(nd + 1) * n + c] = w.p;
    }
}

/* --------------------------------------------------- a5 domain boundaries */
/* Three ghost layers per side (reading): FARFIELD = free stream, EXTRAP =
 * copy of the adjacent interior cell, PERIODIC = wrap.  x sides first over
 * the interior rows, then y sides over the x-extended rows, then z sides
 * over the x,y-extended planes, so corner ghosts are filled consistently. */
static void freestream_prim(const orc *o, prim_t *w)
{
    w->rho = 1.0;
    for (int d = 0; d < 3; d++)
        w->u[d] = o->uinf[d];
    w->p = o->pinf;
    w->T = 1.0;
}

void orc_bc(orc *o, double *q)
{
    int nd = o->ndim, nv = o->nv;
    long vs = o->vstride;
    int n[3] = {o->ni, o->nj, o->nk};
    prim_t fs;
    freestream_prim(o, &fs);
    real qfs[5];
    {
        /* the free stream in the state's own variables */
        real tmp[5 * 1];
        (void)tmp;
        if (o->scheme == ORC_RK3)
            prim_cons(o, fs, qfs);
        else {
            qfs[0] = 0.0;
            for (int d = 0; d < nd; d++)
                qfs[1 + d] = fs.u[d];
            qfs[nd + 1] = 0.0;
        }
    }
    for (int ax = 0; ax < nd; ax++) {
        int lo[3], hi[3];
        for (int d = 0; d < 3; d++) {
            int h = d < nd ? (d < 2 ? 3 : o->hz) : 0;
            if (d < ax) {
                lo[d] = -h;
                hi[d] = n[d] + h;
            } else {
                lo[d] = 0;
                hi[d] = n[d];
            }
        }
        for (int side = 0; side < 2; side++) {
            int type = o->bc[2 * ax + side];
            for (int g = 1; g <= 3; g++) {
                int a = side == 0 ? -g : n[ax] - 1 + g;
                int src = type == ORC_BC_PERIODIC ? (side == 0 ? n[ax] - g : g - 1)
                                                   : (side == 0 ? 0 : n[ax] - 1);
                int c0[3], e0 = lo[(ax + 1) % 3], e1 = hi[(ax + 1) % 3];
                int f0 = lo[(ax + 2) % 3], f1 = hi[(ax + 2) % 3];
                for (int u = e0; u < e1; u++)
                    for (int w = f0; w < f1; w++) {
                        c0[ax] = a;
                        c0[(ax + 1) % 3] = u;
                        c0[(ax + 2) % 3] = w;
                        if (nd == 2)
                            c0[2] = 0;
                        long dst = sidx(o, c0[0], c0[1], c0[2]);
                        c0[ax] = src;
                        long sv = sidx(o, c0[0], c0[1], c0[2]);
                        for (int v = 0; v < nv; v++)
                            q[dst + v * vs] = type == ORC_BC_FARFIELD ? qfs[v] : q[sv + v * vs];
                    }
            }
        }
    }
}

/* ------------------------------------------------------------- a5 IB fill */
/* Boundary conditions along the local-normal line (section 4.4):
 *   velocity: Dirichlet, the body velocity (eq.4);
 *   pressure: Neumann, dp/dn = -rho n . a_body, n into the fluid (eqs 5-6,
 *             read with that sign), zero for a stationary body;
 *   temperature: Neumann, dT/dn = 0 (eq.8).
 * Linear family (compressible, sections 4.6 and 5): forcing nodes use an
 * inverse-distance-weighted probe and ghost nodes the image point, both with
 * a linear profile along the line.  Quadratic family (incompressible,
 * sections 4.5 and 5): two multilinear probes and a quadratic profile.
 * Forcing nodes are filled first (they read FLUID cells only), then all ghost
 * layers (they read FLUID and FORCING cells); each pass is Jacobi. */
/* The value at a probe: the weighted mean sum_m w_m phi_m / sum_m w_m of
 * (p, u.., T) over its corners (multilinear or inverse-distance weights,
 * sections 4.5-4.6).  The weights of a probe sum to one; dividing by their
 * computed sum reproduces a constant field exactly, whatever the rounding of
 * the weights (at low Mach p is p_inf plus a perturbation some 1e6 times
 * smaller, so a sum of weights off by an ulp would otherwise shift p by
 * that ulp of p_inf). */
static void probe_value(const orc *o, const double *q, const int32_t *ids, const double *w,
                        real *phi)
{
    int nd = o->ndim;
    real wsum = 0.0;
    for (int v = 0; v < nd + 2; v++)
        phi[v] = 0.0;
    for (int m = 0; m < (1 << nd); m++) {
        if (ids[m] < 0 || w[m] == 0.0)
            continue;
        long c = ids[m];
        int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
        prim_t p = state_prim(o, q, sidx(o, i, j, k));
        phi[0] += w[m] * p.p;
        for (int d = 0; d < nd; d++)
            phi[1 + d] += w[m] * p.u[d];
        phi[nd + 1] += w[m] * p.T;
        wsum += w[m];
    }
    if (wsum > 0.0)
        for (int v = 0; v < nd + 2; v++)
            phi[v] /= wsum;
}

static void fill_range(orc *o, double *q, int r0, int r1, double t)
{
    int nd = o->ndim, quad = o->family == ORC_IB_QUADRATIC;
    real ub[3] = {0, 0, 0}, ab[3] = {0, 0, 0};
    if (o->motion) {
        ub[o->maxis] = pose_vel(o, t);
        ab[o->maxis] = pose_acc(o, t);
    }
    int nr = r1 - r0;
    prim_t *out = (prim_t *)malloc(sizeof(prim_t) * (nr > 0 ? nr : 1));
    for (int r = r0; r < r1; r++) {
        const int32_t *ir = o->irec + (long)IREC * r;
        const double *dr = o->drec + (long)DREC * r;
        const double *n = dr;
        real sx = dr[6], s1 = dr[7], s2 = dr[8];
        real phi1[5], phi2[5];
        prim_t res;
        res.u[0] = res.u[1] = res.u[2] = 0.0;
        if (ir[4] == 2) { /* no valid probe corner at all: counted fallback */
            res.p = o->pinf;
            res.T = 1.0;
            for (int d = 0; d < nd; d++)
                res.u[d] = ub[d];
        } else {
            probe_value(o, q, ir + 7, dr + 9, phi1);
            real rho1 = phi1[0] / (o->R * phi1[nd + 1]);
            real an = 0.0;
            for (int d = 0; d < nd; d++)
                an += n[d] * ab[d];
            real gp = -rho1 * an, gT = 0.0;
            if (o->wallp == ORC_WALL_EQ7 && nd == 2) {
                /* eq.7 (reading: the normal momentum balance at the wall, n
                 * into the fluid): dp/dn = rho u_t^2 kappa - rho a_n, u_t the
                 * tangential velocity relative to the wall at probe 1 */
                real ut = -(phi1[1] - ub[0]) * n[1] + (phi1[2] - ub[1]) * n[0];
                gp = rho1 * ut * ut * dr[26] - rho1 * an;
            }
            if (!quad || ir[5] == 2) {
                for (int d = 0; d < nd; d++)
                    res.u[d] = ub[d] + (phi1[1 + d] - ub[d]) * sx / s1;
                res.p = phi1[0] + gp * (sx - s1);
                res.T = phi1[nd + 1] + gT * (sx - s1);
            } else {
                probe_value(o, q, ir + 15, dr + 17, phi2);
                /* Dirichlet: parabola through (0, phiB), (s1, phi1), (s2, phi2) */
                real L0 = (sx - s1) * (sx - s2) / (s1 * s2);
                real L1 = sx * (sx - s2) / (s1 * (s1 - s2));
                real L2 = sx * (sx - s1) / (s2 * (s2 - s1));
                for (int d = 0; d < nd; d++)
                    res.u[d] = ub[d] * L0 + phi1[1 + d] * L1 + phi2[1 + d] * L2;
                /* Neumann: phi = c0 + g s + c2 s^2 through the two probes */
                real c2p = (phi2[0] - phi1[0] - gp * (s2 - s1)) / (s2 * s2 - s1 * s1);
                real c0p = phi1[0] - gp * s1 - c2p * s1 * s1;
                res.p = c0p + gp * sx + c2p * sx * sx;
                real c2T = (phi2[nd + 1] - phi1[nd + 1] - gT * (s2 - s1)) / (s2 * s2 - s1 * s1);
                real c0T = phi1[nd + 1] - gT * s1 - c2T * s1 * s1;
                res.T = c0T + gT * sx + c2T * sx * sx;
            }
        }
        res.rho = res.p / (o->R * res.T);
        out[r - r0] = res;
    }
    for (int r = r0; r < r1; r++) {
        long c = o->irec[(long)IREC * r];
        int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
        prim_state(o, out[r - r0], q, sidx(o, i, j, k));
    }
    free(out);
}

void orc_fill(orc *o, double *q, double t)
{
    fill_range(o, q, 0, o->nF, t);
    fill_range(o, q, o->nF, o->nF + o->nG, t);
}

/* ------------------------------------------------------------ a7 WENO5 */
/* Fifth-order WENO (section 2, [74]); reading: the Jiang-Shu weights with
 * eps = 1e-6 and linear weights (0.1, 0.6, 0.3).  Left state at i+1/2 from
 * v(i-2 .. i+2); the right state is the same function of v(i+3 .. i-1). */
/* Second-order TVD reconstruction (section 2 names the scheme, not its
 * limiter; reading: MUSCL with the minmod limiter): the state at the face
 * between b and c seen from b's side, b + (1/2) minmod(b - a, c - b). */
static real minmod(real x, real y)
{
    if (x > 0.0 && y > 0.0)
        return x < y ? x : y;
    if (x < 0.0 && y < 0.0)
        return x > y ? x : y;
    return 0.0;
}

static real tvd2_r(real a, real b, real c)
{
    return b + 0.5 * minmod(b - a, c - b);
}

static real weno5_r(real a, real b, real c, real d, real e)
{
    real q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
    real q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
    real q2 = (2.0 * c + 5.0 * d - e) / 6.0;
    real b0 = 13.0 / 12.0 * (a - 2.0 * b + c) * (a - 2.0 * b + c) +
                0.25 * (a - 4.0 * b + 3.0 * c) * (a - 4.0 * b + 3.0 * c);
    real b1 = 13.0 / 12.0 * (b - 2.0 * c + d) * (b - 2.0 * c + d) + 0.25 * (b - d) * (b - d);
    real b2 = 13.0 / 12.0 * (c - 2.0 * d + e) * (c - 2.0 * d + e) +
                0.25 * (3.0 * c - 4.0 * d + e) * (3.0 * c - 4.0 * d + e);
    real a0 = 0.1 / ((WENO_EPS + b0) * (WENO_EPS + b0));
    real a1 = 0.6 / ((WENO_EPS + b1) * (WENO_EPS + b1));
    real a2 = 0.3 / ((WENO_EPS + b2) * (WENO_EPS + b2));
    real s = a0 + a1 + a2;
    return (a0 / s) * q0 + (a1 / s) * q1 + (a2 / s) * q2;
}

/* -------------------------------------------------- a8 LDFSS + precond. */
/* Low-diffusion flux splitting (section 2, [73]).  Reading: Edwards'
 * LDFSS(0) with the interface speed of sound replaced, in dual-time mode, by
 * the Weiss-Smith preconditioned one
 *   eps = min(1, max(|u_L|^2/2 + |u_R|^2/2, U_c^2) / a_half^2),
 *   a~  = (1/2) RSQRT((1 - eps)^2 Ubar^2 + 4 eps a_half^2),
 * and the split pressure taken on the unpreconditioned interface Mach numbers
 * U / a_half, with its velocity-diffusion part p_bar (D+ + D- - 1) scaled by
 * a~ / a_half, so that the pressure dissipation is of the order of the
 * dynamic pressure, rho U_r U, at low Mach.
 * With eps = 1 (or outside dual time) this is exactly LDFSS(0).
 * w = (rho, u, v[, w], p); nrm = unit normal; flux per unit area. */
static real sgn1(real m) { return m >= 0.0 ? 1.0 : -1.0; }

static void ldfss_r(int ndim, const real *wl, const real *wr, const double *nrm, double gamma,
                    int precond, double uc2, real *flux)
{
    int nv = ndim + 2;
    real rl = wl[0], rr = wr[0], pl = wl[nv - 1], pr = wr[nv - 1];
    real UL = 0.0, UR = 0.0, ql2 = 0.0, qr2 = 0.0;
    for (int d = 0; d < ndim; d++) {
        UL += wl[1 + d] * nrm[d];
        UR += wr[1 + d] * nrm[d];
        ql2 += wl[1 + d] * wl[1 + d];
        qr2 += wr[1 + d] * wr[1 + d];
    }
    real al = RSQRT(gamma * pl / rl), ar = RSQRT(gamma * pr / rr);
    real ah = 0.5 * (al + ar);
    real at = ah, eps = 1.0;
    if (precond) {
        eps = RFMIN(1.0, RFMAX(0.5 * ql2 + 0.5 * qr2, uc2) / (ah * ah));
        if (eps < 1.0) {
            real ub = 0.5 * (UL + UR);
            at = 0.5 * RSQRT((1.0 - eps) * (1.0 - eps) * ub * ub + 4.0 * eps * ah * ah);
        }
    }
    real ML = UL / at, MR = UR / at;
    real apl = 0.5 * (1.0 + sgn1(ML)), amr = 0.5 * (1.0 - sgn1(MR));
    real bl = -RFMAX(0.0, 1.0 - RFLOOR(RFABS(ML))), br = -RFMAX(0.0, 1.0 - RFLOOR(RFABS(MR)));
    real mpl = 0.25 * (ML + 1.0) * (ML + 1.0), mmr = -0.25 * (MR - 1.0) * (MR - 1.0);
    real cp = apl * (1.0 + bl) * ML - bl * mpl;
    real cm = amr * (1.0 + br) * MR - br * mmr;
    real mh = 0.25 * bl * br * (RSQRT(0.5 * (ML * ML + MR * MR)) - 1.0) *
                (RSQRT(0.5 * (ML * ML + MR * MR)) - 1.0);
    real dp = pl - pr;
    real mhp = mh * (1.0 - (dp + RFABS(dp)) / (2.0 * rl * at * at));
    real mhm = mh * (1.0 + (dp - RFABS(dp)) / (2.0 * rr * at * at));
    real chp = cp - mhp, chm = cm + mhm;
    real ppl = 0.25 * (ML + 1.0) * (ML + 1.0) * (2.0 - ML);
    real pmr = 0.25 * (MR - 1.0) * (MR - 1.0) * (2.0 + MR);
    real dpl = apl * (1.0 + bl) - bl * ppl;
    real dmr = amr * (1.0 + br) - br * pmr;
    real Hl = gamma / (gamma - 1.0) * pl / rl + 0.5 * ql2;
    real Hr = gamma / (gamma - 1.0) * pr / rr + 0.5 * qr2;
    real fl = at * rl * chp, fr = at * rr * chm;
    real pf;
    if (eps >= 1.0)
        pf = dpl * pl + dmr * pr;
    else {
        /* pressure split on the unpreconditioned interface Mach numbers,
         * velocity-diffusion part scaled by a~ / a_half */
        real mL = UL / ah, mR = UR / ah;
        real aL = 0.5 * (1.0 + sgn1(mL)), aR = 0.5 * (1.0 - sgn1(mR));
        real gL = -RFMAX(0.0, 1.0 - RFLOOR(RFABS(mL))), gR = -RFMAX(0.0, 1.0 - RFLOOR(RFABS(mR)));
        real qL = 0.25 * (mL + 1.0) * (mL + 1.0) * (2.0 - mL);
        real qR = 0.25 * (mR - 1.0) * (mR - 1.0) * (2.0 + mR);
        real eL = aL * (1.0 + gL) - gL * qL;
        real eR = aR * (1.0 + gR) - gR * qR;
        real pbar = 0.5 * (pl + pr);
        pf = pbar + 0.5 * (eL - eR) * (pl - pr) + at / ah * pbar * (eL + eR - 1.0);
    }
    flux[0] = fl + fr;
    for (int d = 0; d < ndim; d++)
        flux[1 + d] = fl * wl[1 + d] + fr * wr[1 + d] + pf * nrm[d];
    flux[nv - 1] = fl * Hl + fr * Hr;
}

/* ------------------------------------------------------- a6-a9 residual */
/* Cell-centred finite volume on a rectilinear grid (section 2): WENO5 in
 * index space on the primitive variables (rho, u, v[, w], p) (reading), the
 * LDFSS flux above, and second-order central viscous fluxes: normal
 * gradient from the two cell values, tangential gradients as the mean of the
 * two cells' central differences, face velocity the mean of the two cells,
 * constant mu, tau = mu (grad u + grad u^T - 2/3 div u I), q = -k grad T. */
static void face_flux(const orc *o, const double *q, int i, int j, int k, int ax, real *F)
{
    int nd = o->ndim, nv = o->nv;
    int off[3] = {0, 0, 0};
    off[ax] = 1;
    /* primitive values of the six stencil cells L-2 .. L+3 */
    prim_t st[6];
    for (int m = 0; m < 6; m++) {
        int s = m - 2;
        st[m] = state_prim(o, q, sidx(o, i + s * off[0], j + s * off[1], k + s * off[2]));
        (void)st[m];
    }
    real v[6][5];
    for (int m = 0; m < 6; m++) {
        v[m][0] = st[m].rho;
        for (int d = 0; d < nd; d++)
            v[m][1 + d] = st[m].u[d];
        v[m][nv - 1] = st[m].p;
    }
    real wl[5], wr[5];
    for (int var = 0; var < nv; var++) {
        if (o->recon == ORC_RECON_TVD2) {
            wl[var] = tvd2_r(v[1][var], v[2][var], v[3][var]);
            wr[var] = tvd2_r(v[4][var], v[3][var], v[2][var]);
        } else {
            wl[var] = weno5_r(v[0][var], v[1][var], v[2][var], v[3][var], v[4][var]);
            wr[var] = weno5_r(v[5][var], v[4][var], v[3][var], v[2][var], v[1][var]);
        }
    }
    double nrm[3] = {0, 0, 0};
    nrm[ax] = 1.0;
    real fi[5];
    ldfss_r(nd, wl, wr, nrm, o->gamma, o->scheme == ORC_DUAL, o->uc2, fi);

    /* viscous flux */
    const double *cc[3] = {o->xc, o->yc, o->zc};
    int lo[3] = {i, j, k}, hi[3] = {i + off[0], j + off[1], k + off[2]};
    prim_t PL = st[2], PR = st[3];
    real grad[4][3]; /* d(u_m)/dx_d for m < 3, dT/dx_d in row 3 */
    int idx_lo = lo[ax] + 3, idx_hi = hi[ax] + 3;
    real dn = cc[ax][idx_hi] - cc[ax][idx_lo];
    for (int m = 0; m < 3; m++)
        grad[m][ax] = (PR.u[m] - PL.u[m]) / dn;
    grad[3][ax] = (PR.T - PL.T) / dn;
    for (int e = 0; e < nd; e++) {
        if (e == ax)
            continue;
        real g[4] = {0, 0, 0, 0};
        for (int side = 0; side < 2; side++) {
            int b[3] = {side ? hi[0] : lo[0], side ? hi[1] : lo[1], side ? hi[2] : lo[2]};
            int p1[3] = {b[0], b[1], b[2]}, m1[3] = {b[0], b[1], b[2]};
            p1[e] += 1;
            m1[e] -= 1;
            prim_t A = state_prim(o, q, sidx(o, p1[0], p1[1], p1[2]));
            prim_t B = state_prim(o, q, sidx(o, m1[0], m1[1], m1[2]));
            real de = cc[e][b[e] + 4] - cc[e][b[e] + 2];
            for (int m = 0; m < 3; m++)
                g[m] += 0.5 * (A.u[m] - B.u[m]) / de;
            g[3] += 0.5 * (A.T - B.T) / de;
        }
        for (int m = 0; m < 4; m++)
            grad[m][e] = g[m];
    }
    for (int m = 0; m < 4; m++)
        for (int e = nd; e < 3; e++)
            grad[m][e] = 0.0;
    real div = 0.0;
    for (int d = 0; d < nd; d++)
        div += grad[d][d];
    real uf[3];
    for (int m = 0; m < 3; m++)
        uf[m] = 0.5 * (PL.u[m] + PR.u[m]);
    real tau[3]; /* tau_{m, ax} */
    for (int m = 0; m < 3; m++)
        tau[m] = o->mu * (grad[m][ax] + grad[ax][m] - (m == ax ? 2.0 / 3.0 * div : 0.0));
    real qn = -o->kc * grad[3][ax];
    real fv[5];
    fv[0] = 0.0;
    real work = 0.0;
    for (int d = 0; d < nd; d++) {
        fv[1 + d] = tau[d];
        work += uf[d] * tau[d];
    }
    fv[nv - 1] = work - qn;
    for (int var = 0; var < nv; var++)
        F[var] = fi[var] - fv[var];
}

static int is_solid_at(const orc *o, int i, int j, int k)
{
    int n[3] = {o->ni, o->nj, o->nk}, c[3] = {i, j, k};
    for (int d = 0; d < o->ndim; d++)
        if (c[d] < 0 || c[d] >= n[d])
            return 0; /* domain ghost */
    return o->cls[cidx(o, i, j, k)] == ORC_SOLID;
}

static void residual_r(orc *o, const double *q, real *r)
{
    int nd = o->ndim, nv = o->nv;
    long n = (long)o->ni * o->nj * o->nk;
    i64 viol = 0;
#pragma omp parallel for schedule(static) reduction(+ : viol)
    for (long c = 0; c < n; c++) {
        for (int v = 0; v < nv; v++)
            r[v * n + c] = 0.0;
        if (o->cls[c] != ORC_FLUID)
            continue;
        int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
        /* stencil check: no cell read by this cell's fluxes may be SOLID */
        for (int ax = 0; ax < nd; ax++)
            for (int s = -3; s <= 3; s++) {
                int p[3] = {i, j, k};
                p[ax] += s;
                if (is_solid_at(o, p[0], p[1], p[2]))
                    viol++;
            }
        for (int a = 0; a < nd; a++)
            for (int b = a + 1; b < nd; b++)
                for (int sa = -1; sa <= 1; sa += 2)
                    for (int sb = -1; sb <= 1; sb += 2) {
                        int p[3] = {i, j, k};
                        p[a] += sa;
                        p[b] += sb;
                        if (is_solid_at(o, p[0], p[1], p[2]))
                            viol++;
                    }
        real dx[3] = {o->xf[i + 4] - o->xf[i + 3], o->yf[j + 4] - o->yf[j + 3],
                        o->zf[k + 4] - o->zf[k + 3]};
        real vol = dx[0] * dx[1] * dx[2];
        real acc[5] = {0, 0, 0, 0, 0};
        for (int ax = 0; ax < nd; ax++) {
            real area = vol / dx[ax];
            real Fp[5], Fm[5];
            int off[3] = {0, 0, 0};
            off[ax] = 1;
            face_flux(o, q, i, j, k, ax, Fp);
            face_flux(o, q, i - off[0], j - off[1], k - off[2], ax, Fm);
            for (int v = 0; v < nv; v++)
                acc[v] += (Fp[v] - Fm[v]) * area;
        }
        for (int v = 0; v < nv; v++)
            r[v * n + c] = acc[v] / vol;
    }
    o->stat_stencil_violation += viol;
}

/* The exported evaluations take and return double; the arithmetic runs in
 * the oracle's scalar type. */
void orc_residual(orc *o, const double *q, double *r)
{
    long n = (long)o->ni * o->nj * o->nk * o->nv;
    real *rr = (real *)malloc(sizeof(real) * n);
    residual_r(o, q, rr);
    for (long m = 0; m < n; m++)
        r[m] = (double)rr[m];
    free(rr);
}

double orc_weno5(double a, double b, double c, double d, double e)
{
    return (double)weno5_r(a, b, c, d, e);
}

double orc_tvd2(double a, double b, double c) { return (double)tvd2_r(a, b, c); }

void orc_ldfss(int ndim, const double *wl, const double *wr, const double *nrm, double gamma,
               int precond, double uc2, double *flux)
{
    real a[5] = {0, 0, 0, 0, 0}, b[5] = {0, 0, 0, 0, 0}, f[5];
    for (int m = 0; m < ndim + 2; m++) {
        a[m] = wl[m];
        b[m] = wr[m];
    }
    ldfss_r(ndim, a, b, nrm, gamma, precond, uc2, f);
    for (int m = 0; m < ndim + 2; m++)
        flux[m] = (double)f[m];
}

size_t orc_real_bytes(void) { return sizeof(real); }

/* ------------------------------------------------------ a10 SSP-RK3 step */
/* Shu-Osher three-stage SSP Runge-Kutta (the explicit scheme of the
 * workload; not in the paper):
 *   Q1 = Q^n - dt R(Q^n);  Q2 = 3/4 Q^n + 1/4 (Q1 - dt R(Q1));
 *   Q^{n+1} = 1/3 Q^n + 2/3 (Q2 - dt R(Q2)).
 * Before every residual: domain ghosts, then the IB fill at the stage time
 * (t, t + dt, t + dt/2).  FLUID cells take the update; FORCING and ghost
 * cells copy the stage input, so a cell uncovered by a moving body keeps its
 * latest ghost-extended state; SOLID cells are left untouched.  For a moving
 * body, classification and geometry are redone at the pose of t^n. */
static void rk_stage(orc *o, const double *qn, const double *qin, double *qout, double a,
                     double b)
{
    int nv = o->nv;
    long n = (long)o->ni * o->nj * o->nk, vs = o->vstride;
    real *r = (real *)malloc(sizeof(real) * nv * n);
    residual_r(o, qin, r);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; c++) {
        int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
        long s = sidx(o, i, j, k);
        uint8_t t = o->cls[c];
        if (t == ORC_FLUID) {
            for (int v = 0; v < nv; v++)
                qout[s + v * vs] = (real)a * qn[s + v * vs] + (real)b * (qin[s + v * vs] - o->dt * r[v * n + c]);
        } else if (t != ORC_SOLID) {
            for (int v = 0; v < nv; v++)
                qout[s + v * vs] = qin[s + v * vs];
        }
    }
    free(r);
}

void orc_rk3_step(orc *o, double *q, double *q1, double *q2, double t)
{
    if (o->motion) {
        orc_set_pose(o, t);
        orc_classify(o);
        orc_geometry(o);
    }
    double dt = o->dt;
    /* each stage: IB fill (its probes read interior cells only), then the
     * domain ghost layers as images of the filled interior */
    orc_fill(o, q, t);
    orc_bc(o, q);
    rk_stage(o, q, q, q1, 0.0, 1.0);
    orc_fill(o, q1, t + dt);
    orc_bc(o, q1);
    rk_stage(o, q, q1, q2, 0.75, 0.25);
    orc_fill(o, q2, t + 0.5 * dt);
    orc_bc(o, q2);
    rk_stage(o, q, q2, q, 1.0 / 3.0, 2.0 / 3.0);
}

/* ------------------------------------------------------ a10 dual time */
/* Dual time stepping (section 2): three-point (BDF2) physical-time
 * derivative, two-point Euler pseudo-time derivative, preconditioned
 * (section 1: all-speed solver; [72]).  Reading: a point-implicit pseudo
 * step per FLUID cell,
 *   [Gamma / dtau + b0 / dt * P] dQp = -[(b0 (Q - Q^n) - b2 (Q^n - Q^{n-1})) / dt + R],
 * with Qp = (p, u, v[, w], T), P = dQ/dQp, Gamma = P with rho_p replaced by
 * theta = 1/U_r^2 + 1/(c_p T) (Weiss-Smith), U_r^2 = min(a^2, max(|u|^2,
 * U_c^2)); BDF2 (b0, b2) = (3/2, 1/2), BDF1 (1, 0) for the first physical
 * step; dtau = CFL_tau / sum_d [(|U'_d| + c'_d) / dx_d + 2 nu_v / dx_d^2] with
 * U' = (1 + eps) u_d / 2, c' = RSQRT((1 - eps)^2 u_d^2 + 4 eps a^2) / 2,
 * eps = U_r^2 / a^2, nu_v = mu / rho max(4/3, gamma / Pr).  The system is
 * solved by Gaussian elimination with partial pivoting. */
static void gauss_solve(int n, real A[5][5], real *b)
{
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int r = c + 1; r < n; r++)
            if (RFABS(A[r][c]) > RFABS(A[piv][c]))
                piv = r;
        if (piv != c) {
            for (int m = 0; m < n; m++) {
                real t = A[c][m];
                A[c][m] = A[piv][m];
                A[piv][m] = t;
            }
            real t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < n; r++) {
            real f = A[r][c] / A[c][c];
            for (int m = c; m < n; m++)
                A[r][m] -= f * A[c][m];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; r--) {
        real s = b[r];
        for (int m = r + 1; m < n; m++)
            s -= A[r][m] * b[m];
        b[r] = s / A[r][r];
    }
}

static void conserved_of_state(orc *o, const double *q, real *Q)
{
    int nv = o->nv;
    long n = (long)o->ni * o->nj * o->nk;
    for (long c = 0; c < n; c++) {
        int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
        prim_t w = state_prim(o, q, sidx(o, i, j, k));
        real v[5];
        prim_cons(o, w, v);
        for (int m = 0; m < nv; m++)
            Q[m * n + c] = v[m];
    }
}

/* Start of a physical step: history rotation Q^{n-1} <- Q^n, Q^n <- Q(W). */
void orc_dual_begin(orc *o, const double *w, real *qn, real *qnm1, int first, double t_new)
{
    long n = (long)o->ni * o->nj * o->nk;
    if (o->motion) {
        orc_set_pose(o, t_new);
        orc_classify(o);
        orc_geometry(o);
    }
    if (!first)
        memcpy(qnm1, qn, sizeof(real) * o->nv * n);
    conserved_of_state(o, w, qn);
}

/* n_iter pseudo-time iterations of the current physical step. */
void orc_dual_iterate(orc *o, double *w, double *wtmp, const real *qn, const real *qnm1,
                      int first, double t_new, int n_iter)
{
    int nd = o->ndim, nv = o->nv;
    long n = (long)o->ni * o->nj * o->nk, vs = o->vstride;
    /* (b0 Q - (b0 + b2) Q^n + b2 Q^{n-1}) / dt: BDF2 (3/2, 1/2), BDF1 (1, 0) */
    real b0 = first ? 1.0 : 1.5, b2 = first ? 0.0 : 0.5;
    real *r = (real *)malloc(sizeof(real) * nv * n);
    for (int it = 0; it < n_iter; it++) {
        orc_fill(o, w, t_new);
        orc_bc(o, w);
        residual_r(o, w, r);
        memcpy(wtmp, w, sizeof(double) * nv * vs);
#pragma omp parallel for schedule(static)
        for (long c = 0; c < n; c++) {
            if (o->cls[c] != ORC_FLUID)
                continue;
            int i = (int)(c % o->ni), j = (int)((c / o->ni) % o->nj), k = (int)(c / ((long)o->ni * o->nj));
            long s = sidx(o, i, j, k);
            prim_t P = state_prim(o, w, s);
            real Q[5];
            prim_cons(o, P, Q);
            real q2 = 0.0;
            for (int d = 0; d < nd; d++)
                q2 += P.u[d] * P.u[d];
            real a2 = o->gamma * P.p / P.rho;
            real ur2 = RFMIN(a2, RFMAX(q2, o->uc2));
            real eps = ur2 / a2;
            double dx[3] = {o->xf[i + 4] - o->xf[i + 3], o->yf[j + 4] - o->yf[j + 3],
                            o->zf[k + 4] - o->zf[k + 3]};
            real nuv = o->mu / P.rho * RFMAX(4.0 / 3.0, o->gamma / o->pr);
            real lam = 0.0;
            for (int d = 0; d < nd; d++) {
                real ud = P.u[d];
                real up = 0.5 * (1.0 + eps) * RFABS(ud);
                real cpr = 0.5 * RSQRT((1.0 - eps) * (1.0 - eps) * ud * ud + 4.0 * eps * a2);
                lam += (up + cpr) / dx[d] + 2.0 * nuv / (dx[d] * dx[d]);
            }
            real dtau = o->cfl_tau / lam;
            real H = o->cp * P.T + 0.5 * q2;
            real rp = 1.0 / (o->R * P.T), rT = -P.rho / P.T;
            real th = 1.0 / ur2 + 1.0 / (o->cp * P.T);
            real Pm[5][5], Gm[5][5], A[5][5];
            memset(Pm, 0, sizeof Pm);
            memset(Gm, 0, sizeof Gm);
            int e = nv - 1;
            for (int pass = 0; pass < 2; pass++) {
                real (*M)[5] = pass == 0 ? Pm : Gm;
                real x = pass == 0 ? rp : th;
                M[0][0] = x;
                M[0][e] = rT;
                for (int d = 0; d < nd; d++) {
                    M[1 + d][0] = P.u[d] * x;
                    M[1 + d][1 + d] = P.rho;
                    M[1 + d][e] = P.u[d] * rT;
                    M[e][1 + d] = P.rho * P.u[d];
                }
                M[e][0] = H * x - 1.0;
                M[e][e] = H * rT + P.rho * o->cp;
            }
            for (int m = 0; m < nv; m++)
                for (int l = 0; l < nv; l++)
                    A[m][l] = Gm[m][l] / dtau + b0 / o->dt * Pm[m][l];
            real rhs[5];
            for (int m = 0; m < nv; m++)
                rhs[m] = -((b0 * (Q[m] - qn[m * n + c]) - b2 * (qn[m * n + c] - qnm1[m * n + c])) /
                               o->dt +
                           r[m * n + c]);
            gauss_solve(nv, A, rhs);
            for (int m = 0; m < nv; m++)
                wtmp[s + m * vs] = w[s + m * vs] + rhs[m];
        }
        memcpy(w, wtmp, sizeof(double) * nv * vs);
    }
    free(r);
}

void orc_dual_step(orc *o, double *w, double *wtmp, real *qn, real *qnm1, int first,
                   double t_new)
{
    orc_dual_begin(o, w, qn, qnm1, first, t_new);
    orc_dual_iterate(o, w, wtmp, qn, qnm1, first, t_new, o->n_inner);
}

/* --------------------------------------------------------- surface forces */
/* p - p_inf of the state at offset s, without forming p_inf + p' for dual
 * time (whose state holds p' itself). */
static double state_pprime(const orc *o, const double *q, long s)
{
    if (o->scheme == ORC_DUAL)
        return q[s];
    return state_prim(o, q, s).p - o->pinf;
}

/* Section 6, eq.9: the force on the body, F_i = integral over the surface of
 * (-P delta_ij + tau_ij) n_j, with the surface values sampled by inverse
 * distance weighting (section 4.6).  The paper gives no quadrature; the
 * reading:
 *  - one point per facet: its centroid (2D: the segment midpoint), weighted
 *    by the facet's length (2D, per unit span) or area, with the facet's
 *    outward unit normal;
 *  - P enters as P - p_inf: the constant adds -p_inf times the sum of the
 *    facets' area vectors, zero for a closed surface (or a prism periodic
 *    along its axis), and is left out so that nothing of size p_inf is
 *    rounded at low Mach;
 *  - P - p_inf and the velocity gradient at the point: weights 1/r^2 over
 *    the centres of the enclosing cell box (4 or 8 cells; periodic axes
 *    wrap) that are FLUID or FORCING, normalised; a centre at r = 0 takes the
 *    whole weight; a point with no such centre adds nothing and is counted;
 *  - the gradient at a cell: central differences over its face neighbours
 *    (halo cells included), (u(+) - u(-)) / (x(+) - x(-));
 *  - tau_ij = mu (d_j u_i + d_i u_j - 2/3 delta_ij div u), formed at the point
 *    from the interpolated gradient.
 * q must be filled (IB nodes and halo).  F[0..2] (F_z = 0 in 2D); per facet
 * (facet_out may be NULL): P - p_inf, (tau n)_x, (tau n)_y, (tau n)_z, the
 * facet's area.  Returns the number of facets with no valid centre. */
int orc_forces(orc *o, const double *q, double *F, double *facet_out)
{
    int nd = o->ndim, nc = 1 << nd, missed = 0;
    int per[3] = {o->bc[0] == ORC_BC_PERIODIC, o->bc[2] == ORC_BC_PERIODIC, o->bc[4] == ORC_BC_PERIODIC};
    const double *cen[3] = {o->xc, o->yc, o->zc};
    int nn[3] = {o->ni, o->nj, o->nk};
    F[0] = F[1] = F[2] = 0.0;
    for (int f = 0; f < o->nfacet; f++) {
        /* centroid, measure, outward normal */
        double y[3] = {0.0, 0.0, 0.0}, area;
        const int *fv = o->facet + nd * f;
        for (int m = 0; m < nd; m++)
            for (int d = 0; d < nd; d++)
                y[d] += o->v[nd * fv[m] + d] / nd;
        if (nd == 2) {
            double ex = o->v[2 * fv[1]] - o->v[2 * fv[0]], ey = o->v[2 * fv[1] + 1] - o->v[2 * fv[0] + 1];
            area = sqrt(ex * ex + ey * ey);
        } else {
            double e1[3], e2[3], cr[3];
            for (int d = 0; d < 3; d++) {
                e1[d] = o->v[3 * fv[1] + d] - o->v[3 * fv[0] + d];
                e2[d] = o->v[3 * fv[2] + d] - o->v[3 * fv[0] + d];
            }
            cross3(e1, e2, cr);
            area = 0.5 * sqrt(dot3(cr, cr));
        }
        const double *n = o->fnrm + 3 * f;
        /* enclosing box and inverse-distance weights */
        int i0[3] = {0, 0, 0}, ok = 1;
        double fr[3];
        for (int d = 0; d < nd && ok; d++)
            ok = locate(cen[d], nn[d], per[d], y[d], &i0[d], &fr[d]);
        double w[8] = {0.0}, wsum = 0.0;
        long cs[8] = {0};
        int zero = -1, nvalid = 0;
        for (int m = 0; m < nc && ok; m++) {
            int b[3] = {m & 1, (m >> 1) & 1, (m >> 2) & 1}, ci[3] = {0, 0, 0};
            double r2 = 0.0;
            for (int d = 0; d < nd; d++) {
                ci[d] = wrap(i0[d] + b[d], nn[d]);
                double dx = y[d] - cen[d][i0[d] + b[d] + 3];
                r2 += dx * dx;
            }
            uint8_t t = o->cls[cidx(o, ci[0], ci[1], ci[2])];
            cs[m] = sidx(o, ci[0], ci[1], ci[2]);
            if (t != ORC_FLUID && t != ORC_FORCING)
                continue;
            nvalid++;
            if (r2 == 0.0 && zero < 0)
                zero = m;
            w[m] = r2 > 0.0 ? 1.0 / r2 : 0.0;
        }
        double pp = 0.0, g[3][3] = {{0.0}};
        if (!ok || nvalid == 0) {
            missed++;
            area = 0.0;
        } else {
            if (zero >= 0)
                for (int m = 0; m < nc; m++)
                    w[m] = m == zero ? 1.0 : 0.0;
            for (int m = 0; m < nc; m++)
                wsum += w[m];
            for (int m = 0; m < nc; m++) {
                if (w[m] == 0.0)
                    continue;
                double wm = w[m] / wsum;
                int b[3] = {m & 1, (m >> 1) & 1, (m >> 2) & 1}, ci[3] = {0, 0, 0};
                for (int d = 0; d < nd; d++)
                    ci[d] = wrap(i0[d] + b[d], nn[d]);
                pp += wm * state_pprime(o, q, cs[m]);
                for (int d = 0; d < nd; d++) {
                    int cp[3] = {ci[0], ci[1], ci[2]}, cm[3] = {ci[0], ci[1], ci[2]};
                    cp[d] += 1;
                    cm[d] -= 1;
                    prim_t wp = state_prim(o, q, sidx(o, cp[0], cp[1], cp[2]));
                    prim_t wmn = state_prim(o, q, sidx(o, cm[0], cm[1], cm[2]));
                    double dxd = cen[d][ci[d] + 4] - cen[d][ci[d] + 2];
                    for (int i = 0; i < nd; i++)
                        g[i][d] += wm * (wp.u[i] - wmn.u[i]) / dxd;
                }
            }
        }
        double div = 0.0;
        for (int d = 0; d < nd; d++)
            div += g[d][d];
        double tn[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < nd; i++)
            for (int j = 0; j < nd; j++) {
                double tau = o->mu * (g[i][j] + g[j][i] - (i == j ? 2.0 / 3.0 * div : 0.0));
                tn[i] += tau * n[j];
            }
        for (int i = 0; i < nd; i++)
            F[i] += area * (-pp * n[i] + tn[i]);
        if (facet_out) {
            double *fo = facet_out + 5 * f;
            fo[0] = pp;
            fo[1] = tn[0];
            fo[2] = tn[1];
            fo[3] = tn[2];
            fo[4] = area;
        }
    }
    return missed;
}

/* ------------------------------------------------------------ threading */
/* Threads of the OpenMP loops (1 without OpenMP); results do not depend on it. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* -------------------------------------------------------------- accessors */
void orc_get_class(orc *o, uint8_t *cls)
{
    memcpy(cls, o->cls, (size_t)o->ni * o->nj * o->nk);
}

int orc_get_lists(orc *o, int32_t *listF, int32_t *listG, int32_t *counts)
{
    if (listF)
        memcpy(listF, o->listF, sizeof(int32_t) * o->nF);
    if (listG)
        memcpy(listG, o->listG, sizeof(int32_t) * o->nG);
    if (counts) {
        counts[0] = o->nF;
        counts[1] = o->nG1;
        counts[2] = o->nG2;
        counts[3] = o->nG3;
        counts[4] = o->nG;
    }
    return o->nF + o->nG;
}

void orc_get_records(orc *o, int which, int32_t *ifeat, double *dfeat)
{
    (void)which;
    int nrec = o->nF + o->nG;
    if (ifeat)
        memcpy(ifeat, o->irec, sizeof(int32_t) * IREC * nrec);
    if (dfeat)
        memcpy(dfeat, o->drec, sizeof(double) * DREC * nrec);
}

void orc_get_stats(orc *o, int64_t *s)
{
    s[0] = o->stat_fallback_pprime;
    s[1] = o->stat_fallback_probe;
    s[2] = o->stat_fallback_none;
    s[3] = o->stat_stencil_violation;
    s[4] = o->stat_fresh_cleared;
    s[5] = o->stat_fresh_violation;
}

double orc_get_param(orc *o, int which)
{
    switch (which) {
    case 0: return o->pinf;
    case 1: return o->R;
    case 2: return o->cp;
    case 3: return o->mu;
    case 4: return o->kc;
    case 5: return o->uc2;
    case 6: return (double)o->disp / LAT_SCALE;
    default: return 0.0;
    }
}
