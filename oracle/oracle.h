/*
 * CPU oracle for the all-speed sharp-interface immersed-boundary finite-volume
 * step (Seshadri & De, arXiv 1912.11908).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this code: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.  It is a plain, slow, FP64 implementation written from
 * the paper's description (sections 2-6) and the readings listed with each
 * function; it shares no source with the HIP path.
 *
 * Layout conventions used by every entry point:
 *   - state arrays are [nv][nk + 2*hz][nj + 6][ni + 6] doubles (i fastest),
 *     nv = ndim + 2, 3 halo cells per side in x and y, hz = 3 in 3D, 0 in 2D;
 *   - residual arrays are [nv][nk][nj][ni] (interior cells only);
 *   - class arrays are uint8 [nk][nj][ni].
 */
#ifndef IBM_ORACLE_H
#define IBM_ORACLE_H
#include <stddef.h>
#include <stdint.h>

/* scalar type of the flow half: double unless a wider build sets it */
#ifndef ORC_REAL
#define ORC_REAL double
#endif
typedef ORC_REAL orc_real;

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc orc;

enum { ORC_FLUID = 0, ORC_FORCING = 1, ORC_G1 = 2, ORC_G2 = 3, ORC_G3 = 4, ORC_SOLID = 5 };
enum { ORC_BC_FARFIELD = 0, ORC_BC_EXTRAP = 1, ORC_BC_PERIODIC = 2 };
enum { ORC_RK3 = 0, ORC_DUAL = 1 };
enum { ORC_IB_LINEAR = 0, ORC_IB_QUADRATIC = 1 };
enum { ORC_WALL_EQ6 = 0, ORC_WALL_EQ7 = 1 };
enum { ORC_RECON_WENO5 = 0, ORC_RECON_TVD2 = 1 };
/* RTLN: ray-tracing classification and local normals (the paper's
 * framework); SDSN: signed-distance classification and surface normals (the
 * standard HCIB/GC it is compared with; 2D) */
enum { ORC_FRAME_RTLN = 0, ORC_FRAME_SDSN = 1 };

orc *orc_create(int ndim, int ni, int nj, int nk, const double *xf, const double *yf,
                const double *zf, const int *bc, int nvert, int nfacet, const double *vert,
                const int *facet, double mach, double re, double pr, double gamma, int scheme,
                int family, double dt, double cfl_tau, int n_inner, int motion,
                const double *mpar, const double *uinf, int wall_pressure, int reconstruction,
                int framework);
void orc_destroy(orc *o);

/* a1: body pose at time t (no-op for a stationary body). */
void orc_set_pose(orc *o, double t);
/* free body (motion 2): displacement, velocity and acceleration along the
 * motion axis used by the next pose and fills */
void orc_set_body(orc *o, double x, double u, double a);
/* a2 + a3: classification, tagging and list compaction; returns 0 or <0. */
int orc_classify(orc *o);
/* a4: closest feature, local normal, boundary point and probes per listed node. */
int orc_geometry(orc *o);
/* a5: domain ghost layers and immersed-boundary fill at time t. */
void orc_bc(orc *o, double *q);
void orc_fill(orc *o, double *q, double t);
/* a6-a9: residual R = (1/V) sum_f (F_inv - F_visc) . S on FLUID cells. */
void orc_residual(orc *o, const double *q, double *r);
/* a10: one SSP-RK3 step (3 stages), or one physical dual-time step. */
void orc_rk3_step(orc *o, double *q, double *q1, double *q2, double t);
/* qn, qnm1: the step history Q^n, Q^{n-1}, conserved, [nv][nk][nj][ni], in the
 * flow half's scalar type (orc_real_bytes() bytes per value) */
void orc_dual_step(orc *o, double *w, double *wtmp, orc_real *qn, orc_real *qnm1, int first,
                   double t_new);
void orc_dual_begin(orc *o, const double *w, orc_real *qn, orc_real *qnm1, int first, double t_new);
void orc_dual_iterate(orc *o, double *w, double *wtmp, const orc_real *qn, const orc_real *qnm1,
                      int first, double t_new, int n_iter);
size_t orc_real_bytes(void);
/* state <-> primitive (rho, u, v[, w], p) on interior cells. */
void orc_prim_to_state(orc *o, const double *prim, double *q);
void orc_state_to_prim(orc *o, const double *q, double *prim);

/* accessors for tests */
/* section 6, eq.9: force on the body of a filled state; returns the number
 * of facets with no FLUID / FORCING centre around their centroid */
int orc_forces(orc *o, const double *q, double *F, double *facet_out);
void orc_get_class(orc *o, uint8_t *cls);
int orc_get_lists(orc *o, int32_t *listF, int32_t *listG, int32_t *counts);
void orc_get_records(orc *o, int which, int32_t *ifeat, double *dfeat);
void orc_get_stats(orc *o, int64_t *stats);
double orc_get_param(orc *o, int which);

/* OpenMP threads of the cell loops (timing only; results do not depend on it) */
void orc_set_threads(int n);
int orc_get_threads(void);

/* pins */
double orc_weno5(double a, double b, double c, double d, double e);
/* second-order TVD face state (MUSCL, minmod) seen from b, between b and c */
double orc_tvd2(double a, double b, double c);
void orc_ldfss(int ndim, const double *wl, const double *wr, const double *nrm, double gamma,
               int precond, double uc2, double *flux);

#ifdef __cplusplus
}
#endif
#endif
