/*
 * ibm.h -- C ABI of the MI355X (gfx950) immersed-boundary step library.
 *
 * The library advances the compressible Navier-Stokes equations on a
 * rectilinear cell-centred finite-volume grid with a sharp-interface
 * immersed body, following Seshadri & De, "A novel sharp interface immersed
 * boundary framework for viscous flow simulations at arbitrary Mach number
 * involving complex and moving boundaries" (arXiv 1912.11908):
 *   - node classification by ray casting with crossing parity (section 3.2),
 *   - forcing (IB) and three ghost layers (sections 3.2 and 5),
 *   - closest feature, angle-weighted pseudo-normals and the local-normal
 *     reconstruction direction (section 4, eqs 1-3),
 *   - boundary conditions eqs 4-6 and 8 with inverse-distance / image-point
 *     (compressible) or quadratic (incompressible) reconstruction
 *     (sections 4.4-4.6 and 5),
 *   - WENO5 reconstruction, low-diffusion flux splitting with low-Mach
 *     preconditioning and central viscous fluxes (section 2),
 *   - explicit SSP-RK3 or preconditioned dual time stepping (section 2).
 *
 * Conventions shared by every entry point
 *   Units: rho_inf = U_inf = T_inf = 1, U_inf along +x, p_inf = 1/(gamma M^2),
 *     gas constant R = p_inf, mu = 1/Re (constant), conductivity mu c_p / Pr.
 *   State layout (device, double): [nv][nk + 2*hz][nj + 6][ni + 6], i fastest,
 *     nv = ndim + 2, three halo cells per side in x and y, hz = 3 in 3D and 0
 *     in 2D.  For IBM_RK3 the state is conserved (rho, rho u, rho v[, rho w],
 *     rho E); for IBM_DUAL it is the primitive perturbation
 *     (p - p_inf, u, v[, w], T - 1).
 *   Interior arrays (residuals, primitives, classes): [..][nk][nj][ni].
 *   Classes: IBM_FLUID, IBM_FORCING (fluid cell with a solid face
 *     neighbour), IBM_G1..IBM_G3 (ghost layers), IBM_SOLID.
 *   Streams are hipStream_t passed as void*; NULL means the default stream.
 *   Every device buffer is allocated by the caller and must stay valid while
 *   work that uses it is in flight; the library never allocates or frees
 *   device memory.  The workspace handed to ibm_create belongs to the context
 *   until ibm_destroy.
 *   Calls enqueue work asynchronously and do not synchronise, except
 *   ibm_create (uploads the geometry), ibm_status and ibm_read_counts.
 *   One context is used by one host thread at a time; distinct contexts are
 *   independent.
 *   Return codes: IBM_OK (0) or a negative IBM_E* code; ibm_last_error gives
 *   a message.  Nothing aborts and no C++ exception crosses the ABI.
 */
#ifndef IBM_H
#define IBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IBM_OK 0
#define IBM_EINVAL (-1)      /* bad argument, shape or descriptor             */
#define IBM_EGEOM (-2)       /* body out of the lattice range or degenerate   */
#define IBM_EDEVICE (-3)     /* HIP error (code in ibm_last_error)            */
#define IBM_ENONFINITE (-4)  /* non-finite or non-positive rho/p in a cell    */
#define IBM_ENOSPACE (-5)    /* workspace smaller than ibm_workspace_bytes    */
#define IBM_ECAPACITY (-6)   /* more IB nodes than the workspace can hold     */

enum { IBM_BC_FARFIELD = 0, IBM_BC_EXTRAP = 1, IBM_BC_PERIODIC = 2 };
enum { IBM_RK3 = 0, IBM_DUAL = 1 };
enum { IBM_IB_LINEAR = 0, IBM_IB_QUADRATIC = 1 };
enum { IBM_FP64 = 0, IBM_MIXED = 1 };
enum { IBM_FLUID = 0, IBM_FORCING = 1, IBM_G1 = 2, IBM_G2 = 3, IBM_G3 = 4, IBM_SOLID = 5 };
enum { IBM_WALL_EQ6 = 0, IBM_WALL_EQ7 = 1 };
enum { IBM_RECON_WENO5 = 0, IBM_RECON_TVD2 = 1 };
/* IB framework: ray-tracing classification with local normals (sections 3-4),
 * or the standard HCIB/GC one it is compared with in section 7: signed-distance
 * classification (inside where (X - P0) . n_f < 0, n_f the outward normal of
 * the closest facet, lowest id among equals) with the facet normal through the
 * closest point as the reconstruction direction. */
enum { IBM_FRAME_RTLN = 0, IBM_FRAME_SDSN = 1 };

/* Case descriptor; all pointers are host pointers, copied by ibm_create. */
typedef struct ibm_case {
    int ndim;                 /* 2 or 3                                            */
    int ni, nj, nk;           /* interior cells per axis (nk = 1 when ndim = 2)    */
    const double *xf, *yf, *zf; /* face coordinates, ni+1 / nj+1 / nk+1, increasing */
    int bc[6];                /* x-, x+, y-, y+, z-, z+: IBM_BC_*                   */
    int nvert, nfacet;        /* body size (0 facets: no body)                     */
    const double *vert;       /* nvert * ndim coordinates (rest pose)              */
    const int32_t *facet;     /* 2D: nfacet * 2 vertex ids, counter-clockwise      */
                              /* polygon; 3D: nfacet * 3 ids, counter-clockwise    */
                              /* seen from outside                                 */
    int motion;               /* 0: stationary; 1: prescribed translation along    */
                              /* one axis; 2: free translation along one axis      */
                              /* (section 6, eq.10; IBM_RK3 only)                  */
    double motion_par[4];     /* 1: axis, amplitude A, frequency f, phase:         */
                              /* x_axis(t) = A cos(2 pi f t + phase) + V t         */
                              /* (section 8.2.2; V = motion_vel, section 8.2.3);   */
                              /* 2: axis, mass (rho_inf L^ndim units; 2D: per unit */
                              /* span), -, -; motion_vel is the initial velocity   */
    double mach, reynolds, prandtl, gamma;
    int scheme;               /* IBM_RK3 or IBM_DUAL                               */
    int ib_family;            /* IBM_IB_LINEAR (IDW + image point) or QUADRATIC    */
    int precision;            /* IBM_FP64, or IBM_MIXED: FP32 reconstruction and   */
                              /* fluxes on perturbation variables, FP64 update     */
    double dt;                /* physical time step                                */
    double cfl_tau;           /* pseudo-time CFL (dual time)                       */
    int n_inner;              /* pseudo-iterations per physical step (dual time)   */
    double u_inf[3];          /* free-stream velocity (unused components 0); M and */
                              /* Re take unit reference speed: |u_inf| = 1, or     */
                              /* u_inf = 0 for a body moving in still fluid        */
    double motion_vel;        /* V: constant speed along the motion axis           */
    int wall_pressure;        /* IBM_WALL_EQ6: dp/dn = -rho a_n (eq.6);            */
                              /* IBM_WALL_EQ7: dp/dn = rho u_t^2 / R - rho a_n     */
                              /* (eq.7, supersonic moving bodies; 2D only)         */
    int reconstruction;       /* IBM_RECON_WENO5 (fifth order) or IBM_RECON_TVD2   */
                              /* (second-order MUSCL, minmod limiter) (section 2)  */
    int ib_framework;         /* IBM_FRAME_RTLN or IBM_FRAME_SDSN                  */
} ibm_case;

typedef struct ibm_ctx ibm_ctx;

/* Device pointers into the context's workspace, for inspection. */
typedef struct ibm_info {
    int ndim, ni, nj, nk, nv;
    long long state_elems;    /* doubles per state array (nv * extended cells)     */
    long long ncell;          /* interior cells                                    */
    int cap_nodes;            /* capacity of each IB node list                     */
    int region[6];            /* IB region box [i0,i1) [j0,j1) [k0,k1)             */
    uint8_t *cls;             /* class per interior cell                           */
    int32_t *counts;          /* nF, nG1, nG2, nG3, nG, status, fallbacks x2       */
    int32_t *list_forcing;    /* cell ids of FORCING nodes, raster order           */
    int32_t *list_ghost;      /* cell ids of G1..G3 nodes, raster order            */
    int32_t *rec_int;         /* per record (forcing first, then ghosts):          */
                              /* IBM_REC_INT int32s                                */
    double *rec_dbl;          /* per record IBM_REC_DBL doubles                    */
    double time;              /* current solution time                             */
} ibm_info;

#define IBM_REC_INT 24
#define IBM_REC_DBL 32

/* Bytes of device workspace a case needs (host-only; no device work).
 * Returns IBM_EINVAL for an invalid descriptor. */
int ibm_workspace_bytes(const ibm_case *c, size_t *bytes);

/* Create a context bound to the current HIP device.  Copies the descriptor's
 * host arrays, builds facet normals and the pseudo-normals of eqs 2-3 on the
 * host, and uploads grid and body data into d_workspace (synchronous).
 * bytes must be at least ibm_workspace_bytes(c). */
int ibm_create(const ibm_case *c, void *d_workspace, size_t bytes, ibm_ctx **out);
void ibm_destroy(ibm_ctx *ctx);

/* Solution time used by the next ibm_classify / ibm_advance call: the pose
 * of a moving body (the prescribed translation of section 8.2.2, at
 * constant speed in section 8.2.3) and the body velocity and acceleration
 * of the wall conditions (eqs 4-7, section 4.4) are evaluated at it.
 * IBM_EINVAL for a non-finite t; no device work. */
int ibm_set_time(ibm_ctx *ctx, double t);

/* a1-a4: pose the body at the context time, classify every cell by ray
 * parity (section 3.2), tag FORCING and G1-G3, compact the node lists in
 * raster order, and build per-node reconstruction records: closest feature,
 * local normal, boundary point P' and probe stencils (section 4). */
int ibm_classify(ibm_ctx *ctx, void *stream);

/* a5: fill the immersed-boundary nodes of d_q at time t (FORCING first, then
 * the ghost layers G1-G3), eqs 4-6 and 8, and then the domain ghost layers
 * (three per side) as images of the filled interior. */
int ibm_fill(ibm_ctx *ctx, double *d_q, double t, void *stream);

/* a6-a9 (section 2: cell-centred finite volumes with fifth-order WENO face
 * states, low-diffusion flux splitting, preconditioned in dual time, and
 * second-order central viscous fluxes; the unknowns of section 4.4):
 * residual R = (1/V) sum_faces (F_inv - F_visc) . S of d_q on FLUID cells
 * (zero elsewhere), in conserved form, device interior layout
 * [nv][nk][nj][ni] (caller-owned, nv * ncell doubles).  d_q's IB nodes must
 * already be filled (ibm_fill); its halo is not read: stencils resolve
 * domain ghost cells from the interior by the rules of the boundary types.
 * IBM_EINVAL for null pointers; asynchronous on stream. */
int ibm_residual(ibm_ctx *ctx, const double *d_q, double *d_r, void *stream);

/* Section 6, eq.9: the force on the body, F_i = surface integral of
 * (-P delta_ij + tau_ij) n_j, from the state d_q, whose IB nodes and halo
 * must be filled (ibm_fill), at the pose of the last classification.  One
 * point per facet (centroid; 2D: segment midpoint) weighted by the facet's
 * length (per unit span) or area, outward unit normal; P - p_inf and the
 * velocity gradient at the point by inverse-distance weights (1/r^2) over the
 * centres of the enclosing cell box that are FLUID or FORCING (a centre at
 * r = 0 takes the whole weight), the gradient at a cell by central
 * differences over its face neighbours; tau = mu (grad u + grad u^T -
 * 2/3 div u I).  Nondimensional (rho_inf U_inf^2 L^(ndim-1)).
 * d_force: device, 3 doubles (F_z = 0 in 2D).  d_facet: device or NULL,
 * nfacet rows of 5 doubles: P - p_inf, (tau n)_x, (tau n)_y, (tau n)_z, area.
 * d_missed: device int32 or NULL: facets with no FLUID / FORCING centre
 * around them (they add nothing).  Asynchronous on stream; the sums are
 * taken in a fixed order (reproducible).  IBM_EINVAL without a body. */
int ibm_forces(ibm_ctx *ctx, const double *d_q, double *d_force, double *d_facet, int32_t *d_missed,
               void *stream);

/* For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * force of ibm_forces, same arguments and bit-identical results, whose
 * reduction scratch (block sums and, when d_missed is NULL, the
 * facets-missed counter) lives in a fixed device array of the library
 * instead of the context's workspace; nothing is allocated, no memset is
 * enqueued.  Limit: IBM_FORCES_STATIC_MAX_FACETS facets (IBM_EINVAL beyond
 * it); the context's device must be current.  The array is per device and
 * shared by every call on that device: calls whose work overlaps on one
 * device (other streams, other threads) race and must be serialised by the
 * caller. */
#define IBM_FORCES_STATIC_MAX_FACETS 262144
int ibm_forces_static(ibm_ctx *ctx, const double *d_q, double *d_force, double *d_facet, int32_t *d_missed,
                      void *stream);

/* Free body (motion 2): displacement, velocity and acceleration along the
 * axis after the last step, and the axial force of that step (host out[4]).
 * Each step of a free body: pose at x^n, fill and ibm_forces at t^n (the
 * only host synchronisation of the step), a^n = F^n / M, the RK3 stages with
 * the body moving at u^n and accelerating at a^n, then eq.10 with the 1/2 of
 * the standard Verlet form: x^{n+1} = x^n + u^n dt + dt^2 a^n / 2,
 * u^{n+1} = u^n + dt a^n.  IBM_EINVAL for other motions. */
int ibm_body_state(const ibm_ctx *ctx, double *out);

/* a1-a10: advance nsteps SSP-RK3 steps (IBM_RK3) or physical dual-time steps
 * of n_inner pseudo-iterations each (IBM_DUAL; section 2: three-point
 * physical-time and two-point pseudo-time differencing), in place on d_q,
 * each stage filling the IB nodes first (sections 4.4-5).  Moving bodies
 * are reclassified at every step (sections 3.2 and 5), at the pose of the
 * step's start time (RK3) or end time (dual time).  The interior (IB nodes
 * included) is advanced; d_q's halo is neither read nor written (call
 * ibm_fill for a filled halo).  IBM_EINVAL for a null state or nsteps < 0;
 * device errors and non-finite states are reported by ibm_status. */
int ibm_advance(ibm_ctx *ctx, double *d_q, int nsteps, void *stream);

/* Serving (several independent solves, e.g. under continuous batching):
 * advance each ctx[m] by nsteps steps on its state d_q[m], as ibm_advance
 * would, with bit-identical results.  Stationary-body solves that share
 * ndim, precision and scheme advance together: every stage of one step of
 * all of them is one launch over all their tiles, so many small solves fill
 * the GPU as one large one does.  Moving-body solves advance one after
 * another.  Contexts must be distinct and on the current device;
 * n <= IBM_BATCH_MAX.  The first call with a new d_q[m] copies that solve's
 * launch arguments into its workspace (asynchronously, on stream). */
int ibm_batch_advance(ibm_ctx *const *ctx, double *const *d_q, int n, int nsteps, void *stream);

/* Primitive (rho, u, v[, w], p) interior array -> state (halo untouched),
 * and back. */
int ibm_init_state(ibm_ctx *ctx, const double *d_prim, double *d_q, void *stream);
int ibm_state_to_prim(ibm_ctx *ctx, const double *d_q, double *d_prim, void *stream);

/* Synchronise the stream and report the sticky device status: IBM_OK,
 * IBM_ENONFINITE or IBM_ECAPACITY. */
int ibm_status(ibm_ctx *ctx, void *stream);

/* Copy the counts word array (8 int32) to host memory; synchronises. */
int ibm_read_counts(ibm_ctx *ctx, int32_t *host_counts, void *stream);

int ibm_info_get(const ibm_ctx *ctx, ibm_info *out);

/* Options.  IBM_OPT_GRAPHS (default 1): ibm_advance replays each step of a
 * stationary-body solve as a captured HIP graph (launched on the caller's
 * stream) instead of enqueuing its kernels one by one; 0 enqueues eagerly.
 * Both give bit-identical results. */
#define IBM_OPT_GRAPHS 1
/* IBM_OPT_CORNER_LISTS (default 1): each tile near the body fills, before
 * its ghost nodes, the FORCING probe corners they read outside its loaded
 * cells, listed at classification; 0 makes every ghost node fill its own
 * FORCING corners instead (the path a tile takes when its list does not
 * fit).  Both give bit-identical results; takes effect at the next
 * classification. */
#define IBM_OPT_CORNER_LISTS 2
/* IBM_OPT_STAGE_TIMING (default 0): value n > 0 makes the next n stage
 * launches of ibm_advance (each RK3 stage or dual-time pseudo-iteration of
 * the fused residual-and-update kernel, section 2) record HIP events at
 * their start and end (a 3D FP64 stage with a body: from the start of its
 * two fill launches to the end of its stage kernel), read back by
 * ibm_stage_timing; while it is on, steps
 * are enqueued eagerly (no graph replay).  0 turns it off.  At most
 * IBM_STAGE_TIMING_MAX.  Changing it discards unread timings. */
#define IBM_OPT_STAGE_TIMING 3
/* IBM_OPT_PIPELINE (default 1): a prescribed-motion solve classifies the
 * next step (pose, ray parity, tags, lists, records) on a stream of its own
 * into a second set of buffers while the current step's stages run on the
 * caller's stream (joined by events); 0 classifies each step on the
 * caller's stream before its stages.  Both give bit-identical results. */
#define IBM_OPT_PIPELINE 4
#define IBM_STAGE_TIMING_MAX 100000
#define IBM_BATCH_MAX 64
int ibm_set_option(ibm_ctx *ctx, int option, int value);
const char *ibm_last_error(const ibm_ctx *ctx);

/* Stage timing (section 2's residual and update, one launch per RK3 stage
 * or pseudo-iteration): synchronises on the last timed launch and returns
 * the summed device time of the stage launches timed since the option was
 * set or since the last call (total_ms, host), their number (launches) and,
 * if not NULL, the shortest and longest (min_ms, max_ms); then starts
 * counting again.  Zero launches when the option is off. */
int ibm_stage_timing(ibm_ctx *ctx, float *total_ms, int *launches, float *min_ms, float *max_ms);

/* Average device time in milliseconds of one launch of the fused
 * residual-and-update kernel (section 2) of the given RK3 stage (1..3) or of
 * one dual-time pseudo-iteration (stage 0, BDF2 coefficients), measured with
 * HIP events around nrep launches on stream.  It is the kernel a step
 * launches, on the same tiles: with a body, the tile list whose near tiles
 * fill the IB nodes they read (body at the context time); for a 3D FP64
 * solve with a body, the two fill launches on a copy of d_q in the
 * context's scratch, then the kernel over every tile (the time spans the
 * three).  d_q is the input; the output goes to the context's scratch stage
 * buffer, so neither d_q nor the solve's dual-time history changes.  Dual
 * time needs one advanced step first (IBM_EINVAL otherwise).  Synchronises. */
int ibm_time_update_kernel(ibm_ctx *ctx, const double *d_q, int stage, int nrep, void *stream,
                           float *avg_ms);

#ifdef __cplusplus
}
#endif
#endif
