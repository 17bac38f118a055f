// Internal structures shared by the host orchestration (api.cpp) and the
// HIP kernels (geometry.hip, flow.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ibm.h"

namespace ibm {

constexpr double kLatScale = 16777216.0;  // 2^24: lattice of the exact predicates
constexpr int kRecI = IBM_REC_INT;
constexpr int kRecD = IBM_REC_DBL;

// counts[] words on the device
enum { CNT_F = 0, CNT_G1 = 1, CNT_G2 = 2, CNT_G3 = 3, CNT_G = 4, CNT_STATUS = 5,
       CNT_FB_PPRIME = 6, CNT_FB_PROBE = 7, CNT_WORDS = 8 };
enum { ST_NONFINITE = 1, ST_CAPACITY = 2 };

// Grid description in device memory.  Extended per-axis arrays hold the
// three halo cells on each side: centre index i lives at [i + 3].
struct Grid {
    int ndim, ni, nj, nk, nv, hz;
    int sx, sy, sz;          // extended sizes
    long long vs;            // doubles per state variable
    long long ncell;         // interior cells
    int bc[6];
    const double *xc[3];     // extended centres (n + 6)
    const double *xf[3];     // extended faces (n + 7), face f at [f + 3]
    const double *rdx[3];    // 1 / cell width, extended (n + 6)
    const double *rdxc[3];   // 1 / (xc[i+1] - xc[i]), index [i + 3]
    const double *rdtc[3];   // 1 / (xc[i+1] - xc[i-1]), index [i + 3]
    const float *rdx_f[3], *rdxc_f[3], *rdtc_f[3];
    const long long *Xc[3];  // lattice centres, interior
};

struct Body {
    int nvert, nfacet, nedge;
    const long long *V0;     // lattice vertices at rest (nvert * ndim)
    long long *V;            // posed lattice vertices
    double *v;               // posed vertices (exact V / 2^24)
    const int *facet;        // nfacet * ndim
    const double *fnrm;      // nfacet * 3
    const double *vnrm;      // nvert * 3
    const double *enrm;      // nedge * 3 (3D)
    const int *edge_of;      // nfacet * 3 (3D): global edge id per facet edge
    const double *fcurv;     // 2D: signed curvature per segment (eq.7)
    const double *vcurv;     // 2D: signed curvature per vertex
    // 3D facet bins in the rest frame (uniform cubes of side bin_h from
    // bin_o; a facet is listed in every bin its bounding box meets), CSR:
    // bin_start[nbin + 1], bin_facet; nbin = 0 for brute-force search
    double bin_o[3], bin_h;
    int bin_n[3], nbin;
    const int *bin_start, *bin_facet;
    // per bin listing (beside bin_facet): the listed facet's rest-frame
    // bounding box lo[3], hi[3], rounded outward to float
    const float *bin_box;
    double disp[3];          // current displacement of the pose (exact)
    // IBM_FRAME_*; for the signed-distance classification the posed lattice
    // box of the vertices (cells outside it are outside the body)
    int frame;
    long long lat_lo[3], lat_hi[3];
};

struct Flow {
    double gamma, pinf, R, cp, mu, kc, pr, uc2, Hinf, dt, cfl_tau;
    double uinf[3], uinf2;   // free-stream velocity and its square
    double rR, gm1inv;       // 1 / R and 1 / (gamma - 1)
    int scheme, family, precision;
    int wallp;               // IBM_WALL_EQ6 / IBM_WALL_EQ7
    int recon;               // IBM_RECON_WENO5 / IBM_RECON_TVD2
};

// Immersed-boundary work area.
struct IB {
    int region[6];           // [i0,i1) [j0,j1) [k0,k1)
    int rw, rh, rd;          // region extents
    int words_per_row;       // toggle bitmask words per region row
    int cap;                 // capacity of each list and of the records
    uint8_t *cls;            // class per interior cell
    uint8_t *inside;         // inside flag per region cell
    uint32_t *toggle;        // crossing toggles per region row
    int32_t *counts;         // CNT_* words
    // the other classification buffer's counts (null with one buffer): the
    // sticky status bits are set in both, so either buffer's word is whole
    int32_t *counts_other;
    int32_t *blk;            // per-block counts: FORCING, ghosts (scanned), G1, G2, G3 (5 * nblk)
    int nblk;
    int32_t *listF, *listG;
    int32_t *rec_i;          // cap * kRecI
    double *rec_d;           // cap * kRecD
    // fill plan (structure of arrays, cap entries each): state offsets of the
    // node and of its probe corners (unused corners point at the node with
    // weight 0), weights, line geometry n0 n1 n2 s_X s1 s2, modes
    int32_t *plan_node;      // cap
    int32_t *plan_off;       // 16 * cap: probe 1 corners 0..7, probe 2 corners 8..15
    double *plan_w;          // 16 * cap
    double *plan_geo;        // 6 * cap
    int32_t *plan_mode;      // cap: mode1 | mode2 << 4
    // 16 * cap, ghost records: the FORCING record of each weighted probe
    // corner that is a FORCING node (-1 otherwise, and for FORCING records)
    int32_t *plan_frec;
    double *plan_kappa;      // cap: surface curvature at the node's feature (2D, eq.7)
    double *fval;            // NV * cap: filled values of FORCING corners, by record
    int32_t *rmap;           // cap: record index per region cell (IB nodes only)
    // cap: per region cell, the closest facet that the last 3D search from
    // it found.  The next search starts from that facet's distance, which
    // bounds the minimum from above whatever facet it is, so an entry only
    // speeds the search up (out-of-range entries are ignored).
    int32_t *hint;
    // per near tile ("slot", a tile whose stencils reach the region): the
    // IB nodes (FORCING and G1-G3) among the cells it loads, as (tile-local
    // cell, record); rebuilt after every classification
    const int32_t *tile_slot;  // slot per tile id, -1 for the other tiles
    const int32_t *slot_tile;  // tile id per slot
    int32_t *tg_cnt;           // nslot
    int32_t *tg_t, *tg_rec;    // nslot * tg_stride
    // per slot: FORCING records outside the loaded cells that its ghost
    // nodes read as probe corners (repeats allowed; count -1 if they did
    // not fit, and the ghosts then fill those corners themselves)
    int32_t *tj_cnt;           // nslot
    int32_t *tj_rec;           // nslot * tg_stride
    int nslot, tg_stride;
};

// quotient and remainder of 0 <= x < 2^31 by n > 0 through the FP64
// reciprocal (a quotient off by at most one), then corrected exactly
__device__ inline int divmod_rcp(int x, int n, double rn, int &r)
{
    int q = (int)((double)x * rn);
    int rr = x - q * n;
    if (rr < 0) {
        --q;
        rr += n;
    } else if (rr >= n) {
        ++q;
        rr -= n;
    }
    r = rr;
    return q;
}

// (i, j, k) of cell id c = (k nj + j) ni + i
__device__ inline void split_cell(const Grid &g, int c, int &i, int &j, int &k)
{
    int q = divmod_rcp(c, g.ni, 1.0 / g.ni, i);
    k = divmod_rcp(q, g.nj, 1.0 / g.nj, j);
}

// The by-value argument block of a kernel whose only argument it is, read in
// place through a pointer into the constant kernel-argument segment: the
// compiler then loads each field where it is used instead of holding the
// whole block in scalar registers, which it would otherwise spill into
// vector-register lanes (a VALU instruction per reload).
template <typename T> __device__ __forceinline__ const T &kernarg_block()
{
    unsigned long long pa = reinterpret_cast<unsigned long long>(__builtin_amdgcn_kernarg_segment_ptr());
    unsigned plo = __builtin_amdgcn_readfirstlane((unsigned)pa);
    unsigned phi = __builtin_amdgcn_readfirstlane((unsigned)(pa >> 32));
    using Const = __attribute__((address_space(4))) const T;
    const Const *ap = (const Const *)(((unsigned long long)phi << 32) | plo);
    return *(const T *)ap;
}

// Set sticky status bits (ST_*) in the counts of every classification buffer.
__device__ inline void raise_status(const IB &ib, int32_t *counts, int bits)
{
    atomicOr(&counts[CNT_STATUS], bits);
    if (ib.counts_other)
        atomicOr(&ib.counts_other[CNT_STATUS], bits);
}

// Tiles of the fused residual/update kernel: cells per block along x, y, z.
constexpr int kTile2[3] = {16, 15, 1};  // 255 x-faces, 256 y-faces: one pass each
constexpr int kTile3[3] = {8, 7, 8};  // 504, 512, 504 faces: one pass each for 512 threads
// threads per block of the fused kernel: 2D 256, 3D 512
constexpr int kThreads2 = 256, kThreads3 = 512;

// The launch of the fused residual/update kernel for a stage with a body:
// a list of tiles (the near tiles among them fill, on the fly, the IB nodes
// they read) and the body's motion at the stage time.
struct StagePart {
    const int32_t *tiles;    // tile ids, -1 entries are padding
    int ntiles;
    double ub, ab;           // body velocity and acceleration along `axis`
    int axis;                // motion axis, -1 for a stationary body
    // when set, the launch records these events at its start and end (stage
    // timing); null otherwise
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    // 3D FP64: the stage fills the IB nodes of its input in place (the
    // standalone fill launches), then runs the plain kernel over every tile;
    // `tiles` is then unused
    bool prefill = false;
};

struct Motion {
    int on, axis;
    double amp, freq, phase, vel;
    // free rigid body (section 6): mass, and the displacement, velocity,
    // acceleration and axial force of its last step
    int free;
    double mass, x, u, a, force;
};

// ------------------------------------------------------------ launchers
// geometry.hip
hipError_t launch_pose(const Grid &g, Body &b, long long disp, int axis, hipStream_t s);
hipError_t launch_classify(const Grid &g, const Body &b, IB &ib, hipStream_t s);
hipError_t launch_records(const Grid &g, const Body &b, const Flow &f, IB &ib, hipStream_t s);
// forces.hip: surface force (eq.9) of a filled state; part holds
// 3 * forces_blocks(nfacet) doubles
int forces_blocks(int nfacet);
hipError_t launch_forces(const Grid &g, const Body &b, const Flow &f, const IB &ib, const double *q, double *force,
                         double *facet_out, double *part, int32_t *missed, hipStream_t s);
// the allocation-free variant's scratch on `device` (which must be current):
// room for the block sums of IBM_FORCES_STATIC_MAX_FACETS facets and the
// facets-missed counter
hipError_t forces_static_scratch(int device, double **part, int32_t **missed);
// *p = 0 by a one-thread kernel (no memset node when a caller captures)
hipError_t launch_zero_i32(int32_t *p, hipStream_t s);
// per near tile IB lists and FORCING corner lists (after the records)
hipError_t launch_ghost_lists(const Grid &g, const IB &ib, bool quad, bool corner_lists, hipStream_t s);
// cells a tile's stencils load (tile plus its halo) for this dimension
int tile_load_cells(int ndim);

// flow.hip
hipError_t launch_domain_bc(const Grid &g, const Flow &f, double *q, hipStream_t s);
// The IB nodes of q filled in place: FORCING nodes, then the ghost layers
// that read them (two launches; ev_start, when set, records the start of the
// first).
hipError_t launch_ib_fill(const Grid &g, const Flow &f, const IB &ib, double *q, double ub_axis, double ab_axis,
                          int axis, hipStream_t s, hipEvent_t ev_start);
hipError_t launch_bc_fill(const Grid &g, const Flow &f, const IB &ib, double *q, double ub_axis,
                          double ab_axis, int axis, hipStream_t s);
hipError_t launch_residual(const Grid &g, const Flow &f, const IB &ib, const double *q, double *r,
                           hipStream_t s);
// part: null runs every tile with no fill; the stencils resolve domain ghost
// cells on the fly, so the state's halo is never read
hipError_t launch_rk_stage(const Grid &g, const Flow &f, const IB &ib, const double *qn,
                           double *qin, double *qout, double a, double b, hipStream_t s,
                           const StagePart *part = nullptr);
hipError_t launch_dual_iter(const Grid &g, const Flow &f, const IB &ib, double *w,
                            double *wout, const double *qn, const double *qnm1, double b0,
                            double b2, hipStream_t s, const StagePart *part = nullptr);
hipError_t launch_dual_begin(const Grid &g, const Flow &f, const double *w, double *qn,
                             double *qnm1, int first, hipStream_t s);
hipError_t launch_prim_to_state(const Grid &g, const Flow &f, const double *prim, double *q,
                                hipStream_t s);
hipError_t launch_state_to_prim(const Grid &g, const Flow &f, const double *q, double *prim,
                                hipStream_t s);
hipError_t launch_copy_state(const Grid &g, const double *src, double *dst, hipStream_t s);

// Batched stages (several solves per launch): the arguments of one stage
// launch of a solve are written as stage_args_bytes() opaque bytes to host
// memory `dst` (to be copied to device memory); the return value is the
// launch's block count.  launch_stage_batch runs n prepared launches (device
// argument blocks d_args[m], block counts nblk[m]) of solves that share
// ndim, precision and scheme as one launch; ghosts selects the second
// launch of a stage.
size_t stage_args_bytes();
int stage_args(const Grid &g, const Flow &f, const IB &ib, double *qin, const double *qn,
               const double *qnm1, double *out, double a, double b, const StagePart *part, void *dst);
hipError_t launch_stage_batch(int ndim, int precision, int scheme, bool ghosts, int n, const void *const *d_args,
                              const int *nblk, hipStream_t s, hipEvent_t ev_start = nullptr,
                              hipEvent_t ev_stop = nullptr);

}  // namespace ibm
