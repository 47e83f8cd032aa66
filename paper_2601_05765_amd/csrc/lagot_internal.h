// lagot_internal.h -- device data layout and launch wrappers shared by the
// HIP kernel files and the C-ABI host driver (api.cpp). Not a public header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lagot {

// Facet storage: row-major blocks of FCAP entries per cell (cell i owns
// [i*FCAP, i*FCAP + fcnt[i])). The same layout holds the Hessian rows.
constexpr int FCAP = 64;
// Learned warm start: nearest sites per input, network sizes, flat parameter layout
// (W1 64x128, b1, W2 128x128, b2, W3 128x128, b3, w4 128, b4), float32.
constexpr int N_NEI = 16;
constexpr int MLP_IN = 64, MLP_HID = 128;
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = 8192, MLP_OFF_W2 = 8320, MLP_OFF_B2 = 24704, MLP_OFF_W3 = 24832,
              MLP_OFF_B3 = 41216, MLP_OFF_W4 = 41344, MLP_OFF_B4 = 41472, MLP_NPARAMS = 41473;
// Fast-path capacities of the cell kernel (float32, G lanes per cell).
constexpr int FAST_CMAX = 48;   // candidate bisectors (incl. walls) per cell
constexpr int FAST_PMAX = 32;   // planes of the polytope (6 auxiliary + cutting ones)
constexpr int FAST_VMAX = 64;   // polytope vertices (triangles of the dual)
// Large-capacity float64 path for cells flagged by the fast path.
constexpr int BIG_CMAX = 256;
constexpr int BIG_PMAX = 64;
constexpr int BIG_VMAX = 128;
constexpr int OVF_CMAX = 96;     // float64 pass for the cells the fast pass defers (crowded cells)
constexpr int OVF_PMAX = 64;
constexpr int OVF_VMAX = 128;
constexpr int OVERFLOW_ROUNDS = 8;  // clip rounds for cells with more candidates than CMAX
constexpr int CROWD_ROUNDS = 32;    // ... in the crowded pass (no threshold on t: rounds end when no
                                    // candidate cuts the polytope)
constexpr int SEED_CMAX = 64;    // seed pass of a crowded cell: its nearest sites (float32, 64 lanes)
constexpr int SEED_PMAX = 64;
constexpr int SEED_VMAX = 128;
// The fast pass defers a cell whose search block (sites within r + r_max) holds more
// sites than this: such a cell is crowded, and its neighbours are found from the
// geometry of the cells instead (seed pass, cell boxes, box-overlap candidates).
constexpr int FAST_SCAN_MAX = 1024;
// Box grids: QLEV levels of bucket size h 4^l (h: 1.2 site spacings). A cell box is
// registered at the finest level where it spans at most QREG_MAX buckets; boxes too
// large for every level go to a per-call list that every crowded cell tests directly.
constexpr int QREG_MAX = 27;
constexpr int QLEV = 3;

// Per-cell status bits written by the cell kernel.
enum CellFlag : uint32_t {
    CF_EMPTY = 1u << 0,     // the cell is empty (legitimate result)
    CF_CAND = 1u << 1,      // too many candidate planes
    CF_PLANES = 1u << 2,    // too many polytope planes
    CF_VERTS = 1u << 3,     // too many polytope vertices
    CF_TOPO = 1u << 4,      // inconsistent clip combinatorics (near-degenerate float geometry)
    CF_WALK = 1u << 5,      // facet polygon walk did not close
    CF_FACETS = 1u << 6,    // more than FCAP facets
    CF_PREC = 1u << 7,      // volume small against its ball: float32 pyramid sums cancel, redo in float64
    CF_FAIL_MASK = CF_CAND | CF_PLANES | CF_VERTS | CF_TOPO | CF_WALK | CF_FACETS,
};

struct GridDesc {
    float lo[3];      // box low corner
    float inv_s;      // 1 / grid cell size
    float s;          // grid cell size
    int dim[3];       // cells per axis
    int ncell;        // dim[0]*dim[1]*dim[2]
    int base;         // first entry of this grid in the shared cell_start array
    float hsp;        // typical site spacing of the instance: cbrt(sum nu / n), else cbrt(|box| / n)
    int pad;
};

struct BoxF {
    float lo[3], hi[3];
};

// ---- instances -------------------------------------------------------------
// A call solves B independent instances (B = 1 for lagot_solve). Instance b owns
// rows [off[b], off[b+1]) in caller order and in grid order alike: each instance
// has its own grid over its own box, and the spatial sort never moves a site out
// of its instance's range. Row-parallel kernels run over TILE-row tiles that
// never straddle two instances, so per-instance reductions are sums over a
// contiguous run of tile partials (fixed order, deterministic). A tile is one
// workgroup: TILE threads for row-wise kernels, 4 x TILE for the sparse products.
constexpr int TILE = 256;

// Per-instance control phase (device array, read by every kernel that may skip
// an instance).
enum Phase : int32_t {
    PH_DONE = 0,     // converged (or a single step taken): nothing more to do
    PH_ACTIVE = 1,   // accepted iterate above tolerance: needs a Newton direction
    PH_TRIAL = 2,    // in the step-size search
    PH_ACCEPT = 3,   // trial accepted in this round (transient)
    PH_FAILED = 4,   // stopped with an error status
    PH_START = 5,    // initial evaluation pending
    PH_RESTART = 6,  // empty start cell after a repair: restart from the default weights
    PH_REPAIR = 7,   // empty start cell: raise the weights of the empty cells to the default
};

struct Batch {
    int B;                       // instances
    int T;                       // tiles
    const int32_t *off;          // [B+1] first row of each instance
    const int32_t *tile_inst;    // [T] instance of each tile
    const int32_t *tile_row;     // [T] first row of each tile
    const int32_t *first_tile;   // [B+1] first tile of each instance
    const int32_t *inst;         // [n] instance of each row
    const GridDesc *grid;        // [B]
    const BoxF *box;             // [B]
    const double *rmax;          // [B] max sqrt(psi) over the instance (weights being evaluated)
    const int32_t *phase;        // [B] Phase
    const float4 *dom;           // [ndom] convex domain planes (unit outward normal, offset c: n.x <= c)
    int ndom;                    // 0: the box walls bound the cells
    // a union of convex pieces (npieces > 0): piece k holds planes dom[dom_off[k] .. dom_off[k+1]),
    // dom_wid[w] is plane w's wall (-1: a plane between pieces); the cell passes see one piece
    // at a time (npieces 0, dom and ndom of that piece)
    int npieces;
    const int32_t *dom_off;
    const int32_t *dom_wid;
    // local reach (null: r_max of the instance bounds every ball): ir[cgrid base + c] bounds
    // the radius of every ball whose site lies within twice its radius of coarse cell c
    const GridDesc *cgrid;       // [B] coarse grids (laid end to end)
    const float *ir;
};

constexpr int DOM_MAX = 32;      // planes of a convex polyhedral domain
constexpr int PIECE_MAX = 16;    // convex pieces of a non-convex domain
constexpr int PIECE_PLANES_MAX = 64;  // planes of all its pieces together
constexpr int AUX_PLANE_ID = -1000000;  // ids of the clipper's auxiliary cube planes (walls: -1-w)

// Workgroups are dealt to the 8 XCDs round-robin (workgroup w runs on XCD w mod 8),
// and each XCD has its own L2. This maps the hardware workgroup id to a logical one
// so that each XCD works through one contiguous run of logical ids: neighbouring
// rows (grid order = space order) then share an L2. A bijection on [0, n).
constexpr int NXCD = 8;
__device__ inline int xcd_block(int w, int n) {
    const int per = n / NXCD, rem = n % NXCD;  // XCD x gets per + (x < rem) ids
    const int x = w % NXCD, k = w / NXCD;
    if (k < per) return x * per + min(x, rem) + k;
    // the last round (w >= per * NXCD): only XCDs x < rem have an id left
    return x * per + x + per;
}

// Does instance b take part in a launch that selects phase `want` (< 0: all)?
__device__ inline bool selected(const Batch &bt, int want, int b) { return want < 0 || bt.phase[b] == want; }

// Newton state of one instance (device, one record per instance).
struct InstCtl {
    double eps0;       // KMT volume floor: 0.5 min(min nu, min V(psi_start))
    double alpha;      // current step length of the step-size search
    double gnorm;      // ||nu - V||_2 at the accepted iterate
    double maxrel;     // max |V - nu| / nu at the accepted iterate
    double minV;       // min V at the accepted iterate
    double sumV;       // sum V at the accepted iterate
    double tminV;      // min V and ||nu - V||_2 at the last step-size trial (diagnostic)
    double tgnorm;
    int iters, evals, halvings, hstep, cg_iters, status, default_start, learned;
    int restore;       // the float32 shadow must be reset to the accepted weights
    int repaired;      // empty start cells were given the default weight
    int iter_base;     // iterations before the current continuation stage (the limit counts from here)
    int pad;
    double alpha_acc;  // last accepted step length (1 at a start or a stage start)
    double alpha_first;  // the first accepted step length of the current continuation stage (0: none)
    double gnorm0;       // ||nu - V||_2 at the start of the current continuation stage
    double gnorm_prev;   // ||nu - V||_2 at the accepted iterate before the current one (0: none)
};

// Newton options as the device control kernels see them.
struct CtlOpts {
    double tol;
    int max_newton, max_halvings, single, allow_restart, residual_test;
    int repair_more;  // a repaired start that still has an empty cell is repaired again
    int stage_carry;  // a continuation stage's step search starts at the last stage's first accepted step
    double gtol;      // > 0: an intermediate stage also ends when ||nu - V||_2 <= gtol x its start value
};

// Views of the evaluation outputs (sorted site order).
struct EvalOut {
    double *V;        // [n] volume
    double *K;        // [n] spherical area
    float *wall;      // [6n] wall facet areas (may be null)
    int32_t *fcol;    // [n*FCAP] neighbour (sorted index)
    float *farea;     // [n*FCAP] facet area
    int32_t *fcnt;    // [n] facet count
    uint32_t *flags;  // [n] CellFlag bits
    int32_t *fb_list; // [n] cells to redo on the float64 path
    int32_t *fb_count;// [1] length of fb_list (device counter)
    int32_t *fb_inst; // [B] cells sent to the float64 path, per instance (accumulates over a call)
    int32_t *fail_inst; // [B] cells that failed the float64 path too, per instance (per evaluation)
    int32_t *ovf_list;  // [n] cells with more candidates than the fast kernel holds
    int32_t *ovf_count; // [1] length of ovf_list (device counter)
    double *cen;        // [3n] centroids in caller order (null: not computed)
};

// Cell boxes and the box grid of the crowded-cell pass (section 4, "Finding
// Contributing Neighbors"). Every evaluated cell writes an axis-aligned box that holds
// its restricted cell: the exact cell for cells finished by the fast pass, a superset
// (the cell clipped by its nearest sites only) for deferred ones. If sites i and j share
// a facet, the facet lies in both cells, so their boxes overlap: the candidates of a
// crowded cell are the sites whose boxes overlap its own. Boxes are registered in the
// buckets of a uniform grid (one per instance, GridDesc qgrid[b]) they overlap.
struct QBoxes {
    float4 *box;        // [2n] grid order: (lo.x, lo.y, lo.z, 0), (hi.x, hi.y, hi.z, 0); empty: lo > hi
    const GridDesc *qgrid;  // [B * QLEV] bucket grids (instance-major), laid end to end (base) in start/count/cursor
    int32_t *count;     // [nq + 1] boxes per bucket
    int32_t *start;     // [nq + 1] exclusive scan of count
    int32_t *cursor;    // [nq] fill cursors
    int32_t *ent;       // [QREG_MAX * n] cell ids per bucket
    int32_t *large;     // [n] cells whose boxes span more than QREG_MAX buckets
    int32_t *nlarge;    // [1]
    int32_t *tmp;       // [max(nq, n) / 1024 + 16] scan workspace
    int32_t *dcnt, *dstart;  // [n + 1] deferred-cell marks and their scan (the list in grid order)
    int nq;             // buckets over all instances
};

// Conjugate-gradient vectors and scalars (Chronopoulos-Gear form, one kernel per
// iteration). Per row, r, w = A u, s = A p and the Jacobi diagonal D form one 32-byte
// record, kept for two iterations (slot k % 2 is read by iteration k, slot (k+1) % 2
// written), so that a row can rebuild the next preconditioned residual of any
// neighbour from one record load; p and x are touched by their own row only.
struct RWSD {
    double r, w, s, d;
};
struct CgBufs {
    RWSD *rws[2];
    double *p, *x;           // x: the Newton direction
    double *part;            // partials per quarter tile (NS = 4T): gamma[2][NS], delta[2][NS],
                             // rho[2][NS], rho0[NS]
    double *cgs;             // [B][4] alpha and gamma of iterations k%2 = 0, 1
    double *sc;              // [B][2][4] gamma, delta, rho, rho0 summed from the partials of slot 0, 1
    int32_t *cgst;           // [B][4] iterations done, breakdown, converged, unused
    int32_t *kbase;          // [1] index of the first iteration of the next chunk
    int32_t *remaining;      // [1] instances still iterating after the last chunk
    int32_t *maxit;          // [1] most iterations any instance has done in this solve
    double *u;               // [n] u_{k+1} of every row (the split iteration's product input)
};

// Parameters of the velocity system of the fluid step (section 5, eq. (4)).
struct FluidPrm {
    double dt;        // time step
    double inv_eps2;  // 1 / eps^2 of the pressure spring (force m (c - p) / eps^2)
    double gamma;     // surface tension
    double mu;        // viscosity of every site when no per-site array is given
    double g[3];      // gravity (acceleration)
};

// Bounds of the position update: per-axis clamp interval, and the inward margin kept
// from every domain plane.
struct AdvectBounds {
    double lo[3], hi[3];
    double plane_margin;
};

// Jacobi-PCG of the three coordinates of the fluid velocity system at once (fluid.hip).
struct Rec3 {
    double r[3], w[3], s[3], d;  // per row and slot: r, w = A u, s = A p of 3 coordinates, diagonal
};
struct Cg3Bufs {
    Rec3 *rec[2];        // [n] per slot (iteration parity)
    double *p, *x;       // [3n] row-major (x: the solution)
    double *part;        // [21 nb]: per slot gamma[3], delta[3], rho[3] per block, then rho0[3]
    double *cgs;         // [2][3][2]: alpha and gamma per slot and coordinate
    double *sc;          // [2][12]: gamma[3], delta[3], rho[3], rho0[3] summed from the partials of a slot
    int32_t *st;         // [3][4]: iterations, breakdown, converged, unused
    int32_t *kbase;      // index of the first iteration of the next chunk
    int32_t *remaining;  // coordinates still iterating after the last chunk
    int nb;              // blocks (rows / 128, rounded up)
};

// ---- launch wrappers (defined in the .hip files) ----
// grid.hip
void launch_fill_inst(hipStream_t st, const Batch &bt, int32_t *inst);
void launch_zero_i32(hipStream_t st, int32_t *p, int64_t count);
// Non-convex domains (a union of convex pieces): the per-piece evaluation outputs are
// summed into accumulators (volume, area, facet lists merged by neighbour, walls by wall
// id, first moments), which the last call writes back as the evaluation's outputs.
struct PieceAcc {
    double *V, *K, *mom;   // [n], [n], [3n] (caller order: the first moments sum V_k c_k)
    int32_t *fcol;         // [n*FCAP]
    float *farea;          // [n*FCAP]
    int32_t *fcnt;         // [n]
    uint32_t *flags;       // [n]
    float *wall;           // [nwalls*n]
    double *cen;           // [3n] the piece pass's centroids (caller order)
};
void launch_piece_begin(hipStream_t st, bool first, int32_t *fb_count, int32_t *ovf_count, int32_t *ovf_sum);
void launch_zero_f32(hipStream_t st, float *p, int64_t count);
void launch_piece_accum(hipStream_t st, int64_t n, const Batch &bt, int want, bool first, const EvalOut &o,
                        int nw_piece, const int32_t *wid_piece, int nwalls, const int32_t *perm, PieceAcc acc);
void launch_piece_final(hipStream_t st, int64_t n, const Batch &bt, int want, const EvalOut &o, int nwalls,
                        const int32_t *perm, const float4 *pos_s, double *cen_out, PieceAcc acc);
void launch_validate(hipStream_t st, int64_t n, const Batch &bt, const float *x, const float *y, const float *z,
                     const double *psi, const double *nu, int32_t *bad_inst);
void launch_gather_sites(hipStream_t st, int64_t n, const float *x, const float *y, const float *z,
                         const double *psi, float4 *pos_orig);
// rmax[b] = max sqrt(max(psi, 0)) over the rows of every selected instance
void launch_rmax(hipStream_t st, const Batch &bt, int want, const double *psi, double *rmax);
// moved sites (lagot_solve_moved): p = float(p0 + t (p1 - p0)) per coordinate (exactly p1 at t = 1)
void launch_lerp_sites(hipStream_t st, int64_t n, const float *x0, const float *y0, const float *z0, const float *x1,
                       const float *y1, const float *z1, double t, float *x, float *y, float *z);
// weights carried with moved sites: psi_out = psi - 2 d.(c - pa) + |d|^2, d = pb - pa (caller order;
// cen [3n] site-major)
void launch_carry_weights(hipStream_t st, int64_t n, const float *xa, const float *ya, const float *za,
                          const float *xb, const float *yb, const float *zb, const double *cen, const double *psi,
                          double *psi_out);
// local reach of the selected instances from the float32 weights in pos_s.w: rmc[c] = the
// largest ball radius of the sites in coarse cell c, ir[c] = the largest rmc[c'] of the coarse
// cells c' within 2 rmc[c'] of c (work arrays of nc_total entries; ir as bt.ir)
void launch_local_reach(hipStream_t st, int64_t n, const Batch &bt, int want, int nc_total, const float4 *pos_s,
                        uint32_t *rmc, uint32_t *ir);
void launch_grid_build(hipStream_t st, int64_t n, const Batch &bt, int ncell_total, const float4 *pos_orig,
                       int32_t *keys, int32_t *cell_count, int32_t *cell_start, int32_t *scan_tmp, int32_t *perm,
                       int32_t *cursor);
void launch_permute_in(hipStream_t st, int64_t n, const int32_t *perm, const float4 *pos_orig, const double *psi,
                       const double *nu, float4 *pos_s, double *psi_s, double *nu_s);
void launch_psi_shadow(hipStream_t st, int64_t n, const double *psi_s, float4 *pos_s);
void launch_scatter_out_f64(hipStream_t st, int64_t n, const int32_t *perm, const double *src_s, double *dst);
void launch_scan_i32(hipStream_t st, const int32_t *in, int32_t *out, int n, int32_t *tmp);
// sorts data[start[c] .. start[c+1]) ascending for every c < nseg
void launch_sort_segments(hipStream_t st, int nseg, const int32_t *start, int32_t *data);
void launch_csr_count(hipStream_t st, int64_t n, const int32_t *perm, const int32_t *fcnt, int32_t *cnt_orig);
void launch_csr_fill(hipStream_t st, int64_t n, const int32_t *perm, const int32_t *fcol, const float *farea,
                     const int32_t *fcnt, const int32_t *start, int32_t *col, float *area, int64_t *row_ptr);
void launch_scatter_walls(hipStream_t st, int64_t n, int nw, const int32_t *perm, const float *wall_s, float *wall);
void launch_scatter_rows(hipStream_t st, int64_t n, int row_bytes, const int32_t *perm, const void *src, void *dst);
void launch_default_start(hipStream_t st, const Batch &bt, int want, const double *ev_nu, double *psi_s,
                          float4 *pos_s);
// psi_out = psi_s, except that empty cells (V <= 0) of the selected instances get
// max(psi, default weight, weights of the neighbours whose power region contains the ball)
// instances of phase `want` with more than 64, and more than 1%, of their cells empty
// (V <= 0) -> PH_RESTART,
// the phase histogram counts updated (nempty: [B] scratch)
void launch_repair_gate(hipStream_t st, const Batch &bt, int want, const double *V, int32_t *nempty, int32_t *phase,
                        int32_t *counts);
void launch_repair_empty(hipStream_t st, const Batch &bt, int want, const double *V, const double *nu_s,
                         const int32_t *cell_start, const double *psi_s, double *psi_out, float4 *pos_s);

// cells.hip
// Cells of the selected instances at the float64 weights psi (float32 shadow in pos_s.w).
void launch_eval_begin(hipStream_t st, const Batch &bt, int want, EvalOut out);
void launch_cells(hipStream_t st, int64_t n, const Batch &bt, int want, const float4 *pos_s, const double *psi,
                  const int32_t *perm, const int32_t *cell_start, EvalOut out, const QBoxes &qb, int tpc,
                  bool crowd);
// The passes after the fast one: the crowded cells it deferred (seed boxes, box grid,
// box-overlap candidates, float64), then the cells flagged for the float64 pass.
// crowd = false (no crowded cell expected): the fast pass writes no boxes and the float64
// pass takes the deferred cells too. Events e0, e1 (may be null) bracket the crowded pass.
// every cell on the float64 path with |K| by section 3.3's own route (lagot_cells_paper_k)
void launch_cells_kroute(hipStream_t st, int64_t n, const Batch &bt, const float4 *pos_s, const double *psi,
                         const int32_t *perm, const int32_t *cell_start, EvalOut out, const QBoxes &qb);
void launch_cells_fallback(hipStream_t st, int64_t n, const Batch &bt, int want, const float4 *pos_s,
                           const double *psi, const int32_t *perm, const int32_t *cell_start, EvalOut out,
                           const QBoxes &qb, bool crowd, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                           int32_t *start_gate = nullptr);

// newton.hip
// ev[4b..4b+3] = sum V, max |V - nu| / nu, ||nu - V||_2, min V of every selected instance
void launch_eval_reduce(hipStream_t st, const Batch &bt, int want, const double *V, const double *nu, double *part,
                        double *ev);
void launch_hess_assemble(hipStream_t st, int64_t n, const Batch &bt, int want, const float4 *pos_s,
                          const int32_t *fcol, const float *farea, const int32_t *fcnt, int32_t *hcol, float *hval,
                          int32_t *xcnt, int32_t *herr);
// Row lengths, sorted rows and the diagonal of -Hess K; with ent given (else null), the
// rows are also packed per tile: row i at ent[tile * TILE * FCAP + hrow[i].x], hrow[i].y
// entries of (column, float bits of the value)
void launch_hess_finish(hipStream_t st, const Batch &bt, int want, const double *psi_s, const double *K,
                        const int32_t *fcnt, const int32_t *xcnt, int32_t *hcnt, int32_t *hcol, float *hval,
                        double *diag, int2 *hrow, int2 *ent);
// CG block shape: `lanes` lanes per row (1, 2, 4 or 8), `sub` rows per block (64, 128
// or 256; 8 lanes with at most 128 rows)
bool cg_shape_ok(int lanes, int sub);
void launch_cg_init(hipStream_t st, const Batch &bt, int lanes, int sub, const double *V, const double *nu,
                    const double *diag, const int2 *hrow, const int2 *ent, CgBufs cg);
// one PCG iteration in two launches (own update, then the product on u_{k+1})
void launch_cg_split_iter(hipStream_t st, const Batch &bt, int lanes, int sub, int m, double rtol2, int cap,
                          const int2 *hrow, const int2 *ent, CgBufs cg);
void launch_cg_iter(hipStream_t st, const Batch &bt, int lanes, int sub, int m, double rtol2, int cap,
                    const int2 *hrow, const int2 *ent, CgBufs cg);
void launch_cg_advance(hipStream_t st, const Batch &bt, int chunk, int cap, CgBufs cg);
// The scalars of the next PCG iteration from the partials just written (after launch_cg_init:
// m = -1; after launch_cg_iter with m: the same m), one block per instance with more than
// cg_sum_in_block_max() partials (the others are summed inside the iteration's blocks)
void launch_cg_scalars(hipStream_t st, const Batch &bt, int sub, int m, int cap, CgBufs cg);
int cg_sum_in_block_max();
// step_start 1: the step search starts at min(1, 2 alpha_acc) instead of 1
void launch_cg_finish(hipStream_t st, const Batch &bt, int sub, double rtol2, int step_start, CgBufs cg,
                      const int32_t *herr, InstCtl *ctl, int32_t *phase);
void launch_ctl_init(hipStream_t st, const Batch &bt, InstCtl *ctl, int32_t *phase);
// ev: statistics of the first iterate; ev_floor: of the given start weights (eps0)
void launch_ctl_start(hipStream_t st, const Batch &bt, CtlOpts o, int from_phase, const double *ev,
                      const double *ev_nu, const double *ev_floor, const int32_t *fail_inst, InstCtl *ctl,
                      int32_t *phase, int32_t *counts);
void launch_axpy_trial(hipStream_t st, const Batch &bt, const InstCtl *ctl, const double *psi_s, const double *u,
                       double *psi_trial, float4 *pos_s);
void launch_ctl_decide(hipStream_t st, const Batch &bt, CtlOpts o, const double *ev, const int32_t *fail_inst,
                       InstCtl *ctl, int32_t *phase);
void launch_accept_rows(hipStream_t st, const Batch &bt, const InstCtl *ctl, double *psi_s, const double *psi_trial,
                        float4 *pos_s);
void launch_ctl_commit(hipStream_t st, const Batch &bt, CtlOpts o, InstCtl *ctl, int32_t *phase, int32_t *counts);
// Near convergence a full Newton step that fails to halve ||nu - V|| has reached the rounding
// of the float32 cells: the cells still off by more than tol/4 are marked (prec, sorted
// order), and the evaluations of the rest of the call finish them on the float64 path.
void launch_mark_precise(hipStream_t st, const Batch &bt, CtlOpts o, const InstCtl *ctl, const double *V,
                         const double *nu, uint8_t *prec);
void launch_add_precise(hipStream_t st, int64_t n, const Batch &bt, int want, const uint8_t *prec, EvalOut o);
// One instance's start evaluation: when the cell boxes after the seed pass show more empty
// cells than the repair gate allows (more than 64 and more than 1%), the crowded and float64
// passes are skipped.
void launch_start_gate(hipStream_t st, const Batch &bt, int want, const float4 *box, double *V, int32_t *nempty,
                       int32_t *fb_count, int32_t *ovf_count);
// Start of a continuation stage (every instance): the current iterate, with statistics
// ev against the stage's prescribed volumes (statistics ev_nu), becomes the stage's
// start: status cleared, eps0 = 0.5 min(min nu_s, min V), the iteration limit counted
// from here; DONE if it already meets o.tol.
void launch_ctl_stage(hipStream_t st, const Batch &bt, CtlOpts o, const double *ev, const double *ev_nu,
                      const int32_t *fail_inst, InstCtl *ctl, int32_t *phase, int32_t *counts);
// nu_s = (1 - s) v0 + s nu over n rows
void launch_nu_stage(hipStream_t st, int64_t n, double s, const double *v0, const double *nu, double *nu_s);

// fluid.hip
// Rows of the velocity system in grid order: rescales hval from w_ij to mu_ij w_ij,
// diag = m/dt + row sum, b[c*n + i] = right-hand side of coordinate c; bad counts
// invalid masses, viscosities and velocities.
void launch_fluid_rows(hipStream_t st, int64_t n, const int32_t *perm, const float4 *pos_s, const int32_t *hcol,
                       float *hval, const int32_t *hcnt, const double *mass, const double *mu, const FluidPrm &fp,
                       const double *v, const double *cen, double *diag, double *b, int32_t *bad);
// out = Lap_mu u (caller order, [3n]); mu == null: mu_ij = mu0
void launch_p1_laplacian(hipStream_t st, int64_t n, const int32_t *perm, const int32_t *hcol, const float *hval,
                         const int32_t *hcnt, const double *mu, double mu0, const double *u, double *out,
                         int32_t *bad);
int cg3_blocks(int64_t n);
// bad += entries with nu <= 0, mass <= 0, a non-finite velocity, or a viscosity < 0 (mu may be null)
void launch_fluid_check(hipStream_t st, int64_t n, const double *nu, const double *mass, const double *mu,
                        const double *v, int32_t *bad);
// packed rows: rp [n+1] (exclusive scan of hcnt), ent [rp[n]] = (column, float bits of the value)
void launch_pack_rows(hipStream_t st, int64_t n, const int32_t *hcol, const float *hval, const int32_t *hcnt,
                      const int32_t *rp, int2 *ent);
void launch_cg3_init(hipStream_t st, int64_t n, const int32_t *rp, const int2 *ent, const double *diag,
                     const double *b, const Cg3Bufs &g);
void launch_cg3_iter(hipStream_t st, int64_t n, int m, double rtol2, int cap, const int32_t *rp, const int2 *ent,
                     const Cg3Bufs &g);
void launch_cg3_advance(hipStream_t st, int chunk, int cap, const Cg3Bufs &g);
// the scalars of the next iteration from the partials just written (m = -1 after init)
void launch_cg3_scalars(hipStream_t st, int m, int cap, const Cg3Bufs &g);
// out[3 perm[i] + q] = x[3 i + q]
void launch_scatter3(hipStream_t st, int64_t n, const int32_t *perm, const double *x, double *out);
// x += dt v, clamped into the box and the domain planes (see k_advect)
void launch_advect(hipStream_t st, int64_t n, float *x, float *y, float *z, const double *v, double dt,
                   const AdvectBounds &bd, const float4 *dom, int ndom, const int32_t *dom_off, int npieces);

// mlp.hip
void launch_knn_features(hipStream_t st, int64_t n, const float4 *pos_s, const int32_t *perm,
                         const int32_t *cell_start, GridDesc g, const double *psi_prev_s, const double *nu_s,
                         const double *nu_sum, const double *V_s, int32_t *nbr, uint16_t *feat, int32_t *err);
void launch_gemm(hipStream_t st, bool ta, bool tb, int epi, const uint16_t *A, const uint16_t *B, int M, int N, int K,
                 float *C, uint16_t *Cb, const float *bias, const float *Zaux);
void launch_out_layer(hipStream_t st, int m, const uint16_t *H, const float *w4, const float *b4, float *y,
                      const float *t, float *dy, float *loss_part);
void launch_out_back(hipStream_t st, int m, const float *dy, const float *w4, const float *Z, float *dZ,
                     uint16_t *dZb);
void launch_colsum(hipStream_t st, int m, int ncol, const float *X, const uint16_t *Xb, const float *w, float *part,
                   int max_part_blocks, float *out);
void launch_adam(hipStream_t st, int64_t np, float *p, const float *g, float *m1, float *m2, float lr, float b1,
                 float b2, float eps, float c1, float c2, uint16_t *pb);
void launch_to_bf16(hipStream_t st, int64_t n, const float *x, uint16_t *y);
void launch_gather_rows(hipStream_t st, int m, const int32_t *idx, const uint16_t *F, const float *T, uint16_t *Fb,
                        float *Tb);
void launch_apply_guess(hipStream_t st, int64_t n, const double *psi_prev, const double *nu, const float *out, double beta,
                        double *psi_new, float4 *pos_s);
enum { MLP_EPI_STORE = 0, MLP_EPI_BIAS_GELU = 1, MLP_EPI_GELU_BACK = 2 };

}  // namespace lagot
