// api.cpp -- C-ABI of liblagot (declared in include/lagot.h): context and
// workspace management, input validation, the per-instance spatial sort, cell
// evaluations, and the host side of the damped Newton loop of Algorithm 1
// (KMT step control) around the Jacobi-PCG direction solve.
//
// Every solve is a batch of B >= 1 independent instances (lagot_solve is the
// case B = 1). Everything between the caller's arrays runs in grid order on the
// device; the decisions of Algorithm 1 (stop, accept, halve, fail) are taken per
// instance by device control kernels, and the host only reads a histogram of
// instance phases between the steps of a Newton iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "lagot.h"
#include "lagot_internal.h"

using namespace lagot;

// Device memory of lagot_mlp_forward_noalloc: the two hidden-activation buffers of at most
// LAGOT_NOALLOC_MAX_ROWS rows, one copy per GPU. Host code never passes this name to a
// kernel (on the host it is only a stand-in for the symbol); it uses the per-device address
// that hipGetSymbolAddress returns (noalloc_scratch_ptr).
static __device__ __align__(256) uint16_t scratch[2 * (size_t)LAGOT_NOALLOC_MAX_ROWS * MLP_HID];

namespace {

template <typename T> hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, sizeof(T) * (count ? count : 1));
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct lagot_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t cap_n = 0;
    int cap_cells = 0;
    int cap_B = 0, cap_T = 0;
    int tpc = 32;
    int tpc_default = 32;  // lanes per cell when the options leave it to the library
    struct Tuned {
        int tpc = 32, cg_lanes = 4, cg_sub = 64;
        bool cg = false;  // the CG shape has been timed too
    };
    std::map<int, Tuned> tuned;    // autotuner: size/density class -> shapes
    int tune_key = -1;             // class whose CG shape the next direction solve times
    int cg_chunk = 16;             // PCG launches between host checks (adapted per solve)
    int cg_lanes = 4, cg_sub = 64; // PCG block shape of the current call: lanes per row, rows per block
    int cg_lanes_def = 4, cg_sub_def = 64;  // ... when the options do not ask for the autotuner

    // the current call: B instances, T tiles, n rows
    int B = 0, T = 0;
    int64_t n = 0;
    int max_inst_tiles = 0;  // tiles of the largest instance of the call
    int ncell_total = 0;
    std::vector<GridDesc> h_grid;

    // sites (caller order, then grid order)
    float4 *pos_orig = nullptr, *pos_s = nullptr;
    double *psi_s = nullptr, *nu_s = nullptr, *psi_trial = nullptr;
    int32_t *keys = nullptr, *perm = nullptr, *inst = nullptr;
    int32_t *cell_count = nullptr, *cell_start = nullptr, *cursor = nullptr, *scan_tmp = nullptr;
    // instances and tiles
    int32_t *off = nullptr, *tile_inst = nullptr, *tile_row = nullptr, *first_tile = nullptr;
    GridDesc *grid = nullptr;
    BoxF *box = nullptr;
    double *rmax = nullptr;
    int32_t *phase = nullptr;
    InstCtl *ctl = nullptr;
    double *ev = nullptr, *ev2 = nullptr, *ev_nu = nullptr, *part_ev = nullptr;
    int32_t *fb_inst = nullptr, *fail_inst = nullptr, *bad_inst = nullptr, *herr = nullptr, *counts = nullptr;
    int32_t *nempty = nullptr;  // [cap_B] empty start cells per instance
    int32_t *misc = nullptr;  // [0] float64 work-list length [1] feature errors [2] kbase [3] remaining
                              // [4] overflow work-list length [5] large cell boxes
    // cell boxes and the box grid of the crowded-cell pass
    float4 *qbox = nullptr;                 // [2n]
    int32_t *qent = nullptr, *qlarge = nullptr;  // [QREG_MAX n], [n]
    int32_t *qcount = nullptr, *qstart = nullptr, *qcursor = nullptr, *qtmp = nullptr;  // bucket arrays
    int32_t *qdstart = nullptr;             // [n + 1] scan of the deferred-cell marks
    int64_t cap_qtmp_n = 0;                 // rows the scan workspace qtmp serves
    GridDesc *qgrid = nullptr;              // [B]
    int nq = 0, cap_nq = 0;
    // crowded pass on for this call: some site grid was capped by the spacing (a few large
    // balls), or an evaluation of this call or of the last one deferred cells
    bool crowd = false, crowd_seen = false;
    // local reach (crowded calls): coarse grids, largest radius per coarse cell, spread bound
    GridDesc *cgrid = nullptr;              // [B]
    uint32_t *lr_rmc = nullptr, *lr_ir = nullptr;
    int nc = 0, cap_nc = 0;
    bool eval_crowd = false;  // the crowded pass ran in the last evaluation
    // evaluation outputs (grid order)
    double *V = nullptr, *K = nullptr;
    float *wall = nullptr;
    int32_t *fcol = nullptr, *fcnt = nullptr, *fb_list = nullptr, *ovf_list = nullptr;
    double *cen_out = nullptr;  // caller's centroid array during a lagot_centroids call
    double *cont_buf = nullptr; // continuation: start volumes, prescribed volumes, last accepted weights [3n]
    int64_t cap_cont = 0;
    double *mv_buf = nullptr;   // lagot_solve_moved: centroids [3n], volumes [n], accepted / trial weights [2n]
    float *mv_pos = nullptr;    // ... positions of the accepted part and of the trial part [6n]
    int64_t cap_mv = 0;
    double *fl_buf = nullptr;   // fluid step: PCG records and vectors, right-hand sides, centroids
    int32_t *fl_int = nullptr;  // fluid step: PCG status per coordinate, chunk counters
    int2 *fl_ent = nullptr;     // fluid step: matrix rows packed back to back
    int64_t cap_ent = 0;
    int64_t cap_fl = 0;
    int fl_chunk = 32;          // fluid PCG launches between host checks (adapted per call)
    bool fl_reuse = false;      // lagot_fluid_step's velocity update: reuse its solve's sorted sites
    float4 *dom_d = nullptr;    // [PIECE_PLANES_MAX] domain planes (lagot_set_domain, lagot_set_domain_pieces)
    int ndom = 0;
    // a non-convex domain as a union of convex pieces (lagot_set_domain_pieces; 0: convex)
    int npieces = 0, nwalls = 0;
    uint8_t *prec = nullptr;    // [n + 4] cells a solve finishes on the float64 path (sorted order)
    bool prec_on = false;       // set while a solve runs
    bool start_gate = false;    // set for a one-instance start evaluation (hopeless starts skip the slow passes)
    int32_t h_dom_off[PIECE_MAX + 1] = {0};
    int32_t *dom_off_d = nullptr, *dom_wid_d = nullptr;  // [PIECE_MAX + 1], [PIECE_PLANES_MAX]
    // per-piece accumulators of an evaluation (allocated with the sites when pieces are set)
    double *pa_V = nullptr, *pa_K = nullptr, *pa_mom = nullptr, *pa_cen = nullptr;
    int32_t *pa_fcol = nullptr, *pa_fcnt = nullptr;
    float *pa_farea = nullptr, *pa_wall = nullptr;
    uint32_t *pa_flags = nullptr;
    int64_t cap_piece = 0;
    int cap_piece_w = 0;
    int wall_w = 6;             // wall areas per site in the wall buffer (6, or the domain's planes)
    float *farea = nullptr;
    uint32_t *flags = nullptr;
    // second set of evaluation outputs (learned guess: evaluated aside, swapped in if kept)
    double *V2 = nullptr, *K2 = nullptr;
    int32_t *fcol2 = nullptr, *fcnt2 = nullptr;
    float *farea2 = nullptr;
    uint32_t *flags2 = nullptr;
    int64_t cap_alt = 0;
    // Hessian and PCG
    int32_t *hcol = nullptr, *hcnt = nullptr, *xcnt = nullptr;
    float *hval = nullptr;
    double *diag = nullptr;
    int2 *hrow = nullptr;       // packed Hessian rows: (start within the tile's region, length)
    int2 *hent = nullptr;       // [cap_hent_T * TILE * FCAP] packed entries, one region per tile
    int cap_hent_T = 0;
    double *cg_vec = nullptr;   // rws[2] (4 doubles per row each), p, x, u: 11 doubles per row
    int cg_split = 0;           // PCG iteration: 0 two launches for large instances, 1 always one, 2 always two
    double *cg_part = nullptr;  // 7 * 4 * cap_T
    double *cg_cgs = nullptr;   // 4 * cap_B
    double *cg_sc = nullptr;    // 8 * cap_B
    int32_t *cg_cgst = nullptr; // 4 * cap_B
    // pinned host staging (uploads) and read-back
    char *h_stage = nullptr;
    size_t cap_stage = 0;
    char *h_rd = nullptr;
    size_t cap_rd = 0;
    int32_t *h_cnt = nullptr;  // [16]
    // CSR staging for lagot_cells
    int32_t *csr_cnt = nullptr, *csr_start = nullptr;
    int32_t *csr_tmp = nullptr;
    // statistics of the current call
    int last_fb = 0;
    // learned warm start: float32 master parameters, bf16 copy, Adam moments
    float *mlp_p = nullptr, *mlp_g = nullptr, *mlp_m1 = nullptr, *mlp_m2 = nullptr;
    uint16_t *mlp_pb = nullptr;
    int mlp_t = 0;
    bool mlp_set = false;
    int32_t *nbr_s = nullptr;        // [n*16] grid order (caller indices)
    uint16_t *feat_s = nullptr;      // [n*64] bf16 inputs, grid order
    uint16_t *inf_a = nullptr, *inf_b = nullptr;  // [n*128] bf16 hidden activations
    float *mlp_out = nullptr;        // [n]
    int64_t cap_inf = 0;
    // training workspace (batch rows)
    int cap_batch = 0;
    uint16_t *tX = nullptr, *tH1 = nullptr, *tH2 = nullptr, *tH3 = nullptr, *tdZb = nullptr;
    float *tZ1 = nullptr, *tZ2 = nullptr, *tZ3 = nullptr, *tdZ = nullptr, *ty = nullptr, *tt = nullptr,
          *tdy = nullptr, *tpart = nullptr, *tloss = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around the float32 cell kernel
    hipEvent_t evc0 = nullptr, evc1 = nullptr;  // around the crowded pass
    // graph mode: a private stream (default priority) and the graphs of the current call
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr;
    hipGraphExec_t g_dir = nullptr, g_trial = nullptr;
    std::map<int, hipGraphExec_t> g_cg;  // by chunk length
    bool graph_events = true;            // event records can be captured (timing inside graphs)
    bool capturing = false;
    bool ev_pending = false;
    double ms_cell = 0.0;
    int cell_launches = 0;
    bool ev_crowd_pending = false;
    double ms_crowd = 0.0;      // summed duration of the crowded pass in the current call
    int crowd_launches = 0;
    int64_t crowd_cells = 0;    // cells the timed crowded-pass launches processed
    uint16_t *noalloc = nullptr;  // this device's copy of the static scratch array
};

namespace {

#define HIP_TRY(expr)                                       \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) {                             \
            fprintf(stderr, "lagot: %s failed: %s\n", #expr, hipGetErrorString(e_)); \
            return LAGOT_EHIP;                              \
        }                                                   \
    } while (0)

template <typename... P> void free_ptrs(P *&...ps) {
    ((ps ? (void)hipFree((void *)ps) : (void)0), ...);
    ((ps = nullptr), ...);
}

void free_sites(lagot_ctx *c) {
    free_ptrs(c->pos_orig, c->pos_s, c->psi_s, c->nu_s, c->psi_trial, c->keys, c->perm, c->inst, c->V, c->K, c->wall,
              c->fcol, c->fcnt, c->fb_list, c->ovf_list, c->farea, c->flags, c->hcol, c->hcnt, c->xcnt, c->hval, c->diag,
              c->cg_vec, c->csr_cnt, c->csr_start, c->csr_tmp, c->hrow, c->qbox, c->qent, c->qlarge, c->qdstart);
    free_ptrs(c->prec);
    c->cap_n = 0;
}

void free_pieces(lagot_ctx *c) {
    free_ptrs(c->pa_V, c->pa_K, c->pa_mom, c->pa_cen, c->pa_fcol, c->pa_fcnt, c->pa_farea, c->pa_wall, c->pa_flags);
    c->cap_piece = 0;
    c->cap_piece_w = 0;
}

void free_inst(lagot_ctx *c) {
    free_ptrs(c->off, c->tile_inst, c->tile_row, c->first_tile, c->grid, c->box, c->rmax, c->phase, c->ctl, c->ev,
              c->ev2, c->ev_nu, c->part_ev, c->fb_inst, c->fail_inst, c->bad_inst, c->herr, c->cg_part, c->cg_cgs,
              c->cg_cgst, c->qgrid, c->cg_sc, c->cgrid, c->nempty);
}

void free_alt(lagot_ctx *c) {
    free_ptrs(c->V2, c->K2, c->fcol2, c->fcnt2, c->farea2, c->flags2);
    c->cap_alt = 0;
}

// The second output set is either not allocated (cap_alt = 0) or exactly as large as
// the first (cap_alt = cap_n): the two sets are swapped by pointer, so after a kept
// learned guess either one may serve as the primary set, and both must hold cap_n rows.
// ensure_sites frees both sets whenever it grows the first.
int ensure_alt(lagot_ctx *c) {
    if (c->cap_alt == c->cap_n) return LAGOT_OK;
    free_alt(c);
    const size_t N = (size_t)c->cap_n;
    HIP_TRY(dalloc(&c->V2, N));
    HIP_TRY(dalloc(&c->K2, N));
    HIP_TRY(dalloc(&c->fcol2, FCAP * N));
    HIP_TRY(dalloc(&c->farea2, FCAP * N));
    HIP_TRY(dalloc(&c->fcnt2, N));
    HIP_TRY(dalloc(&c->flags2, N));
    c->cap_alt = c->cap_n;
    return LAGOT_OK;
}

void swap_alt(lagot_ctx *c) {
    std::swap(c->V, c->V2);
    std::swap(c->K, c->K2);
    std::swap(c->fcol, c->fcol2);
    std::swap(c->farea, c->farea2);
    std::swap(c->fcnt, c->fcnt2);
    std::swap(c->flags, c->flags2);
}

void free_all(lagot_ctx *c) {
    free_alt(c);
    free_sites(c);
    free_inst(c);
    c->cap_qtmp_n = 0;
    free_pieces(c);
    free_ptrs(c->dom_off_d, c->dom_wid_d);
    free_ptrs(c->cell_count, c->cell_start, c->cursor, c->scan_tmp, c->counts, c->misc, c->dom_d, c->fl_buf, c->fl_int, c->fl_ent,
              c->hent, c->qcount, c->qstart, c->qcursor, c->qtmp, c->cont_buf, c->lr_rmc, c->lr_ir, c->mv_buf,
              c->mv_pos);
    c->cap_mv = 0;
    c->cap_cont = 0;
    c->cap_nc = 0;
    c->cap_nq = 0;
    c->cap_ent = 0;
    c->cap_hent_T = 0;
    c->cap_fl = 0;
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    if (c->h_rd) (void)hipHostFree(c->h_rd);
    if (c->h_cnt) (void)hipHostFree(c->h_cnt);
    free_ptrs(c->mlp_p, c->mlp_g, c->mlp_m1, c->mlp_m2, c->mlp_pb, c->nbr_s, c->feat_s, c->inf_a, c->inf_b,
              c->mlp_out, c->tX, c->tH1, c->tH2, c->tH3, c->tdZb, c->tZ1, c->tZ2, c->tZ3, c->tdZ, c->ty, c->tt,
              c->tdy, c->tpart, c->tloss);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->evc0) (void)hipEventDestroy(c->evc0);
    if (c->evc1) (void)hipEventDestroy(c->evc1);
}

// Add the duration of the last recorded cell-kernel launch (call after a stream sync).
void collect_cell_time(lagot_ctx *c) {
    if (!c->ev_pending) return;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) {
        c->ms_cell += ms;
        c->cell_launches++;
    }
    if (c->ev_crowd_pending && hipEventElapsedTime(&ms, c->evc0, c->evc1) == hipSuccess) {
        int32_t cnt = 0;
        if (hipMemcpy(&cnt, c->misc + 4, sizeof(cnt), hipMemcpyDeviceToHost) == hipSuccess) {
            c->ms_crowd += ms;
            c->crowd_launches++;
            c->crowd_cells += cnt;
        }
    }
    c->ev_crowd_pending = false;
    c->ev_pending = false;
    c->ev_crowd_pending = false;
}

int ensure_sites(lagot_ctx *c, int64_t n) {
    if (n <= c->cap_n) return LAGOT_OK;
    free_alt(c);  // either set may be the primary one (see ensure_alt): both go
    free_sites(c);
    const size_t N = (size_t)n;
    HIP_TRY(dalloc(&c->pos_orig, N));
    HIP_TRY(dalloc(&c->pos_s, N));
    HIP_TRY(dalloc(&c->psi_s, N));
    HIP_TRY(dalloc(&c->nu_s, N));
    HIP_TRY(dalloc(&c->psi_trial, N));
    HIP_TRY(dalloc(&c->keys, N));
    HIP_TRY(dalloc(&c->perm, N));
    HIP_TRY(dalloc(&c->inst, N));
    HIP_TRY(dalloc(&c->V, N));
    HIP_TRY(dalloc(&c->K, N));
    HIP_TRY(dalloc(&c->wall, (size_t)c->wall_w * N));
    HIP_TRY(dalloc(&c->fcol, FCAP * N));
    HIP_TRY(dalloc(&c->farea, FCAP * N));
    HIP_TRY(dalloc(&c->fcnt, N));
    HIP_TRY(dalloc(&c->fb_list, N));
    HIP_TRY(dalloc(&c->ovf_list, N));
    HIP_TRY(dalloc(&c->flags, N));
    HIP_TRY(dalloc(&c->hcol, FCAP * N));
    HIP_TRY(dalloc(&c->hval, FCAP * N));
    HIP_TRY(dalloc(&c->hcnt, N));
    HIP_TRY(dalloc(&c->xcnt, N));
    HIP_TRY(dalloc(&c->diag, N));
    HIP_TRY(dalloc(&c->hrow, N));
    HIP_TRY(dalloc(&c->qbox, 2 * N));
    HIP_TRY(dalloc(&c->qent, (size_t)QREG_MAX * N));
    HIP_TRY(dalloc(&c->qlarge, N));
    HIP_TRY(dalloc(&c->qdstart, N + 1));
    HIP_TRY(dalloc(&c->cg_vec, 11 * N));
    HIP_TRY(dalloc(&c->csr_cnt, N + 1));
    HIP_TRY(dalloc(&c->csr_start, N + 1));
    HIP_TRY(dalloc(&c->csr_tmp, N / 1024 + 16));
    HIP_TRY(dalloc(&c->prec, N + 4));
    c->cap_n = n;
    return LAGOT_OK;
}

// accumulators of the per-piece evaluations of a non-convex domain
int ensure_pieces(lagot_ctx *c, int64_t n) {
    if (c->npieces == 0 || (n <= c->cap_piece && c->nwalls <= c->cap_piece_w)) return LAGOT_OK;
    free_pieces(c);
    const size_t N = (size_t)std::max(n, c->cap_n);
    const int w = std::max(c->nwalls, 1);
    HIP_TRY(dalloc(&c->pa_V, N));
    HIP_TRY(dalloc(&c->pa_K, N));
    HIP_TRY(dalloc(&c->pa_mom, 3 * N));
    HIP_TRY(dalloc(&c->pa_cen, 3 * N));
    HIP_TRY(dalloc(&c->pa_fcol, FCAP * N));
    HIP_TRY(dalloc(&c->pa_farea, FCAP * N));
    HIP_TRY(dalloc(&c->pa_fcnt, N));
    HIP_TRY(dalloc(&c->pa_flags, N));
    HIP_TRY(dalloc(&c->pa_wall, (size_t)w * N));
    c->cap_piece = (int64_t)N;
    c->cap_piece_w = w;
    return LAGOT_OK;
}

int ensure_inst(lagot_ctx *c, int B, int T) {
    if (B <= c->cap_B && T <= c->cap_T) return LAGOT_OK;
    free_inst(c);
    B = std::max(B, c->cap_B);
    T = std::max(T, c->cap_T);
    c->cap_B = c->cap_T = 0;
    const size_t b = (size_t)B, t = (size_t)T;
    HIP_TRY(dalloc(&c->off, b + 1));
    HIP_TRY(dalloc(&c->tile_inst, t));
    HIP_TRY(dalloc(&c->tile_row, t));
    HIP_TRY(dalloc(&c->first_tile, b + 1));
    HIP_TRY(dalloc(&c->grid, b));
    HIP_TRY(dalloc(&c->box, b));
    HIP_TRY(dalloc(&c->rmax, b));
    HIP_TRY(dalloc(&c->phase, b));
    HIP_TRY(dalloc(&c->ctl, b));
    HIP_TRY(dalloc(&c->ev, 4 * b));
    HIP_TRY(dalloc(&c->ev2, 4 * b));
    HIP_TRY(dalloc(&c->ev_nu, 4 * b));
    HIP_TRY(dalloc(&c->part_ev, 4 * t));
    HIP_TRY(dalloc(&c->fb_inst, b));
    HIP_TRY(dalloc(&c->fail_inst, b));
    HIP_TRY(dalloc(&c->bad_inst, b));
    HIP_TRY(dalloc(&c->herr, b));
    HIP_TRY(dalloc(&c->cg_part, 7 * 4 * t));  // per quarter tile
    HIP_TRY(dalloc(&c->cg_cgs, 4 * b));
    HIP_TRY(dalloc(&c->cg_sc, 8 * b));
    HIP_TRY(dalloc(&c->cg_cgst, 4 * b));
    HIP_TRY(dalloc(&c->qgrid, (size_t)QLEV * b));
    HIP_TRY(dalloc(&c->cgrid, b));
    HIP_TRY(dalloc(&c->nempty, b));
    c->cap_B = B;
    c->cap_T = T;
    return LAGOT_OK;
}

int ensure_cells(lagot_ctx *c, int ncell) {
    if (ncell <= c->cap_cells) return LAGOT_OK;
    free_ptrs(c->cell_count, c->cell_start, c->cursor, c->scan_tmp);
    c->cap_cells = 0;
    HIP_TRY(dalloc(&c->cell_count, (size_t)ncell + 1));
    HIP_TRY(dalloc(&c->cell_start, (size_t)ncell + 1));
    HIP_TRY(dalloc(&c->cursor, (size_t)ncell + 1));
    HIP_TRY(dalloc(&c->scan_tmp, (size_t)ncell / 1024 + 16));
    c->cap_cells = ncell;
    return LAGOT_OK;
}

int ensure_coarse(lagot_ctx *c, int nc) {
    if (nc <= c->cap_nc) return LAGOT_OK;
    free_ptrs(c->lr_rmc, c->lr_ir);
    c->cap_nc = 0;
    HIP_TRY(dalloc(&c->lr_rmc, (size_t)nc));
    HIP_TRY(dalloc(&c->lr_ir, (size_t)nc));
    c->cap_nc = nc;
    return LAGOT_OK;
}

int ensure_buckets(lagot_ctx *c, int nq) {
    if (nq <= c->cap_nq && c->cap_n <= c->cap_qtmp_n) return LAGOT_OK;
    nq = std::max(nq, c->cap_nq);
    free_ptrs(c->qcount, c->qstart, c->qcursor, c->qtmp);
    c->cap_nq = 0;
    HIP_TRY(dalloc(&c->qcount, (size_t)nq + 1));
    HIP_TRY(dalloc(&c->qstart, (size_t)nq + 1));
    HIP_TRY(dalloc(&c->qcursor, (size_t)nq + 1));
    HIP_TRY(dalloc(&c->qtmp, (size_t)std::max<int64_t>(nq, c->cap_n) / 1024 + 16));
    c->cap_nq = nq;
    c->cap_qtmp_n = c->cap_n;
    return LAGOT_OK;
}

int ensure_pinned(char **p, size_t *cap, size_t bytes) {
    if (bytes <= *cap) return LAGOT_OK;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    bytes = std::max<size_t>(bytes, 4096);
    HIP_TRY(hipHostMalloc((void **)p, bytes));
    *cap = bytes;
    return LAGOT_OK;
}

bool box_ok(const lagot_box &b) {
    for (int a = 0; a < 3; ++a)
        if (!(b.hi[a] > b.lo[a]) || !std::isfinite(b.lo[a]) || !std::isfinite(b.hi[a])) return false;
    return true;
}

double box_volume(const lagot_box &b) {
    return (b.hi[0] - b.lo[0]) * (b.hi[1] - b.lo[1]) * (b.hi[2] - b.lo[2]);
}

int sync(lagot_ctx *c) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    collect_cell_time(c);
    return LAGOT_OK;
}

Batch batch(const lagot_ctx *c) {
    Batch b;
    b.B = c->B;
    b.T = c->T;
    b.off = c->off;
    b.tile_inst = c->tile_inst;
    b.tile_row = c->tile_row;
    b.first_tile = c->first_tile;
    b.inst = c->inst;
    b.grid = c->grid;
    b.box = c->box;
    b.rmax = c->rmax;
    b.phase = c->phase;
    b.dom = c->dom_d;
    b.ndom = c->ndom;
    b.npieces = c->npieces;
    b.dom_off = c->dom_off_d;
    b.dom_wid = c->dom_wid_d;
    b.cgrid = c->cgrid;
    b.ir = c->crowd ? reinterpret_cast<const float *>(c->lr_ir) : nullptr;
    return b;
}

CgBufs cg_bufs(const lagot_ctx *c) {
    CgBufs g;
    const size_t N = (size_t)c->cap_n;
    for (int q = 0; q < 2; ++q) g.rws[q] = reinterpret_cast<RWSD *>(c->cg_vec + 4 * q * N);
    g.p = c->cg_vec + 8 * N;
    g.x = c->cg_vec + 9 * N;
    g.u = c->cg_vec + 10 * N;
    g.part = c->cg_part;
    g.cgs = c->cg_cgs;
    g.sc = c->cg_sc;
    g.cgst = c->cg_cgst;
    g.kbase = c->misc + 2;
    g.remaining = c->misc + 3;
    g.maxit = c->misc + 7;
    return g;
}

// Validate the instances and sort each one spatially. On return the grid-order
// arrays pos_s (with float32 psi), psi_s (and nu_s) are filled, rmax[b] holds
// max sqrt(psi) of each instance, ev_nu[4b+0] = sum nu and ev_nu[4b+3] = min nu
// (when nu is given). bad (host, B entries, may be null) flags invalid instances.
int prepare(lagot_ctx *c, int B, const int64_t *offs, const float *x, const float *y, const float *z,
            const double *psi, const double *nu, const lagot_box *boxes, std::vector<int> *bad) {
    if (B <= 0 || !offs || !boxes || !x || !y || !z || !psi) return LAGOT_EINVAL;
    if (offs[0] != 0) return LAGOT_EINVAL;
    for (int b = 0; b < B; ++b)
        if (!(offs[b + 1] > offs[b]) || !box_ok(boxes[b])) return LAGOT_EINVAL;
    const int64_t n = offs[B];
    if (n > (int64_t)INT32_MAX / FCAP) return LAGOT_EINVAL;
    int64_t T64 = 0;
    for (int b = 0; b < B; ++b) T64 += (offs[b + 1] - offs[b] + TILE - 1) / TILE;
    const int T = (int)T64;
    int rc = ensure_sites(c, n);
    if (!rc) rc = ensure_pieces(c, n);
    if (!rc) rc = ensure_inst(c, B, T);
    if (rc) return rc;
    c->B = B;
    c->T = T;
    c->n = n;
    // tile table, boxes and (below) grids, staged in pinned memory
    const size_t stage = sizeof(int32_t) * (2 * (size_t)(B + 1) + 2 * (size_t)T) + sizeof(BoxF) * B +
                         (2 + QLEV) * sizeof(GridDesc) * B + 64;
    rc = ensure_pinned(&c->h_stage, &c->cap_stage, stage);
    if (rc) return rc;
    int32_t *h_off = (int32_t *)c->h_stage;
    int32_t *h_first = h_off + (B + 1);
    int32_t *h_tinst = h_first + (B + 1);
    int32_t *h_trow = h_tinst + T;
    BoxF *h_box = (BoxF *)(h_trow + T);
    GridDesc *h_g = (GridDesc *)(h_box + B);
    int t = 0;
    c->max_inst_tiles = 0;
    for (int b = 0; b < B; ++b) {
        h_off[b] = (int32_t)offs[b];
        h_first[b] = t;
        c->max_inst_tiles = std::max(c->max_inst_tiles, (int)((offs[b + 1] - offs[b] + TILE - 1) / TILE));
        for (int64_t r = offs[b]; r < offs[b + 1]; r += TILE) {
            h_tinst[t] = b;
            h_trow[t] = (int32_t)r;
            ++t;
        }
        for (int a = 0; a < 3; ++a) {
            h_box[b].lo[a] = (float)boxes[b].lo[a];
            h_box[b].hi[a] = (float)boxes[b].hi[a];
        }
    }
    h_off[B] = (int32_t)n;
    h_first[B] = T;
    hipStream_t st = c->stream;
    HIP_TRY(hipMemcpyAsync(c->off, h_off, sizeof(int32_t) * (B + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->first_tile, h_first, sizeof(int32_t) * (B + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->tile_inst, h_tinst, sizeof(int32_t) * T, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->tile_row, h_trow, sizeof(int32_t) * T, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->box, h_box, sizeof(BoxF) * B, hipMemcpyHostToDevice, st));
    const Batch bt = batch(c);
    launch_fill_inst(st, bt, c->inst);
    launch_zero_i32(st, c->bad_inst, B);
    launch_validate(st, n, bt, x, y, z, psi, nu, c->bad_inst);
    launch_gather_sites(st, n, x, y, z, psi, c->pos_orig);
    launch_rmax(st, bt, -1, psi, c->rmax);
    if (nu) launch_eval_reduce(st, bt, -1, nu, nu, c->part_ev, c->ev_nu);
    // read back: bad counts, r_max, nu statistics
    const size_t ibytes = ((sizeof(int32_t) * B + 63) / 64) * 64;
    rc = ensure_pinned(&c->h_rd, &c->cap_rd, ibytes + sizeof(double) * 5 * B + 64);
    if (rc) return rc;
    int32_t *r_bad = (int32_t *)c->h_rd;
    double *r_rmax = (double *)(c->h_rd + ibytes);
    double *r_nu = r_rmax + B;
    HIP_TRY(hipMemcpyAsync(r_bad, c->bad_inst, sizeof(int32_t) * B, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(r_rmax, c->rmax, sizeof(double) * B, hipMemcpyDeviceToHost, st));
    if (nu) HIP_TRY(hipMemcpyAsync(r_nu, c->ev_nu, sizeof(double) * 4 * B, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    bool any_bad = false;
    for (int b = 0; b < B; ++b) {
        // every site strictly inside its box, no NaN, nu > 0, and room for air: sum nu < |box|
        bool ok = r_bad[b] == 0 && std::isfinite(r_rmax[b]);
        if (nu) ok = ok && r_nu[4 * b] < box_volume(boxes[b]);
        if (bad) (*bad)[b] = !ok;
        any_bad = any_bad || !ok;
    }
    if (any_bad) return LAGOT_EINVAL;
    // One grid of sites per instance: cell size 2 r_max (the 3x3x3 neighbourhood then
    // covers every bisector that can cut a ball), but no coarser than 1.5 times the mean
    // spacing of the instance's sites in its box: where a few balls are much larger than
    // the rest (crowded scenes), a grid sized by them would put thousands of sites in
    // every cell. At most 512 cells per axis and 2^24 cells. The typical site spacing h
    // (cube root of the mean prescribed volume, else of the box volume per site) sets the
    // seed radius of crowded cells and the box grids: QLEV levels of buckets 1.2 h 4^l,
    // at most 1024 buckets per axis and 2^24 per level.
    c->h_grid.resize(B);
    std::vector<GridDesc> qg((size_t)B * QLEV), cgv(B);
    int64_t total = 0, qtotal = 0, ctotal = 0;
    bool capped = false;
    auto make_grid = [](const lagot_box &bx, double s, int maxdim, int64_t base, GridDesc *g) {
        int dim[3];
        for (;;) {
            int64_t tot = 1;
            bool ok = true;
            for (int a = 0; a < 3; ++a) {
                dim[a] = std::max(1, (int)std::ceil((bx.hi[a] - bx.lo[a]) / s));
                ok = ok && dim[a] <= maxdim;
                tot *= dim[a];
            }
            if (ok && tot <= (1 << 24)) break;
            s *= 1.25;
        }
        for (int a = 0; a < 3; ++a) {
            g->lo[a] = (float)bx.lo[a];
            g->dim[a] = dim[a];
        }
        g->s = (float)s;
        g->inv_s = (float)(1.0 / s);
        g->ncell = dim[0] * dim[1] * dim[2];
        g->base = (int)base;
        g->hsp = 0.f;
        g->pad = 0;
    };
    for (int b = 0; b < B; ++b) {
        const lagot_box &bx = boxes[b];
        double ext = 0.0;
        for (int a = 0; a < 3; ++a) ext = std::max(ext, bx.hi[a] - bx.lo[a]);
        const double nb = (double)(offs[b + 1] - offs[b]);
        const double hsp = std::cbrt((nu ? r_nu[4 * b] : box_volume(bx)) / nb);
        double s = std::min(2.0 * r_rmax[b], 1.5 * std::cbrt(box_volume(bx) / nb));
        s = std::max(s, ext / 512.0);
        capped = capped || s < 2.0 * r_rmax[b];
        GridDesc g;
        make_grid(bx, s, 512, total, &g);
        g.hsp = (float)hsp;
        total += g.ncell;
        if (total > ((int64_t)1 << 28)) return LAGOT_ECAPACITY;
        c->h_grid[b] = g;
        make_grid(bx, 4.0 * (double)g.s, 256, ctotal, &cgv[b]);  // coarse grid of the local reach
        ctotal += cgv[b].ncell;
        double sq = std::max(1.2 * hsp, ext / 1024.0);
        for (int l = 0; l < QLEV; ++l, sq *= 4.0) {
            GridDesc &q = qg[(size_t)b * QLEV + l];
            make_grid(bx, sq, 1024, qtotal, &q);
            q.hsp = (float)hsp;
            qtotal += q.ncell;
        }
        if (qtotal > ((int64_t)1 << 28)) return LAGOT_ECAPACITY;
    }
    c->ncell_total = (int)total;
    c->nq = (int)qtotal;
    c->nc = (int)ctotal;
    c->crowd = c->crowd_seen || capped;
    c->crowd_seen = false;
    rc = ensure_cells(c, c->ncell_total);
    if (!rc) rc = ensure_buckets(c, c->nq);
    if (!rc) rc = ensure_coarse(c, c->nc);
    if (rc) return rc;
    std::memcpy(h_g, c->h_grid.data(), sizeof(GridDesc) * B);
    std::memcpy(h_g + B, qg.data(), sizeof(GridDesc) * B * QLEV);
    HIP_TRY(hipMemcpyAsync(c->grid, h_g, sizeof(GridDesc) * B, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->qgrid, h_g + B, sizeof(GridDesc) * B * QLEV, hipMemcpyHostToDevice, st));
    std::memcpy(h_g + B + (size_t)B * QLEV, cgv.data(), sizeof(GridDesc) * B);
    HIP_TRY(hipMemcpyAsync(c->cgrid, h_g + B + (size_t)B * QLEV, sizeof(GridDesc) * B, hipMemcpyHostToDevice, st));
    launch_grid_build(st, n, bt, c->ncell_total, c->pos_orig, c->keys, c->cell_count, c->cell_start, c->scan_tmp,
                      c->perm, c->cursor);
    launch_permute_in(st, n, c->perm, c->pos_orig, psi, nu, c->pos_s, c->psi_s, nu ? c->nu_s : nullptr);
    return LAGOT_OK;
}

QBoxes qboxes(lagot_ctx *c) {
    QBoxes q;
    q.box = c->qbox;
    q.qgrid = c->qgrid;
    q.count = c->qcount;
    q.start = c->qstart;
    q.cursor = c->qcursor;
    q.ent = c->qent;
    q.large = c->qlarge;
    q.nlarge = c->misc + 5;
    q.tmp = c->qtmp;
    q.dcnt = c->csr_cnt;
    q.dstart = c->qdstart;
    q.nq = c->nq;
    return q;
}

EvalOut eval_out(lagot_ctx *c, bool walls) {
    EvalOut o{c->V, c->K, walls ? c->wall : nullptr, c->fcol, c->farea, c->fcnt, c->flags, c->fb_list, c->misc + 0,
              c->fb_inst, c->fail_inst, c->ovf_list, c->misc + 4, c->cen_out};
    return o;
}

// Cells of the instances in phase `want` (< 0: all) at the float64 weights psi_eval
// (grid order; float32 shadow in pos_s.w, r_max per instance on the device); the
// per-instance statistics go to ev_out when it is given.
// wall areas per site: 6 box walls, a convex domain's planes, or a non-convex domain's walls
int wall_count(const lagot_ctx *c) { return c->npieces > 0 ? c->nwalls : (c->ndom > 0 ? c->ndom : 6); }

PieceAcc piece_acc(const lagot_ctx *c) {
    PieceAcc a;
    a.V = c->pa_V;
    a.K = c->pa_K;
    a.mom = c->pa_mom;
    a.fcol = c->pa_fcol;
    a.farea = c->pa_farea;
    a.fcnt = c->pa_fcnt;
    a.flags = c->pa_flags;
    a.wall = c->pa_wall;
    a.cen = c->pa_cen;
    return a;
}

// A non-convex domain (a union of convex pieces with disjoint interiors): the restricted
// cell is the union of its parts in the pieces, so volume, spherical area, facet areas,
// wall areas and first moments are sums over the pieces. Each piece is evaluated as a
// convex domain (all passes), and its outputs are added to the accumulators; the sums are
// then written back as the evaluation's outputs (section 6: cells in polyhedral domains).
void evaluate_pieces(lagot_ctx *c, int want, const double *psi_eval, bool walls, const Batch &bt, const EvalOut &o,
                     bool timed) {
    hipStream_t st = c->stream;
    const QBoxes qb = qboxes(c);
    const PieceAcc acc = piece_acc(c);
    c->eval_crowd = c->crowd;
    if (c->crowd) launch_local_reach(st, c->n, bt, want, c->nc, c->pos_s, c->lr_rmc, c->lr_ir);
    if (timed) (void)hipEventRecord(c->ev0, st);
    for (int k = 0; k < c->npieces; ++k) {
        Batch bk = bt;
        bk.dom = c->dom_d + c->h_dom_off[k];
        bk.ndom = c->h_dom_off[k + 1] - c->h_dom_off[k];
        bk.npieces = 0;
        EvalOut ok = o;
        ok.cen = o.cen ? acc.cen : nullptr;
        launch_piece_begin(st, k == 0, o.fb_count, o.ovf_count, c->misc + 8);
        if (walls) launch_zero_f32(st, c->wall, (int64_t)bk.ndom * c->n);
        launch_cells(st, c->n, bk, want, c->pos_s, psi_eval, c->perm, c->cell_start, ok, qb, c->tpc, c->crowd);
        if (c->prec_on) launch_add_precise(st, c->n, bt, want, c->prec, ok);
        launch_cells_fallback(st, c->n, bk, want, c->pos_s, psi_eval, c->perm, c->cell_start, ok, qb, c->crowd,
                              nullptr, nullptr);
        launch_piece_accum(st, c->n, bt, want, k == 0, ok, bk.ndom, c->dom_wid_d + c->h_dom_off[k], c->nwalls, c->perm,
                           acc);
    }
    launch_piece_final(st, c->n, bt, want, o, c->nwalls, c->perm, c->pos_s, o.cen, acc);
    // the deferred cells of all pieces as the evaluation's count (it turns the crowded pass on)
    launch_piece_begin(st, false, nullptr, o.ovf_count, c->misc + 8);
    if (timed) (void)hipEventRecord(c->ev1, st);
    if (!c->capturing) c->ev_pending = true;
}

void evaluate(lagot_ctx *c, int want, const double *psi_eval, bool walls, double *ev_out) {
    const Batch bt = batch(c);
    const EvalOut o = eval_out(c, walls);
    const bool timed = !c->capturing || c->graph_events;
    launch_eval_begin(c->stream, bt, want, o);
    if (c->npieces > 0) {
        evaluate_pieces(c, want, psi_eval, walls, bt, o, timed);
        if (ev_out) launch_eval_reduce(c->stream, bt, want, c->V, c->nu_s, c->part_ev, ev_out);
        return;
    }
    if (walls)
        (void)hipMemsetAsync(c->wall, 0, (size_t)(c->ndom > 0 ? c->ndom : 6) * sizeof(float) * (size_t)c->n,
                             c->stream);
    const QBoxes qb = qboxes(c);
    c->eval_crowd = c->crowd;
    if (c->crowd) launch_local_reach(c->stream, c->n, bt, want, c->nc, c->pos_s, c->lr_rmc, c->lr_ir);
    if (timed) (void)hipEventRecord(c->ev0, c->stream);
    launch_cells(c->stream, c->n, bt, want, c->pos_s, psi_eval, c->perm, c->cell_start, o, qb, c->tpc, c->crowd);
    if (timed) (void)hipEventRecord(c->ev1, c->stream);
    if (c->prec_on) launch_add_precise(c->stream, c->n, bt, want, c->prec, o);
    if (!c->capturing) c->ev_pending = true;
    const bool tc = timed && c->crowd && !c->capturing;  // the crowded pass is timed outside graphs
    launch_cells_fallback(c->stream, c->n, bt, want, c->pos_s, psi_eval, c->perm, c->cell_start, o, qb, c->crowd,
                          tc ? c->evc0 : nullptr, tc ? c->evc1 : nullptr, c->start_gate ? c->nempty : nullptr);
    if (tc) c->ev_crowd_pending = true;
    if (ev_out) launch_eval_reduce(c->stream, bt, want, c->V, c->nu_s, c->part_ev, ev_out);
}

// Per-bit counts of the cell flags of the last evaluation (bits 0..7: final, 8..15: the
// reasons that sent cells to the float64 pass).
int flag_hist(lagot_ctx *c, int64_t *counts) {
    std::vector<uint32_t> f((size_t)c->n);
    HIP_TRY(hipMemcpyAsync(f.data(), c->flags, sizeof(uint32_t) * (size_t)c->n, hipMemcpyDeviceToHost, c->stream));
    const int rc = sync(c);
    if (rc) return rc;
    for (int k = 0; k < 16; ++k) counts[k] = 0;
    for (uint32_t v : f)
        for (int k = 0; k < 16; ++k) counts[k] += (v >> k) & 1u;
    return LAGOT_OK;
}

void drop_graphs(lagot_ctx *c);

// After a synchronisation: cells deferred by the last evaluation turn the crowded pass on
// for the rest of the call and for the next call (graphs captured without it are dropped).
void note_deferred(lagot_ctx *c, int32_t deferred) {
    if (deferred <= 0) return;
    c->crowd_seen = true;
    if (!c->crowd) {
        c->crowd = true;
        drop_graphs(c);
    }
}

// Phase histogram written by the last control kernel -> h_cnt[0..7]; the cells the last
// evaluation deferred -> h_cnt[9].
int read_counts(lagot_ctx *c) {
    HIP_TRY(hipMemcpyAsync(c->h_cnt, c->counts, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->h_cnt + 9, c->misc + 4, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    const int rc = sync(c);
    if (!rc) note_deferred(c, c->h_cnt[9]);
    return rc;
}

// ---- learned warm start ------------------------------------------------------
int ensure_mlp(lagot_ctx *c) {
    if (c->mlp_p) return LAGOT_OK;
    HIP_TRY(dalloc(&c->mlp_p, MLP_NPARAMS));
    HIP_TRY(dalloc(&c->mlp_g, MLP_NPARAMS));
    HIP_TRY(dalloc(&c->mlp_m1, MLP_NPARAMS));
    HIP_TRY(dalloc(&c->mlp_m2, MLP_NPARAMS));
    HIP_TRY(dalloc(&c->mlp_pb, MLP_NPARAMS));
    return LAGOT_OK;
}

int ensure_inference(lagot_ctx *c, int64_t n) {
    if (n <= c->cap_inf) return LAGOT_OK;
    free_ptrs(c->nbr_s, c->feat_s, c->inf_a, c->inf_b, c->mlp_out);
    c->cap_inf = 0;
    HIP_TRY(dalloc(&c->nbr_s, (size_t)n * N_NEI));
    HIP_TRY(dalloc(&c->feat_s, (size_t)n * MLP_IN));
    HIP_TRY(dalloc(&c->inf_a, (size_t)n * MLP_HID));
    HIP_TRY(dalloc(&c->inf_b, (size_t)n * MLP_HID));
    HIP_TRY(dalloc(&c->mlp_out, (size_t)n));
    c->cap_inf = n;
    return LAGOT_OK;
}

int ensure_batch(lagot_ctx *c, int b) {
    if (b <= c->cap_batch) return LAGOT_OK;
    free_ptrs(c->tX, c->tH1, c->tH2, c->tH3, c->tdZb, c->tZ1, c->tZ2, c->tZ3, c->tdZ, c->ty, c->tt, c->tdy, c->tpart,
              c->tloss);
    c->cap_batch = 0;
    const size_t B = (size_t)b;
    HIP_TRY(dalloc(&c->tX, B * MLP_IN));
    HIP_TRY(dalloc(&c->tH1, B * MLP_HID));
    HIP_TRY(dalloc(&c->tH2, B * MLP_HID));
    HIP_TRY(dalloc(&c->tH3, B * MLP_HID));
    HIP_TRY(dalloc(&c->tdZb, B * MLP_HID));
    HIP_TRY(dalloc(&c->tZ1, B * MLP_HID));
    HIP_TRY(dalloc(&c->tZ2, B * MLP_HID));
    HIP_TRY(dalloc(&c->tZ3, B * MLP_HID));
    HIP_TRY(dalloc(&c->tdZ, B * MLP_HID));
    HIP_TRY(dalloc(&c->ty, B));
    HIP_TRY(dalloc(&c->tt, B));
    HIP_TRY(dalloc(&c->tdy, B));
    HIP_TRY(dalloc(&c->tpart, 4096 * (size_t)MLP_HID + B));
    HIP_TRY(dalloc(&c->tloss, B / 256 + 8));
    c->cap_batch = b;
    return LAGOT_OK;
}

// forward of m rows of bf16 inputs X into out (float32); hidden activations ping-pong in a/b
void mlp_forward_dev(lagot_ctx *c, int m, const uint16_t *X, uint16_t *a, uint16_t *b, float *out) {
    const float *P = c->mlp_p;
    const uint16_t *PB = c->mlp_pb;
    launch_gemm(c->stream, false, false, MLP_EPI_BIAS_GELU, X, PB + MLP_OFF_W1, m, MLP_HID, MLP_IN, nullptr, a,
                P + MLP_OFF_B1, nullptr);
    launch_gemm(c->stream, false, false, MLP_EPI_BIAS_GELU, a, PB + MLP_OFF_W2, m, MLP_HID, MLP_HID, nullptr, b,
                P + MLP_OFF_B2, nullptr);
    launch_gemm(c->stream, false, false, MLP_EPI_BIAS_GELU, b, PB + MLP_OFF_W3, m, MLP_HID, MLP_HID, nullptr, a,
                P + MLP_OFF_B3, nullptr);
    launch_out_layer(c->stream, m, a, P + MLP_OFF_W4, P + MLP_OFF_B4, out, nullptr, nullptr, nullptr);
}

// Inputs of every site in grid order (one instance; needs prepare() with psi =
// psi_prev and nu, and the cell volumes at psi_prev in c->V).
int build_features(lagot_ctx *c) {
    int rc = ensure_inference(c, c->n);
    if (rc) return rc;
    launch_zero_i32(c->stream, c->misc + 1, 1);
    // ev_nu[0] holds sum nu of the (single) instance
    launch_knn_features(c->stream, c->n, c->pos_s, c->perm, c->cell_start, c->h_grid[0], c->psi_s, c->nu_s, c->ev_nu,
                        c->V, c->nbr_s, c->feat_s, c->misc + 1);
    return LAGOT_OK;
}

void fill_defaults(lagot_opts *o) {
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-5;
    o->max_newton = 100;
    o->max_halvings = 30;
    o->cg_rtol = 1e-6;
    o->cg_max_iter = 1000;
    o->threads_per_cell = 0;
    o->verbose = 0;
    o->use_learned = 0;
    o->empty_start_fallback = 1;
    o->autotune = 0;
    o->residual_test = 1;
    o->continuation = 0;
    o->stage_newton = 8;
    o->stage_tol = 1e-2;
    o->step_start = 0;
    o->reserved = 0;
    o->stage_step = 0.25;
    o->stage_gtol = 0.0;
}

bool valid_tpc(int t) { return t == 8 || t == 16 || t == 32 || t == 64; }

int check_opts(const lagot_opts &o) {
    if (!(o.tol > 0) || o.max_newton < 0 || o.max_halvings < 0 || !(o.cg_rtol > 0) || o.cg_max_iter < 1)
        return LAGOT_EINVAL;
    if (!valid_tpc(o.threads_per_cell) && o.threads_per_cell != 0) return LAGOT_EINVAL;
    if (o.continuation != 0 && o.continuation != 1) return LAGOT_EINVAL;
    if (o.continuation && (o.stage_newton < 1 || !(o.stage_tol > 0))) return LAGOT_EINVAL;
    if (o.step_start < 0 || o.step_start > 2 || o.reserved != 0) return LAGOT_EINVAL;
    if (o.continuation && !(o.stage_step > 0.0 && o.stage_step <= 1.0)) return LAGOT_EINVAL;
    if (!(o.stage_gtol >= 0.0 && o.stage_gtol < 1.0)) return LAGOT_EINVAL;
    return LAGOT_OK;
}

// Autotuner: time the float32 cell kernel with 16, 32 and 64 lanes per cell at the
// start weights and keep the fastest for this class of problem (log2 of the mean
// instance size, log2 of the sites per ball volume); later calls of the class reuse it.
int autotune_tpc(lagot_ctx *c) {
    std::vector<double> r(c->B);
    HIP_TRY(hipMemcpyAsync(r.data(), c->rmax, sizeof(double) * c->B, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    double rm = 0.0, vol = 0.0;
    for (int b = 0; b < c->B; ++b) {
        rm = std::max(rm, r[b]);
        const GridDesc &g = c->h_grid[b];
        vol += (double)g.dim[0] * g.dim[1] * g.dim[2] * g.s * g.s * g.s;
    }
    const double per_ball = (double)c->n * (4.0 / 3.0) * M_PI * rm * rm * rm / std::max(vol, 1e-300);
    const int key = (int)std::floor(std::log2((double)c->n / c->B)) * 64 +
                    std::min(63, std::max(0, (int)std::floor(std::log2(per_ball + 1e-30)) + 32));
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) {
        c->tpc = it->second.tpc;
        if (it->second.cg) {
            c->cg_lanes = it->second.cg_lanes;
            c->cg_sub = it->second.cg_sub;
        } else {
            c->tune_key = key;
        }
        return LAGOT_OK;
    }
    const int cand[3] = {16, 32, 64};
    float best = 1e30f;
    int best_t = c->tpc_default;
    for (int t : cand) {
        c->tpc = t;
        for (int rep = 0; rep < 2; ++rep) {  // the second run is timed
            evaluate(c, -1, c->psi_s, false, nullptr);
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        c->ev_pending = false;
        c->ev_crowd_pending = false;
        if (ms < best) {
            best = ms;
            best_t = t;
        }
    }
    c->tpc = best_t;
    c->tuned[key].tpc = best_t;
    c->tune_key = key;
    return LAGOT_OK;
}

// Inward margin of the fluid step's position update, relative to the box extent.
constexpr double ADVECT_MARGIN = 1e-6;

// spacing of float32 numbers at |v|
double ulp32(double v) {
    const float f = (float)std::fabs(v);
    return (double)std::nextafter(f, INFINITY) - (double)f;
}

// ---- graph mode ---------------------------------------------------------------
void drop_graphs(lagot_ctx *c) {
    if (c->g_dir) (void)hipGraphExecDestroy(c->g_dir);
    if (c->g_trial) (void)hipGraphExecDestroy(c->g_trial);
    for (auto &kv : c->g_cg) (void)hipGraphExecDestroy(kv.second);
    c->g_dir = c->g_trial = nullptr;
    c->g_cg.clear();
}

// Capture what `enqueue` launches on the context stream into an executable graph.
template <typename F> int capture(lagot_ctx *c, F &&enqueue, hipGraphExec_t *out) {
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    enqueue();
    c->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || !g) {
        fprintf(stderr, "lagot: graph capture failed: %s\n", hipGetErrorString(e));
        return LAGOT_EHIP;
    }
    const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        fprintf(stderr, "lagot: graph instantiation failed: %s\n", hipGetErrorString(e2));
        return LAGOT_EHIP;
    }
    return LAGOT_OK;
}

// The PCG scalars need their own kernel when an instance has more partials (sub-tiles)
// than the iteration's blocks sum themselves.
bool cg_scalar_launch(const lagot_ctx *c) {
    return (int64_t)c->max_inst_tiles * (TILE / c->cg_sub) > cg_sum_in_block_max();
}

// Jacobi-PCG for every ACTIVE instance with the context's block shape: chunks of
// launches, then the count of instances still iterating is read back.
int run_cg(lagot_ctx *c, const lagot_opts &o, int *launched, bool with_init, bool graph) {
    const Batch bt = batch(c);
    const CgBufs cg = cg_bufs(c);
    hipStream_t st = c->stream;
    if (with_init)
    {
        launch_cg_init(st, bt, c->cg_lanes, c->cg_sub, c->V, c->nu_s, c->diag, c->hrow, c->hent, cg);
        if (cg_scalar_launch(c)) launch_cg_scalars(st, bt, c->cg_sub, -1, o.cg_max_iter, cg);
    }
    const double rtol2 = o.cg_rtol * o.cg_rtol;
    const int cap = o.cg_max_iter;
    int k = 0;
    while (k < cap) {
        const int m = std::min(c->cg_chunk, cap - k);
        const bool split = c->cg_split == 2 || (c->cg_split == 0 && cg_scalar_launch(c));
        auto chunk = [&]() {
            for (int q = 0; q < m; ++q) {
                if (split)
                    launch_cg_split_iter(c->stream, bt, c->cg_lanes, c->cg_sub, q, rtol2, cap, c->hrow, c->hent, cg);
                else
                    launch_cg_iter(c->stream, bt, c->cg_lanes, c->cg_sub, q, rtol2, cap, c->hrow, c->hent, cg);
                if (cg_scalar_launch(c)) launch_cg_scalars(c->stream, bt, c->cg_sub, q, cap, cg);
            }
            launch_cg_advance(c->stream, bt, m, cap, cg);
        };
        if (graph) {
            hipGraphExec_t &ex = c->g_cg[m];
            if (!ex) {
                int rc = capture(c, chunk, &ex);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(ex, st));
        } else {
            chunk();
        }
        k += m;
        HIP_TRY(hipMemcpyAsync(c->h_cnt + 8, c->misc + 3, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(c->h_cnt + 10, c->misc + 7, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        int rc = sync(c);
        if (rc) return rc;
        if (c->h_cnt[8] == 0) break;
    }
    *launched = k;
    return LAGOT_OK;
}

// One Jacobi-PCG direction solve for every ACTIVE instance, then ACTIVE -> TRIAL.
// When the autotuner asks for it, the solve is first run with each candidate block
// shape (the same system each time) and the fastest shape is kept for the class.
int newton_direction(lagot_ctx *c, const lagot_opts &o, bool graph) {
    const Batch bt = batch(c);
    hipStream_t st = c->stream;
    if (c->cap_hent_T < c->T) {  // one TILE * FCAP region of packed Hessian entries per tile
        if (graph) drop_graphs(c);   // captured launches hold the old buffer
        free_ptrs(c->hent);
        c->cap_hent_T = 0;
        HIP_TRY(dalloc(&c->hent, (size_t)c->T * TILE * FCAP));
        c->cap_hent_T = c->T;
    }
    auto assemble = [&](bool with_init) {
        launch_hess_assemble(c->stream, c->n, bt, PH_ACTIVE, c->pos_s, c->fcol, c->farea, c->fcnt, c->hcol, c->hval,
                             c->xcnt, c->herr);
        launch_hess_finish(c->stream, bt, PH_ACTIVE, c->psi_s, c->K, c->fcnt, c->xcnt, c->hcnt, c->hcol, c->hval,
                           c->diag, c->hrow, c->hent);
        if (with_init) {
            launch_cg_init(c->stream, bt, c->cg_lanes, c->cg_sub, c->V, c->nu_s, c->diag, c->hrow, c->hent,
                           cg_bufs(c));
            if (cg_scalar_launch(c)) launch_cg_scalars(c->stream, bt, c->cg_sub, -1, o.cg_max_iter, cg_bufs(c));
        }
    };
    int k = 0, rc;
    if (c->tune_key < 0) {
        // Hessian, PCG set-up, PCG chunks
        if (graph) {
            if (!c->g_dir) {
                rc = capture(c, [&]() { assemble(true); }, &c->g_dir);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(c->g_dir, st));
        } else {
            assemble(true);
        }
        rc = run_cg(c, o, &k, false, graph);
        if (rc) return rc;
    } else {
        assemble(false);
        static const int shapes[4][2] = {{2, 128}, {4, 128}, {2, 64}, {4, 64}};
        double best = 1e300;
        int bl = c->cg_lanes, bs = c->cg_sub;
        for (const auto &sh : shapes) {
            c->cg_lanes = sh[0];
            c->cg_sub = sh[1];
            rc = sync(c);
            if (rc) return rc;
            const double t0 = now_ms();
            rc = run_cg(c, o, &k, true, false);
            if (rc) return rc;
            const double ms = now_ms() - t0;
            if (ms < best) {
                best = ms;
                bl = sh[0];
                bs = sh[1];
            }
        }
        auto &tu = c->tuned[c->tune_key];
        tu.cg_lanes = bl;
        tu.cg_sub = bs;
        tu.cg = true;
        c->tune_key = -1;
        c->cg_lanes = bl;
        c->cg_sub = bs;
        if (!(bl == shapes[3][0] && bs == shapes[3][1])) {
            rc = run_cg(c, o, &k, true, false);  // the direction of the kept shape
            if (rc) return rc;
        }
    }
    // chunk length for the next direction: this solve's iteration count (the iterations
    // it ran, not the launches: a launch after convergence returns at once but is not
    // free) plus two, in steps of four (graph mode captures one chunk per length)
    c->cg_chunk = std::min(64, std::max(4, (c->h_cnt[10] + 2 + 3) / 4 * 4));
    launch_cg_finish(st, bt, c->cg_sub, o.cg_rtol * o.cg_rtol, o.step_start, cg_bufs(c), c->herr, c->ctl, c->phase);
    return LAGOT_OK;
}

struct CallTimes {
    double eval = 0, lin = 0, learned = 0;
    int extra_evals = 0;
};

// Learned guess for a single instance, taken like a Newton step from the start weights:
// psi + beta s^2 out for beta = 1, 1/2, 1/4 (Algorithm 1's step halving applied to the
// network's correction, so that a few outlying weights that empty cells at the full step
// do not throw the whole guess away), each evaluated into the second set of outputs; the
// first that keeps every cell above eps0 and lowers both the residual norm and the largest
// relative volume error (the stop test) is kept. *accepted = 1 + the halvings taken, or 0.
int learned_guess(lagot_ctx *c, CallTimes &tm, int *accepted) {
    *accepted = 0;
    const Batch bt = batch(c);
    hipStream_t st = c->stream;
    double *h = (double *)c->h_rd;  // [0..3] start, [4..7] guess, [8] min nu
    int32_t *hf = (int32_t *)(h + 12);
    HIP_TRY(hipMemcpyAsync(h, c->ev, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(h + 8, c->ev_nu + 3, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hf, c->fail_inst, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    int rc = sync(c);
    if (rc) return rc;
    const double eps0 = 0.5 * std::min(h[8], h[3]);
    if (hf[0] != 0 || !(eps0 > 0.0)) return LAGOT_OK;  // Newton handles this start itself
    const double t0 = now_ms();
    rc = build_features(c);
    if (!rc) rc = ensure_alt(c);
    if (rc) return rc;
    mlp_forward_dev(c, (int)c->n, c->feat_s, c->inf_a, c->inf_b, c->mlp_out);
    constexpr int GUESS_HALVINGS = 2;
    for (int k = 0; k <= GUESS_HALVINGS && !*accepted; ++k) {
        launch_apply_guess(st, c->n, c->psi_s, c->nu_s, c->mlp_out, std::ldexp(1.0, -k), c->psi_trial, c->pos_s);
        launch_rmax(st, bt, -1, c->psi_trial, c->rmax);
        swap_alt(c);  // the guess's cells go to the second output set
        evaluate(c, -1, c->psi_trial, false, c->ev2);
        swap_alt(c);
        tm.extra_evals++;
        HIP_TRY(hipMemcpyAsync(h + 4, c->ev2, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hf + 1, c->fail_inst, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hf + 2, c->misc + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        rc = sync(c);
        if (rc) return rc;
        if (hf[2] == 0 && hf[1] == 0 && h[7] >= eps0 && h[6] < h[2] && h[5] < h[1]) *accepted = 1 + k;
    }
    if (*accepted) {
        HIP_TRY(hipMemcpyAsync(c->psi_s, c->psi_trial, sizeof(double) * c->n, hipMemcpyDeviceToDevice, st));
        swap_alt(c);
    } else {
        // back to the start weights, whose cells are still in the first output set
        launch_psi_shadow(st, c->n, c->psi_s, c->pos_s);
        launch_rmax(st, bt, -1, c->psi_s, c->rmax);
        launch_zero_i32(st, c->fail_inst, 1);  // the start had no failed cell (checked above)
    }
    tm.learned += now_ms() - t0;
    return LAGOT_OK;
}

// Path following on the prescribed volumes (one instance; opts.continuation). From a
// start far from the solution, Algorithm 1's global step length can collapse: some cell
// empties under every long step, and KMT halves the step for all cells. With V0 the
// volumes at the start iterate, the start solves the problem with targets V0 exactly;
// the targets nu(s) = (1 - s) V0 + s nu (sum below the box volume for every s, positive)
// are then solved for s rising to 1, each stage by Algorithm 1 from the weights of the
// last accepted stage. Stage results are accepted only through Newton's own test, so the
// final stage is a plain solve of the problem to the caller's tolerance.
template <typename Loop>
int continuation(lagot_ctx *c, const lagot_opts &o, const CtlOpts &co, CallTimes &tm, Loop &&newton_loop,
                 int *stages_out) {
    const Batch bt = batch(c);
    hipStream_t st = c->stream;
    const int64_t n = c->n;
    if (n > c->cap_cont) {
        free_ptrs(c->cont_buf);
        c->cap_cont = 0;
        HIP_TRY(dalloc(&c->cont_buf, 3 * (size_t)n));
        c->cap_cont = n;
    }
    double *v0 = c->cont_buf, *nu_t = v0 + n, *psi_ok = nu_t + n;
    HIP_TRY(hipMemcpyAsync(v0, c->V, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(nu_t, c->nu_s, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(psi_ok, c->psi_s, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    lagot_opts os = o;
    os.cg_rtol = std::max(o.cg_rtol, 1e-2);  // inexact directions suffice for a loose stage
    os.max_newton = o.stage_newton;
    CtlOpts cs = co;
    cs.tol = o.stage_tol;
    cs.max_newton = o.stage_newton;
    cs.max_halvings = std::min(o.max_halvings, 4);  // a stage that needs short steps is retried closer
    cs.gtol = o.stage_gtol;
    double s = 0.0, ds = o.stage_step;
    int stages = 0, rc = LAGOT_OK;
    for (;;) {
        const double s1 = std::min(1.0, s + ds);
        const bool last = s1 >= 1.0;
        const CtlOpts &cc = last ? co : cs;
        if (o.use_graph) drop_graphs(c);  // captured launches hold the stage's options
        launch_nu_stage(st, n, s1, v0, nu_t, c->nu_s);
        launch_eval_reduce(st, bt, -1, c->nu_s, c->nu_s, c->part_ev, c->ev_nu);
        launch_eval_reduce(st, bt, -1, c->V, c->nu_s, c->part_ev, c->ev);
        launch_ctl_stage(st, bt, cc, c->ev, c->ev_nu, c->fail_inst, c->ctl, c->phase, c->counts);
        InstCtl q0, q1;
        HIP_TRY(hipMemcpyAsync(&q0, c->ctl, sizeof(q0), hipMemcpyDeviceToHost, st));
        rc = read_counts(c);
        if (rc) return rc;
        rc = newton_loop(last ? o : os, cc);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(&q1, c->ctl, sizeof(q1), hipMemcpyDeviceToHost, st));
        rc = sync(c);
        if (rc) return rc;
        const int its = q1.iters - q0.iters, halv = q1.halvings - q0.halvings;
        if (o.verbose)
            fprintf(stderr, "lagot continuation s %.5f (step %.5f): status %d, %d Newton iterations, %d halvings\n", s1,
                    ds, q1.status, its, halv);
        if (q1.status == LAGOT_OK) {
            ++stages;
            s = s1;
            if (last) break;
            HIP_TRY(hipMemcpyAsync(psi_ok, c->psi_s, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            if (its <= 3 && halv == 0) ds *= 2.0;
        } else if (q1.status == LAGOT_ENOCONV || q1.status == LAGOT_ELINESEARCH || q1.status == LAGOT_ECAPACITY) {
            // back to the last accepted stage, with a shorter step in s
            ds *= 0.5;
            if (ds < 1.0 / 4096.0) break;
            HIP_TRY(hipMemcpyAsync(c->psi_s, psi_ok, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            launch_psi_shadow(st, n, c->psi_s, c->pos_s);
            launch_rmax(st, bt, -1, c->psi_s, c->rmax);
            evaluate(c, -1, c->psi_s, false, nullptr);
            tm.extra_evals++;
        } else {
            break;  // empty start cell, capacity, PCG breakdown: the stage's error is the call's
        }
    }
    *stages_out = stages;
    if (s < 1.0) {
        // failed: the call returns the last accepted stage's weights with the failing
        // stage's status and the residuals against the caller's volumes
        InstCtl q;
        HIP_TRY(hipMemcpyAsync(&q, c->ctl, sizeof(q), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(c->psi_s, psi_ok, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(c->nu_s, nu_t, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        launch_psi_shadow(st, n, c->psi_s, c->pos_s);
        launch_rmax(st, bt, -1, c->psi_s, c->rmax);
        evaluate(c, -1, c->psi_s, false, c->ev);
        tm.extra_evals++;
        double e[4];
        HIP_TRY(hipMemcpyAsync(e, c->ev, sizeof(e), hipMemcpyDeviceToHost, st));
        rc = sync(c);
        if (rc) return rc;
        q.sumV = e[0];
        q.maxrel = e[1];
        q.gnorm = e[2];
        q.minV = e[3];
        if (q.status == LAGOT_OK) q.status = LAGOT_ENOCONV;
        const int32_t failed = PH_FAILED;
        HIP_TRY(hipMemcpyAsync(c->ctl, &q, sizeof(q), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(c->phase, &failed, sizeof(failed), hipMemcpyHostToDevice, st));
        rc = sync(c);
        if (rc) return rc;
    }
    return LAGOT_OK;
}

// Damped Newton (Algorithm 1, KMT step control) for every instance of the call;
// single = true takes at most one Newton iteration per instance.
int newton_run_impl(lagot_ctx *c, int B, const int64_t *offs, const float *x, const float *y, const float *z,
                    const double *nu, const lagot_box *boxes, double *psi, const lagot_opts &o, lagot_stats *stats,
                    bool single, double t0) {
    const bool graph = o.use_graph != 0;
    std::vector<int> bad(std::max(B, 1), 0);
    auto fail_all = [&](int rc) {
        if (stats)
            for (int b = 0; b < B; ++b) {
                std::memset(&stats[b], 0, sizeof(lagot_stats));
                stats[b].status = rc;
                stats[b].ms_total = now_ms() - t0;
            }
        return rc;
    };
    int rc = check_opts(o);
    if (!rc && (!nu || !psi)) rc = LAGOT_EINVAL;
    if (!rc && o.use_learned && B != 1) rc = LAGOT_EINVAL;
    if (!rc && o.continuation && B != 1) rc = LAGOT_EINVAL;
    if (rc) return fail_all(rc);
    c->tpc = o.threads_per_cell ? o.threads_per_cell : c->tpc_default;
    c->ms_cell = 0.0;
    c->ms_crowd = 0.0;
    c->crowd_launches = 0;
    c->crowd_cells = 0;
    c->cell_launches = 0;
    c->ev_pending = false;
    c->ev_crowd_pending = false;
    rc = prepare(c, B, offs, x, y, z, psi, nu, boxes, &bad);
    if (rc) return fail_all(rc);
    // cells marked for the float64 path at a stalled final iteration stay marked for the call
    struct PrecScope {
        lagot_ctx *c;
        ~PrecScope() { c->prec_on = false; }
    } prec_scope{c};
    launch_zero_i32(c->stream, reinterpret_cast<int32_t *>(c->prec), (c->n + 3) / 4);
    c->prec_on = true;
    c->tune_key = -1;
    c->cg_lanes = c->cg_lanes_def;
    c->cg_sub = c->cg_sub_def;
    if (o.autotune && o.threads_per_cell == 0) {
        rc = autotune_tpc(c);
        if (rc) return fail_all(rc);
        c->ms_cell = 0.0;
        c->ms_crowd = 0.0;
        c->crowd_launches = 0;
        c->crowd_cells = 0;
        c->cell_launches = 0;
    }
    const Batch bt = batch(c);
    hipStream_t st = c->stream;
    CtlOpts co{o.tol, o.max_newton, o.max_halvings, single ? 1 : 0, o.empty_start_fallback ? 1 : 0,
               o.residual_test ? 1 : 0, 0, o.step_start == 2 ? 1 : 0, 0.0};
    CallTimes tm;
    int learned = 0;
    launch_zero_i32(st, c->fb_inst, B);
    launch_ctl_init(st, bt, c->ctl, c->phase);
    double te = now_ms();
    // a start that the repair gate will send to the restart anyway (judged from the float32
    // pass's empty cells) skips the crowded and float64 passes of its evaluation
    c->start_gate = B == 1 && o.empty_start_fallback && !(o.use_learned && c->mlp_set) && c->npieces == 0;
    evaluate(c, PH_START, c->psi_s, false, c->ev);
    c->start_gate = false;
    if (o.use_learned && c->mlp_set) {
        rc = learned_guess(c, tm, &learned);
        if (rc) return fail_all(rc);
    }
    // the KMT floor eps0 comes from the given start weights (ev); a kept guess supplies
    // the statistics of the first iterate (ev2)
    launch_ctl_start(st, bt, co, PH_START, learned ? c->ev2 : c->ev, c->ev_nu, c->ev, c->fail_inst, c->ctl, c->phase,
                     c->counts);
    rc = read_counts(c);
    if (rc) return fail_all(rc);
    // the repair is for a few empty start cells: an instance with more than 64 empty cells,
    // and more than 1% of its cells (a warm start from weights of much moved sites), goes to
    // the restart at once
    if (c->h_cnt[PH_REPAIR] > 0) {
        launch_repair_gate(st, bt, PH_REPAIR, c->V, c->nempty, c->phase, c->counts);
        rc = read_counts(c);
        if (rc) return fail_all(rc);
    }
    // repair rounds: raising one cell can empty a neighbour's, so a repaired start is
    // checked and repaired again, up to REPAIR_ROUNDS times, before the full restart
    constexpr int REPAIR_ROUNDS = 2;
    for (int round = 0; round < REPAIR_ROUNDS && c->h_cnt[PH_REPAIR] > 0; ++round) {
        launch_repair_empty(st, bt, PH_REPAIR, c->V, c->nu_s, c->cell_start, c->psi_s, c->psi_trial, c->pos_s);
        std::swap(c->psi_s, c->psi_trial);
        launch_rmax(st, bt, PH_REPAIR, c->psi_s, c->rmax);
        evaluate(c, PH_REPAIR, c->psi_s, false, c->ev);
        CtlOpts cr = co;
        cr.repair_more = round + 1 < REPAIR_ROUNDS ? 1 : 0;
        launch_ctl_start(st, bt, cr, PH_REPAIR, c->ev, c->ev_nu, c->ev, c->fail_inst, c->ctl, c->phase, c->counts);
        rc = read_counts(c);
        if (rc) return fail_all(rc);
    }
    if (c->h_cnt[PH_RESTART] > 0) {
        launch_default_start(st, bt, PH_RESTART, c->ev_nu, c->psi_s, c->pos_s);
        launch_rmax(st, bt, PH_RESTART, c->psi_s, c->rmax);
        evaluate(c, PH_RESTART, c->psi_s, false, c->ev);
        launch_ctl_start(st, bt, co, PH_RESTART, c->ev, c->ev_nu, c->ev, c->fail_inst, c->ctl, c->phase, c->counts);
        rc = read_counts(c);
        if (rc) return fail_all(rc);
    }
    tm.eval += now_ms() - te - tm.learned;
    int round = 0;
    // Newton iterations of every ACTIVE instance until none is left (Algorithm 1 with the
    // step control on the device), with options o and control options co
    auto newton_loop = [&](const lagot_opts &o, const CtlOpts &co) -> int {
    while (c->h_cnt[PH_ACTIVE] > 0) {
        const double tl = now_ms();
        rc = newton_direction(c, o, graph);
        if (rc) return rc;
        tm.lin += now_ms() - tl;
        te = now_ms();
        // one step-size trial of every instance in the search (Alg. 1, KMT test on the device)
        auto trial = [&]() {
            launch_axpy_trial(c->stream, bt, c->ctl, c->psi_s, cg_bufs(c).x, c->psi_trial, c->pos_s);
            launch_rmax(c->stream, bt, PH_TRIAL, c->psi_trial, c->rmax);
            evaluate(c, PH_TRIAL, c->psi_trial, false, c->ev);
            launch_ctl_decide(c->stream, bt, co, c->ev, c->fail_inst, c->ctl, c->phase);
            launch_accept_rows(c->stream, bt, c->ctl, c->psi_s, c->psi_trial, c->pos_s);
            launch_ctl_commit(c->stream, bt, co, c->ctl, c->phase, c->counts);
            launch_mark_precise(c->stream, bt, co, c->ctl, c->V, c->nu_s, c->prec);
        };
        for (int h = 0; h <= o.max_halvings; ++h) {
            if (graph) {
                if (!c->g_trial) {
                    rc = capture(c, trial, &c->g_trial);
                    if (rc && c->graph_events) {  // no event nodes on this runtime: capture untimed
                        c->graph_events = false;
                        rc = capture(c, trial, &c->g_trial);
                    }
                    if (rc) return rc;
                }
                if (hipGraphLaunch(c->g_trial, st) != hipSuccess) return LAGOT_EHIP;
                c->ev_pending = c->graph_events;
            } else {
                trial();
            }
            rc = read_counts(c);
            if (rc) return rc;
            if (o.verbose > 2) {  // every step-size trial of the first instance
                InstCtl q;
                HIP_TRY(hipMemcpy(&q, c->ctl, sizeof(q), hipMemcpyDeviceToHost));
                fprintf(stderr, "    trial %d: minV %.4e (eps0 %.4e) |g| %.6e (accepted |g| %.6e) -> %s\n", h, q.tminV,
                        q.eps0, q.tgnorm, q.gnorm, c->h_cnt[PH_TRIAL] == 0 ? "kept" : "halved");
                int32_t fl = 0;
                HIP_TRY(hipMemcpy(&fl, c->fail_inst, sizeof(fl), hipMemcpyDeviceToHost));
                if (fl) {  // cells that failed every pass: their flags (final, and first-pass reasons)
                    int64_t h16[16];
                    rc = flag_hist(c, h16);
                    if (rc) return rc;
                    fprintf(stderr, "      %d failed cells; flag bits:", fl);
                    for (int k = 0; k < 16; ++k) fprintf(stderr, " %lld", (long long)h16[k]);
                    fprintf(stderr, "\n");
                }
            }
            if (c->h_cnt[PH_TRIAL] == 0) break;
        }
        tm.eval += now_ms() - te;
        ++round;
        if (o.verbose) {
            fprintf(stderr, "lagot newton round %d: active %d done %d failed %d (linear %.1f ms, eval %.1f ms)\n",
                    round, c->h_cnt[PH_ACTIVE], c->h_cnt[PH_DONE], c->h_cnt[PH_FAILED], tm.lin, tm.eval);
            if (o.verbose > 1) {  // state of the first instance
                InstCtl q;
                int32_t fb = 0, fl = 0;
                double rm = 0.0;
                HIP_TRY(hipMemcpyAsync(&q, c->ctl, sizeof(q), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipMemcpyAsync(&fb, c->fb_inst, sizeof(fb), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipMemcpyAsync(&fl, c->fail_inst, sizeof(fl), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipMemcpyAsync(&rm, c->rmax, sizeof(rm), hipMemcpyDeviceToHost, st));
                rc = sync(c);
                if (rc) return rc;
                fprintf(stderr,
                        "  inst 0: alpha %.3g |g| %.3e maxrel %.3e minV %.3e eps0 %.3e evals %d halvings %d cg %d "
                        "fallback %d failed (last evaluation) %d r_max %.4g cell kernel %.1f ms; last trial: "
                        "minV %.3e |g| %.3e\n",
                        q.alpha, q.gnorm, q.maxrel, q.minV, q.eps0, q.evals, q.halvings, q.cg_iters, fb, fl, rm, c->ms_cell,
                        q.tminV, q.tgnorm);
            }
        }
    }
    return LAGOT_OK;
    };
    int stages = 0;
    if (o.continuation && !single && c->h_cnt[PH_ACTIVE] > 0) {
        rc = continuation(c, o, co, tm, newton_loop, &stages);
    } else {
        rc = newton_loop(o, co);
    }
    if (rc) return fail_all(rc);

    // weights back to caller order (every instance holds its last accepted iterate)
    launch_scatter_out_f64(st, c->n, c->perm, c->psi_s, psi);
    std::vector<InstCtl> hc(B);
    std::vector<int32_t> hfb(B), hfail(B);
    HIP_TRY(hipMemcpyAsync(hc.data(), c->ctl, sizeof(InstCtl) * B, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hfb.data(), c->fb_inst, sizeof(int32_t) * B, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hfail.data(), c->fail_inst, sizeof(int32_t) * B, hipMemcpyDeviceToHost, st));
    rc = sync(c);
    if (rc) return fail_all(rc);
    const double ms_total = now_ms() - t0;
    int first = LAGOT_OK;
    for (int b = 0; b < B; ++b) {
        const InstCtl &q = hc[b];
        if (first == LAGOT_OK && q.status != LAGOT_OK) first = q.status;
        if (!stats) continue;
        lagot_stats &S = stats[b];
        std::memset(&S, 0, sizeof(S));
        S.status = q.status;
        S.newton_iters = q.iters;
        S.evals = q.evals + (B == 1 ? tm.extra_evals : 0);
        S.halvings = q.halvings;
        S.cg_iters = q.cg_iters;
        S.fallback_cells = hfb[b];
        S.failed_cells = hfail[b];
        S.cell_launches = c->cell_launches;
        S.learned_accepted = learned;
        S.default_start = q.default_start;
        S.repaired_start = q.repaired;
        S.stages = stages;
        S.max_rel_err = q.maxrel;
        S.grad_norm = q.gnorm;
        S.ms_total = ms_total;
        S.ms_eval = tm.eval;
        S.ms_linear = tm.lin;
        S.ms_cell_kernel = c->ms_cell;
        S.ms_learned = tm.learned;
    }
    return first;
}

int newton_run(lagot_ctx *c, int B, const int64_t *offs, const float *x, const float *y, const float *z,
               const double *nu, const lagot_box *boxes, double *psi, const lagot_opts *opts_in,
               lagot_stats *stats, bool single) {
    const double t0 = now_ms();
    lagot_opts o;
    if (opts_in)
        o = *opts_in;
    else
        fill_defaults(&o);
    if (!o.use_graph) return newton_run_impl(c, B, offs, x, y, z, nu, boxes, psi, o, stats, single, t0);
    // graph mode: the call runs on the context's private stream (a legacy default stream
    // cannot be captured), after everything already enqueued on the context's stream
    if (!c->gstream) {
        HIP_TRY(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    }
    HIP_TRY(hipEventRecord(c->ev_in, c->stream));
    HIP_TRY(hipStreamWaitEvent(c->gstream, c->ev_in, 0));
    hipStream_t user = c->stream;
    c->stream = c->gstream;
    const int rc = newton_run_impl(c, B, offs, x, y, z, nu, boxes, psi, o, stats, single, t0);
    (void)hipStreamSynchronize(c->gstream);
    c->stream = user;
    drop_graphs(c);
    return rc;
}

int single_instance(lagot_ctx *c, int64_t n, const float *x, const float *y, const float *z, const double *nu,
                    const lagot_box &box, double *psi, const lagot_opts *opts, lagot_stats *stats, bool single) {
    if (n <= 0) {
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->status = LAGOT_EINVAL;
        }
        return LAGOT_EINVAL;
    }
    const int64_t offs[2] = {0, n};
    lagot_stats S;
    const int rc = newton_run(c, 1, offs, x, y, z, nu, &box, psi, opts, &S, single);
    if (stats) *stats = S;
    return rc;
}

// Parameters of the velocity update: dt > 0, eps > 0 (+inf allowed), gamma >= 0, the
// scalar viscosity >= 0 when no per-site array is given, finite gravity, a PCG tolerance
// in (0, 1) and at least one PCG iteration.
bool fluid_params_ok(const lagot_fluid_params &p, bool per_site_mu) {
    bool ok = p.dt > 0.0 && std::isfinite(p.dt) && p.eps > 0.0 && !std::isnan(p.eps) && p.gamma >= 0.0 &&
              std::isfinite(p.gamma) && p.cg_rtol > 0.0 && p.cg_rtol < 1.0 && p.cg_max_iter >= 1 &&
              (per_site_mu || (p.mu >= 0.0 && std::isfinite(p.mu)));
    for (int a = 0; a < 3; ++a) ok = ok && std::isfinite(p.gravity[a]);
    return ok;
}

// Cells at (x, psi) with their facet weights: the P1 Laplacian's w_ij in hcol/hval/hcnt
// (grid order, sorted rows), and the centroids into cen (caller order) when given.
int fluid_cells(lagot_ctx *c, int64_t n, const float *x, const float *y, const float *z, const double *psi,
                const lagot_box &box, double *cen) {
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    c->ms_cell = 0.0;
    c->ms_crowd = 0.0;
    c->crowd_launches = 0;
    c->crowd_cells = 0;
    c->cell_launches = 0;
    c->ev_pending = false;
    c->ev_crowd_pending = false;
    hipStream_t st = c->stream;
    int rc = LAGOT_OK;
    if (c->fl_reuse) {
        // the solve that just ran on this context sorted these sites and left the final
        // weights in psi_s (float32 shadow in pos_s.w): only r_max follows the weights
        if (c->n != n || c->B != 1) return LAGOT_EINVAL;
        launch_rmax(st, batch(c), -1, c->psi_s, c->rmax);
    } else {
        c->tpc = c->tpc_default;
        const int64_t offs[2] = {0, n};
        rc = prepare(c, 1, offs, x, y, z, psi, nullptr, &box, nullptr);
        if (rc) return rc;
    }
    launch_zero_i32(st, c->fb_inst, 1);
    c->cen_out = cen;
    evaluate(c, -1, c->psi_s, false, nullptr);
    c->cen_out = nullptr;
    const Batch bt = batch(c);
    launch_hess_assemble(st, n, bt, -1, c->pos_s, c->fcol, c->farea, c->fcnt, c->hcol, c->hval, c->xcnt, c->herr);
    launch_hess_finish(st, bt, -1, c->psi_s, c->K, c->fcnt, c->xcnt, c->hcnt, c->hcol, c->hval, c->diag, nullptr,
                       nullptr);
    HIP_TRY(hipMemcpyAsync(c->h_cnt, c->misc, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(c->h_cnt + 1, c->fail_inst, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(c->h_cnt + 2, c->herr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(c->h_cnt + 9, c->misc + 4, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    rc = sync(c);
    if (rc) return rc;
    note_deferred(c, c->h_cnt[9]);
    c->last_fb = c->h_cnt[0];
    if (c->h_cnt[1] != 0 || c->h_cnt[2] != 0) return LAGOT_ECAPACITY;
    return LAGOT_OK;
}

}  // namespace

extern "C" {

void lagot_default_opts(lagot_opts *opts) {
    if (opts) fill_defaults(opts);
}

// Address of this device's copy of the static scratch array, looked up once per device
// (with that device current) and kept for the life of the process.
static int noalloc_scratch_ptr(int device, uint16_t **out) {
    static std::mutex mu;
    static std::map<int, uint16_t *> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            fprintf(stderr, "lagot: hipGetSymbolAddress(scratch) failed on device %d: %s\n", device,
                    hipGetErrorString(e));
            return LAGOT_EHIP;
        }
        it = addr.emplace(device, static_cast<uint16_t *>(ptr)).first;
    }
    *out = it->second;
    return LAGOT_OK;
}

int lagot_create(lagot_ctx **out, int device, void *stream) {
    if (!out) return LAGOT_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LAGOT_EHIP;
    if (hipSetDevice(device) != hipSuccess) return LAGOT_EHIP;
    uint16_t *noalloc = nullptr;
    if (noalloc_scratch_ptr(device, &noalloc) != LAGOT_OK) return LAGOT_EHIP;
    lagot_ctx *c = new lagot_ctx();
    c->device = device;
    c->noalloc = noalloc;
    c->stream = (hipStream_t)stream;
    if (dalloc(&c->counts, 8) != hipSuccess || dalloc(&c->misc, 16) != hipSuccess ||
        hipHostMalloc((void **)&c->h_cnt, 16 * sizeof(int32_t)) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreate(&c->evc0) != hipSuccess || hipEventCreate(&c->evc1) != hipSuccess) {
        free_all(c);
        delete c;
        return LAGOT_EHIP;
    }
    *out = c;
    return LAGOT_OK;
}

void lagot_destroy(lagot_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
}

int lagot_centroids(lagot_ctx *c, int64_t n, const float *x, const float *y, const float *z, const double *psi,
                    lagot_box box, double *vol, double *centroid) {
    if (!c || !vol || !centroid || n <= 0) return LAGOT_EINVAL;
    c->cen_out = centroid;
    const int rc = lagot_cells(c, n, x, y, z, psi, box, vol, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                               nullptr);
    c->cen_out = nullptr;
    return rc;
}

int lagot_cells(lagot_ctx *c, int64_t n, const float *x, const float *y, const float *z, const double *psi,
                lagot_box box, double *vol, double *sph_area, float *wall_area, int64_t *row_ptr, int32_t *col,
                float *facet_area, int64_t nnz_cap, int64_t *nnz_out) {
    if (!c || !vol || n <= 0) return LAGOT_EINVAL;
    const bool csr = row_ptr || col || facet_area;
    if (csr && !(row_ptr && col && facet_area && nnz_cap >= 0)) return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    c->tpc = c->tpc_default;
    c->ms_cell = 0.0;
    c->ms_crowd = 0.0;
    c->crowd_launches = 0;
    c->crowd_cells = 0;
    c->cell_launches = 0;
    c->ev_pending = false;
    c->ev_crowd_pending = false;
    const int64_t offs[2] = {0, n};
    int rc = prepare(c, 1, offs, x, y, z, psi, nullptr, &box, nullptr);
    if (rc) return rc;
    hipStream_t st = c->stream;
    launch_zero_i32(st, c->fb_inst, 1);
    evaluate(c, -1, c->psi_s, wall_area != nullptr, nullptr);
    launch_scatter_out_f64(st, n, c->perm, c->V, vol);
    if (sph_area) launch_scatter_out_f64(st, n, c->perm, c->K, sph_area);
    if (wall_area) launch_scatter_walls(st, n, wall_count(c), c->perm, c->wall, wall_area);
    HIP_TRY(hipMemcpyAsync(c->h_cnt, c->misc, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(c->h_cnt + 1, c->fail_inst, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (csr || nnz_out) {
        launch_csr_count(st, n, c->perm, c->fcnt, c->csr_cnt);
        launch_scan_i32(st, c->csr_cnt, c->csr_start, (int)n, c->csr_tmp);
        HIP_TRY(hipMemcpyAsync(c->h_cnt + 4, c->csr_start + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipMemcpyAsync(c->h_cnt + 9, c->misc + 4, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    rc = sync(c);
    if (rc) return rc;
    note_deferred(c, c->h_cnt[9]);
    c->last_fb = c->h_cnt[0];
    if (c->h_cnt[1] != 0) return LAGOT_ECAPACITY;
    if (csr || nnz_out) {
        const int64_t nnz = c->h_cnt[4];
        if (nnz_out) *nnz_out = nnz;
        if (csr) {
            if (nnz > nnz_cap) return LAGOT_ECAPACITY;
            launch_csr_fill(st, n, c->perm, c->fcol, c->farea, c->fcnt, c->csr_start, col, facet_area, row_ptr);
            HIP_TRY(hipStreamSynchronize(st));
        }
    }
    return LAGOT_OK;
}

int lagot_cells_paper_k(lagot_ctx *c, int64_t n, const float *x, const float *y, const float *z, const double *psi,
                        lagot_box box, double *vol, double *sph_area) {
    if (!c || !vol || !sph_area || n <= 0) return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    c->tpc = c->tpc_default;
    c->ms_cell = 0.0;
    c->ms_crowd = 0.0;
    c->crowd_launches = 0;
    c->crowd_cells = 0;
    c->cell_launches = 0;
    c->ev_pending = false;
    c->ev_crowd_pending = false;
    const int64_t offs[2] = {0, n};
    int rc = prepare(c, 1, offs, x, y, z, psi, nullptr, &box, nullptr);
    if (rc) return rc;
    hipStream_t st = c->stream;
    const Batch bt = batch(c);
    const EvalOut o = eval_out(c, false);
    launch_zero_i32(st, c->fb_inst, 1);
    launch_eval_begin(st, bt, -1, o);
    if (c->crowd) launch_local_reach(st, c->n, bt, -1, c->nc, c->pos_s, c->lr_rmc, c->lr_ir);
    (void)hipEventRecord(c->ev0, st);
    if (c->npieces > 0) {
        // a non-convex domain: the route in each convex piece, V and K summed over the pieces
        const PieceAcc acc = piece_acc(c);
        for (int k = 0; k < c->npieces; ++k) {
            Batch bk = bt;
            bk.dom = c->dom_d + c->h_dom_off[k];
            bk.ndom = c->h_dom_off[k + 1] - c->h_dom_off[k];
            bk.npieces = 0;
            launch_cells_kroute(st, n, bk, c->pos_s, c->psi_s, c->perm, c->cell_start, o, qboxes(c));
            launch_piece_accum(st, n, bt, -1, k == 0, o, bk.ndom, c->dom_wid_d + c->h_dom_off[k], c->nwalls,
                               c->perm, acc);
        }
        launch_piece_final(st, n, bt, -1, o, c->nwalls, c->perm, c->pos_s, nullptr, acc);
    } else {
        launch_cells_kroute(st, n, bt, c->pos_s, c->psi_s, c->perm, c->cell_start, o, qboxes(c));
    }
    (void)hipEventRecord(c->ev1, st);
    c->ev_pending = true;
    launch_scatter_out_f64(st, n, c->perm, c->V, vol);
    launch_scatter_out_f64(st, n, c->perm, c->K, sph_area);
    HIP_TRY(hipMemcpyAsync(c->h_cnt + 1, c->fail_inst, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    rc = sync(c);
    if (rc) return rc;
    return c->h_cnt[1] != 0 ? LAGOT_ECAPACITY : LAGOT_OK;
}

int lagot_newton_step(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const double *nu,
                      lagot_box box, double *psi_inout, const lagot_opts *opts, lagot_stats *stats) {
    if (!ctx || !psi_inout) return LAGOT_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return LAGOT_EHIP;
    return single_instance(ctx, n, x, y, z, nu, box, psi_inout, opts, stats, true);
}

int lagot_solve(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const double *nu,
                lagot_box box, double *psi_inout, const lagot_opts *opts, lagot_stats *stats) {
    if (!ctx || !psi_inout) return LAGOT_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return LAGOT_EHIP;
    return single_instance(ctx, n, x, y, z, nu, box, psi_inout, opts, stats, false);
}

int lagot_solve_moved(lagot_ctx *c, int64_t n, const float *x0, const float *y0, const float *z0, const float *x1,
                      const float *y1, const float *z1, const double *nu, lagot_box box, double *psi_inout,
                      const lagot_opts *opts, lagot_stats *stats) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (!c || !x0 || !y0 || !z0 || !x1 || !y1 || !z1 || !nu || !psi_inout || n <= 0) {
        if (stats) stats->status = LAGOT_EINVAL;
        return LAGOT_EINVAL;
    }
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    const double t_start = now_ms();
    lagot_opts o;
    if (opts)
        o = *opts;
    else
        fill_defaults(&o);
    int rc = check_opts(o);
    if (!rc && o.use_learned) rc = LAGOT_EINVAL;
    if (rc) {
        if (stats) stats->status = rc;
        return rc;
    }
    if (n > c->cap_mv) {
        free_ptrs(c->mv_buf, c->mv_pos);
        c->cap_mv = 0;
        HIP_TRY(dalloc(&c->mv_buf, 6 * (size_t)n));
        HIP_TRY(dalloc(&c->mv_pos, 6 * (size_t)n));
        c->cap_mv = n;
    }
    double *cen = c->mv_buf, *vol = cen + 3 * n, *psi_a = vol + n, *psi_b = psi_a + n;
    float *xa = c->mv_pos, *ya = xa + n, *za = ya + n, *xb = za + n, *yb = xb + n, *zb = yb + n;
    hipStream_t st = c->stream;
    HIP_TRY(hipMemcpyAsync(xa, x0, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(ya, y0, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(za, z0, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(psi_a, psi_inout, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    // Parts of the move: the weights of the last accepted positions are carried to the next
    // ones (centroids of their cells), and Algorithm 1 solves there, to stage_tol for a part
    // short of the end. A carried start with an empty cell (EEMPTY: the repair is off while
    // the move can still be split) or a part that does not converge halves the part.
    double tau = 0.0, dtau = 1.0;
    bool have_cen = false;
    int parts = 0, rc_last = LAGOT_OK;
    lagot_stats acc, S;
    std::memset(&acc, 0, sizeof(acc));
    constexpr double MIN_PART = 1.0 / 64.0;
    while (tau < 1.0) {
        const double t1 = std::min(1.0, tau + dtau);
        const bool last = t1 >= 1.0;
        if (!have_cen) {
            rc = lagot_centroids(c, n, xa, ya, za, psi_a, box, vol, cen);
            if (rc) break;
            acc.evals += 1;
            have_cen = true;
        }
        launch_lerp_sites(st, n, x0, y0, z0, x1, y1, z1, t1, xb, yb, zb);
        launch_carry_weights(st, n, xa, ya, za, xb, yb, zb, cen, psi_a, psi_b);
        lagot_opts op = o;
        op.empty_start_fallback = dtau <= MIN_PART ? o.empty_start_fallback : 0;
        if (!last) op.tol = std::max(o.tol, o.stage_tol);
        rc = single_instance(c, n, xb, yb, zb, nu, box, psi_b, &op, &S, false);
        acc.newton_iters += S.newton_iters;
        acc.evals += S.evals;
        acc.halvings += S.halvings;
        acc.cg_iters += S.cg_iters;
        acc.fallback_cells += S.fallback_cells;
        acc.cell_launches += S.cell_launches;
        acc.default_start |= S.default_start;
        acc.repaired_start |= S.repaired_start;
        acc.ms_eval += S.ms_eval;
        acc.ms_linear += S.ms_linear;
        acc.ms_cell_kernel += S.ms_cell_kernel;
        acc.failed_cells = S.failed_cells;
        acc.max_rel_err = S.max_rel_err;
        acc.grad_norm = S.grad_norm;
        rc_last = rc;
        if (o.verbose)
            fprintf(stderr, "lagot moved sites: part to %.4f (step %.4f): status %d, %d Newton iterations\n", t1, dtau,
                    rc, S.newton_iters);
        if (rc == LAGOT_OK) {
            ++parts;
            tau = t1;
            HIP_TRY(hipMemcpyAsync(psi_a, psi_b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            std::swap(xa, xb);
            std::swap(ya, yb);
            std::swap(za, zb);
            have_cen = false;
            dtau = std::min(2.0 * dtau, 1.0);
        } else if ((rc == LAGOT_EEMPTY || rc == LAGOT_ENOCONV || rc == LAGOT_ELINESEARCH || rc == LAGOT_ECAPACITY) &&
                   dtau > MIN_PART) {
            dtau *= 0.5;
        } else {
            break;
        }
    }
    if (tau >= 1.0) {
        rc = LAGOT_OK;
        HIP_TRY(hipMemcpyAsync(psi_inout, psi_a, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    } else if (!rc) {
        rc = rc_last ? rc_last : LAGOT_ENOCONV;
    }
    if (stats) {
        *stats = acc;
        stats->status = rc;
        stats->stages = parts;
        stats->ms_total = now_ms() - t_start;
    }
    return rc;
}

int lagot_solve_batched(lagot_ctx *ctx, int32_t n_inst, const int64_t *offsets, const float *x, const float *y,
                        const float *z, const double *nu, const lagot_box *boxes, double *psi_inout,
                        const lagot_opts *opts, lagot_stats *per_inst) {
    if (!ctx || !psi_inout || n_inst <= 0 || !offsets || !boxes) return LAGOT_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return LAGOT_EHIP;
    return newton_run(ctx, n_inst, offsets, x, y, z, nu, boxes, psi_inout, opts, per_inst, false);
}

int lagot_mlp_set_params(lagot_ctx *c, const float *params) {
    if (!c || !params) return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    int rc = ensure_mlp(c);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(c->mlp_p, params, sizeof(float) * MLP_NPARAMS, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(c->mlp_m1, 0, sizeof(float) * MLP_NPARAMS, c->stream));
    HIP_TRY(hipMemsetAsync(c->mlp_m2, 0, sizeof(float) * MLP_NPARAMS, c->stream));
    launch_to_bf16(c->stream, MLP_NPARAMS, c->mlp_p, c->mlp_pb);
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->mlp_t = 0;
    c->mlp_set = true;
    return LAGOT_OK;
}

int lagot_mlp_get_params(lagot_ctx *c, float *params) {
    if (!c || !params || !c->mlp_set) return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    HIP_TRY(hipMemcpyAsync(params, c->mlp_p, sizeof(float) * MLP_NPARAMS, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LAGOT_OK;
}

int lagot_features(lagot_ctx *c, int64_t n, const float *x, const float *y, const float *z, const double *psi_prev,
                   const double *nu, lagot_box box, int32_t *nbr, uint16_t *feats) {
    if (!c || !nu || (!nbr && !feats) || n <= 0) return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    c->tpc = c->tpc_default;
    c->ev_pending = false;
    c->ev_crowd_pending = false;
    const int64_t offs[2] = {0, n};
    int rc = prepare(c, 1, offs, x, y, z, psi_prev, nu, &box, nullptr);
    if (rc) return rc;
    launch_zero_i32(c->stream, c->fb_inst, 1);
    evaluate(c, -1, c->psi_s, false, nullptr);  // volumes under the previous weights are inputs too
    rc = build_features(c);
    if (rc) return rc;
    if (nbr) launch_scatter_rows(c->stream, n, N_NEI * 4, c->perm, c->nbr_s, nbr);
    if (feats) launch_scatter_rows(c->stream, n, MLP_IN * 2, c->perm, c->feat_s, feats);
    HIP_TRY(hipMemcpyAsync(c->h_cnt + 7, c->misc + 1, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    rc = sync(c);
    if (rc) return rc;
    return c->h_cnt[7] ? LAGOT_ECAPACITY : LAGOT_OK;
}

int lagot_mlp_forward(lagot_ctx *c, int64_t m, const uint16_t *feats, float *out) {
    if (!c || !feats || !out || m <= 0 || m > INT32_MAX / MLP_HID || !c->mlp_set) return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    int rc = ensure_inference(c, m);
    if (rc) return rc;
    mlp_forward_dev(c, (int)m, feats, c->inf_a, c->inf_b, out);
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LAGOT_OK;
}

int lagot_mlp_forward_noalloc(lagot_ctx *c, int64_t m, const uint16_t *feats, float *out) {
    if (!c || !feats || !out || m <= 0 || !c->mlp_set) return LAGOT_EINVAL;
    if (m > LAGOT_NOALLOC_MAX_ROWS) {
        fprintf(stderr, "lagot: lagot_mlp_forward_noalloc: %lld rows exceed its static buffers (%d rows)\n",
                (long long)m, LAGOT_NOALLOC_MAX_ROWS);
        return LAGOT_ECAPACITY;
    }
    if (hipSetDevice(c->device) != hipSuccess || !c->noalloc) return LAGOT_EHIP;
    // the two activation buffers: rows [0, m) of each half of the device's array
    uint16_t *a = c->noalloc;
    uint16_t *b = c->noalloc + (size_t)LAGOT_NOALLOC_MAX_ROWS * MLP_HID;
    mlp_forward_dev(c, (int)m, feats, a, b, out);
    HIP_TRY(hipGetLastError());
    return LAGOT_OK;
}

int lagot_mlp_train_step(lagot_ctx *c, int64_t nrows, const uint16_t *feats, const float *targets,
                         const int32_t *batch_idx, int32_t batch, float lr, float *loss) {
    if (!c || !feats || !targets || !batch_idx || batch <= 0 || nrows <= 0 || !c->mlp_set || !(lr > 0.f))
        return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    int rc = ensure_batch(c, batch);
    if (rc) return rc;
    hipStream_t st = c->stream;
    const int B = batch;
    float *P = c->mlp_p, *G = c->mlp_g;
    const uint16_t *PB = c->mlp_pb;
    launch_gather_rows(st, B, batch_idx, feats, targets, c->tX, c->tt);
    // forward, keeping pre-activations
    launch_gemm(st, false, false, MLP_EPI_BIAS_GELU, c->tX, PB + MLP_OFF_W1, B, MLP_HID, MLP_IN, c->tZ1, c->tH1,
                P + MLP_OFF_B1, nullptr);
    launch_gemm(st, false, false, MLP_EPI_BIAS_GELU, c->tH1, PB + MLP_OFF_W2, B, MLP_HID, MLP_HID, c->tZ2, c->tH2,
                P + MLP_OFF_B2, nullptr);
    launch_gemm(st, false, false, MLP_EPI_BIAS_GELU, c->tH2, PB + MLP_OFF_W3, B, MLP_HID, MLP_HID, c->tZ3, c->tH3,
                P + MLP_OFF_B3, nullptr);
    launch_out_layer(st, B, c->tH3, P + MLP_OFF_W4, P + MLP_OFF_B4, c->ty, c->tt, c->tdy, c->tloss);
    // backward
    launch_colsum(st, B, MLP_HID, nullptr, c->tH3, c->tdy, c->tpart, 4096, G + MLP_OFF_W4);
    launch_colsum(st, B, 1, c->tdy, nullptr, nullptr, c->tpart, 4096, G + MLP_OFF_B4);
    launch_out_back(st, B, c->tdy, P + MLP_OFF_W4, c->tZ3, c->tdZ, c->tdZb);
    launch_gemm(st, true, false, MLP_EPI_STORE, c->tH2, c->tdZb, MLP_HID, MLP_HID, B, G + MLP_OFF_W3, nullptr, nullptr,
                nullptr);
    launch_colsum(st, B, MLP_HID, c->tdZ, nullptr, nullptr, c->tpart, 4096, G + MLP_OFF_B3);
    launch_gemm(st, false, true, MLP_EPI_GELU_BACK, c->tdZb, PB + MLP_OFF_W3, B, MLP_HID, MLP_HID, c->tdZ, c->tdZb,
                nullptr, c->tZ2);
    launch_gemm(st, true, false, MLP_EPI_STORE, c->tH1, c->tdZb, MLP_HID, MLP_HID, B, G + MLP_OFF_W2, nullptr, nullptr,
                nullptr);
    launch_colsum(st, B, MLP_HID, c->tdZ, nullptr, nullptr, c->tpart, 4096, G + MLP_OFF_B2);
    launch_gemm(st, false, true, MLP_EPI_GELU_BACK, c->tdZb, PB + MLP_OFF_W2, B, MLP_HID, MLP_HID, c->tdZ, c->tdZb,
                nullptr, c->tZ1);
    launch_gemm(st, true, false, MLP_EPI_STORE, c->tX, c->tdZb, MLP_IN, MLP_HID, B, G + MLP_OFF_W1, nullptr, nullptr,
                nullptr);
    launch_colsum(st, B, MLP_HID, c->tdZ, nullptr, nullptr, c->tpart, 4096, G + MLP_OFF_B1);
    // Adam
    c->mlp_t++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)c->mlp_t), c2 = 1.f - powf(b2, (float)c->mlp_t);
    launch_adam(st, MLP_NPARAMS, P, G, c->mlp_m1, c->mlp_m2, lr, b1, b2, 1e-8f, c1, c2, c->mlp_pb);
    if (loss) {
        const int nlb = (B + 255) / 256;
        std::vector<float> h(nlb);
        HIP_TRY(hipMemcpyAsync(h.data(), c->tloss, sizeof(float) * nlb, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        double sum = 0.0;
        for (float v : h) sum += v;
        *loss = (float)(sum / B);
    }
    return LAGOT_OK;
}

int lagot_mlp_last_grads(lagot_ctx *c, float *grads) {
    if (!c || !grads || !c->mlp_set) return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    HIP_TRY(hipMemcpyAsync(grads, c->mlp_g, sizeof(float) * MLP_NPARAMS, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LAGOT_OK;
}

int lagot_set_threads_per_cell(lagot_ctx *ctx, int threads_per_cell) {
    if (!ctx || !valid_tpc(threads_per_cell)) return LAGOT_EINVAL;
    ctx->tpc_default = threads_per_cell;
    return LAGOT_OK;
}

int lagot_set_cg_shape(lagot_ctx *ctx, int lanes_per_row, int rows_per_block) {
    if (!ctx || !cg_shape_ok(lanes_per_row, rows_per_block)) return LAGOT_EINVAL;
    ctx->cg_lanes = ctx->cg_lanes_def = lanes_per_row;
    ctx->cg_sub = ctx->cg_sub_def = rows_per_block;
    return LAGOT_OK;
}

int lagot_set_cg_split(lagot_ctx *ctx, int mode) {
    if (!ctx || mode < 0 || mode > 2) return LAGOT_EINVAL;
    if (mode != ctx->cg_split) drop_graphs(ctx);  // captured chunks hold the other kernels
    ctx->cg_split = mode;
    return LAGOT_OK;
}

int lagot_last_fallback_cells(const lagot_ctx *ctx) { return ctx ? ctx->last_fb : -1; }

int lagot_last_pass_counts(lagot_ctx *ctx, int64_t *counts) {
    if (!ctx || !counts || ctx->n <= 0 || !ctx->misc) return LAGOT_EINVAL;
    int32_t m[5];
    HIP_TRY(hipMemcpyAsync(m, ctx->misc, sizeof(m), hipMemcpyDeviceToHost, ctx->stream));
    const int rc = sync(ctx);
    if (rc) return rc;
    counts[0] = m[4];
    counts[1] = m[0];
    counts[2] = ctx->eval_crowd ? 1 : 0;
    return LAGOT_OK;
}

// a wall buffer of at least w areas per site for the next calls
static int widen_walls(lagot_ctx *c, int w) {
    if (w <= c->wall_w) return LAGOT_OK;
    if (c->stream) HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->wall) (void)hipFree(c->wall);
    c->wall = nullptr;
    c->wall_w = w;
    if (c->cap_n > 0) HIP_TRY(dalloc(&c->wall, (size_t)w * (size_t)c->cap_n));
    return LAGOT_OK;
}

int lagot_set_domain(lagot_ctx *c, int nplanes, const double *planes) {
    if (!c || nplanes < 0 || nplanes > DOM_MAX || (nplanes > 0 && !planes)) return LAGOT_EINVAL;
    float4 h[DOM_MAX];
    for (int w = 0; w < nplanes; ++w) {
        const double *q = planes + 4 * w;
        const double len = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        if (!(std::fabs(len - 1.0) <= 1e-6) || !std::isfinite(q[3])) return LAGOT_EINVAL;
        h[w] = make_float4((float)q[0], (float)q[1], (float)q[2], (float)q[3]);
    }
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    if (!c->dom_d) HIP_TRY(dalloc(&c->dom_d, PIECE_PLANES_MAX));
    if (nplanes > 0) {
        HIP_TRY(hipMemcpyAsync(c->dom_d, h, sizeof(float4) * nplanes, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    const int rc = widen_walls(c, std::max(6, nplanes));
    if (rc) return rc;
    c->ndom = nplanes;
    c->npieces = 0;
    c->nwalls = 0;
    return LAGOT_OK;
}

int lagot_set_domain_pieces(lagot_ctx *c, int npieces, const int32_t *piece_off, const double *planes,
                            const int32_t *wall_id, int nwalls) {
    if (!c || npieces < 1 || npieces > PIECE_MAX || !piece_off || !planes || !wall_id) return LAGOT_EINVAL;
    if (nwalls < 1 || nwalls > PIECE_PLANES_MAX || piece_off[0] != 0) return LAGOT_EINVAL;
    int widest = 0;
    for (int k = 0; k < npieces; ++k) {
        const int m = piece_off[k + 1] - piece_off[k];
        if (m < 1 || m > DOM_MAX) return LAGOT_EINVAL;
        widest = std::max(widest, m);
    }
    const int total = piece_off[npieces];
    if (total > PIECE_PLANES_MAX) return LAGOT_EINVAL;
    float4 h[PIECE_PLANES_MAX];
    for (int w = 0; w < total; ++w) {
        const double *q = planes + 4 * w;
        const double len = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        if (!(std::fabs(len - 1.0) <= 1e-6) || !std::isfinite(q[3])) return LAGOT_EINVAL;
        if (wall_id[w] < -1 || wall_id[w] >= nwalls) return LAGOT_EINVAL;
        h[w] = make_float4((float)q[0], (float)q[1], (float)q[2], (float)q[3]);
    }
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    if (c->stream) HIP_TRY(hipStreamSynchronize(c->stream));
    if (!c->dom_d) HIP_TRY(dalloc(&c->dom_d, PIECE_PLANES_MAX));
    if (!c->dom_off_d) HIP_TRY(dalloc(&c->dom_off_d, PIECE_MAX + 1));
    if (!c->dom_wid_d) HIP_TRY(dalloc(&c->dom_wid_d, PIECE_PLANES_MAX));
    HIP_TRY(hipMemcpyAsync(c->dom_d, h, sizeof(float4) * total, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->dom_off_d, piece_off, sizeof(int32_t) * (npieces + 1), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->dom_wid_d, wall_id, sizeof(int32_t) * total, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const int rc = widen_walls(c, std::max(6, std::max(widest, nwalls)));
    if (rc) return rc;
    for (int k = 0; k <= npieces; ++k) c->h_dom_off[k] = piece_off[k];
    c->ndom = total;
    c->npieces = npieces;
    c->nwalls = nwalls;
    return LAGOT_OK;
}

int lagot_last_flag_counts(lagot_ctx *ctx, int64_t *counts) {
    if (!ctx || !counts || ctx->n <= 0 || !ctx->flags) return LAGOT_EINVAL;
    return flag_hist(ctx, counts);
}

double lagot_last_cell_kernel_ms(const lagot_ctx *ctx) { return ctx ? ctx->ms_cell : -1.0; }

int lagot_last_kernel_times(const lagot_ctx *ctx, double *out) {
    if (!ctx || !out) return LAGOT_EINVAL;
    out[0] = ctx->ms_cell;
    out[1] = ctx->cell_launches;
    out[2] = ctx->ms_crowd;
    out[3] = ctx->crowd_launches;
    out[4] = (double)ctx->crowd_cells;
    return LAGOT_OK;
}

int lagot_last_deferred(lagot_ctx *ctx, int32_t *idx, int64_t cap, int64_t *count) {
    if (!ctx || !count || (cap > 0 && !idx) || ctx->n <= 0 || !ctx->misc) return LAGOT_EINVAL;
    int32_t m = 0;
    HIP_TRY(hipMemcpyAsync(&m, ctx->misc + 4, sizeof(m), hipMemcpyDeviceToHost, ctx->stream));
    int rc = sync(ctx);
    if (rc) return rc;
    *count = m;
    const int64_t k = std::min<int64_t>(m, cap);
    if (k <= 0) return LAGOT_OK;
    std::vector<int32_t> rows((size_t)k), perm((size_t)ctx->n);
    HIP_TRY(hipMemcpyAsync(rows.data(), ctx->ovf_list, sizeof(int32_t) * (size_t)k, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipMemcpyAsync(perm.data(), ctx->perm, sizeof(int32_t) * (size_t)ctx->n, hipMemcpyDeviceToHost,
                           ctx->stream));
    rc = sync(ctx);
    if (rc) return rc;
    for (int64_t q = 0; q < k; ++q) idx[q] = perm[(size_t)rows[(size_t)q]];
    return LAGOT_OK;
}

void lagot_default_fluid_params(lagot_fluid_params *prm) {
    if (!prm) return;
    *prm = lagot_fluid_params{};
    prm->dt = 1e-3;
    prm->eps = 1.0;
    prm->gamma = 0.0;
    prm->mu = 0.0;
    prm->gravity[2] = -9.81;
    prm->cg_rtol = 1e-10;
    prm->cg_max_iter = 2000;
}

int lagot_p1_laplacian(lagot_ctx *c, int64_t n, const float *x, const float *y, const float *z, const double *psi,
                       lagot_box box, const double *mu, double mu0, const double *u, double *lap_u) {
    if (!c || !u || !lap_u || n <= 0) return LAGOT_EINVAL;
    if (!mu && !(mu0 >= 0.0 && std::isfinite(mu0))) return LAGOT_EINVAL;
    int rc = fluid_cells(c, n, x, y, z, psi, box, nullptr);
    if (rc) return rc;
    hipStream_t st = c->stream;
    launch_zero_i32(st, c->bad_inst, 1);
    launch_p1_laplacian(st, n, c->perm, c->hcol, c->hval, c->hcnt, mu, mu0, u, lap_u, c->bad_inst);
    HIP_TRY(hipMemcpyAsync(c->h_cnt, c->bad_inst, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    rc = sync(c);
    if (rc) return rc;
    return c->h_cnt[0] ? LAGOT_EINVAL : LAGOT_OK;
}

int lagot_fluid_velocity(lagot_ctx *c, int64_t n, const float *x, const float *y, const float *z,
                         const double *psi, lagot_box box, const double *mass, const double *mu, const double *v_in,
                         const lagot_fluid_params *prm, double *v_out, double *centroid, int32_t *cg_iters) {
    if (!c || !mass || !v_in || !prm || !v_out || n <= 0) return LAGOT_EINVAL;
    const lagot_fluid_params &p = *prm;
    if (!fluid_params_ok(p, mu != nullptr)) return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    const int nb3 = cg3_blocks(n);
    if (n > c->cap_fl) {
        free_ptrs(c->fl_buf, c->fl_int);
        c->cap_fl = 0;
        HIP_TRY(dalloc(&c->fl_buf, 32 * (size_t)n + 21 * (size_t)nb3 + 40));
        HIP_TRY(dalloc(&c->fl_int, 16));
        c->cap_fl = n;
    }
    // layout (doubles): records of the two slots [10n each], p [3n], x [3n], b [3n],
    // centroids [3n], partials [21 nb], step scalars [12], summed partials [24]; the records
    // come first (16-byte aligned)
    double *fb = c->fl_buf;
    Cg3Bufs g;
    g.rec[0] = reinterpret_cast<Rec3 *>(fb);
    g.rec[1] = reinterpret_cast<Rec3 *>(fb + 10 * n);
    g.p = fb + 20 * n;
    g.x = fb + 23 * n;
    double *b = fb + 26 * n;
    double *cen = centroid ? centroid : fb + 29 * n;
    g.part = fb + 32 * n;
    g.cgs = fb + 32 * n + 21 * (int64_t)nb3;
    g.sc = g.cgs + 12;
    g.st = c->fl_int;
    g.kbase = c->fl_int + 12;
    g.remaining = c->fl_int + 13;
    g.nb = nb3;
    int rc = fluid_cells(c, n, x, y, z, psi, box, cen);
    if (rc) return rc;
    hipStream_t st = c->stream;
    FluidPrm fp;
    fp.dt = p.dt;
    fp.inv_eps2 = 1.0 / (p.eps * p.eps);
    fp.gamma = p.gamma;
    fp.mu = p.mu;
    for (int a = 0; a < 3; ++a) fp.g[a] = p.gravity[a];
    launch_zero_i32(st, c->bad_inst, 1);
    launch_fluid_rows(st, n, c->perm, c->pos_s, c->hcol, c->hval, c->hcnt, mass, mu, fp, v_in, cen, c->diag, b,
                      c->bad_inst);
    // the scaled rows packed back to back for the PCG (row offsets: scan of the counts)
    int32_t *rp = c->csr_start;
    launch_scan_i32(st, c->hcnt, rp, (int)n, c->csr_tmp);
    HIP_TRY(hipMemcpyAsync(c->h_cnt, c->bad_inst, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(c->h_cnt + 1, rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    rc = sync(c);
    if (rc) return rc;
    if (c->h_cnt[0]) return LAGOT_EINVAL;
    const int64_t nnz = c->h_cnt[1];
    if (nnz > c->cap_ent) {
        free_ptrs(c->fl_ent);
        c->cap_ent = 0;
        HIP_TRY(dalloc(&c->fl_ent, (size_t)std::max<int64_t>(nnz, 1)));
        c->cap_ent = nnz;
    }
    launch_pack_rows(st, n, c->hcol, c->hval, c->hcnt, rp, c->fl_ent);
    // the three coordinates in one Jacobi-PCG (x_0 = 0, stop at ||r|| <= cg_rtol ||b||
    // per coordinate), in chunks of launches with a read-back of the count still iterating
    launch_cg3_init(st, n, rp, c->fl_ent, c->diag, b, g);
    launch_cg3_scalars(st, -1, p.cg_max_iter, g);
    const double rtol2 = p.cg_rtol * p.cg_rtol;
    const int cap = p.cg_max_iter;
    int k = 0;
    while (k < cap) {
        const int m = std::min(c->fl_chunk, cap - k);
        for (int q = 0; q < m; ++q) {
            launch_cg3_iter(st, n, q, rtol2, cap, rp, c->fl_ent, g);
            launch_cg3_scalars(st, q, cap, g);
        }
        launch_cg3_advance(st, m, cap, g);
        k += m;
        HIP_TRY(hipMemcpyAsync(c->h_cnt, c->fl_int, 14 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        rc = sync(c);
        if (rc) return rc;
        if (c->h_cnt[13] == 0) break;
    }
    launch_scatter3(st, n, c->perm, g.x, v_out);
    rc = sync(c);
    if (rc) return rc;
    int status = LAGOT_OK, most = 0;
    for (int q = 0; q < 3; ++q) {
        const int it = c->h_cnt[4 * q], brk = c->h_cnt[4 * q + 1], conv = c->h_cnt[4 * q + 2];
        if (cg_iters) cg_iters[q] = it;
        most = std::max(most, it);
        if (!conv && status == LAGOT_OK) status = brk ? LAGOT_ESINGULAR : LAGOT_ENOCONV;
    }
    // next call's chunk: this solve's iteration count and a margin, so that a like call
    // needs one read-back and few launches that find every coordinate done
    c->fl_chunk = std::min(256, std::max(8, (most + 4 + 3) / 4 * 4));
    return status;
}

int lagot_fluid_step(lagot_ctx *c, int64_t n, float *x, float *y, float *z, const double *nu, lagot_box box,
                     double *psi_inout, const double *mass, const double *mu, double *v_inout,
                     const lagot_fluid_params *prm, const lagot_opts *opts, lagot_stats *stats, int32_t *cg_iters) {
    if (!c || !x || !y || !z || !nu || !psi_inout || !mass || !v_inout || !prm || n <= 0) return LAGOT_EINVAL;
    if (!box_ok(box) || !fluid_params_ok(*prm, mu != nullptr)) return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    {
        // every input is checked before a site moves: options, prescribed volumes,
        // masses, velocities and viscosities
        lagot_opts o;
        if (opts)
            o = *opts;
        else
            fill_defaults(&o);
        if (check_opts(o) || o.use_learned) return LAGOT_EINVAL;
        launch_zero_i32(c->stream, c->misc + 6, 1);
        launch_fluid_check(c->stream, n, nu, mass, mu, v_inout, c->misc + 6);
        int32_t bad = 0;
        HIP_TRY(hipMemcpyAsync(&bad, c->misc + 6, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (bad) return LAGOT_EINVAL;
    }
    AdvectBounds bd;
    double ext = 0.0, big = 0.0;
    for (int a = 0; a < 3; ++a) {
        ext = std::max(ext, box.hi[a] - box.lo[a]);
        big = std::max(big, std::max(std::fabs(box.lo[a]), std::fabs(box.hi[a])));
    }
    // the margin also exceeds a few float32 ulps of the bounds, so that the rounding of a
    // clamped coordinate to float32 keeps it strictly inside
    const double ulps = 4.0 * ulp32(big);
    for (int a = 0; a < 3; ++a) {
        const double m = std::max(ADVECT_MARGIN * (box.hi[a] - box.lo[a]), ulps);
        bd.lo[a] = box.lo[a] + m;
        bd.hi[a] = box.hi[a] - m;
    }
    bd.plane_margin = std::max(ADVECT_MARGIN * ext, ulps);
    launch_advect(c->stream, n, x, y, z, v_inout, prm->dt, bd, c->dom_d, c->ndom, c->dom_off_d, c->npieces);
    int rc = single_instance(c, n, x, y, z, nu, box, psi_inout, opts, stats, false);
    if (rc) return rc;
    c->fl_reuse = true;
    rc = lagot_fluid_velocity(c, n, x, y, z, psi_inout, box, mass, mu, v_inout, prm, v_inout, nullptr, cg_iters);
    c->fl_reuse = false;
    return rc;
}

const char *lagot_strerror(int code) {
    switch (code) {
        case LAGOT_OK: return "ok";
        case LAGOT_EINVAL: return "invalid argument";
        case LAGOT_EEMPTY: return "a start cell is empty";
        case LAGOT_ENOCONV: return "Newton iteration limit reached";
        case LAGOT_ELINESEARCH: return "step halving limit reached";
        case LAGOT_ECAPACITY: return "capacity exceeded";
        case LAGOT_ESINGULAR: return "conjugate-gradient breakdown";
        case LAGOT_EHIP: return "HIP runtime error";
        default: return "unknown error";
    }
}

}  // extern "C"
