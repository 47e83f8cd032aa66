// api.cpp -- C-ABI of liblagot (declared in include/lagot.h): context and
// workspace management, input validation, the spatial sort, one evaluation of
// all cells, and the host side of the damped Newton loop of Algorithm 1 (KMT
// step control) around the Jacobi-PCG direction solve.
//
// Everything between the caller's arrays runs in grid order on the device; the
// host only reads a few float64 scalars per evaluation / PCG chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lagot.h"
#include "lagot_internal.h"

using namespace lagot;

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
    int tpc = 32;
    int tpc_default = 32;  // lanes per cell when the options leave it to the library

    // sites (caller order, then grid order)
    float4 *pos_orig = nullptr, *pos_s = nullptr;
    double *psi_s = nullptr, *nu_s = nullptr, *psi_trial = nullptr;
    int32_t *keys = nullptr, *perm = nullptr;
    int32_t *cell_count = nullptr, *cell_start = nullptr, *cursor = nullptr, *scan_tmp = nullptr;
    GridDesc grid{};
    // evaluation outputs (grid order)
    double *V = nullptr, *K = nullptr;
    float *wall = nullptr;
    int32_t *fcol = nullptr, *fcnt = nullptr, *fb_list = nullptr;
    float *farea = nullptr;
    uint32_t *flags = nullptr;
    int32_t *counters = nullptr;  // [0] fallback count [1] fail count [2] bad inputs [3] hessian overflow
    // Hessian and PCG
    int32_t *hcol = nullptr, *hcnt = nullptr, *xcnt = nullptr;
    float *hval = nullptr;
    double *diag = nullptr, *g = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    double *p2 = nullptr;
    double *partial = nullptr, *scal = nullptr, *red4 = nullptr, *rmax = nullptr, *rmax_partial = nullptr;
    int cap_blocks = 0;
    // pinned host mirrors
    double *h_scal = nullptr;
    int32_t *h_cnt = nullptr;
    // CSR staging for lagot_cells
    int32_t *csr_cnt = nullptr, *csr_start = nullptr;
    int64_t *csr_start64 = nullptr;
    int32_t *csr_tmp = nullptr;
    // statistics of the current call
    int fb_total = 0;
    int last_fb = 0;
    // learned warm start: float32 master parameters, bf16 copy, Adam moments
    float *mlp_p = nullptr, *mlp_g = nullptr, *mlp_m1 = nullptr, *mlp_m2 = nullptr;
    uint16_t *mlp_pb = nullptr;
    int mlp_t = 0;
    bool mlp_set = false;
    double *nusum = nullptr;
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
    bool ev_pending = false;
    double ms_cell = 0.0;
    int cell_launches = 0;
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

void free_all(lagot_ctx *c) {
    void *bufs[] = {c->pos_orig, c->pos_s, c->psi_s, c->nu_s, c->psi_trial, c->keys, c->perm, c->cell_count,
                    c->cell_start, c->cursor, c->scan_tmp, c->V, c->K, c->wall, c->fcol, c->fcnt, c->fb_list,
                    c->farea, c->flags, c->counters, c->hcol, c->hcnt, c->xcnt, c->hval, c->diag, c->g, c->x,
                    c->r, c->z, c->p, c->q, c->partial, c->scal, c->red4, c->rmax, c->rmax_partial, c->csr_cnt,
                    c->csr_start, c->csr_start64, c->csr_tmp, c->p2};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (c->h_scal) (void)hipHostFree(c->h_scal);
    if (c->h_cnt) (void)hipHostFree(c->h_cnt);
    void *mbufs[] = {c->mlp_p, c->mlp_g, c->mlp_m1, c->mlp_m2, c->mlp_pb, c->nusum, c->nbr_s, c->feat_s, c->inf_a,
                     c->inf_b, c->mlp_out, c->tX, c->tH1, c->tH2, c->tH3, c->tdZb, c->tZ1, c->tZ2, c->tZ3, c->tdZ,
                     c->ty, c->tt, c->tdy, c->tpart, c->tloss};
    for (void *b : mbufs)
        if (b) (void)hipFree(b);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
}

// Add the duration of the last recorded cell-kernel launch (call after a stream sync).
void collect_cell_time(lagot_ctx *c) {
    if (!c->ev_pending) return;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) {
        c->ms_cell += ms;
        c->cell_launches++;
    }
    c->ev_pending = false;
}

int nblk256(int64_t n) { return (int)((n + 255) / 256); }

int ensure_sites(lagot_ctx *c, int64_t n) {
    if (n <= c->cap_n) return LAGOT_OK;
    void *bufs[] = {c->pos_orig, c->pos_s, c->psi_s, c->nu_s, c->psi_trial, c->keys, c->perm, c->V, c->K, c->wall,
                    c->fcol, c->fcnt, c->fb_list, c->farea, c->flags, c->hcol, c->hcnt, c->xcnt, c->hval, c->diag,
                    c->g, c->x, c->r, c->z, c->p, c->q, c->partial, c->rmax_partial, c->csr_cnt, c->csr_start,
                    c->csr_start64, c->csr_tmp, c->p2};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    const size_t N = (size_t)n;
    const int nb = nblk256(n);
    HIP_TRY(dalloc(&c->pos_orig, N));
    HIP_TRY(dalloc(&c->pos_s, N));
    HIP_TRY(dalloc(&c->psi_s, N));
    HIP_TRY(dalloc(&c->nu_s, N));
    HIP_TRY(dalloc(&c->psi_trial, N));
    HIP_TRY(dalloc(&c->keys, N));
    HIP_TRY(dalloc(&c->perm, N));
    HIP_TRY(dalloc(&c->V, N));
    HIP_TRY(dalloc(&c->K, N));
    HIP_TRY(dalloc(&c->wall, 6 * N));
    HIP_TRY(dalloc(&c->fcol, FCAP * N));
    HIP_TRY(dalloc(&c->farea, FCAP * N));
    HIP_TRY(dalloc(&c->fcnt, N));
    HIP_TRY(dalloc(&c->fb_list, N));
    HIP_TRY(dalloc(&c->flags, N));
    HIP_TRY(dalloc(&c->hcol, FCAP * N));
    HIP_TRY(dalloc(&c->hval, FCAP * N));
    HIP_TRY(dalloc(&c->hcnt, N));
    HIP_TRY(dalloc(&c->xcnt, N));
    HIP_TRY(dalloc(&c->diag, N));
    HIP_TRY(dalloc(&c->g, N));
    HIP_TRY(dalloc(&c->x, N));
    HIP_TRY(dalloc(&c->r, N));
    HIP_TRY(dalloc(&c->z, N));
    HIP_TRY(dalloc(&c->p, N));
    HIP_TRY(dalloc(&c->q, N));
    HIP_TRY(dalloc(&c->p2, N));
    HIP_TRY(dalloc(&c->partial, std::max<size_t>(4 * (size_t)nb, 5 * 512 + (size_t)spmv_blocks(n) + 64)));
    HIP_TRY(dalloc(&c->rmax_partial, (size_t)nb));
    HIP_TRY(dalloc(&c->csr_cnt, N + 1));
    HIP_TRY(dalloc(&c->csr_start, N + 1));
    HIP_TRY(dalloc(&c->csr_start64, N + 1));
    HIP_TRY(dalloc(&c->csr_tmp, N / 1024 + 16));
    c->cap_n = n;
    c->cap_blocks = nb;
    return LAGOT_OK;
}

int ensure_cells(lagot_ctx *c, int ncell) {
    if (ncell <= c->cap_cells) return LAGOT_OK;
    void *bufs[] = {c->cell_count, c->cell_start, c->cursor, c->scan_tmp};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    HIP_TRY(dalloc(&c->cell_count, (size_t)ncell + 1));
    HIP_TRY(dalloc(&c->cell_start, (size_t)ncell + 1));
    HIP_TRY(dalloc(&c->cursor, (size_t)ncell + 1));
    HIP_TRY(dalloc(&c->scan_tmp, (size_t)ncell / 1024 + 16));
    c->cap_cells = ncell;
    return LAGOT_OK;
}

BoxF to_boxf(const lagot_box &b) {
    BoxF f;
    for (int a = 0; a < 3; ++a) {
        f.lo[a] = (float)b.lo[a];
        f.hi[a] = (float)b.hi[a];
    }
    return f;
}

bool box_ok(const lagot_box &b) {
    for (int a = 0; a < 3; ++a)
        if (!(b.hi[a] > b.lo[a]) || !std::isfinite(b.lo[a]) || !std::isfinite(b.hi[a])) return false;
    return true;
}

int sync_read(lagot_ctx *c, const void *dev, void *host, size_t bytes) {
    HIP_TRY(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LAGOT_OK;
}

// Validate, gather, spatially sort. nu may be null (cells-only). On return the
// grid-order arrays pos_s (with float32 psi), psi_s (and nu_s) are filled and
// c->rmax holds max sqrt(psi).
int prepare(lagot_ctx *c, int64_t n, const float *x, const float *y, const float *z, const double *psi,
            const double *nu, const lagot_box &box) {
    if (n <= 0 || n > (int64_t)INT32_MAX / FCAP || !x || !y || !z || !psi || !box_ok(box)) return LAGOT_EINVAL;
    int rc = ensure_sites(c, n);
    if (rc) return rc;
    const BoxF bf = to_boxf(box);
    HIP_TRY(hipMemsetAsync(c->counters, 0, 8 * sizeof(int32_t), c->stream));
    launch_validate(c->stream, n, x, y, z, psi, nu, bf, c->counters + 2);
    const int nb = nblk256(n);
    launch_gather_sites(c->stream, n, x, y, z, psi, c->pos_orig, c->rmax_partial, nb);
    launch_reduce_max(c->stream, c->rmax_partial, nb, c->rmax);
    HIP_TRY(hipMemcpyAsync(c->h_scal, c->rmax, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->h_cnt, c->counters, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->h_cnt[2] != 0) return LAGOT_EINVAL;
    const double rmax = c->h_scal[0];
    // grid cell size: 2 r_max (the 3x3x3 neighbourhood then covers every bisector
    // that can cut a ball), but at most 512 cells per axis and 2^24 cells in all
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = std::max(ext, box.hi[a] - box.lo[a]);
    double s = std::max(2.0 * rmax, ext / 512.0);
    int dim[3];
    for (;;) {
        int64_t tot = 1;
        for (int a = 0; a < 3; ++a) {
            dim[a] = std::max(1, (int)std::ceil((box.hi[a] - box.lo[a]) / s));
            tot *= dim[a];
        }
        if (tot <= (1 << 24)) break;
        s *= 1.25;
    }
    GridDesc g;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = (float)box.lo[a];
        g.dim[a] = dim[a];
    }
    g.s = (float)s;
    g.inv_s = (float)(1.0 / s);
    g.ncell = dim[0] * dim[1] * dim[2];
    c->grid = g;
    rc = ensure_cells(c, g.ncell);
    if (rc) return rc;
    launch_grid_build(c->stream, n, c->pos_orig, g, c->keys, c->cell_count, c->cell_start, c->scan_tmp, c->perm,
                      c->cursor);
    launch_permute_in(c->stream, n, c->perm, c->pos_orig, psi, nu, c->pos_s, c->psi_s, nu ? c->nu_s : nullptr);
    return LAGOT_OK;
}

// One evaluation of all cells at the float64 weights psi_eval (grid order), whose
// float32 shadow is pos_s.w (r_max on device).
void evaluate(lagot_ctx *c, int64_t n, const lagot_box &box, bool walls, const double *psi_eval) {
    const BoxF bf = to_boxf(box);
    (void)hipMemsetAsync(c->counters, 0, 2 * sizeof(int32_t), c->stream);
    if (walls) (void)hipMemsetAsync(c->wall, 0, 6 * sizeof(float) * (size_t)n, c->stream);
    EvalOut o{c->V, c->K, walls ? c->wall : nullptr, c->fcol, c->farea, c->fcnt, c->flags, c->fb_list,
              c->counters + 0, c->counters + 1};
    (void)hipEventRecord(c->ev0, c->stream);
    launch_cells(c->stream, n, c->pos_s, psi_eval, c->perm, c->cell_start, c->grid, bf, c->rmax, o, c->tpc);
    (void)hipEventRecord(c->ev1, c->stream);
    c->ev_pending = true;
    launch_cells_fallback(c->stream, n, c->pos_s, psi_eval, c->perm, c->cell_start, c->grid, bf, c->rmax, o);
}

struct EvalStats {
    double sumV, maxrel, gnorm, minV;
    int fb, fail;
};

int evaluate_reduce(lagot_ctx *c, int64_t n, const lagot_box &box, EvalStats *es, const double *psi_eval) {
    evaluate(c, n, box, false, psi_eval);
    const int nb = nblk256(n);
    launch_eval_reduce(c->stream, n, c->V, c->nu_s, c->partial, nb, c->red4);
    HIP_TRY(hipMemcpyAsync(c->h_scal, c->red4, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->h_cnt, c->counters, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    collect_cell_time(c);
    es->sumV = c->h_scal[0];
    es->maxrel = c->h_scal[1];
    es->gnorm = c->h_scal[2];
    es->minV = c->h_scal[3];
    es->fb = c->h_cnt[0];
    es->fail = c->h_cnt[1];
    c->fb_total += es->fb;
    return LAGOT_OK;
}

// Newton direction: assemble -Hess K, Jacobi-PCG for (-Hess K) u = nu - V, u in c->x.
// Iterations are enqueued in chunks without host syncs; the kernels of a chunk
// turn into no-ops once the residual meets the tolerance (device-side test).
int newton_direction(lagot_ctx *c, int64_t n, const lagot_opts &o, int *cg_iters) {
    HIP_TRY(hipMemsetAsync(c->counters + 3, 0, sizeof(int32_t), c->stream));
    launch_hess_assemble(c->stream, n, c->pos_s, c->psi_s, c->K, c->fcol, c->farea, c->fcnt, c->hcol, c->hval,
                         c->xcnt, c->diag, c->counters + 3);
    launch_hess_finish(c->stream, n, c->psi_s, c->K, c->fcnt, c->xcnt, c->hcnt, c->hval, c->diag);
    const int nb = pcg_blocks(n);
    double *RZ = c->partial, *RR = c->partial + 2 * nb, *R0 = c->partial + 4 * nb, *PQ = c->partial + 5 * nb;
    // PQ holds one partial per SpMV block
    int32_t *state = c->counters + 4;
    const double rtol2 = o.cg_rtol * o.cg_rtol;
    launch_pcg_init(c->stream, n, nb, c->V, c->nu_s, c->diag, c->g, c->x, c->r, c->z, RZ, RR, R0, state);
    *cg_iters = 0;
    double *pb[2] = {c->p, c->p2};
    const int chunk = 16;
    int k = 0;
    for (;;) {
        for (int m = 0; m < chunk && k < o.cg_max_iter; ++m, ++k) {
            launch_pcg_spmv(c->stream, n, k, nb, rtol2, R0, c->hcol, c->hval, c->hcnt, c->diag, c->z,
                            pb[(k + 1) & 1], pb[k & 1], c->q, RZ, RR, PQ, state);
            launch_pcg_update(c->stream, n, k, nb, rtol2, R0, c->diag, c->x, c->r, c->z, pb[k & 1], c->q, RZ, RR,
                              PQ, state);
        }
        HIP_TRY(hipMemcpyAsync(c->h_cnt + 3, c->counters + 3, 4 * sizeof(int32_t), hipMemcpyDeviceToHost,
                               c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (c->h_cnt[3] != 0) return LAGOT_ECAPACITY;
        const int done_iters = c->h_cnt[4], breakdown = c->h_cnt[5], converged = c->h_cnt[6];
        *cg_iters = done_iters;
        if (breakdown) {
            // non-positive curvature before the tolerance was met
            launch_pcg_status(c->stream, nb, RR, R0, state, c->scal);
            int rc = sync_read(c, c->scal, c->h_scal, 2 * sizeof(double));
            if (rc) return rc;
            if (!(c->h_scal[0] <= rtol2 * c->h_scal[1])) return LAGOT_ESINGULAR;
            break;
        }
        if (converged || done_iters < k || k >= o.cg_max_iter) break;
    }
    return LAGOT_OK;  // at the iteration cap the direction is inexact; the step control still guards it
}

// ---- learned warm start ------------------------------------------------------
int ensure_mlp(lagot_ctx *c) {
    if (c->mlp_p) return LAGOT_OK;
    HIP_TRY(dalloc(&c->mlp_p, MLP_NPARAMS));
    HIP_TRY(dalloc(&c->mlp_g, MLP_NPARAMS));
    HIP_TRY(dalloc(&c->mlp_m1, MLP_NPARAMS));
    HIP_TRY(dalloc(&c->mlp_m2, MLP_NPARAMS));
    HIP_TRY(dalloc(&c->mlp_pb, MLP_NPARAMS));
    if (!c->nusum) HIP_TRY(dalloc(&c->nusum, 1));
    return LAGOT_OK;
}

int ensure_inference(lagot_ctx *c, int64_t n) {
    if (!c->nusum) HIP_TRY(dalloc(&c->nusum, 1));
    if (n <= c->cap_inf) return LAGOT_OK;
    void *bufs[] = {c->nbr_s, c->feat_s, c->inf_a, c->inf_b, c->mlp_out};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
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
    void *bufs[] = {c->tX, c->tH1, c->tH2, c->tH3, c->tdZb, c->tZ1, c->tZ2, c->tZ3, c->tdZ, c->ty, c->tt, c->tdy,
                    c->tpart, c->tloss};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
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

// Inputs of every site in grid order (needs prepare() with psi = psi_prev and nu, and
// the cell volumes at psi_prev in c->V).
int build_features(lagot_ctx *c, int64_t n) {
    int rc = ensure_inference(c, n);
    if (rc) return rc;
    const int nb = nblk256(n);
    launch_eval_reduce(c->stream, n, c->nu_s, c->nu_s, c->partial, nb, c->red4);
    HIP_TRY(hipMemcpyAsync(c->nusum, c->red4, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(c->counters + 7, 0, sizeof(int32_t), c->stream));
    launch_knn_features(c->stream, n, c->pos_s, c->perm, c->cell_start, c->grid, c->psi_s, c->nu_s, c->nusum, c->V,
                        c->nbr_s, c->feat_s, c->counters + 7);
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
}

bool valid_tpc(int t) { return t == 8 || t == 16 || t == 32 || t == 64; }

int check_opts(const lagot_opts &o) {
    if (!(o.tol > 0) || o.max_newton < 0 || o.max_halvings < 0 || !(o.cg_rtol > 0) || o.cg_max_iter < 1)
        return LAGOT_EINVAL;
    if (!valid_tpc(o.threads_per_cell) && o.threads_per_cell != 0) return LAGOT_EINVAL;
    return LAGOT_OK;
}

// Damped Newton (Algorithm 1, KMT step control); max_iters = 1 for a single step.
int newton_run(lagot_ctx *c, int64_t n, const float *x, const float *y, const float *z, const double *nu,
               const lagot_box &box, double *psi, const lagot_opts *opts_in, lagot_stats *st, bool single) {
    const double t0 = now_ms();
    lagot_stats S;
    std::memset(&S, 0, sizeof(S));
    lagot_opts o;
    if (opts_in)
        o = *opts_in;
    else
        fill_defaults(&o);
    int rc = check_opts(o);
    if (!rc && !nu) rc = LAGOT_EINVAL;
    if (!rc) {
        c->tpc = o.threads_per_cell ? o.threads_per_cell : c->tpc_default;
        c->fb_total = 0;
        c->ms_cell = 0.0;
        c->cell_launches = 0;
        rc = prepare(c, n, x, y, z, psi, nu, box);
    }
    double ms_eval = 0, ms_lin = 0;
    if (!rc) {
        // total prescribed volume must leave room for air: sum nu < |box|
        const int nb = nblk256(n);
        launch_eval_reduce(c->stream, n, c->nu_s, c->nu_s, c->partial, nb, c->red4);
        rc = sync_read(c, c->red4, c->h_scal, 4 * sizeof(double));
        const double box_vol = (box.hi[0] - box.lo[0]) * (box.hi[1] - box.lo[1]) * (box.hi[2] - box.lo[2]);
        const double sum_nu = c->h_scal[0], min_nu = c->h_scal[3];
        if (!rc && !(sum_nu < box_vol)) rc = LAGOT_EINVAL;
        EvalStats es{};
        if (!rc) {
            const double te = now_ms();
            rc = evaluate_reduce(c, n, box, &es, c->psi_s);
            ms_eval += now_ms() - te;
            S.evals = 1;
        }
        // learned warm start: accepted only if every cell keeps volume and ||nu - V|| drops
        if (!rc && !single && o.use_learned && c->mlp_set && es.fail == 0) {
            const double tg = now_ms();
            rc = build_features(c, n);
            if (!rc) {
                mlp_forward_dev(c, (int)n, c->feat_s, c->inf_a, c->inf_b, c->mlp_out);
                launch_apply_guess(c->stream, n, c->psi_s, c->nu_s, c->mlp_out, c->psi_trial, c->pos_s,
                                   c->rmax_partial);
                launch_reduce_max(c->stream, c->rmax_partial, nblk256(n), c->rmax);
                EvalStats eg{};
                rc = evaluate_reduce(c, n, box, &eg, c->psi_trial);
                S.evals++;
                if (!rc && eg.fail == 0 && eg.minV > 0.0 && eg.gnorm < es.gnorm) {
                    std::swap(c->psi_s, c->psi_trial);
                    es = eg;
                    S.learned_accepted = 1;
                } else if (!rc) {
                    launch_psi_shadow(c->stream, n, c->psi_s, c->pos_s);
                    launch_gather_rmax(c->stream, n, c->psi_s, c->rmax_partial);
                    launch_reduce_max(c->stream, c->rmax_partial, nblk256(n), c->rmax);
                }
            }
            S.ms_learned = now_ms() - tg;
        }
        // a start with an empty cell (eps0 = 0) is replaced by the default start weights
        if (!rc && !(es.minV > 0.0) && o.empty_start_fallback) {
            launch_default_start(c->stream, n, c->nu_s, c->psi_s, c->pos_s, c->rmax_partial);
            launch_reduce_max(c->stream, c->rmax_partial, nblk256(n), c->rmax);
            rc = evaluate_reduce(c, n, box, &es, c->psi_s);
            S.evals++;
            S.default_start = 1;
        }
        double eps0 = 0.5 * std::min(min_nu, es.minV);
        if (!rc && !(eps0 > 0.0)) rc = LAGOT_EEMPTY;
        if (!rc && es.fail) rc = LAGOT_ECAPACITY;
        int it = 0;
        while (!rc) {
            S.max_rel_err = es.maxrel;
            S.grad_norm = es.gnorm;
            if (o.verbose)
                fprintf(stderr, "lagot newton it=%d max_rel_err=%.3e |g|=%.3e minV=%.3e fallback=%d\n", it,
                        es.maxrel, es.gnorm, es.minV, es.fb);
            if (es.maxrel <= o.tol) break;
            if (it >= o.max_newton || (single && it >= 1)) {
                rc = single ? LAGOT_OK : LAGOT_ENOCONV;
                break;
            }
            const double tl = now_ms();
            int cgi = 0;
            rc = newton_direction(c, n, o, &cgi);
            ms_lin += now_ms() - tl;
            S.cg_iters += cgi;
            if (rc) break;
            double alpha = 1.0;
            bool accepted = false;
            EvalStats et{};
            for (int h = 0; h <= o.max_halvings; ++h) {
                const int nb2 = nblk256(n);
                launch_axpy_trial(c->stream, n, c->psi_s, c->x, alpha, c->psi_trial, c->pos_s, c->rmax_partial);
                launch_reduce_max(c->stream, c->rmax_partial, nb2, c->rmax);
                const double te = now_ms();
                rc = evaluate_reduce(c, n, box, &et, c->psi_trial);
                ms_eval += now_ms() - te;
                S.evals++;
                if (rc) break;
                if (et.fail == 0 && et.minV >= eps0 && et.gnorm <= (1.0 - 0.5 * alpha) * es.gnorm) {
                    accepted = true;
                    break;
                }
                alpha *= 0.5;
                S.halvings++;
            }
            if (rc) break;
            if (!accepted) {
                // restore the float32 shadow and r_max of the last accepted weights
                launch_psi_shadow(c->stream, n, c->psi_s, c->pos_s);
                launch_gather_rmax(c->stream, n, c->psi_s, c->rmax_partial);
                launch_reduce_max(c->stream, c->rmax_partial, nblk256(n), c->rmax);
                rc = et.fail ? LAGOT_ECAPACITY : LAGOT_ELINESEARCH;
                break;
            }
            std::swap(c->psi_s, c->psi_trial);
            es = et;
            ++it;
            S.newton_iters = it;
        }
        S.max_rel_err = es.maxrel;
        S.grad_norm = es.gnorm;
        if (rc != LAGOT_EINVAL && rc != LAGOT_EHIP) {
            launch_scatter_out_f64(c->stream, n, c->perm, c->psi_s, psi);
            if (hipStreamSynchronize(c->stream) != hipSuccess) rc = LAGOT_EHIP;
        }
    }
    S.fallback_cells = c->fb_total;
    S.cell_launches = c->cell_launches;
    S.ms_cell_kernel = c->ms_cell;
    S.status = rc;
    S.ms_eval = ms_eval;
    S.ms_linear = ms_lin;
    S.ms_total = now_ms() - t0;
    if (st) *st = S;
    return rc;
}

}  // namespace

extern "C" {

void lagot_default_opts(lagot_opts *opts) {
    if (opts) fill_defaults(opts);
}

int lagot_create(lagot_ctx **out, int device, void *stream) {
    if (!out) return LAGOT_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LAGOT_EHIP;
    if (hipSetDevice(device) != hipSuccess) return LAGOT_EHIP;
    lagot_ctx *c = new lagot_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    if (dalloc(&c->counters, 8) != hipSuccess || dalloc(&c->scal, 16) != hipSuccess ||
        dalloc(&c->red4, 4) != hipSuccess || dalloc(&c->rmax, 1) != hipSuccess ||
        hipHostMalloc((void **)&c->h_scal, 16 * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&c->h_cnt, 16 * sizeof(int32_t)) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
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

int lagot_cells(lagot_ctx *c, int64_t n, const float *x, const float *y, const float *z, const double *psi,
                lagot_box box, double *vol, double *sph_area, float *wall_area, int64_t *row_ptr, int32_t *col,
                float *facet_area, int64_t nnz_cap, int64_t *nnz_out) {
    if (!c || !vol) return LAGOT_EINVAL;
    const bool csr = row_ptr || col || facet_area;
    if (csr && !(row_ptr && col && facet_area && nnz_cap >= 0)) return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    c->fb_total = 0;
    c->tpc = c->tpc_default;
    int rc = prepare(c, n, x, y, z, psi, nullptr, box);
    if (rc) return rc;
    evaluate(c, n, box, wall_area != nullptr, c->psi_s);
    launch_scatter_out_f64(c->stream, n, c->perm, c->V, vol);
    if (sph_area) launch_scatter_out_f64(c->stream, n, c->perm, c->K, sph_area);
    if (wall_area) launch_scatter_walls(c->stream, n, c->perm, c->wall, wall_area);
    HIP_TRY(hipMemcpyAsync(c->h_cnt, c->counters, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    if (csr || nnz_out) {
        launch_csr_count(c->stream, n, c->perm, c->fcnt, c->csr_cnt);
        launch_scan_i32(c->stream, c->csr_cnt, c->csr_start, (int)n, c->csr_tmp);
        HIP_TRY(hipMemcpyAsync(c->h_cnt + 4, c->csr_start + n, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->ms_cell = 0.0;
    c->cell_launches = 0;
    collect_cell_time(c);
    c->last_fb = c->h_cnt[0];
    if (c->h_cnt[1] != 0) return LAGOT_ECAPACITY;
    if (csr || nnz_out) {
        const int64_t nnz = c->h_cnt[4];
        if (nnz_out) *nnz_out = nnz;
        if (csr) {
            if (nnz > nnz_cap) return LAGOT_ECAPACITY;
            launch_csr_fill(c->stream, n, c->perm, c->fcol, c->farea, c->fcnt, c->csr_start, col, facet_area,
                            row_ptr);
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
    }
    return LAGOT_OK;
}

int lagot_newton_step(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const double *nu,
                      lagot_box box, double *psi_inout, const lagot_opts *opts, lagot_stats *stats) {
    if (!ctx || !psi_inout) return LAGOT_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return LAGOT_EHIP;
    return newton_run(ctx, n, x, y, z, nu, box, psi_inout, opts, stats, true);
}

int lagot_solve(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const double *nu,
                lagot_box box, double *psi_inout, const lagot_opts *opts, lagot_stats *stats) {
    if (!ctx || !psi_inout) return LAGOT_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return LAGOT_EHIP;
    return newton_run(ctx, n, x, y, z, nu, box, psi_inout, opts, stats, false);
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
    if (!c || !nu || (!nbr && !feats)) return LAGOT_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAGOT_EHIP;
    int rc = prepare(c, n, x, y, z, psi_prev, nu, box);
    if (rc) return rc;
    evaluate(c, n, box, false, c->psi_s);  // volumes under the previous weights are inputs too
    rc = build_features(c, n);
    if (rc) return rc;
    if (nbr) launch_scatter_rows(c->stream, n, N_NEI * 4, c->perm, c->nbr_s, nbr);
    if (feats) launch_scatter_rows(c->stream, n, MLP_IN * 2, c->perm, c->feat_s, feats);
    HIP_TRY(hipMemcpyAsync(c->h_cnt + 7, c->counters + 7, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
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

int lagot_last_fallback_cells(const lagot_ctx *ctx) { return ctx ? ctx->last_fb : -1; }

double lagot_last_cell_kernel_ms(const lagot_ctx *ctx) { return ctx ? ctx->ms_cell : -1.0; }

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
