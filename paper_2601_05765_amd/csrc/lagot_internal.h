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
};

struct BoxF {
    float lo[3], hi[3];
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
    int32_t *fail_count; // [1] cells that failed the float64 path too
};

// ---- launch wrappers (defined in the .hip files) ----
// grid.hip
void launch_gather_sites(hipStream_t st, int64_t n, const float *x, const float *y, const float *z,
                         const double *psi, float4 *pos_orig, double *rmax_partial, int nblk);
void launch_reduce_max(hipStream_t st, const double *partial, int nblk, double *out);
void launch_grid_build(hipStream_t st, int64_t n, const float4 *pos_orig, GridDesc g, int32_t *keys,
                       int32_t *cell_count, int32_t *cell_start, int32_t *scan_tmp, int32_t *perm,
                       int32_t *cursor);
void launch_permute_in(hipStream_t st, int64_t n, const int32_t *perm, const float4 *pos_orig, const double *psi,
                       const double *nu, float4 *pos_s, double *psi_s, double *nu_s);
void launch_psi_shadow(hipStream_t st, int64_t n, const double *psi_s, float4 *pos_s);
void launch_scatter_out_f64(hipStream_t st, int64_t n, const int32_t *perm, const double *src_s, double *dst);
void launch_validate(hipStream_t st, int64_t n, const float *x, const float *y, const float *z, const double *psi,
                     const double *nu, BoxF box, int32_t *bad);
void launch_scan_i32(hipStream_t st, const int32_t *in, int32_t *out, int n, int32_t *tmp);
void launch_csr_count(hipStream_t st, int64_t n, const int32_t *perm, const int32_t *fcnt, int32_t *cnt_orig);
void launch_csr_fill(hipStream_t st, int64_t n, const int32_t *perm, const int32_t *fcol, const float *farea,
                     const int32_t *fcnt, const int32_t *start, int32_t *col, float *area, int64_t *row_ptr);
void launch_scatter_walls(hipStream_t st, int64_t n, const int32_t *perm, const float *wall_s, float *wall);
void launch_scatter_rows(hipStream_t st, int64_t n, int row_bytes, const int32_t *perm, const void *src, void *dst);
void launch_gather_rmax(hipStream_t st, int64_t n, const double *psi, double *partial);

// cells.hip
void launch_cells(hipStream_t st, int64_t n, const float4 *pos_s, const double *psi_s, const int32_t *perm,
                  const int32_t *cell_start, GridDesc g, BoxF box, const double *rmax, EvalOut out, int tpc);
void launch_cells_fallback(hipStream_t st, int64_t n, const float4 *pos_s, const double *psi_s, const int32_t *perm,
                           const int32_t *cell_start, GridDesc g, BoxF box, const double *rmax, EvalOut out);

// newton.hip
void launch_eval_reduce(hipStream_t st, int64_t n, const double *V, const double *nu, double *partial, int nblk,
                        double *out4);
void launch_hess_assemble(hipStream_t st, int64_t n, const float4 *pos_s, const double *psi_s, const double *K,
                          const int32_t *fcol, const float *farea, const int32_t *fcnt, int32_t *hcol, float *hval,
                          int32_t *xcnt, double *diag, int32_t *err);
void launch_hess_finish(hipStream_t st, int64_t n, const double *psi_s, const double *K, const int32_t *fcnt,
                        const int32_t *xcnt, int32_t *hcnt, const float *hval, double *diag);
int pcg_blocks(int64_t n);
int spmv_blocks(int64_t n);
void launch_pcg_init(hipStream_t st, int64_t n, int nb, const double *V, const double *nu, const double *diag,
                     double *g, double *x, double *r, double *z, double *RZ, double *RR, double *R0, int32_t *state);
void launch_pcg_spmv(hipStream_t st, int64_t n, int k, int nb, double rtol2, const double *R0, const int32_t *hcol,
                     const float *hval, const int32_t *hcnt, const double *diag, const double *z, const double *p_old,
                     double *p_new, double *q, const double *RZ, const double *RR, double *PQ, const int32_t *state);
void launch_pcg_update(hipStream_t st, int64_t n, int k, int nb, double rtol2, const double *R0, const double *diag,
                       double *x, double *r, double *z, const double *p, const double *q, double *RZ, double *RR,
                       const double *PQ, int32_t *state);
void launch_pcg_status(hipStream_t st, int nb, const double *RR, const double *R0, const int32_t *state,
                       double *scal);
void launch_axpy_trial(hipStream_t st, int64_t n, const double *psi_s, const double *u, double alpha,
                       double *psi_trial, float4 *pos_s, double *rmax_partial);

// mlp.hip
void launch_knn_features(hipStream_t st, int64_t n, const float4 *pos_s, const int32_t *perm,
                         const int32_t *cell_start, GridDesc g, const double *psi_prev_s, const double *nu_s,
                         const double *nu_sum, const double *V_s, int32_t *nbr, uint16_t *feat, int32_t *err);
void launch_default_start(hipStream_t st, int64_t n, const double *nu_s, double *psi_s, float4 *pos_s,
                          double *rmax_partial);
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
void launch_apply_guess(hipStream_t st, int64_t n, const double *psi_prev, const double *nu, const float *out,
                        double *psi_new, float4 *pos_s, double *rmax_partial);
enum { MLP_EPI_STORE = 0, MLP_EPI_BIAS_GELU = 1, MLP_EPI_GELU_BACK = 2 };

}  // namespace lagot
