/*
 * lagot.h -- C-ABI of the MI355X (gfx950) solver for semi-discrete partial
 * optimal transport with analytic restricted Laguerre cells
 * ("More Power to the Particles", arXiv 2601.05765).
 *
 * Problem (paper, section 2.2 "Volume-Constrained Lagrangian Mesh" and
 * "Free Surface", eq. (1); Algorithm 1): given sites p_i in a box, prescribed
 * volumes nu_i and weights psi_i, the generalized Laguerre cell of site i is
 *
 *   C_i = box ∩ B(p_i, sqrt(psi_i)) ∩ { x : |x-p_i|^2 - psi_i <= |x-p_j|^2 - psi_j  for all j != i }
 *
 * (the air object has weight 0). The solver finds the unique weights with
 * |C_i| = nu_i for all i by damped Newton on the Kantorovich functional, whose
 * gradient is nu_i - |C_i| and whose Hessian is eq. (2) (section 3.1). Around the
 * solve, the fluid model of section 5 (cell centroids, the P1 Laplacian of eq. (3),
 * the semi-implicit velocity update of eq. (4) and the whole step) reuses the same
 * cells, facet weights and conjugate gradients.
 *
 * Conventions for every entry point below
 *   - Array arguments are DEVICE pointers (for example torch tensor storage on
 *     the same GPU); all work is enqueued on the stream given to lagot_create.
 *   - Arrays are in the caller's site order; the library never keeps a
 *     caller pointer after a call returns. The caller owns every array; the
 *     library owns only its context workspace (grown on demand, freed by
 *     lagot_destroy).
 *   - Positions are float32 (x, y, z separate arrays), weights and volumes are
 *     float64. Geometry runs in float32; totals, residuals, CG inner products
 *     and the step-acceptance test run in float64 on the GPU. Cells whose float32
 *     result would lose accuracy are redone in float64; in a solve, once a full
 *     Newton step near the tolerance (max relative error < 100 tol, tol <= 1e-4) fails
 *     to halve ||nu - V||_2, the cells still off by more than tol/4 are finished in
 *     float64 for the rest of the call, so tolerances below float32 rounding converge.
 *   - Return value: LAGOT_OK (0) or one of the negative codes below. On a
 *     Newton error, psi_inout holds the last accepted iterate.
 *   - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef LAGOT_H
#define LAGOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LAGOT_OK 0
#define LAGOT_EINVAL (-1)       /* null pointer, n <= 0, site not strictly inside the box, nu <= 0,
                                   sum(nu) >= box volume, NaN input, bad option */
#define LAGOT_EEMPTY (-2)       /* some start cell is empty, so the KMT floor eps0 is 0 */
#define LAGOT_ENOCONV (-3)      /* max_newton iterations reached before the tolerance */
#define LAGOT_ELINESEARCH (-4)  /* max_halvings step halvings without an acceptable step */
#define LAGOT_ECAPACITY (-5)    /* output capacity too small (nnz_cap) or a cell exceeded even the
                                   large-capacity path */
#define LAGOT_ESINGULAR (-6)    /* conjugate-gradient breakdown (non-positive curvature) */
#define LAGOT_EHIP (-7)         /* HIP runtime error */

typedef struct lagot_ctx lagot_ctx;

typedef struct {
    double lo[3];
    double hi[3];
} lagot_box;

typedef struct {
    double tol;          /* stop when max_i |V_i - nu_i| / nu_i <= tol            (default 1e-5)  */
    int max_newton;      /* Newton iteration limit (section 6: 100)                (default 100)   */
    int max_halvings;    /* step halvings per iteration                           (default 30)    */
    double cg_rtol;      /* relative residual of the Jacobi-PCG direction solve   (default 1e-6)  */
    int cg_max_iter;     /* PCG iteration limit                                    (default 1000)  */
    int threads_per_cell;/* lanes per cell in the cell kernel: 0 = the context's default, else 8, 16,
                            32 or 64                                                             */
    int verbose;         /* 1: one line per Newton iteration to stderr; 2: also the first instance's
                            step length, residuals, fallback count and r_max; 3: also every
                            step-size trial of the first instance                                */
    int use_learned;     /* 1: try the learned warm start (lagot_mlp_set_params) before Newton       */
    int empty_start_fallback; /* 1 (default): if a start cell is empty (KMT needs eps0 > 0), give
                            each empty cell the weight of the neighbour j* that swallows its site
                            most (max psi_j - d_ij^2), so that their bisector is the mid-plane
                            (bounded so no other neighbour loses its site, and by twice the
                            local mean weight), and if a cell is still empty restart from the
                            default start: the common weight (1.2 (3 nu_mean / 4 pi)^(1/3))^2 of
                            the instance (a Voronoi start, no empty cell). An instance with more
                            than 64 empty start cells, and more than 1% of its cells, restarts
                            at once (no repair); 0: LAGOT_EEMPTY                                 */
    int autotune;        /* 1: when threads_per_cell is 0, time the cell kernel with 16, 32 and 64
                            lanes per cell, and the PCG kernels with four block shapes, on the
                            first solve of each size and density class, and keep the fastest in
                            the context (default 0: the context's defaults)                    */
    int use_graph;       /* 1: capture the launch sequences of a Newton iteration (Hessian + PCG set-up,
                            a chunk of PCG iterations, one step-size trial) as HIP graphs once per
                            call and replay them; the call then runs on a private stream of the
                            context, ordered after earlier work on the context's stream. Results
                            are identical to eager launches (default 0)                         */
    int residual_test;   /* 1 (default): a step size is kept only if min V >= eps0 and
                            ||nu - V||_2 drops by the factor (1 - alpha/2) (the KMT method the paper
                            cites); 0: the min-volume test alone, as Algorithm 1 prints it          */
    int continuation;    /* 1: path following on the prescribed volumes for starts far from the
                            solution (lagot_solve, one instance): with V0 the volumes at the start
                            weights, the targets nu(s) = (1 - s) V0 + s nu are solved by Algorithm 1
                            for s rising from 0 to 1, each stage from the previous one's weights:
                            intermediate stages to stage_tol (or stage_gtol) with at most stage_newton iterations
                            and 4 step halvings per iteration (PCG tolerance max(cg_rtol, 1e-2)),
                            the last (s = 1) to tol. The step in s starts at stage_step, doubles after
                            a stage of at most 3 iterations without halving, and halves after a stage
                            that fails to converge (or whose step search ends on a cell the kernels
                            cannot finish), whose weights are discarded; below 2^-12 the call fails
                            with that stage's error and the last accepted stage's weights.
                            0 (default): Algorithm 1 from the start weights                       */
    int stage_newton;    /* Newton iteration limit of an intermediate stage        (default 8)    */
    double stage_tol;    /* tolerance of the intermediate stages                   (default 1e-2) */
    int step_start;      /* 0 (default): each Newton iteration's step search starts at alpha = 1;
                            1: at min(1, 2 x the step length accepted by the previous iteration
                            of the call or continuation stage) -- Algorithm 1 does not say where
                            the search restarts; after short accepted steps this saves the
                            evaluations of trials that would be halved again; 2: as 1, and the
                            first iteration of each continuation stage after the first starts at
                            the first step length accepted in the stage before (not at 1)        */
    int reserved;        /* must be 0                                                            */
    double stage_step;   /* first step in s of the path following, in (0, 1]      (default 0.25) */
    double stage_gtol;   /* an intermediate stage also ends when ||nu(s) - V||_2 falls to stage_gtol
                            times its value at the stage's start (the largest relative error is set
                            by a few small cells; the bulk of the path is tracked by the norm);
                            0 (default): stage_tol alone; else in (0, 1)                         */
} lagot_opts;

typedef struct {
    int status;          /* LAGOT_* code of the call (of the instance, for a batched call) */
    int newton_iters;    /* accepted Newton iterations                                     */
    int evals;           /* full cell evaluations (start + one per step trial)             */
    int halvings;        /* total step halvings                                            */
    int cg_iters;        /* total PCG iterations                                           */
    int fallback_cells;  /* cells redone on the large-capacity float64 path (all evals)    */
    int failed_cells;    /* cells that exceeded even the large-capacity path (last eval)   */
    int cell_launches;   /* launches of the float32 cell kernel (one per evaluation)      */
    int learned_accepted;/* 0, or 1 + the halvings of the network's correction when the
                            learned guess replaced the start weights                   */
    int default_start;   /* 1 if an empty start cell forced the default start weights     */
    int repaired_start;  /* 1 if empty start cells were given the default weight (the other
                            weights kept)                                                   */
    int stages;          /* continuation stages accepted (opts.continuation), else 0      */
    double max_rel_err;  /* max_i |V_i - nu_i| / nu_i at the returned weights              */
    double grad_norm;    /* || nu - V ||_2 at the returned weights                         */
    double ms_total;     /* wall time of the call (host clock, stream synchronised)       */
    double ms_eval;      /* of which cell evaluations incl. reductions (host clock)        */
    double ms_linear;    /* of which Hessian assembly and PCG (host clock)                 */
    double ms_cell_kernel; /* summed duration of the float32 cell-kernel launches (HIP events
                              on the context stream)                                        */
    double ms_learned;   /* of which the learned warm start (features, network, its check) */
    double reserved_d[1];
} lagot_stats;

/* Fill *opts with the defaults listed above. */
void lagot_default_opts(lagot_opts *opts);

/* Create a context on HIP device `device`, enqueuing on `stream` (a hipStream_t;
 * NULL = the legacy default stream). Returns LAGOT_EINVAL if out is NULL,
 * LAGOT_EHIP if the device cannot be used. */
int lagot_create(lagot_ctx **out, int device, void *stream);

/* Release the context and its workspace. NULL is ignored. */
void lagot_destroy(lagot_ctx *ctx);

/*
 * One evaluation of all generalized Laguerre cells (paper section 3,
 * Algorithm 2; section 4 "Cell Update", "Restriction").
 *   in : n sites x,y,z [n] float32, psi [n] float64 (psi <= 0 gives an empty cell)
 *   out: vol [n] float64        |C_i|
 *        sph_area [n] float64   |∂B_i ∩ C_i|, the free-surface area K_i (may be NULL)
 *        wall_area [6n] float32 facet areas on the walls -x,+x,-y,+y,-z,+z, site-major
 *                               (may be NULL)
 *        row_ptr [n+1] int64, col [nnz_cap] int32, facet_area [nnz_cap] float32:
 *                               CSR of the restricted Laguerre facets |B_ij| > 0 as seen
 *                               from cell i, rows in site order, columns ascending
 *                               (all three NULL to skip; then nnz_out may be NULL)
 *        nnz_out (HOST pointer)  number of facets written; the call synchronises the
 *                               stream when it is requested.
 * Errors: LAGOT_EINVAL (bad pointer/size, site outside the box), LAGOT_ECAPACITY
 * (more facets than nnz_cap; *nnz_out still reports the count needed).
 */
int lagot_cells(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const double *psi,
                lagot_box box, double *vol, double *sph_area, float *wall_area, int64_t *row_ptr, int32_t *col,
                float *facet_area, int64_t nnz_cap, int64_t *nnz_out);

/*
 * One evaluation of all cells that also returns their centroids c_i = (1/|C_i|)
 * integral over C_i of x dx, the cell centroid that the paper's pressure model pulls
 * each site towards (section 5, "Incompressibility"). The first moment comes from the
 * same facet fans as the volume (divergence theorem: 4 integral of x dV = surface
 * integral of x (x.n) dA).
 *   in : as lagot_cells; out: vol [n] float64, centroid [3n] float64 (x, y, z per site,
 *        site-major; the site itself for an empty cell). Device pointers owned by the
 *        caller. Synchronises the stream.
 * Errors: as lagot_cells (LAGOT_EINVAL also for a NULL centroid).
 */
int lagot_centroids(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const double *psi,
                    lagot_box box, double *vol, double *centroid);

/*
 * One evaluation of all cells with the spherical area |K_i| by section 3.3's own route
 * (Algorithm 2: c = point_in(C_i), then |K_i| = |Sigma_i| - sum_f |Proj(B_f, Sigma_i, c)|):
 * c is the mean of the midpoints of the chords cast from each restricted facet's area
 * centroid along its inward normal; each restricted facet is projected from c onto the
 * sphere and the projected area taken by Gauss-Bonnet (geodesic curvature of a circle
 * at distance e from the centre e / (r rho), the corrected form of the printed one;
 * turning angles at the corners). A cell with no restricted facet is the whole sphere
 * if p_i is in its cell and empty otherwise. V_i = (sum_f t_f |B_f| + r |K_i|) / 3 as in
 * lagot_cells. Every cell is evaluated on the float64 path: this is the A/B variant of
 * the signed solid-angle form lagot_cells uses (same cells, same facets; the two agree
 * to rounding), slower by design.
 *   in : as lagot_cells; out: vol [n], sph_area [n] float64 in site order (device
 *        pointers owned by the caller). Synchronises the stream; the cell kernel's
 *        time is then lagot_last_cell_kernel_ms.
 * Errors: LAGOT_EINVAL (NULL output, n <= 0, site outside the box), LAGOT_ECAPACITY
 * (a cell beyond the float64 path's capacities).
 */
int lagot_cells_paper_k(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                        const double *psi, lagot_box box, double *vol, double *sph_area);

/*
 * One damped Newton iteration of Algorithm 1: evaluate the cells at psi, stop
 * if the tolerance already holds, else solve (-Hess K) u = nu - V by
 * Jacobi-PCG (eq. (2); walls do not enter) and halve the step from alpha = 1
 * until min V >= eps0 and ||nu - V||_2 decreases by the factor (1 - alpha/2)
 * (Kitagawa-Merigot-Thibert control; eps0 = 1/2 min(min nu, min V(psi)) here,
 * since a single step has no earlier start). psi_inout is updated in place.
 *   in : x,y,z [n] float32, nu [n] float64, psi_inout [n] float64, opts (NULL =
 *        defaults); out: psi_inout, *stats (HOST pointer, may be NULL).
 * Synchronises the stream. Errors: EINVAL, EEMPTY, ELINESEARCH, ESINGULAR, EHIP.
 */
int lagot_newton_step(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const double *nu,
                      lagot_box box, double *psi_inout, const lagot_opts *opts, lagot_stats *stats);

/*
 * Full solve of Algorithm 1 from the start weights in psi_inout to
 * max_i |V_i - nu_i| / nu_i <= opts->tol, with eps0 = 1/2 min(min nu, min V(psi_start)).
 * Same arguments as lagot_newton_step. Synchronises the stream.
 * Errors: EINVAL, EEMPTY, ENOCONV, ELINESEARCH, ESINGULAR, ECAPACITY, EHIP.
 */
int lagot_solve(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const double *nu,
                lagot_box box, double *psi_inout, const lagot_opts *opts, lagot_stats *stats);

/*
 * Solve at moved sites from the weights that solved the problem before the move (the
 * advect-and-solve step of a particle simulation; the warm start is not in the paper).
 * psi_inout holds the solution at positions p0 = (x0, y0, z0); the sites move to
 * p1 = (x1, y1, z1). Each weight is carried with its site: with c_i the centroid of cell
 * i before the move and d_i = p1_i - p0_i, psi_i - 2 d_i.(c_i - p0_i) + |d_i|^2 keeps the
 * power of the site at its old centroid, so the cell follows its centroid to first order
 * instead of being swept by the site's motion; Algorithm 1 (lagot_solve, opts) then solves
 * from these weights. If the carried weights leave a cell empty, or the solve does not
 * converge, the move is split: the sites go part of the way, float(p0 + t (p1 - p0)), are
 * solved there to max(tol, stage_tol), and the rest of the move starts from that solution;
 * the part halves after a failure and doubles after a success, down to 1/64 of the move,
 * where the empty-start repair of lagot_solve (opts.empty_start_fallback) takes over.
 *   in : x0, y0, z0, x1, y1, z1 [n] float32 (device; every site strictly inside the box at
 *        both ends), nu [n] float64, psi_inout [n] float64 (the solution at p0); opts as for
 *        lagot_solve (use_learned must be 0; continuation applies to each part).
 *   out: psi_inout (the solution at p1; unchanged on error); *stats (HOST, may be NULL):
 *        summed over the parts (evals include one centroid evaluation per accepted part),
 *        stages = parts solved, residuals of the last solve. Synchronises the stream.
 * Errors: as lagot_solve (the last part's error when even 1/64 of the move fails).
 */
int lagot_solve_moved(lagot_ctx *ctx, int64_t n, const float *x0, const float *y0, const float *z0,
                      const float *x1, const float *y1, const float *z1, const double *nu, lagot_box box,
                      double *psi_inout, const lagot_opts *opts, lagot_stats *stats);

/*
 * Many independent solves in one call (each instance is a full lagot_solve problem:
 * its own sites, prescribed volumes, box and start weights). Instance b owns the rows
 * [offsets[b], offsets[b+1]) of the concatenated arrays x, y, z, nu, psi_inout.
 * Every kernel serves all instances at once (one launch per step of Algorithm 1 for
 * the whole batch); each instance keeps its own eps0, step length, iteration count and
 * stopping test, and stops independently.
 *   in : n_inst >= 1; offsets (HOST, int64 [n_inst+1], offsets[0] = 0, strictly
 *        increasing: every instance has at least one site); boxes (HOST, [n_inst]);
 *        x, y, z [N] float32, nu [N] float64, psi_inout [N] float64 (device, N =
 *        offsets[n_inst]); opts as for lagot_solve (use_learned must be 0).
 *   out: psi_inout; per_inst (HOST, [n_inst], may be NULL): the statistics of each
 *        instance (status, iterations, evaluations, residuals; the ms_* fields are
 *        those of the whole call).
 * Returns LAGOT_OK if every instance converged, else the status of the first
 * instance that did not. The call validates every instance before solving any:
 * one invalid instance makes the call return LAGOT_EINVAL with nothing solved.
 * Synchronises the stream.
 */
int lagot_solve_batched(lagot_ctx *ctx, int32_t n_inst, const int64_t *offsets, const float *x, const float *y,
                        const float *z, const double *nu, const lagot_box *boxes, double *psi_inout,
                        const lagot_opts *opts, lagot_stats *per_inst);

/*
 * Learned warm start (not part of the paper's method). With opts->use_learned set,
 * lagot_solve takes the network's correction like a Newton step from the given start
 * weights: psi_start + beta s^2 out for beta = 1, 1/2, 1/4 (Algorithm 1's step halving),
 * the first trial that keeps every cell at least at the KMT floor
 * eps0 = 1/2 min(min nu, min V(psi_start)) and makes both ||nu - V||_2 and
 * max_i |V_i - nu_i| / nu_i smaller than at the start replaces the start (stats
 * learned_accepted = 1 + the halvings); eps0 stays that of the given start, and Newton
 * then runs to the tolerance as usual. A start with an empty cell is left to the repair
 * and restart of empty_start_fallback (no guess is tried).
 * Inputs of site i (64 bf16, row-major n x 64): offsets (p_j - p_i)/s_i of its 16 nearest
 * sites in ascending (distance, index), psi_prev_i / s_i^2, nu_i / mean(nu), and the
 * relative volume mismatch (nu - V)/nu under the previous weights of site i and of its
 * 13 nearest sites; s_i = nu_i^(1/3). Network 64 -> 128 -> 128 -> 128 -> 1 with GELU (erf form), output
 * (psi_new_i - psi_prev_i) / s_i^2. Parameters: LAGOT_MLP_NPARAMS float32 laid out as
 * W1[64][128], b1[128], W2[128][128], b2[128], W3[128][128], b3[128], w4[128], b4[1]
 * (row-major, input index first). Products run in bf16 on MFMA with float32 accumulation.
 */
#define LAGOT_MLP_NPARAMS 41473

/* Load float32 parameters (device pointer, LAGOT_MLP_NPARAMS values) into the context
 * and reset the Adam state. Errors: EINVAL, EHIP. */
int lagot_mlp_set_params(lagot_ctx *ctx, const float *params);

/* Copy the context's float32 parameters to `params` (device). EINVAL if none are set. */
int lagot_mlp_get_params(lagot_ctx *ctx, float *params);

/* The 16 nearest sites (caller indices, int32 [n x 16], may be NULL) and the network
 * inputs (bf16 as uint16 [n x 64], may be NULL) of every site, in caller order, from
 * positions, previous weights psi_prev [n] float64 and volumes nu [n] float64 (the
 * cells are evaluated at psi_prev for the mismatch inputs).
 * Errors: EINVAL, ECAPACITY (fewer than 17 sites), EHIP. */
int lagot_features(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const double *psi_prev,
                   const double *nu, lagot_box box, int32_t *nbr, uint16_t *feats);

/* Network output for m input rows (bf16 [m x 64], device) into out [m] float32.
 * Synchronises the stream. Errors: EINVAL (no parameters), EHIP. */
int lagot_mlp_forward(lagot_ctx *ctx, int64_t m, const uint16_t *feats, float *out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lagot_mlp_forward without any
 * allocation. Same arguments, kernels and results. The two bf16 hidden-activation buffers
 * (2 x m x 128 values) live in one static device array of the library, of
 * LAGOT_NOALLOC_MAX_ROWS rows (16 MiB; each GPU the library runs on holds its own copy until
 * the process ends); the parameters are the context's (lagot_mlp_set_params, called before).
 * The call only enqueues the kernels on the context's stream: out is ready when the stream
 * reaches that point (it does not synchronise). Every call on one GPU shares that GPU's array,
 * so calls that overlap on one GPU (two contexts, or streams that run concurrently) race and
 * must be ordered by the caller. Errors: EINVAL (NULL pointer, m <= 0, no parameters),
 * ECAPACITY (m > LAGOT_NOALLOC_MAX_ROWS), EHIP. */
#define LAGOT_NOALLOC_MAX_ROWS 32768
int lagot_mlp_forward_noalloc(lagot_ctx *ctx, int64_t m, const uint16_t *feats, float *out);

/* One Adam step (lr; beta 0.9, 0.999; eps 1e-8) on the mean squared error of the rows
 * batch_idx[0..batch) (device int32) of feats [nrows x 64] against targets [nrows]
 * (float32, device). *loss (HOST, may be NULL) receives the batch loss before the
 * step (the call then synchronises). Errors: EINVAL, EHIP. */
int lagot_mlp_train_step(lagot_ctx *ctx, int64_t nrows, const uint16_t *feats, const float *targets,
                         const int32_t *batch_idx, int32_t batch, float lr, float *loss);

/* Gradient of the last lagot_mlp_train_step's batch loss with respect to the parameters
 * (device float32 [LAGOT_MLP_NPARAMS]; diagnostic). */
int lagot_mlp_last_grads(lagot_ctx *ctx, float *grads);

/* Lanes per cell (8, 16, 32 or 64) used by lagot_cells and by solves whose options leave
 * threads_per_cell at 0 (default 32). Returns LAGOT_EINVAL for other values. */
int lagot_set_threads_per_cell(lagot_ctx *ctx, int threads_per_cell);

/* Block shape of the Jacobi-PCG kernels (one kernel per CG iteration) for solves whose
 * options do not set autotune: lanes per matrix row (1, 2, 4 or 8) and rows per
 * workgroup (64, 128 or 256; at most 128 with 8 lanes). Default 4 and 64. With
 * opts->autotune the first direction solve of each size/density class times the shapes
 * 2x128, 4x128, 2x64 and 4x64 and keeps the fastest. Affects speed only.
 * Returns LAGOT_EINVAL for other shapes. */
int lagot_set_cg_shape(lagot_ctx *ctx, int lanes_per_row, int rows_per_block);

/* How a Jacobi-PCG iteration of the Newton direction is launched. One kernel per iteration
 * forms each neighbour's direction entry from its whole 32-byte record (one global
 * synchronisation per iteration, but 32 bytes gathered per matrix entry); two kernels
 * write every row's entry first (8 bytes per row) and then take the product from those
 * (8 bytes gathered per entry, one more launch). mode 0 (default): two kernels when an
 * instance of the call has more than 2048 partial sums (about 131,000 rows), else one;
 * 1: always one; 2: always two. The same arithmetic per row: the directions agree to the
 * rounding of the partial sums. Affects speed only. Errors: LAGOT_EINVAL. */
int lagot_set_cg_split(lagot_ctx *ctx, int mode);

/*
 * Convex polyhedral domain {x : n_w . x <= c_w, w < nplanes} in place of the box walls
 * for every later call on this context (the paper evaluates its cells in polyhedral
 * domains, section 6; a convex one is an intersection of half-spaces). The domain's
 * planes bound the cells, enter V, K and the wall areas, and not the Hessian (they do
 * not move with psi). The box argument of the calls must still contain the domain (it
 * bounds the neighbour grid); sites must lie strictly inside both. With a domain,
 * lagot_cells' wall_area holds nplanes areas per site (site-major, in plane order).
 *   in : planes [4 nplanes] float64 HOST array (n_x, n_y, n_z, c) per plane, unit outward
 *        normals (|n| within 1e-6 of 1); 0 <= nplanes <= 32; nplanes = 0 restores the box.
 * Applies to every instance of a batch. Synchronises the stream.
 * Errors: LAGOT_EINVAL (NULL ctx or planes, nplanes out of range, normal not unit, c not
 * finite), LAGOT_EHIP.
 */
int lagot_set_domain(lagot_ctx *ctx, int nplanes, const double *planes);

/*
 * Non-convex polyhedral domain (section 6: cells in polyhedral domains, e.g. a pipe) as
 * the union of npieces convex pieces with disjoint interiors, for every later call on
 * this context. Piece k is {x : n_w . x <= c_w, piece_off[k] <= w < piece_off[k+1]}.
 * Each plane is either a wall of the domain (wall_id[w] in [0, nwalls): its facet areas
 * go to that wall; a wall may span several pieces) or a plane between two pieces
 * (wall_id[w] = -1: no wall area). The restricted cell is the union of its parts in the
 * pieces, so V, K, the facet areas (and with them the Hessian) and the centroids are the
 * sums over the pieces; each piece is evaluated like a convex domain, so a call costs up
 * to npieces evaluations. With pieces, lagot_cells' wall_area holds nwalls areas per site
 * (site-major, by wall id). Sites must lie strictly inside some piece: not on a plane
 * between pieces either (the solid angle of a facet seen from a site on its plane depends
 * on the side it is approached from), so the cuts between pieces should avoid the sites.
 * Every plane of a piece must lie wholly on the domain's boundary or wholly between two
 * pieces. The box argument must contain the domain. lagot_set_domain (any nplanes, 0
 * included) goes back to a convex domain.
 *   in : piece_off [npieces + 1] int32 HOST (piece_off[0] = 0, 1 to 32 planes per piece,
 *        at most 64 planes in all); planes [4 piece_off[npieces]] float64 HOST, (n_x, n_y,
 *        n_z, c) per plane, unit outward normals (|n| within 1e-6 of 1); wall_id
 *        [piece_off[npieces]] int32 HOST; 1 <= npieces <= 16, 1 <= nwalls <= 64.
 * lagot_cells_paper_k runs its route in each piece and sums. The crowded pass is not timed
 * per piece (lagot_last_kernel_times reports no crowded-pass time); lagot_last_pass_counts
 * gives the crowded cells summed over the pieces and the last piece's float64 count.
 * Synchronises the stream.
 * Errors: LAGOT_EINVAL (NULL pointers, counts out of range, a normal not unit, c not
 * finite, a wall id out of range), LAGOT_EHIP.
 */
int lagot_set_domain_pieces(lagot_ctx *ctx, int npieces, const int32_t *piece_off, const double *planes,
                            const int32_t *wall_id, int nwalls);

/*
 * The P1 Laplacian over the restricted Laguerre facets (section 5, eq. (3)):
 *   (Lap u)_i = sum_j mu_ij w_ij (u_j - u_i),  w_ij = |V_ij| / (2 |p_j - p_i|),
 * mu_ij = (mu_i + mu_j) / 2 (one reading of the paper's per-pair coefficients). |V_ij|
 * is the facet area seen from the two cells, averaged (a facet that only one side
 * lists keeps that side's area); wall and spherical facets do not enter.
 *   in : the cells as lagot_cells (x, y, z [n] float32, psi [n] float64, box); mu [n]
 *        float64 per-site coefficients or NULL (then mu_ij = mu0); u [3n] float64
 *        (three values per site, site-major).
 *   out: lap_u [3n] float64, site-major. Device pointers owned by the caller; u and
 *        lap_u must not overlap. Synchronises the stream.
 * Errors: EINVAL (as lagot_cells, or a negative or non-finite mu), ECAPACITY, EHIP.
 */
int lagot_p1_laplacian(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const double *psi,
                       lagot_box box, const double *mu, double mu0, const double *u, double *lap_u);

typedef struct {
    double dt;          /* time step (> 0)                                                     */
    double eps;         /* pressure spring F_p = m_i (c_i - p_i) / eps^2 (> 0; +inf: none)     */
    double gamma;       /* surface tension F_t = gamma Lap p (>= 0)                            */
    double mu;          /* viscosity of every site when the per-site array is NULL (>= 0)      */
    double gravity[3];  /* gravity (acceleration): F_g = m_i g                                 */
    double cg_rtol;     /* PCG stop ||r|| <= cg_rtol ||b|| per coordinate   (default 1e-10)    */
    int cg_max_iter;    /* PCG iteration limit per coordinate               (default 2000)     */
    int reserved;
} lagot_fluid_params;

/* dt 1e-3, eps 1, gamma 0, mu 0, gravity (0, 0, -9.81), cg_rtol 1e-10, cg_max_iter 2000 */
void lagot_default_fluid_params(lagot_fluid_params *prm);

/*
 * Velocity update of the fluid step (section 5, "Numerical integration", eq. (4)):
 * with the cells at the sites p and weights psi (normally the OT solution there) and
 * their centroids c_i,
 *   F_p = m_i (c_i - p_i) / eps^2,  F_g = m_i g,  F_t = gamma Lap p  (mu_ij = 1 here),
 *   (m_i/dt) v_i - (Lap_mu v)_i = (m_i/dt) v_in_i + F_p + F_g + F_t,
 * solved for v by Jacobi-PCG, the three coordinates together, each stopping at
 * ||r|| <= cg_rtol ||b|| (Lap_mu as lagot_p1_laplacian; the system is symmetric
 * positive definite). Positions are not moved: the step's
 * position update x += dt v is the caller's. Wall terms (fluid-boundary affinities)
 * do not enter.
 *   in : x, y, z [n] float32, psi [n] float64, box; mass [n] float64 (> 0); mu [n]
 *        float64 per-site viscosity or NULL (then prm->mu); v_in [3n] float64
 *        site-major; prm HOST pointer.
 *   out: v_out [3n] float64 site-major (may equal v_in); centroid [3n] float64 or NULL;
 *        cg_iters [3] HOST int32 PCG iterations per coordinate, or NULL. Device
 *        pointers owned by the caller. Synchronises the stream.
 * Errors: EINVAL (as lagot_cells, bad parameters, a mass <= 0, a negative mu, a
 *         non-finite value), ENOCONV (cg_max_iter iterations without the tolerance),
 *         ESINGULAR (PCG breakdown), ECAPACITY, EHIP.
 */
int lagot_fluid_velocity(lagot_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                         const double *psi, lagot_box box, const double *mass, const double *mu, const double *v_in,
                         const lagot_fluid_params *prm, double *v_out, double *centroid, int32_t *cg_iters);

/*
 * One whole fluid step (section 5, "Numerical integration"): the positions move with the
 * old velocities, x <- x + dt v, the weights are re-solved at the new positions
 * (Algorithm 1 from psi_inout, as lagot_solve), and the velocities are updated at the
 * new cells as lagot_fluid_velocity. The moved positions are kept inside the domain:
 * each coordinate is clamped to [lo + m_a, hi - m_a], m_a = max(1e-6 (hi_a - lo_a), u)
 * with u = 4 float32 spacings at the largest |bound| (so the rounding to float32 keeps a
 * clamped site strictly inside), and, with convex domain planes (lagot_set_domain), a
 * site beyond n.x = c - m (m = max(1e-6 times the largest box extent, u)) is moved along
 * -n onto that plane, in two passes over the planes. With a non-convex domain
 * (lagot_set_domain_pieces) a site stays where it is if that rule, applied with the planes
 * of some piece, leaves it in place; else it moves to the nearest of the places the rule
 * gives with each piece's planes (ties to the first piece). The update x + dt v is formed
 * in float64 with separate roundings and rounded once to float32.
 *   in/out: x, y, z [n] float32 (device), psi_inout [n] float64, v_inout [3n] float64
 *           site-major; in: nu [n] float64, mass [n] float64 (> 0), mu [n] or NULL,
 *           prm, opts (NULL = defaults) HOST; out: stats (the solve's, HOST, may be
 *           NULL), cg_iters [3] HOST int32 or NULL.
 * Errors: those of lagot_solve and lagot_fluid_velocity; invalid parameters, options,
 *         prescribed volumes (<= 0), masses (<= 0), velocities (not finite) and
 *         viscosities (< 0) are rejected (EINVAL) before anything moves; a NaN weight or a
 *         site outside the box is found by the solve. After a solve error the positions have moved,
 *         psi_inout holds the solve's last accepted weights and v_inout is unchanged.
 *         Synchronises the stream.
 */
int lagot_fluid_step(lagot_ctx *ctx, int64_t n, float *x, float *y, float *z, const double *nu, lagot_box box,
                     double *psi_inout, const double *mass, const double *mu, double *v_inout,
                     const lagot_fluid_params *prm, const lagot_opts *opts, lagot_stats *stats, int32_t *cg_iters);

/* Number of cells that the last lagot_cells call on this context redid on the
 * large-capacity float64 path (diagnostic; -1 if ctx is NULL). */
int lagot_last_fallback_cells(const lagot_ctx *ctx);

/* Per-bit cell counts of the last evaluation on this context (lagot_cells or the
 * last evaluation of a solve), a diagnostic of why cells took the float64 path.
 * counts[k] for k < 8: cells whose final result has bit k; counts[8 + k]: cells that
 * the float32 pass sent to the float64 path with reason bit k. Bits: 0 empty cell,
 * 1 too many candidate bisectors, 2 too many polytope planes, 3 too many vertices,
 * 4 inconsistent clip combinatorics, 5 facet walk not closed, 6 too many facets,
 * 7 float32 relative accuracy insufficient (volume small against its terms).
 *   out: counts [16] HOST array. Synchronises the stream.
 * Errors: EINVAL (null pointer or nothing evaluated yet), EHIP. */
int lagot_last_flag_counts(lagot_ctx *ctx, int64_t *counts);

/* Cells of the last evaluation on this context that took the later passes (section 4,
 * "Finding Contributing Neighbors"): counts[0] the crowded cells the float32 pass
 * deferred (search block of more than 1024 sites, or more than 48 candidate bisectors);
 * counts[1] the cells listed for the float64 large-capacity path. A deferred cell takes
 * the crowded pass (candidates from the overlap of cell boxes) when the call expects
 * crowded cells -- a site grid refined below 2 r_max because a few balls are much larger
 * than the spacing, or cells deferred earlier in the call or in the context's last call
 * -- and the float64 pass otherwise (same cells, slower); counts[2] is 1 if the crowded
 * pass ran. Diagnostic.
 *   out: counts [3] HOST array. Synchronises the stream.
 * Errors: EINVAL (null pointer or nothing evaluated yet), EHIP. */
int lagot_last_pass_counts(lagot_ctx *ctx, int64_t *counts);

/* Kernel times of the last call on this context (HIP events on its stream, outside graph
 * capture): out[0] summed ms of the float32 cell-kernel launches, out[1] their number,
 * out[2] summed ms of the crowded-cell pass (box-overlap candidates, float64), out[3]
 * its launches, out[4] the cells those launches processed. Diagnostic; valid after the
 * call returned (it synchronises).
 *   out: out [5] HOST array. Errors: EINVAL (null pointer). */
int lagot_last_kernel_times(const lagot_ctx *ctx, double *out);

/* The cells the float32 pass deferred as crowded in the last evaluation on this context,
 * as caller indices (in the order the pass listed them). Diagnostic.
 *   out: idx [min(count, cap)] HOST int32 (may be NULL when cap = 0); *count HOST = the
 *        number of deferred cells. Synchronises the stream.
 * Errors: EINVAL (null pointer or nothing evaluated yet), EHIP. */
int lagot_last_deferred(lagot_ctx *ctx, int32_t *idx, int64_t cap, int64_t *count);

/* Duration in ms of the float32 cell-kernel launch of the last lagot_cells call
 * (HIP events on the context stream; diagnostic; -1 if ctx is NULL). */
double lagot_last_cell_kernel_ms(const lagot_ctx *ctx);

/* Human-readable text for a LAGOT_* code (static storage). */
const char *lagot_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LAGOT_H */
