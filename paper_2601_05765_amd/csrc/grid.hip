// grid.hip -- uniform-grid spatial sort of the sites (grid_knn, construction
// part) and the gathers/scatters between caller order and grid order.
//
// The bisectors that cut ball i come from the grid cells within r_i + r_max of
// site i (section 4 "Finding Contributing Neighbors": the ball bound replaces the
// security radius and is exact for restricted cells); cells whose block is crowded
// take the box-overlap pass of cells.hip instead. Sites are counting-sorted by grid
// cell (z fastest), and within a grid
// cell by caller index, so the order is deterministic. In a batched call every
// instance has its own grid (its own box and r_max); the grids are laid end to
// end in one cell array, so one sort orders all instances and keeps each one in
// its own row range.
#include "lagot_internal.h"

namespace lagot {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ inline int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one tile; returns the tile total through bsum.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(const int32_t *__restrict__ in,
                                                              int32_t *__restrict__ out,
                                                              int32_t *__restrict__ bsum, int n) {
    __shared__ int wsum[SCAN_THREADS / 64];
    const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int tsum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        tsum += v[k];
    }
    int incl = wave_incl_scan(tsum);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int woff = 0;
    for (int k = 0; k < w; ++k) woff += wsum[k];
    int run = woff + incl - tsum;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == SCAN_THREADS - 1) bsum[blockIdx.x] = run;
}

// Single-block exclusive scan of the tile totals (any count).
__global__ __launch_bounds__(1024) void k_scan_sums(int32_t *bsum, int nb, int32_t *total) {
    __shared__ int wsum[16];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        int i = base + threadIdx.x;
        int v = (i < nb) ? bsum[i] : 0;
        int incl = wave_incl_scan(v);
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int woff = 0;
        for (int k = 0; k < w; ++k) woff += wsum[k];
        int c = carry;
        if (i < nb) bsum[i] = c + woff + incl - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry = c + woff + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(int32_t *out, const int32_t *bsum, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += bsum[i / SCAN_TILE];
}

// exclusive scan of in[0..n) into out[0..n), out[n] = total
void exclusive_scan(hipStream_t st, const int32_t *in, int32_t *out, int n, int32_t *tmp) {
    int nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(SCAN_THREADS), 0, st, in, out, tmp, n);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, tmp, nb, out + n);
    hipLaunchKernelGGL(k_scan_add, dim3((n + 255) / 256), dim3(256), 0, st, out, tmp, n);
}

__global__ void k_gather_sites(int64_t n, const float *__restrict__ x, const float *__restrict__ y,
                               const float *__restrict__ z, const double *__restrict__ psi,
                               float4 *__restrict__ pos) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pos[i] = make_float4(x[i], y[i], z[i], (float)psi[i]);
}

__global__ void k_zero_i32(int32_t *p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// instance of every row, from the tile table (one 64-lane block per tile)
__global__ __launch_bounds__(TILE) void k_fill_inst(Batch bt, int32_t *__restrict__ inst) {
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    const int row = bt.tile_row[t] + (int)threadIdx.x;
    if (row < bt.off[b + 1]) inst[row] = b;
}

__global__ __launch_bounds__(1024) void k_rmax_zero(Batch bt, int want, double *__restrict__ rmax) {
    for (int b = threadIdx.x; b < bt.B; b += 1024)
        if (selected(bt, want, b)) rmax[b] = 0.0;
}

// rmax[b] = max over rows of sqrt(psi). A tile lies in one instance: a block-wide
// max and one atomic per tile (max is order-independent: deterministic).
__global__ __launch_bounds__(TILE) void k_rmax_tiles(Batch bt, int want, const double *__restrict__ psi,
                                                      double *__restrict__ rmax) {
    __shared__ double sh[TILE / 64];
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    if (!selected(bt, want, b)) return;
    const int row = bt.tile_row[t] + (int)threadIdx.x;
    double r = 0.0;
    if (row < bt.off[b + 1]) {
        const double p = psi[row];
        r = p > 0.0 ? sqrt(p) : 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < TILE / 64; ++w) r = fmax(r, sh[w]);
        // non-negative doubles order like their bit patterns
        atomicMax(reinterpret_cast<unsigned long long *>(rmax + b), (unsigned long long)__double_as_longlong(r));
    }
}

__device__ inline int grid_key(const GridDesc &g, float px, float py, float pz) {
    int ix = (int)floorf((px - g.lo[0]) * g.inv_s);
    int iy = (int)floorf((py - g.lo[1]) * g.inv_s);
    int iz = (int)floorf((pz - g.lo[2]) * g.inv_s);
    ix = min(max(ix, 0), g.dim[0] - 1);
    iy = min(max(iy, 0), g.dim[1] - 1);
    iz = min(max(iz, 0), g.dim[2] - 1);
    return (ix * g.dim[1] + iy) * g.dim[2] + iz;
}

__global__ void k_keys_count(int64_t n, Batch bt, const float4 *__restrict__ pos, int32_t *__restrict__ keys,
                             int32_t *__restrict__ count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const GridDesc g = bt.grid[bt.inst[i]];
    float4 p = pos[i];
    int k = g.base + grid_key(g, p.x, p.y, p.z);
    keys[i] = k;
    atomicAdd(&count[k], 1);
}

__global__ void k_scatter(int64_t n, const int32_t *__restrict__ keys, int32_t *__restrict__ cursor,
                          int32_t *__restrict__ perm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int slot = atomicAdd(&cursor[keys[i]], 1);
    perm[slot] = (int32_t)i;
}

// Order each grid cell's sites by caller index, so that the grid order does not depend
// on the order of the scatter's atomics. Cells usually hold a few sites (insertion
// sort); crowded scenes with large weights get cells of thousands of sites, which are
// heap-sorted (O(k log k) instead of O(k^2) per thread).
__device__ inline void sift_down(int32_t *a, int root, int end) {
    for (;;) {
        int child = 2 * root + 1;
        if (child >= end) return;
        if (child + 1 < end && a[child + 1] > a[child]) ++child;
        if (a[root] >= a[child]) return;
        const int32_t t = a[root];
        a[root] = a[child];
        a[child] = t;
        root = child;
    }
}

__global__ void k_sort_cells(int ncell, const int32_t *__restrict__ start, int32_t *__restrict__ perm) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int b = start[c], e = start[c + 1];
    const int m = e - b;
    if (m > 32) {
        int32_t *a = perm + b;
        for (int r = m / 2 - 1; r >= 0; --r) sift_down(a, r, m);
        for (int last = m - 1; last > 0; --last) {
            const int32_t t = a[0];
            a[0] = a[last];
            a[last] = t;
            sift_down(a, 0, last);
        }
        return;
    }
    for (int a = b + 1; a < e; ++a) {
        int v = perm[a];
        int k = a - 1;
        while (k >= b && perm[k] > v) {
            perm[k + 1] = perm[k];
            --k;
        }
        perm[k + 1] = v;
    }
}

__global__ void k_permute_in(int64_t n, const int32_t *__restrict__ perm, const float4 *__restrict__ pos_orig,
                             const double *__restrict__ psi, const double *__restrict__ nu, float4 *__restrict__ pos_s,
                             double *__restrict__ psi_s, double *__restrict__ nu_s) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int i = perm[k];
    pos_s[k] = pos_orig[i];
    psi_s[k] = psi[i];
    if (nu) nu_s[k] = nu[i];
}

__global__ void k_psi_shadow(int64_t n, const double *__restrict__ psi_s, float4 *__restrict__ pos_s) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    pos_s[k].w = (float)psi_s[k];
}

__global__ void k_scatter_out(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ src,
                              double *__restrict__ dst) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    dst[perm[k]] = src[k];
}

// Count invalid inputs per instance: NaN, site not strictly inside its box, nu <= 0.
__global__ void k_validate(int64_t n, Batch bt, const float *__restrict__ x, const float *__restrict__ y,
                           const float *__restrict__ z, const double *__restrict__ psi, const double *__restrict__ nu,
                           int32_t *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = bt.inst[i];
    const BoxF box = bt.box[b];
    float p[3] = {x[i], y[i], z[i]};
    bool ok = true;
    for (int a = 0; a < 3; ++a) ok = ok && (p[a] > box.lo[a]) && (p[a] < box.hi[a]);  // false for NaN
    if (bt.npieces > 0) {
        // strictly inside some piece (a site on a plane of a piece would see that plane's
        // facet at a solid angle that depends on the side it is approached from)
        bool in_any = false;
        for (int k = 0; k < bt.npieces; ++k) {
            bool in = true;
            for (int w = bt.dom_off[k]; w < bt.dom_off[k + 1]; ++w) {
                const float4 q = bt.dom[w];
                in = in && (q.x * p[0] + q.y * p[1] + q.z * p[2] < q.w);
            }
            in_any = in_any || in;
        }
        ok = ok && in_any;
    } else {
        for (int w = 0; w < bt.ndom; ++w) {  // strictly inside every domain plane
            const float4 q = bt.dom[w];
            ok = ok && (q.x * p[0] + q.y * p[1] + q.z * p[2] < q.w);
        }
    }
    if (psi) ok = ok && !isnan(psi[i]);
    if (nu) ok = ok && (nu[i] > 0.0);
    if (!ok) atomicAdd(bad + b, 1);
}

__global__ void k_zero_f32(float *p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.f;
}

// Before each piece's passes: the last piece's deferred cells are added to the sum (which
// the first piece starts at 0) and the list counters are cleared. Called once more after
// the last piece without fb_count: the count then holds the sum over all pieces.
__global__ void k_piece_begin(int first, int32_t *fb_count, int32_t *ovf_count, int32_t *ovf_sum) {
    const int32_t s = first ? 0 : *ovf_sum + *ovf_count;
    *ovf_sum = s;
    if (fb_count) {
        *fb_count = 0;
        *ovf_count = 0;
    } else {
        *ovf_count = s;
    }
}

// One piece's outputs into the accumulators (grid row k; the rows of the selected
// instances): volume, spherical area and first moment added, facets merged by neighbour
// (areas of the same neighbour summed), wall areas added by wall id (planes between
// pieces dropped), flags or-ed. A merged list longer than FCAP is a capacity failure.
__global__ void k_piece_accum(int64_t n, Batch bt, int want, int first, EvalOut o, int nwp,
                              const int32_t *__restrict__ wid, int nwalls, const int32_t *__restrict__ perm,
                              PieceAcc a) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int b = bt.inst[k];
    if (!selected(bt, want, b)) return;
    const double V = o.V[k];
    const int64_t ci = perm[k];
    const int cnt = o.fcnt[k];
    if (first) {
        a.V[k] = V;
        a.K[k] = o.K[k];
        a.flags[k] = o.flags[k];
        for (int f = 0; f < cnt; ++f) {
            a.fcol[k * FCAP + f] = o.fcol[k * FCAP + f];
            a.farea[k * FCAP + f] = o.farea[k * FCAP + f];
        }
        a.fcnt[k] = cnt;
        if (o.cen)
            for (int q = 0; q < 3; ++q) a.mom[3 * ci + q] = V * o.cen[3 * ci + q];
        if (o.wall)
            for (int w = 0; w < nwalls; ++w) a.wall[k * nwalls + w] = 0.f;
    } else {
        a.V[k] += V;
        a.K[k] += o.K[k];
        uint32_t fl = a.flags[k] | o.flags[k];
        int m = a.fcnt[k];
        const int m0 = m;
        for (int f = 0; f < cnt; ++f) {
            const int j = o.fcol[k * FCAP + f];
            const float ar = o.farea[k * FCAP + f];
            int g = 0;
            while (g < m0 && a.fcol[k * FCAP + g] != j) ++g;
            if (g < m0) {
                a.farea[k * FCAP + g] += ar;
            } else if (m < FCAP) {
                a.fcol[k * FCAP + m] = j;
                a.farea[k * FCAP + m] = ar;
                ++m;
            } else if (!(fl & CF_FACETS)) {
                fl |= CF_FACETS;
                atomicAdd(o.fail_inst + b, 1);
            }
        }
        a.fcnt[k] = m;
        a.flags[k] = fl;
        if (o.cen)
            for (int q = 0; q < 3; ++q) a.mom[3 * ci + q] += V * o.cen[3 * ci + q];
    }
    if (o.wall)
        for (int p = 0; p < nwp; ++p)
            if (wid[p] >= 0) a.wall[k * nwalls + wid[p]] += o.wall[k * nwp + p];
}

// Marked cells that the float32 pass finished go to the float64 list as well.
__global__ void k_add_precise(int64_t n, Batch bt, int want, const uint8_t *__restrict__ prec, EvalOut o) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || !prec[k]) return;
    const int b = bt.inst[k];
    if (!selected(bt, want, b)) return;
    if (o.flags[k] & (CF_FAIL_MASK | CF_PREC | CF_CAND | CF_EMPTY)) return;  // listed, deferred or empty
    o.flags[k] |= CF_PREC;
    o.fb_list[atomicAdd(o.fb_count, 1)] = (int32_t)k;
    atomicAdd(o.fb_inst + b, 1);
}

// The accumulated sums as the evaluation's outputs; a cell is empty when its parts are.
__global__ void k_piece_final(int64_t n, Batch bt, int want, EvalOut o, int nwalls, const int32_t *__restrict__ perm,
                              const float4 *__restrict__ pos_s, double *__restrict__ cen_out, PieceAcc a) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (!selected(bt, want, bt.inst[k])) return;
    const double V = a.V[k];
    o.V[k] = V;
    o.K[k] = a.K[k];
    const int cnt = a.fcnt[k];
    for (int f = 0; f < cnt; ++f) {
        o.fcol[k * FCAP + f] = a.fcol[k * FCAP + f];
        o.farea[k * FCAP + f] = a.farea[k * FCAP + f];
    }
    o.fcnt[k] = cnt;
    o.flags[k] = (a.flags[k] & ~(uint32_t)CF_EMPTY) | (V > 0.0 ? 0u : (uint32_t)CF_EMPTY);
    if (o.wall)
        for (int w = 0; w < nwalls; ++w) o.wall[k * nwalls + w] = a.wall[k * nwalls + w];
    if (cen_out) {
        const int64_t ci = perm[k];
        const float4 p = pos_s[k];
        const double ps[3] = {(double)p.x, (double)p.y, (double)p.z};
        for (int q = 0; q < 3; ++q) cen_out[3 * ci + q] = V > 0.0 ? a.mom[3 * ci + q] / V : ps[q];
    }
}

// facet counts per caller row
__global__ void k_csr_count(int64_t n, const int32_t *__restrict__ perm, const int32_t *__restrict__ fcnt,
                            int32_t *__restrict__ cnt) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    cnt[perm[k]] = fcnt[k];
}

// facets of grid row k -> caller row perm[k], columns mapped to caller indices and sorted
__global__ void k_csr_fill(int64_t n, const int32_t *__restrict__ perm, const int32_t *__restrict__ fcol,
                           const float *__restrict__ farea, const int32_t *__restrict__ fcnt,
                           const int32_t *__restrict__ start, int32_t *__restrict__ col, float *__restrict__ area,
                           int64_t *__restrict__ row_ptr) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int i = perm[k];
    const int64_t b = start[i];
    const int c = fcnt[k];
    row_ptr[i] = b;
    if (i == 0) row_ptr[n] = start[n];
    for (int f = 0; f < c; ++f) {
        const int v = perm[fcol[k * FCAP + f]];
        const float a = farea[k * FCAP + f];
        int64_t m = b + f - 1;
        while (m >= b && col[m] > v) {
            col[m + 1] = col[m];
            area[m + 1] = area[m];
            --m;
        }
        col[m + 1] = v;
        area[m + 1] = a;
    }
}

__global__ void k_scatter_walls(int64_t n, int nw, const int32_t *__restrict__ perm, const float *__restrict__ ws,
                                float *__restrict__ w) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t i = perm[k];
    for (int a = 0; a < nw; ++a) w[i * nw + a] = ws[k * nw + a];
}

// Default start weights of the selected instances: one common weight per instance,
// the square of 1.2 (3 nu_mean / 4 pi)^(1/3). With equal weights the power diagram is
// the Voronoi diagram, whose cells contain their sites, so no start cell is empty
// (exactly coincident sites aside); per-site radii from nu_i can swallow a light site
// next to a heavy one in a crowded region. ev_nu[4b] holds the instance's sum of nu.
__global__ __launch_bounds__(TILE) void k_default_start(Batch bt, int want, const double *__restrict__ ev_nu,
                                                         double *__restrict__ psi, float4 *__restrict__ pos) {
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    if (!selected(bt, want, b)) return;
    const int i = bt.tile_row[t] + (int)threadIdx.x;
    if (i >= bt.off[b + 1]) return;
    const double nu_mean = ev_nu[4 * b] / (double)(bt.off[b + 1] - bt.off[b]);
    const double r = 1.2 * cbrt(3.0 * nu_mean / (4.0 * 3.14159265358979323846));
    psi[i] = r * r;
    pos[i].w = (float)(r * r);
}

__global__ void k_zero_n(int n, int32_t *__restrict__ a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

// empty cells (V <= 0) of the instances in phase `want`, per instance
__global__ __launch_bounds__(TILE) void k_count_empty(Batch bt, int want, const double *__restrict__ V,
                                                       int32_t *__restrict__ nempty) {
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    if (!selected(bt, want, b)) return;
    const int i = bt.tile_row[t] + (int)threadIdx.x;
    const int e = __syncthreads_count(i < bt.off[b + 1] && !(V[i] > 0.0));
    if (threadIdx.x == 0 && e > 0) atomicAdd(&nempty[b], e);
}

// the repair is meant for a few empty cells: more than 64 and more than 1% of the
// instance's cells send it to the restart
__global__ void k_repair_gate(Batch bt, int want, const int32_t *__restrict__ nempty, int32_t *__restrict__ phase,
                              int32_t *__restrict__ counts) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bt.B || phase[b] != want) return;
    const int64_t nb = bt.off[b + 1] - bt.off[b];
    if (nempty[b] > 64 && 100 * (int64_t)nempty[b] > nb) {
        phase[b] = PH_RESTART;
        atomicSub(&counts[want], 1);
        atomicAdd(&counts[PH_RESTART], 1);
    }
}

// A one-instance start with more than 64 cells, and more than 1% of the cells, certainly
// empty goes to the restart whatever the other passes find (the repair gate's rule). After
// the seed pass every cell's box holds it (the exact cell, or for a crowded cell the cell
// clipped by its nearest sites): an empty box is an empty cell. Such a start skips the
// crowded and float64 passes of its evaluation (their lists are emptied). Every empty-box
// cell gets its volume 0 here (what the crowded pass would write), so the skipped start
// shows its empty cells to the step control and the repair gate.
__global__ __launch_bounds__(TILE) void k_count_empty_boxes(Batch bt, int want, const float4 *__restrict__ box,
                                                             double *__restrict__ V, int32_t *__restrict__ nempty) {
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    if (!selected(bt, want, b)) return;
    const int i = bt.tile_row[t] + (int)threadIdx.x;
    bool e = false;
    if (i < bt.off[b + 1]) {
        const float4 lo = box[2 * (int64_t)i], hi = box[2 * (int64_t)i + 1];
        e = !(lo.x <= hi.x && lo.y <= hi.y && lo.z <= hi.z);
        if (e) V[i] = 0.0;
    }
    const int cnt = __syncthreads_count(e);
    if (threadIdx.x == 0 && cnt > 0) atomicAdd(&nempty[b], cnt);
}

__global__ void k_start_gate(Batch bt, const int32_t *__restrict__ nempty, int32_t *__restrict__ fb_count,
                             int32_t *__restrict__ ovf_count) {
    const int64_t nb = bt.off[1] - bt.off[0];
    if (nempty[0] > 64 && 100 * (int64_t)nempty[0] > nb) {
        *fb_count = 0;
        *ovf_count = 0;
    }
}

// A start cell that is empty gets a weight that puts its site strictly inside every
// power half-space. Let j* maximise psi_j - d_ij^2 over the other sites (value L).
// With w = psi_j*, every bisector has t_ij = (d_ij^2 + w - psi_j) / (2 d_ij) > 0
// (psi_j - d_ij^2 <= L < w), and the bisector with j* is the mid-plane, so the cell
// gets a share of the space between the two sites, not a sliver. A neighbour k keeps
// its own site only while w < psi_k + d_ik^2 (minimum U over the sites searched);
// if psi_j* >= U the weight falls back to (L + U) / 2 when U > L, else to L (the
// nearest bisector then passes through p_i). The result is at least psi_i, the
// default weight if not positive, and at most twice the larger of the default weight
// and the mean weight of the sites searched (a neighbour much heavier than its
// surroundings is left to the full restart). Only sites within 2 r_max can swallow
// p_i or be swallowed. The other weights keep the warm start. One thread per row;
// weights are read from psi and written to psi_out (every row: a copy where nothing
// changes), so the result does not depend on the order in which rows are repaired.
__global__ __launch_bounds__(TILE) void k_repair_empty(Batch bt, int want, const double *__restrict__ V,
                                                        const double *__restrict__ nu, const int32_t *__restrict__ cell_start,
                                                        const double *__restrict__ psi, double *__restrict__ psi_out,
                                                        float4 *__restrict__ pos) {
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    const int i = bt.tile_row[t] + (int)threadIdx.x;
    if (i >= bt.off[b + 1]) return;
    if (!selected(bt, want, b) || V[i] > 0.0) {
        psi_out[i] = psi[i];
        return;
    }
    const double rd2 = pow(1.2 * cbrt(3.0 * nu[i] / (4.0 * 3.14159265358979323846)), 2.0);
    const double p0 = psi[i];
    const GridDesc g = bt.grid[b];
    const float4 pi = pos[i];
    const float reach = 2.0f * (float)bt.rmax[b] * 1.0001f;
    const float pp[3] = {pi.x, pi.y, pi.z};
    int lo3[3], hi3[3];
    for (int a = 0; a < 3; ++a) {
        lo3[a] = max((int)floorf((pp[a] - reach - g.lo[a]) * g.inv_s), 0);
        hi3[a] = min((int)floorf((pp[a] + reach - g.lo[a]) * g.inv_s), g.dim[a] - 1);
    }
    double m = -1e300, wstar = 0.0, u = 1e300, wsum = 0.0;
    int wn = 0;
    for (int ix = lo3[0]; ix <= hi3[0]; ++ix)
        for (int iy = lo3[1]; iy <= hi3[1]; ++iy) {
            const int col = g.base + (ix * g.dim[1] + iy) * g.dim[2];
            const int beg = cell_start[col + lo3[2]], end = cell_start[col + hi3[2] + 1];
            for (int j = beg; j < end; ++j) {
                if (j == i) continue;
                const float4 q = pos[j];  // x, y, z only (.w of repaired rows changes)
                const double dx = (double)q.x - pi.x, dy = (double)q.y - pi.y, dz = (double)q.z - pi.z;
                const double pj = psi[j], d2 = dx * dx + dy * dy + dz * dz;
                if (pj - d2 > m) {
                    m = pj - d2;
                    wstar = pj;
                }
                u = fmin(u, pj + d2);
                wsum += pj;
                ++wn;
            }
        }
    const double cap = fmax(p0, 2.0 * fmax(rd2, wn > 0 ? wsum / wn : 0.0));
    double w = p0;
    if (m > p0) w = wstar < u ? wstar : (u > m ? 0.5 * (m + u) : m);
    if (!(w > 0.0)) w = rd2;
    w = fmin(w, cap);
    psi_out[i] = w;
    pos[i].w = (float)w;
}

// dst row perm[k] = src row k, rows of `chunks` 16-byte words
__global__ void k_scatter_rows(int64_t n, int chunks, const int32_t *__restrict__ perm, const uint4 *__restrict__ src,
                               uint4 *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * chunks) return;
    const int64_t k = e / chunks;
    const int c = (int)(e % chunks);
    dst[(int64_t)perm[k] * chunks + c] = src[k * chunks + c];
}

// Local reach. A bisector of (i, j) cuts ball i only if d_ij < r_i + r_j. For r_j <= r_i
// that is within 2 r_i; for r_j > r_i the site p_i lies within 2 r_j of p_j, so the coarse
// cell of p_i is within 2 r_j of the coarse cell of p_j. Each coarse cell c' therefore
// spreads the largest radius of its sites, rmc[c'], to every coarse cell within 2 rmc[c'],
// and the search reach of site i is r_i + max(r_i, ir[coarse cell of p_i]): where a few
// balls are much larger than the rest, only the sites near them search far. Radii are
// non-negative floats, ordered like their bit patterns (integer atomic max).
__global__ void k_lr_zero(int nc, uint32_t *__restrict__ rmc, uint32_t *__restrict__ ir) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nc) {
        rmc[k] = 0u;
        ir[k] = 0u;
    }
}

__global__ void k_lr_rmax(int64_t n, Batch bt, int want, const float4 *__restrict__ pos, uint32_t *__restrict__ rmc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = bt.inst[i];
    if (!selected(bt, want, b)) return;
    const float4 p = pos[i];
    const float r = p.w > 0.f ? sqrtf(p.w) : 0.f;
    const GridDesc g = bt.cgrid[b];
    atomicMax(rmc + g.base + grid_key(g, p.x, p.y, p.z), __float_as_uint(r));
}

// one thread per coarse cell of the selected instances (instance found by the bases)
__global__ void k_lr_spread(Batch bt, int want, int nc, const uint32_t *__restrict__ rmc, uint32_t *__restrict__ ir) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nc) return;
    const uint32_t rb = rmc[k];
    if (rb == 0u) return;
    int lo = 0, hi = bt.B - 1;  // the instance whose coarse grid holds k
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (bt.cgrid[mid].base <= k) lo = mid; else hi = mid - 1;
    }
    if (!selected(bt, want, lo)) return;
    const GridDesc g = bt.cgrid[lo];
    const int c = k - g.base;
    const int cz = c % g.dim[2], cy = (c / g.dim[2]) % g.dim[1], cx = c / (g.dim[2] * g.dim[1]);
    const int m = (int)ceilf(2.0f * __uint_as_float(rb) * g.inv_s * 1.0001f);
    for (int ix = max(cx - m, 0); ix <= min(cx + m, g.dim[0] - 1); ++ix)
        for (int iy = max(cy - m, 0); iy <= min(cy + m, g.dim[1] - 1); ++iy)
            for (int iz = max(cz - m, 0); iz <= min(cz + m, g.dim[2] - 1); ++iz)
                atomicMax(ir + g.base + (ix * g.dim[1] + iy) * g.dim[2] + iz, rb);
}

__global__ void k_lerp_sites(int64_t n, const float *__restrict__ x0, const float *__restrict__ y0,
                             const float *__restrict__ z0, const float *__restrict__ x1, const float *__restrict__ y1,
                             const float *__restrict__ z1, double t, float *__restrict__ x, float *__restrict__ y,
                             float *__restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // the differences of floats are exact in float64, and p0 + 1 * (p1 - p0) = p1
    x[i] = (float)((double)x0[i] + t * ((double)x1[i] - (double)x0[i]));
    y[i] = (float)((double)y0[i] + t * ((double)y1[i] - (double)y0[i]));
    z[i] = (float)((double)z0[i] + t * ((double)z1[i] - (double)z0[i]));
}

// The power of a moved site at its old cell's centroid c is kept: |c - pb|^2 - psi' =
// |c - pa|^2 - psi gives psi' = psi - 2 d.(c - pa) + |d|^2 with d = pb - pa; the cell then
// moves with its centroid to first order instead of being swept by the site's motion.
__global__ void k_carry_weights(int64_t n, const float *__restrict__ xa, const float *__restrict__ ya,
                                const float *__restrict__ za, const float *__restrict__ xb, const float *__restrict__ yb,
                                const float *__restrict__ zb, const double *__restrict__ cen,
                                const double *__restrict__ psi, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ax = xa[i], ay = ya[i], az = za[i];
    const double dx = (double)xb[i] - ax, dy = (double)yb[i] - ay, dz = (double)zb[i] - az;
    const double cx = cen[3 * i] - ax, cy = cen[3 * i + 1] - ay, cz = cen[3 * i + 2] - az;
    out[i] = psi[i] - 2.0 * (dx * cx + dy * cy + dz * cz) + (dx * dx + dy * dy + dz * dz);
}

inline int nblocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void launch_lerp_sites(hipStream_t st, int64_t n, const float *x0, const float *y0, const float *z0, const float *x1,
                       const float *y1, const float *z1, double t, float *x, float *y, float *z) {
    hipLaunchKernelGGL(k_lerp_sites, dim3(nblocks(n, 256)), dim3(256), 0, st, n, x0, y0, z0, x1, y1, z1, t, x, y, z);
}

void launch_carry_weights(hipStream_t st, int64_t n, const float *xa, const float *ya, const float *za,
                          const float *xb, const float *yb, const float *zb, const double *cen, const double *psi,
                          double *psi_out) {
    hipLaunchKernelGGL(k_carry_weights, dim3(nblocks(n, 256)), dim3(256), 0, st, n, xa, ya, za, xb, yb, zb, cen, psi,
                       psi_out);
}

void launch_local_reach(hipStream_t st, int64_t n, const Batch &bt, int want, int nc_total, const float4 *pos_s,
                        uint32_t *rmc, uint32_t *ir) {
    hipLaunchKernelGGL(k_lr_zero, dim3(nblocks(nc_total, 256)), dim3(256), 0, st, nc_total, rmc, ir);
    hipLaunchKernelGGL(k_lr_rmax, dim3(nblocks(n, 256)), dim3(256), 0, st, n, bt, want, pos_s, rmc);
    hipLaunchKernelGGL(k_lr_spread, dim3(nblocks(nc_total, 256)), dim3(256), 0, st, bt, want, nc_total, rmc, ir);
}

void launch_default_start(hipStream_t st, const Batch &bt, int want, const double *ev_nu, double *psi_s,
                          float4 *pos_s) {
    hipLaunchKernelGGL(k_default_start, dim3(bt.T), dim3(TILE), 0, st, bt, want, ev_nu, psi_s, pos_s);
}

void launch_repair_gate(hipStream_t st, const Batch &bt, int want, const double *V, int32_t *nempty, int32_t *phase,
                        int32_t *counts) {
    hipLaunchKernelGGL(k_zero_n, dim3(nblocks(bt.B, 256)), dim3(256), 0, st, bt.B, nempty);
    hipLaunchKernelGGL(k_count_empty, dim3(bt.T), dim3(TILE), 0, st, bt, want, V, nempty);
    hipLaunchKernelGGL(k_repair_gate, dim3(nblocks(bt.B, 256)), dim3(256), 0, st, bt, want, nempty, phase, counts);
}

void launch_start_gate(hipStream_t st, const Batch &bt, int want, const float4 *box, double *V, int32_t *nempty,
                       int32_t *fb_count, int32_t *ovf_count) {
    hipLaunchKernelGGL(k_zero_n, dim3(1), dim3(256), 0, st, 1, nempty);
    hipLaunchKernelGGL(k_count_empty_boxes, dim3(bt.T), dim3(TILE), 0, st, bt, want, box, V, nempty);
    hipLaunchKernelGGL(k_start_gate, dim3(1), dim3(1), 0, st, bt, nempty, fb_count, ovf_count);
}

void launch_repair_empty(hipStream_t st, const Batch &bt, int want, const double *V, const double *nu_s,
                         const int32_t *cell_start, const double *psi_s, double *psi_out, float4 *pos_s) {
    hipLaunchKernelGGL(k_repair_empty, dim3(bt.T), dim3(TILE), 0, st, bt, want, V, nu_s, cell_start, psi_s, psi_out,
                       pos_s);
}

void launch_fill_inst(hipStream_t st, const Batch &bt, int32_t *inst) {
    hipLaunchKernelGGL(k_fill_inst, dim3(bt.T), dim3(TILE), 0, st, bt, inst);
}

void launch_zero_i32(hipStream_t st, int32_t *p, int64_t count) {
    hipLaunchKernelGGL(k_zero_i32, dim3(nblocks(count, 256)), dim3(256), 0, st, p, count);
}

void launch_zero_f32(hipStream_t st, float *p, int64_t count) {
    hipLaunchKernelGGL(k_zero_f32, dim3(nblocks(count, 256)), dim3(256), 0, st, p, count);
}

void launch_piece_begin(hipStream_t st, bool first, int32_t *fb_count, int32_t *ovf_count, int32_t *ovf_sum) {
    hipLaunchKernelGGL(k_piece_begin, dim3(1), dim3(1), 0, st, first ? 1 : 0, fb_count, ovf_count, ovf_sum);
}

void launch_piece_accum(hipStream_t st, int64_t n, const Batch &bt, int want, bool first, const EvalOut &o,
                        int nw_piece, const int32_t *wid_piece, int nwalls, const int32_t *perm, PieceAcc acc) {
    hipLaunchKernelGGL(k_piece_accum, dim3(nblocks(n, 256)), dim3(256), 0, st, n, bt, want, first ? 1 : 0, o,
                       nw_piece, wid_piece, nwalls, perm, acc);
}

void launch_add_precise(hipStream_t st, int64_t n, const Batch &bt, int want, const uint8_t *prec, EvalOut o) {
    hipLaunchKernelGGL(k_add_precise, dim3(nblocks(n, 256)), dim3(256), 0, st, n, bt, want, prec, o);
}

void launch_piece_final(hipStream_t st, int64_t n, const Batch &bt, int want, const EvalOut &o, int nwalls,
                        const int32_t *perm, const float4 *pos_s, double *cen_out, PieceAcc acc) {
    hipLaunchKernelGGL(k_piece_final, dim3(nblocks(n, 256)), dim3(256), 0, st, n, bt, want, o, nwalls, perm, pos_s,
                       cen_out, acc);
}

void launch_rmax(hipStream_t st, const Batch &bt, int want, const double *psi, double *rmax) {
    hipLaunchKernelGGL(k_rmax_zero, dim3(1), dim3(1024), 0, st, bt, want, rmax);
    hipLaunchKernelGGL(k_rmax_tiles, dim3(bt.T), dim3(TILE), 0, st, bt, want, psi, rmax);
}

void launch_scatter_rows(hipStream_t st, int64_t n, int row_bytes, const int32_t *perm, const void *src, void *dst) {
    const int chunks = row_bytes / 16;
    hipLaunchKernelGGL(k_scatter_rows, dim3(nblocks(n * chunks, 256)), dim3(256), 0, st, n, chunks, perm,
                       (const uint4 *)src, (uint4 *)dst);
}

void launch_scan_i32(hipStream_t st, const int32_t *in, int32_t *out, int n, int32_t *tmp) {
    exclusive_scan(st, in, out, n, tmp);
}

void launch_sort_segments(hipStream_t st, int nseg, const int32_t *start, int32_t *data) {
    hipLaunchKernelGGL(k_sort_cells, dim3(nblocks(nseg, 256)), dim3(256), 0, st, nseg, start, data);
}

void launch_csr_count(hipStream_t st, int64_t n, const int32_t *perm, const int32_t *fcnt, int32_t *cnt_orig) {
    hipLaunchKernelGGL(k_csr_count, dim3(nblocks(n, 256)), dim3(256), 0, st, n, perm, fcnt, cnt_orig);
}

void launch_csr_fill(hipStream_t st, int64_t n, const int32_t *perm, const int32_t *fcol, const float *farea,
                     const int32_t *fcnt, const int32_t *start, int32_t *col, float *area, int64_t *row_ptr) {
    hipLaunchKernelGGL(k_csr_fill, dim3(nblocks(n, 256)), dim3(256), 0, st, n, perm, fcol, farea, fcnt, start, col,
                       area, row_ptr);
}

void launch_scatter_walls(hipStream_t st, int64_t n, int nw, const int32_t *perm, const float *wall_s, float *wall) {
    hipLaunchKernelGGL(k_scatter_walls, dim3(nblocks(n, 256)), dim3(256), 0, st, n, nw, perm, wall_s, wall);
}

void launch_gather_sites(hipStream_t st, int64_t n, const float *x, const float *y, const float *z,
                         const double *psi, float4 *pos_orig) {
    hipLaunchKernelGGL(k_gather_sites, dim3(nblocks(n, 256)), dim3(256), 0, st, n, x, y, z, psi, pos_orig);
}

// Counting sort by (instance grid base + cell): cell_count is cleared with a
// kernel, not a memset, so the sequence can be captured in a graph.
void launch_grid_build(hipStream_t st, int64_t n, const Batch &bt, int ncell_total, const float4 *pos_orig,
                       int32_t *keys, int32_t *cell_count, int32_t *cell_start, int32_t *scan_tmp, int32_t *perm,
                       int32_t *cursor) {
    launch_zero_i32(st, cell_count, ncell_total);
    hipLaunchKernelGGL(k_keys_count, dim3(nblocks(n, 256)), dim3(256), 0, st, n, bt, pos_orig, keys, cell_count);
    exclusive_scan(st, cell_count, cell_start, ncell_total, scan_tmp);
    (void)hipMemcpyAsync(cursor, cell_start, sizeof(int32_t) * (size_t)ncell_total, hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(k_scatter, dim3(nblocks(n, 256)), dim3(256), 0, st, n, keys, cursor, perm);
    hipLaunchKernelGGL(k_sort_cells, dim3(nblocks(ncell_total, 256)), dim3(256), 0, st, ncell_total, cell_start,
                       perm);
}

void launch_permute_in(hipStream_t st, int64_t n, const int32_t *perm, const float4 *pos_orig, const double *psi,
                       const double *nu, float4 *pos_s, double *psi_s, double *nu_s) {
    hipLaunchKernelGGL(k_permute_in, dim3(nblocks(n, 256)), dim3(256), 0, st, n, perm, pos_orig, psi, nu, pos_s,
                       psi_s, nu_s);
}

void launch_psi_shadow(hipStream_t st, int64_t n, const double *psi_s, float4 *pos_s) {
    hipLaunchKernelGGL(k_psi_shadow, dim3(nblocks(n, 256)), dim3(256), 0, st, n, psi_s, pos_s);
}

void launch_scatter_out_f64(hipStream_t st, int64_t n, const int32_t *perm, const double *src_s, double *dst) {
    hipLaunchKernelGGL(k_scatter_out, dim3(nblocks(n, 256)), dim3(256), 0, st, n, perm, src_s, dst);
}

void launch_validate(hipStream_t st, int64_t n, const Batch &bt, const float *x, const float *y, const float *z,
                     const double *psi, const double *nu, int32_t *bad_inst) {
    hipLaunchKernelGGL(k_validate, dim3(nblocks(n, 256)), dim3(256), 0, st, n, bt, x, y, z, psi, nu, bad_inst);
}

}  // namespace lagot
