// newton.hip -- Hessian assembly (hess_assemble) and the Jacobi-PCG / damped
// Newton building blocks (ot_newton) of Algorithm 1.
//
// Gradient (section 3.1): g_i = nu_i - V_i. Hessian (eq. (2)): the solve uses
// -Hess K = D - W with W_ij = Abar_ij / (2 |p_j - p_i|) over the restricted
// Laguerre facets and D_i = sum_j W_ij + K_i / (2 sqrt(psi_i)); box walls do not
// move with psi and do not enter. Abar is the mean of the facet area seen from
// the two cells (float32 geometry is not bit-symmetric); a facet seen from one
// side only keeps that side's value, in both rows (union pattern).
//
// Precision: facet areas and matrix values are float32; V, K, the diagonal,
// every vector of the conjugate gradients, every inner product and every
// reduction are float64, with fixed-order two-level reductions (deterministic).
//
// Batches: every kernel serves B independent instances at once. Row kernels run
// over the tile table (a tile lies in one instance) and skip instances whose
// control phase is not the one a launch selects; per-instance reductions sum the
// instance's run of tile partials; the step-size control of Algorithm 1 runs per
// instance in small control kernels, so the host only reads phase counts.
#include <algorithm>

#include "lagot_internal.h"

namespace lagot {
namespace {

constexpr int RB = 256;  // threads per block of the vector kernels

__device__ inline double block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
    return s;
}

__device__ inline double block_max(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double s = sh[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) s = fmax(s, sh[k]);
    return s;
}

__device__ inline double block_min(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double s = sh[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) s = fmin(s, sh[k]);
    return s;
}

// ---- per-instance evaluation statistics ----------------------------------------
// part[q*T + t], q = 0..3: sum V, max |V-nu|/nu, sum (nu-V)^2, min V over tile t
__global__ __launch_bounds__(TILE) void k_eval_partial(Batch bt, int want, const double *__restrict__ V,
                                                        const double *__restrict__ nu, double *__restrict__ part) {
    __shared__ double sh[TILE / 64];
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    if (!selected(bt, want, b)) return;
    const int i = bt.tile_row[t] + (int)threadIdx.x;
    double sv = 0.0, mx = 0.0, g2 = 0.0, mn = 1e300;
    if (i < bt.off[b + 1]) {
        const double v = V[i], c = nu[i];
        sv = v;
        mx = fabs(v - c) / c;
        g2 = (c - v) * (c - v);
        mn = v;
    }
    sv = block_sum(sv, sh);
    mx = block_max(mx, sh);
    g2 = block_sum(g2, sh);
    mn = block_min(mn, sh);
    if (threadIdx.x == 0) {
        const int T = bt.T;
        part[t] = sv;
        part[T + t] = mx;
        part[2 * T + t] = g2;
        part[3 * T + t] = mn;
    }
}

__global__ __launch_bounds__(RB) void k_eval_final(Batch bt, int want, const double *__restrict__ part,
                                                    double *__restrict__ ev) {
    __shared__ double sh[RB / 64];
    const int b = blockIdx.x;
    if (!selected(bt, want, b)) return;
    const int T = bt.T, t0 = bt.first_tile[b], t1 = bt.first_tile[b + 1];
    double sv = 0.0, mx = 0.0, g2 = 0.0, mn = 1e300;
    for (int t = t0 + (int)threadIdx.x; t < t1; t += RB) {
        sv += part[t];
        mx = fmax(mx, part[T + t]);
        g2 += part[2 * T + t];
        mn = fmin(mn, part[3 * T + t]);
    }
    sv = block_sum(sv, sh);
    mx = block_max(mx, sh);
    g2 = block_sum(g2, sh);
    mn = block_min(mn, sh);
    if (threadIdx.x == 0) {
        ev[4 * b + 0] = sv;
        ev[4 * b + 1] = mx;
        ev[4 * b + 2] = sqrt(g2);
        ev[4 * b + 3] = mn;
    }
}

// ---- Hessian assembly ---------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_hess_begin(Batch bt, int want, int32_t *__restrict__ xcnt,
                                                      int32_t *__restrict__ herr) {
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    if (!selected(bt, want, b)) return;
    const int i = bt.tile_row[t] + (int)threadIdx.x;
    if (i < bt.off[b + 1]) xcnt[i] = 0;
    if (t == bt.first_tile[b] && threadIdx.x == 0) herr[b] = 0;
}

// Row i of -Hess K: one entry per facet of cell i; a facet that cell j does not
// list is appended to row j as well (union pattern). One thread per facet slot;
// the partner row is read with 16-byte loads and searched in registers.
__global__ void k_hess_assemble(int64_t n, Batch bt, int want, const float4 *__restrict__ pos,
                                const int32_t *__restrict__ fcol, const float *__restrict__ farea,
                                const int32_t *__restrict__ fcnt, int32_t *__restrict__ hcol,
                                float *__restrict__ hval, int32_t *__restrict__ xcnt, int32_t *__restrict__ herr) {
    const int64_t t = (int64_t)xcd_block((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t i = t / 16;
    const int f0 = (int)(t & 15);
    if (i >= n) return;
    const int b = bt.inst[i];
    if (!selected(bt, want, b)) return;
    const int ci = fcnt[i];
    for (int f = f0; f < ci; f += 16) {
        const int j = fcol[i * FCAP + f];
        const float a = farea[i * FCAP + f];
        const int cj = fcnt[j];
        const int4 *rowj = reinterpret_cast<const int4 *>(fcol + (int64_t)j * FCAP);
        int pos2 = -1;
        for (int q = 0; q < (cj + 3) / 4 && pos2 < 0; ++q) {
            const int4 v = rowj[q];
            if (v.x == (int32_t)i && 4 * q + 0 < cj) pos2 = 4 * q + 0;
            else if (v.y == (int32_t)i && 4 * q + 1 < cj) pos2 = 4 * q + 1;
            else if (v.z == (int32_t)i && 4 * q + 2 < cj) pos2 = 4 * q + 2;
            else if (v.w == (int32_t)i && 4 * q + 3 < cj) pos2 = 4 * q + 3;
        }
        const float a2 = pos2 >= 0 ? farea[(int64_t)j * FCAP + pos2] : -1.f;
        const float4 pi = pos[i], pj = pos[j];
        const float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
        const float d = sqrtf(dx * dx + dy * dy + dz * dz);
        const float abar = (a2 >= 0.f) ? 0.5f * (a + a2) : a;
        const float w = abar / (2.f * d);
        hcol[i * FCAP + f] = j;
        hval[i * FCAP + f] = w;
        if (a2 < 0.f) {
            const int x = atomicAdd(&xcnt[j], 1);
            const int slot = cj + x;
            if (slot < FCAP) {
                hcol[(int64_t)j * FCAP + slot] = (int32_t)i;
                hval[(int64_t)j * FCAP + slot] = w;
            } else {
                atomicAdd(herr + b, 1);
            }
        }
    }
}

// Row length, diagonal; the entries appended by the union pattern arrive in atomic
// order and are sorted by column here, so every later sum over the row is in a fixed
// order (deterministic results). One block per tile. With ent given, the tile's rows
// are also packed back to back as (column, float bits of the value) pairs into the
// tile's region ent[t * TILE * FCAP ...], row i starting at hrow[i].x within it
// (hrow[i].y = its length): the conjugate gradients then read every row's entries
// from consecutive addresses instead of one 64-entry block per row.
__global__ __launch_bounds__(TILE) void k_hess_finish(Batch bt, int want, const double *__restrict__ psi,
                                                       const double *__restrict__ K, const int32_t *__restrict__ fcnt,
                                                       const int32_t *__restrict__ xcnt, int32_t *__restrict__ hcnt,
                                                       int32_t *__restrict__ hcol, float *__restrict__ hval,
                                                       double *__restrict__ diag, int2 *__restrict__ hrow,
                                                       int2 *__restrict__ ent) {
    __shared__ int wsum[TILE / 64];
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    if (!selected(bt, want, b)) return;
    const int64_t i = bt.tile_row[t] + (int)threadIdx.x;
    const bool has = i < bt.off[b + 1];
    int c = 0;
    if (has) {
        const int f0 = fcnt[i];
        c = min(f0 + xcnt[i], FCAP);
        hcnt[i] = c;
        int32_t *cr = hcol + i * FCAP;
        float *vr = hval + i * FCAP;
        for (int a = f0 + 1; a < c; ++a) {
            const int32_t key = cr[a];
            const float v = vr[a];
            int q = a - 1;
            while (q >= f0 && cr[q] > key) {
                cr[q + 1] = cr[q];
                vr[q + 1] = vr[q];
                --q;
            }
            cr[q + 1] = key;
            vr[q + 1] = v;
        }
        double s = 0.0;
        for (int f = 0; f < c; ++f) s += (double)vr[f];
        const double p = psi[i];
        if (p > 0.0) s += K[i] / (2.0 * sqrt(p));
        diag[i] = s;
    }
    if (!ent) return;
    // exclusive scan of the row lengths over the tile
    int incl = c;
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int excl = incl - c;
    for (int k = 0; k < w; ++k) excl += wsum[k];
    if (!has) return;
    hrow[i] = make_int2(excl, c);
    const int32_t *cr = hcol + i * FCAP;
    const float *vr = hval + i * FCAP;
    int2 *er = ent + (int64_t)t * (TILE * FCAP) + excl;
    for (int f = 0; f < c; ++f) er[f] = make_int2(cr[f], __float_as_int(vr[f]));
}

// ---- Jacobi-PCG, one kernel per iteration (Chronopoulos-Gear form) ------------
// Preconditioned CG on (D - W) x = g with M = diag(D - W). With u = M^-1 r and
// w = A u, one iteration k needs only gamma_k = (r_k, u_k) and
// delta_k = (w_k, u_k), both summed in the same pass:
//   beta_k = gamma_k / gamma_{k-1},  alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1})
//   p_k = u_k + beta_k p_{k-1},  s_k = w_k + beta_k s_{k-1}  (= A p_k)
//   x_{k+1} = x_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k s_k,  w_{k+1} = A u_{k+1}.
// A row needs u_{k+1} of its neighbours; it rebuilds it from their stored r_k, w_k,
// s_{k-1} and the two scalars (same arithmetic as the owner), so no grid-wide
// barrier separates the vector update from the product. Every block recomputes
// the scalars from its instance's tile partials in a fixed order: deterministic,
// no atomics, no device-scope fences (a device-scope fence writes back the XCD's
// L2 on this part). The stop test is ||r_k|| <= rtol ||r_0||.
// Block shapes of the conjugate-gradient kernels: LANES lanes per row (rows hold
// ~6-20 entries) and SUB rows per block (a block covers a sub-tile; partials are kept
// per sub-tile, so SUB sets how many partials every block sums). Chosen per context
// (lagot_set_cg_shape / the autotuner); the partial buffers are sized for SUB = 64.
constexpr int PF = 4;              // row entries per lane fetched before the scalars are known
// An instance with at most this many partials has every block of an iteration sum them
// (no extra launch); larger ones get them summed once per iteration by k_cg_scalars.
constexpr int CG_SUM_IN_BLOCK = 2048;
constexpr int SCB = 1024;          // threads of k_cg_scalars

// Four fixed-order sums over the partials t0..t1-1 (any block size, multiple of 64;
// sh holds one row per wave).
__device__ inline void sum_range(const double *a, const double *b, const double *c, const double *d, int t0, int t1,
                                 double *out, double (*sh)[4]) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = t0 + (int)threadIdx.x; t < t1; t += (int)blockDim.x) {
        s[0] += a[t];
        s[1] += b[t];
        s[2] += c[t];
        s[3] += d[t];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        for (int o = 32; o > 0; o >>= 1) s[q] += __shfl_xor(s[q], o, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 4; ++q) sh[w][q] = s[q];
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
        double v = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) v += sh[k][q];
        out[q] = v;
    }
}

__device__ inline void block_sum3(double &a, double &b, double &c, double (*sh)[4]) {
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sh[w][0] = a;
        sh[w][1] = b;
        sh[w][2] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
        a += sh[k][0];
        b += sh[k][1];
        c += sh[k][2];
    }
}

__device__ inline RWSD load_rwsd(const RWSD *a, int i) {
    const double2 *p = reinterpret_cast<const double2 *>(a + i);
    const double2 lo = p[0], hi = p[1];
    return RWSD{lo.x, lo.y, hi.x, hi.y};
}
__device__ inline void store_rwsd(RWSD *a, int i, double r, double w, double s, double d) {
    double2 *p = reinterpret_cast<double2 *>(a + i);
    p[0] = make_double2(r, w);
    p[1] = make_double2(s, d);
}

// partial slots (per sub-tile, NS = SPT * T of them): gamma[2][NS], delta[2][NS],
// rho[2][NS], rho0[NS]
__device__ inline double *P_GAM(const CgBufs &cg, int NS, int slot) { return cg.part + slot * NS; }
__device__ inline double *P_DEL(const CgBufs &cg, int NS, int slot) { return cg.part + (2 + slot) * NS; }
__device__ inline double *P_RHO(const CgBufs &cg, int NS, int slot) { return cg.part + (4 + slot) * NS; }
__device__ inline double *P_RHO0(const CgBufs &cg, int NS) { return cg.part + 6 * NS; }

// r_0 = g = nu - V (0 on empty rows), u_0 = r_0 / D, w_0 = A u_0, s_{-1} = p_{-1} = x_0 = 0
template <int LANES, int SUB>
__global__ __launch_bounds__(LANES * SUB) void k_cg_init(Batch bt, const double *__restrict__ V, const double *__restrict__ nu,
                                                 const double *__restrict__ diag, const int2 *__restrict__ hrow,
                                                 const int2 *__restrict__ ent, CgBufs cg) {
    constexpr int SPT = TILE / SUB;
    __shared__ double sh[LANES * SUB / 64][4];
    const int q = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int t = q / SPT;
    if (q == 0 && threadIdx.x == 0) *cg.kbase = 0;
    const int b = bt.tile_inst[t];
    if (bt.phase[b] != PH_ACTIVE) return;
    const int NS = SPT * bt.T;
    const int l = threadIdx.x & (LANES - 1);
    const int row = bt.tile_row[t] + (q % SPT) * SUB + (int)(threadIdx.x / LANES);
    const bool has = row < bt.off[b + 1];
    double acc = 0.0;
    if (has) {
        const int2 hr = hrow[row];
        const int2 *er = ent + (int64_t)t * (TILE * FCAP) + hr.x;
        for (int f = l; f < hr.y; f += LANES) {
            const int2 e = er[f];
            const double dj = diag[e.x];
            const double uj = dj > 0.0 ? (nu[e.x] - V[e.x]) / dj : 0.0;
            acc += (double)__int_as_float(e.y) * uj;
        }
    }
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LANES);
    double gp = 0.0, dp = 0.0, rp = 0.0;
    if (has && l == 0) {
        const double d = diag[row];
        const double g = d > 0.0 ? nu[row] - V[row] : 0.0;
        const double u = d > 0.0 ? (nu[row] - V[row]) / d : 0.0;
        const double w = d * u - acc;
        store_rwsd(cg.rws[0], row, g, w, 0.0, d);
        cg.p[row] = 0.0;
        cg.x[row] = 0.0;
        gp = g * u;
        dp = w * u;
        rp = g * g;
    }
    block_sum3(gp, dp, rp, sh);
    if (threadIdx.x == 0) {
        P_GAM(cg, NS, 0)[q] = gp;
        P_DEL(cg, NS, 0)[q] = dp;
        P_RHO(cg, NS, 0)[q] = rp;
        P_RHO0(cg, NS)[q] = rp;
    }
    if (q == SPT * bt.first_tile[b] && threadIdx.x == 0) {
        int32_t *st = cg.cgst + 4 * b;
        st[0] = 0;
        st[1] = 0;
        st[2] = 0;
        st[3] = 0;
    }
}

// Iteration k = *kbase + m (the host advances kbase after a chunk of launches, so a
// chunk has fixed arguments and can be replayed as a graph). The loads that do not
// depend on the iteration's scalars (the row's entries, the neighbours' r, w, s, D)
// are issued before the partial sums that give the scalars, so their latencies overlap.
template <int LANES, int SUB>
__global__ __launch_bounds__(LANES * SUB) void k_cg_iter(Batch bt, int m, double rtol2, int cap,
                                                 const int2 *__restrict__ hrow, const int2 *__restrict__ ent,
                                                 CgBufs cg) {
    constexpr int SPT = TILE / SUB;
    __shared__ double sh[LANES * SUB / 64][4];
    const int q = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int t = q / SPT;
    const int b = bt.tile_inst[t];
    const int row = bt.tile_row[t] + (q % SPT) * SUB + (int)(threadIdx.x / LANES);
    const int k = *cg.kbase + m;
    int32_t *st = cg.cgst + 4 * b;
    const int4 st4 = *reinterpret_cast<const int4 *>(st);
    if (bt.phase[b] != PH_ACTIVE || st4.y != 0 || st4.z != 0 || k >= cap) return;
    const int NS = SPT * bt.T;
    const int t0 = SPT * bt.first_tile[b];
    const int end = bt.off[b + 1];
    const int cur = k & 1, nxt = cur ^ 1;
    const double2 prev = *reinterpret_cast<const double2 *>(cg.cgs + 4 * b + 2 * nxt);  // alpha, gamma of k-1
    const RWSD *cur_rec = cg.rws[cur];
    const int l = threadIdx.x & (LANES - 1);
    const bool has = row < end;
    // scalar-independent loads
    int c = 0;
    RWSD own{0.0, 0.0, 0.0, 0.0};
    double pk_1 = 0.0, xk = 0.0;
    int2 hr = make_int2(0, 0);
    float vv[PF];
    RWSD nb[PF];
    if (has) {
        hr = hrow[row];
        c = hr.y;
        own = load_rwsd(cur_rec, row);
        pk_1 = cg.p[row];
        xk = cg.x[row];
    }
    const int2 *er = ent + (int64_t)t * (TILE * FCAP) + hr.x;
#pragma unroll
    for (int e = 0; e < PF; ++e) {
        const int f = l + LANES * e;
        vv[e] = 0.f;
        nb[e] = RWSD{0.0, 0.0, 0.0, 0.0};
        if (f < c) {
            const int2 en = er[f];
            vv[e] = __int_as_float(en.y);
            nb[e] = load_rwsd(cur_rec, en.x);
        }
    }
    const double d = own.d, rk = own.r, wk = own.w, sk_1 = own.s;
    // the iteration's scalars: summed by the block itself from the instance's partials when
    // they are few, else once per iteration by k_cg_scalars
    double gam, del, rho, rho0;
    const int t1 = SPT * bt.first_tile[b + 1];
    if (t1 - t0 <= CG_SUM_IN_BLOCK) {
        double S[4];
        sum_range(P_GAM(cg, NS, cur), P_DEL(cg, NS, cur), P_RHO(cg, NS, cur), P_RHO0(cg, NS), t0, t1, S, sh);
        gam = S[0];
        del = S[1];
        rho = S[2];
        rho0 = S[3];
    } else {
        const double2 s01 = *reinterpret_cast<const double2 *>(cg.sc + 8 * b + 4 * cur);
        const double2 s23 = *reinterpret_cast<const double2 *>(cg.sc + 8 * b + 4 * cur + 2);
        gam = s01.x;
        del = s01.y;
        rho = s23.x;
        rho0 = s23.y;
    }
    const bool lead = q == t0 && threadIdx.x == 0;
    if (rho <= rtol2 * rho0) {
        if (lead) {
            st[2] = 1;
            st[0] = k;
        }
        return;
    }
    double alpha, beta = 0.0;
    if (k == 0) {
        alpha = gam / del;
    } else {
        beta = gam / prev.y;
        alpha = gam / (del - beta * gam / prev.x);
    }
    if (!(alpha > 0.0) || !(alpha < 1e300)) {  // non-positive curvature (or NaN)
        if (lead) {
            st[1] = 1;
            st[0] = k;
        }
        return;
    }
    if (lead) {
        cg.cgs[4 * b + 2 * cur] = alpha;
        cg.cgs[4 * b + 2 * cur + 1] = gam;
        st[0] = k + 1;
    }
    // u_{k+1} of a neighbour from its stored r_k, w_k, s_{k-1} (same arithmetic as its owner)
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < PF; ++e) {
        const double s1 = fma(beta, nb[e].s, nb[e].w);
        const double uj = nb[e].d > 0.0 ? fma(-alpha, s1, nb[e].r) / nb[e].d : 0.0;
        acc += (double)vv[e] * uj;
    }
    for (int f = l + LANES * PF; f < c; f += LANES) {
        const int2 en = er[f];
        const RWSD o = load_rwsd(cur_rec, en.x);
        const double s1 = fma(beta, o.s, o.w);
        const double uj = o.d > 0.0 ? fma(-alpha, s1, o.r) / o.d : 0.0;
        acc += (double)__int_as_float(en.y) * uj;
    }
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LANES);
    double gp = 0.0, dp = 0.0, rp = 0.0;
    if (has && l == 0) {
        const double uk = d > 0.0 ? rk / d : 0.0;
        const double pk = fma(beta, pk_1, uk);
        const double sk = fma(beta, sk_1, wk);
        cg.x[row] = fma(alpha, pk, xk);
        const double r1 = fma(-alpha, sk, rk);
        const double u1 = d > 0.0 ? r1 / d : 0.0;
        const double w1 = d * u1 - acc;
        cg.p[row] = pk;
        store_rwsd(cg.rws[nxt], row, r1, w1, sk, d);
        gp = r1 * u1;
        dp = w1 * u1;
        rp = r1 * r1;
    }
    block_sum3(gp, dp, rp, sh);
    if (threadIdx.x == 0) {
        P_GAM(cg, NS, nxt)[q] = gp;
        P_DEL(cg, NS, nxt)[q] = dp;
        P_RHO(cg, NS, nxt)[q] = rp;
    }
}

// ---- the same iteration in two launches (large instances) ----------------------------
// k_cg_iter forms a neighbour's u_{k+1} from its whole (r, w, s, D) record: one launch per
// iteration, but 32 bytes gathered per matrix entry, which at millions of rows no longer
// stay in L2. Split, the first launch does the scalars and every row's own update and
// writes u_{k+1} (8 bytes per row), the second the product w_{k+1} = A u_{k+1} from those
// values. Same arithmetic per row (u_{k+1} bit for bit); the partial sums are taken in
// other block shapes, so the scalars differ from k_cg_iter's in the last bits.
template <int SUB>
__global__ __launch_bounds__(SUB) void k_cg_update(Batch bt, int m, double rtol2, int cap, CgBufs cg) {
    constexpr int SPT = TILE / SUB;
    __shared__ double sh[SUB / 64][4];
    const int q = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int t = q / SPT;
    const int b = bt.tile_inst[t];
    const int row = bt.tile_row[t] + (q % SPT) * SUB + (int)threadIdx.x;
    const int k = *cg.kbase + m;
    int32_t *st = cg.cgst + 4 * b;
    const int4 st4 = *reinterpret_cast<const int4 *>(st);
    if (bt.phase[b] != PH_ACTIVE || st4.y != 0 || st4.z != 0 || k >= cap) return;
    const int NS = SPT * bt.T;
    const int t0 = SPT * bt.first_tile[b], t1 = SPT * bt.first_tile[b + 1];
    const int end = bt.off[b + 1];
    const int cur = k & 1, nxt = cur ^ 1;
    const double2 prev = *reinterpret_cast<const double2 *>(cg.cgs + 4 * b + 2 * nxt);  // alpha, gamma of k-1
    const bool has = row < end;
    RWSD own{0.0, 0.0, 0.0, 0.0};
    double pk_1 = 0.0, xk = 0.0;
    if (has) {
        own = load_rwsd(cg.rws[cur], row);
        pk_1 = cg.p[row];
        xk = cg.x[row];
    }
    double gam, del, rho, rho0;
    if (t1 - t0 <= CG_SUM_IN_BLOCK) {
        double S[4];
        sum_range(P_GAM(cg, NS, cur), P_DEL(cg, NS, cur), P_RHO(cg, NS, cur), P_RHO0(cg, NS), t0, t1, S, sh);
        gam = S[0];
        del = S[1];
        rho = S[2];
        rho0 = S[3];
    } else {
        const double2 s01 = *reinterpret_cast<const double2 *>(cg.sc + 8 * b + 4 * cur);
        const double2 s23 = *reinterpret_cast<const double2 *>(cg.sc + 8 * b + 4 * cur + 2);
        gam = s01.x;
        del = s01.y;
        rho = s23.x;
        rho0 = s23.y;
    }
    const bool lead = q == t0 && threadIdx.x == 0;
    if (rho <= rtol2 * rho0) {
        if (lead) {
            st[2] = 1;
            st[0] = k;
        }
        return;
    }
    double alpha, beta = 0.0;
    if (k == 0) {
        alpha = gam / del;
    } else {
        beta = gam / prev.y;
        alpha = gam / (del - beta * gam / prev.x);
    }
    if (!(alpha > 0.0) || !(alpha < 1e300)) {  // non-positive curvature (or NaN)
        if (lead) {
            st[1] = 1;
            st[0] = k;
        }
        return;
    }
    if (lead) {
        cg.cgs[4 * b + 2 * cur] = alpha;
        cg.cgs[4 * b + 2 * cur + 1] = gam;
        st[0] = k + 1;
    }
    double gp = 0.0, rp = 0.0, unused = 0.0;
    if (has) {
        const double d = own.d;
        const double uk = d > 0.0 ? own.r / d : 0.0;
        const double pk = fma(beta, pk_1, uk);
        const double sk = fma(beta, own.s, own.w);
        cg.x[row] = fma(alpha, pk, xk);
        const double r1 = fma(-alpha, sk, own.r);
        const double u1 = d > 0.0 ? r1 / d : 0.0;
        cg.p[row] = pk;
        cg.u[row] = u1;
        // r, s and D of the new record; its w comes from the product
        double *rec = reinterpret_cast<double *>(cg.rws[nxt] + row);
        rec[0] = r1;
        *reinterpret_cast<double2 *>(rec + 2) = make_double2(sk, d);
        gp = r1 * u1;
        rp = r1 * r1;
    }
    block_sum3(gp, rp, unused, sh);
    if (threadIdx.x == 0) {
        P_GAM(cg, NS, nxt)[q] = gp;
        P_RHO(cg, NS, nxt)[q] = rp;
    }
}

// second launch of the split iteration: w_{k+1} = D u_{k+1} - sum_j v_ij u_{k+1,j} and the
// delta partials, for the instances whose update ran (iteration count advanced to k + 1)
template <int LANES, int SUB>
__global__ __launch_bounds__(LANES * SUB) void k_cg_product(Batch bt, int m, int cap, const int2 *__restrict__ hrow,
                                                    const int2 *__restrict__ ent, CgBufs cg) {
    constexpr int SPT = TILE / SUB;
    __shared__ double sh[LANES * SUB / 64][4];
    const int q = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int t = q / SPT;
    const int b = bt.tile_inst[t];
    const int row = bt.tile_row[t] + (q % SPT) * SUB + (int)(threadIdx.x / LANES);
    const int k = *cg.kbase + m;
    const int4 st4 = *reinterpret_cast<const int4 *>(cg.cgst + 4 * b);
    if (bt.phase[b] != PH_ACTIVE || st4.y != 0 || st4.z != 0 || st4.x != k + 1 || k >= cap) return;
    const int NS = SPT * bt.T;
    const int nxt = (k & 1) ^ 1;
    const int l = threadIdx.x & (LANES - 1);
    const bool has = row < bt.off[b + 1];
    int2 hr = make_int2(0, 0);
    if (has) hr = hrow[row];
    const int2 *er = ent + (int64_t)t * (TILE * FCAP) + hr.x;
    double acc = 0.0;
    for (int f = l; f < hr.y; f += LANES) {
        const int2 en = er[f];
        acc += (double)__int_as_float(en.y) * cg.u[en.x];
    }
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LANES);
    double dp = 0.0, u1 = 0.0, z1 = 0.0;
    if (has && l == 0) {
        double *rec = reinterpret_cast<double *>(cg.rws[nxt] + row);
        u1 = cg.u[row];
        const double w1 = rec[3] * u1 - acc;
        rec[1] = w1;
        dp = w1 * u1;
    }
    block_sum3(dp, u1, z1, sh);
    if (threadIdx.x == 0) P_DEL(cg, NS, nxt)[q] = dp;
}

// The scalars gamma, delta, rho (and rho0) of the next iteration: the instance's sub-tile
// partials of the slot just written, summed once, in a fixed order (deterministic), by
// one block per instance, instead of by every block of the next iteration (which made
// the reduction quadratic in the number of tiles).
__global__ __launch_bounds__(SCB) void k_cg_scalars(Batch bt, int spt, int m, int cap, CgBufs cg) {
    __shared__ double sh[SCB / 64][4];
    const int b = blockIdx.x;
    if (bt.phase[b] != PH_ACTIVE) return;
    if (spt * (bt.first_tile[b + 1] - bt.first_tile[b]) <= CG_SUM_IN_BLOCK) return;  // summed in the blocks
    int slot = 0;
    if (m >= 0) {
        const int32_t *st = cg.cgst + 4 * b;
        const int k = *cg.kbase + m;
        if (st[1] != 0 || st[2] != 0 || k >= cap) return;  // iteration k wrote no partials
        slot = (k + 1) & 1;
    }
    const int NS = spt * bt.T;
    double S[4];
    sum_range(P_GAM(cg, NS, slot), P_DEL(cg, NS, slot), P_RHO(cg, NS, slot), P_RHO0(cg, NS),
              spt * bt.first_tile[b], spt * bt.first_tile[b + 1], S, sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) cg.sc[8 * b + 4 * slot + q] = S[q];
}

// After a chunk: advance kbase; count instances still iterating; the most iterations
// any active instance has done (sizes the next solve's chunks).
__global__ __launch_bounds__(1024) void k_cg_advance(Batch bt, int chunk, int cap, CgBufs cg) {
    __shared__ int cnt, mx;
    if (threadIdx.x == 0) cnt = mx = 0;
    __syncthreads();
    int mine = 0, most = 0;
    for (int b = threadIdx.x; b < bt.B; b += 1024) {
        const int32_t *st = cg.cgst + 4 * b;
        if (bt.phase[b] != PH_ACTIVE) continue;
        mine += st[1] == 0 && st[2] == 0 && st[0] < cap;
        most = max(most, st[0]);
    }
    if (mine) atomicAdd(&cnt, mine);
    if (most) atomicMax(&mx, most);
    __syncthreads();
    if (threadIdx.x == 0) {
        *cg.kbase += chunk;
        *cg.remaining = cnt;
        *cg.maxit = mx;
    }
}

// End of the direction solve: ACTIVE -> TRIAL with alpha = 1 (with step_start:
// min(1, 2 x the last accepted step length)), or FAILED.
__global__ __launch_bounds__(RB) void k_cg_finish(Batch bt, int SPT, double rtol2, int step_start, CgBufs cg,
                                                   const int32_t *__restrict__ herr, InstCtl *__restrict__ ctl,
                                                   int32_t *__restrict__ phase) {
    __shared__ double sh[RB / 64][4];
    const int b = blockIdx.x;
    if (phase[b] != PH_ACTIVE) return;
    const int32_t *st = cg.cgst + 4 * b;
    const int it = st[0];
    const int NS = SPT * bt.T;
    double S[4];
    sum_range(P_RHO(cg, NS, it & 1), P_RHO0(cg, NS), P_RHO0(cg, NS), P_RHO0(cg, NS), SPT * bt.first_tile[b],
              SPT * bt.first_tile[b + 1], S, sh);
    if (threadIdx.x != 0) return;
    InstCtl &c = ctl[b];
    c.cg_iters += it;
    // a breakdown is harmless once the residual already meets the tolerance
    const bool singular = st[1] != 0 && !(S[0] <= rtol2 * S[1]);
    if (herr[b] != 0) {
        c.status = -5;  // LAGOT_ECAPACITY
        phase[b] = PH_FAILED;
    } else if (singular) {
        c.status = -6;  // LAGOT_ESINGULAR
        phase[b] = PH_FAILED;
    } else {
        c.alpha = step_start ? fmin(1.0, 2.0 * c.alpha_acc) : 1.0;
        c.hstep = 0;
        phase[b] = PH_TRIAL;
    }
}

// ---- step-size control of Algorithm 1, per instance -----------------------------
__device__ inline void count_phases(const int32_t *phase, int B, int32_t *counts) {
    __shared__ int h[8];
    if (threadIdx.x < 8) h[threadIdx.x] = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += blockDim.x) atomicAdd(&h[phase[b] & 7], 1);
    __syncthreads();
    if (threadIdx.x < 8) counts[threadIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(1024) void k_ctl_init(Batch bt, InstCtl *__restrict__ ctl, int32_t *__restrict__ phase) {
    for (int b = threadIdx.x; b < bt.B; b += 1024) {
        InstCtl c{};
        c.alpha = 1.0;
        c.alpha_acc = 1.0;
        ctl[b] = c;
        phase[b] = PH_START;
    }
}

// After the evaluation at the start weights: eps0 = 0.5 min(min nu, min V(psi_start))
// with psi_start the given start (ev_floor); ev describes the first iterate (the given
// start, or a kept learned guess).
__global__ __launch_bounds__(1024) void k_ctl_start(Batch bt, CtlOpts o, int from_phase, const double *__restrict__ ev,
                                                     const double *__restrict__ ev_nu,
                                                     const double *__restrict__ ev_floor,
                                                     const int32_t *__restrict__ fail_inst, InstCtl *__restrict__ ctl,
                                                     int32_t *__restrict__ phase, int32_t *__restrict__ counts) {
    for (int b = threadIdx.x; b < bt.B; b += 1024) {
        if (phase[b] != from_phase) continue;
        InstCtl &c = ctl[b];
        c.evals += 1;
        if (from_phase == PH_REPAIR) c.repaired = 1;
        if (from_phase == PH_RESTART) c.default_start = 1;
        c.sumV = ev[4 * b + 0];
        c.maxrel = ev[4 * b + 1];
        c.gnorm = ev[4 * b + 2];
        c.gnorm_prev = 0.0;
        c.minV = ev[4 * b + 3];
        // an empty start cell: first raise the empty cells' weights (again while the
        // host allows more rounds), then restart from the default weights, then give up
        // (eps0 would be 0)
        if (!(c.minV > 0.0) && o.allow_restart && from_phase != PH_RESTART) {
            phase[b] = (from_phase == PH_START || o.repair_more) ? PH_REPAIR : PH_RESTART;
            continue;
        }
        c.eps0 = 0.5 * fmin(ev_nu[4 * b + 3], ev_floor[4 * b + 3]);
        int ph = PH_ACTIVE;
        if (!(c.eps0 > 0.0)) {
            c.status = -2;  // LAGOT_EEMPTY
            ph = PH_FAILED;
        } else if (fail_inst[b] != 0) {
            c.status = -5;  // LAGOT_ECAPACITY
            ph = PH_FAILED;
        } else if (c.maxrel <= o.tol) {
            ph = PH_DONE;
        } else if (o.max_newton <= 0) {
            if (!o.single) c.status = -3;  // LAGOT_ENOCONV
            ph = o.single ? PH_DONE : PH_FAILED;
        }
        phase[b] = ph;
    }
    __syncthreads();
    count_phases(phase, bt.B, counts);
}

// trial weights psi + alpha u of every instance in the step-size search
__global__ __launch_bounds__(TILE) void k_axpy_trial(Batch bt, const InstCtl *__restrict__ ctl,
                                                      const double *__restrict__ psi, const double *__restrict__ u,
                                                      double *__restrict__ out, float4 *__restrict__ pos) {
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    if (bt.phase[b] != PH_TRIAL) return;
    const int i = bt.tile_row[t] + (int)threadIdx.x;
    if (i >= bt.off[b + 1]) return;
    const double v = fma(ctl[b].alpha, u[i], psi[i]);
    out[i] = v;
    pos[i].w = (float)v;
}

// KMT test of the trial: every cell keeps volume eps0 and ||g|| <= (1 - alpha/2) ||g_accepted||.
__global__ __launch_bounds__(1024) void k_ctl_decide(Batch bt, CtlOpts o, const double *__restrict__ ev,
                                                      const int32_t *__restrict__ fail_inst,
                                                      InstCtl *__restrict__ ctl, int32_t *__restrict__ phase) {
    for (int b = threadIdx.x; b < bt.B; b += 1024) {
        if (phase[b] != PH_TRIAL) continue;
        InstCtl &c = ctl[b];
        c.evals += 1;
        const double sumV = ev[4 * b + 0], maxrel = ev[4 * b + 1], gnorm = ev[4 * b + 2], minV = ev[4 * b + 3];
        c.tminV = minV;
        c.tgnorm = gnorm;
        if (fail_inst[b] == 0 && minV >= c.eps0 && (!o.residual_test || gnorm <= (1.0 - 0.5 * c.alpha) * c.gnorm)) {
            c.sumV = sumV;
            c.maxrel = maxrel;
            c.gnorm_prev = c.gnorm;
            c.gnorm = gnorm;
            c.minV = minV;
            c.alpha_acc = c.alpha;
            if (c.iters == c.iter_base) c.alpha_first = c.alpha;
            phase[b] = PH_ACCEPT;
        } else {
            c.alpha *= 0.5;
            c.halvings += 1;
            c.hstep += 1;
            if (c.hstep > o.max_halvings) {
                c.status = fail_inst[b] != 0 ? -5 : -4;  // LAGOT_ECAPACITY : LAGOT_ELINESEARCH
                c.restore = 1;
                phase[b] = PH_FAILED;
            }
        }
    }
}

// accepted trials become the iterate; a failed search puts back the float32 shadow
// Rows of instances that took a full step (alpha 1) to max relative error < 100 tol (tol
// <= 1e-4: a final solve) without halving ||nu - V||: the cells off by more than tol/4.
__global__ __launch_bounds__(TILE) void k_mark_precise(Batch bt, CtlOpts o, const InstCtl *__restrict__ ctl,
                                                        const double *__restrict__ V, const double *__restrict__ nu,
                                                        uint8_t *__restrict__ prec) {
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    if (bt.phase[b] != PH_ACTIVE || !(o.tol <= 1e-4)) return;
    const InstCtl &c = ctl[b];
    if (!(c.alpha_acc == 1.0 && c.gnorm_prev > 0.0 && c.gnorm > 0.5 * c.gnorm_prev && c.maxrel < 100.0 * o.tol)) return;
    const int i = bt.tile_row[t] + (int)threadIdx.x;
    if (i >= bt.off[b + 1]) return;
    if (fabs(V[i] - nu[i]) > 0.25 * o.tol * nu[i]) prec[i] = 1;
}

__global__ __launch_bounds__(TILE) void k_accept_rows(Batch bt, const InstCtl *__restrict__ ctl,
                                                       double *__restrict__ psi, const double *__restrict__ trial,
                                                       float4 *__restrict__ pos) {
    const int t = blockIdx.x;
    const int b = bt.tile_inst[t];
    const int ph = bt.phase[b];
    const bool acc = ph == PH_ACCEPT, rst = ph == PH_FAILED && ctl[b].restore;
    if (!acc && !rst) return;
    const int i = bt.tile_row[t] + (int)threadIdx.x;
    if (i >= bt.off[b + 1]) return;
    if (acc)
        psi[i] = trial[i];
    else
        pos[i].w = (float)psi[i];
}

__global__ __launch_bounds__(1024) void k_ctl_commit(Batch bt, CtlOpts o, InstCtl *__restrict__ ctl,
                                                      int32_t *__restrict__ phase, int32_t *__restrict__ counts) {
    for (int b = threadIdx.x; b < bt.B; b += 1024) {
        InstCtl &c = ctl[b];
        c.restore = 0;
        if (phase[b] != PH_ACCEPT) continue;
        c.iters += 1;
        int ph = PH_ACTIVE;
        if (c.maxrel <= o.tol || o.single || (o.gtol > 0.0 && c.gnorm <= o.gtol * c.gnorm0)) {
            ph = PH_DONE;
        } else if (c.iters - c.iter_base >= o.max_newton) {
            c.status = -3;  // LAGOT_ENOCONV
            ph = PH_FAILED;
        }
        phase[b] = ph;
    }
    __syncthreads();
    count_phases(phase, bt.B, counts);
}

__global__ __launch_bounds__(1024) void k_ctl_stage(Batch bt, CtlOpts o, const double *__restrict__ ev,
                                                     const double *__restrict__ ev_nu,
                                                     const int32_t *__restrict__ fail_inst, InstCtl *__restrict__ ctl,
                                                     int32_t *__restrict__ phase, int32_t *__restrict__ counts) {
    for (int b = threadIdx.x; b < bt.B; b += 1024) {
        InstCtl &c = ctl[b];
        c.status = 0;
        c.restore = 0;
        c.iter_base = c.iters;
        c.alpha = 1.0;
        // the search of the stage's first iteration starts at min(1, 2 alpha_acc)
        c.alpha_acc = (o.stage_carry && c.alpha_first > 0.0) ? 0.5 * c.alpha_first : 1.0;
        c.sumV = ev[4 * b + 0];
        c.maxrel = ev[4 * b + 1];
        c.gnorm = ev[4 * b + 2];
        c.minV = ev[4 * b + 3];
        c.gnorm0 = c.gnorm;
        c.gnorm_prev = 0.0;
        c.eps0 = 0.5 * fmin(ev_nu[4 * b + 3], ev[4 * b + 3]);
        int ph = PH_ACTIVE;
        if (!(c.eps0 > 0.0)) {
            c.status = -2;  // LAGOT_EEMPTY
            ph = PH_FAILED;
        } else if (fail_inst[b] != 0) {
            c.status = -5;  // LAGOT_ECAPACITY
            ph = PH_FAILED;
        } else if (c.maxrel <= o.tol) {
            ph = PH_DONE;
        }
        phase[b] = ph;
    }
    __syncthreads();
    count_phases(phase, bt.B, counts);
}

__global__ __launch_bounds__(256) void k_nu_stage(int64_t n, double s, const double *__restrict__ v0,
                                                   const double *__restrict__ nu, double *__restrict__ nu_s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) nu_s[i] = (1.0 - s) * v0[i] + s * nu[i];
}

inline int nblocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void launch_mark_precise(hipStream_t st, const Batch &bt, CtlOpts o, const InstCtl *ctl, const double *V,
                         const double *nu, uint8_t *prec) {
    hipLaunchKernelGGL(k_mark_precise, dim3(bt.T), dim3(TILE), 0, st, bt, o, ctl, V, nu, prec);
}

void launch_ctl_stage(hipStream_t st, const Batch &bt, CtlOpts o, const double *ev, const double *ev_nu,
                      const int32_t *fail_inst, InstCtl *ctl, int32_t *phase, int32_t *counts) {
    hipLaunchKernelGGL(k_ctl_stage, dim3(1), dim3(1024), 0, st, bt, o, ev, ev_nu, fail_inst, ctl, phase, counts);
}

void launch_nu_stage(hipStream_t st, int64_t n, double s, const double *v0, const double *nu, double *nu_s) {
    hipLaunchKernelGGL(k_nu_stage, dim3(nblocks(n, 256)), dim3(256), 0, st, n, s, v0, nu, nu_s);
}

void launch_eval_reduce(hipStream_t st, const Batch &bt, int want, const double *V, const double *nu, double *part,
                        double *ev) {
    hipLaunchKernelGGL(k_eval_partial, dim3(bt.T), dim3(TILE), 0, st, bt, want, V, nu, part);
    hipLaunchKernelGGL(k_eval_final, dim3(bt.B), dim3(RB), 0, st, bt, want, part, ev);
}

void launch_hess_assemble(hipStream_t st, int64_t n, const Batch &bt, int want, const float4 *pos_s,
                          const int32_t *fcol, const float *farea, const int32_t *fcnt, int32_t *hcol, float *hval,
                          int32_t *xcnt, int32_t *herr) {
    hipLaunchKernelGGL(k_hess_begin, dim3(bt.T), dim3(TILE), 0, st, bt, want, xcnt, herr);
    hipLaunchKernelGGL(k_hess_assemble, dim3(nblocks(n * 16, 256)), dim3(256), 0, st, n, bt, want, pos_s, fcol, farea,
                       fcnt, hcol, hval, xcnt, herr);
}

void launch_hess_finish(hipStream_t st, const Batch &bt, int want, const double *psi_s, const double *K,
                        const int32_t *fcnt, const int32_t *xcnt, int32_t *hcnt, int32_t *hcol, float *hval,
                        double *diag, int2 *hrow, int2 *ent) {
    hipLaunchKernelGGL(k_hess_finish, dim3(bt.T), dim3(TILE), 0, st, bt, want, psi_s, K, fcnt, xcnt, hcnt, hcol, hval,
                       diag, hrow, ent);
}

// shape = 4 * log2(lanes) + log2(SUB / 64): lanes in {1, 2, 4, 8}, SUB in {64, 128, 256}
#define LAGOT_CG_SHAPES(X) X(1, 64) X(1, 128) X(1, 256) X(2, 64) X(2, 128) X(2, 256) X(4, 64) X(4, 128) X(4, 256) \
    X(8, 64) X(8, 128)

bool cg_shape_ok(int lanes, int sub) {
#define X(L, S) if (lanes == L && sub == S) return true;
    LAGOT_CG_SHAPES(X)
#undef X
    return false;
}

void launch_cg_init(hipStream_t st, const Batch &bt, int lanes, int sub, const double *V, const double *nu,
                    const double *diag, const int2 *hrow, const int2 *ent, CgBufs cg) {
    const dim3 grid((TILE / sub) * bt.T), block(lanes * sub);
#define X(L, S) \
    if (lanes == L && sub == S) { hipLaunchKernelGGL((k_cg_init<L, S>), grid, block, 0, st, bt, V, nu, diag, hrow, ent, cg); return; }
    LAGOT_CG_SHAPES(X)
#undef X
}

void launch_cg_iter(hipStream_t st, const Batch &bt, int lanes, int sub, int m, double rtol2, int cap,
                    const int2 *hrow, const int2 *ent, CgBufs cg) {
    const dim3 grid((TILE / sub) * bt.T), block(lanes * sub);
#define X(L, S) \
    if (lanes == L && sub == S) { hipLaunchKernelGGL((k_cg_iter<L, S>), grid, block, 0, st, bt, m, rtol2, cap, hrow, ent, cg); return; }
    LAGOT_CG_SHAPES(X)
#undef X
}

int cg_sum_in_block_max() { return CG_SUM_IN_BLOCK; }

void launch_cg_split_iter(hipStream_t st, const Batch &bt, int lanes, int sub, int m, double rtol2, int cap,
                          const int2 *hrow, const int2 *ent, CgBufs cg) {
    const dim3 grid((TILE / sub) * bt.T);
    if (sub == 64)
        hipLaunchKernelGGL((k_cg_update<64>), grid, dim3(64), 0, st, bt, m, rtol2, cap, cg);
    else if (sub == 128)
        hipLaunchKernelGGL((k_cg_update<128>), grid, dim3(128), 0, st, bt, m, rtol2, cap, cg);
    else
        hipLaunchKernelGGL((k_cg_update<256>), grid, dim3(256), 0, st, bt, m, rtol2, cap, cg);
    const dim3 block(lanes * sub);
#define X(L, S) \
    if (lanes == L && sub == S) { hipLaunchKernelGGL((k_cg_product<L, S>), grid, block, 0, st, bt, m, cap, hrow, ent, cg); return; }
    LAGOT_CG_SHAPES(X)
#undef X
}

void launch_cg_scalars(hipStream_t st, const Batch &bt, int sub, int m, int cap, CgBufs cg) {
    hipLaunchKernelGGL(k_cg_scalars, dim3(bt.B), dim3(SCB), 0, st, bt, TILE / sub, m, cap, cg);
}

void launch_cg_advance(hipStream_t st, const Batch &bt, int chunk, int cap, CgBufs cg) {
    hipLaunchKernelGGL(k_cg_advance, dim3(1), dim3(1024), 0, st, bt, chunk, cap, cg);
}

void launch_cg_finish(hipStream_t st, const Batch &bt, int sub, double rtol2, int step_start, CgBufs cg,
                      const int32_t *herr, InstCtl *ctl, int32_t *phase) {
    hipLaunchKernelGGL(k_cg_finish, dim3(bt.B), dim3(RB), 0, st, bt, TILE / sub, rtol2, step_start, cg, herr, ctl,
                       phase);
}

void launch_ctl_init(hipStream_t st, const Batch &bt, InstCtl *ctl, int32_t *phase) {
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1024), 0, st, bt, ctl, phase);
}

void launch_ctl_start(hipStream_t st, const Batch &bt, CtlOpts o, int from_phase, const double *ev,
                      const double *ev_nu, const double *ev_floor, const int32_t *fail_inst, InstCtl *ctl,
                      int32_t *phase, int32_t *counts) {
    hipLaunchKernelGGL(k_ctl_start, dim3(1), dim3(1024), 0, st, bt, o, from_phase, ev, ev_nu, ev_floor, fail_inst, ctl,
                       phase, counts);
}

void launch_axpy_trial(hipStream_t st, const Batch &bt, const InstCtl *ctl, const double *psi_s, const double *u,
                       double *psi_trial, float4 *pos_s) {
    hipLaunchKernelGGL(k_axpy_trial, dim3(bt.T), dim3(TILE), 0, st, bt, ctl, psi_s, u, psi_trial, pos_s);
}

void launch_ctl_decide(hipStream_t st, const Batch &bt, CtlOpts o, const double *ev, const int32_t *fail_inst,
                       InstCtl *ctl, int32_t *phase) {
    hipLaunchKernelGGL(k_ctl_decide, dim3(1), dim3(1024), 0, st, bt, o, ev, fail_inst, ctl, phase);
}

void launch_accept_rows(hipStream_t st, const Batch &bt, const InstCtl *ctl, double *psi_s, const double *psi_trial,
                        float4 *pos_s) {
    hipLaunchKernelGGL(k_accept_rows, dim3(bt.T), dim3(TILE), 0, st, bt, ctl, psi_s, psi_trial, pos_s);
}

void launch_ctl_commit(hipStream_t st, const Batch &bt, CtlOpts o, InstCtl *ctl, int32_t *phase, int32_t *counts) {
    hipLaunchKernelGGL(k_ctl_commit, dim3(1), dim3(1024), 0, st, bt, o, ctl, phase, counts);
}

}  // namespace lagot
