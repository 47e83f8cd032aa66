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

// partial[0*nb+b] = sum V, [1] = max |V-nu|/nu, [2] = sum (nu-V)^2, [3] = min V
__global__ __launch_bounds__(RB) void k_eval_partial(int64_t n, const double *__restrict__ V,
                                                      const double *__restrict__ nu, double *__restrict__ partial) {
    __shared__ double sh[RB / 64];
    double sv = 0.0, mx = 0.0, g2 = 0.0, mn = 1e300;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
        const double v = V[i], b = nu[i];
        sv += v;
        mx = fmax(mx, fabs(v - b) / b);
        g2 += (b - v) * (b - v);
        mn = fmin(mn, v);
    }
    const int nb = gridDim.x;
    sv = block_sum(sv, sh);
    mx = block_max(mx, sh);
    g2 = block_sum(g2, sh);
    mn = block_min(mn, sh);
    if (threadIdx.x == 0) {
        partial[0 * nb + blockIdx.x] = sv;
        partial[1 * nb + blockIdx.x] = mx;
        partial[2 * nb + blockIdx.x] = g2;
        partial[3 * nb + blockIdx.x] = mn;
    }
}

__global__ __launch_bounds__(1024) void k_eval_final(const double *partial, int nb, double *out4) {
    __shared__ double sh[16];
    double sv = 0.0, mx = 0.0, g2 = 0.0, mn = 1e300;
    for (int b = threadIdx.x; b < nb; b += 1024) {
        sv += partial[b];
        mx = fmax(mx, partial[nb + b]);
        g2 += partial[2 * nb + b];
        mn = fmin(mn, partial[3 * nb + b]);
    }
    sv = block_sum(sv, sh);
    mx = block_max(mx, sh);
    g2 = block_sum(g2, sh);
    mn = block_min(mn, sh);
    if (threadIdx.x == 0) {
        out4[0] = sv;
        out4[1] = mx;
        out4[2] = sqrt(g2);
        out4[3] = mn;
    }
}

// Row i of -Hess K: one entry per facet of cell i; a facet that cell j does not
// list is appended to row j as well (union pattern). One thread per facet slot;
// the partner row is read with 16-byte loads and searched in registers.
__global__ void k_hess_assemble(int64_t n, const float4 *__restrict__ pos, const int32_t *__restrict__ fcol,
                                const float *__restrict__ farea, const int32_t *__restrict__ fcnt,
                                int32_t *__restrict__ hcol, float *__restrict__ hval, int32_t *__restrict__ xcnt,
                                int32_t *__restrict__ err) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / 16;
    const int f0 = (int)(t & 15);
    if (i >= n) return;
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
                atomicAdd(err, 1);
            }
        }
    }
}

__global__ void k_hess_finish(int64_t n, const double *__restrict__ psi, const double *__restrict__ K,
                              const int32_t *__restrict__ fcnt, const int32_t *__restrict__ xcnt,
                              int32_t *__restrict__ hcnt, const float *__restrict__ hval, double *__restrict__ diag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = min(fcnt[i] + xcnt[i], FCAP);
    hcnt[i] = c;
    double s = 0.0;
    for (int f = 0; f < c; ++f) s += (double)hval[i * FCAP + f];
    const double p = psi[i];
    if (p > 0.0) s += K[i] / (2.0 * sqrt(p));
    diag[i] = s;
}



// ---- Jacobi-PCG, two fused kernels per iteration -----------------------------
// Every kernel runs a fixed grid of nb <= 512 blocks (grid-stride loops) and
// leaves one partial per block. The scalars an iteration needs (alpha, beta, the
// stop test) are recomputed by every block from the previous kernel's partials,
// summed in block order: deterministic, with no atomics and no device fences
// (a device-scope fence writes back the XCD's L2 on this part).
// Partials: RZ[2][nb], RR[2][nb] (slot k%2 holds the residual of iteration k), PQ[nb].
// state (int32): [0] iterations done, [1] breakdown, [2] converged.

__device__ inline double sum_partials(const double *v, int nb, double *sh) {
    double s = 0.0;
    for (int k = threadIdx.x; k < nb; k += RB) s += v[k];
    return block_sum(s, sh);
}

// Four block-ordered sums in one pass and one block reduction (lanes fold in a fixed order).
__device__ inline void sum_partials4(const double *a, const double *b, const double *c, const double *d, int na,
                                     int nd, double *out, double (*sh)[4]) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < na; k += RB) {
        s[0] += a[k];
        s[1] += b[k];
        s[2] += c[k];
    }
    for (int k = threadIdx.x; k < nd; k += RB) s[3] += d[k];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        for (int o = 32; o > 0; o >>= 1) s[q] += __shfl_xor(s[q], o, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 4; ++q) sh[w][q] = s[q];
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
        double t = 0.0;
        for (int k = 0; k < RB / 64; ++k) t += sh[k][q];
        out[q] = t;
    }
}

// g = nu - V (0 on empty rows), x = 0, r = g, z = r / D ; partials of r.z, r.r into slot 0
__global__ __launch_bounds__(RB) void k_pcg_init(int64_t n, int nb, const double *__restrict__ V,
                                                  const double *__restrict__ nu, const double *__restrict__ diag,
                                                  double *__restrict__ g, double *__restrict__ x,
                                                  double *__restrict__ r, double *__restrict__ z,
                                                  double *__restrict__ RZ, double *__restrict__ RR,
                                                  double *__restrict__ R0, int32_t *__restrict__ state) {
    __shared__ double sh[RB / 64];
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)nb * RB) {
        const double d = diag[i];
        const double gi = d > 0.0 ? nu[i] - V[i] : 0.0;
        const double zi = d > 0.0 ? gi / d : 0.0;
        g[i] = gi;
        x[i] = 0.0;
        r[i] = gi;
        z[i] = zi;
        rz += gi * zi;
        rr += gi * gi;
    }
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        RZ[blockIdx.x] = rz;
        RR[blockIdx.x] = rr;
        R0[blockIdx.x] = rr;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        state[0] = 0;
        state[1] = 0;
        state[2] = 0;
    }
}

// p_k = z + beta p_{k-1} (p_0 = z); q = (D - W) p_k; one partial of p.q per block.
// Four lanes per row (rows hold ~6-20 facets), one row per lane quad, no grid stride:
// the gathers of a row are issued together and every row is in flight at once.
constexpr int SPMV_LANES = 4;
constexpr int SPMV_ROWS = RB / SPMV_LANES;

__global__ __launch_bounds__(RB) void k_pcg_spmv(int64_t n, int k, int nb, double rtol2, const double *__restrict__ R0,
                                                  const int32_t *__restrict__ hcol, const float *__restrict__ hval,
                                                  const int32_t *__restrict__ hcnt, const double *__restrict__ diag,
                                                  const double *__restrict__ z, const double *__restrict__ p_old,
                                                  double *__restrict__ p_new, double *__restrict__ q,
                                                  const double *__restrict__ RZ, const double *__restrict__ RR,
                                                  double *__restrict__ PQ, const int32_t *__restrict__ state) {
    __shared__ double sh[RB / 64];
    __shared__ double sh4[RB / 64][4];
    if (state[1] != 0) return;
    double S4[4];
    sum_partials4(R0, RR + (k & 1) * nb, RZ + (k & 1) * nb, RZ + ((k + 1) & 1) * nb, nb, k > 0 ? nb : 0, S4, sh4);
    const double stop = rtol2 * S4[0], rr = S4[1], rz = S4[2], rz_old = S4[3];
    if (rr <= stop) return;
    const double beta = (k > 0 && rz_old > 0.0) ? rz / rz_old : 0.0;
    const int l = threadIdx.x & (SPMV_LANES - 1);
    const int64_t row = (int64_t)blockIdx.x * SPMV_ROWS + (threadIdx.x / SPMV_LANES);
    double acc = 0.0, pq = 0.0;
    if (row < n) {
        const int c = hcnt[row];
        const int32_t *cr = hcol + row * FCAP;
        const float *vr = hval + row * FCAP;
#pragma unroll 4
        for (int f = l; f < c; f += SPMV_LANES) {
            const int j = cr[f];
            const double pj = k == 0 ? z[j] : z[j] + beta * p_old[j];
            acc += (double)vr[f] * pj;
        }
    }
#pragma unroll
    for (int o = SPMV_LANES / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, SPMV_LANES);
    if (row < n && l == 0) {
        const double pi = k == 0 ? z[row] : z[row] + beta * p_old[row];
        const double qi = diag[row] * pi - acc;
        p_new[row] = pi;
        q[row] = qi;
        pq = pi * qi;
    }
    pq = block_sum(pq, sh);
    if (threadIdx.x == 0) PQ[blockIdx.x] = pq;
}

// alpha = rz / (p.q); x += alpha p; r -= alpha q; z = r / D; partials of r.z, r.r into slot (k+1)%2
__global__ __launch_bounds__(RB) void k_pcg_update(int64_t n, int k, int nb, int npq, double rtol2,
                                                    const double *__restrict__ R0,
                                                    const double *__restrict__ diag, double *__restrict__ x,
                                                    double *__restrict__ r, double *__restrict__ z,
                                                    const double *__restrict__ p, const double *__restrict__ q,
                                                    double *__restrict__ RZ, double *__restrict__ RR,
                                                    const double *__restrict__ PQ, int32_t *__restrict__ state) {
    __shared__ double sh[RB / 64];
    __shared__ double sh4[RB / 64][4];
    if (state[1] != 0) return;
    double S4[4];
    sum_partials4(R0, RR + (k & 1) * nb, RZ + (k & 1) * nb, PQ, nb, npq, S4, sh4);
    const double stop = rtol2 * S4[0], rr = S4[1], rz = S4[2], pq = S4[3];
    if (rr <= stop) {
        if (blockIdx.x == 0 && threadIdx.x == 0) state[2] = 1;
        return;
    }
    if (!(pq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) state[1] = 1;
        return;
    }
    const double alpha = rz / pq;
    double rzn = 0.0, rrn = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)nb * RB) {
        const double d = diag[i];
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        const double zi = d > 0.0 ? ri / d : 0.0;
        z[i] = zi;
        rzn += ri * zi;
        rrn += ri * ri;
    }
    rzn = block_sum(rzn, sh);
    rrn = block_sum(rrn, sh);
    if (threadIdx.x == 0) {
        RZ[((k + 1) & 1) * nb + blockIdx.x] = rzn;
        RR[((k + 1) & 1) * nb + blockIdx.x] = rrn;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) state[0] = k + 1;
}

// Residual of the latest iterate into scal: [0] r.r, [1] r0.r0
__global__ __launch_bounds__(RB) void k_pcg_status(int nb, const double *__restrict__ RR, const double *__restrict__ R0,
                                                    const int32_t *__restrict__ state, double *__restrict__ scal) {
    __shared__ double sh[RB / 64];
    const int it = state[0];
    const double rr = sum_partials(RR + (it & 1) * nb, nb, sh);
    const double r0 = sum_partials(R0, nb, sh);
    if (threadIdx.x == 0) {
        scal[0] = rr;
        scal[1] = r0;
    }
}

__global__ void k_axpy_trial(int64_t n, const double *__restrict__ psi, const double *__restrict__ u, double alpha,
                             double *__restrict__ out, float4 *__restrict__ pos_s, double *__restrict__ rmax_partial) {
    __shared__ double red[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if (i < n) {
        const double v = psi[i] + alpha * u[i];
        out[i] = v;
        pos_s[i].w = (float)v;
        rr = v > 0.0 ? sqrt(v) : 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) rr = fmax(rr, __shfl_xor(rr, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rr;
    __syncthreads();
    if (threadIdx.x == 0) rmax_partial[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

inline int nblocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void launch_eval_reduce(hipStream_t st, int64_t n, const double *V, const double *nu, double *partial, int nblk,
                        double *out4) {
    hipLaunchKernelGGL(k_eval_partial, dim3(nblk), dim3(RB), 0, st, n, V, nu, partial);
    hipLaunchKernelGGL(k_eval_final, dim3(1), dim3(1024), 0, st, partial, nblk, out4);
}

void launch_hess_assemble(hipStream_t st, int64_t n, const float4 *pos_s, const double *psi_s, const double *K,
                          const int32_t *fcol, const float *farea, const int32_t *fcnt, int32_t *hcol, float *hval,
                          int32_t *xcnt, double *diag, int32_t *err) {
    (void)psi_s;
    (void)K;
    (void)diag;
    (void)hipMemsetAsync(xcnt, 0, sizeof(int32_t) * (size_t)n, st);
    hipLaunchKernelGGL(k_hess_assemble, dim3(nblocks(n * 16, 256)), dim3(256), 0, st, n, pos_s, fcol, farea, fcnt,
                       hcol, hval, xcnt, err);
}

void launch_hess_finish(hipStream_t st, int64_t n, const double *psi_s, const double *K, const int32_t *fcnt,
                        const int32_t *xcnt, int32_t *hcnt, const float *hval, double *diag) {
    hipLaunchKernelGGL(k_hess_finish, dim3(nblocks(n, 256)), dim3(256), 0, st, n, psi_s, K, fcnt, xcnt, hcnt, hval,
                       diag);
}

int pcg_blocks(int64_t n) { return (int)std::min<int64_t>(512, std::max<int64_t>(1, (n + RB - 1) / RB)); }
int spmv_blocks(int64_t n) { return (int)((n + SPMV_ROWS - 1) / SPMV_ROWS); }

void launch_pcg_init(hipStream_t st, int64_t n, int nb, const double *V, const double *nu, const double *diag,
                     double *g, double *x, double *r, double *z, double *RZ, double *RR, double *R0, int32_t *state) {
    hipLaunchKernelGGL(k_pcg_init, dim3(nb), dim3(RB), 0, st, n, nb, V, nu, diag, g, x, r, z, RZ, RR, R0, state);
}

void launch_pcg_spmv(hipStream_t st, int64_t n, int k, int nb, double rtol2, const double *R0, const int32_t *hcol,
                     const float *hval, const int32_t *hcnt, const double *diag, const double *z, const double *p_old,
                     double *p_new, double *q, const double *RZ, const double *RR, double *PQ, const int32_t *state) {
    hipLaunchKernelGGL(k_pcg_spmv, dim3(spmv_blocks(n)), dim3(RB), 0, st, n, k, nb, rtol2, R0, hcol, hval, hcnt, diag, z, p_old, p_new,
                       q, RZ, RR, PQ, state);
}

void launch_pcg_update(hipStream_t st, int64_t n, int k, int nb, double rtol2, const double *R0, const double *diag,
                       double *x, double *r, double *z, const double *p, const double *q, double *RZ, double *RR,
                       const double *PQ, int32_t *state) {
    hipLaunchKernelGGL(k_pcg_update, dim3(nb), dim3(RB), 0, st, n, k, nb, spmv_blocks(n), rtol2, R0, diag, x, r, z, p, q, RZ, RR, PQ,
                       state);
}

void launch_pcg_status(hipStream_t st, int nb, const double *RR, const double *R0, const int32_t *state,
                       double *scal) {
    hipLaunchKernelGGL(k_pcg_status, dim3(1), dim3(RB), 0, st, nb, RR, R0, state, scal);
}

void launch_axpy_trial(hipStream_t st, int64_t n, const double *psi_s, const double *u, double alpha,
                       double *psi_trial, float4 *pos_s, double *rmax_partial) {
    hipLaunchKernelGGL(k_axpy_trial, dim3(nblocks(n, 256)), dim3(256), 0, st, n, psi_s, u, alpha, psi_trial, pos_s,
                       rmax_partial);
}

}  // namespace lagot
