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
// list is appended to row j as well (union pattern).
__global__ void k_hess_assemble(int64_t n, const float4 *__restrict__ pos, const int32_t *__restrict__ fcol,
                                const float *__restrict__ farea, const int32_t *__restrict__ fcnt,
                                int32_t *__restrict__ hcol, float *__restrict__ hval, int32_t *__restrict__ xcnt,
                                int32_t *__restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ci = fcnt[i];
    const float4 pi = pos[i];
    for (int f = 0; f < ci; ++f) {
        const int j = fcol[i * FCAP + f];
        const float a = farea[i * FCAP + f];
        const int cj = fcnt[j];
        float a2 = -1.f;
        for (int f2 = 0; f2 < cj; ++f2) {
            if (fcol[(int64_t)j * FCAP + f2] == (int32_t)i) {
                a2 = farea[(int64_t)j * FCAP + f2];
                break;
            }
        }
        const float4 pj = pos[j];
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

// q = (D - W) p ; partial sums of p.q
__global__ __launch_bounds__(RB) void k_spmv_dot(int64_t n, const int32_t *__restrict__ hcol,
                                                  const float *__restrict__ hval, const int32_t *__restrict__ hcnt,
                                                  const double *__restrict__ diag, const double *__restrict__ p,
                                                  double *__restrict__ q, double *__restrict__ partial) {
    __shared__ double sh[RB / 64];
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    double pq = 0.0;
    if (i < n) {
        const double pi = p[i];
        double acc = diag[i] * pi;
        const int c = hcnt[i];
        for (int f = 0; f < c; ++f) acc -= (double)hval[i * FCAP + f] * p[hcol[i * FCAP + f]];
        q[i] = acc;
        pq = pi * acc;
    }
    pq = block_sum(pq, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = pq;
}

__global__ __launch_bounds__(1024) void k_reduce_sum(const double *partial, int nb, int ncomp, double *out) {
    __shared__ double sh[16];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += 1024) s += partial[c * nb + b];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) out[c] = s;
        __syncthreads();
    }
}

// g = nu - V (0 on empty rows), x = 0, r = g, z = r / D, p = z ; partials of r.z and r.r
__global__ __launch_bounds__(RB) void k_pcg_init(int64_t n, const double *__restrict__ V,
                                                  const double *__restrict__ nu, const double *__restrict__ diag,
                                                  double *__restrict__ g, double *__restrict__ x,
                                                  double *__restrict__ r, double *__restrict__ z,
                                                  double *__restrict__ p, double *__restrict__ partial) {
    __shared__ double sh[RB / 64];
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < n) {
        const double d = diag[i];
        const double gi = d > 0.0 ? nu[i] - V[i] : 0.0;
        const double zi = d > 0.0 ? gi / d : 0.0;
        g[i] = gi;
        x[i] = 0.0;
        r[i] = gi;
        z[i] = zi;
        p[i] = zi;
        rz = gi * zi;
        rr = gi * gi;
    }
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = rz;
        partial[gridDim.x + blockIdx.x] = rr;
    }
}

// scal: [0] rz  [1] rr  [2] pq  [3] alpha  [4] beta  [5] breakdown flag
// x += alpha p ; r -= alpha q ; z = r / D ; partials of r.z, r.r
__global__ __launch_bounds__(RB) void k_pcg_update(int64_t n, const double *__restrict__ scal,
                                                    const double *__restrict__ diag, double *__restrict__ x,
                                                    double *__restrict__ r, double *__restrict__ z,
                                                    const double *__restrict__ p, const double *__restrict__ q,
                                                    double *__restrict__ partial) {
    __shared__ double sh[RB / 64];
    const double alpha = scal[3];
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < n) {
        const double d = diag[i];
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        const double zi = d > 0.0 ? ri / d : 0.0;
        z[i] = zi;
        rz = ri * zi;
        rr = ri * ri;
    }
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = rz;
        partial[gridDim.x + blockIdx.x] = rr;
    }
}

// mode 0: pq partials -> scal[2], alpha = rz / pq -> scal[3]
// mode 1: (rz_new, rr_new) partials -> beta = rz_new / rz -> scal[4], scal[0] = rz_new, scal[1] = rr_new
// mode 2: (rz, rr) partials of the initial residual -> scal[0], scal[1]
__global__ __launch_bounds__(1024) void k_pcg_scalars(const double *partial, int nb, int mode, double *scal) {
    __shared__ double sh[16];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nb; k += 1024) {
        a += partial[k];
        if (mode != 0) b += partial[nb + k];
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            scal[2] = a;
            if (!(a > 0.0)) {
                scal[5] = 1.0;
                scal[3] = 0.0;
            } else {
                scal[3] = scal[0] / a;
            }
        } else if (mode == 1) {
            scal[4] = scal[0] > 0.0 ? a / scal[0] : 0.0;
            scal[0] = a;
            scal[1] = b;
        } else {
            scal[0] = a;
            scal[1] = b;
            scal[5] = 0.0;
        }
    }
}

__global__ void k_pcg_direction(int64_t n, const double *__restrict__ scal, const double *__restrict__ z,
                                double *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    p[i] = z[i] + scal[4] * p[i];
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
    hipLaunchKernelGGL(k_hess_assemble, dim3(nblocks(n, 128)), dim3(128), 0, st, n, pos_s, fcol, farea, fcnt, hcol,
                       hval, xcnt, err);
}

void launch_hess_finish(hipStream_t st, int64_t n, const double *psi_s, const double *K, const int32_t *fcnt,
                        const int32_t *xcnt, int32_t *hcnt, const float *hval, double *diag) {
    hipLaunchKernelGGL(k_hess_finish, dim3(nblocks(n, 256)), dim3(256), 0, st, n, psi_s, K, fcnt, xcnt, hcnt, hval,
                       diag);
}

void launch_spmv_dot(hipStream_t st, int64_t n, const int32_t *hcol, const float *hval, const int32_t *hcnt,
                     const double *diag, const double *p, double *q, double *partial, int nblk) {
    hipLaunchKernelGGL(k_spmv_dot, dim3(nblk), dim3(RB), 0, st, n, hcol, hval, hcnt, diag, p, q, partial);
}

void launch_reduce_sum(hipStream_t st, const double *partial, int nblk, int ncomp, double *out) {
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(1024), 0, st, partial, nblk, ncomp, out);
}

void launch_pcg_init(hipStream_t st, int64_t n, const double *V, const double *nu, const double *diag, double *g,
                     double *x, double *r, double *z, double *p, double *partial, int nblk) {
    hipLaunchKernelGGL(k_pcg_init, dim3(nblk), dim3(RB), 0, st, n, V, nu, diag, g, x, r, z, p, partial);
}

void launch_pcg_update(hipStream_t st, int64_t n, const double *scal, const double *diag, double *x, double *r,
                       double *z, const double *p, const double *q, double *partial, int nblk) {
    hipLaunchKernelGGL(k_pcg_update, dim3(nblk), dim3(RB), 0, st, n, scal, diag, x, r, z, p, q, partial);
}

void launch_pcg_scalars(hipStream_t st, const double *partial, int nblk, int mode, double *scal) {
    hipLaunchKernelGGL(k_pcg_scalars, dim3(1), dim3(1024), 0, st, partial, nblk, mode, scal);
}

void launch_pcg_direction(hipStream_t st, int64_t n, const double *scal, const double *z, double *p) {
    hipLaunchKernelGGL(k_pcg_direction, dim3(nblocks(n, 256)), dim3(256), 0, st, n, scal, z, p);
}

void launch_axpy_trial(hipStream_t st, int64_t n, const double *psi_s, const double *u, double alpha,
                       double *psi_trial, float4 *pos_s, double *rmax_partial) {
    hipLaunchKernelGGL(k_axpy_trial, dim3(nblocks(n, 256)), dim3(256), 0, st, n, psi_s, u, alpha, psi_trial, pos_s,
                       rmax_partial);
}

}  // namespace lagot
