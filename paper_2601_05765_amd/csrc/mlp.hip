// mlp.hip -- learned warm start: the 16 nearest sites of every site (grid
// search), the 64 network inputs, and the network 64 -> 128 -> 128 -> 128 -> 1
// (GELU, erf form) with BF16 MFMA products and FP32 accumulation, its backward
// pass and Adam. The network predicts (psi_new - psi_prev) / s_i^2 with
// s_i = nu_i^(1/3); its guess is only a start for the Newton solve.
//
// Inputs of site i (64): the offsets (p_j - p_i) / s_i of its 16 nearest sites in
// ascending (distance, caller index), psi_prev_i / s_i^2, nu_i / mean(nu), and the
// relative volume mismatch (nu - V) / nu under the previous weights of the site and
// of its 13 nearest sites.
#include <algorithm>

#include "lagot_internal.h"

namespace lagot {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * __expf(-0.5f * x * x) * 0.39894228040143268f;
}

// ---------------- 16 nearest sites and the network inputs ----------------
// One thread per site (grid order). Sorted top-16 kept in registers (static
// indices). Distances in float64 without contraction (the float32 inputs make
// the differences and their squares exact), ties by caller index. The search
// grows by shells of grid cells (ring R adds the cells at Chebyshev distance R
// from the site's cell) and stops once the 16th distance is within R cell sizes,
// which every unvisited cell is beyond. A candidate is compared with the current
// 16th entry first; only closer ones run the insertion pass.
__device__ inline void knn_offer(double kd, int ki, int kj, double (&D)[N_NEI], int (&I)[N_NEI], int (&J)[N_NEI]) {
    if (!(kd < D[N_NEI - 1] || (kd == D[N_NEI - 1] && ki < I[N_NEI - 1]))) return;
#pragma unroll
    for (int m = 0; m < N_NEI; ++m) {
        const bool less = kd < D[m] || (kd == D[m] && ki < I[m]);
        if (less) {
            const double td = D[m];
            const int ti = I[m], tj = J[m];
            D[m] = kd;
            I[m] = ki;
            J[m] = kj;
            kd = td;
            ki = ti;
            kj = tj;
        }
    }
}

__global__ __launch_bounds__(256) void k_knn_features(int64_t n, const float4 *__restrict__ pos_s,
                                                       const int32_t *__restrict__ perm,
                                                       const int32_t *__restrict__ cell_start, GridDesc g,
                                                       const double *__restrict__ psi_prev_s,
                                                       const double *__restrict__ nu_s, const double *__restrict__ nu_sum,
                                                       const double *__restrict__ V_s,
                                                       int32_t *__restrict__ nbr_out, uint16_t *__restrict__ feat,
                                                       int32_t *__restrict__ err) {
    const int64_t k = (int64_t)xcd_block((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float4 p = pos_s[k];
    double D[N_NEI];
    int I[N_NEI], J[N_NEI];
#pragma unroll
    for (int m = 0; m < N_NEI; ++m) {
        D[m] = 1e300;
        I[m] = 0x7FFFFFFF;
        J[m] = -1;
    }
    int c3[3];
    const float pp[3] = {p.x, p.y, p.z};
    for (int a = 0; a < 3; ++a) c3[a] = min(max((int)floorf((pp[a] - g.lo[a]) * g.inv_s), 0), g.dim[a] - 1);
    int found = 0;
    for (int R = 0;; ++R) {
        const int x0 = max(c3[0] - R, 0), x1 = min(c3[0] + R, g.dim[0] - 1);
        const int y0 = max(c3[1] - R, 0), y1 = min(c3[1] + R, g.dim[1] - 1);
        const int z0 = max(c3[2] - R, 0), z1 = min(c3[2] + R, g.dim[2] - 1);
        for (int ix = x0; ix <= x1; ++ix)
            for (int iy = y0; iy <= y1; ++iy) {
                const int col = (ix * g.dim[1] + iy) * g.dim[2];
                // columns inside the previous ring contribute only their two new end cells
                const bool inner = abs(ix - c3[0]) < R && abs(iy - c3[1]) < R;
                for (int part = 0; part < (inner ? 2 : 1); ++part) {
                    int za = z0, zb = z1;
                    if (inner) {
                        za = zb = part == 0 ? c3[2] - R : c3[2] + R;
                        if (za < 0 || za >= g.dim[2]) continue;
                    }
                    const int beg = cell_start[col + za], end = cell_start[col + zb + 1];
                    for (int j = beg; j < end; ++j) {
                        if (j == k) continue;
                        const float4 q = pos_s[j];
                        const double dx = (double)q.x - (double)p.x, dy = (double)q.y - (double)p.y,
                                     dz = (double)q.z - (double)p.z;
                        const double kd =
                            __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
                        ++found;
                        knn_offer(kd, perm[j], j, D, I, J);
                    }
                }
            }
        const double reach = (double)R * (double)g.s;
        const bool whole = x0 == 0 && y0 == 0 && z0 == 0 && x1 == g.dim[0] - 1 && y1 == g.dim[1] - 1 &&
                           z1 == g.dim[2] - 1;
        if ((found >= N_NEI && D[N_NEI - 1] <= reach * reach) || whole) break;
    }
    if (found < N_NEI) atomicAdd(err, 1);
    // inputs
    const double s = cbrt(nu_s[k]);
    const float inv_s = (float)(1.0 / s);
    uint16_t f[64];
#pragma unroll
    for (int m = 0; m < N_NEI; ++m) {
        float ox = 0.f, oy = 0.f, oz = 0.f;
        if (J[m] >= 0) {
            const float4 q = pos_s[J[m]];
            ox = (q.x - p.x) * inv_s;
            oy = (q.y - p.y) * inv_s;
            oz = (q.z - p.z) * inv_s;
        }
        f[3 * m] = f2bf(ox);
        f[3 * m + 1] = f2bf(oy);
        f[3 * m + 2] = f2bf(oz);
        if (nbr_out) nbr_out[k * N_NEI + m] = I[m] == 0x7FFFFFFF ? -1 : I[m];
    }
    f[48] = f2bf((float)(psi_prev_s[k] / (s * s)));
    f[49] = f2bf((float)(nu_s[k] * (double)n / *nu_sum));
    f[50] = f2bf((float)((nu_s[k] - V_s[k]) / nu_s[k]));
#pragma unroll
    for (int m = 0; m < 13; ++m) {
        const int j = J[m];
        f[51 + m] = j >= 0 ? f2bf((float)((nu_s[j] - V_s[j]) / nu_s[j])) : (uint16_t)0;
    }
    uint4 *dst = reinterpret_cast<uint4 *>(feat + k * 64);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        uint4 w;
        w.x = (uint32_t)f[8 * v] | ((uint32_t)f[8 * v + 1] << 16);
        w.y = (uint32_t)f[8 * v + 2] | ((uint32_t)f[8 * v + 3] << 16);
        w.z = (uint32_t)f[8 * v + 4] | ((uint32_t)f[8 * v + 5] << 16);
        w.w = (uint32_t)f[8 * v + 6] | ((uint32_t)f[8 * v + 7] << 16);
        dst[v] = w;
    }
}

// ---------------- BF16 MFMA product with fused epilogues ----------------
// C[M x N] = op(A)[M x K] . op(B)[K x N]; A is M x K (or K x M when TA), B is
// K x N (or N x K when TB); bf16 operands, fp32 accumulation. 64 x 64 tile per
// 256-thread block, four waves of 32 x 32 (2 x 2 v_mfma_f32_16x16x32_bf16).
enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_GELU_BACK = 2 };
constexpr int TK = 32, LDK = TK + 8;

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B, int M,
                                               int N, int K, float *__restrict__ C, uint16_t *__restrict__ Cb,
                                               const float *__restrict__ bias, const float *__restrict__ Zaux) {
    __shared__ __attribute__((aligned(16))) uint16_t As[64][LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[64][LDK];  // [n][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = tid * 8 + e;
            const int r = idx / TK, kk = idx % TK;
            const int gm = m0 + r, gk = k0 + kk;
            uint16_t v = 0;
            if (gm < M && gk < K) v = TA ? A[(int64_t)gk * M + gm] : A[(int64_t)gm * K + gk];
            As[r][kk] = v;
            const int gn = n0 + r;
            uint16_t w = 0;
            if (gn < N && gk < K) w = TB ? B[(int64_t)gn * K + gk] : B[(int64_t)gk * N + gn];
            Bs[r][kk] = w;
        }
        __syncthreads();
        const int kq = 8 * (lane >> 4);
#pragma unroll
        for (int tm = 0; tm < 2; ++tm) {
            const uint4 ua = *reinterpret_cast<const uint4 *>(&As[wm + tm * 16 + (lane & 15)][kq]);
            const bf16x8 a = __builtin_bit_cast(bf16x8, ua);
#pragma unroll
            for (int tn = 0; tn < 2; ++tn) {
                const uint4 ub = *reinterpret_cast<const uint4 *>(&Bs[wn + tn * 16 + (lane & 15)][kq]);
                const bf16x8 b = __builtin_bit_cast(bf16x8, ub);
                acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[tm][tn], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int tm = 0; tm < 2; ++tm)
#pragma unroll
        for (int tn = 0; tn < 2; ++tn)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + wm + tm * 16 + 4 * (lane >> 4) + i;
                const int col = n0 + wn + tn * 16 + (lane & 15);
                if (row >= M || col >= N) continue;
                const int64_t o = (int64_t)row * N + col;
                const float v = acc[tm][tn][i];
                if (EPI == EPI_STORE) {
                    C[o] = v;
                } else if (EPI == EPI_BIAS_GELU) {
                    const float z = v + bias[col];
                    if (C) C[o] = z;
                    Cb[o] = f2bf(gelu(z));
                } else {
                    const float d = v * gelu_grad(Zaux[o]);
                    C[o] = d;
                    Cb[o] = f2bf(d);
                }
            }
}

// ---------------- output layer, loss, small reductions, Adam ----------------
// y = h . w4 + b4 (one thread per row); with targets: dy = 2 (y - t) / m and
// block partials of (y - t)^2.
__global__ __launch_bounds__(256) void k_out_layer(int m, const uint16_t *__restrict__ H, const float *__restrict__ w4,
                                                    const float *__restrict__ b4, float *__restrict__ y,
                                                    const float *__restrict__ t, float *__restrict__ dy,
                                                    float *__restrict__ loss_part) {
    __shared__ float sh[4];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    float e2 = 0.f;
    if (r < m) {
        const uint4 *h = reinterpret_cast<const uint4 *>(H + (int64_t)r * 128);
        float s = b4[0];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const uint4 u = h[v];
            const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                s += bf2f((uint16_t)(w[q] & 0xFFFF)) * w4[8 * v + 2 * q];
                s += bf2f((uint16_t)(w[q] >> 16)) * w4[8 * v + 2 * q + 1];
            }
        }
        y[r] = s;
        if (t) {
            const float e = s - t[r];
            dy[r] = 2.f * e / (float)m;
            e2 = e * e;
        }
    }
    if (loss_part) {
        for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = e2;
        __syncthreads();
        if (threadIdx.x == 0) loss_part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
    }
}

// dZ3 = (dy w4^T) * gelu'(Z3): [m x 128]
__global__ void k_out_back(int m, const float *__restrict__ dy, const float *__restrict__ w4,
                           const float *__restrict__ Z, float *__restrict__ dZ, uint16_t *__restrict__ dZb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * 128) return;
    const int r = (int)(e / 128), c = (int)(e % 128);
    const float d = dy[r] * w4[c] * gelu_grad(Z[e]);
    dZ[e] = d;
    dZb[e] = f2bf(d);
}

// Column sums of X [m x ncol] (optionally weighted by w[m]) into part[block][ncol]; ncol <= 128.
__global__ __launch_bounds__(128) void k_colsum_part(int m, int ncol, const float *__restrict__ X,
                                                      const uint16_t *__restrict__ Xb, const float *__restrict__ w,
                                                      int rows_per_block, float *__restrict__ part) {
    const int c = threadIdx.x;
    if (c >= ncol) return;
    const int r0 = blockIdx.x * rows_per_block, r1 = min(m, r0 + rows_per_block);
    float s = 0.f;
    for (int r = r0; r < r1; ++r) {
        const float v = X ? X[(int64_t)r * ncol + c] : bf2f(Xb[(int64_t)r * ncol + c]);
        s += w ? v * w[r] : v;
    }
    part[(int64_t)blockIdx.x * ncol + c] = s;
}

__global__ void k_colsum_final(int nblk, int ncol, const float *__restrict__ part, float *__restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * ncol + c];
    out[c] = s;
}

// Adam on the float32 master parameters; refreshes the bf16 copy of the matrices.
__global__ void k_adam(int64_t np, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2,
                       uint16_t *__restrict__ pb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float v = p[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    p[i] = v;
    pb[i] = f2bf(v);
}

__global__ void k_to_bf16(int64_t n, const float *__restrict__ x, uint16_t *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// gather rows idx[0..m) of the inputs (64 bf16) and targets
__global__ void k_gather_rows(int m, const int32_t *__restrict__ idx, const uint16_t *__restrict__ F,
                              const float *__restrict__ T, uint16_t *__restrict__ Fb, float *__restrict__ Tb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * 8) return;
    const int r = (int)(e / 8), v = (int)(e % 8);
    const int64_t src = idx[r];
    reinterpret_cast<uint4 *>(Fb + (int64_t)r * 64)[v] = reinterpret_cast<const uint4 *>(F + src * 64)[v];
    if (v == 0 && T) Tb[r] = T[src];
}

// psi_guess = psi_prev + beta s^2 out, s = nu^(1/3) (grid order; beta: the step along the
// network's correction)
__global__ void k_apply_guess(int64_t n, const double *__restrict__ psi_prev, const double *__restrict__ nu,
                              const float *__restrict__ out, double beta, double *__restrict__ psi_new,
                              float4 *__restrict__ pos_s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = cbrt(nu[i]);
    const double v = psi_prev[i] + beta * s * s * (double)out[i];
    psi_new[i] = v;
    pos_s[i].w = (float)v;
}

inline int nblocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void launch_knn_features(hipStream_t st, int64_t n, const float4 *pos_s, const int32_t *perm,
                         const int32_t *cell_start, GridDesc g, const double *psi_prev_s, const double *nu_s,
                         const double *nu_sum, const double *V_s, int32_t *nbr, uint16_t *feat, int32_t *err) {
    hipLaunchKernelGGL(k_knn_features, dim3(nblocks(n, 256)), dim3(256), 0, st, n, pos_s, perm, cell_start, g,
                       psi_prev_s, nu_s, nu_sum, V_s, nbr, feat, err);
}

void launch_gemm(hipStream_t st, bool ta, bool tb, int epi, const uint16_t *A, const uint16_t *B, int M, int N, int K,
                 float *C, uint16_t *Cb, const float *bias, const float *Zaux) {
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
#define LAGOT_GEMM(TA, TB, E) hipLaunchKernelGGL((k_gemm<TA, TB, E>), grid, dim3(256), 0, st, A, B, M, N, K, C, Cb, bias, Zaux)
    if (!ta && !tb && epi == EPI_BIAS_GELU) LAGOT_GEMM(false, false, EPI_BIAS_GELU);
    else if (!ta && tb && epi == EPI_GELU_BACK) LAGOT_GEMM(false, true, EPI_GELU_BACK);
    else if (ta && !tb && epi == EPI_STORE) LAGOT_GEMM(true, false, EPI_STORE);
    else if (!ta && !tb && epi == EPI_STORE) LAGOT_GEMM(false, false, EPI_STORE);
#undef LAGOT_GEMM
}

void launch_out_layer(hipStream_t st, int m, const uint16_t *H, const float *w4, const float *b4, float *y,
                      const float *t, float *dy, float *loss_part) {
    hipLaunchKernelGGL(k_out_layer, dim3(nblocks(m, 256)), dim3(256), 0, st, m, H, w4, b4, y, t, dy, loss_part);
}

void launch_out_back(hipStream_t st, int m, const float *dy, const float *w4, const float *Z, float *dZ,
                     uint16_t *dZb) {
    hipLaunchKernelGGL(k_out_back, dim3(nblocks((int64_t)m * 128, 256)), dim3(256), 0, st, m, dy, w4, Z, dZ, dZb);
}

void launch_colsum(hipStream_t st, int m, int ncol, const float *X, const uint16_t *Xb, const float *w, float *part,
                   int max_part_blocks, float *out) {
    const int rpb = std::max(64, (m + max_part_blocks - 1) / max_part_blocks);
    const int nblk = (m + rpb - 1) / rpb;
    hipLaunchKernelGGL(k_colsum_part, dim3(nblk), dim3(128), 0, st, m, ncol, X, Xb, w, rpb, part);
    hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(128), 0, st, nblk, ncol, part, out);
}

void launch_adam(hipStream_t st, int64_t np, float *p, const float *g, float *m1, float *m2, float lr, float b1,
                 float b2, float eps, float c1, float c2, uint16_t *pb) {
    hipLaunchKernelGGL(k_adam, dim3(nblocks(np, 256)), dim3(256), 0, st, np, p, g, m1, m2, lr, b1, b2, eps, c1, c2,
                       pb);
}

void launch_to_bf16(hipStream_t st, int64_t n, const float *x, uint16_t *y) {
    hipLaunchKernelGGL(k_to_bf16, dim3(nblocks(n, 256)), dim3(256), 0, st, n, x, y);
}

void launch_gather_rows(hipStream_t st, int m, const int32_t *idx, const uint16_t *F, const float *T, uint16_t *Fb,
                        float *Tb) {
    hipLaunchKernelGGL(k_gather_rows, dim3(nblocks((int64_t)m * 8, 256)), dim3(256), 0, st, m, idx, F, T, Fb, Tb);
}

void launch_apply_guess(hipStream_t st, int64_t n, const double *psi_prev, const double *nu, const float *out,
                        double beta, double *psi_new, float4 *pos_s) {
    hipLaunchKernelGGL(k_apply_guess, dim3(nblocks(n, 256)), dim3(256), 0, st, n, psi_prev, nu, out, beta, psi_new,
                       pos_s);
}

}  // namespace lagot
