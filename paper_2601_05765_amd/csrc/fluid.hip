// fluid.hip -- the fluid model around the OT solve (section 5): the P1 Laplacian of
// eq. (3) over the restricted Laguerre facets, and the rows of the semi-implicit
// velocity system of eq. (4).
//
// The facet weights w_ij = Abar_ij / (2 |p_j - p_i|) are the off-diagonal entries of
// -Hess K, assembled by the Hessian kernels (union pattern, sorted rows, float32
// values, bit-symmetric). With mu_ij = (mu_i + mu_j) / 2 the velocity system is
//   (m_i/dt + sum_j mu_ij w_ij) v_i - sum_j mu_ij w_ij v_j = b_i,
//   b_i = (m_i/dt) v^k_i + m_i (c_i - p_i) / eps^2 + m_i g + gamma (Lap p)_i,
// symmetric positive definite, solved per coordinate by the Jacobi-PCG of the Newton
// direction. The diagonal is the row sum of the stored float32 off-diagonals plus
// m_i/dt, so every row of the viscous operator sums to zero exactly as stored and the
// solve conserves momentum up to its residual.
//
// Rows are in grid order (the solver's sort); caller-order arrays are read and written
// through perm (perm[i] = caller index of grid row i).
#include "lagot_internal.h"

namespace lagot {
namespace {

constexpr int FB = 256;  // threads per block, one row per thread

// One row of the velocity system. Also rescales the row's stored weights from w_ij to
// mu_ij w_ij (in place: a row is read and written by its own thread only). bad counts
// rows with a non-positive or non-finite mass, a negative or non-finite viscosity or
// a non-finite velocity.
__global__ __launch_bounds__(FB) void k_fluid_rows(int64_t n, const int32_t *__restrict__ perm,
                                                   const float4 *__restrict__ pos_s, const int32_t *__restrict__ hcol,
                                                   float *__restrict__ hval, const int32_t *__restrict__ hcnt,
                                                   const double *__restrict__ mass, const double *__restrict__ mu,
                                                   FluidPrm fp, const double *__restrict__ v,
                                                   const double *__restrict__ cen, double *__restrict__ diag,
                                                   double *__restrict__ b, int32_t *__restrict__ bad) {
    const int64_t i = (int64_t)xcd_block((int)blockIdx.x, (int)gridDim.x) * FB + threadIdx.x;
    if (i >= n) return;
    const int o = perm[i];
    const double m = mass[o];
    const double mui = mu ? mu[o] : fp.mu;
    const double vx = v[3 * (int64_t)o], vy = v[3 * (int64_t)o + 1], vz = v[3 * (int64_t)o + 2];
    if (!(m > 0.0) || !(m < INFINITY) || !(mui >= 0.0) || !(mui < INFINITY) || !isfinite(vx) || !isfinite(vy) ||
        !isfinite(vz))
        atomicAdd(bad, 1);
    const float4 pf = pos_s[i];
    const double px = pf.x, py = pf.y, pz = pf.z;
    const int c = hcnt[i];
    const int32_t *cr = hcol + i * FCAP;
    float *vr = hval + i * FCAP;
    double lx = 0.0, ly = 0.0, lz = 0.0, dsum = 0.0;
    for (int f = 0; f < c; ++f) {
        const int j = cr[f];
        const double w = vr[f];
        const float4 q = pos_s[j];
        lx = fma(w, (double)q.x - px, lx);
        ly = fma(w, (double)q.y - py, ly);
        lz = fma(w, (double)q.z - pz, lz);
        const double muj = mu ? mu[perm[j]] : fp.mu;
        const float wm = (float)(0.5 * (mui + muj) * w);
        vr[f] = wm;
        dsum += (double)wm;
    }
    const double mdt = m / fp.dt;
    diag[i] = mdt + dsum;
    const double cx = cen[3 * (int64_t)o], cy = cen[3 * (int64_t)o + 1], cz = cen[3 * (int64_t)o + 2];
    b[i] = mdt * vx + m * (cx - px) * fp.inv_eps2 + m * fp.g[0] + fp.gamma * lx;
    b[n + i] = mdt * vy + m * (cy - py) * fp.inv_eps2 + m * fp.g[1] + fp.gamma * ly;
    b[2 * n + i] = mdt * vz + m * (cz - pz) * fp.inv_eps2 + m * fp.g[2] + fp.gamma * lz;
}

// (Lap_mu u)_i = sum_j mu_ij w_ij (u_j - u_i) for a caller-order field u [3n]; the
// result goes to out [3n] in caller order. mu == null: mu_ij = mu0.
__global__ __launch_bounds__(FB) void k_p1_laplacian(int64_t n, const int32_t *__restrict__ perm,
                                                     const int32_t *__restrict__ hcol, const float *__restrict__ hval,
                                                     const int32_t *__restrict__ hcnt, const double *__restrict__ mu,
                                                     double mu0, const double *__restrict__ u,
                                                     double *__restrict__ out, int32_t *__restrict__ bad) {
    const int64_t i = (int64_t)xcd_block((int)blockIdx.x, (int)gridDim.x) * FB + threadIdx.x;
    if (i >= n) return;
    const int o = perm[i];
    const double mui = mu ? mu[o] : mu0;
    if (!(mui >= 0.0) || !(mui < INFINITY)) atomicAdd(bad, 1);
    const double ux = u[3 * (int64_t)o], uy = u[3 * (int64_t)o + 1], uz = u[3 * (int64_t)o + 2];
    const int c = hcnt[i];
    const int32_t *cr = hcol + i * FCAP;
    const float *vr = hval + i * FCAP;
    double lx = 0.0, ly = 0.0, lz = 0.0;
    for (int f = 0; f < c; ++f) {
        const int oj = perm[cr[f]];
        const double muj = mu ? mu[oj] : mu0;
        const double w = 0.5 * (mui + muj) * (double)vr[f];
        lx = fma(w, u[3 * (int64_t)oj] - ux, lx);
        ly = fma(w, u[3 * (int64_t)oj + 1] - uy, ly);
        lz = fma(w, u[3 * (int64_t)oj + 2] - uz, lz);
    }
    out[3 * (int64_t)o] = lx;
    out[3 * (int64_t)o + 1] = ly;
    out[3 * (int64_t)o + 2] = lz;
}

// out[3 perm[i] + comp] = x[i]
__global__ __launch_bounds__(FB) void k_scatter_comp(int64_t n, const int32_t *__restrict__ perm,
                                                     const double *__restrict__ x, int comp, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * FB + threadIdx.x;
    if (i < n) out[3 * (int64_t)perm[i] + comp] = x[i];
}

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t value) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

__global__ void k_zero_f64(double *p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

// Position update of the fluid step, x += dt v (section 5), kept inside the domain: each
// coordinate is clamped to [lo + m_a, hi - m_a] (m_a = margin * (hi_a - lo_a)), then, with
// convex domain planes n.x <= c, a site with n.x > c - m (m = margin * largest extent)
// is moved along -n onto n.x = c - m, in two passes over the planes. Every product and
// sum is rounded separately (no contraction), so the result is reproducible on any
// IEEE double implementation before the final rounding to float32.
__global__ __launch_bounds__(FB) void k_advect(int64_t n, float *__restrict__ x, float *__restrict__ y,
                                               float *__restrict__ z, const double *__restrict__ v, double dt,
                                               AdvectBounds bd, const float4 *__restrict__ dom, int ndom) {
    const int64_t i = (int64_t)blockIdx.x * FB + threadIdx.x;
    if (i >= n) return;
    double p[3] = {(double)x[i], (double)y[i], (double)z[i]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double q = __dadd_rn(p[a], __dmul_rn(dt, v[3 * i + a]));
        p[a] = fmin(fmax(q, bd.lo[a]), bd.hi[a]);
    }
    for (int pass = 0; pass < 2; ++pass)
        for (int w = 0; w < ndom; ++w) {
            const float4 h = dom[w];
            const double nx = h.x, ny = h.y, nz = h.z;
            const double s = __dsub_rn(__dadd_rn(__dadd_rn(__dmul_rn(nx, p[0]), __dmul_rn(ny, p[1])),
                                                 __dmul_rn(nz, p[2])),
                                       (double)h.w);
            const double e = __dadd_rn(s, bd.plane_margin);
            if (e > 0.0) {
                p[0] = __dsub_rn(p[0], __dmul_rn(e, nx));
                p[1] = __dsub_rn(p[1], __dmul_rn(e, ny));
                p[2] = __dsub_rn(p[2], __dmul_rn(e, nz));
            }
        }
    x[i] = (float)p[0];
    y[i] = (float)p[1];
    z[i] = (float)p[2];
}

inline unsigned nb(int64_t n) { return (unsigned)((n + FB - 1) / FB); }

}  // namespace

void launch_fluid_rows(hipStream_t st, int64_t n, const int32_t *perm, const float4 *pos_s, const int32_t *hcol,
                       float *hval, const int32_t *hcnt, const double *mass, const double *mu, const FluidPrm &fp,
                       const double *v, const double *cen, double *diag, double *b, int32_t *bad) {
    hipLaunchKernelGGL(k_fluid_rows, dim3(nb(n)), dim3(FB), 0, st, n, perm, pos_s, hcol, hval, hcnt, mass, mu, fp, v,
                       cen, diag, b, bad);
}

void launch_p1_laplacian(hipStream_t st, int64_t n, const int32_t *perm, const int32_t *hcol, const float *hval,
                         const int32_t *hcnt, const double *mu, double mu0, const double *u, double *out,
                         int32_t *bad) {
    hipLaunchKernelGGL(k_p1_laplacian, dim3(nb(n)), dim3(FB), 0, st, n, perm, hcol, hval, hcnt, mu, mu0, u, out, bad);
}

void launch_scatter_comp(hipStream_t st, int64_t n, const int32_t *perm, const double *x, int comp, double *out) {
    hipLaunchKernelGGL(k_scatter_comp, dim3(nb(n)), dim3(FB), 0, st, n, perm, x, comp, out);
}

void launch_fill_i32(hipStream_t st, int32_t *p, int64_t count, int32_t value) {
    hipLaunchKernelGGL(k_fill_i32, dim3(nb(count)), dim3(FB), 0, st, p, count, value);
}

void launch_advect(hipStream_t st, int64_t n, float *x, float *y, float *z, const double *v, double dt,
                   const AdvectBounds &bd, const float4 *dom, int ndom) {
    hipLaunchKernelGGL(k_advect, dim3(nb(n)), dim3(FB), 0, st, n, x, y, z, v, dt, bd, dom, ndom);
}

void launch_zero_f64(hipStream_t st, double *p, int64_t count) {
    hipLaunchKernelGGL(k_zero_f64, dim3(nb(count)), dim3(FB), 0, st, p, count);
}

}  // namespace lagot
