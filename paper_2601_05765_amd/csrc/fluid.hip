// fluid.hip -- the fluid model around the OT solve (section 5): the P1 Laplacian of
// eq. (3) over the restricted Laguerre facets, and the rows of the semi-implicit
// velocity system of eq. (4).
//
// The facet weights w_ij = Abar_ij / (2 |p_j - p_i|) are the off-diagonal entries of
// -Hess K, assembled by the Hessian kernels (union pattern, sorted rows, float32
// values, bit-symmetric). With mu_ij = (mu_i + mu_j) / 2 the velocity system is
//   (m_i/dt + sum_j mu_ij w_ij) v_i - sum_j mu_ij w_ij v_j = b_i,
//   b_i = (m_i/dt) v^k_i + m_i (c_i - p_i) / eps^2 + m_i g + gamma (Lap p)_i,
// symmetric positive definite, solved for the three coordinates at once by a Jacobi-PCG
// of the Newton direction's form (k_cg3_*). The diagonal is the row sum of the stored
// float32 off-diagonals plus m_i/dt, so every row of the viscous operator sums to zero
// exactly as stored and the solve conserves momentum up to its residual.
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

// Position update of the fluid step, x += dt v (section 5), kept inside the domain: each
// coordinate is clamped to [lo + m_a, hi - m_a] (m_a = margin * (hi_a - lo_a)), then, with
// convex domain planes n.x <= c, a site with n.x > c - m (m = margin * largest extent)
// is moved along -n onto n.x = c - m, in two passes over the planes. Every product and
// sum is rounded separately (no contraction), so the result is reproducible on any
// IEEE double implementation before the final rounding to float32.
// Inputs of the fluid step that must be valid before any site moves.
__global__ __launch_bounds__(FB) void k_fluid_check(int64_t n, const double *__restrict__ nu,
                                                    const double *__restrict__ mass, const double *__restrict__ mu,
                                                    const double *__restrict__ v, int32_t *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * FB + threadIdx.x;
    if (i >= n) return;
    bool ok = nu[i] > 0.0 && isfinite(nu[i]) && mass[i] > 0.0 && isfinite(mass[i]);
    for (int a = 0; a < 3; ++a) ok = ok && isfinite(v[3 * i + a]);
    if (mu) ok = ok && mu[i] >= 0.0 && isfinite(mu[i]);
    if (!ok) atomicAdd(bad, 1);
}

// The convex rule: a site beyond n.x = c - margin is moved along -n onto that plane, in
// two passes over the planes in order (every product and sum rounded separately).
__device__ inline void keep_in_planes(double p[3], const float4 *__restrict__ dom, int m, double margin) {
    for (int pass = 0; pass < 2; ++pass)
        for (int w = 0; w < m; ++w) {
            const float4 h = dom[w];
            const double nx = h.x, ny = h.y, nz = h.z;
            const double s = __dsub_rn(__dadd_rn(__dadd_rn(__dmul_rn(nx, p[0]), __dmul_rn(ny, p[1])),
                                                 __dmul_rn(nz, p[2])),
                                       (double)h.w);
            const double e = __dadd_rn(s, margin);
            if (e > 0.0) {
                p[0] = __dsub_rn(p[0], __dmul_rn(e, nx));
                p[1] = __dsub_rn(p[1], __dmul_rn(e, ny));
                p[2] = __dsub_rn(p[2], __dmul_rn(e, nz));
            }
        }
}

__global__ __launch_bounds__(FB) void k_advect(int64_t n, float *__restrict__ x, float *__restrict__ y,
                                               float *__restrict__ z, const double *__restrict__ v, double dt,
                                               AdvectBounds bd, const float4 *__restrict__ dom, int ndom,
                                               const int32_t *__restrict__ dom_off, int npieces) {
    const int64_t i = (int64_t)blockIdx.x * FB + threadIdx.x;
    if (i >= n) return;
    double p[3] = {(double)x[i], (double)y[i], (double)z[i]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double q = __dadd_rn(p[a], __dmul_rn(dt, v[3 * i + a]));
        p[a] = fmin(fmax(q, bd.lo[a]), bd.hi[a]);
    }
    if (npieces > 0) {
        // a union of convex pieces: the site stays if the convex rule of some piece leaves
        // it in place (it lies inside that piece by the margin), else it takes the nearest
        // of its places under the pieces' rules (ties to the first piece)
        double best[3] = {p[0], p[1], p[2]};
        double bestd = INFINITY;
        bool done = false;
        for (int k = 0; k < npieces && !done; ++k) {
            double q[3] = {p[0], p[1], p[2]};
            keep_in_planes(q, dom + dom_off[k], dom_off[k + 1] - dom_off[k], bd.plane_margin);
            const double dx = __dsub_rn(q[0], p[0]), dy = __dsub_rn(q[1], p[1]), dz = __dsub_rn(q[2], p[2]);
            const double d = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
            if (d < bestd) {
                best[0] = q[0];
                best[1] = q[1];
                best[2] = q[2];
                bestd = d;
            }
            done = d == 0.0;
        }
        p[0] = best[0];
        p[1] = best[1];
        p[2] = best[2];
    } else {
        keep_in_planes(p, dom, ndom, bd.plane_margin);
    }
    x[i] = (float)p[0];
    y[i] = (float)p[1];
    z[i] = (float)p[2];
}

// ---- three right-hand sides at once: Jacobi-PCG, Chronopoulos-Gear form ----------
// The three coordinates of the velocity system share the matrix, so one kernel per
// iteration advances all three (same recurrences as the Newton direction's PCG, with
// scalars, convergence and breakdown per coordinate): the row's entries and the
// neighbour indices are loaded once for the three, and the launch count drops by 3x.
// Per row and slot (iteration parity) one 80-byte record holds r, w = A u, s = A p of
// the three coordinates and the diagonal D. Every block sums the per-block partials
// in a fixed order (deterministic, no atomics, no device-scope fences).
constexpr int C3L = 2;             // lanes per row
constexpr int C3S = 128;           // rows per block
constexpr int C3B = C3L * C3S;     // threads per block
constexpr int CG3_SUM_IN_BLOCK = 2048;  // up to this many blocks, each block sums the partials itself

__device__ inline void load_rec3(const Rec3 *a, int64_t i, double *r, double *w, double *s, double &d) {
    const double2 *p = reinterpret_cast<const double2 *>(a + i);
    const double2 q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3], q4 = p[4];
    r[0] = q0.x; r[1] = q0.y; r[2] = q1.x;
    w[0] = q1.y; w[1] = q2.x; w[2] = q2.y;
    s[0] = q3.x; s[1] = q3.y; s[2] = q4.x;
    d = q4.y;
}

__device__ inline void store_rec3(Rec3 *a, int64_t i, const double *r, const double *w, const double *s, double d) {
    double2 *p = reinterpret_cast<double2 *>(a + i);
    p[0] = make_double2(r[0], r[1]);
    p[1] = make_double2(r[2], w[0]);
    p[2] = make_double2(w[1], w[2]);
    p[3] = make_double2(s[0], s[1]);
    p[4] = make_double2(s[2], d);
}

// Block sum of NV values per thread (one row of sh per wave); every thread gets the sums.
template <int NV> __device__ inline void block_sums(double *v, double (*sh)[NV]) {
#pragma unroll
    for (int q = 0; q < NV; ++q)
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    const int wv = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) sh[wv][q] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = 0.0;
        for (int k = 0; k < C3B / 64; ++k) t += sh[k][q];
        v[q] = t;
    }
}

// partial slots: [slot][9][NB] (gamma[3], delta[3], rho[3]) then rho0[3][NB]
__device__ inline double *P3(const Cg3Bufs &g, int slot, int q) { return g.part + ((int64_t)slot * 9 + q) * g.nb; }
__device__ inline double *P3_RHO0(const Cg3Bufs &g, int c) { return g.part + ((int64_t)18 + c) * g.nb; }

// r_0 = b, u_0 = r_0 / D, w_0 = A u_0, p_{-1} = s_{-1} = x_0 = 0
__global__ __launch_bounds__(C3B) void k_cg3_init(int64_t n, const int32_t *__restrict__ rp,
                                                  const int2 *__restrict__ ent, const double *__restrict__ diag,
                                                  const double *__restrict__ b, Cg3Bufs g) {
    __shared__ double sh[C3B / 64][12];
    const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);  // row blocks of one XCD are contiguous
    if (blk == 0 && threadIdx.x < 16) {
        if (threadIdx.x < 12) g.st[threadIdx.x] = 0;
        if (threadIdx.x == 12) *g.kbase = 0;
    }
    const int64_t row = (int64_t)blk * C3S + (int)(threadIdx.x / C3L);
    const int l = threadIdx.x & (C3L - 1);
    const bool has = row < n;
    double acc[3] = {0.0, 0.0, 0.0};
    if (has) {
        const int e1 = rp[row + 1];
        for (int f = rp[row] + l; f < e1; f += C3L) {
            const int2 e = ent[f];
            const int j = e.x;
            const double v = (double)__int_as_float(e.y) / diag[j];
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[q] = fma(v, b[q * n + j], acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
        for (int o = C3L / 2; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, C3L);
    double part[12] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (has && l == 0) {
        const double d = diag[row];
        double r[3], w[3], z[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            r[q] = b[q * n + row];
            const double u = r[q] / d;
            w[q] = d * u - acc[q];
            part[q] = r[q] * u;          // gamma
            part[3 + q] = w[q] * u;      // delta
            part[6 + q] = r[q] * r[q];   // rho
            g.p[3 * row + q] = 0.0;
            g.x[3 * row + q] = 0.0;
        }
        store_rec3(g.rec[0], row, r, w, z, d);
    }
    block_sums<12>(part, sh);
    if (threadIdx.x == 0) {
        for (int q = 0; q < 9; ++q) P3(g, 0, q)[blk] = part[q];
        for (int q = 0; q < 3; ++q) P3_RHO0(g, q)[blk] = part[6 + q];
    }
}

// Iteration k = *kbase + m of the three systems (the host advances kbase per chunk).
__global__ __launch_bounds__(C3B) void k_cg3_iter(int64_t n, int m, double rtol2, int cap,
                                                  const int32_t *__restrict__ rp, const int2 *__restrict__ ent,
                                                  Cg3Bufs g) {
    __shared__ double sh[C3B / 64][12];
    const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);  // row blocks of one XCD are contiguous
    const int k = *g.kbase + m;
    if (k >= cap) return;
    bool act[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) act[q] = g.st[4 * q + 1] == 0 && g.st[4 * q + 2] == 0;
    if (!act[0] && !act[1] && !act[2]) return;
    const int cur = k & 1, nxt = cur ^ 1;
    const int64_t row = (int64_t)blk * C3S + (int)(threadIdx.x / C3L);
    const int l = threadIdx.x & (C3L - 1);
    const bool has = row < n;
    // scalars of iteration k: summed by the block itself from every block's partials when
    // the blocks are few, else once per iteration by k_cg3_scalars
    double S[12];
    if (g.nb <= CG3_SUM_IN_BLOCK) {
#pragma unroll
        for (int q = 0; q < 12; ++q) S[q] = 0.0;
        for (int t = (int)threadIdx.x; t < g.nb; t += C3B) {
#pragma unroll
            for (int q = 0; q < 9; ++q) S[q] += P3(g, cur, q)[t];
#pragma unroll
            for (int q = 0; q < 3; ++q) S[9 + q] += P3_RHO0(g, q)[t];
        }
        block_sums<12>(S, sh);
    } else {
#pragma unroll
        for (int q = 0; q < 12; ++q) S[q] = g.sc[12 * cur + q];
    }
    const bool lead = blk == 0 && threadIdx.x == 0;
    double alpha[3] = {0.0, 0.0, 0.0}, beta[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (!act[q]) continue;
        const double gam = S[q], del = S[3 + q], rho = S[6 + q], rho0 = S[9 + q];
        if (rho <= rtol2 * rho0) {
            act[q] = false;
            if (lead) {
                g.st[4 * q + 2] = 1;
                g.st[4 * q + 0] = k;
            }
            continue;
        }
        if (k == 0) {
            alpha[q] = gam / del;
        } else {
            const double pa = g.cgs[6 * nxt + 2 * q], pg = g.cgs[6 * nxt + 2 * q + 1];  // alpha, gamma of k-1
            beta[q] = gam / pg;
            alpha[q] = gam / (del - beta[q] * gam / pa);
        }
        if (!(alpha[q] > 0.0) || !(alpha[q] < 1e300)) {  // non-positive curvature (or NaN)
            act[q] = false;
            if (lead) {
                g.st[4 * q + 1] = 1;
                g.st[4 * q + 0] = k;
            }
            continue;
        }
        if (lead) {
            g.cgs[6 * cur + 2 * q] = alpha[q];
            g.cgs[6 * cur + 2 * q + 1] = gam;
            g.st[4 * q + 0] = k + 1;
        }
    }
    if (!act[0] && !act[1] && !act[2]) return;  // the same decision in every block
    const Rec3 *crec = g.rec[cur];
    // u_{k+1} of each neighbour from its stored r_k, w_k, s_{k-1}
    double acc[3] = {0.0, 0.0, 0.0};
    if (has) {
        const int e1 = rp[row + 1];
        for (int f = rp[row] + l; f < e1; f += C3L) {
            const int2 e = ent[f];
            double r[3], w[3], s[3], d;
            load_rec3(crec, e.x, r, w, s, d);
            const double v = (double)__int_as_float(e.y) / d;
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[q] = fma(v, fma(-alpha[q], fma(beta[q], s[q], w[q]), r[q]), acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
        for (int o = C3L / 2; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, C3L);
    double part[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (has && l == 0) {
        double r[3], w[3], s[3], d;
        load_rec3(crec, row, r, w, s, d);
        double r1[3], w1[3], s1[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (act[q]) {
                const double uk = r[q] / d;
                const double pk = fma(beta[q], g.p[3 * row + q], uk);
                const double sk = fma(beta[q], s[q], w[q]);
                g.x[3 * row + q] = fma(alpha[q], pk, g.x[3 * row + q]);
                g.p[3 * row + q] = pk;
                r1[q] = fma(-alpha[q], sk, r[q]);
                const double u1 = r1[q] / d;
                w1[q] = d * u1 - acc[q];
                s1[q] = sk;
                part[q] = r1[q] * u1;
                part[3 + q] = w1[q] * u1;
                part[6 + q] = r1[q] * r1[q];
            } else {
                r1[q] = r[q];
                w1[q] = w[q];
                s1[q] = s[q];
            }
        }
        store_rec3(g.rec[nxt], row, r1, w1, s1, d);
    }
    block_sums<9>(part, reinterpret_cast<double (*)[9]>(&sh[0][0]));
    if (threadIdx.x == 0)
        for (int q = 0; q < 9; ++q) P3(g, nxt, q)[blk] = part[q];
}

// The scalars of the next iteration: the partials of the slot just written, summed once
// in a fixed order (deterministic) by one block, instead of by every block of the next
// iteration (quadratic in the number of blocks).
__global__ __launch_bounds__(C3B) void k_cg3_scalars(int m, int cap, Cg3Bufs g) {
    __shared__ double sh[C3B / 64][12];
    int slot = 0;
    if (m >= 0) {
        const int k = *g.kbase + m;
        if (k >= cap) return;
        slot = (k + 1) & 1;
    }
    double S[12] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int t = (int)threadIdx.x; t < g.nb; t += C3B) {
#pragma unroll
        for (int q = 0; q < 9; ++q) S[q] += P3(g, slot, q)[t];
#pragma unroll
        for (int q = 0; q < 3; ++q) S[9 + q] += P3_RHO0(g, q)[t];
    }
    block_sums<12>(S, sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < 12; ++q) g.sc[12 * slot + q] = S[q];
}

// After a chunk: advance kbase; count the coordinates still iterating.
__global__ void k_cg3_advance(int chunk, int cap, Cg3Bufs g) {
    if (threadIdx.x != 0) return;
    int cnt = 0;
    for (int q = 0; q < 3; ++q) cnt += g.st[4 * q + 1] == 0 && g.st[4 * q + 2] == 0 && g.st[4 * q] < cap;
    *g.kbase += chunk;
    *g.remaining = cnt;
}

// The rows of the scaled matrix packed back to back, (column, value bits) per entry:
// the PCG then reads one contiguous run per row instead of two 64-entry row blocks.
__global__ __launch_bounds__(FB) void k_pack_rows(int64_t n, const int32_t *__restrict__ hcol,
                                                  const float *__restrict__ hval, const int32_t *__restrict__ hcnt,
                                                  const int32_t *__restrict__ rp, int2 *__restrict__ ent) {
    const int64_t i = (int64_t)xcd_block((int)blockIdx.x, (int)gridDim.x) * FB + threadIdx.x;
    if (i >= n) return;
    const int c = hcnt[i], o = rp[i];
    for (int f = 0; f < c; ++f) ent[o + f] = make_int2(hcol[i * FCAP + f], __float_as_int(hval[i * FCAP + f]));
}

// out[3 perm[i] + q] = x[3 i + q]
__global__ __launch_bounds__(FB) void k_scatter3(int64_t n, const int32_t *__restrict__ perm,
                                                 const double *__restrict__ x, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * FB + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
#pragma unroll
    for (int q = 0; q < 3; ++q) out[3 * o + q] = x[3 * i + q];
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

void launch_fluid_check(hipStream_t st, int64_t n, const double *nu, const double *mass, const double *mu,
                        const double *v, int32_t *bad) {
    hipLaunchKernelGGL(k_fluid_check, dim3(nb(n)), dim3(FB), 0, st, n, nu, mass, mu, v, bad);
}

void launch_advect(hipStream_t st, int64_t n, float *x, float *y, float *z, const double *v, double dt,
                   const AdvectBounds &bd, const float4 *dom, int ndom, const int32_t *dom_off, int npieces) {
    hipLaunchKernelGGL(k_advect, dim3(nb(n)), dim3(FB), 0, st, n, x, y, z, v, dt, bd, dom, ndom, dom_off, npieces);
}

int cg3_blocks(int64_t n) { return (int)((n + C3S - 1) / C3S); }

void launch_pack_rows(hipStream_t st, int64_t n, const int32_t *hcol, const float *hval, const int32_t *hcnt,
                      const int32_t *rp, int2 *ent) {
    hipLaunchKernelGGL(k_pack_rows, dim3(nb(n)), dim3(FB), 0, st, n, hcol, hval, hcnt, rp, ent);
}

void launch_cg3_init(hipStream_t st, int64_t n, const int32_t *rp, const int2 *ent, const double *diag,
                     const double *b, const Cg3Bufs &g) {
    hipLaunchKernelGGL(k_cg3_init, dim3(cg3_blocks(n)), dim3(C3B), 0, st, n, rp, ent, diag, b, g);
}

void launch_cg3_iter(hipStream_t st, int64_t n, int m, double rtol2, int cap, const int32_t *rp, const int2 *ent,
                     const Cg3Bufs &g) {
    hipLaunchKernelGGL(k_cg3_iter, dim3(cg3_blocks(n)), dim3(C3B), 0, st, n, m, rtol2, cap, rp, ent, g);
}

void launch_cg3_scalars(hipStream_t st, int m, int cap, const Cg3Bufs &g) {
    if (g.nb <= CG3_SUM_IN_BLOCK) return;  // the iteration's blocks sum the partials themselves
    hipLaunchKernelGGL(k_cg3_scalars, dim3(1), dim3(C3B), 0, st, m, cap, g);
}

void launch_cg3_advance(hipStream_t st, int chunk, int cap, const Cg3Bufs &g) {
    hipLaunchKernelGGL(k_cg3_advance, dim3(1), dim3(64), 0, st, chunk, cap, g);
}

void launch_scatter3(hipStream_t st, int64_t n, const int32_t *perm, const double *x, double *out) {
    hipLaunchKernelGGL(k_scatter3, dim3(nb(n)), dim3(FB), 0, st, n, perm, x, out);
}

}  // namespace lagot
