// cells.hip -- evaluation of every generalized Laguerre cell
//   C_i = box ∩ B(p_i, sqrt(psi_i)) ∩ {power_i <= power_j  for all j}      (eq. (1))
// fused in one kernel: candidate bisectors (cell_clip input), convex clipping
// (cell_clip, section 4 "Cell Update"), and the analytic restriction to the
// ball (ball_cell_integrate, section 3.2-3.3 and Algorithm 2).
//
// Mapping (MI355X, wave64): one 64-lane workgroup holds 64/G cells, G lanes per
// cell. A cell lives in LDS: its candidate planes, the polytope as a set of
// vertex triangles (each vertex stores the three planes meeting there, in
// counter-clockwise order seen from outside, plus its position), and small
// per-plane tables. Lanes of a group own strided vertex slots and planes;
// ballots give ranks; all cross-lane traffic goes through LDS.
//
// Clipping by a plane k: vertices beyond k are marked; for every plane x the
// removed triangles around it give an out-set and an in-set of neighbour planes
// (bitmasks); x lies on the cut boundary iff out \ in is a single plane y, and
// the new vertex on edge x∩y is interpolated between the kept and the removed
// end of that edge. The new triangles are (x, y, k). Euler's relation
// T = 2F - 4 checks the combinatorics after every cut; a violation, or any
// capacity overflow, flags the cell for the float64 large-capacity path.
//
// Restriction (section 3.2 "triangles and circular sectors", section 3.3 occlusion
// identity with the projection centre at p_i, section 3.2 pyramids): each face
// polygon is walked counter-clockwise; every edge (P,Q) contributes the signed
// fan piece triangle(q,P,Q) ∩ disk(q, rho), q = t n, split into at most two
// circular sectors and one triangle. Planar area and the solid angle seen from
// p_i are summed per face; then
//   K = r^2 (4 pi [p_i in C_i] - sum_f sgn(t_f) Omega_f),  V = (sum_f t_f A_f + r K) / 3.
#include "lagot_internal.h"

namespace lagot {
namespace {

constexpr uint32_t TRI_INVALID = 0xFFFFFFFFu;
constexpr uint32_t TRI_REMOVED = 0x80000000u;
constexpr double PI_D = 3.14159265358979323846;

template <int PMAX> struct MaskType { using T = uint32_t; };
template <> struct MaskType<64> { using T = unsigned long long; };

__device__ inline int popc(uint32_t v) { return __popc(v); }
__device__ inline int popc(unsigned long long v) { return __popcll(v); }
__device__ inline int ctz_(uint32_t v) { return __ffs(v) - 1; }
__device__ inline int ctz_(unsigned long long v) { return __ffsll(v) - 1; }

__device__ inline uint32_t pack3(int a, int b, int c) { return (uint32_t)a | ((uint32_t)b << 8) | ((uint32_t)c << 16); }

template <int G> __device__ inline unsigned long long gballot(bool pred) {
    unsigned long long b = __ballot(pred);
    if constexpr (G == 64) {
        return b;
    } else {
        const int base = (int)(threadIdx.x & (64 - G));
        return (b >> base) & ((1ull << G) - 1ull);
    }
}

template <int G> __device__ inline unsigned long long lanes_below() {
    const int gl = (int)(threadIdx.x & (G - 1));
    return (1ull << gl) - 1ull;
}

template <int G, typename T> __device__ inline T gsum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int G> __device__ inline int gmax(int v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

template <typename R> __device__ inline R dot3(R ax, R ay, R az, R bx, R by, R bz) { return ax * bx + ay * by + az * bz; }

template <typename R> __device__ inline R rsqrt_(R v);
template <> __device__ inline float rsqrt_<float>(float v) { return rsqrtf(v); }
template <> __device__ inline double rsqrt_<double>(double v) { return 1.0 / sqrt(v); }
template <typename R> __device__ inline R atan2_(R y, R x);
template <> __device__ inline float atan2_<float>(float y, float x) { return atan2f(y, x); }
template <> __device__ inline double atan2_<double>(double y, double x) { return atan2(y, x); }

// Signed circular sector of the disk between in-plane directions u and v.
template <typename R>
__device__ inline void sector(R ux, R uy, R uz, R vx, R vy, R vz, R nx, R ny, R nz, R half_rho2, R cone, R &A,
                              R &Om) {
    R cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    R phi = atan2_<R>(dot3(nx, ny, nz, cx, cy, cz), dot3(ux, uy, uz, vx, vy, vz));
    A += half_rho2 * phi;
    Om += cone * phi;
}

// One fan piece: triangle (q, q+u, q+v) ∩ disk(q, rho). h = |t|, cone = 1 - h/r.
template <typename R>
__device__ inline void fan_piece(R ux, R uy, R uz, R vx, R vy, R vz, R nx, R ny, R nz, R rho2, R h, R cone, R &A,
                                 R &Om) {
    const R wx = vx - ux, wy = vy - uy, wz = vz - uz;
    const R a = dot3(wx, wy, wz, wx, wy, wz);
    if (!(a > R(0))) return;
    const R b = dot3(ux, uy, uz, wx, wy, wz);
    const R c = dot3(ux, uy, uz, ux, uy, uz) - rho2;
    const R disc = b * b - a * c;
    R lo = R(1), hi = R(0);
    if (disc > R(0)) {
        const R sq = sqrt(disc);
        const R ia = R(1) / a;
        lo = fmax((-b - sq) * ia, R(0));
        hi = fmin((-b + sq) * ia, R(1));
    }
    const R half_rho2 = R(0.5) * rho2;
    if (!(lo < hi)) {
        sector<R>(ux, uy, uz, vx, vy, vz, nx, ny, nz, half_rho2, cone, A, Om);
        return;
    }
    const R ax = ux + lo * wx, ay = uy + lo * wy, az = uz + lo * wz;
    const R bx = ux + hi * wx, by = uy + hi * wy, bz = uz + hi * wz;
    sector<R>(ux, uy, uz, ax, ay, az, nx, ny, nz, half_rho2, cone, A, Om);
    sector<R>(bx, by, bz, vx, vy, vz, nx, ny, nz, half_rho2, cone, A, Om);
    // triangle (q, q+a, q+b) inside the disk: planar area and Van Oosterom-Strackee solid angle
    const R cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
    const R s = dot3(nx, ny, nz, cx, cy, cz);
    A += R(0.5) * s;
    const R h2 = h * h;
    const R la = sqrt(dot3(ax, ay, az, ax, ay, az) + h2);
    const R lb = sqrt(dot3(bx, by, bz, bx, by, bz) + h2);
    Om += R(2) * atan2_<R>(s, la * lb + h * (la + lb) + h2 + dot3(ax, ay, az, bx, by, bz));
}

template <typename R, int CMAX, int PMAX, int VMAX> struct CellSmem {
    using M = typename MaskType<PMAX>::T;
    R cand[CMAX][4];       // candidate plane: unit normal, signed distance t
    int32_t cid[CMAX];     // neighbour (grid-order index) or -1-w for wall w
    uint8_t corder[CMAX];  // candidates in ascending t
    R pl[PMAX][4];         // polytope planes (0..5 auxiliary cube)
    int32_t pid[PMAX];
    uint32_t tri[VMAX];    // vertex = planes (a,b,c) packed, TRI_INVALID if free
    R vp[VMAX][3];         // vertex position relative to p_i
    union {
        struct {
            M mout[PMAX];
            M min[PMAX];
            uint8_t nxt[PMAX];
            uint8_t newl[PMAX];
            uint8_t rslot[PMAX];
            uint8_t kslot[PMAX];
            R newpos[PMAX][3];  // positions of the new vertices, by rank
        } c;
        struct {
            uint8_t eslot[PMAX][PMAX];  // directed edge a->b  ->  vertex slot holding it
            uint8_t fstart[PMAX];
            R farea[PMAX];
        } g;
    } u;
};

struct CellArgs {
    int64_t n;
    const float4 *pos_s;      // x, y, z, float32 psi (grid order)
    const double *psi_s;      // float64 psi (grid order); used by the float64 path
    const int32_t *perm;      // grid order -> caller index (tie rule for coincident sites)
    const int32_t *cell_start;
    GridDesc g;
    BoxF box;
    const double *rmax;
    EvalOut out;
};

template <typename R, int G, int CMAX, int PMAX, int VMAX>
__device__ void cell_body(int64_t cell, const CellArgs &A, CellSmem<R, CMAX, PMAX, VMAX> &S, bool fast) {
    using M = typename MaskType<PMAX>::T;
    static_assert(VMAX <= 255 && PMAX <= 64 && CMAX <= 256, "slot indices are bytes");
    const int gl = (int)(threadIdx.x & (G - 1));
    const unsigned long long below = lanes_below<G>();
    const bool act = cell >= 0;
    uint32_t flags = 0;

    R px = 0, py = 0, pz = 0, psi_i = 0;
    if (act) {
        const float4 p4 = A.pos_s[cell];
        px = p4.x;
        py = p4.y;
        pz = p4.z;
        psi_i = fast ? (R)p4.w : (R)A.psi_s[cell];
    }
    bool live = act && (psi_i > R(0));
    if (act && !live) flags |= CF_EMPTY;
    const R r = live ? sqrt(psi_i) : R(0);

    // ---------------- candidate bisectors: grid cells within r + r_max ----------------
    int ncand = 0;
    bool inside = true;
    bool empty = false;
    if (live) {
        const float reach = ((float)r + (float)(*A.rmax)) * 1.0001f;
        int lo3[3], hi3[3];
        const float pp[3] = {(float)px, (float)py, (float)pz};
        for (int a = 0; a < 3; ++a) {
            lo3[a] = max((int)floorf((pp[a] - reach - A.g.lo[a]) * A.g.inv_s), 0);
            hi3[a] = min((int)floorf((pp[a] + reach - A.g.lo[a]) * A.g.inv_s), A.g.dim[a] - 1);
        }
        for (int ix = lo3[0]; ix <= hi3[0]; ++ix) {
            for (int iy = lo3[1]; iy <= hi3[1]; ++iy) {
                const int col = (ix * A.g.dim[1] + iy) * A.g.dim[2];
                const int beg = A.cell_start[col + lo3[2]];
                const int end = A.cell_start[col + hi3[2] + 1];
                for (int base = beg; base < end; base += G) {
                    const int j = base + gl;
                    bool keep = false, kill = false, neg = false;
                    R nx = 0, ny = 0, nz = 0, t = 0;
                    if (j < end && j != cell) {
                        const float4 q4 = A.pos_s[j];
                        const R psi_j = fast ? (R)q4.w : (R)A.psi_s[j];
                        const R dx = (R)q4.x - px, dy = (R)q4.y - py, dz = (R)q4.z - pz;
                        const R d2 = dot3(dx, dy, dz, dx, dy, dz);
                        if (d2 > R(0)) {
                            const R id = rsqrt_<R>(d2);
                            t = (d2 + psi_i - psi_j) * (R(0.5) * id);
                            if (t <= -r) {
                                kill = true;
                            } else if (t < r) {
                                keep = true;
                                neg = t < R(0);
                                nx = dx * id;
                                ny = dy * id;
                                nz = dz * id;
                            }
                        } else {
                            // coincident sites: the larger weight, then the lower caller index, owns the point
                            kill = psi_j > psi_i || (psi_j == psi_i && A.perm[j] < A.perm[cell]);
                        }
                    }
                    const unsigned long long b = gballot<G>(keep);
                    if (keep) {
                        const int c = ncand + popc(b & below);
                        if (c < CMAX) {
                            S.cand[c][0] = nx;
                            S.cand[c][1] = ny;
                            S.cand[c][2] = nz;
                            S.cand[c][3] = t;
                            S.cid[c] = j;
                        }
                    }
                    ncand += popc(b);
                    if (gballot<G>(kill)) empty = true;
                    if (gballot<G>(neg)) inside = false;
                }
            }
        }
        // box walls -x,+x,-y,+y,-z,+z: t = distance from p_i to the wall
        {
            bool keep = false;
            R t = 0;
            if (gl < 6) {
                const int ax = gl >> 1;
                const R pc = ax == 0 ? px : (ax == 1 ? py : pz);
                t = (gl & 1) ? (R)A.box.hi[ax] - pc : pc - (R)A.box.lo[ax];
                keep = t < r;
            }
            const unsigned long long b = gballot<G>(keep);
            if (keep) {
                const int c = ncand + popc(b & below);
                if (c < CMAX) {
                    const int ax = gl >> 1;
                    S.cand[c][0] = ax == 0 ? ((gl & 1) ? R(1) : R(-1)) : R(0);
                    S.cand[c][1] = ax == 1 ? ((gl & 1) ? R(1) : R(-1)) : R(0);
                    S.cand[c][2] = ax == 2 ? ((gl & 1) ? R(1) : R(-1)) : R(0);
                    S.cand[c][3] = t;
                    S.cid[c] = -1 - gl;
                }
            }
            ncand += popc(b);
        }
        if (empty) {
            flags |= CF_EMPTY;
            live = false;
        } else if (ncand > CMAX) {
            flags |= CF_CAND;
            live = false;
        }
    }
    __syncthreads();

    // ---------------- order candidates by t (ties by id) ----------------
    if (live) {
        for (int c = gl; c < ncand; c += G) {
            const R tc = S.cand[c][3];
            const int ic = S.cid[c];
            int rank = 0;
            for (int c2 = 0; c2 < ncand; ++c2) {
                const R t2 = S.cand[c2][3];
                rank += (t2 < tc) || (t2 == tc && S.cid[c2] < ic);
            }
            S.corder[rank] = (uint8_t)c;
        }
        // auxiliary cube p_i +- L (outside the ball, never a facet)
        const R L = R(1.05) * r;
        if (gl < 6) {
            const int ax = gl >> 1;
            const R sg = (gl & 1) ? R(1) : R(-1);
            S.pl[gl][0] = ax == 0 ? sg : R(0);
            S.pl[gl][1] = ax == 1 ? sg : R(0);
            S.pl[gl][2] = ax == 2 ? sg : R(0);
            S.pl[gl][3] = L;
            S.pid[gl] = -7 - gl;
        }
        if (gl < 8) {
            const int sx = (gl & 1) ? 1 : -1, sy = (gl & 2) ? 1 : -1, sz = (gl & 4) ? 1 : -1;
            const int a = sx < 0 ? 0 : 1, b = sy < 0 ? 2 : 3, c = sz < 0 ? 4 : 5;
            S.tri[gl] = (sx * sy * sz > 0) ? pack3(a, b, c) : pack3(a, c, b);
            S.vp[gl][0] = sx * L;
            S.vp[gl][1] = sy * L;
            S.vp[gl][2] = sz * L;
        }
    }
    int np = 6, ntri = 8, hw = 8, nface = 6;
    __syncthreads();

    // ---------------- clip by the candidates in ascending t ----------------
    const int maxc = gmax<64>(live ? ncand : 0);
    for (int it = 0; it < maxc; ++it) {
        const bool go = live && it < ncand;
        R nx = 0, ny = 0, nz = 0, t = 0;
        int cidx = 0;
        if (go) {
            cidx = min((int)S.corder[it], CMAX - 1);
            nx = S.cand[cidx][0];
            ny = S.cand[cidx][1];
            nz = S.cand[cidx][2];
            t = S.cand[cidx][3];
        }
        int nrem = 0;
        if (go) {
            for (int s = gl; s - gl < hw; s += G) {
                bool out = false;
                if (s < hw) {
                    const uint32_t u = S.tri[s];
                    if (u != TRI_INVALID) {
                        out = dot3(nx, ny, nz, S.vp[s][0], S.vp[s][1], S.vp[s][2]) > t;
                        if (out) S.tri[s] = u | TRI_REMOVED;
                    }
                }
                nrem += popc(gballot<G>(out));
            }
        }
        bool cut = go && nrem > 0;
        if (cut && nrem == ntri) {  // the half-space misses the polytope: empty cell
            flags |= CF_EMPTY;
            live = false;
            cut = false;
        }
        if (cut && np >= PMAX) {
            flags |= CF_PLANES;
            live = false;
            cut = false;
        }
        __syncthreads();
        if (cut) {
            for (int p = gl; p < np; p += G) {
                S.u.c.mout[p] = 0;
                S.u.c.min[p] = 0;
                S.u.c.nxt[p] = 0xFF;
                S.u.c.rslot[p] = 0;
                S.u.c.kslot[p] = 0;
            }
        }
        __syncthreads();
        if (cut) {
            for (int s = gl; s < hw; s += G) {
                const uint32_t u = S.tri[s];
                if (u != TRI_INVALID && (u & TRI_REMOVED)) {
                    const int a = u & 0xFF, b = (u >> 8) & 0xFF, c = (u >> 16) & 0xFF;
                    atomicOr(&S.u.c.mout[a], (M)1 << b);
                    atomicOr(&S.u.c.mout[b], (M)1 << c);
                    atomicOr(&S.u.c.mout[c], (M)1 << a);
                    atomicOr(&S.u.c.min[b], (M)1 << a);
                    atomicOr(&S.u.c.min[c], (M)1 << b);
                    atomicOr(&S.u.c.min[a], (M)1 << c);
                }
            }
        }
        __syncthreads();
        int nnew = 0, ninterior = 0;
        bool bad = false;
        if (cut) {
            for (int p = gl; p - gl < np; p += G) {
                bool bnd = false, intr = false;
                if (p < np) {
                    const M mo = S.u.c.mout[p], mi = S.u.c.min[p];
                    const M e = mo & ~mi;
                    if (e) {
                        bnd = true;
                        bad = bad || popc(e) != 1 || popc((M)(mi & ~mo)) != 1;
                        S.u.c.nxt[p] = (uint8_t)ctz_(e);
                    } else if (mo) {
                        intr = true;
                    }
                }
                const unsigned long long b = gballot<G>(bnd);
                if (bnd) S.u.c.newl[nnew + popc(b & below)] = (uint8_t)p;
                nnew += popc(b);
                ninterior += popc(gballot<G>(intr));
            }
            bad = gballot<G>(bad) != 0;
        }
        __syncthreads();
        if (cut) {
            for (int s = gl; s < hw; s += G) {
                const uint32_t u = S.tri[s];
                if (u == TRI_INVALID) continue;
                const int a = u & 0xFF, b = (u >> 8) & 0xFF, c = (u >> 16) & 0xFF;
                if (u & TRI_REMOVED) {
                    if (S.u.c.nxt[a] == b) S.u.c.rslot[a] = (uint8_t)s;
                    if (S.u.c.nxt[b] == c) S.u.c.rslot[b] = (uint8_t)s;
                    if (S.u.c.nxt[c] == a) S.u.c.rslot[c] = (uint8_t)s;
                } else {
                    if (S.u.c.nxt[b] == a) S.u.c.kslot[b] = (uint8_t)s;
                    if (S.u.c.nxt[c] == b) S.u.c.kslot[c] = (uint8_t)s;
                    if (S.u.c.nxt[a] == c) S.u.c.kslot[a] = (uint8_t)s;
                }
            }
        }
        __syncthreads();
        // new vertices: on edge x∩nxt[x], between its kept and its removed end.
        // All positions are read before any slot is reused (removed slots are free).
        if (cut) {
            for (int k = gl; k < nnew; k += G) {
                const int p = S.u.c.newl[k];
                const int ks = S.u.c.kslot[p], rs = S.u.c.rslot[p];
                const R ax = S.vp[ks][0], ay = S.vp[ks][1], az = S.vp[ks][2];
                const R bx = S.vp[rs][0], by = S.vp[rs][1], bz = S.vp[rs][2];
                const R sa = dot3(nx, ny, nz, ax, ay, az) - t;
                const R sb = dot3(nx, ny, nz, bx, by, bz) - t;
                const R lam = (sb > sa) ? sa / (sa - sb) : R(0.5);
                S.u.c.newpos[k][0] = ax + lam * (bx - ax);
                S.u.c.newpos[k][1] = ay + lam * (by - ay);
                S.u.c.newpos[k][2] = az + lam * (bz - az);
            }
        }
        __syncthreads();
        if (cut) {
            const int knew = np;
            if (gl == 0) {
                S.pl[knew][0] = nx;
                S.pl[knew][1] = ny;
                S.pl[knew][2] = nz;
                S.pl[knew][3] = t;
                S.pid[knew] = S.cid[cidx];
            }
            int fbase = 0, top = 0;
            for (int j = 0; j * G < VMAX; ++j) {
                const int s = j * G + gl;
                const uint32_t u = (s < hw) ? S.tri[s] : TRI_INVALID;
                const bool isfree = (u == TRI_INVALID) || (u & TRI_REMOVED);
                const unsigned long long b = gballot<G>(isfree);
                const int frank = fbase + popc(b & below);
                fbase += popc(b);
                if (isfree) {
                    if (frank < nnew) {
                        const int p = S.u.c.newl[frank];
                        const int q = S.u.c.nxt[p];
                        S.vp[s][0] = S.u.c.newpos[frank][0];
                        S.vp[s][1] = S.u.c.newpos[frank][1];
                        S.vp[s][2] = S.u.c.newpos[frank][2];
                        S.tri[s] = pack3(p, q, knew);
                        top = s + 1;
                    } else if (s < hw) {
                        S.tri[s] = TRI_INVALID;
                    }
                }
            }
            hw = max(hw, gmax<G>(top));
            if (fbase < nnew) {
                flags |= CF_VERTS;
                live = false;
            }
            ntri = ntri - nrem + nnew;
            nface = nface - ninterior + 1;
            np++;
            if (bad || ntri != 2 * nface - 4) {
                flags |= CF_TOPO;
                live = false;
            }
        }
        __syncthreads();
    }

    // ---------------- restriction to the ball and integration ----------------
    if (live) {
        for (int p = gl; p < np; p += G) S.u.g.fstart[p] = 0xFF;
    }
    __syncthreads();
    if (live) {
        for (int s = gl; s < hw; s += G) {
            const uint32_t u = S.tri[s];
            if (u == TRI_INVALID) continue;
            const int a = u & 0xFF, b = (u >> 8) & 0xFF, c = (u >> 16) & 0xFF;
            S.u.g.eslot[a][b] = (uint8_t)s;
            S.u.g.eslot[b][c] = (uint8_t)s;
            S.u.g.eslot[c][a] = (uint8_t)s;
            S.u.g.fstart[a] = (uint8_t)s;
            S.u.g.fstart[b] = (uint8_t)s;
            S.u.g.fstart[c] = (uint8_t)s;
        }
    }
    __syncthreads();
    double sum_tA = 0.0, sum_om = 0.0;
    bool walk_bad = false;
    if (live) {
        const R cone_den = R(1) / r;
        for (int p = gl; p < np; p += G) {
            R Af = 0, Of = 0;
            const int s0 = S.u.g.fstart[p];
            if (p >= 6 && s0 != 0xFF) {
                const R nx = S.pl[p][0], ny = S.pl[p][1], nz = S.pl[p][2], t = S.pl[p][3];
                const R h = fabs(t);
                const R rho2 = (r - t) * (r + t);
                const R cone = R(1) - h * cone_den;
                const R qx = t * nx, qy = t * ny, qz = t * nz;
                int s = s0, steps = 0;
                R ux = S.vp[s][0] - qx, uy = S.vp[s][1] - qy, uz = S.vp[s][2] - qz;
                do {
                    const uint32_t u = S.tri[s];
                    const int a = u & 0xFF, b = (u >> 8) & 0xFF, c = (u >> 16) & 0xFF;
                    const int third = (a == p) ? c : ((b == p) ? a : ((c == p) ? b : -1));
                    if (third < 0 || u == TRI_INVALID) {
                        walk_bad = true;
                        break;
                    }
                    const int sn = S.u.g.eslot[p][third];
                    if (sn >= hw || ++steps > VMAX) {
                        walk_bad = true;
                        break;
                    }
                    const R vx = S.vp[sn][0] - qx, vy = S.vp[sn][1] - qy, vz = S.vp[sn][2] - qz;
                    fan_piece<R>(ux, uy, uz, vx, vy, vz, nx, ny, nz, rho2, h, cone, Af, Of);
                    ux = vx;
                    uy = vy;
                    uz = vz;
                    s = sn;
                } while (s != s0);
                sum_tA += (double)t * (double)Af;
                sum_om += (t >= R(0)) ? (double)Of : -(double)Of;
            }
            S.u.g.farea[p] = Af;
        }
        if (gballot<G>(walk_bad)) {
            flags |= CF_WALK;
            live = false;
        }
    }
    sum_tA = gsum<G>(sum_tA);
    sum_om = gsum<G>(sum_om);
    __syncthreads();

    // ---------------- outputs ----------------
    if (!act) return;
    const EvalOut &o = A.out;
    int nf = 0;
    if (live) {
        for (int p = gl; p - gl < np; p += G) {
            bool isf = false;
            float a = 0.f;
            int id = -100;
            if (p < np && p >= 6) {
                a = (float)S.u.g.farea[p];
                id = S.pid[p];
                isf = id >= 0 && a > 0.f;
                if (id < 0 && o.wall) o.wall[cell * 6 + (-1 - id)] = a;
            }
            const unsigned long long b = gballot<G>(isf);
            if (isf) {
                const int slot = nf + popc(b & below);
                if (slot < FCAP) {
                    o.fcol[cell * FCAP + slot] = id;
                    o.farea[cell * FCAP + slot] = a;
                }
            }
            nf += popc(b);
        }
        if (nf > FCAP) {
            flags |= CF_FACETS;
            nf = FCAP;
        }
    }
    if (gl == 0) {
        double V = 0.0, K = 0.0;
        if (live) {
            const double rd = (double)r;
            K = rd * rd * (4.0 * PI_D * (inside ? 1.0 : 0.0) - sum_om);
            V = (sum_tA + rd * K) / 3.0;
        }
        // a cell much smaller than its ball is a difference of large pyramid terms:
        // float32 would lose the relative accuracy, so it is redone in float64
        if (fast && live && V < 0.05 * (4.0 / 3.0) * PI_D * (double)r * (double)r * (double)r) flags |= CF_PREC;
        o.V[cell] = V;
        o.K[cell] = K;
        o.fcnt[cell] = live ? nf : 0;
        o.flags[cell] = flags;
        if (fast && (flags & (CF_FAIL_MASK | CF_PREC))) {
            const int slot = atomicAdd(o.fb_count, 1);
            o.fb_list[slot] = (int32_t)cell;
        } else if (!fast && (flags & CF_FAIL_MASK)) {
            atomicAdd(o.fail_count, 1);
        }
    }
}

template <int G>
__global__ __launch_bounds__(64) void k_cells_fast(CellArgs A) {
    __shared__ CellSmem<float, FAST_CMAX, FAST_PMAX, FAST_VMAX> smem[64 / G];
    const int gi = (int)(threadIdx.x / G);
    const int64_t cell = (int64_t)blockIdx.x * (64 / G) + gi;
    cell_body<float, G, FAST_CMAX, FAST_PMAX, FAST_VMAX>(cell < A.n ? cell : -1, A, smem[gi], true);
}

__global__ __launch_bounds__(64) void k_cells_big(CellArgs A) {
    __shared__ CellSmem<double, BIG_CMAX, BIG_PMAX, BIG_VMAX> smem[1];
    const int count = *A.out.fb_count;
    for (int k = blockIdx.x; k < count; k += gridDim.x) {
        const int64_t cell = A.out.fb_list[k];
        cell_body<double, 64, BIG_CMAX, BIG_PMAX, BIG_VMAX>(cell, A, smem[0], false);
        __syncthreads();
    }
}

}  // namespace

void launch_cells(hipStream_t st, int64_t n, const float4 *pos_s, const int32_t *perm, const int32_t *cell_start,
                  GridDesc g, BoxF box, const double *rmax, EvalOut out, int tpc) {
    CellArgs a{n, pos_s, nullptr, perm, cell_start, g, box, rmax, out};
    if (tpc == 32) {
        hipLaunchKernelGGL(k_cells_fast<32>, dim3((unsigned)((n + 1) / 2)), dim3(64), 0, st, a);
    } else if (tpc == 64) {
        hipLaunchKernelGGL(k_cells_fast<64>, dim3((unsigned)n), dim3(64), 0, st, a);
    } else {
        hipLaunchKernelGGL(k_cells_fast<16>, dim3((unsigned)((n + 3) / 4)), dim3(64), 0, st, a);
    }
}

void launch_cells_fallback(hipStream_t st, int64_t n, const float4 *pos_s, const double *psi_s, const int32_t *perm,
                           const int32_t *cell_start, GridDesc g, BoxF box, const double *rmax, EvalOut out) {
    CellArgs a{n, pos_s, psi_s, perm, cell_start, g, box, rmax, out};
    hipLaunchKernelGGL(k_cells_big, dim3(512), dim3(64), 0, st, a);
}

}  // namespace lagot
