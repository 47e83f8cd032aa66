// cells.hip -- evaluation of every generalized Laguerre cell
//   C_i = box ∩ B(p_i, sqrt(psi_i)) ∩ {power_i <= power_j  for all j}      (eq. (1))
// fused in one kernel: candidate bisectors (cell_clip input), convex clipping
// (cell_clip, section 4 "Cell Update"), and the analytic restriction to the
// ball (ball_cell_integrate, section 3.2-3.3 and Algorithm 2).
//
// Mapping (MI355X, wave64): one 64-lane workgroup holds 64/G cells, G lanes per
// cell. The polytope is a set of vertex triangles (each vertex stores the three
// planes meeting there, counter-clockwise seen from outside, and its position
// relative to p_i); lane l of a group keeps vertex slots l, l+G, ... in
// registers. LDS holds only what lanes exchange: the candidate planes, the
// plane table, per-plane bitmasks and the two ends of every cut edge, and for
// the integration the vertex records and a directed-edge -> slot table.
// Ballots give ranks; three barriers per clipping plane.
//
// Clipping by a plane k: vertices beyond k are marked; for every plane x the
// removed triangles around it give an out-set and an in-set of neighbour planes
// (bitmasks); x lies on the cut boundary iff out \ in is a single plane y, and
// the new vertex on edge x∩y is interpolated between the kept and the removed
// end of that edge. The new triangles are (x, y, k). Euler's relation
// T = 2F - 4 checks the combinatorics after every cut; a violation, or any
// capacity overflow, flags the cell for the float64 large-capacity path.
//
// Crowded cells (section 4, "Finding Contributing Neighbors"): where a few balls are
// much larger than the rest, a cell's search block holds thousands of sites, most of
// whose bisectors never touch the cell. The fast pass defers such a cell; a seed pass
// clips it by its nearest sites only (a superset of the cell) and writes its box, every
// other cell writes the box of its exact cell, the boxes are registered in bucket grids,
// and the crowded pass (float64) clips each deferred cell by the sites whose boxes
// overlap its own, starting from its box. This candidate set is exact: a point of the
// result outside the true cell has a site of lower power whose own cell holds the point,
// so the two boxes overlap and that site was a candidate.
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

template <typename R> __device__ inline R rcp_(R v);
template <> __device__ inline float rcp_<float>(float v) { return __builtin_amdgcn_rcpf(v); }
template <> __device__ inline double rcp_<double>(double v) { return 1.0 / v; }

// One fan piece: triangle (q, q+u, q+v) ∩ disk(q, rho), signed by the orientation of
// (u, v) about n. h = |t|, cone = 1 - h/r. Returns its planar area A and the solid
// angle Om it subtends at p_i (apex at height h above q).
//   - no crossing of the circle: one circular sector of angle phi = angle(u, v):
//       area rho^2 phi / 2, solid angle phi (1 - h/r)
//   - crossing at a = u + lo w, b = u + hi w: sectors (u, a) and (b, v) plus the
//     triangle (q, a, b) inside the disk (Van Oosterom-Strackee with the apex at h).
//     The two sector angles are parts of one angle below pi, so they are summed as
//     the argument of the product of their complex numbers (one atan2).
// With MOM it also returns the piece's first moment about q (an in-plane vector)
// (Mx, My, Mz): a sector of radius rho from the unit direction e through the angle phi
// has the moment rho^3/3 (e sin phi + (n x e)(1 - cos phi)), with sin and cos from the
// normalised cross and dot products (no angle needed); a triangle (q, q+a, q+b) has its
// signed area times (a + b)/3.
// One fan piece's planar area A, solid angle Om and (with MOM) first moment (Mx, My, Mz),
// returned by value: the accumulators stay in registers whatever the optimiser does with
// the branches.
template <typename R> struct PieceSum {
    R A, Om, Mx, My, Mz;
};

template <typename R>
__device__ __attribute__((always_inline)) inline void sector_moment(R ex, R ey, R ez, R cphi, R sphi, R nx, R ny, R nz, R k,
                                                                    PieceSum<R> &p) {
    const R wx = ny * ez - nz * ey, wy = nz * ex - nx * ez, wz = nx * ey - ny * ex;
    const R oc = R(1) - cphi;
    p.Mx += k * (ex * sphi + wx * oc);
    p.My += k * (ey * sphi + wy * oc);
    p.Mz += k * (ez * sphi + wz * oc);
}

template <typename R, bool MOM = false>
__device__ __attribute__((always_inline)) inline PieceSum<R> fan_piece(R ux, R uy, R uz, R vx, R vy, R vz, R nx, R ny, R nz,
                                                                        R rho2, R h, R cone) {
    PieceSum<R> p{R(0), R(0), R(0), R(0), R(0)};
    const R wx = vx - ux, wy = vy - uy, wz = vz - uz;
    const R a = dot3(wx, wy, wz, wx, wy, wz);
    if (!(a > R(0))) return p;
    const R b = dot3(ux, uy, uz, wx, wy, wz);
    const R c = dot3(ux, uy, uz, ux, uy, uz) - rho2;
    const R disc = b * b - a * c;
    R lo = R(1), hi = R(0);
    if (disc > R(0)) {
        const R sq = sqrt(disc);
        const R ia = rcp_<R>(a);
        lo = fmax((-b - sq) * ia, R(0));
        hi = fmin((-b + sq) * ia, R(1));
    }
    const R half_rho2 = R(0.5) * rho2;
    if (!(lo < hi)) {
        const R cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
        const R sn = dot3(nx, ny, nz, cx, cy, cz), cs = dot3(ux, uy, uz, vx, vy, vz);
        const R phi = atan2_<R>(sn, cs);
        p.A += half_rho2 * phi;
        p.Om += cone * phi;
        if constexpr (MOM) {
            const R lu = sqrt(dot3(ux, uy, uz, ux, uy, uz)), luv = lu * sqrt(dot3(vx, vy, vz, vx, vy, vz));
            if (luv > R(0)) {
                const R il = rcp_<R>(lu), iuv = rcp_<R>(luv);
                sector_moment<R>(ux * il, uy * il, uz * il, cs * iuv, sn * iuv, nx, ny, nz,
                                 rho2 * sqrt(rho2) * R(1.0 / 3.0), p);
            }
        }
        return p;
    }
    const R ax = ux + lo * wx, ay = uy + lo * wy, az = uz + lo * wz;
    const R bx = ux + hi * wx, by = uy + hi * wy, bz = uz + hi * wz;
    // sector (u, a) and sector (b, v) as complex numbers (cos-part, sin-part)
    R c1 = dot3(ux, uy, uz, ax, ay, az);
    R s1 = nx * (uy * az - uz * ay) + ny * (uz * ax - ux * az) + nz * (ux * ay - uy * ax);
    R c2 = dot3(bx, by, bz, vx, vy, vz);
    R s2 = nx * (by * vz - bz * vy) + ny * (bz * vx - bx * vz) + nz * (bx * vy - by * vx);
    if (c1 == R(0) && s1 == R(0)) c1 = R(1);
    if (c2 == R(0) && s2 == R(0)) c2 = R(1);
    if constexpr (MOM) {
        // sector (u, a) from the direction of u and sector (b, v) from the direction of b;
        // a = u when u is inside the disk (and b = v when v is): angle 0, no moment
        const R k = rho2 * sqrt(rho2) * R(1.0 / 3.0);
        const R lu = sqrt(dot3(ux, uy, uz, ux, uy, uz)), la = sqrt(dot3(ax, ay, az, ax, ay, az));
        const R lb = sqrt(dot3(bx, by, bz, bx, by, bz)), lv = sqrt(dot3(vx, vy, vz, vx, vy, vz));
        if (lo > R(0) && lu * la > R(0)) {
            const R il = rcp_<R>(lu), d = rcp_<R>(lu * la);
            sector_moment<R>(ux * il, uy * il, uz * il, c1 * d, s1 * d, nx, ny, nz, k, p);
        }
        if (hi < R(1) && lb * lv > R(0)) {
            const R il = rcp_<R>(lb), d = rcp_<R>(lb * lv);
            sector_moment<R>(bx * il, by * il, bz * il, c2 * d, s2 * d, nx, ny, nz, k, p);
        }
    }
    const R phi = atan2_<R>(c1 * s2 + s1 * c2, c1 * c2 - s1 * s2);
    p.A += half_rho2 * phi;
    p.Om += cone * phi;
    // triangle (q, q+a, q+b) inside the disk: planar area and solid angle
    const R cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
    const R st = dot3(nx, ny, nz, cx, cy, cz);
    p.A += R(0.5) * st;
    if constexpr (MOM) {
        const R w = st * R(1.0 / 6.0);
        p.Mx += w * (ax + bx);
        p.My += w * (ay + by);
        p.Mz += w * (az + bz);
    }
    const R h2 = h * h;
    const R la = sqrt(dot3(ax, ay, az, ax, ay, az) + h2);
    const R lb = sqrt(dot3(bx, by, bz, bx, by, bz) + h2);
    p.Om += R(2) * atan2_<R>(st, la * lb + h * (la + lb) + h2 + dot3(ax, ay, az, bx, by, bz));
    return p;
}

// ---- section 3.3's own route to |K| (Algorithm 2: point_in, occluded patches) ----
// From a point c inside the (convex) restricted cell every ray leaves through one
// boundary point, on the sphere or on a restricted facet B_f, so the sphere is tiled by
// K and the projections of the B_f from c: |K| = 4 pi r^2 - sum_f |Proj(B_f)|. A
// projected facet is bounded by circle arcs: a straight boundary piece of B_f projects
// into the circle cut by the plane through c and the piece; a boundary arc of B_f (on
// the facet's circle) stays. Gauss-Bonnet gives |Proj(B_f)| = r^2 (2 pi - G_f) with
// G_f = sum k_g len + sum turning angles, k_g = e / (r rho) for a circle at signed
// distance e from the centre (positive on the smaller cap: the corrected form of the
// printed curvature), so k_g len = e theta / r for an arc of angle theta.
// Per fan piece (the facet edge P -> Q, counter-clockwise about n seen from outside),
// G_f is split into parts that need only the piece and the next vertex X on the facet:
//   - the facet circle's arcs: (t / r) times the piece's signed sector angle about q;
//     over the facet these sum to the angle of the circle inside the polygon (the same
//     winding argument as the signed fan), i.e. to the arcs of B_f's boundary;
//   - the projection of the piece's part inside the ball [A, B] (plane through c, A, B);
//   - the turning angles at A (from the circle arc, if A is where the edge enters the
//     ball) and at B (to the circle arc if the edge leaves the ball, else to the next
//     piece's projection at the vertex Q).
// A vertex is inside the ball by one test (|Q| < r) for both pieces that meet there.
template <typename R> __device__ inline void kr_unit(R &x, R &y, R &z) {
    const R l = sqrt(x * x + y * y + z * z);
    const R il = l > R(0) ? R(1) / l : R(0);
    x *= il;
    y *= il;
    z *= il;
}

// the ray c + s (a - c), s > 0, on the sphere |y| = r (c inside the ball)
template <typename R> __device__ inline void kr_project(R cx, R cy, R cz, R ax, R ay, R az, R r, R &ox, R &oy, R &oz) {
    const R ex = ax - cx, ey = ay - cy, ez = az - cz;
    const R qa = dot3(ex, ey, ez, ex, ey, ez), qb = dot3(cx, cy, cz, ex, ey, ez);
    const R qc = dot3(cx, cy, cz, cx, cy, cz) - r * r;
    const R s = (-qb + sqrt(fmax(qb * qb - qa * qc, R(0)))) / qa;
    ox = cx + s * ex;
    oy = cy + s * ey;
    oz = cz + s * ez;
}

// signed turning angle at the sphere point x from tangent T1 to tangent T2
template <typename R> __device__ inline R kr_turn(R t1x, R t1y, R t1z, R t2x, R t2y, R t2z, R x, R y, R z) {
    const R wx = t1y * t2z - t1z * t2y, wy = t1z * t2x - t1x * t2z, wz = t1x * t2y - t1y * t2x;
    return atan2_<R>(dot3(wx, wy, wz, x, y, z), dot3(t1x, t1y, t1z, t2x, t2y, t2z) * sqrt(dot3(x, y, z, x, y, z)));
}

// unit tangent at x of a circle traversed positively about the unit axis u
template <typename R> __device__ inline void kr_tangent(R ux, R uy, R uz, R x, R y, R z, R &tx, R &ty, R &tz) {
    tx = uy * z - uz * y;
    ty = uz * x - ux * z;
    tz = ux * y - uy * x;
    kr_unit(tx, ty, tz);
}

// The piece P -> Q against the ball: the part inside [lo, hi] of P + s (Q - P) (empty if
// lo >= hi), and the piece's signed sector angle phi about the circle centre q = t n
// (the parts of the piece outside the ball). A facet's restricted part is not empty iff
// one of its pieces has a part inside, or its circle lies inside the polygon (sum of phi
// 2 pi rather than 0): a combinatorial test, not the sign of a cancelling area sum.
template <typename R> struct KRArc {
    R lo, hi, phi;
    bool inP, inQ;
};

template <typename R>
__device__ KRArc<R> kr_arc(R px, R py, R pz, R qx, R qy, R qz, R nx, R ny, R nz, R t, R r) {
    KRArc<R> k;
    const R r2 = r * r;
    k.inP = dot3(px, py, pz, px, py, pz) < r2;
    k.inQ = dot3(qx, qy, qz, qx, qy, qz) < r2;
    const bool inP = k.inP, inQ = k.inQ;
    const R wx = qx - px, wy = qy - py, wz = qz - pz;
    const R a = dot3(wx, wy, wz, wx, wy, wz);
    k.lo = R(1);
    k.hi = R(0);
    k.phi = R(0);
    if (!(a > R(0))) return k;
    R lo = R(1), hi = R(0);
    {
        const R b = dot3(px, py, pz, wx, wy, wz), c0 = dot3(px, py, pz, px, py, pz) - r2;
        const R disc = b * b - a * c0;
        if (disc > R(0)) {
            const R sq = sqrt(disc);
            lo = inP ? R(0) : fmin(fmax((-b - sq) / a, R(0)), R(1));
            hi = inQ ? R(1) : fmin(fmax((-b + sq) / a, R(0)), R(1));
        }
        if (inP && inQ) {
            lo = R(0);
            hi = R(1);
        }
    }
    k.lo = lo;
    k.hi = hi;
    const bool seg = lo < hi;
    const R ox = t * nx, oy = t * ny, oz = t * nz;
    const R ux = px - ox, uy = py - oy, uz = pz - oz, vx = qx - ox, vy = qy - oy, vz = qz - oz;
    if (!seg) {
        k.phi = atan2_<R>(nx * (uy * vz - uz * vy) + ny * (uz * vx - ux * vz) + nz * (ux * vy - uy * vx),
                          dot3(ux, uy, uz, vx, vy, vz));
    } else {
        const R aqx = px + lo * wx - ox, aqy = py + lo * wy - oy, aqz = pz + lo * wz - oz;
        const R bqx = px + hi * wx - ox, bqy = py + hi * wy - oy, bqz = pz + hi * wz - oz;
        if (!inP)
            k.phi += atan2_<R>(nx * (uy * aqz - uz * aqy) + ny * (uz * aqx - ux * aqz) + nz * (ux * aqy - uy * aqx),
                               dot3(ux, uy, uz, aqx, aqy, aqz));
        if (!inQ)
            k.phi += atan2_<R>(nx * (bqy * vz - bqz * vy) + ny * (bqz * vx - bqx * vz) + nz * (bqx * vy - bqy * vx),
                               dot3(bqx, bqy, bqz, vx, vy, vz));
    }
    return k;
}

// G_f share of one fan piece P -> Q (next vertex X on the facet); positions relative to p_i
template <typename R>
__device__ R kr_piece(R px, R py, R pz, R qx, R qy, R qz, R xx, R xy, R xz, R nx, R ny, R nz, R t, R r, R cx, R cy,
                      R cz) {
    const KRArc<R> k = kr_arc<R>(px, py, pz, qx, qy, qz, nx, ny, nz, t, r);
    R g = t * k.phi / r;
    if (!(k.lo < k.hi)) return g;
    const bool inP = k.inP, inQ = k.inQ;
    const R wx = qx - px, wy = qy - py, wz = qz - pz;
    const R ax = px + k.lo * wx, ay = py + k.lo * wy, az = pz + k.lo * wz;
    const R bx = px + k.hi * wx, by = py + k.hi * wy, bz = pz + k.hi * wz;
    // projection of [A, B] from c: the circle of the plane through c, A, B (axis m)
    R pax, pay, paz, pbx, pby, pbz;
    kr_project<R>(cx, cy, cz, ax, ay, az, r, pax, pay, paz);
    kr_project<R>(cx, cy, cz, bx, by, bz, r, pbx, pby, pbz);
    const R eax = ax - cx, eay = ay - cy, eaz = az - cz, ebx = bx - cx, eby = by - cy, ebz = bz - cz;
    R mx = eay * ebz - eaz * eby, my = eaz * ebx - eax * ebz, mz = eax * eby - eay * ebx;
    kr_unit(mx, my, mz);
    const R e = dot3(cx, cy, cz, mx, my, mz);
    const R ocx = e * mx, ocy = e * my, ocz = e * mz;
    {
        const R sx = pax - ocx, sy = pay - ocy, sz = paz - ocz, fx = pbx - ocx, fy = pby - ocy, fz = pbz - ocz;
        R th = atan2_<R>(mx * (sy * fz - sz * fy) + my * (sz * fx - sx * fz) + mz * (sx * fy - sy * fx),
                         dot3(sx, sy, sz, fx, fy, fz));
        if (th < R(0)) th += R(2.0 * PI_D);
        g += e * th / r;
    }
    R tax, tay, taz, tbx, tby, tbz;
    kr_tangent<R>(mx, my, mz, pax, pay, paz, tax, tay, taz);
    kr_tangent<R>(mx, my, mz, pbx, pby, pbz, tbx, tby, tbz);
    if (!inP) {  // entry from the facet circle's arc
        R cxa, cya, cza;
        kr_tangent<R>(nx, ny, nz, ax, ay, az, cxa, cya, cza);
        g += kr_turn<R>(cxa, cya, cza, tax, tay, taz, ax, ay, az);
    }
    if (!inQ) {  // exit onto the facet circle's arc
        R cxb, cyb, czb;
        kr_tangent<R>(nx, ny, nz, bx, by, bz, cxb, cyb, czb);
        g += kr_turn<R>(tbx, tby, tbz, cxb, cyb, czb, bx, by, bz);
    } else {     // the vertex Q: on to the projection of the next piece Q -> X
        const R fx = qx - cx, fy = qy - cy, fz = qz - cz, hx = xx - cx, hy = xy - cy, hz = xz - cz;
        R m2x = fy * hz - fz * hy, m2y = fz * hx - fx * hz, m2z = fx * hy - fy * hx;
        kr_unit(m2x, m2y, m2z);
        R t2x, t2y, t2z;
        kr_tangent<R>(m2x, m2y, m2z, pbx, pby, pbz, t2x, t2y, t2z);
        g += kr_turn<R>(tbx, tby, tbz, t2x, t2y, t2z, pbx, pby, pbz);
    }
    return g;
}

// per-piece first moments and areas, per-face chord midpoints (the route's scratch)
template <typename R, int PMAX, int VMAX> struct KRSmem {
    R pm[3 * VMAX][6];  // piece: first moment about q (3), planar area, sector angle, 1 if a part is inside
    R fm[PMAX][4];      // face: chord midpoint (3), 1 if the restricted facet is not empty
};

// Vertex record of the integration phase: position relative to p_i and its three planes.
template <typename R> struct alignas(16) VRec {
    R x, y, z;
    uint32_t t;
};

template <typename R, int CMAX, int PMAX, int VMAX> struct CellSmem {
    using M = typename MaskType<PMAX>::T;
    R pl[PMAX][4];   // planes of the polytope (0..5: auxiliary cube): unit normal, t
    int32_t pid[PMAX];
    union {
        struct {
            R csort[CMAX][4];   // candidate planes in ascending t
            int32_t csid[CMAX]; // neighbour (grid-order index) or -1-w for wall w
            union {
                struct {        // discovery order
                    R cand[CMAX][4];
                    int32_t cid[CMAX];
                } d;
                struct {        // clipping
                    M mout[PMAX];       // per plane: heads of the removed triangles' edges leaving it
                    M min[PMAX];        //            tails of the removed triangles' edges entering it
                    uint8_t nxt[PMAX];  // boundary plane -> next plane along the cut (0xFF otherwise)
                    uint8_t newl[PMAX]; // boundary planes by rank
                    R kpos[PMAX][3];    // kept end of the cut edge x∩nxt[x]
                    R rpos[PMAX][3];    // removed end
                } k;
            } x;
        } c;
        struct {            // integration
            // rec and eslot are contiguous: once the successors are known, eslot holds the
            // list of fan pieces, and then both hold the pieces' (area, solid angle)
            VRec<R> rec[VMAX];
            uint8_t eslot[PMAX][PMAX];   // directed edge a->b -> slot of the vertex holding it
            uint32_t succ[VMAX];         // successor slot on each of the vertex's three faces
            uint32_t trs[VMAX];          // the vertex's three planes (packed)
            uint32_t fstart[PMAX];
            R farea[PMAX];
        } g;
    } u;
};

struct CellArgs {
    int64_t n;
    const float4 *pos_s;      // x, y, z, float32 psi (grid order)
    const double *psi_s;      // float64 psi being evaluated (grid order)
    const int32_t *perm;      // grid order -> caller index (tie rule for coincident sites)
    const int32_t *cell_start;
    Batch bt;                 // instance of each row, its grid, box and r_max
    int want;                 // evaluate the instances in this phase (< 0: all)
    EvalOut out;
    QBoxes qb;                // cell boxes and their bucket grid (crowded cells)
    int crowd;                // 1: the crowded pass runs (boxes written); 0: deferred cells go to
                              // the float64 pass
};

template <typename R, int G, int CMAX, int PMAX, int VMAX, int MODE, bool MOM, bool KR = false>
__device__ void cell_body(int64_t cell, const CellArgs &A, CellSmem<R, CMAX, PMAX, VMAX> &S,
                          KRSmem<R, PMAX, VMAX> *KS = nullptr) {
    // KR: |K| by section 3.3's own route (kr_piece) in place of the signed solid angles
    // MODE 0: the fast pass (a crowded cell -- more than CMAX candidates, or a search
    // block of more than FAST_SCAN_MAX sites -- is deferred to the overflow list; every
    // other cell writes its box); 3: the seed pass of a deferred cell (clipped by its
    // nearest sites only: a superset of the cell, whose box it writes); 1: the crowded
    // pass (candidates are the sites whose boxes overlap the cell's, threshold ladder and
    // clip rounds when they exceed CMAX); 2: the large-capacity pass for the cells that
    // passes 0 and 1 cannot finish (capacity, or float32 accuracy).
    constexpr bool fast = MODE != 2;
    constexpr bool rounds = MODE == 1 || MODE == 2;
    constexpr bool seed = MODE == 3;
    bool deferred = false;
    using M = typename MaskType<PMAX>::T;
    constexpr int NS = VMAX / G;  // vertex slots per lane (registers); slot id = k * G + lane
    static_assert(NS * G == VMAX, "VMAX must be a multiple of G");
    static_assert(VMAX <= 255 && PMAX <= 64 && CMAX <= 256, "slot and plane indices are bytes");
    const int gl = (int)(threadIdx.x & (G - 1));
    const unsigned long long below = lanes_below<G>();
    const bool act = cell >= 0;
    uint32_t flags = 0;
    auto &D = S.u.c.x.d;
    auto &KT = S.u.c.x.k;
    auto &GT = S.u.g;

    R px = 0, py = 0, pz = 0, psi_i = 0;
    double psi_i64 = 0.0;
    const int inst = act ? A.bt.inst[cell] : 0;
    if (act) {
        const float4 p4 = A.pos_s[cell];
        px = p4.x;
        py = p4.y;
        pz = p4.z;
        psi_i64 = A.psi_s[cell];
        psi_i = (R)psi_i64;
    }
    bool live = act && (psi_i > R(0));
    if (act && !live) flags |= CF_EMPTY;
    const R r = live ? sqrt(psi_i) : R(0);

    // ---------------- candidate bisectors: sites within r + r_max ----------------
    // Normally every candidate (|t| < r) is kept. When there are more than CMAX, a
    // counting pass picks tau = r 2^(-k/2), the largest with at most CMAX candidates
    // below it, and only those are kept. After clipping, a restricted cell that stays
    // within distance tau of p_i cannot be cut by the others (exact); otherwise the
    // others are tested against the polytope and the ones that cut it are clipped too.
    int ncand = 0;
    bool inside = true;
    bool empty = false;
    R tau = r;
    bool overflow = false;
    GridDesc gd{};
    int lo3[3] = {0, 0, 0}, hi3[3] = {-1, -1, -1};
    int nyc = 1, ncol = 0;
    const int gbase = (int)(threadIdx.x & (64 - G));
    // the crowded pass starts from the cell's box (a superset of the cell written by the
    // seed pass; an empty box is an empty cell)
    float qlo[3] = {0.f, 0.f, 0.f}, qhi[3] = {0.f, 0.f, 0.f};
    if constexpr (MODE == 1) {
        if (live) {
            const float4 a = A.qb.box[2 * cell], b = A.qb.box[2 * cell + 1];
            qlo[0] = a.x;
            qlo[1] = a.y;
            qlo[2] = a.z;
            qhi[0] = b.x;
            qhi[1] = b.y;
            qhi[2] = b.z;
            if (!(a.x <= b.x && a.y <= b.y && a.z <= b.z)) empty = true;
        }
    }
    if (live && !empty) {
        const float pp[3] = {(float)px, (float)py, (float)pz};
        if constexpr (MODE == 1) {
            // the buckets are visited level by level (scan sets the block of each level)
            gd = A.qb.qgrid[inst * QLEV];
        } else if constexpr (seed) {
            // the sites within 2.5 spacings
            gd = A.bt.grid[inst];
            const float reach = 2.5f * gd.hsp;
            for (int a = 0; a < 3; ++a) {
                lo3[a] = max((int)floorf((pp[a] - reach - gd.lo[a]) * gd.inv_s), 0);
                hi3[a] = min((int)floorf((pp[a] + reach - gd.lo[a]) * gd.inv_s), gd.dim[a] - 1);
            }
        } else {
            // every site whose ball can meet this one: within r + r_max, or r + max(r, local
            // bound of the larger balls) when the local reach is known
            gd = A.bt.grid[inst];
            float rj = (float)A.bt.rmax[inst];
            if (A.bt.ir) {
                const GridDesc cg = A.bt.cgrid[inst];
                int k3[3];
                for (int a = 0; a < 3; ++a)
                    k3[a] = min(max((int)floorf((pp[a] - cg.lo[a]) * cg.inv_s), 0), cg.dim[a] - 1);
                rj = fmaxf((float)r, A.bt.ir[cg.base + (k3[0] * cg.dim[1] + k3[1]) * cg.dim[2] + k3[2]]);
            }
            const float reach = ((float)r + rj) * 1.0001f;
            for (int a = 0; a < 3; ++a) {
                lo3[a] = max((int)floorf((pp[a] - reach - gd.lo[a]) * gd.inv_s), 0);
                hi3[a] = min((int)floorf((pp[a] + reach - gd.lo[a]) * gd.inv_s), gd.dim[a] - 1);
            }
        }
        if constexpr (MODE != 1) {
            nyc = hi3[1] - lo3[1] + 1;
            ncol = (hi3[0] - lo3[0] + 1) * nyc;
        }
    }
    // bucket block of the cell's box at box-grid level lev (crowded pass)
    auto bucket_block = [&](int lev) {
        gd = A.qb.qgrid[inst * QLEV + lev];
        for (int a = 0; a < 3; ++a) {
            lo3[a] = min(max((int)floorf((qlo[a] - gd.lo[a]) * gd.inv_s), 0), gd.dim[a] - 1);
            hi3[a] = min(max((int)floorf((qhi[a] - gd.lo[a]) * gd.inv_s), 0), gd.dim[a] - 1);
        }
        nyc = hi3[1] - lo3[1] + 1;
        ncol = (hi3[0] - lo3[0] + 1) * nyc;
    };
    // The bisector of (i, j) as a candidate plane: keep (|t| < r), kill (the site empties
    // the cell), neg (p_i is behind the bisector), the unit normal and t, and d^2.
    auto site = [&](bool valid, int j, auto &&f) {
        bool keep = false, kill = false, neg = false;
        R nx = 0, ny = 0, nz = 0, t = 0, d2o = 0;
        if (valid) {
            const float4 q4 = A.pos_s[j];
            // the weight difference is formed from the float64 weights: for close
            // sites t ~ (psi_i - psi_j) / 2d amplifies any rounding of the weights
            const double psi_j64 = A.psi_s[j];
            const R dpsi = (R)(psi_i64 - psi_j64);
            const R dx = (R)q4.x - px, dy = (R)q4.y - py, dz = (R)q4.z - pz;
            const R d2 = dot3(dx, dy, dz, dx, dy, dz);
            d2o = d2;
            if (d2 > R(0)) {
                const R id = rsqrt_<R>(d2);
                t = (d2 + dpsi) * (R(0.5) * id);
                if constexpr (sizeof(R) == 4) {
                    // d^2 and the weight difference nearly cancel (large weights):
                    // the float32 offset would carry their rounding, so it is
                    // formed in float64 (the float32 differences are exact there)
                    if (fabs(dpsi) > d2 && t > -r && t < r) {
                        const double ex = (double)q4.x - (double)px, ey = (double)q4.y - (double)py,
                                     ez = (double)q4.z - (double)pz;
                        const double e2 = ex * ex + ey * ey + ez * ez;
                        t = (R)((e2 + (psi_i64 - psi_j64)) / (2.0 * sqrt(e2)));
                    }
                }
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
                kill = psi_j64 > psi_i64 || (psi_j64 == psi_i64 && A.perm[j] < A.perm[cell]);
            }
        }
        f(keep, kill, neg, nx, ny, nz, t, j, d2o);
    };
    // Does the box of cell j overlap this cell's box? With `dedup`, a pair is reported
    // only in the bucket that holds the low corner of the two boxes' intersection (the
    // entry e of column (ix, iy), start index col), so a site registered in several
    // of the buckets visited is a candidate once.
    auto box_hit = [&](int j, bool dedup, int ix, int iy, int col, int e) -> bool {
        const float4 a = A.qb.box[2 * (int64_t)j], b = A.qb.box[2 * (int64_t)j + 1];
        if (!(a.x <= qhi[0] && qlo[0] <= b.x && a.y <= qhi[1] && qlo[1] <= b.y && a.z <= qhi[2] && qlo[2] <= b.z))
            return false;
        if (!dedup) return true;
        const float m[3] = {fmaxf(a.x, qlo[0]), fmaxf(a.y, qlo[1]), fmaxf(a.z, qlo[2])};
        int mb[3];
        for (int q = 0; q < 3; ++q)
            mb[q] = min(max((int)floorf((m[q] - gd.lo[q]) * gd.inv_s), 0), gd.dim[q] - 1);
        if (mb[0] != ix || mb[1] != iy) return false;
        return A.qb.start[col + mb[2]] <= e && e < A.qb.start[col + mb[2] + 1];
    };
    // Visit every candidate site, G at a time, then the walls. The sites (the entries of
    // the buckets, in the crowded pass) of up to G grid columns are numbered
    // consecutively (prefix sum over the lanes); each lane finds its column by a binary
    // search over shuffled sums.
    const int32_t *colstart = (MODE == 1) ? A.qb.start : A.cell_start;
    auto scan = [&](auto &&f) {
      const bool any = ncol > 0 || (MODE == 1 && live && !empty);
      for (int lev = 0; lev < (MODE == 1 ? QLEV : 1) && any; ++lev) {
        if constexpr (MODE == 1) bucket_block(lev);
        for (int c0 = 0; c0 < ncol; c0 += G) {
            int cbeg = 0, cnt = 0;
            if (c0 + gl < ncol) {
                const int ix = lo3[0] + (c0 + gl) / nyc, iy = lo3[1] + (c0 + gl) % nyc;
                const int col = gd.base + (ix * gd.dim[1] + iy) * gd.dim[2];
                cbeg = colstart[col + lo3[2]];
                cnt = colstart[col + hi3[2] + 1] - cbeg;
            }
            int incl = cnt;
#pragma unroll
            for (int o = 1; o < G; o <<= 1) {
                const int v = __shfl_up(incl, o, G);
                if (gl >= o) incl += v;
            }
            const int excl = incl - cnt;
            const int total = __shfl(incl, gbase + G - 1, 64);
            for (int b0 = 0; b0 < total; b0 += G) {
                const int idx = b0 + gl;
                int cidx = 0;  // number of columns whose sites all come before idx
#pragma unroll
                for (int step = G / 2; step >= 1; step >>= 1) {
                    const int v = __shfl(incl, gbase + cidx + step - 1, 64);
                    if (v <= idx) cidx += step;
                }
                const int e = __shfl(cbeg, gbase + cidx, 64) + (idx - __shfl(excl, gbase + cidx, 64));
                bool valid = idx < total;
                int j = e;
                if constexpr (MODE == 1) {
                    j = valid ? A.qb.ent[e] : -1;
                    const int ix = lo3[0] + (c0 + cidx) / nyc, iy = lo3[1] + (c0 + cidx) % nyc;
                    valid = valid && j != cell &&
                            box_hit(j, true, ix, iy, gd.base + (ix * gd.dim[1] + iy) * gd.dim[2], e);
                }
                site(valid && j != cell, j, f);
            }
        }
      }
        if constexpr (MODE == 1) {
            // cells whose boxes are too large for the buckets: tested one by one
            const int nl = *A.qb.nlarge;
            for (int k0 = 0; k0 < nl; k0 += G) {
                const int k = k0 + gl;
                int j = -1;
                bool valid = false;
                if (k < nl) {
                    j = A.qb.large[k];
                    valid = j != cell && A.bt.inst[j] == inst && box_hit(j, false, 0, 0, 0, 0);
                }
                site(valid, j, f);
            }
        }
        if (A.bt.ndom > 0) {
            // walls of a convex polyhedral domain n.x <= c: t = c - n.p_i, G planes at a time
            for (int w0 = 0; w0 < A.bt.ndom; w0 += G) {
                const int w = w0 + gl;
                bool keep = false;
                R nx = 0, ny = 0, nz = 0, t = 0;
                if (live && w < A.bt.ndom) {
                    const float4 q = A.bt.dom[w];
                    nx = (R)q.x;
                    ny = (R)q.y;
                    nz = (R)q.z;
                    t = (R)q.w - (nx * px + ny * py + nz * pz);
                    keep = t < r;
                }
                // the site may lie outside the domain's convex piece: behind the plane (t < 0),
                // and beyond the ball's reach (t <= -r: the cell has no part in the piece)
                f(keep, live && w < A.bt.ndom && t <= -r, keep && t < R(0), nx, ny, nz, t, -1 - w, R(0));
            }
            return;
        }
        // box walls -x,+x,-y,+y,-z,+z: t = distance from p_i to the wall; lane gl < 6 reads
        // its own bound (lo[0..2], hi[0..2]) straight from the box array
        bool keep = false;
        R nx = 0, ny = 0, nz = 0, t = 0;
        if (live && gl < 6) {
            const float *bnd = &A.bt.box[inst].lo[0];
            const int ax = gl >> 1;
            // select values, not the captured references (a select of references becomes
            // an indexed load from the closure, which then stays in scratch memory)
            const R cx = px, cy = py, cz = pz;
            const R pc = ax == 0 ? cx : (ax == 1 ? cy : cz);
            const R w = (R)bnd[(gl & 1) * 3 + ax];
            t = (gl & 1) ? w - pc : pc - w;
            keep = t < r;
            const R sg = (gl & 1) ? R(1) : R(-1);
            nx = ax == 0 ? sg : R(0);
            ny = ax == 1 ? sg : R(0);
            nz = ax == 2 ? sg : R(0);
        }
        f(keep, false, false, nx, ny, nz, t, -1 - gl, R(0));
    };
    // keep the candidates with t < thr. nnear counts the kept planes within 0.1 r of p_i:
    // where two such planes meet, the cell's shape near p_i is set by offsets far below r,
    // which float32 coordinates (relative to p_i, absolute error ~6e-8 r) resolve only to
    // ~6e-8 r / max(|t1|, |t2|); such cells are finished in float64.
    int nnear = 0;
    // the seed pass keeps the sites within dsel of p_i only (the walls always)
    R dsel2 = R(0);
    auto collect = [&](R thr) {
        ncand = 0;
        nnear = 0;
        scan([&](bool keep, bool kill, bool neg, R nx, R ny, R nz, R t, int id, R d2) {
            bool k2 = keep && t < thr;
            if constexpr (seed) k2 = k2 && (id < 0 || d2 < dsel2);
            if constexpr (sizeof(R) == 4) nnear += popc(gballot<G>(k2 && fabs(t) < R(0.1) * r));
            const unsigned long long b = gballot<G>(k2);
            if (k2) {
                const int c = ncand + popc(b & below);
                if (c < CMAX) {
                    D.cand[c][0] = nx;
                    D.cand[c][1] = ny;
                    D.cand[c][2] = nz;
                    D.cand[c][3] = t;
                    D.cid[c] = id;
                }
            }
            ncand += popc(b);
            if (gballot<G>(kill)) empty = true;
            if (gballot<G>(neg)) inside = false;
        });
    };
    // a convex piece of the domain that the ball cannot reach (t <= -r for one of its
    // planes): the cell has no part in it, and no candidate needs to be scanned
    if (A.bt.ndom > 0 && live && !empty) {
        bool out = false;
        for (int w = gl; w < A.bt.ndom; w += G) {
            const float4 q = A.bt.dom[w];
            const R nx = (R)q.x, ny = (R)q.y, nz = (R)q.z;
            out = out || (R)q.w - (nx * px + ny * py + nz * pz) <= -r;
        }
        if (gballot<G>(out)) empty = true;
    }
    if constexpr (MODE == 0) {
        // a search block holding more than FAST_SCAN_MAX sites: crowded, deferred
        if (live && !empty) {
            int tot = 0;
            for (int c0 = 0; c0 < ncol; c0 += G) {
                int cnt = 0;
                if (c0 + gl < ncol) {
                    const int ix = lo3[0] + (c0 + gl) / nyc, iy = lo3[1] + (c0 + gl) % nyc;
                    const int col = gd.base + (ix * gd.dim[1] + iy) * gd.dim[2];
                    cnt = A.cell_start[col + hi3[2] + 1] - A.cell_start[col + lo3[2]];
                }
                tot += gsum<G>(cnt);
            }
            if (tot > FAST_SCAN_MAX) {
                deferred = true;
                live = false;
            }
        }
    }
    if constexpr (seed) {
        // the nearest sites: the largest radius 2.5 h 2^(-k/3) (h = site spacing; the sphere
        // lies in the block) holding at most CMAX candidates. Any subset of the
        // bisectors gives a superset of the cell, so if even the smallest radius holds
        // more, the first CMAX found are kept.
        if (live && !empty) {
            constexpr int ND = 12;
            int cnt[ND];
            R d2k[ND];
            R f = R(2.5) * (R)gd.hsp;
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                d2k[k] = f * f;
                cnt[k] = 0;
                f *= R(0.79370052598409974);
            }
            scan([&](bool keep, bool, bool, R, R, R, R, int id, R d2) {
#pragma unroll
                for (int k = 0; k < ND; ++k) cnt[k] += (keep && id >= 0 && d2 < d2k[k]) ? 1 : 0;
            });
            int kk = ND - 1;
#pragma unroll
            for (int k = ND - 1; k >= 0; --k)
                if (gsum<G>(cnt[k]) <= CMAX - 6) kk = k;
#pragma unroll
            for (int k = 0; k < ND; ++k)
                if (k == kk) dsel2 = d2k[k];
        }
    }
    if (live && !empty) collect(r);
    if constexpr (seed) ncand = min(ncand, CMAX);
    if (!rounds && live && !empty && ncand > CMAX) {
        deferred = true;
        live = false;
    }
    if (MODE == 1 && live && !empty && ncand > CMAX) {
        // Crowded pass: the polytope starts from the cell's box, which already holds the
        // cell tightly, so the first CMAX candidates found are clipped and the clip rounds
        // then take every candidate that still cuts the polytope (tau = -r: no threshold).
        // (A threshold on t would assume the site lies near its cell; a crowded site often
        // lies far outside it, behind many of its bisectors.)
        tau = -r;
        overflow = true;
        ncand = CMAX;
    }
    if (MODE == 2 && live && !empty && ncand > CMAX) {
        constexpr int NT = 18;  // tau = r 2^(-k/3), k = 1..18 (down to r / 64)
        R thr[NT];
        int cnt[NT];
        R f = R(0.79370052598409974);
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            thr[k] = r * f;
            cnt[k] = 0;
            f *= R(0.79370052598409974);
        }
        scan([&](bool keep, bool, bool, R, R, R, R t, int, R) {
#pragma unroll
            for (int k = 0; k < NT; ++k) cnt[k] += (keep && t < thr[k]) ? 1 : 0;
        });
        int kk = -1;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            const int tot = gsum<G>(cnt[k]);
            if (kk < 0 && tot <= CMAX) kk = k;
        }
        if (kk >= 0) {
#pragma unroll
            for (int k = 0; k < NT; ++k)
                if (k == kk) tau = thr[k];
            overflow = true;
            collect(tau);
        }
    }
    if (empty) {
        flags |= CF_EMPTY;
        live = false;
    } else if (live && ncand > CMAX) {
        flags |= CF_CAND;
        live = false;
    }
    __syncthreads();

    // ---------------- candidates in ascending t (ties by id); masks cleared ----------------
    auto rank_round = [&](int count) {
        if (live) {
            for (int c = gl; c < count; c += G) {
                const R tc = D.cand[c][3];
                const int ic = D.cid[c];
                int rank = 0;
                for (int c2 = 0; c2 < count; ++c2) {
                    const R t2 = D.cand[c2][3];
                    rank += (t2 < tc) || (t2 == tc && D.cid[c2] < ic);
                }
                rank = min(rank, CMAX - 1);
                S.u.c.csort[rank][0] = D.cand[c][0];
                S.u.c.csort[rank][1] = D.cand[c][1];
                S.u.c.csort[rank][2] = D.cand[c][2];
                S.u.c.csort[rank][3] = tc;
                S.u.c.csid[rank] = ic;
            }
        }
        __syncthreads();  // the discovery staging is dead from here on (the clip tables overlap it)
        if (live) {
            for (int p = gl; p < PMAX; p += G) {
                KT.mout[p] = 0;
                KT.min[p] = 0;
            }
        }
    };
    // auxiliary box (never a facet); planes 0..5 = -x,+x,-y,+y,-z,+z. Normally the cube
    // p_i +- L, outside the ball. The crowded pass starts from the cell's box instead: it
    // holds the cell with a margin, so its faces never touch the restricted cell, and the
    // clipped polytope stays inside the box, where every bisector that can cut the cell
    // is among the box-overlap candidates.
    const R L = R(1.05) * r;
    R ax0 = -L, ax1 = L, ay0 = -L, ay1 = L, az0 = -L, az1 = L;
    if constexpr (MODE == 1) {
        ax0 = fmax(-L, (R)qlo[0] - px);
        ax1 = fmin(L, (R)qhi[0] - px);
        ay0 = fmax(-L, (R)qlo[1] - py);
        ay1 = fmin(L, (R)qhi[1] - py);
        az0 = fmax(-L, (R)qlo[2] - pz);
        az1 = fmin(L, (R)qhi[2] - pz);
    }
    if (live && gl < 6) {
        const int ax = gl >> 1;
        const R sg = (gl & 1) ? R(1) : R(-1);
        const R lo = ax == 0 ? ax0 : (ax == 1 ? ay0 : az0), hi = ax == 0 ? ax1 : (ax == 1 ? ay1 : az1);
        S.pl[gl][0] = ax == 0 ? sg : R(0);
        S.pl[gl][1] = ax == 1 ? sg : R(0);
        S.pl[gl][2] = ax == 2 ? sg : R(0);
        S.pl[gl][3] = (gl & 1) ? hi : -lo;
        S.pid[gl] = AUX_PLANE_ID - gl;
    }
    // vertex slots in registers; the box's corners go to slots 0..7
    uint32_t tri[NS];
    R vx[NS], vy[NS], vz[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        tri[k] = TRI_INVALID;
        vx[k] = vy[k] = vz[k] = R(0);
        const int s = k * G + gl;
        if (live && s < 8) {
            const int sx = (s & 1) ? 1 : -1, sy = (s & 2) ? 1 : -1, sz = (s & 4) ? 1 : -1;
            const int a = sx < 0 ? 0 : 1, b = sy < 0 ? 2 : 3, c = sz < 0 ? 4 : 5;
            tri[k] = (sx * sy * sz > 0) ? pack3(a, b, c) : pack3(a, c, b);
            vx[k] = sx < 0 ? ax0 : ax1;
            vy[k] = sy < 0 ? ay0 : ay1;
            vz[k] = sz < 0 ? az0 : az1;
        }
    }
    int np = 6, ntri = 8, nface = 6;
    __syncthreads();
    // Drops the planes (index >= 6) that no vertex uses any more: a plane that cut
    // the polytope can lose its whole face to later planes, and long clip sequences
    // would otherwise run out of plane slots. Between clip steps the cut tables are
    // free: nxt flags the planes in use, newl maps old to new index, kpos/rpos hold
    // the kept planes and min their ids (min is cleared again for the next step).
    // Called by every lane of the workgroup (it holds barriers).
    auto compact = [&]() {
        uint8_t *used = KT.nxt;
        uint8_t *map = KT.newl;
        R *tpl = &KT.kpos[0][0];
        int32_t *tid = reinterpret_cast<int32_t *>(&KT.min[0]);
        static_assert(sizeof(KT.kpos) + sizeof(KT.rpos) >= sizeof(R) * 4 * PMAX, "plane staging");
        static_assert(sizeof(KT.min) >= sizeof(int32_t) * PMAX, "id staging");
        if (live)
            for (int p = gl; p < np; p += G) used[p] = p < 6 ? 1 : 0;
        __syncthreads();
        if (live) {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const uint32_t u = tri[k];
                if (u == TRI_INVALID) continue;
                used[u & 0xFF] = 1;
                used[(u >> 8) & 0xFF] = 1;
                used[(u >> 16) & 0xFF] = 1;
            }
        }
        __syncthreads();
        int nk = 0;
        if (live) {
            for (int p = gl; p - gl < np; p += G) {
                const bool keep = p < np && used[p];
                const unsigned long long b = gballot<G>(keep);
                const int to = nk + popc(b & below);
                nk += popc(b);
                if (p < np) map[p] = keep ? (uint8_t)to : (uint8_t)0xFF;
                if (keep) {
                    tpl[4 * to + 0] = S.pl[p][0];
                    tpl[4 * to + 1] = S.pl[p][1];
                    tpl[4 * to + 2] = S.pl[p][2];
                    tpl[4 * to + 3] = S.pl[p][3];
                    tid[to] = S.pid[p];
                }
            }
        }
        __syncthreads();
        if (live) {
            for (int p = gl; p < nk; p += G) {
                S.pl[p][0] = tpl[4 * p + 0];
                S.pl[p][1] = tpl[4 * p + 1];
                S.pl[p][2] = tpl[4 * p + 2];
                S.pl[p][3] = tpl[4 * p + 3];
                S.pid[p] = tid[p];
            }
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const uint32_t u = tri[k];
                if (u == TRI_INVALID) continue;
                tri[k] = pack3(map[u & 0xFF], map[(u >> 8) & 0xFF], map[(u >> 16) & 0xFF]);
            }
        }
        __syncthreads();
        if (live) {
            for (int p = gl; p < PMAX; p += G) KT.min[p] = 0;
            np = nk;
        }
        __syncthreads();
    };
    // clip by the planes csort[0..count) in ascending t (every lane of the workgroup
    // runs the same number of iterations: the loop holds barriers)
    auto clip_round = [&](int count) {
        const int maxc = gmax<64>(live ? count : 0);
        for (int it = 0; it < maxc; ++it) {
            if constexpr (rounds) {  // long clip sequences: free the slots of dead planes
                if (__any(live && it < count && np >= PMAX - 1)) compact();
            }
            const bool go = live && it < count;
            R nx = 0, ny = 0, nz = 0, t = 0;
            if (go) {
                nx = S.u.c.csort[it][0];
                ny = S.u.c.csort[it][1];
                nz = S.u.c.csort[it][2];
                t = S.u.c.csort[it][3];
            }
            // vertices beyond the plane
            bool rem[NS];
            int nrem = 0;
    #pragma unroll
            for (int k = 0; k < NS; ++k) {
                rem[k] = go && tri[k] != TRI_INVALID && (nx * vx[k] + ny * vy[k] + nz * vz[k] > t);
                nrem += popc(gballot<G>(rem[k]));
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
            // edges of the removed triangles, per plane
            if (cut) {
    #pragma unroll
                for (int k = 0; k < NS; ++k) {
                    if (rem[k]) {
                        const uint32_t u = tri[k];
                        const int a = u & 0xFF, b = (u >> 8) & 0xFF, c = (u >> 16) & 0xFF;
                        atomicOr(&KT.mout[a], (M)1 << b);
                        atomicOr(&KT.mout[b], (M)1 << c);
                        atomicOr(&KT.mout[c], (M)1 << a);
                        atomicOr(&KT.min[b], (M)1 << a);
                        atomicOr(&KT.min[c], (M)1 << b);
                        atomicOr(&KT.min[a], (M)1 << c);
                    }
                }
            }
            __syncthreads();
            // boundary of the cut: plane x with out \ in = {y}; masks are cleared for the next plane
            int nnew = 0, ninterior = 0;
            bool bad = false;
            if (cut) {
                for (int p = gl; p - gl < np; p += G) {
                    bool bnd = false, intr = false;
                    if (p < np) {
                        const M mo = KT.mout[p], mi = KT.min[p];
                        KT.mout[p] = 0;
                        KT.min[p] = 0;
                        const M e = mo & ~mi;
                        uint8_t nx8 = 0xFF;
                        if (e) {
                            bnd = true;
                            bad = bad || popc(e) != 1 || popc((M)(mi & ~mo)) != 1;
                            nx8 = (uint8_t)ctz_(e);
                        } else if (mo) {
                            intr = true;
                        }
                        KT.nxt[p] = nx8;
                    }
                    const unsigned long long b = gballot<G>(bnd);
                    if (bnd) KT.newl[nnew + popc(b & below)] = (uint8_t)p;
                    nnew += popc(b);
                    ninterior += popc(gballot<G>(intr));
                }
                bad = gballot<G>(bad) != 0;
            }
            __syncthreads();
            // the two ends of every cut edge; removed slots are freed
            if (cut) {
    #pragma unroll
                for (int k = 0; k < NS; ++k) {
                    const uint32_t u = tri[k];
                    if (u == TRI_INVALID) continue;
                    const int a = u & 0xFF, b = (u >> 8) & 0xFF, c = (u >> 16) & 0xFF;
                    const int na = KT.nxt[a], nb = KT.nxt[b], nc = KT.nxt[c];
                    if (rem[k]) {
                        if (na == b) { KT.rpos[a][0] = vx[k]; KT.rpos[a][1] = vy[k]; KT.rpos[a][2] = vz[k]; }
                        if (nb == c) { KT.rpos[b][0] = vx[k]; KT.rpos[b][1] = vy[k]; KT.rpos[b][2] = vz[k]; }
                        if (nc == a) { KT.rpos[c][0] = vx[k]; KT.rpos[c][1] = vy[k]; KT.rpos[c][2] = vz[k]; }
                        tri[k] = TRI_INVALID;
                    } else {
                        if (nb == a) { KT.kpos[b][0] = vx[k]; KT.kpos[b][1] = vy[k]; KT.kpos[b][2] = vz[k]; }
                        if (nc == b) { KT.kpos[c][0] = vx[k]; KT.kpos[c][1] = vy[k]; KT.kpos[c][2] = vz[k]; }
                        if (na == c) { KT.kpos[a][0] = vx[k]; KT.kpos[a][1] = vy[k]; KT.kpos[a][2] = vz[k]; }
                    }
                }
            }
            __syncthreads();
            // new vertices (x, nxt[x], k) into free slots, in rank order
            if (cut) {
                const int knew = np;
                if (gl == 0) {
                    S.pl[knew][0] = nx;
                    S.pl[knew][1] = ny;
                    S.pl[knew][2] = nz;
                    S.pl[knew][3] = t;
                    S.pid[knew] = S.u.c.csid[it];
                }
                int fbase = 0;
    #pragma unroll
                for (int k = 0; k < NS; ++k) {
                    const bool isfree = tri[k] == TRI_INVALID;
                    const unsigned long long b = gballot<G>(isfree);
                    const int frank = fbase + popc(b & below);
                    fbase += popc(b);
                    if (isfree && frank < nnew) {
                        const int p = KT.newl[frank];
                        const int q = KT.nxt[p];
                        const R ax = KT.kpos[p][0], ay = KT.kpos[p][1], az = KT.kpos[p][2];
                        const R bx = KT.rpos[p][0], by = KT.rpos[p][1], bz = KT.rpos[p][2];
                        const R sa = nx * ax + ny * ay + nz * az - t;
                        const R sb = nx * bx + ny * by + nz * bz - t;
                        const R lam = (sb > sa) ? sa * rcp_<R>(sa - sb) : R(0.5);
                        vx[k] = ax + lam * (bx - ax);
                        vy[k] = ay + lam * (by - ay);
                        vz[k] = az + lam * (bz - az);
                        tri[k] = pack3(p, q, knew);
                    }
                }
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
        }
    };

    // Clip rounds. Round 0 clips the discovered candidates. A cell whose discovery
    // overflowed then runs rounds over the candidates with tau <= t < r_eff (r_eff
    // bounds the current polytope) that cut the polytope and are not yet among its
    // planes: the first CMAX found are clipped in ascending t, and a round that leaves
    // none out is its last. Clipping by any subset is exact (the cell is the
    // intersection of all the half-spaces); each round only shrinks the polytope.
    // One loop holds the only copy of the clipping code.
    int count = ncand, nclip = ncand;
    bool more = overflow && live;
    for (int round = 0;; ++round) {
        rank_round(count);
        __syncthreads();
        clip_round(nclip);
        if (!rounds || round >= (MODE == 1 ? CROWD_ROUNDS : OVERFLOW_ROUNDS) || !__any(more && live)) break;
        compact();
        R v2 = R(0);
#pragma unroll
        for (int k = 0; k < NS; ++k)
            if (tri[k] != TRI_INVALID) v2 = fmax(v2, vx[k] * vx[k] + vy[k] * vy[k] + vz[k] * vz[k]);
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) v2 = fmax(v2, __shfl_xor(v2, o, 64));
        // the restricted cell lies within min(max vertex distance, r) of p_i
        const R reff = v2 > r * r ? r : sqrt(v2);
        int nc2 = 0;
        __syncthreads();  // the clip tables become the staging list
        if (more && live && reff >= tau) {
            const int npl = np;
            scan([&](bool keep, bool, bool, R nx, R ny, R nz, R t, int id, R) {
                unsigned long long pm = gballot<G>(keep && t >= tau && t < reff);
                while (pm) {
                    const int q = __ffsll((long long)pm) - 1;
                    pm &= pm - 1;
                    const R qx = __shfl(nx, gbase + q, 64), qy = __shfl(ny, gbase + q, 64),
                            qz = __shfl(nz, gbase + q, 64), qt = __shfl(t, gbase + q, 64);
                    const int qid = __shfl(id, gbase + q, 64);
                    bool beyond = false;
#pragma unroll
                    for (int k = 0; k < NS; ++k)
                        beyond = beyond || (tri[k] != TRI_INVALID && qx * vx[k] + qy * vy[k] + qz * vz[k] > qt);
                    if (!gballot<G>(beyond)) continue;
                    bool known = false;  // a plane of the polytope (rounding can put its vertices beyond it)
                    for (int pp = 6 + gl; pp < npl; pp += G) known = known || S.pid[pp] == qid;
                    if (gballot<G>(known)) continue;
                    if (gl == 0 && nc2 < CMAX) {
                        D.cand[nc2][0] = qx;
                        D.cand[nc2][1] = qy;
                        D.cand[nc2][2] = qz;
                        D.cand[nc2][3] = qt;
                        D.cid[nc2] = qid;
                    }
                    ++nc2;
                }
            });
        }
        __syncthreads();
        // the nearest (in t) of the collected cutters, as many as free plane slots allow
        count = (more && live) ? min(nc2, CMAX) : 0;
        nclip = min(count, PMAX - 1 - np);
        more = more && live && nc2 > nclip;
        if (more && nclip <= 0) {
            flags |= CF_PLANES;
            live = false;
            more = false;
        }
    }
    if (more && live) {
        flags |= CF_CAND;
        live = false;
    }
    // Each vertex again from its three planes (Cramer's rule): clipping places new
    // vertices by interpolation along edges whose ends carry the rounding of earlier
    // clips, which compounds over long clip sequences. Kept where the planes are well
    // conditioned (|det| of the unit normals > 0.05), else the interpolated position.
    if (live) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const uint32_t u = tri[k];
            if (u == TRI_INVALID) continue;
            const int a = u & 0xFF, b = (u >> 8) & 0xFF, c = (u >> 16) & 0xFF;
            const R ax = S.pl[a][0], ay = S.pl[a][1], az = S.pl[a][2], at = S.pl[a][3];
            const R bx = S.pl[b][0], by = S.pl[b][1], bz = S.pl[b][2], bt = S.pl[b][3];
            const R cx = S.pl[c][0], cy = S.pl[c][1], cz = S.pl[c][2], ct = S.pl[c][3];
            const R bcx = by * cz - bz * cy, bcy = bz * cx - bx * cz, bcz = bx * cy - by * cx;
            const R cax = cy * az - cz * ay, cay = cz * ax - cx * az, caz = cx * ay - cy * ax;
            const R abx = ay * bz - az * by, aby = az * bx - ax * bz, abz = ax * by - ay * bx;
            const R det = ax * bcx + ay * bcy + az * bcz;
            if (fabs(det) > R(0.05)) {
                const R inv = R(1) / det;
                vx[k] = (at * bcx + bt * cax + ct * abx) * inv;
                vy[k] = (at * bcy + bt * cay + ct * aby) * inv;
                vz[k] = (at * bcz + bt * caz + ct * abz) * inv;
            }
        }
    }

    // ---------------- the cell's box (fast and seed passes) ----------------
    // The polytope's vertex bounds clamped to the ball's bounds, widened by a margin for
    // float32 rounding (relative to r, and to the coordinates): a box that holds the
    // restricted cell (the exact cell in the fast pass, a superset in the seed pass).
    // Cells that failed get the ball's bounds, empty cells an empty box.
    if ((MODE == 0 && A.crowd) || seed) {
        R b0x = R(3e38), b0y = R(3e38), b0z = R(3e38), b1x = R(-3e38), b1y = R(-3e38), b1z = R(-3e38);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (tri[k] == TRI_INVALID) continue;
            b0x = fmin(b0x, vx[k]);
            b0y = fmin(b0y, vy[k]);
            b0z = fmin(b0z, vz[k]);
            b1x = fmax(b1x, vx[k]);
            b1y = fmax(b1y, vy[k]);
            b1z = fmax(b1z, vz[k]);
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
            b0x = fmin(b0x, __shfl_xor(b0x, o, 64));
            b0y = fmin(b0y, __shfl_xor(b0y, o, 64));
            b0z = fmin(b0z, __shfl_xor(b0z, o, 64));
            b1x = fmax(b1x, __shfl_xor(b1x, o, 64));
            b1y = fmax(b1y, __shfl_xor(b1y, o, 64));
            b1z = fmax(b1z, __shfl_xor(b1z, o, 64));
        }
        if (act && !deferred && gl == 0) {
            const float mg = 2e-5f * (float)r + 2e-7f * (fabsf((float)px) + fabsf((float)py) + fabsf((float)pz));
            float4 lo = make_float4(3e38f, 3e38f, 3e38f, 0.f), hi = make_float4(-3e38f, -3e38f, -3e38f, 0.f);
            if (live) {
                lo = make_float4((float)(px + fmax(b0x, -r)) - mg, (float)(py + fmax(b0y, -r)) - mg,
                                 (float)(pz + fmax(b0z, -r)) - mg, 0.f);
                hi = make_float4((float)(px + fmin(b1x, r)) + mg, (float)(py + fmin(b1y, r)) + mg,
                                 (float)(pz + fmin(b1z, r)) + mg, 0.f);
            } else if (!(flags & CF_EMPTY) && r > R(0)) {
                const float rr = (float)r * 1.00002f + mg;
                lo = make_float4((float)px - rr, (float)py - rr, (float)pz - rr, 0.f);
                hi = make_float4((float)px + rr, (float)py + rr, (float)pz + rr, 0.f);
            }
            A.qb.box[2 * cell] = lo;
            A.qb.box[2 * cell + 1] = hi;
        }
        if (seed) return;
    }

    // ---------------- restriction to the ball and integration ----------------
    // Every (vertex, facet through it) pair is one fan piece: the edge from the vertex to
    // its counter-clockwise successor on that facet. The pieces are listed, spread over
    // all lanes of the cell, and summed per facet in the facet's walk order (fixed order:
    // deterministic).
    static_assert(sizeof(GT.rec) + sizeof(GT.eslot) >= sizeof(R) * 6 * VMAX, "piece storage");
    static_assert(sizeof(GT.eslot) >= sizeof(uint16_t) * 3 * VMAX, "piece list storage");
    __syncthreads();
    if (live) {
        for (int p = gl; p < np; p += G) GT.fstart[p] = 0xFFu;
    }
    __syncthreads();
    if (live) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const uint32_t u = tri[k];
            if (u == TRI_INVALID) continue;
            const int s = k * G + gl;
            const int a = u & 0xFF, b = (u >> 8) & 0xFF, c = (u >> 16) & 0xFF;
            GT.rec[s] = VRec<R>{vx[k], vy[k], vz[k], u};
            GT.trs[s] = u;
            GT.eslot[a][b] = (uint8_t)s;
            GT.eslot[b][c] = (uint8_t)s;
            GT.eslot[c][a] = (uint8_t)s;
            atomicMin(&GT.fstart[a], (uint32_t)s);
            atomicMin(&GT.fstart[b], (uint32_t)s);
            atomicMin(&GT.fstart[c], (uint32_t)s);
        }
    }
    __syncthreads();
    // successor of vertex (a,b,c) counter-clockwise on face a is the vertex holding edge a->c
    uint32_t sc_k[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        sc_k[k] = 0xFFFFFFFFu;
        const uint32_t u = tri[k];
        if (live && u != TRI_INVALID) {
            const int a = u & 0xFF, b = (u >> 8) & 0xFF, c = (u >> 16) & 0xFF;
            sc_k[k] = (uint32_t)GT.eslot[a][c] | ((uint32_t)GT.eslot[b][a] << 8) | ((uint32_t)GT.eslot[c][b] << 16);
        }
    }
    __syncthreads();  // eslot is dead from here on: it takes the piece list
    uint16_t *plist = reinterpret_cast<uint16_t *>(&GT.eslot[0][0]);
    int npc = 0;
    if (live) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const uint32_t u = tri[k];
            const int s = k * G + gl;
            if (u != TRI_INVALID) GT.succ[s] = sc_k[k];
#pragma unroll
            for (int rot = 0; rot < 3; ++rot) {
                const bool want = u != TRI_INVALID && (int)((u >> (8 * rot)) & 0xFFu) >= 6;
                const unsigned long long bm = gballot<G>(want);
                if (want) plist[npc + popc(bm & below)] = (uint16_t)(3 * s + rot);
                npc += popc(bm);
            }
        }
    }
    __syncthreads();
    // a polytope whose vertices all lie in the ball lies in it (both convex): the cell
    // has no spherical part (K = 0 exactly, not the difference 4 pi - sum of solid
    // angles) and V is the pyramid sum alone
    R v2max = R(0);
#pragma unroll
    for (int k = 0; k < NS; ++k)
        if (tri[k] != TRI_INVALID) v2max = fmax(v2max, vx[k] * vx[k] + vy[k] * vy[k] + vz[k] * vz[k]);
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v2max = fmax(v2max, __shfl_xor(v2max, o, 64));
    const bool in_ball = v2max < r * r;
    // the pieces, G at a time; with MOM each lane also sums its pieces' share of the
    // first moment: 4 integral of x dV = sum_f [t (t n A + m) - r^2 n A] over the facets
    // (x.n = t on a facet, whose moment about p_i is t n A + m; on the sphere x.n = r and
    // the vector area of the spherical part is -sum_f n A). In the ball the r^2 term is
    // exactly zero (closed polytope) and is left out.
    constexpr int MAXR = 3 * NS;
    R pa[MAXR], po[MAXR];
    double mom_x = 0.0, mom_y = 0.0, mom_z = 0.0;
    int pc[MAXR];
    bool walk_bad = false;
    const R cone_den = live ? R(1) / r : R(0);
#pragma unroll
    for (int rr = 0; rr < MAXR; ++rr) {
        pa[rr] = po[rr] = R(0);
        pc[rr] = -1;
        const int idx = rr * G + gl;
        if (live && idx < npc) {
            const int code = plist[idx];
            pc[rr] = code;
            const int sv = code / 3, rot = code - 3 * sv;
            const uint32_t u = GT.trs[sv];
            const int f = (int)((u >> (8 * rot)) & 0xFFu);
            const uint32_t sn = (GT.succ[sv] >> (8 * rot)) & 0xFFu;
            if (sn >= (uint32_t)VMAX) {
                walk_bad = true;
            } else {
                const R nx = S.pl[f][0], ny = S.pl[f][1], nz = S.pl[f][2], t = S.pl[f][3];
                const R h = fabs(t);
                const R rho2 = (r - t) * (r + t);
                const R cone = R(1) - h * cone_den;
                const R qx = t * nx, qy = t * ny, qz = t * nz;
                const VRec<R> P = GT.rec[sv], Q = GT.rec[sn];
                const PieceSum<R> ps = fan_piece<R, MOM>(P.x - qx, P.y - qy, P.z - qz, Q.x - qx, Q.y - qy, Q.z - qz,
                                                         nx, ny, nz, rho2, h, cone);
                pa[rr] = ps.A;
                po[rr] = ps.Om;
                const R mx = ps.Mx, my = ps.My, mz = ps.Mz;
                if constexpr (KR) {
                    const KRArc<R> ka = kr_arc<R>(P.x, P.y, P.z, Q.x, Q.y, Q.z, nx, ny, nz, t, r);
                    KS->pm[code][0] = mx;
                    KS->pm[code][1] = my;
                    KS->pm[code][2] = mz;
                    KS->pm[code][3] = ps.A;
                    KS->pm[code][4] = ka.phi;
                    KS->pm[code][5] = ka.lo < ka.hi ? R(1) : R(0);
                }
                if constexpr (MOM) {
                    const double td = (double)t, ar = (double)pa[rr];
                    const double c2 = td * td - (in_ball ? 0.0 : (double)r * (double)r);
                    mom_x += c2 * (double)nx * ar + td * (double)mx;
                    mom_y += c2 * (double)ny * ar + td * (double)my;
                    mom_z += c2 * (double)nz * ar + td * (double)mz;
                }
            }
        }
    }
    // section 3.3's route: c = point_in (a ray from each restricted facet's area centroid
    // along -n to the first of the sphere and the other planes; the mean of the chords'
    // midpoints), then the Gauss-Bonnet shares of the pieces (kr_piece)
    double kr_sum = 0.0;
    int kr_faces = 0;
    if constexpr (KR) {
        static_assert(MOM, "the route needs the pieces' first moments");
        __syncthreads();
        if (live) {
            for (int p = gl; p < np; p += G) {
                R f0 = 0, f1 = 0, f2 = 0, f3 = 0;
                const uint32_t s0 = GT.fstart[p];
                if (p >= 6 && s0 < (uint32_t)VMAX) {
                    R Af = 0, Mx = 0, My = 0, Mz = 0, phi = 0, nseg = 0;
                    uint32_t sv = s0;
                    int steps = 0;
                    do {
                        const uint32_t u = GT.trs[sv];
                        const int rot = ((int)(u & 0xFFu) == p) ? 0
                                      : (((int)((u >> 8) & 0xFFu) == p) ? 1 : (((int)((u >> 16) & 0xFFu) == p) ? 2 : -1));
                        if (rot < 0) break;
                        Mx += KS->pm[3 * sv + rot][0];
                        My += KS->pm[3 * sv + rot][1];
                        Mz += KS->pm[3 * sv + rot][2];
                        Af += KS->pm[3 * sv + rot][3];
                        phi += KS->pm[3 * sv + rot][4];
                        nseg += KS->pm[3 * sv + rot][5];
                        const uint32_t sn = (GT.succ[sv] >> (8 * rot)) & 0xFFu;
                        if (sn >= (uint32_t)VMAX || ++steps > VMAX) break;
                        sv = sn;
                    } while (sv != s0);
                    if ((nseg > R(0) || phi > R(PI_D)) && Af > R(0)) {
                        const R nx = S.pl[p][0], ny = S.pl[p][1], nz = S.pl[p][2], t = S.pl[p][3];
                        const R ia = R(1) / Af;
                        const R gx = t * nx + Mx * ia, gy = t * ny + My * ia, gz = t * nz + Mz * ia;
                        // d = -n: the far root of |g + s d| = r, then the other planes
                        const R gd = -dot3(gx, gy, gz, nx, ny, nz);
                        R lam = -gd + sqrt(fmax(gd * gd - (dot3(gx, gy, gz, gx, gy, gz) - r * r), R(0)));
                        for (int k = 6; k < np; ++k) {
                            if (k == p) continue;
                            const R den = -dot3(S.pl[k][0], S.pl[k][1], S.pl[k][2], nx, ny, nz);
                            if (den > R(0)) {
                                const R l = (S.pl[k][3] - dot3(S.pl[k][0], S.pl[k][1], S.pl[k][2], gx, gy, gz)) / den;
                                lam = fmin(lam, l);
                            }
                        }
                        lam = fmax(lam, R(0));
                        f0 = gx - R(0.5) * lam * nx;
                        f1 = gy - R(0.5) * lam * ny;
                        f2 = gz - R(0.5) * lam * nz;
                        f3 = R(1);
                    }
                }
                KS->fm[p][0] = f0;
                KS->fm[p][1] = f1;
                KS->fm[p][2] = f2;
                KS->fm[p][3] = f3;
            }
        }
        __syncthreads();
        double csx = 0.0, csy = 0.0, csz = 0.0;
        if (live) {
            for (int p = gl; p < np; p += G) {
                if (KS->fm[p][3] > R(0)) {
                    csx += (double)KS->fm[p][0];
                    csy += (double)KS->fm[p][1];
                    csz += (double)KS->fm[p][2];
                    ++kr_faces;
                }
            }
        }
        csx = gsum<G>(csx);
        csy = gsum<G>(csy);
        csz = gsum<G>(csz);
        kr_faces = (int)gsum<G>((double)kr_faces);
        const R ccx = kr_faces ? (R)(csx / kr_faces) : R(0), ccy = kr_faces ? (R)(csy / kr_faces) : R(0),
                ccz = kr_faces ? (R)(csz / kr_faces) : R(0);
#pragma unroll
        for (int rr = 0; rr < MAXR; ++rr) {
            const int idx = rr * G + gl;
            if (live && idx < npc && kr_faces > 0) {
                const int code = plist[idx];
                const int sv = code / 3, rot = code - 3 * sv;
                const uint32_t u = GT.trs[sv];
                const int f = (int)((u >> (8 * rot)) & 0xFFu);
                const uint32_t sn = (GT.succ[sv] >> (8 * rot)) & 0xFFu;
                if (sn < (uint32_t)VMAX && KS->fm[f][3] > R(0)) {
                    const uint32_t un = GT.trs[sn];
                    const int rot2 = ((int)(un & 0xFFu) == f) ? 0 : (((int)((un >> 8) & 0xFFu) == f) ? 1 : 2);
                    const uint32_t sx = (GT.succ[sn] >> (8 * rot2)) & 0xFFu;
                    if (sx < (uint32_t)VMAX) {
                        const VRec<R> P = GT.rec[sv], Q = GT.rec[sn], X = GT.rec[sx];
                        kr_sum += (double)kr_piece<R>(P.x, P.y, P.z, Q.x, Q.y, Q.z, X.x, X.y, X.z, S.pl[f][0],
                                                      S.pl[f][1], S.pl[f][2], S.pl[f][3], r, ccx, ccy, ccz);
                    } else {
                        walk_bad = true;
                    }
                }
            }
        }
        kr_sum = gsum<G>(kr_sum);
    }
    __syncthreads();  // rec and the list are dead: they take the pieces
    R(*pieces)[2] = reinterpret_cast<R(*)[2]>(&GT.rec[0]);
#pragma unroll
    for (int rr = 0; rr < MAXR; ++rr) {
        if (pc[rr] >= 0) {
            pieces[pc[rr]][0] = pa[rr];
            pieces[pc[rr]][1] = po[rr];
        }
    }
    __syncthreads();
    // per facet: sum its pieces in walk order from its lowest slot
    double sum_tA = 0.0, sum_om = 0.0, sum_tA_abs = 0.0;
    if (live) {
        for (int p = gl; p < np; p += G) {
            R Af = 0, Of = 0;
            const uint32_t s0 = GT.fstart[p];
            if (p >= 6 && s0 < (uint32_t)VMAX) {
                uint32_t sv = s0;
                int steps = 0;
                do {
                    const uint32_t u = GT.trs[sv];
                    const int rot = ((int)(u & 0xFFu) == p) ? 0
                                  : (((int)((u >> 8) & 0xFFu) == p) ? 1 : (((int)((u >> 16) & 0xFFu) == p) ? 2 : -1));
                    if (rot < 0) {
                        walk_bad = true;
                        break;
                    }
                    Af += pieces[3 * sv + rot][0];
                    Of += pieces[3 * sv + rot][1];
                    const uint32_t sn = (GT.succ[sv] >> (8 * rot)) & 0xFFu;
                    if (sn >= (uint32_t)VMAX || ++steps > VMAX) {
                        walk_bad = true;
                        break;
                    }
                    sv = sn;
                } while (sv != s0);
                const R t = S.pl[p][3];
                sum_tA += (double)t * (double)Af;
                sum_tA_abs += fabs((double)t * (double)Af);
                sum_om += (t >= R(0)) ? (double)Of : -(double)Of;
            }
            GT.farea[p] = Af;
        }
    }
    if (gballot<G>(walk_bad)) {
        flags |= CF_WALK;
        live = false;
    }
    sum_tA = gsum<G>(sum_tA);
    sum_tA_abs = gsum<G>(sum_tA_abs);
    if constexpr (MOM) {
        mom_x = gsum<G>(mom_x);
        mom_y = gsum<G>(mom_y);
        mom_z = gsum<G>(mom_z);
    }
    sum_om = gsum<G>(sum_om);
    __syncthreads();

    // ---------------- outputs ----------------
    if (!act) return;
    const EvalOut &o = A.out;
    if (deferred) {
        if (gl == 0) {
            o.ovf_list[atomicAdd(o.ovf_count, 1)] = (int32_t)cell;
            o.flags[cell] = CF_CAND;  // the reason, kept by a float64 pass
        }
        return;
    }
    int nf = 0;
    if (live) {
        for (int p = gl; p - gl < np; p += G) {
            bool isf = false;
            float a = 0.f;
            int id = -100;
            if (p < np && p >= 6) {
                a = (float)GT.farea[p];
                id = S.pid[p];
                isf = id >= 0 && a > 0.f;
                if (id < 0 && o.wall) o.wall[cell * (A.bt.ndom > 0 ? A.bt.ndom : 6) + (-1 - id)] = a;
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
            if constexpr (KR) {
                // no restricted facet: the whole sphere if p_i is in the cell, else nothing
                K = kr_faces == 0 ? rd * rd * 4.0 * PI_D * (inside ? 1.0 : 0.0)
                                  : rd * rd * (4.0 * PI_D - 2.0 * PI_D * kr_faces + kr_sum);
            } else {
                K = in_ball ? 0.0 : rd * rd * (4.0 * PI_D * (inside ? 1.0 : 0.0) - sum_om);
            }
            V = (sum_tA + rd * K) / 3.0;
            if (!(V == V) || !(K == K)) flags |= CF_TOPO;
        }
        // a cell much smaller than its terms is a difference of large ones (with a
        // spherical part: of the ball's size; without: pyramids from a site far from its
        // cell): float32 would lose the relative accuracy, so it is redone in float64
        if (MOM && o.cen) {
            // centroid in caller order: the site plus the first moment over the volume
            const int64_t ci = A.perm[cell];
            const double f = V > 0.0 ? 0.25 / V : 0.0;
            o.cen[3 * ci + 0] = (double)px + f * mom_x;
            o.cen[3 * ci + 1] = (double)py + f * mom_y;
            o.cen[3 * ci + 2] = (double)pz + f * mom_z;
        }
        const double scale = in_ball ? sum_tA_abs / 3.0 : (4.0 / 3.0) * PI_D * (double)r * (double)r * (double)r;
        if (fast && sizeof(R) == 4 && live && (V < 0.05 * scale || nnear >= 2)) flags |= CF_PREC;
        o.V[cell] = V;
        o.K[cell] = K;
        o.fcnt[cell] = live ? nf : 0;
        // the float64 pass keeps the float32 pass's reasons in bits 8..15
        o.flags[cell] = (fast || KR) ? flags : (flags | (o.flags[cell] << 8));
        if (fast && (flags & (CF_FAIL_MASK | CF_PREC))) {
            const int slot = atomicAdd(o.fb_count, 1);
            o.fb_list[slot] = (int32_t)cell;
            atomicAdd(o.fb_inst + inst, 1);
        } else if (!fast && (flags & CF_FAIL_MASK)) {
            atomicAdd(o.fail_inst + inst, 1);
        }
    }
}

template <int G, bool MOM>
__global__ __launch_bounds__(64) void k_cells_fast(CellArgs A) {
    __shared__ CellSmem<float, FAST_CMAX, FAST_PMAX, FAST_VMAX> smem[64 / G];
    const int gi = (int)(threadIdx.x / G);
    int64_t cell = (int64_t)xcd_block((int)blockIdx.x, (int)gridDim.x) * (64 / G) + gi;
    if (cell >= A.n || !selected(A.bt, A.want, A.bt.inst[cell])) cell = -1;
    cell_body<float, G, FAST_CMAX, FAST_PMAX, FAST_VMAX, 0, MOM>(cell, A, smem[gi]);
}

// Seed pass of the cells deferred by the fast pass (crowded cells), one per wavefront:
// each is clipped by its nearest sites only, and writes the box of that superset of
// its cell. The list length is read on the device and the blocks stride over it.
// Work-list loops: the list is split into NXCD contiguous parts, one per XCD (workgroup w
// runs on XCD w mod NXCD), and the workgroups of an XCD stride over its part, so cells
// that are neighbours in the list (and in space) run on the same XCD and share its L2.
#define XCD_LIST_LOOP(k, count)                                                                \
    const int xcd_ = (int)(blockIdx.x % NXCD), per_ = (int)(gridDim.x / NXCD);                 \
    const int lo_ = (int)((int64_t)(count) * xcd_ / NXCD), hi_ = (int)((int64_t)(count) * (xcd_ + 1) / NXCD); \
    for (int k = lo_ + (int)(blockIdx.x / NXCD); k < hi_; k += per_)

__global__ __launch_bounds__(64) void k_cells_seed(CellArgs A) {
    __shared__ CellSmem<float, SEED_CMAX, SEED_PMAX, SEED_VMAX> smem[1];
    const int count = *A.out.ovf_count;
    XCD_LIST_LOOP(k, count) {
        const int64_t cell = A.out.ovf_list[k];
        cell_body<float, 64, SEED_CMAX, SEED_PMAX, SEED_VMAX, 3, false>(cell, A, smem[0]);
        __syncthreads();
    }
}

// The deferred cells in grid order (the fast pass appends them in the order its atomics
// happen): a deferred cell is the only one whose fast-pass flags are exactly CF_CAND.
// Grid order is space order, so the seed and crowded passes then read neighbouring data.
__global__ __launch_bounds__(256) void k_defer_mark(int64_t n, Batch bt, int want, const uint32_t *__restrict__ flags,
                                                    const int32_t *__restrict__ ovf_count, int32_t *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cnt[i] = (*ovf_count > 0 && selected(bt, want, bt.inst[i]) && flags[i] == CF_CAND) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_defer_fill(int64_t n, const int32_t *__restrict__ cnt,
                                                    const int32_t *__restrict__ start, int32_t *__restrict__ list) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && cnt[i]) list[start[i]] = (int32_t)i;
}

// Registration of the cell boxes in the buckets of the box grid (every cell of the
// selected instances; nothing to do when no cell was deferred). A box spanning more
// than QREG_MAX buckets goes to the list of large boxes instead.
struct BucketRange {
    int lo[3], hi[3], count;
};
__device__ inline BucketRange bucket_range(const GridDesc &g, float4 lo, float4 hi) {
    BucketRange br;
    const float l[3] = {lo.x, lo.y, lo.z}, h[3] = {hi.x, hi.y, hi.z};
    br.count = 1;
    for (int a = 0; a < 3; ++a) {
        br.lo[a] = min(max((int)floorf((l[a] - g.lo[a]) * g.inv_s), 0), g.dim[a] - 1);
        br.hi[a] = min(max((int)floorf((h[a] - g.lo[a]) * g.inv_s), 0), g.dim[a] - 1);
        br.count *= br.hi[a] - br.lo[a] + 1;
    }
    return br;
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_qbox_register(int64_t n, Batch bt, int want, const int32_t *__restrict__ ovf_count,
                                                       QBoxes qb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || *ovf_count == 0) return;
    const int b = bt.inst[i];
    if (!selected(bt, want, b)) return;
    const float4 lo = qb.box[2 * i], hi = qb.box[2 * i + 1];
    if (!(lo.x <= hi.x && lo.y <= hi.y && lo.z <= hi.z)) return;  // empty cell
    GridDesc g;
    BucketRange br;
    int lev = 0;
    for (; lev < QLEV; ++lev) {
        g = qb.qgrid[b * QLEV + lev];
        br = bucket_range(g, lo, hi);
        if (br.count <= QREG_MAX) break;
    }
    if (lev == QLEV) {
        if (!FILL) qb.large[atomicAdd(qb.nlarge, 1)] = (int32_t)i;
        return;
    }
    for (int ix = br.lo[0]; ix <= br.hi[0]; ++ix)
        for (int iy = br.lo[1]; iy <= br.hi[1]; ++iy)
            for (int iz = br.lo[2]; iz <= br.hi[2]; ++iz) {
                const int key = g.base + (ix * g.dim[1] + iy) * g.dim[2] + iz;
                if (FILL)
                    qb.ent[qb.start[key] + atomicAdd(qb.cursor + key, 1)] = (int32_t)i;
                else
                    atomicAdd(qb.count + key, 1);
            }
}

// counts (and the large list) before the count pass, fill cursors before the fill pass
__global__ __launch_bounds__(256) void k_qbox_zero(QBoxes qb, bool cursors) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cursors) {
        if (k < qb.nq) qb.cursor[k] = 0;
        return;
    }
    if (k <= qb.nq) qb.count[k] = 0;
    if (k == 0) *qb.nlarge = 0;
}

// The list of large boxes in ascending order (its length is small; one thread, heap sort),
// so that the candidates do not depend on the order of the atomics.
__global__ __launch_bounds__(64) void k_qbox_sort_large(QBoxes qb) {
    if (threadIdx.x != 0) return;
    int32_t *a = qb.large;
    const int m = *qb.nlarge;
    auto sift = [&](int root, int end) {
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
    };
    for (int r = m / 2 - 1; r >= 0; --r) sift(r, m);
    for (int last = m - 1; last > 0; --last) {
        const int32_t t = a[0];
        a[0] = a[last];
        a[last] = t;
        sift(0, last);
    }
}

// Crowded pass: the deferred cells, one per wavefront, in float64 (a crowded cell's site
// often lies well outside its cell, where the pyramid terms of float32 coordinates
// cancel), with the candidates whose boxes overlap the cell's box, the threshold ladder
// and clip rounds when they exceed the capacity.
__global__ __launch_bounds__(64) void k_cells_overflow(CellArgs A) {
    __shared__ CellSmem<double, OVF_CMAX, OVF_PMAX, OVF_VMAX> smem[1];
    const int count = *A.out.ovf_count;
    XCD_LIST_LOOP(k, count) {
        const int64_t cell = A.out.ovf_list[k];
        cell_body<double, 64, OVF_CMAX, OVF_PMAX, OVF_VMAX, 1, true>(cell, A, smem[0]);
        __syncthreads();
    }
}

// The float64 large-capacity pass: the cells the earlier passes listed, and, when the
// crowded pass is off, the cells the fast pass deferred.
__global__ __launch_bounds__(64) void k_cells_big(CellArgs A) {
    __shared__ CellSmem<double, BIG_CMAX, BIG_PMAX, BIG_VMAX> smem[1];
    const int count = *A.out.fb_count;
    const int total = count + (A.crowd ? 0 : *A.out.ovf_count);
    XCD_LIST_LOOP(k, total) {
        const int64_t cell = k < count ? A.out.fb_list[k] : A.out.ovf_list[k - count];
        cell_body<double, 64, BIG_CMAX, BIG_PMAX, BIG_VMAX, 2, true>(cell, A, smem[0]);
        __syncthreads();
    }
}

// Every cell on the float64 path with |K| by section 3.3's own route (interior point,
// projected facets, Gauss-Bonnet): the A/B variant of the signed solid-angle form.
__global__ __launch_bounds__(64) void k_cells_kroute(CellArgs A) {
    __shared__ CellSmem<double, BIG_CMAX, BIG_PMAX, BIG_VMAX> smem[1];
    __shared__ KRSmem<double, BIG_PMAX, BIG_VMAX> krs[1];
    XCD_LIST_LOOP(k, A.n) {
        cell_body<double, 64, BIG_CMAX, BIG_PMAX, BIG_VMAX, 2, true, true>(k, A, smem[0], &krs[0]);
        __syncthreads();
    }
}

// Clears the per-evaluation counters: the overflow and float64 work lists and the
// failure counts of the selected instances (a kernel, so the sequence can be captured).
__global__ __launch_bounds__(1024) void k_eval_begin(Batch bt, int want, EvalOut o) {
    if (threadIdx.x == 0) {
        *o.fb_count = 0;
        *o.ovf_count = 0;
    }
    for (int b = threadIdx.x; b < bt.B; b += 1024)
        if (selected(bt, want, b)) o.fail_inst[b] = 0;
}

}  // namespace

void launch_cells_kroute(hipStream_t st, int64_t n, const Batch &bt, const float4 *pos_s, const double *psi,
                         const int32_t *perm, const int32_t *cell_start, EvalOut out, const QBoxes &qb) {
    CellArgs a{n, pos_s, psi, perm, cell_start, bt, -1, out, qb, 0};
    hipLaunchKernelGGL(k_cells_kroute, dim3(4096), dim3(64), 0, st, a);
}

void launch_eval_begin(hipStream_t st, const Batch &bt, int want, EvalOut out) {
    hipLaunchKernelGGL(k_eval_begin, dim3(1), dim3(1024), 0, st, bt, want, out);
}

void launch_cells(hipStream_t st, int64_t n, const Batch &bt, int want, const float4 *pos_s, const double *psi,
                  const int32_t *perm, const int32_t *cell_start, EvalOut out, const QBoxes &qb, int tpc, bool crowd) {
    CellArgs a{n, pos_s, psi, perm, cell_start, bt, want, out, qb, crowd ? 1 : 0};
    if (out.cen) {  // centroids: one instantiation (32 lanes per cell)
        hipLaunchKernelGGL((k_cells_fast<32, true>), dim3((unsigned)((n + 1) / 2)), dim3(64), 0, st, a);
    } else if (tpc == 8) {
        hipLaunchKernelGGL((k_cells_fast<8, false>), dim3((unsigned)((n + 7) / 8)), dim3(64), 0, st, a);
    } else if (tpc == 32) {
        hipLaunchKernelGGL((k_cells_fast<32, false>), dim3((unsigned)((n + 1) / 2)), dim3(64), 0, st, a);
    } else if (tpc == 64) {
        hipLaunchKernelGGL((k_cells_fast<64, false>), dim3((unsigned)n), dim3(64), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_cells_fast<16, false>), dim3((unsigned)((n + 3) / 4)), dim3(64), 0, st, a);
    }
}

// The crowded cells deferred by the fast pass (seed boxes, box grid, box-overlap
// candidates), then the cells listed for the float64 pass by both; the passes read the
// list lengths on the device (no host synchronisation).
void launch_cells_fallback(hipStream_t st, int64_t n, const Batch &bt, int want, const float4 *pos_s,
                           const double *psi, const int32_t *perm, const int32_t *cell_start, EvalOut out,
                           const QBoxes &qb, bool crowd, hipEvent_t e0, hipEvent_t e1, int32_t *start_gate) {
    CellArgs a{n, pos_s, psi, perm, cell_start, bt, want, out, qb, crowd ? 1 : 0};
    if (!crowd) {
        hipLaunchKernelGGL(k_cells_big, dim3(2048), dim3(64), 0, st, a);
        return;
    }
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_defer_mark, dim3(nb), dim3(256), 0, st, n, bt, want, out.flags, out.ovf_count, qb.dcnt);
    launch_scan_i32(st, qb.dcnt, qb.dstart, (int)n, qb.tmp);
    hipLaunchKernelGGL(k_defer_fill, dim3(nb), dim3(256), 0, st, n, qb.dcnt, qb.dstart, out.ovf_list);
    hipLaunchKernelGGL(k_cells_seed, dim3(4096), dim3(64), 0, st, a);
    // a start that the repair gate would send to the restart skips the rest (empty boxes)
    if (start_gate) launch_start_gate(st, bt, want, qb.box, out.V, start_gate, out.fb_count, out.ovf_count);
    const unsigned nz = (unsigned)((qb.nq + 256) / 256);
    hipLaunchKernelGGL(k_qbox_zero, dim3(nz), dim3(256), 0, st, qb, false);
    hipLaunchKernelGGL(k_qbox_register<false>, dim3(nb), dim3(256), 0, st, n, bt, want, out.ovf_count, qb);
    launch_scan_i32(st, qb.count, qb.start, qb.nq, qb.tmp);
    hipLaunchKernelGGL(k_qbox_zero, dim3(nz), dim3(256), 0, st, qb, true);
    hipLaunchKernelGGL(k_qbox_register<true>, dim3(nb), dim3(256), 0, st, n, bt, want, out.ovf_count, qb);
    launch_sort_segments(st, qb.nq, qb.start, qb.ent);
    hipLaunchKernelGGL(k_qbox_sort_large, dim3(1), dim3(64), 0, st, qb);
    if (e0) (void)hipEventRecord(e0, st);
    hipLaunchKernelGGL(k_cells_overflow, dim3(4096), dim3(64), 0, st, a);
    if (e1) (void)hipEventRecord(e1, st);
    hipLaunchKernelGGL(k_cells_big, dim3(2048), dim3(64), 0, st, a);
}

}  // namespace lagot
