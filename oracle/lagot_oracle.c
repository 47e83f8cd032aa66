/*
 * lagot_oracle.c -- plain FP64 CPU reference ("oracle") for the generalized
 * Laguerre cells of semi-discrete partial optimal transport.
 *
 * TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg of
 * the benchmark call this file; the product path never does. It shares no code
 * with the HIP kernels.
 *
 * What it computes (paper: section 2.2 "Free Surface", eq. (1); section 3.2
 * "Pyramid Decomposition"; section 3.3 "Area of Spherical Patches";
 * Algorithm 2 "Facets areas and volume of a Laguerre cell restricted to a
 * sphere"):
 *
 *   C_i = box  ∩  B(p_i, sqrt(psi_i))  ∩  { x : |x-p_i|^2 - psi_i <= |x-p_j|^2 - psi_j  for all j != i }
 *
 * and, for each site i,
 *   V_i  = |C_i|                       volume
 *   K_i  = |∂B_i ∩ C_i|               free (spherical) surface area
 *   A_ij = |C_i ∩ bisector(i,j)|       restricted Laguerre facet areas
 *   W_iw = |C_i ∩ wall w|              box-wall facet areas (w = -x,+x,-y,+y,-z,+z)
 *
 * Route (written plainly, no blocking or reordering beyond the definition):
 *   1. neighbours by brute force over all j; the bisector of (i,j) in coordinates
 *      local to p_i is { y : n_ij . y = t_ij } with n_ij = (p_j-p_i)/d_ij and
 *      t_ij = (d_ij^2 + psi_i - psi_j) / (2 d_ij)  (section 3.2, h_ij read as a
 *      signed scalar with its factor 1/2);
 *   2. the polytope box ∩ cube(p_i, 2r) ∩ half-spaces is built as explicit face
 *      polygons by Sutherland-Hodgman clipping of every face, in ascending t;
 *   3. every facet polygon is restricted to its disk (centre q = t n, radius
 *      rho = sqrt(r^2 - t^2)) by the signed fan of triangles and circular sectors
 *      around q (section 3.2: "triangles and circular sectors"); the same fan
 *      gives the solid angle the restricted facet subtends at p_i;
 *   4. occlusion identity (section 3.3, |K_i| = |Sigma_i| - sum of projected
 *      facets) with the projection centre c = p_i and signed solid angles:
 *      K_i = r^2 (4 pi [p_i in C_i] - sum_f sgn(t_f) Omega_f);
 *   5. pyramid decomposition with F = (x - p_i)/3 (section 3.2):
 *      V_i = (1/3) (sum_f t_f A_f + r K_i).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

enum { OR_OK = 0, OR_EMPTY = 1, OR_FACET_CAP = 2 };

typedef struct {
    double n[3]; /* unit outward normal of the half-space n.y <= t (local coords) */
    double t;    /* signed distance of the plane from p_i                        */
    long id;     /* >= 0 neighbour site, -1..-6 box wall, -7..-12 auxiliary cube  */
} oplane;

typedef struct {
    int plane;   /* index into the plane table */
    int nv, cap;
    double *v;   /* nv * 3 vertices, counter-clockwise seen from outside */
} oface;

typedef struct {
    int nf, cap;
    oface *f;
} opoly;

/* Work units of one cell evaluation (for cost models; not part of the result):
 * [0] bisector planes cutting the ball, [1] vertex-versus-plane tests,
 * [2] vertices created by clipping, [3] restricted facets (neighbour + wall faces),
 * [4] facet polygon edges integrated, [5] of which cross the facet's circle. */
enum { W_CAND = 0, W_TESTS, W_NEWV, W_FACES, W_EDGES, W_CROSS, W_N };
static __thread long *g_work = NULL;

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void face_push(oface *f, const double *p)
{
    if (f->nv == f->cap) {
        f->cap = f->cap ? 2 * f->cap : 8;
        f->v = (double *)realloc(f->v, sizeof(double) * 3 * (size_t)f->cap);
    }
    memcpy(f->v + 3 * f->nv, p, 3 * sizeof(double));
    f->nv++;
}

static oface *poly_new_face(opoly *P, int plane)
{
    if (P->nf == P->cap) {
        P->cap = P->cap ? 2 * P->cap : 16;
        P->f = (oface *)realloc(P->f, sizeof(oface) * (size_t)P->cap);
    }
    oface *f = &P->f[P->nf++];
    f->plane = plane;
    f->nv = 0;
    f->cap = 0;
    f->v = NULL;
    return f;
}

static void poly_free(opoly *P)
{
    for (int k = 0; k < P->nf; ++k) free(P->f[k].v);
    free(P->f);
    P->f = NULL;
    P->nf = P->cap = 0;
}

/* --- ordering of points of a planar convex set, counter-clockwise about n --- */
typedef struct {
    double ang;
    double p[3];
} angpt;

static int cmp_angpt(const void *a, const void *b)
{
    const angpt *u = (const angpt *)a, *v = (const angpt *)b;
    if (u->ang < v->ang) return -1;
    if (u->ang > v->ang) return 1;
    for (int k = 0; k < 3; ++k) {
        if (u->p[k] < v->p[k]) return -1;
        if (u->p[k] > v->p[k]) return 1;
    }
    return 0;
}

static void plane_frame(const double *n, double *e1, double *e2)
{
    /* e1 perpendicular to n, e2 = n x e1, so that increasing angle is counter-clockwise about n */
    double a[3] = {0, 0, 0};
    int k = (fabs(n[0]) <= fabs(n[1]) && fabs(n[0]) <= fabs(n[2])) ? 0 : (fabs(n[1]) <= fabs(n[2]) ? 1 : 2);
    a[k] = 1.0;
    double c[3];
    cross3(n, a, c);
    double l = sqrt(dot3(c, c));
    for (int m = 0; m < 3; ++m) e1[m] = c[m] / l;
    cross3(n, e1, e2);
}

/* Sort pts (count m) counter-clockwise about n, drop exact duplicates; returns new count. */
static int order_ccw(angpt *pts, int m, const double *n)
{
    if (m == 0) return 0;
    double c[3] = {0, 0, 0}, e1[3], e2[3];
    for (int k = 0; k < m; ++k)
        for (int q = 0; q < 3; ++q) c[q] += pts[k].p[q] / m;
    plane_frame(n, e1, e2);
    for (int k = 0; k < m; ++k) {
        double d[3] = {pts[k].p[0] - c[0], pts[k].p[1] - c[1], pts[k].p[2] - c[2]};
        pts[k].ang = atan2(dot3(d, e2), dot3(d, e1));
    }
    qsort(pts, (size_t)m, sizeof(angpt), cmp_angpt);
    int w = 0;
    for (int k = 0; k < m; ++k) {
        if (w > 0 && memcmp(pts[w - 1].p, pts[k].p, sizeof(pts[k].p)) == 0) continue;
        pts[w++] = pts[k];
    }
    if (w > 1 && memcmp(pts[0].p, pts[w - 1].p, sizeof(pts[0].p)) == 0) w--;
    return w;
}

/* Point where the segment a-b meets plane (n,t); endpoints taken in a fixed
 * (lexicographic) order so that the two faces sharing an edge get the same bits. */
static void edge_cut(const double *a, const double *b, const oplane *pl, double *out)
{
    const double *A = a, *B = b;
    for (int k = 0; k < 3; ++k) {
        if (a[k] < b[k]) break;
        if (a[k] > b[k]) {
            A = b;
            B = a;
            break;
        }
    }
    double sA = dot3(pl->n, A) - pl->t, sB = dot3(pl->n, B) - pl->t;
    double s = sA / (sA - sB);
    for (int k = 0; k < 3; ++k) out[k] = A[k] + (B[k] - A[k]) * s;
}

/* Clip polytope P by half-space n.y <= t of plane index pidx (table pl). */
static void poly_clip(opoly *P, const oplane *pl, int pidx)
{
    const oplane *h = &pl[pidx];
    if (g_work) {
        long nv = 0;
        for (int k = 0; k < P->nf; ++k) nv += P->f[k].nv;
        g_work[W_TESTS] += nv / 3;
    }
    int cutcap = 64, ncut = 0;
    angpt *cut = (angpt *)malloc(sizeof(angpt) * (size_t)cutcap);
    int w = 0;
    for (int k = 0; k < P->nf; ++k) {
        oface *f = &P->f[k];
        oface g = {f->plane, 0, 0, NULL};
        for (int e = 0; e < f->nv; ++e) {
            const double *a = f->v + 3 * e;
            const double *b = f->v + 3 * ((e + 1) % f->nv);
            double sa = dot3(h->n, a) - h->t;
            double sb = dot3(h->n, b) - h->t;
            if (sa <= 0.0) face_push(&g, a);
            double ip[3];
            int has_cut = 0;
            if (sa == 0.0) {
                memcpy(ip, a, sizeof(ip));
                has_cut = 1;
            }
            if ((sa < 0.0 && sb > 0.0) || (sa > 0.0 && sb < 0.0)) {
                edge_cut(a, b, h, ip);
                face_push(&g, ip);
                has_cut = 1;
            }
            if (has_cut) {
                if (ncut == cutcap) {
                    cutcap *= 2;
                    cut = (angpt *)realloc(cut, sizeof(angpt) * (size_t)cutcap);
                }
                memcpy(cut[ncut++].p, ip, sizeof(ip));
            }
        }
        free(f->v);
        if (g.nv >= 3) {
            P->f[w++] = g;
        } else {
            free(g.v);
        }
    }
    P->nf = w;
    int m = order_ccw(cut, ncut, h->n);
    if (g_work && m >= 3) g_work[W_NEWV] += m;
    if (m >= 3) {
        oface *nf = poly_new_face(P, pidx);
        for (int k = 0; k < m; ++k) face_push(nf, cut[k].p);
    }
    free(cut);
}

/* --- restriction of one facet polygon to its disk: signed fan around q --- */
typedef struct {
    double area;  /* planar area of the restricted facet              */
    double omega; /* solid angle it subtends at p_i (sign of orientation only) */
    double m[3];  /* first moment of the restricted facet about its disk centre q */
} fanacc;

/* circular sector of the disk between in-plane directions u and v */
static void fan_sector(const double *u, const double *v, const double *n, double rho2, double h, double r, fanacc *acc)
{
    double c[3];
    cross3(u, v, c);
    double phi = atan2(dot3(n, c), dot3(u, v));
    acc->area += 0.5 * rho2 * phi;
    acc->omega += phi * (1.0 - h / r);
    /* first moment of the sector: with a the unit direction of u and b = n x a, the
       integral of (rho' cos s a + rho' sin s b) rho' drho' ds over [0, rho] x [0, phi] */
    double lu = sqrt(dot3(u, u));
    if (lu > 0.0) {
        double a[3] = {u[0] / lu, u[1] / lu, u[2] / lu}, b[3];
        cross3(n, a, b);
        double k = rho2 * sqrt(rho2) / 3.0, sp = sin(phi), cp = 1.0 - cos(phi);
        for (int j = 0; j < 3; ++j) acc->m[j] += k * (a[j] * sp + b[j] * cp);
    }
}

/* triangle (q, q+A, q+B) fully inside the disk */
static void fan_triangle(const double *A, const double *B, const double *n, double h, fanacc *acc)
{
    double c[3];
    cross3(A, B, c);
    double s = dot3(n, c);
    acc->area += 0.5 * s;
    /* first moment of the triangle (0, A, B): its signed area times its centroid (A + B) / 3 */
    for (int j = 0; j < 3; ++j) acc->m[j] += 0.5 * s * (A[j] + B[j]) / 3.0;
    double la = sqrt(dot3(A, A) + h * h), lb = sqrt(dot3(B, B) + h * h);
    /* Van Oosterom-Strackee solid angle of the triangle with apex at height h above q */
    acc->omega += 2.0 * atan2(s, la * lb + h * (la + lb) + h * h + dot3(A, B));
}

/* one fan piece: triangle (q, q+u, q+v) intersected with the disk of radius rho */
static void fan_piece(const double *u, const double *v, const double *n, double rho2, double h, double r, fanacc *acc)
{
    double w[3] = {v[0] - u[0], v[1] - u[1], v[2] - u[2]};
    double a = dot3(w, w);
    if (a == 0.0) return;
    double b = dot3(u, w);
    double c = dot3(u, u) - rho2;
    double disc = b * b - a * c;
    double lo = 1.0, hi = 0.0;
    if (disc > 0.0) {
        double sq = sqrt(disc);
        double s1 = (-b - sq) / a, s2 = (-b + sq) / a;
        lo = s1 > 0.0 ? s1 : 0.0;
        hi = s2 < 1.0 ? s2 : 1.0;
    }
    if (g_work) g_work[W_EDGES]++;
    if (!(lo < hi)) {
        fan_sector(u, v, n, rho2, h, r, acc);
        return;
    }
    if (g_work) g_work[W_CROSS]++;
    double A[3], B[3];
    for (int k = 0; k < 3; ++k) {
        A[k] = u[k] + lo * w[k];
        B[k] = u[k] + hi * w[k];
    }
    fan_sector(u, A, n, rho2, h, r, acc);
    fan_triangle(A, B, n, h, acc);
    fan_sector(B, v, n, rho2, h, r, acc);
}

static fanacc restrict_face(const oface *f, const oplane *pl, double r)
{
    fanacc acc = {0.0, 0.0, {0.0, 0.0, 0.0}};
    double t = pl->t, h = fabs(t);
    double rho2 = (r - t) * (r + t);
    if (!(rho2 > 0.0)) return acc;
    double q[3] = {t * pl->n[0], t * pl->n[1], t * pl->n[2]};
    for (int e = 0; e < f->nv; ++e) {
        const double *a = f->v + 3 * e;
        const double *b = f->v + 3 * ((e + 1) % f->nv);
        double u[3] = {a[0] - q[0], a[1] - q[1], a[2] - q[2]};
        double v[3] = {b[0] - q[0], b[1] - q[1], b[2] - q[2]};
        fan_piece(u, v, pl->n, rho2, h, r, &acc);
    }
    return acc;
}

/* auxiliary cube planes carry ids at or below this (never facets, never walls) */
#define AUX_ID (-1000000)

/* ---- section 3.3's own route to |K_i| (point_in, occluded patches, Gauss-Bonnet) ----
 *
 * The restricted cell is convex, so from a point c inside it every ray leaves through
 * exactly one boundary point: on the spherical part K_i, or on a restricted facet B_f.
 * The sphere is therefore tiled by K_i and the central projections from c of the B_f:
 * |K_i| = |Sigma_i| - sum_f |Proj(B_f, Sigma_i, c)|. Each projected facet is a region of
 * the sphere bounded by circle arcs (a straight boundary piece of B_f projects into the
 * circle cut from the sphere by the plane through c and the piece; a boundary arc of
 * B_f, on the facet's own circle, stays where it is); its area follows from
 * Gauss-Bonnet, |R| / r^2 = 2 pi - sum k_g len - sum turning angles, with the
 * geodesic curvature of a circle at distance e from the centre k_g = e / (r rho)
 * (reading of the printed formula, whose radicand is negative), signed positive when
 * the region is on the circle's smaller cap.
 */
typedef struct {
    int arc;         /* 0: straight piece A->B of an edge; 1: arc of the facet circle A->B (ccw about n) */
    int full;        /* the whole facet circle */
    double A[3], B[3];
} kpiece;

/* end points (parameters lo < hi on a + s (b - a)) of the part of edge ab in the ball |y| < r */
static int seg_in_ball(const double *a, const double *b, double r, double *lo, double *hi)
{
    double w[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double qa = dot3(w, w);
    if (!(qa > 0.0)) return 0;
    double qb = dot3(a, w), qc = dot3(a, a) - r * r;
    double disc = qb * qb - qa * qc;
    if (!(disc > 0.0)) return 0;
    double sq = sqrt(disc);
    double s1 = (-qb - sq) / qa, s2 = (-qb + sq) / qa;
    *lo = s1 > 0.0 ? s1 : 0.0;
    *hi = s2 < 1.0 ? s2 : 1.0;
    return *lo < *hi;
}

/* boundary of face f restricted to the ball, in order (counter-clockwise about n seen from
   outside); returns the piece count (0: the restricted facet is empty) */
static int restricted_boundary(const oface *f, const oplane *pl, double r, kpiece *out, int cap)
{
    double t = pl->t;
    if (!(fabs(t) < r)) return 0;
    int m = 0, first_entry = -1;
    for (int e = 0; e < f->nv; ++e) {
        const double *a = f->v + 3 * e, *b = f->v + 3 * ((e + 1) % f->nv);
        double lo, hi;
        if (!seg_in_ball(a, b, r, &lo, &hi)) continue;
        if (m + 2 > cap) return -1;
        kpiece sp;
        sp.arc = 0;
        sp.full = 0;
        for (int k = 0; k < 3; ++k) {
            sp.A[k] = a[k] + lo * (b[k] - a[k]);
            sp.B[k] = a[k] + hi * (b[k] - a[k]);
        }
        /* an entry point: the boundary came along the circle from the last exit */
        if (lo > 0.0 && m > 0) {
            kpiece ap = {1, 0, {0, 0, 0}, {0, 0, 0}};
            memcpy(ap.A, out[m - 1].B, sizeof(ap.A));
            memcpy(ap.B, sp.A, sizeof(ap.B));
            out[m++] = ap;
        }
        if (m == 0) first_entry = lo > 0.0;
        out[m++] = sp;
    }
    if (m == 0) {
        /* no edge meets the ball: the facet circle lies wholly inside or outside the polygon;
           inside iff its centre q = t n is on the inner side of every edge */
        double q[3] = {t * pl->n[0], t * pl->n[1], t * pl->n[2]};
        for (int e = 0; e < f->nv; ++e) {
            const double *a = f->v + 3 * e, *b = f->v + 3 * ((e + 1) % f->nv);
            double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, v[3] = {q[0] - a[0], q[1] - a[1], q[2] - a[2]}, c[3];
            cross3(u, v, c);
            if (dot3(c, pl->n) < 0.0) return 0;
        }
        kpiece fp = {1, 1, {0, 0, 0}, {0, 0, 0}};
        out[0] = fp;
        return 1;
    }
    /* closing arc from the last exit to the first entry */
    if (first_entry) {
        if (m + 1 > cap) return -1;
        kpiece ap = {1, 0, {0, 0, 0}, {0, 0, 0}};
        memcpy(ap.A, out[m - 1].B, sizeof(ap.A));
        memcpy(ap.B, out[0].A, sizeof(ap.B));
        out[m++] = ap;
    }
    return m;
}

/* point of the ray c + s (x - c), s > 0, on the sphere |y| = r (c inside the ball) */
static void project_from(const double *c, const double *x, double r, double *out)
{
    double e[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    double a = dot3(e, e), b = dot3(c, e), cc = dot3(c, c) - r * r;
    double s = (-b + sqrt(b * b - a * cc)) / a;
    for (int k = 0; k < 3; ++k) out[k] = c[k] + s * e[k];
}

/* positive angle in [0, 2 pi) from x to y about the unit axis u (x, y taken about the
   circle centre o) */
static double angle_about(const double *x, const double *y, const double *o, const double *u)
{
    double a[3] = {x[0] - o[0], x[1] - o[1], x[2] - o[2]}, b[3] = {y[0] - o[0], y[1] - o[1], y[2] - o[2]}, c[3];
    cross3(a, b, c);
    double th = atan2(dot3(c, u), dot3(a, b));
    return th < 0.0 ? th + 2.0 * OR_PI : th;
}

/* unit tangent at the sphere point x of a circle traversed positively about the axis u */
static void tangent_about(const double *u, const double *x, double *T)
{
    cross3(u, x, T);
    double l = sqrt(dot3(T, T));
    for (int k = 0; k < 3; ++k) T[k] /= l;
}

/* area of the projection from c of one restricted facet (pieces kp[0..m)) */
static double projected_patch(const kpiece *kp, int m, const oplane *pl, const double *c, double r)
{
    if (m == 1 && kp[0].full) {
        /* the cap beyond the facet plane: 2 pi r (r - t) */
        return 2.0 * OR_PI * r * (r - pl->t);
    }
    double kl = 0.0, turn = 0.0;
    double T0[3] = {0.0, 0.0, 0.0}, Tprev[3] = {0.0, 0.0, 0.0}, Pfirst[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < m; ++k) {
        const kpiece *q = &kp[k];
        double Ps[3], Pe[3], u[3], e, Ts[3], Te[3];
        if (q->arc) {
            memcpy(Ps, q->A, sizeof(Ps));
            memcpy(Pe, q->B, sizeof(Pe));
            memcpy(u, pl->n, sizeof(u));
            e = pl->t;
        } else {
            project_from(c, q->A, r, Ps);
            project_from(c, q->B, r, Pe);
            double a[3] = {q->A[0] - c[0], q->A[1] - c[1], q->A[2] - c[2]};
            double b[3] = {q->B[0] - c[0], q->B[1] - c[1], q->B[2] - c[2]};
            cross3(a, b, u);
            double l = sqrt(dot3(u, u));
            for (int j = 0; j < 3; ++j) u[j] /= l;
            e = dot3(c, u);
        }
        double o[3] = {e * u[0], e * u[1], e * u[2]};
        kl += e * angle_about(Ps, Pe, o, u) / r;
        tangent_about(u, Ps, Ts);
        tangent_about(u, Pe, Te);
        if (k == 0) {
            memcpy(T0, Ts, sizeof(T0));
            memcpy(Pfirst, Ps, sizeof(Pfirst));
        } else {
            double x[3];
            cross3(Tprev, Ts, x);
            turn += atan2(dot3(x, Ps) / r, dot3(Tprev, Ts));
        }
        memcpy(Tprev, Te, sizeof(Tprev));
    }
    double x[3];
    cross3(Tprev, T0, x);
    turn += atan2(dot3(x, Pfirst) / r, dot3(Tprev, T0));
    return r * r * (2.0 * OR_PI - kl - turn);
}

/* K_i by the route above, with c = point_in(C_i): from the area centroid of each
   restricted facet a ray along -n_f to the first of the sphere and the other planes;
   c = the mean of the chords' midpoints. Returns K; c (local coordinates) in cin. */
static double paper_k(const opoly *P, const oplane *pl, int nreal, double r, int inside, double *cin)
{
    int cap = 8, nb = 0;
    kpiece *kp = NULL;
    int *start = (int *)malloc(sizeof(int) * (size_t)(P->nf + 1));
    int *face = (int *)malloc(sizeof(int) * (size_t)(P->nf + 1));
    start[0] = 0;
    int total = 0;
    for (int k = 0; k < P->nf; ++k) {
        const oface *f = &P->f[k];
        const oplane *p = &pl[f->plane];
        if (p->id <= AUX_ID) continue;
        int m;
        for (;;) {
            kp = (kpiece *)realloc(kp, sizeof(kpiece) * (size_t)(total + cap));
            m = restricted_boundary(f, p, r, kp + total, cap);
            if (m >= 0) break;
            cap *= 2;
        }
        if (m == 0) continue;
        face[nb] = k;
        total += m;
        start[++nb] = total;
    }
    cin[0] = cin[1] = cin[2] = 0.0;
    double K;
    if (nb == 0) {
        K = 4.0 * OR_PI * r * r * inside;
    } else {
        for (int b = 0; b < nb; ++b) {
            const oplane *p = &pl[P->f[face[b]].plane];
            /* the restricted facet's area centroid q + m / area (a point of its relative
               interior, so the ray below has a chord of positive length) */
            fanacc a = restrict_face(&P->f[face[b]], p, r);
            double g[3];
            for (int j = 0; j < 3; ++j) g[j] = p->t * p->n[j] + (a.area > 0.0 ? a.m[j] / a.area : 0.0);
            double d[3] = {-p->n[0], -p->n[1], -p->n[2]};
            double gd = dot3(g, d);
            double lam = -gd + sqrt(gd * gd - (dot3(g, g) - r * r));
            for (int k = 0; k < nreal; ++k) {
                if (&pl[k] == p) continue;
                double den = dot3(pl[k].n, d);
                if (den > 0.0) {
                    double l = (pl[k].t - dot3(pl[k].n, g)) / den;
                    if (l < lam) lam = l;
                }
            }
            if (lam < 0.0) lam = 0.0;
            for (int j = 0; j < 3; ++j) cin[j] += g[j] + 0.5 * lam * d[j];
        }
        for (int j = 0; j < 3; ++j) cin[j] /= nb;
        double occluded = 0.0;
        for (int b = 0; b < nb; ++b)
            occluded += projected_patch(kp + start[b], start[b + 1] - start[b], &pl[P->f[face[b]].plane], cin, r);
        K = 4.0 * OR_PI * r * r - occluded;
    }
    free(kp);
    free(start);
    free(face);
    return K;
}

static int cmp_plane_t(const void *a, const void *b)
{
    const oplane *u = (const oplane *)a, *v = (const oplane *)b;
    if (u->t < v->t) return -1;
    if (u->t > v->t) return 1;
    return (u->id < v->id) ? -1 : (u->id > v->id);
}

/*
 * Evaluate one cell. Outputs: V, K, the 6 wall areas, up to fcap neighbour
 * facets (id, area) with area > 0, the facet count (may exceed fcap -> status
 * OR_FACET_CAP), and the number of planes that cut the ball (ncand).
 */

static int oracle_cell(long i, long n, const double *x, const double *y, const double *z, const double *psi,
                       const double *box, const double *dom, int ndom, double *V, double *K, double *wall, long *fj,
                       double *fA, int fcap, int *fcount, int *ncand, double *cen, double *Kp, double *cin)
{
    const int nwall = ndom > 0 ? ndom : 6;
    *V = 0.0;
    *K = 0.0;
    cen[0] = x[i];
    cen[1] = y[i];
    cen[2] = z[i];
    if (Kp) {
        *Kp = 0.0;
        cin[0] = x[i];
        cin[1] = y[i];
        cin[2] = z[i];
    }
    for (int k = 0; k < nwall; ++k) wall[k] = 0.0;
    *fcount = 0;
    *ncand = 0;
    if (!(psi[i] > 0.0)) return OR_EMPTY;
    const double r = sqrt(psi[i]);
    const double pi3[3] = {x[i], y[i], z[i]};

    int pcap = 64, np = 0;
    oplane *pl = (oplane *)malloc(sizeof(oplane) * (size_t)pcap);
    for (long j = 0; j < n; ++j) {
        if (j == i) continue;
        double d3[3] = {x[j] - pi3[0], y[j] - pi3[1], z[j] - pi3[2]};
        double d2 = dot3(d3, d3);
        if (d2 == 0.0) {
            /* coincident sites: the one with the larger weight (then lower index) owns everything */
            if (psi[j] > psi[i] || (psi[j] == psi[i] && j < i)) {
                free(pl);
                return OR_EMPTY;
            }
            continue;
        }
        double d = sqrt(d2);
        double t = (d2 + psi[i] - psi[j]) / (2.0 * d);
        if (t <= -r) {
            free(pl);
            return OR_EMPTY;
        }
        if (t < r) {
            if (np == pcap) {
                pcap *= 2;
                pl = (oplane *)realloc(pl, sizeof(oplane) * (size_t)pcap);
            }
            oplane *p = &pl[np++];
            p->n[0] = d3[0] / d;
            p->n[1] = d3[1] / d;
            p->n[2] = d3[2] / d;
            p->t = t;
            p->id = j;
        }
    }
    *ncand = np;
    if (g_work) g_work[W_CAND] = np;
    /* walls: the box -x,+x,-y,+y,-z,+z, or the planes n.x <= c of a convex polyhedral
       domain (unit outward normals; the paper evaluates cells in polyhedral domains, section
       6, and a convex one is an intersection of half-spaces); t is the distance of p_i to
       the wall */
    for (int w = 0; w < nwall; ++w) {
        double nw[3] = {0.0, 0.0, 0.0}, t;
        if (ndom > 0) {
            const double *q = dom + 4 * w;
            nw[0] = q[0];
            nw[1] = q[1];
            nw[2] = q[2];
            t = q[3] - dot3(nw, pi3);
        } else {
            int ax = w / 2;
            nw[ax] = (w % 2 == 0) ? -1.0 : 1.0;
            t = (w % 2 == 0) ? pi3[ax] - box[ax] : box[3 + ax] - pi3[ax];
        }
        if (t < r) {
            if (np + 1 > pcap) {
                pcap *= 2;
                pl = (oplane *)realloc(pl, sizeof(oplane) * (size_t)pcap);
            }
            oplane *p = &pl[np++];
            p->n[0] = nw[0];
            p->n[1] = nw[1];
            p->n[2] = nw[2];
            p->t = t;
            p->id = -1 - w;
        }
    }
    qsort(pl, (size_t)np, sizeof(oplane), cmp_plane_t);
    int inside = 1;
    for (int k = 0; k < np; ++k)
        if (pl[k].t < 0.0) inside = 0;

    /* auxiliary cube p_i +- 2r (never a facet: it lies outside the ball) */
    const int nreal = np;
    pl = (oplane *)realloc(pl, sizeof(oplane) * (size_t)(np + 6));
    opoly P = {0, 0, NULL};
    const double L = 2.0 * r;
    for (int w = 0; w < 6; ++w) {
        int ax = w / 2;
        double sgn = (w % 2 == 0) ? -1.0 : 1.0;
        oplane *p = &pl[np + w];
        p->n[0] = p->n[1] = p->n[2] = 0.0;
        p->n[ax] = sgn;
        p->t = L;
        p->id = AUX_ID - w;
        angpt c4[4];
        int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3, m = 0;
        for (int s1 = -1; s1 <= 1; s1 += 2)
            for (int s2 = -1; s2 <= 1; s2 += 2) {
                c4[m].p[ax] = sgn * L;
                c4[m].p[a1] = s1 * L;
                c4[m].p[a2] = s2 * L;
                m++;
            }
        m = order_ccw(c4, 4, p->n);
        oface *f = poly_new_face(&P, np + w);
        for (int k = 0; k < m; ++k) face_push(f, c4[k].p);
    }
    for (int k = 0; k < nreal; ++k) {
        poly_clip(&P, pl, k);
        if (P.nf == 0) break;
    }

    /* First moment about p_i (the centroid the pressure model of section 5 uses), by the
       divergence theorem applied to the fields x_k x (divergence 4 x_k):
       4 * integral of x dV = surface integral of x (x.n) dA. On a facet x.n = t and the
       facet's moment is q area + m (q = t n); on the sphere x.n = r and x = r n, whose
       area integral is -sum_f n_f area_f (a closed surface has zero vector area). */
    double sumTA = 0.0, sumOm = 0.0, mom[3] = {0.0, 0.0, 0.0};
    int nf = 0;
    for (int k = 0; k < P.nf; ++k) {
        const oface *f = &P.f[k];
        const oplane *p = &pl[f->plane];
        if (p->id <= AUX_ID) continue;
        if (g_work) g_work[W_FACES]++;
        fanacc a = restrict_face(f, p, r);
        sumTA += p->t * a.area;
        sumOm += (p->t >= 0.0 ? 1.0 : -1.0) * a.omega;
        for (int j = 0; j < 3; ++j)
            mom[j] += p->t * (p->t * p->n[j] * a.area + a.m[j]) - r * r * p->n[j] * a.area;
        if (p->id < 0) {
            wall[-1 - p->id] = a.area;
        } else if (a.area > 0.0) {
            if (nf < fcap) {
                fj[nf] = p->id;
                fA[nf] = a.area;
            }
            nf++;
        }
    }
    if (Kp) {
        double cl[3];
        *Kp = paper_k(&P, pl, nreal, r, inside, cl);
        for (int j = 0; j < 3; ++j) cin[j] = pi3[j] + cl[j];
    }
    poly_free(&P);
    free(pl);
    if (P.nf == 0 && !inside) {
        /* the half-spaces alone are empty inside the cube: no volume, no surface */
    }
    *K = r * r * (4.0 * OR_PI * inside - sumOm);
    *V = (sumTA + r * (*K)) / 3.0;
    if (*V > 0.0) {
        cen[0] = pi3[0] + 0.25 * mom[0] / *V;
        cen[1] = pi3[1] + 0.25 * mom[1] / *V;
        cen[2] = pi3[2] + 0.25 * mom[2] / *V;
    }
    *fcount = nf;
    return nf > fcap ? OR_FACET_CAP : OR_OK;
}

/*
 * Evaluate m cells (indices idx[0..m), or all n cells when idx == NULL), in the box or,
 * when ndom > 0, in the convex domain {x : n_w.x <= c_w} given as dom[4w..4w+4) =
 * (n_w, c_w) with unit outward normals (the box is then not used).
 * Per evaluated cell c: V[c], K[c], wall[W c..W c+W) with W = 6 or ndom, facets fj/fA[c*fcap ..],
 * fcount[c], ncand[c], status[c], the centroid cen[3c..3c+3) (the site itself for an
 * empty cell), and when work != NULL the six work units of each cell at
 * work[6c..6c+6). With Kp != NULL also |K| by section 3.3's own route (point_in and the
 * projected facets, paper_k above) at Kp[c] and its interior point at cin[3c..3c+3).
 * OpenMP over cells.
 */
int oracle_cells(long n, const double *x, const double *y, const double *z, const double *psi,
                 const double *box, const long *idx, long m, double *V, double *K, double *wall, long *fj,
                 double *fA, int fcap, int *fcount, int *ncand, int *status, int nthreads, long *work, double *cen,
                 const double *dom, int ndom, double *Kp, double *cin)
{
    long cnt = idx ? m : n;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (long c = 0; c < cnt; ++c) {
        long i = idx ? idx[c] : c;
        g_work = work ? &work[W_N * c] : NULL;
        if (g_work)
            for (int k = 0; k < W_N; ++k) g_work[k] = 0;
        const int nwall = ndom > 0 ? ndom : 6;
        status[c] = oracle_cell(i, n, x, y, z, psi, box, dom, ndom, &V[c], &K[c], &wall[(size_t)nwall * c],
                                &fj[(size_t)c * fcap], &fA[(size_t)c * fcap], fcap, &fcount[c], &ncand[c],
                                &cen[3 * c], Kp ? &Kp[c] : NULL, cin ? &cin[3 * c] : NULL);
    }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
