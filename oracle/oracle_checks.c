/*
 * oracle_checks.c -- penetration and separation checks used by the tests.
 *
 * TEST INFRASTRUCTURE ONLY (see ccfr_oracle.h).  Deliberately independent of
 * the candidate, closest-point, region and projection code: its own distance
 * routines (by exhaustive characterisation of the minimiser, not the Voronoi
 * walk) and its own sweep-and-prune along x instead of all-pairs loops.
 *
 *  - Interpenetration (Sec. 4.3, the paper's zero remaining violations): an edge
 *    of one triangle passing through another triangle that shares no vertex with
 *    it, decided with FP64 orientation determinants.
 *  - Separation: the minimum distance over non-adjacent vertex-triangle,
 *    edge-edge and free-particle pairs; the method keeps it at least xi.
 */
#include "ccfr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static double d3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* squared distance from p to segment ab */
static double pt_seg2(const double* p, const double* a, const double* b) {
    double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    double L = d3(ab, ab);
    double t = L > 0 ? d3(ap, ab) / L : 0.0;
    t = t < 0 ? 0 : (t > 1 ? 1 : t);
    double q[3] = {a[0] + t * ab[0] - p[0], a[1] + t * ab[1] - p[1], a[2] + t * ab[2] - p[2]};
    return d3(q, q);
}

/* squared distance from p to triangle abc: foot of the perpendicular if it lies
 * inside (barycentrics from the 2x2 normal equations), else the nearest edge */
static double pt_tri2(const double* p, const double* a, const double* b, const double* c) {
    double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double ac[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    double g11 = d3(ab, ab), g12 = d3(ab, ac), g22 = d3(ac, ac);
    double r1 = d3(ab, ap), r2 = d3(ac, ap);
    double det = g11 * g22 - g12 * g12;
    double best = pt_seg2(p, a, b);
    double e2 = pt_seg2(p, b, c), e3 = pt_seg2(p, c, a);
    if (e2 < best) best = e2;
    if (e3 < best) best = e3;
    if (det > 1e-14 * g11 * g22) {
        double u = (g22 * r1 - g12 * r2) / det;
        double v = (g11 * r2 - g12 * r1) / det;
        if (u >= 0 && v >= 0 && u + v <= 1) {
            double f[3] = {a[0] + u * ab[0] + v * ac[0] - p[0], a[1] + u * ab[1] + v * ac[1] - p[1],
                           a[2] + u * ab[2] + v * ac[2] - p[2]};
            double df = d3(f, f);
            if (df < best) best = df;
        }
    }
    return best;
}

/* squared distance between segments ab and cd: interior critical point if it
 * lies in (0,1)^2, and the four endpoint-to-segment distances */
static double seg_seg2(const double* a, const double* b, const double* c, const double* d) {
    double best = pt_seg2(a, c, d);
    double t = pt_seg2(b, c, d);
    if (t < best) best = t;
    t = pt_seg2(c, a, b);
    if (t < best) best = t;
    t = pt_seg2(d, a, b);
    if (t < best) best = t;
    double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double v[3] = {d[0] - c[0], d[1] - c[1], d[2] - c[2]};
    double w[3] = {a[0] - c[0], a[1] - c[1], a[2] - c[2]};
    double uu = d3(u, u), uv = d3(u, v), vv = d3(v, v), uw = d3(u, w), vw = d3(v, w);
    double det = uu * vv - uv * uv;
    if (det > 1e-14 * uu * vv) {
        double s = (uv * vw - vv * uw) / det;
        double r = (uu * vw - uv * uw) / det;
        if (s > 0 && s < 1 && r > 0 && r < 1) {
            double q[3] = {w[0] + s * u[0] - r * v[0], w[1] + s * u[1] - r * v[1], w[2] + s * u[2] - r * v[2]};
            double dq = d3(q, q);
            if (dq < best) best = dq;
        }
    }
    return best;
}

/* ---- exact orientation predicates ----
 *
 * The sign of a 3x3 (2x2) orientation determinant decides the intersection
 * tests below, so it is computed exactly: a floating-point evaluation with a
 * static error bound first, and where that bound cannot certify the sign, an
 * exact evaluation in floating-point expansion arithmetic.  Both are the
 * published method of J. R. Shewchuk, "Adaptive Precision Floating-Point
 * Arithmetic and Fast Robust Geometric Predicates" (Discrete Comput. Geom. 18,
 * 1997): exact sums (Two-Sum), exact products (here through a fused
 * multiply-add), nonoverlapping expansions grown one component at a time
 * (Grow-Expansion), and the first error bound of his orient3d.  The exact
 * stage here does not use his adaptive intermediate stages: it expands the
 * 4x4 (3x3) determinant with a column of ones into its 24 (6) signed products
 * of coordinates, each of which is an exact expansion of four (two) doubles,
 * and sums them exactly.  Inputs are assumed free of overflow and of underflow
 * in the products (coordinates of metres, far from both limits). */

static void two_sum(double a, double b, double* x, double* y) {
    double s = a + b;
    double bv = s - a;
    double av = s - bv;
    *x = s;
    *y = (a - av) + (b - bv);
}

static void two_prod(double a, double b, double* x, double* y) {
    double p = a * b;
    *x = p;
    *y = fma(a, b, -p);
}

/* h = e + b for a nonoverlapping expansion e[0..m) in increasing magnitude;
 * h has m + 1 components and is nonoverlapping too. */
static int grow(const double* e, int m, double b, double* h) {
    double q = b;
    for (int i = 0; i < m; ++i) {
        double qn, hi;
        two_sum(q, e[i], &qn, &hi);
        h[i] = hi;
        q = qn;
    }
    h[m] = q;
    return m + 1;
}

/* sign of a nonoverlapping expansion: that of its largest nonzero component */
static int expansion_sign(const double* e, int m) {
    for (int i = m - 1; i >= 0; --i)
        if (e[i] != 0.0) return e[i] > 0.0 ? 1 : -1;
    return 0;
}

/* exact sign of det [[p_i, 1]] for k + 1 points p_i of dimension k (k = 2, 3) */
static int det_ones_sign(const double* const* p, int k) {
    static const int perm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const int par3[6] = {0, 1, 1, 0, 0, 1};
    double acc[2][100];
    int cur = 0, m = 0;
    /* det = sum over the row o holding the 1 and the bijection of the other
     * rows onto the coordinate columns; the permutation's sign is the parity of
     * the column order times (-1)^(o + k) */
    for (int o = 0; o <= k; ++o) {
        int rows[3], nr = 0;
        for (int i = 0; i <= k; ++i)
            if (i != o) rows[nr++] = i;
        const int sign_o = ((o + k) & 1) ? -1 : 1;
        if (k == 2) {
            for (int q = 0; q < 2; ++q) {
                int c0 = q, c1 = 1 - q;
                int sg = sign_o * (q ? -1 : 1);
                double hi, lo;
                two_prod(p[rows[0]][c0], p[rows[1]][c1], &hi, &lo);
                double t[2] = {sg * lo, sg * hi};
                for (int j = 0; j < 2; ++j) {
                    m = grow(acc[cur], m, t[j], acc[1 - cur]);
                    cur = 1 - cur;
                }
            }
        } else {
            for (int q = 0; q < 6; ++q) {
                int sg = sign_o * (par3[q] ? -1 : 1);
                double a = p[rows[0]][perm3[q][0]], b = p[rows[1]][perm3[q][1]], c = p[rows[2]][perm3[q][2]];
                double h, l, h1, l1, h2, l2;
                two_prod(a, b, &h, &l);      /* a b = h + l exactly         */
                two_prod(h, c, &h1, &l1);    /* h c = h1 + l1               */
                two_prod(l, c, &h2, &l2);    /* l c = h2 + l2               */
                double t[4] = {sg * l2, sg * l1, sg * h2, sg * h1};
                for (int j = 0; j < 4; ++j) {
                    m = grow(acc[cur], m, t[j], acc[1 - cur]);
                    cur = 1 - cur;
                }
            }
        }
    }
    return expansion_sign(acc[cur], m);
}

/* sign of (b - a) . ((c - a) x (d - a)): positive when d lies on the side of
 * plane abc that the right-hand normal (b - a) x (c - a) points to */
int orc_orient3d_sign(const double* a, const double* b, const double* c, const double* d) {
    const double eps = ldexp(1.0, -53);
    const double errA = (7.0 + 56.0 * eps) * eps;
    /* Shewchuk's orient3d first stage, in his form with d as the origin */
    double adx = a[0] - d[0], bdx = b[0] - d[0], cdx = c[0] - d[0];
    double ady = a[1] - d[1], bdy = b[1] - d[1], cdy = c[1] - d[1];
    double adz = a[2] - d[2], bdz = b[2] - d[2], cdz = c[2] - d[2];
    double bdxcdy = bdx * cdy, cdxbdy = cdx * bdy;
    double cdxady = cdx * ady, adxcdy = adx * cdy;
    double adxbdy = adx * bdy, bdxady = bdx * ady;
    double det = adz * (bdxcdy - cdxbdy) + bdz * (cdxady - adxcdy) + cdz * (adxbdy - bdxady);
    double perm = (fabs(bdxcdy) + fabs(cdxbdy)) * fabs(adz) + (fabs(cdxady) + fabs(adxcdy)) * fabs(bdz) +
                  (fabs(adxbdy) + fabs(bdxady)) * fabs(cdz);
    /* det here is det[a-d; b-d; c-d] = det[[a,1];[b,1];[c,1];[d,1]], which is
     * minus the triple product (b - a) . ((c - a) x (d - a)) */
    if (det > errA * perm) return -1;
    if (-det > errA * perm) return 1;
    const double* pts[4] = {a, b, c, d};
    return -det_ones_sign(pts, 3);
}

/* sign of the 2-D cross product (b - a) x (c - a) of 2-vectors, exact */
int orc_orient2d_sign(const double* a, const double* b, const double* c) {
    const double* pts[3] = {a, b, c};
    return det_ones_sign(pts, 2);
}

/* closed segments pq and rs in the plane meet (exact) */
static int seg_seg_2d(const double* p, const double* q, const double* r, const double* s) {
    int d1 = orc_orient2d_sign(r, s, p), d2 = orc_orient2d_sign(r, s, q);
    int d3 = orc_orient2d_sign(p, q, r), d4 = orc_orient2d_sign(p, q, s);
    if (d1 * d2 < 0 && d3 * d4 < 0) return 1;
#define ON_SEG(u, v, w) (fmin(u[0], v[0]) <= w[0] && w[0] <= fmax(u[0], v[0]) && \
                         fmin(u[1], v[1]) <= w[1] && w[1] <= fmax(u[1], v[1]))
    if (d1 == 0 && ON_SEG(r, s, p)) return 1;
    if (d2 == 0 && ON_SEG(r, s, q)) return 1;
    if (d3 == 0 && ON_SEG(p, q, r)) return 1;
    if (d4 == 0 && ON_SEG(p, q, s)) return 1;
#undef ON_SEG
    return 0;
}

/* closed triangle abc (non-degenerate) contains p, in the plane (exact) */
static int tri_has_2d(const double* a, const double* b, const double* c, const double* p) {
    int s1 = orc_orient2d_sign(a, b, p), s2 = orc_orient2d_sign(b, c, p), s3 = orc_orient2d_sign(c, a, p);
    return (s1 >= 0 && s2 >= 0 && s3 >= 0) || (s1 <= 0 && s2 <= 0 && s3 <= 0);
}

/* A segment lying in the plane of triangle abc: drop one coordinate axis along
 * which the projected triangle keeps a non-zero area (incidence is preserved by
 * such a projection) and test in 2-D.  A triangle of zero area is skipped. */
static int coplanar_hit(const double* p0, const double* p1, const double* a, const double* b, const double* c) {
    for (int drop = 2; drop >= 0; --drop) {
        const int i = drop == 0 ? 1 : 0, j = drop == 2 ? 1 : 2;
        double A[2] = {a[i], a[j]}, B[2] = {b[i], b[j]}, Cc[2] = {c[i], c[j]};
        double P[2] = {p0[i], p0[j]}, Q[2] = {p1[i], p1[j]};
        if (orc_orient2d_sign(A, B, Cc) == 0) continue;
        if (tri_has_2d(A, B, Cc, P) || tri_has_2d(A, B, Cc, Q)) return 1;
        return seg_seg_2d(P, Q, A, B) || seg_seg_2d(P, Q, B, Cc) || seg_seg_2d(P, Q, Cc, A);
    }
    return 0;
}

/* the closed segment p0 p1 meets the closed triangle abc */
static int seg_hits_tri(const double* p0, const double* p1, const double* a, const double* b, const double* c) {
    int o0 = orc_orient3d_sign(a, b, c, p0), o1 = orc_orient3d_sign(a, b, c, p1);
    if (o0 * o1 > 0) return 0;
    if (o0 == 0 && o1 == 0) return coplanar_hit(p0, p1, a, b, c);
    /* the line p0 p1 crosses the plane inside the closed segment; it passes
     * through the triangle iff it sees the three edges with one orientation */
    int s1 = orc_orient3d_sign(p0, p1, a, b), s2 = orc_orient3d_sign(p0, p1, b, c),
        s3 = orc_orient3d_sign(p0, p1, c, a);
    return (s1 >= 0 && s2 >= 0 && s3 >= 0) || (s1 <= 0 && s2 <= 0 && s3 <= 0);
}

typedef struct { double lo[3], hi[3]; int32_t kind, id; int32_t stat, pad_; } item_t;

static int cmp_lo(const void* a, const void* b) {
    double x = ((const item_t*)a)->lo[0], y = ((const item_t*)b)->lo[0];
    return x < y ? -1 : (x > y ? 1 : 0);
}

static item_t make_item(const double* x, const int32_t* vids, int nv, double grow, int kind, int id) {
    item_t it;
    for (int k = 0; k < 3; ++k) {
        double mn = x[3 * vids[0] + k], mx = mn;
        for (int i = 1; i < nv; ++i) {
            double c = x[3 * vids[i] + k];
            mn = c < mn ? c : mn;
            mx = c > mx ? c : mx;
        }
        it.lo[k] = mn - grow;
        it.hi[k] = mx + grow;
    }
    it.kind = kind;
    it.id = id;
    it.stat = 0;
    it.pad_ = 0;
    return it;
}

int64_t orc_count_edge_tri_intersections(int32_t n_verts, const double* x, int32_t n_tris,
                                         const int32_t* tris, int32_t n_edges,
                                         const int32_t* edges) {
    (void)n_verts;
    int64_t n = (int64_t)n_tris + n_edges;
    item_t* it = (item_t*)malloc(sizeof(item_t) * (size_t)(n + 1));
    for (int32_t t = 0; t < n_tris; ++t) it[t] = make_item(x, tris + 3 * t, 3, 0.0, 0, t);
    for (int32_t e = 0; e < n_edges; ++e) it[n_tris + e] = make_item(x, edges + 2 * e, 2, 0.0, 1, e);
    qsort(it, (size_t)n, sizeof(item_t), cmp_lo);
    int64_t hits = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : hits)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n && it[j].lo[0] <= it[i].hi[0]; ++j) {
            if (it[i].kind == it[j].kind) continue;
            if (it[j].lo[1] > it[i].hi[1] || it[i].lo[1] > it[j].hi[1]) continue;
            if (it[j].lo[2] > it[i].hi[2] || it[i].lo[2] > it[j].hi[2]) continue;
            const item_t* T = it[i].kind == 0 ? &it[i] : &it[j];
            const item_t* E = it[i].kind == 0 ? &it[j] : &it[i];
            const int32_t* tv = tris + 3 * T->id;
            const int32_t* ev = edges + 2 * E->id;
            int share = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 2; ++b) share |= (tv[a] == ev[b]);
            if (share) continue;
            hits += seg_hits_tri(x + 3 * ev[0], x + 3 * ev[1], x + 3 * tv[0], x + 3 * tv[1], x + 3 * tv[2]);
        }
    }
    free(it);
    return hits;
}

double orc_min_separation(int32_t n_verts, const double* x, const double* inv_mass, int32_t n_tris,
                          const int32_t* tris, int32_t n_edges, const int32_t* edges, double reach,
                          double below, int64_t out_counts[4]) {
    unsigned char* fr = (unsigned char*)malloc((size_t)n_verts + 1);
    memset(fr, 1, (size_t)n_verts);
    for (int32_t t = 0; t < 3 * n_tris; ++t) fr[tris[t]] = 0;
    for (int32_t e = 0; e < 2 * n_edges; ++e) fr[edges[e]] = 0;
    int64_t n = (int64_t)n_verts + n_tris + n_edges;
    item_t* it = (item_t*)malloc(sizeof(item_t) * (size_t)(n + 1));
    const double g = 0.5 * reach;
    for (int32_t v = 0; v < n_verts; ++v) it[v] = make_item(x, &v, 1, g, 0, v);
    for (int32_t t = 0; t < n_tris; ++t) it[n_verts + t] = make_item(x, tris + 3 * t, 3, g, 1, t);
    for (int32_t e = 0; e < n_edges; ++e) it[n_verts + n_tris + e] = make_item(x, edges + 2 * e, 2, g, 2, e);
    /* stat: every vertex of the item has zero inverse mass (two such items
     * never move relative to each other); set before the sort reorders items */
    for (int64_t k = 0; k < n; ++k) {
        const int32_t* vs = it[k].kind == 0 ? &it[k].id : (it[k].kind == 1 ? tris + 3 * it[k].id : edges + 2 * it[k].id);
        int nv = it[k].kind == 0 ? 1 : (it[k].kind == 1 ? 3 : 2);
        int s = 1;
        for (int q = 0; q < nv; ++q) s &= (inv_mass == NULL ? 0 : inv_mass[vs[q]] == 0.0);
        it[k].stat = s;
    }
    qsort(it, (size_t)n, sizeof(item_t), cmp_lo);
    double best2 = reach * reach;
    int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    const double below2 = below * below;
#pragma omp parallel for schedule(dynamic, 256) reduction(min : best2) reduction(+ : c0, c1, c2, c3)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n && it[j].lo[0] <= it[i].hi[0]; ++j) {
            if (it[j].lo[1] > it[i].hi[1] || it[i].lo[1] > it[j].hi[1]) continue;
            if (it[j].lo[2] > it[i].hi[2] || it[i].lo[2] > it[j].hi[2]) continue;
            if (it[i].stat && it[j].stat) continue;
            int ki = it[i].kind, kj = it[j].kind;
            double dist2 = -1.0;
            int kind = -1;
            if ((ki == 0 && kj == 1) || (ki == 1 && kj == 0)) {          /* vertex - triangle */
                int32_t v = ki == 0 ? it[i].id : it[j].id;
                int32_t t = ki == 1 ? it[i].id : it[j].id;
                const int32_t* tv = tris + 3 * t;
                if (tv[0] == v || tv[1] == v || tv[2] == v) continue;
                dist2 = pt_tri2(x + 3 * v, x + 3 * tv[0], x + 3 * tv[1], x + 3 * tv[2]);
                kind = 0;
            } else if (ki == 2 && kj == 2) {                              /* edge - edge */
                const int32_t* a = edges + 2 * it[i].id;
                const int32_t* b = edges + 2 * it[j].id;
                if (a[0] == b[0] || a[0] == b[1] || a[1] == b[0] || a[1] == b[1]) continue;
                dist2 = seg_seg2(x + 3 * a[0], x + 3 * a[1], x + 3 * b[0], x + 3 * b[1]);
                kind = 1;
            } else if (ki == 0 && kj == 0) {                              /* particle - particle */
                int32_t a = it[i].id, b = it[j].id;
                if (!fr[a] || !fr[b]) continue;
                double dv[3] = {x[3 * a] - x[3 * b], x[3 * a + 1] - x[3 * b + 1], x[3 * a + 2] - x[3 * b + 2]};
                dist2 = d3(dv, dv);
                kind = 2;
            } else if ((ki == 0 && kj == 2) || (ki == 2 && kj == 0)) {    /* particle - edge */
                int32_t p = ki == 0 ? it[i].id : it[j].id;
                const int32_t* e = edges + 2 * (ki == 2 ? it[i].id : it[j].id);
                if (!fr[p]) continue;
                dist2 = pt_seg2(x + 3 * p, x + 3 * e[0], x + 3 * e[1]);
                kind = 3;
            } else {
                continue;
            }
            if (dist2 < best2) best2 = dist2;
            if (dist2 < below2) {
                if (kind == 0) c0++;
                else if (kind == 1) c1++;
                else if (kind == 2) c2++;
                else c3++;
            }
        }
    }
    if (out_counts) { out_counts[0] = c0; out_counts[1] = c1; out_counts[2] = c2; out_counts[3] = c3; }
    free(it);
    free(fr);
    return sqrt(best2);
}

/* Certified sampled check of a straight-line motion x(t) = (1 - t) x0 + t x1,
 * t in [0, 1] (one solver iteration moves every vertex along such a line: the
 * anchor update of Alg. 4).  The distance between a vertex and a triangle, two
 * edges, two particles or a particle and an edge whose vertices move
 * linearly changes with t at a rate of at most L = 2 max_v |x1_v - x0_v|, since each closest point is a convex
 * combination of vertices that move at most that far.  So from a sample at t
 * with minimum distance d > floor, no pair can come closer than floor before
 * t + (d - floor) / L: the samples advance by exactly that step (conservative
 * advancement), and reaching t = 1 certifies that the minimum distance stays
 * above `floor` along the whole motion.  Returns the smallest sampled minimum
 * distance (capped at `reach`); *certified = 1 if t = 1 was reached, 0 if a
 * sample came to `floor` or below, or if more than max_samples were needed.
 * *n_samples receives the samples taken, *t_min the time of the smallest. */
double orc_motion_check(int32_t n_verts, const double* x0, const double* x1, const double* inv_mass,
                        int32_t n_tris, const int32_t* tris, int32_t n_edges, const int32_t* edges,
                        double floor_dist, double reach, int64_t max_samples, int32_t* certified,
                        int64_t* n_samples, double* t_min) {
    double L = 0.0;
    for (int32_t v = 0; v < n_verts; ++v) {
        double d[3] = {x1[3 * v] - x0[3 * v], x1[3 * v + 1] - x0[3 * v + 1], x1[3 * v + 2] - x0[3 * v + 2]};
        double m = sqrt(d3(d, d));
        if (m > L) L = m;
    }
    L *= 2.0;
    double* xt = (double*)malloc(sizeof(double) * (3 * (size_t)n_verts + 1));
    double t = 0.0, best = reach, tbest = 0.0;
    int64_t ns = 0;
    int ok = 0;
    while (ns < max_samples) {
        for (size_t k = 0; k < 3 * (size_t)n_verts; ++k) xt[k] = (1.0 - t) * x0[k] + t * x1[k];
        double d = orc_min_separation(n_verts, xt, inv_mass, n_tris, tris, n_edges, edges, reach, 0.0, NULL);
        ++ns;
        if (d < best) { best = d; tbest = t; }
        if (!(d > floor_dist)) break;
        if (t >= 1.0) { ok = 1; break; }
        if (L == 0.0) { ok = 1; break; }
        t += (d - floor_dist) / L;
        if (t > 1.0) t = 1.0;
    }
    free(xt);
    if (certified) *certified = ok;
    if (n_samples) *n_samples = ns;
    if (t_min) *t_min = tbest;
    return best;
}

/* ---- the same separation check for large meshes: a uniform grid ----
 * Items (vertices, triangles, edges, boxes grown by reach / 2) whose largest
 * box extent is at most the cell size h are put in the cell of their box's
 * lower corner; two such boxes can only overlap if those cells are neighbours
 * (each box spans at most h), so every item looks up the 27 cells around its
 * own.  Items larger than h (walls, ground planes) are tested against every
 * item.  Same pairs, rules and results as orc_min_separation. */

typedef struct { uint64_t key; int64_t item; } cell_ref;

static int cmp_cell(const void* a, const void* b) {
    uint64_t x = ((const cell_ref*)a)->key, y = ((const cell_ref*)b)->key;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static uint64_t pack_cell(int64_t cx, int64_t cy, int64_t cz) {
    const int64_t o = (int64_t)1 << 20;
    return ((uint64_t)(cx + o) << 42) | ((uint64_t)(cy + o) << 21) | (uint64_t)(cz + o);
}

static int cmp_dbl(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* distance of one pair of items (kind 0 vertex, 1 triangle, 2 edge), or -1 if
 * the pair is not one the check covers */
static double item_pair_dist2(const item_t* A, const item_t* B, const double* x, const int32_t* tris,
                              const int32_t* edges, const unsigned char* fr, int* kind) {
    int ki = A->kind, kj = B->kind;
    if (A->stat && B->stat) return -1.0;
    if ((ki == 0 && kj == 1) || (ki == 1 && kj == 0)) {
        int32_t v = ki == 0 ? A->id : B->id;
        int32_t t = ki == 1 ? A->id : B->id;
        const int32_t* tv = tris + 3 * t;
        if (tv[0] == v || tv[1] == v || tv[2] == v) return -1.0;
        *kind = 0;
        return pt_tri2(x + 3 * v, x + 3 * tv[0], x + 3 * tv[1], x + 3 * tv[2]);
    }
    if (ki == 2 && kj == 2) {
        const int32_t* a = edges + 2 * A->id;
        const int32_t* b = edges + 2 * B->id;
        if (a[0] == b[0] || a[0] == b[1] || a[1] == b[0] || a[1] == b[1]) return -1.0;
        *kind = 1;
        return seg_seg2(x + 3 * a[0], x + 3 * a[1], x + 3 * b[0], x + 3 * b[1]);
    }
    if (ki == 0 && kj == 0) {
        int32_t a = A->id, b = B->id;
        if (!fr[a] || !fr[b]) return -1.0;
        double dv[3] = {x[3 * a] - x[3 * b], x[3 * a + 1] - x[3 * b + 1], x[3 * a + 2] - x[3 * b + 2]};
        *kind = 2;
        return d3(dv, dv);
    }
    if ((ki == 0 && kj == 2) || (ki == 2 && kj == 0)) {
        int32_t p = ki == 0 ? A->id : B->id;
        const int32_t* e = edges + 2 * (ki == 2 ? A->id : B->id);
        if (!fr[p]) return -1.0;
        *kind = 3;
        return pt_seg2(x + 3 * p, x + 3 * e[0], x + 3 * e[1]);
    }
    return -1.0;
}

static int boxes_overlap(const item_t* A, const item_t* B) {
    for (int k = 0; k < 3; ++k)
        if (A->lo[k] > B->hi[k] || B->lo[k] > A->hi[k]) return 0;
    return 1;
}

double orc_min_separation_grid(int32_t n_verts, const double* x, const double* inv_mass, int32_t n_tris,
                               const int32_t* tris, int32_t n_edges, const int32_t* edges, double reach,
                               double below, int64_t out_counts[4]) {
    unsigned char* fr = (unsigned char*)malloc((size_t)n_verts + 1);
    memset(fr, 1, (size_t)n_verts);
    for (int32_t t = 0; t < 3 * n_tris; ++t) fr[tris[t]] = 0;
    for (int32_t e = 0; e < 2 * n_edges; ++e) fr[edges[e]] = 0;
    const int64_t n = (int64_t)n_verts + n_tris + n_edges;
    item_t* it = (item_t*)malloc(sizeof(item_t) * (size_t)(n + 1));
    const double g = 0.5 * reach;
    for (int32_t v = 0; v < n_verts; ++v) it[v] = make_item(x, &v, 1, g, 0, v);
    for (int32_t t = 0; t < n_tris; ++t) it[n_verts + t] = make_item(x, tris + 3 * t, 3, g, 1, t);
    for (int32_t e = 0; e < n_edges; ++e) it[n_verts + n_tris + e] = make_item(x, edges + 2 * e, 2, g, 2, e);
    double* ext = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    for (int64_t k = 0; k < n; ++k) {
        const int32_t* vs = it[k].kind == 0 ? &it[k].id : (it[k].kind == 1 ? tris + 3 * it[k].id : edges + 2 * it[k].id);
        int nv = it[k].kind == 0 ? 1 : (it[k].kind == 1 ? 3 : 2);
        int s = 1;
        for (int q = 0; q < nv; ++q) s &= (inv_mass == NULL ? 0 : inv_mass[vs[q]] == 0.0);
        it[k].stat = s;
        double e = 0.0;
        for (int a = 0; a < 3; ++a) e = fmax(e, it[k].hi[a] - it[k].lo[a]);
        ext[k] = e;
    }
    /* cell size: the largest extent among items up to 8 times the median */
    double* sorted = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    memcpy(sorted, ext, sizeof(double) * (size_t)n);
    qsort(sorted, (size_t)n, sizeof(double), cmp_dbl);
    double h = n > 0 ? sorted[n / 2] : reach;
    const double cap = 8.0 * h;
    for (int64_t k = 0; k < n; ++k)
        if (sorted[k] <= cap && sorted[k] > h) h = sorted[k];
    if (!(h > 0.0)) h = reach > 0.0 ? reach : 1.0;
    free(sorted);
    int64_t* large = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    cell_ref* cells = (cell_ref*)malloc(sizeof(cell_ref) * (size_t)(n + 1));
    int64_t nl = 0, nc = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (ext[k] > h) { large[nl++] = k; continue; }
        cells[nc].key = pack_cell((int64_t)floor(it[k].lo[0] / h), (int64_t)floor(it[k].lo[1] / h),
                                  (int64_t)floor(it[k].lo[2] / h));
        cells[nc].item = k;
        nc++;
    }
    qsort(cells, (size_t)nc, sizeof(cell_ref), cmp_cell);
    double best2 = reach * reach;
    int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    const double below2 = below * below;
#pragma omp parallel for schedule(dynamic, 512) reduction(min : best2) reduction(+ : c0, c1, c2, c3)
    for (int64_t q = 0; q < nc; ++q) {
        const int64_t i = cells[q].item;
        const int64_t cx = (int64_t)floor(it[i].lo[0] / h), cy = (int64_t)floor(it[i].lo[1] / h),
                      cz = (int64_t)floor(it[i].lo[2] / h);
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    const uint64_t key = pack_cell(cx + dx, cy + dy, cz + dz);
                    int64_t lo = 0, hi = nc;                 /* first entry with this key */
                    while (lo < hi) {
                        int64_t mid = (lo + hi) / 2;
                        if (cells[mid].key < key) lo = mid + 1;
                        else hi = mid;
                    }
                    for (int64_t r = lo; r < nc && cells[r].key == key; ++r) {
                        const int64_t j = cells[r].item;
                        if (j <= i || !boxes_overlap(&it[i], &it[j])) continue;
                        int kind = -1;
                        double dist2 = item_pair_dist2(&it[i], &it[j], x, tris, edges, fr, &kind);
                        if (dist2 < 0.0) continue;
                        if (dist2 < best2) best2 = dist2;
                        if (dist2 < below2) {
                            if (kind == 0) c0++;
                            else if (kind == 1) c1++;
                            else if (kind == 2) c2++;
                            else c3++;
                        }
                    }
                }
    }
    /* large items against every item (each large-large pair once) */
#pragma omp parallel for schedule(dynamic, 4096) reduction(min : best2) reduction(+ : c0, c1, c2, c3)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t a = 0; a < nl; ++a) {
            const int64_t i = large[a];
            if (i == j || (ext[j] > h && j < i)) continue;
            if (!boxes_overlap(&it[i], &it[j])) continue;
            int kind = -1;
            double dist2 = item_pair_dist2(&it[i], &it[j], x, tris, edges, fr, &kind);
            if (dist2 < 0.0) continue;
            if (dist2 < best2) best2 = dist2;
            if (dist2 < below2) { if (kind == 0) c0++; else if (kind == 1) c1++; else if (kind == 2) c2++; else c3++; }
        }
    }
    if (out_counts) { out_counts[0] = c0; out_counts[1] = c1; out_counts[2] = c2; out_counts[3] = c3; }
    free(it); free(fr); free(ext); free(large); free(cells);
    return sqrt(best2);
}
