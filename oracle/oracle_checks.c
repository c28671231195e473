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

static double orient(const double* a, const double* b, const double* c, const double* d) {
    double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double w[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
    return u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) +
           u[2] * (v[0] * w[1] - v[1] * w[0]);
}

static int seg_hits_tri(const double* p0, const double* p1, const double* a, const double* b, const double* c) {
    double o0 = orient(a, b, c, p0), o1 = orient(a, b, c, p1);
    if ((o0 > 0 && o1 > 0) || (o0 < 0 && o1 < 0)) return 0;
    if (o0 == 0 && o1 == 0) {   /* coplanar: touching iff some distance is zero */
        if (pt_tri2(p0, a, b, c) == 0 || pt_tri2(p1, a, b, c) == 0) return 1;
        return seg_seg2(p0, p1, a, b) == 0 || seg_seg2(p0, p1, b, c) == 0 || seg_seg2(p0, p1, c, a) == 0;
    }
    double s1 = orient(p0, p1, a, b), s2 = orient(p0, p1, b, c), s3 = orient(p0, p1, c, a);
    return (s1 >= 0 && s2 >= 0 && s3 >= 0) || (s1 <= 0 && s2 <= 0 && s3 <= 0);
}

typedef struct { double lo[3], hi[3]; int32_t kind, id; } item_t;

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
                          double below, int64_t out_counts[3]) {
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
    /* static[k]: every vertex of item k has zero inverse mass (such pairs never move) */
    unsigned char* st = (unsigned char*)malloc((size_t)n + 1);
    for (int64_t k = 0; k < n; ++k) {
        const int32_t* vs = it[k].kind == 0 ? &it[k].id : (it[k].kind == 1 ? tris + 3 * it[k].id : edges + 2 * it[k].id);
        int nv = it[k].kind == 0 ? 1 : (it[k].kind == 1 ? 3 : 2);
        int s = 1;
        for (int q = 0; q < nv; ++q) s &= (inv_mass == NULL ? 0 : inv_mass[vs[q]] == 0.0);
        st[k] = (unsigned char)s;
    }
    qsort(it, (size_t)n, sizeof(item_t), cmp_lo);
    double best2 = reach * reach;
    int64_t c0 = 0, c1 = 0, c2 = 0;
    const double below2 = below * below;
#pragma omp parallel for schedule(dynamic, 256) reduction(min : best2) reduction(+ : c0, c1, c2)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n && it[j].lo[0] <= it[i].hi[0]; ++j) {
            if (it[j].lo[1] > it[i].hi[1] || it[i].lo[1] > it[j].hi[1]) continue;
            if (it[j].lo[2] > it[i].hi[2] || it[i].lo[2] > it[j].hi[2]) continue;
            if (st[i] && st[j]) continue;
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
            } else {
                continue;
            }
            if (dist2 < best2) best2 = dist2;
            if (dist2 < below2) {
                if (kind == 0) c0++;
                else if (kind == 1) c1++;
                else c2++;
            }
        }
    }
    if (out_counts) { out_counts[0] = c0; out_counts[1] = c1; out_counts[2] = c2; }
    free(it);
    free(fr);
    free(st);
    return sqrt(best2);
}
