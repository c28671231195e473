/*
 * oracle_regions.c -- per-vertex convex regions (App. C, Algorithm 3), FP64.
 *
 * TEST INFRASTRUCTURE ONLY (see ccfr_oracle.h).
 *
 * For an active vertex p with inverse mass w_p > 0, Algorithm 3 walks
 *   (VF) the passive faces f of p:           closest point x_q on f to x_p,
 *        n = x_p - x_q, phi = |n| - xi, kept if phi < 2r,
 *        w_f = sum_v bary_v w_v, d = w_p / (w_p + w_f) phi;
 *   (EE) each incident edge e of p against its passive edges e':
 *        closest points x_A on e and x_B on e', n = x_A - x_B, phi = |n| - xi,
 *        w_e, w_e' barycentric-weighted, d = w_e / (w_e + w_e') phi;
 *   (FV) each incident face f_p of p against its passive vertices q:
 *        closest point x_A on f_p to x_q, phi = |x_A - x_q| - xi,
 *        d = w_f / (w_f + w_q) phi;
 * and stores (d, n / |n|, phi) for p.  This is Eq. 2/3 (Sec. 3.1) written for
 * mesh primitives.  Readings of the printed algorithm:
 *   -   d = s (|n| - xi): the separation after the step is at least xi.
 *   -   (FV) the normal points from the vertex q towards the face,
 *       n = x_A - x_q, and the share is w_f / (w_f + w_q): the printed
 *       x_q - x_A and w_p would let a face vertex move towards q.
 *   -   effective inverse masses are sum bary * w as printed; a pair whose two
 *       sides both have zero effective inverse mass gives no half-space; static
 *       vertices (w = 0) get no region.
 *   -   EE closest points are computed once per pair with the lower edge index
 *       first, so both sides of a pair see the same two points.
 *   -   zero-area triangles, zero-length edges and coincident closest points
 *       are skipped and counted.
 *   VV  free particles i, j (Sec. 4.2 point-point interactions) use Eq. 1-2
 *       directly: n = x_p - x_q, d = w_p / (w_p + w_q) phi.
 *   VE  a free particle p against an edge e (closest point x_B = (1-t) x_a +
 *       t x_b on e): for p, n = x_p - x_B and d = w_p / (w_p + w_e) phi with
 *       w_e = (1-t) w_a + t w_b; for the edge's endpoints (EV, as FV for a
 *       face) n = x_B - x_p and d = w_e / (w_e + w_p) phi.
 * The paper's passive sets T, E, Q come from the broad phase: here they are
 * read from the candidate lists (orc_regions) or recomputed by brute force for
 * one vertex (orc_vertex_region).
 */
#include "ccfr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static uint64_t make_key(int kind, int32_t a, int32_t b) {
    return ((uint64_t)kind << 62) | ((uint64_t)(uint32_t)a << 31) | (uint64_t)(uint32_t)b;
}

static const double* X(const orc_mesh* m, int32_t v) { return m->x + 3 * (size_t)v; }

typedef struct {
    orc_halfspace* out;
    int64_t cap, n, n_degenerate;
} sink_t;

static void emit(sink_t* s, const double nvec[3], double D, double phi, double share, uint64_t key,
                 int fragile) {
    if (s->n < s->cap) {
        orc_halfspace* h = &s->out[s->n];
        for (int k = 0; k < 3; ++k) h->n[k] = nvec[k] / D;
        h->d = share * phi;
        h->phi = phi;
        h->share = share;
        h->key = key;
        h->fragile = fragile;
        h->pad_ = 0;
    }
    s->n++;
}

/* passive sets of one active vertex p */
typedef struct {
    const int32_t* faces; int64_t n_faces;                 /* T: passive faces of p         */
    int n_inc_edges; const int32_t* inc_edges;             /* AdjEdges(p)                   */
    const int32_t** edge_partners; const int64_t* n_edge_partners; /* E per incident edge  */
    int n_inc_faces; const int32_t* inc_faces;             /* AdjFaces(p)                   */
    const int32_t** face_partners; const int64_t* n_face_partners; /* Q per incident face  */
    const int32_t* particles; int64_t n_particles;        /* VV partners                   */
    const int32_t* pedges; int64_t n_pedges;              /* VE: edges passive to particle p */
    const int32_t** edge_particles; const int64_t* n_edge_particles; /* EV per incident edge */
} passive_t;

static void narrow_phase_vertex(const orc_mesh* m, const orc_params* prm, int32_t p,
                                const passive_t* P, sink_t* s) {
    const double* w = m->inv_mass;
    const double r = prm->r, xi = prm->xi;
    if (w[p] == 0.0) return;                                  /* static: no region */

    /* VF: p against its passive faces */
    for (int64_t i = 0; i < P->n_faces; ++i) {
        int32_t f = P->faces[i];
        const int32_t* fv = m->tris + 3 * (size_t)f;
        if (fv[0] == p || fv[1] == p || fv[2] == p) continue;
        double xq[3], bary[3];
        if (orc_closest_point_triangle(X(m, p), X(m, fv[0]), X(m, fv[1]), X(m, fv[2]), xq, bary) < 0) {
            s->n_degenerate++;
            continue;
        }
        double nvec[3] = {X(m, p)[0] - xq[0], X(m, p)[1] - xq[1], X(m, p)[2] - xq[2]};
        double D = sqrt(nvec[0] * nvec[0] + nvec[1] * nvec[1] + nvec[2] * nvec[2]);
        double phi = D - xi;
        if (!(phi < 2.0 * r)) continue;
        if (D == 0.0) { s->n_degenerate++; continue; }
        double wf = bary[0] * w[fv[0]] + bary[1] * w[fv[1]] + bary[2] * w[fv[2]];
        double wsum = w[p] + wf;
        if (wsum == 0.0) continue;
        emit(s, nvec, D, phi, w[p] / wsum, make_key(ORC_KIND_VF, p, f), 0);
    }

    /* EE: each incident edge of p against its passive edges */
    for (int ie = 0; ie < P->n_inc_edges; ++ie) {
        int32_t e = P->inc_edges[ie];
        for (int64_t i = 0; i < P->n_edge_partners[ie]; ++i) {
            int32_t e2 = P->edge_partners[ie][i];
            const int32_t* ea = m->edges + 2 * (size_t)e;
            const int32_t* eb = m->edges + 2 * (size_t)e2;
            if (e == e2 || ea[0] == eb[0] || ea[0] == eb[1] || ea[1] == eb[0] || ea[1] == eb[1]) continue;
            int32_t lo = e < e2 ? e : e2, hi = e < e2 ? e2 : e;
            const int32_t* L = m->edges + 2 * (size_t)lo;
            const int32_t* H = m->edges + 2 * (size_t)hi;
            double sL, tH;
            int rc = orc_closest_points_segments(X(m, L[0]), X(m, L[1]), X(m, H[0]), X(m, H[1]), &sL, &tH);
            if (rc < 0) { s->n_degenerate++; continue; }
            double pL[3], qH[3];
            for (int k = 0; k < 3; ++k) {
                pL[k] = (1.0 - sL) * X(m, L[0])[k] + sL * X(m, L[1])[k];
                qH[k] = (1.0 - tH) * X(m, H[0])[k] + tH * X(m, H[1])[k];
            }
            double wL = (1.0 - sL) * w[L[0]] + sL * w[L[1]];
            double wH = (1.0 - tH) * w[H[0]] + tH * w[H[1]];
            /* x_A on the active edge e, x_B on the passive edge e2 */
            const double* xA = (e == lo) ? pL : qH;
            const double* xB = (e == lo) ? qH : pL;
            double we = (e == lo) ? wL : wH, we2 = (e == lo) ? wH : wL;
            double nvec[3] = {xA[0] - xB[0], xA[1] - xB[1], xA[2] - xB[2]};
            double D = sqrt(nvec[0] * nvec[0] + nvec[1] * nvec[1] + nvec[2] * nvec[2]);
            double phi = D - xi;
            if (!(phi < 2.0 * r)) continue;
            if (D == 0.0) { s->n_degenerate++; continue; }
            double wsum = we + we2;
            if (wsum == 0.0) continue;
            /* near-parallel edges: the closest points are ill-conditioned */
            double d1[3], d2[3], cr[3];
            for (int k = 0; k < 3; ++k) { d1[k] = X(m, L[1])[k] - X(m, L[0])[k]; d2[k] = X(m, H[1])[k] - X(m, H[0])[k]; }
            cr[0] = d1[1] * d2[2] - d1[2] * d2[1];
            cr[1] = d1[2] * d2[0] - d1[0] * d2[2];
            cr[2] = d1[0] * d2[1] - d1[1] * d2[0];
            double a2 = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
            double b2 = d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2];
            double sin2 = (cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]) / (a2 * b2);
            int fragile = (rc == 1) || sin2 < 1e-6;
            emit(s, nvec, D, phi, we / wsum, make_key(ORC_KIND_EE, lo, hi), fragile);
        }
    }

    /* FV: each incident face of p against its passive vertices */
    for (int jf = 0; jf < P->n_inc_faces; ++jf) {
        int32_t f = P->inc_faces[jf];
        const int32_t* fv = m->tris + 3 * (size_t)f;
        for (int64_t i = 0; i < P->n_face_partners[jf]; ++i) {
            int32_t q = P->face_partners[jf][i];
            if (fv[0] == q || fv[1] == q || fv[2] == q) continue;
            double xA[3], bary[3];
            if (orc_closest_point_triangle(X(m, q), X(m, fv[0]), X(m, fv[1]), X(m, fv[2]), xA, bary) < 0) {
                s->n_degenerate++;
                continue;
            }
            double nvec[3] = {xA[0] - X(m, q)[0], xA[1] - X(m, q)[1], xA[2] - X(m, q)[2]};   /* towards the face */
            double D = sqrt(nvec[0] * nvec[0] + nvec[1] * nvec[1] + nvec[2] * nvec[2]);
            double phi = D - xi;
            if (!(phi < 2.0 * r)) continue;
            if (D == 0.0) { s->n_degenerate++; continue; }
            double wf = bary[0] * w[fv[0]] + bary[1] * w[fv[1]] + bary[2] * w[fv[2]];
            double wsum = wf + w[q];                                                      /* face share */
            if (wsum == 0.0) continue;
            emit(s, nvec, D, phi, wf / wsum, make_key(ORC_KIND_VF, q, f), 0);
        }
    }

    /* VE: free particle p against its passive edges */
    for (int64_t i = 0; i < P->n_pedges; ++i) {
        int32_t e = P->pedges[i];
        const int32_t* ev = m->edges + 2 * (size_t)e;
        double t;
        if (orc_closest_point_segment(X(m, p), X(m, ev[0]), X(m, ev[1]), &t) < 0) { s->n_degenerate++; continue; }
        double xb[3];
        for (int k = 0; k < 3; ++k) xb[k] = (1.0 - t) * X(m, ev[0])[k] + t * X(m, ev[1])[k];
        double nvec[3] = {X(m, p)[0] - xb[0], X(m, p)[1] - xb[1], X(m, p)[2] - xb[2]};
        double D = sqrt(nvec[0] * nvec[0] + nvec[1] * nvec[1] + nvec[2] * nvec[2]);
        double phi = D - xi;
        if (!(phi < 2.0 * r)) continue;
        if (D == 0.0) { s->n_degenerate++; continue; }
        double we = (1.0 - t) * w[ev[0]] + t * w[ev[1]];
        double wsum = w[p] + we;
        if (wsum == 0.0) continue;
        emit(s, nvec, D, phi, w[p] / wsum, make_key(ORC_KIND_VE, p, e), 0);
    }

    /* EV: each incident edge of p against its passive particles */
    for (int ie = 0; ie < P->n_inc_edges && P->edge_particles; ++ie) {
        int32_t e = P->inc_edges[ie];
        const int32_t* ev = m->edges + 2 * (size_t)e;
        for (int64_t i = 0; i < P->n_edge_particles[ie]; ++i) {
            int32_t q = P->edge_particles[ie][i];
            double t;
            if (orc_closest_point_segment(X(m, q), X(m, ev[0]), X(m, ev[1]), &t) < 0) { s->n_degenerate++; continue; }
            double xa[3];
            for (int k = 0; k < 3; ++k) xa[k] = (1.0 - t) * X(m, ev[0])[k] + t * X(m, ev[1])[k];
            double nvec[3] = {xa[0] - X(m, q)[0], xa[1] - X(m, q)[1], xa[2] - X(m, q)[2]};
            double D = sqrt(nvec[0] * nvec[0] + nvec[1] * nvec[1] + nvec[2] * nvec[2]);
            double phi = D - xi;
            if (!(phi < 2.0 * r)) continue;
            if (D == 0.0) { s->n_degenerate++; continue; }
            double we = (1.0 - t) * w[ev[0]] + t * w[ev[1]];
            double wsum = we + w[q];
            if (wsum == 0.0) continue;
            emit(s, nvec, D, phi, we / wsum, make_key(ORC_KIND_VE, q, e), 0);
        }
    }

    /* VV: free particle p against its partners (Eq. 1-2) */
    for (int64_t i = 0; i < P->n_particles; ++i) {
        int32_t q = P->particles[i];
        if (q == p) continue;
        double nvec[3] = {X(m, p)[0] - X(m, q)[0], X(m, p)[1] - X(m, q)[1], X(m, p)[2] - X(m, q)[2]};
        double D = sqrt(nvec[0] * nvec[0] + nvec[1] * nvec[1] + nvec[2] * nvec[2]);
        double phi = D - xi;
        if (!(phi < 2.0 * r)) continue;
        if (D == 0.0) { s->n_degenerate++; continue; }
        double wsum = w[p] + w[q];
        if (wsum == 0.0) continue;
        int32_t a = p < q ? p : q, b = p < q ? q : p;
        emit(s, nvec, D, phi, w[p] / wsum, make_key(ORC_KIND_VV, a, b), 0);
    }
}

/* ---------------- CSR helpers ---------------- */

typedef struct { int64_t* off; int32_t* idx; } csr_t;

/* rows[i] receives cols[i] for i < n (both optional to mirror) */
static csr_t csr_build(int64_t n_rows, int64_t n, const int32_t* rows, int rs, const int32_t* cols, int cs) {
    csr_t c;
    c.off = (int64_t*)calloc((size_t)n_rows + 1, sizeof(int64_t));
    c.idx = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < n; ++i) c.off[rows[i * rs] + 1]++;
    for (int64_t r = 0; r < n_rows; ++r) c.off[r + 1] += c.off[r];
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n_rows + 1));
    memcpy(cur, c.off, sizeof(int64_t) * (size_t)n_rows);
    for (int64_t i = 0; i < n; ++i) c.idx[cur[rows[i * rs]]++] = cols[i * cs];
    free(cur);
    return c;
}

static void csr_free(csr_t* c) { free(c->off); free(c->idx); }

int64_t orc_regions(const orc_mesh* m, const orc_params* prm,
                    const int32_t* vf, int64_t n_vf, const int32_t* ee, int64_t n_ee,
                    const int32_t* vv, int64_t n_vv, const int32_t* vpe, int64_t n_ve,
                    int64_t* offsets, orc_halfspace* hs, int64_t cap, int64_t stats[4]) {
    const int32_t N = m->n_verts;
    /* passive faces of each vertex, passive vertices of each face */
    csr_t Tv = csr_build(N, n_vf, vf, 2, vf + 1, 2);
    csr_t Qf = csr_build(m->n_tris, n_vf, vf + 1, 2, vf, 2);
    /* passive edges of each edge: both directions */
    int32_t* ee2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(4 * n_ee + 2));
    for (int64_t i = 0; i < n_ee; ++i) {
        ee2[4 * i + 0] = ee[2 * i]; ee2[4 * i + 1] = ee[2 * i + 1];
        ee2[4 * i + 2] = ee[2 * i + 1]; ee2[4 * i + 3] = ee[2 * i];
    }
    csr_t Ee = csr_build(m->n_edges, 2 * n_ee, ee2, 2, ee2 + 1, 2);
    int32_t* vv2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(4 * n_vv + 2));
    for (int64_t i = 0; i < n_vv; ++i) {
        vv2[4 * i + 0] = vv[2 * i]; vv2[4 * i + 1] = vv[2 * i + 1];
        vv2[4 * i + 2] = vv[2 * i + 1]; vv2[4 * i + 3] = vv[2 * i];
    }
    csr_t Vv = csr_build(N, 2 * n_vv, vv2, 2, vv2 + 1, 2);
    /* VE: the edges of each free particle, the particles of each edge */
    csr_t Pv = csr_build(N, n_ve, vpe, 2, vpe + 1, 2);
    csr_t Pe = csr_build(m->n_edges, n_ve, vpe + 1, 2, vpe, 2);
    /* incidence */
    int32_t* ve = (int32_t*)malloc(sizeof(int32_t) * (size_t)(4 * m->n_edges + 2));
    for (int32_t e = 0; e < m->n_edges; ++e) {
        ve[4 * e + 0] = m->edges[2 * e]; ve[4 * e + 1] = e;
        ve[4 * e + 2] = m->edges[2 * e + 1]; ve[4 * e + 3] = e;
    }
    csr_t AdjE = csr_build(N, 2 * (int64_t)m->n_edges, ve, 2, ve + 1, 2);
    int32_t* vt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(6 * m->n_tris + 2));
    for (int32_t t = 0; t < m->n_tris; ++t)
        for (int k = 0; k < 3; ++k) { vt[6 * t + 2 * k] = m->tris[3 * t + k]; vt[6 * t + 2 * k + 1] = t; }
    csr_t AdjF = csr_build(N, 3 * (int64_t)m->n_tris, vt, 2, vt + 1, 2);

    int64_t* cnt = (int64_t*)calloc((size_t)N + 1, sizeof(int64_t));
    int64_t ndeg_total = 0;
    for (int phase = 0; phase < 2; ++phase) {
#pragma omp parallel for schedule(dynamic, 32) reduction(+ : ndeg_total)
        for (int32_t p = 0; p < N; ++p) {
            int ne = (int)(AdjE.off[p + 1] - AdjE.off[p]);
            int nf = (int)(AdjF.off[p + 1] - AdjF.off[p]);
            const int32_t** ep = (const int32_t**)malloc(sizeof(void*) * (size_t)(ne + 1));
            int64_t* nep = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ne + 1));
            const int32_t** fp = (const int32_t**)malloc(sizeof(void*) * (size_t)(nf + 1));
            int64_t* nfp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nf + 1));
            const int32_t** pp = (const int32_t**)malloc(sizeof(void*) * (size_t)(ne + 1));
            int64_t* npp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ne + 1));
            const int32_t* incE = AdjE.idx + AdjE.off[p];
            const int32_t* incF = AdjF.idx + AdjF.off[p];
            for (int i = 0; i < ne; ++i) {
                ep[i] = Ee.idx + Ee.off[incE[i]];
                nep[i] = Ee.off[incE[i] + 1] - Ee.off[incE[i]];
                pp[i] = Pe.idx + Pe.off[incE[i]];
                npp[i] = Pe.off[incE[i] + 1] - Pe.off[incE[i]];
            }
            for (int i = 0; i < nf; ++i) {
                fp[i] = Qf.idx + Qf.off[incF[i]];
                nfp[i] = Qf.off[incF[i] + 1] - Qf.off[incF[i]];
            }
            passive_t P = {Tv.idx + Tv.off[p], Tv.off[p + 1] - Tv.off[p],
                           ne, incE, ep, nep, nf, incF, fp, nfp,
                           Vv.idx + Vv.off[p], Vv.off[p + 1] - Vv.off[p],
                           Pv.idx + Pv.off[p], Pv.off[p + 1] - Pv.off[p], pp, npp};
            sink_t s;
            if (phase == 0) { s.out = NULL; s.cap = 0; }
            else {
                s.out = hs ? hs + offsets[p] : NULL;
                int64_t room = cap - offsets[p];
                s.cap = hs ? (room < 0 ? 0 : room) : 0;
            }
            s.n = 0;
            s.n_degenerate = 0;
            narrow_phase_vertex(m, prm, p, &P, &s);
            if (phase == 0) { cnt[p + 1] = s.n; ndeg_total += s.n_degenerate; }
            free(ep); free(nep); free(fp); free(nfp); free(pp); free(npp);
        }
        if (phase == 0) {
            for (int32_t p = 0; p < N; ++p) cnt[p + 1] += cnt[p];
            for (int32_t p = 0; p <= N; ++p) offsets[p] = cnt[p];
            if (!hs || cap <= 0) break;
        }
    }
    int64_t H = cnt[N];
    if (stats) { stats[0] = ndeg_total; stats[1] = H; stats[2] = 0; stats[3] = 0; }
    free(cnt);
    csr_free(&Tv); csr_free(&Qf); csr_free(&Ee); csr_free(&Vv); csr_free(&AdjE); csr_free(&AdjF);
    csr_free(&Pv); csr_free(&Pe);
    free(ee2); free(vv2); free(ve); free(vt);
    return H;
}

int64_t orc_vertex_region(const orc_mesh* m, const orc_params* prm, int32_t v,
                          orc_halfspace* hs, int64_t cap) {
    /* incident edges and faces */
    int ne = 0, nf = 0;
    for (int32_t e = 0; e < m->n_edges; ++e) ne += (m->edges[2 * e] == v || m->edges[2 * e + 1] == v);
    for (int32_t t = 0; t < m->n_tris; ++t)
        nf += (m->tris[3 * t] == v || m->tris[3 * t + 1] == v || m->tris[3 * t + 2] == v);
    int32_t* incE = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ne + 1));
    int32_t* incF = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nf + 1));
    ne = nf = 0;
    for (int32_t e = 0; e < m->n_edges; ++e)
        if (m->edges[2 * e] == v || m->edges[2 * e + 1] == v) incE[ne++] = e;
    for (int32_t t = 0; t < m->n_tris; ++t)
        if (m->tris[3 * t] == v || m->tris[3 * t + 1] == v || m->tris[3 * t + 2] == v) incF[nf++] = t;

    const int64_t big = (int64_t)m->n_verts + m->n_tris + m->n_edges + 1;
    int32_t* faces = (int32_t*)malloc(sizeof(int32_t) * (size_t)big);
    int64_t n_faces = orc_vf_tris_of_vertex(m, prm, v, faces, big);
    const int32_t** ep = (const int32_t**)malloc(sizeof(void*) * (size_t)(ne + 1));
    int64_t* nep = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ne + 1));
    for (int i = 0; i < ne; ++i) {
        int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)big);
        nep[i] = orc_ee_partners_of_edge(m, prm, incE[i], buf, big);
        ep[i] = buf;
    }
    const int32_t** fp = (const int32_t**)malloc(sizeof(void*) * (size_t)(nf + 1));
    int64_t* nfp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nf + 1));
    for (int i = 0; i < nf; ++i) {
        int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)big);
        nfp[i] = orc_vf_verts_of_tri(m, prm, incF[i], buf, big);
        fp[i] = buf;
    }
    int32_t* parts = (int32_t*)malloc(sizeof(int32_t) * (size_t)big);
    int64_t n_parts = orc_vv_partners_of_vertex(m, prm, v, parts, big);
    int32_t* pedges = (int32_t*)malloc(sizeof(int32_t) * (size_t)big);
    int64_t n_pedges = orc_ve_edges_of_vertex(m, prm, v, pedges, big);
    const int32_t** pp = (const int32_t**)malloc(sizeof(void*) * (size_t)(ne + 1));
    int64_t* npp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ne + 1));
    for (int i = 0; i < ne; ++i) {
        int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)big);
        npp[i] = orc_ve_verts_of_edge(m, prm, incE[i], buf, big);
        pp[i] = buf;
    }

    passive_t P = {faces, n_faces, ne, incE, ep, nep, nf, incF, fp, nfp, parts, n_parts,
                   pedges, n_pedges, pp, npp};
    sink_t s = {hs, cap, 0, 0};
    narrow_phase_vertex(m, prm, v, &P, &s);

    for (int i = 0; i < ne; ++i) free((void*)ep[i]);
    for (int i = 0; i < ne; ++i) free((void*)pp[i]);
    for (int i = 0; i < nf; ++i) free((void*)fp[i]);
    free(pp); free(npp); free(pedges);
    free(ep); free(nep); free(fp); free(nfp); free(faces); free(parts); free(incE); free(incF);
    return s.n;
}
