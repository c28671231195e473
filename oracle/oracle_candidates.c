/*
 * oracle_candidates.c -- candidate primitive pairs of the broad phase.
 *
 * TEST INFRASTRUCTURE ONLY (see ccfr_oracle.h).
 *
 * Sec. 4.1: every primitive's axis-aligned box is expanded by
 * r + xi/2 + delta/2, and primitive pairs whose expanded boxes overlap are
 * passed to the narrow phase.  The contract this file implements fixes the
 * arithmetic so that the set is exact:
 *
 *   pad = fl32(r + xi/2 + delta/2 + guard)          (sum in FP64, one rounding)
 *   lo  = fl32(min_v x_v - pad),  hi = fl32(max_v x_v + pad)   per axis, with
 *         x_v the FP32 positions and one IEEE single subtraction / addition
 *   candidate  <=>  lo_P <= hi_Q and lo_Q <= hi_P on all three axes.
 *
 * Pair kinds (Alg. 3 inputs plus the point-point interactions of Sec. 4.2):
 *   VF (v, t): v is not a vertex of t;
 *   EE (e, e'), e < e': the edges share no vertex;
 *   VV (i, j), i < j: both are free particles (in no edge and no triangle);
 *   VE (p, e): p is a free particle, e an edge (a particle against a strand
 *       or a cloth edge: no other kind brings the two together).
 * A pair whose vertices all have zero inverse mass is skipped.
 *
 * Everything here is brute force over all primitive pairs: no grid or tree, so
 * the set is the definition itself.
 */
#include "ccfr_oracle.h"

#include <stdlib.h>
#include <string.h>

typedef struct { float lo[3], hi[3]; } fbox;

float orc_box_pad(const orc_params* prm) {
    double s = prm->r + 0.5 * prm->xi + 0.5 * prm->delta + prm->guard;
    return (float)s;
}

static fbox box_of(const orc_mesh* m, const int32_t* vids, int nv, float pad) {
    fbox b;
    for (int k = 0; k < 3; ++k) {
        float mn = (float)m->x[3 * vids[0] + k], mx = mn;
        for (int i = 1; i < nv; ++i) {
            float c = (float)m->x[3 * vids[i] + k];
            if (c < mn) mn = c;
            if (c > mx) mx = c;
        }
        volatile float lo = mn - pad;   /* one FP32 rounding each */
        volatile float hi = mx + pad;
        b.lo[k] = lo;
        b.hi[k] = hi;
    }
    return b;
}

static int overlap(const fbox* p, const fbox* q) {
    for (int k = 0; k < 3; ++k)
        if (!(p->lo[k] <= q->hi[k] && q->lo[k] <= p->hi[k])) return 0;
    return 1;
}

static int all_static(const orc_mesh* m, const int32_t* vids, int nv) {
    for (int i = 0; i < nv; ++i)
        if (m->inv_mass[vids[i]] != 0.0) return 0;
    return 1;
}

/* 1 for vertices in no edge and no triangle */
static unsigned char* free_particle_flags(const orc_mesh* m) {
    unsigned char* f = (unsigned char*)malloc((size_t)m->n_verts + 1);
    memset(f, 1, (size_t)m->n_verts);
    for (int t = 0; t < m->n_tris; ++t)
        for (int k = 0; k < 3; ++k) f[m->tris[3 * t + k]] = 0;
    for (int e = 0; e < m->n_edges; ++e)
        for (int k = 0; k < 2; ++k) f[m->edges[2 * e + k]] = 0;
    return f;
}

static int vert_in_tri(const int32_t* t, int32_t v) { return t[0] == v || t[1] == v || t[2] == v; }
static int edges_share(const int32_t* e, const int32_t* f) {
    return e[0] == f[0] || e[0] == f[1] || e[1] == f[0] || e[1] == f[1];
}

typedef struct {
    float pad;
    fbox* vbox;
    fbox* tbox;
    fbox* ebox;
    unsigned char *vstat, *tstat, *estat, *vfree;
} boxes_t;

static void boxes_build(const orc_mesh* m, const orc_params* prm, boxes_t* B) {
    B->pad = orc_box_pad(prm);
    B->vbox = (fbox*)malloc(sizeof(fbox) * ((size_t)m->n_verts + 1));
    B->tbox = (fbox*)malloc(sizeof(fbox) * ((size_t)m->n_tris + 1));
    B->ebox = (fbox*)malloc(sizeof(fbox) * ((size_t)m->n_edges + 1));
    B->vstat = (unsigned char*)malloc((size_t)m->n_verts + 1);
    B->tstat = (unsigned char*)malloc((size_t)m->n_tris + 1);
    B->estat = (unsigned char*)malloc((size_t)m->n_edges + 1);
    for (int v = 0; v < m->n_verts; ++v) {
        B->vbox[v] = box_of(m, &v, 1, B->pad);
        B->vstat[v] = (unsigned char)all_static(m, &v, 1);
    }
    for (int t = 0; t < m->n_tris; ++t) {
        B->tbox[t] = box_of(m, m->tris + 3 * t, 3, B->pad);
        B->tstat[t] = (unsigned char)all_static(m, m->tris + 3 * t, 3);
    }
    for (int e = 0; e < m->n_edges; ++e) {
        B->ebox[e] = box_of(m, m->edges + 2 * e, 2, B->pad);
        B->estat[e] = (unsigned char)all_static(m, m->edges + 2 * e, 2);
    }
    B->vfree = free_particle_flags(m);
}

static void boxes_free(boxes_t* B) {
    free(B->vbox); free(B->tbox); free(B->ebox);
    free(B->vstat); free(B->tstat); free(B->estat); free(B->vfree);
}

/* the three pair predicates */
static int is_vf(const orc_mesh* m, const boxes_t* B, int32_t v, int32_t t) {
    if (vert_in_tri(m->tris + 3 * t, v)) return 0;
    if (B->vstat[v] && B->tstat[t]) return 0;
    return overlap(&B->vbox[v], &B->tbox[t]);
}
static int is_ee(const orc_mesh* m, const boxes_t* B, int32_t e, int32_t f) {
    if (e == f || edges_share(m->edges + 2 * e, m->edges + 2 * f)) return 0;
    if (B->estat[e] && B->estat[f]) return 0;
    return overlap(&B->ebox[e], &B->ebox[f]);
}
static int is_ve(const boxes_t* B, int32_t p, int32_t e) {
    if (!B->vfree[p]) return 0;
    if (B->vstat[p] && B->estat[e]) return 0;
    return overlap(&B->vbox[p], &B->ebox[e]);
}
static int is_vv(const boxes_t* B, int32_t i, int32_t j) {
    if (i == j || !B->vfree[i] || !B->vfree[j]) return 0;
    if (B->vstat[i] && B->vstat[j]) return 0;
    return overlap(&B->vbox[i], &B->vbox[j]);
}

/* Two passes (count per outer index, then fill at prefix offsets) keep the
 * lists in ascending order whatever the thread schedule. */
void orc_candidates(const orc_mesh* m, const orc_params* prm,
                    int32_t* vf, int64_t cap_vf, int32_t* ee, int64_t cap_ee,
                    int32_t* vv, int64_t cap_vv, int32_t* ve, int64_t cap_ve, int64_t counts[4]) {
    boxes_t B;
    boxes_build(m, prm, &B);
    int nmax = m->n_verts > m->n_edges ? m->n_verts : m->n_edges;
    int64_t* cnt = (int64_t*)calloc((size_t)nmax + 1, sizeof(int64_t));

    /* VF */
#pragma omp parallel for schedule(dynamic, 64)
    for (int v = 0; v < m->n_verts; ++v) {
        int64_t c = 0;
        for (int t = 0; t < m->n_tris; ++t) c += is_vf(m, &B, v, t);
        cnt[v + 1] = c;
    }
    for (int v = 0; v < m->n_verts; ++v) cnt[v + 1] += cnt[v];
    counts[0] = cnt[m->n_verts];
    if (vf && cap_vf > 0) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int v = 0; v < m->n_verts; ++v) {
            int64_t o = cnt[v];
            for (int t = 0; t < m->n_tris; ++t)
                if (is_vf(m, &B, v, t)) {
                    if (o < cap_vf) { vf[2 * o] = v; vf[2 * o + 1] = t; }
                    ++o;
                }
        }
    }

    /* EE */
    memset(cnt, 0, sizeof(int64_t) * ((size_t)nmax + 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int e = 0; e < m->n_edges; ++e) {
        int64_t c = 0;
        for (int f = e + 1; f < m->n_edges; ++f) c += is_ee(m, &B, e, f);
        cnt[e + 1] = c;
    }
    for (int e = 0; e < m->n_edges; ++e) cnt[e + 1] += cnt[e];
    counts[1] = cnt[m->n_edges];
    if (ee && cap_ee > 0) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int e = 0; e < m->n_edges; ++e) {
            int64_t o = cnt[e];
            for (int f = e + 1; f < m->n_edges; ++f)
                if (is_ee(m, &B, e, f)) {
                    if (o < cap_ee) { ee[2 * o] = e; ee[2 * o + 1] = f; }
                    ++o;
                }
        }
    }

    /* VV */
    memset(cnt, 0, sizeof(int64_t) * ((size_t)nmax + 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < m->n_verts; ++i) {
        int64_t c = 0;
        if (B.vfree[i])
            for (int j = i + 1; j < m->n_verts; ++j) c += is_vv(&B, i, j);
        cnt[i + 1] = c;
    }
    for (int i = 0; i < m->n_verts; ++i) cnt[i + 1] += cnt[i];
    counts[2] = cnt[m->n_verts];
    if (vv && cap_vv > 0) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int i = 0; i < m->n_verts; ++i) {
            int64_t o = cnt[i];
            if (!B.vfree[i]) continue;
            for (int j = i + 1; j < m->n_verts; ++j)
                if (is_vv(&B, i, j)) {
                    if (o < cap_vv) { vv[2 * o] = i; vv[2 * o + 1] = j; }
                    ++o;
                }
        }
    }

    /* VE */
    memset(cnt, 0, sizeof(int64_t) * ((size_t)nmax + 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int p = 0; p < m->n_verts; ++p) {
        int64_t c = 0;
        if (B.vfree[p])
            for (int e = 0; e < m->n_edges; ++e) c += is_ve(&B, p, e);
        cnt[p + 1] = c;
    }
    for (int p = 0; p < m->n_verts; ++p) cnt[p + 1] += cnt[p];
    counts[3] = cnt[m->n_verts];
    if (ve && cap_ve > 0) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int p = 0; p < m->n_verts; ++p) {
            int64_t o = cnt[p];
            if (!B.vfree[p]) continue;
            for (int e = 0; e < m->n_edges; ++e)
                if (is_ve(&B, p, e)) {
                    if (o < cap_ve) { ve[2 * o] = p; ve[2 * o + 1] = e; }
                    ++o;
                }
        }
    }
    free(cnt);
    boxes_free(&B);
}

int64_t orc_ve_edges_of_vertex(const orc_mesh* m, const orc_params* prm, int32_t v, int32_t* out, int64_t cap) {
    unsigned char* fr = free_particle_flags(m);
    int64_t n = 0;
    if (fr[v]) {
        float pad = orc_box_pad(prm);
        fbox bv = box_of(m, &v, 1, pad);
        int sv = all_static(m, &v, 1);
        for (int e = 0; e < m->n_edges; ++e) {
            const int32_t* ev = m->edges + 2 * e;
            if (sv && all_static(m, ev, 2)) continue;
            fbox be = box_of(m, ev, 2, pad);
            if (!overlap(&bv, &be)) continue;
            if (n < cap) out[n] = e;
            ++n;
        }
    }
    free(fr);
    return n;
}

int64_t orc_ve_verts_of_edge(const orc_mesh* m, const orc_params* prm, int32_t e, int32_t* out, int64_t cap) {
    unsigned char* fr = free_particle_flags(m);
    float pad = orc_box_pad(prm);
    const int32_t* ev = m->edges + 2 * e;
    fbox be = box_of(m, ev, 2, pad);
    int se = all_static(m, ev, 2);
    int64_t n = 0;
    for (int v = 0; v < m->n_verts; ++v) {
        if (!fr[v]) continue;
        if (se && all_static(m, &v, 1)) continue;
        fbox bv = box_of(m, &v, 1, pad);
        if (!overlap(&bv, &be)) continue;
        if (n < cap) out[n] = v;
        ++n;
    }
    free(fr);
    return n;
}

int64_t orc_vf_tris_of_vertex(const orc_mesh* m, const orc_params* prm, int32_t v,
                              int32_t* out, int64_t cap) {
    float pad = orc_box_pad(prm);
    fbox bv = box_of(m, &v, 1, pad);
    int sv = all_static(m, &v, 1);
    int64_t n = 0;
    for (int t = 0; t < m->n_tris; ++t) {
        const int32_t* tv = m->tris + 3 * t;
        if (vert_in_tri(tv, v)) continue;
        if (sv && all_static(m, tv, 3)) continue;
        fbox bt = box_of(m, tv, 3, pad);
        if (!overlap(&bv, &bt)) continue;
        if (n < cap) out[n] = t;
        ++n;
    }
    return n;
}

int64_t orc_vf_verts_of_tri(const orc_mesh* m, const orc_params* prm, int32_t t,
                            int32_t* out, int64_t cap) {
    float pad = orc_box_pad(prm);
    const int32_t* tv = m->tris + 3 * t;
    fbox bt = box_of(m, tv, 3, pad);
    int st = all_static(m, tv, 3);
    int64_t n = 0;
    for (int v = 0; v < m->n_verts; ++v) {
        if (vert_in_tri(tv, v)) continue;
        if (st && all_static(m, &v, 1)) continue;
        fbox bv = box_of(m, &v, 1, pad);
        if (!overlap(&bv, &bt)) continue;
        if (n < cap) out[n] = v;
        ++n;
    }
    return n;
}

int64_t orc_ee_partners_of_edge(const orc_mesh* m, const orc_params* prm, int32_t e,
                                int32_t* out, int64_t cap) {
    float pad = orc_box_pad(prm);
    const int32_t* ev = m->edges + 2 * e;
    fbox be = box_of(m, ev, 2, pad);
    int se = all_static(m, ev, 2);
    int64_t n = 0;
    for (int f = 0; f < m->n_edges; ++f) {
        const int32_t* fv = m->edges + 2 * f;
        if (f == e || edges_share(ev, fv)) continue;
        if (se && all_static(m, fv, 2)) continue;
        fbox bf = box_of(m, fv, 2, pad);
        if (!overlap(&be, &bf)) continue;
        if (n < cap) out[n] = f;
        ++n;
    }
    return n;
}

int64_t orc_vv_partners_of_vertex(const orc_mesh* m, const orc_params* prm, int32_t v,
                                  int32_t* out, int64_t cap) {
    unsigned char* fr = free_particle_flags(m);
    int64_t n = 0;
    if (fr[v]) {
        float pad = orc_box_pad(prm);
        fbox bv = box_of(m, &v, 1, pad);
        int sv = all_static(m, &v, 1);
        for (int j = 0; j < m->n_verts; ++j) {
            if (j == v || !fr[j]) continue;
            if (sv && all_static(m, &j, 1)) continue;
            fbox bj = box_of(m, &j, 1, pad);
            if (!overlap(&bv, &bj)) continue;
            if (n < cap) out[n] = j;
            ++n;
        }
    }
    free(fr);
    return n;
}
