/*
 * oracle_response.c -- the soft response and friction of Sec. 3.3, applied per
 * vertex between the XPBD constraints and the projection (applyResponse in
 * Alg. 4), FP64.
 *
 * TEST INFRASTRUCTURE ONLY (see ccfr_oracle.h).
 *
 * The paper's response energy E_c = k/2 w_c max(0, delta - d_c)^2 becomes the
 * XPBD constraint C_c = max(0, delta - d_c) with compliance alpha = 1/k; the
 * visibility weight w_c = prod_{j != c} (1 - S((d_c - d_j) / delta_v)), S the
 * cubic smoothstep, lets the innermost contacts occlude farther ones; friction
 * follows Macklin et al. 2014 on the same active contacts.  Readings of what
 * the paper leaves open:
 *   -    d_c is the pair's gap beyond the offset at the vertex's proposal y,
 *        with the two sides advancing in proportion to their shares of the
 *        gap: d_c = rho_c / s_c, rho_c = n_c . y + d_c(half-space), s_c the
 *        vertex side's share (so d_c = phi_c at y = 0).  A contact is active
 *        while d_c < delta, and the vertex takes its share s_c of the pair's
 *        correction: the vertex constraint is s_c C_c = s_c delta - rho_c with
 *        gradient -n_c, one XPBD update per iteration with the multiplier
 *        starting at zero (the constraint set is rebuilt every iteration):
 *        dn = w (s_c C_c) / (w + alpha~_c), alpha~_c = alpha / (w_c dt^2).
 *        A contact with w_c = 0 is fully occluded and skipped.
 *   -    the visibility product runs over the vertex's other active
 *        contacts; delta_v = 0 gives every weight 1.
 *   -    the active contacts are applied one after another, innermost first
 *        (ascending d_c at the proposal, ties by key), each on the
 *        displacement the previous ones left; friction after each: with t the
 *        tangential part of the current displacement, t is removed if
 *        |t| < mu_s dn (static), else scaled down by min(mu_k dn / |t|, 1).
 *   -    the response acts on the pairs of the vertex's region (phi < 2r);
 *        every repulsion range of the paper's scenes is below 2r.
 */
#include "ccfr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* cubic smoothstep on [0, 1] */
static double smoothstep(double t) {
    if (t <= 0.0) return 0.0;
    if (t >= 1.0) return 1.0;
    return t * t * (3.0 - 2.0 * t);
}

typedef struct { double d; uint64_t key; int64_t idx; double weight; } active_t;

static int cmp_active(const void* a, const void* b) {
    const active_t* p = (const active_t*)a;
    const active_t* q = (const active_t*)b;
    if (p->d < q->d) return -1;
    if (p->d > q->d) return 1;
    return p->key < q->key ? -1 : (p->key > q->key ? 1 : 0);
}

void orc_apply_response(const orc_params* prm, double w, const orc_halfspace* C, int64_t nC, double dt,
                        const double y_in[3], double y_out[3]) {
    memcpy(y_out, y_in, sizeof(double) * 3);
    if (!prm->response || w == 0.0 || nC == 0 || !(prm->delta > 0.0)) return;
    active_t* A = (active_t*)malloc(sizeof(active_t) * (size_t)nC);
    int64_t na = 0;
    for (int64_t k = 0; k < nC; ++k) {
        if (!(C[k].share > 0.0)) continue;
        const double rho = dot3(C[k].n, y_in) + C[k].d;
        const double d = rho / C[k].share;                         /* gap at the proposal */
        if (d < prm->delta) {
            A[na].d = d;
            A[na].key = C[k].key;
            A[na].idx = k;
            na++;
        }
    }
    for (int64_t i = 0; i < na; ++i) {                             /* visibility weights */
        double wc = 1.0;
        if (prm->vis_width > 0.0)
            for (int64_t j = 0; j < na; ++j)
                if (j != i) wc *= 1.0 - smoothstep((A[i].d - A[j].d) / prm->vis_width);
        A[i].weight = wc;
    }
    qsort(A, (size_t)na, sizeof(active_t), cmp_active);            /* innermost first */
    double y[3] = {y_in[0], y_in[1], y_in[2]};
    for (int64_t i = 0; i < na; ++i) {
        if (!(A[i].weight > 0.0)) continue;
        const orc_halfspace* c = &C[A[i].idx];
        const double rho = dot3(c->n, y) + c->d;
        const double cv = c->share * prm->delta - rho;             /* s_c C_c */
        if (!(cv > 0.0)) continue;
        const double at = prm->resp_compliance / (A[i].weight * dt * dt);
        const double dn = w * cv / (w + at);
        for (int k = 0; k < 3; ++k) y[k] += dn * c->n[k];
        if (prm->mu_s > 0.0 || prm->mu_k > 0.0) {
            const double yn = dot3(c->n, y);
            double t[3] = {y[0] - yn * c->n[0], y[1] - yn * c->n[1], y[2] - yn * c->n[2]};
            const double lt = sqrt(dot3(t, t));
            double f = 0.0;
            if (lt < prm->mu_s * dn) f = 1.0;
            else if (lt > 0.0) f = fmin(prm->mu_k * dn / lt, 1.0);
            for (int k = 0; k < 3; ++k) y[k] -= f * t[k];
        }
    }
    memcpy(y_out, y, sizeof(double) * 3);
    free(A);
}

void orc_response(const orc_mesh* m, const orc_params* prm, const int64_t* offsets, const orc_halfspace* hs,
                  double dt, const double* y_in, double* y_out) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int32_t v = 0; v < m->n_verts; ++v)
        orc_apply_response(prm, m->inv_mass[v], hs + offsets[v], offsets[v + 1] - offsets[v], dt,
                           y_in + 3 * (size_t)v, y_out + 3 * (size_t)v);
}
