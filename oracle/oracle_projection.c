/*
 * oracle_projection.c -- projection of a proposed vertex position onto its
 * convex region: Algorithm 2 (projectOntoConvexRegion, App. B) calling
 * Algorithm 1 (orthogonalProjection, Plesnik's ERO-line update, App. A), the
 * epsilon retraction and halt fallback of Sec. 3.2, then the r-ball clamp of
 * Algorithm 4.  FP64, in world coordinates, as the paper writes it.
 *
 * TEST INFRASTRUCTURE ONLY (see ccfr_oracle.h).
 *
 * Readings of the printed algorithms:
 *   -    exact duplicate half-spaces (bitwise-equal n and d) are dropped before
 *        sorting; the one with the smallest key is kept.
 *   -    the ascending sort by rho breaks ties by ascending key.
 *   -    in Alg. 1's loop over j = 1..m, entry m is the plane being added
 *        (n_m, b_m), and the plane stored at the end is that same (n_m, b_m).
 *   -    one tolerance eps_plesnik for Alg. 1 and eps_retract for Alg. 2.
 *   -    once three independent planes are stored, Alg. 1 returns its input
 *        unchanged (in R^3 a fourth plane cannot be independent).
 *   -    max_passes is the literal loop count of Alg. 2: a pass that finds no
 *        violated half-space returns the position it started from; after
 *        max_passes passes with violations the vertex falls back to x (halt).
 *   -    the clamp |x* - x| <= r of Alg. 4 is applied after the projection, also
 *        to vertices with no half-space; static vertices (w = 0) do not move.
 *
 * Fragility.  A vertex is reported fragile when one of its discrete decisions
 * (the sign of rho, the order of two violated half-spaces, a comparison with
 * eps_plesnik) sat within a relative margin of its threshold, so that a
 * different rounding order could flip it.  The margins are test-side only.
 * Each such decision is numbered in the order it is met, and a caller may ask
 * for any of them to take its other outcome (orc_project_branches walks every
 * combination): the results of all branches are the results a correct
 * implementation that rounds differently may return.
 */
#include "ccfr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define REL_RHO 1e-9    /* sign of rho, order of near-equal rho        */
#define REL_EPS 1e-6    /* |beta| or |v_new| against eps_plesnik        */

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

typedef struct {
    int m;             /* |V| = |A| = |B| */
    double V[3][3];    /* ERO directions  */
    double A[3][3];    /* plane normals   */
    double B[3];       /* plane RHS       */
} ero_t;

typedef struct {
    int fragile;
    int n_dec;         /* near-threshold decisions met so far                */
    uint64_t flip;     /* decision k takes its other outcome if bit k is set */
} flags_t;

/* which rule flagged a vertex: [0] rho sign, [1] order of violated rho, [2] eps */
static int64_t g_reasons[3];

void orc_fragile_reasons(int64_t out[3], int reset) {
    for (int k = 0; k < 3; ++k) {
        out[k] = g_reasons[k];
        if (reset) g_reasons[k] = 0;
    }
}

/* A discrete decision whose default outcome is `out`: when it sits near its
 * threshold (`near`) the vertex is fragile and the decision may be flipped. */
static int decide(flags_t* f, int out, int near, int reason) {
    if (!f || !near) return out;
    f->fragile = 1;
#pragma omp atomic
    g_reasons[reason]++;
    const int k = f->n_dec++;
    if (k < 64 && ((f->flip >> k) & 1u)) return !out;
    return out;
}

static int near_eps(double mag, double eps) { return fabs(mag - eps) <= REL_EPS * eps; }

static void push(ero_t* S, const double v[3], const double n[3], double b) {
    memcpy(S->V[S->m], v, sizeof(double) * 3);
    memcpy(S->A[S->m], n, sizeof(double) * 3);
    S->B[S->m] = b;
    S->m++;
}

/* Algorithm 1: add plane n . x = b to the stored system and move xt to the
 * orthogonal projection of x0 onto the intersection of all stored planes. */
static void orthogonal_projection(double xt[3], const double x0[3], const double n[3], double b,
                                  ero_t* S, double eps, flags_t* fl) {
    if (S->m == 0) {
        double v0[3] = {n[0], n[1], n[2]};
        double beta0 = dot3(n, v0);
        if (decide(fl, fabs(beta0) < eps, near_eps(fabs(beta0), eps), 2)) return;
        double c = (b - dot3(n, xt)) / beta0;
        for (int k = 0; k < 3; ++k) xt[k] += c * v0[k];
        push(S, v0, n, b);
        return;
    }
    if (S->m == 3) return;                                         /* three planes stored */
    const int m = S->m;
    const double* n0 = S->A[0];
    const double b0 = S->B[0];
    const double* nm = n;
    const double bm = b;
    double dn[3] = {nm[0] - n0[0], nm[1] - n0[1], nm[2] - n0[2]};
    double beta_u = dot3(dn, S->V[m - 1]);
    double alpha_u = bm - dot3(nm, xt);
    if (decide(fl, fabs(beta_u) < eps, near_eps(fabs(beta_u), eps), 2)) return;
    double u[3], w[3];
    for (int k = 0; k < 3; ++k) u[k] = xt[k] + (alpha_u / beta_u) * S->V[m - 1][k];
    for (int k = 0; k < 3; ++k) w[k] = x0[k] + nm[k];
    for (int j = 1; j <= m; ++j) {
        const double* nj = (j < m) ? S->A[j] : nm;                 /* entry m: the new plane */
        const double bj = (j < m) ? S->B[j] : bm;
        double dnj[3] = {nj[0] - n0[0], nj[1] - n0[1], nj[2] - n0[2]};
        double beta_w = dot3(dnj, S->V[j - 1]);
        if (decide(fl, fabs(beta_w) > eps, near_eps(fabs(beta_w), eps), 2)) {
            double alpha_w = bj - b0 - dot3(dnj, w);
            for (int k = 0; k < 3; ++k) w[k] += (alpha_w / beta_w) * S->V[j - 1][k];
        }
    }
    double vnew[3] = {w[0] - u[0], w[1] - u[1], w[2] - u[2]};
    if (decide(fl, norm3(vnew) > eps, near_eps(norm3(vnew), eps), 2)) {
        double beta_new = dot3(n0, vnew);
        if (decide(fl, fabs(beta_new) < eps, near_eps(fabs(beta_new), eps), 2)) {
            memcpy(xt, u, sizeof(double) * 3);
        } else {
            double alpha_new = b0 - dot3(n0, u);
            for (int k = 0; k < 3; ++k) xt[k] = u[k] + (alpha_new / beta_new) * vnew[k];
        }
        push(S, vnew, nm, bm);                                     /* stored: the new plane */
    }
}

void orc_orthogonal_projection(double xt[3], const double x0[3], const double n[3], double b,
                               double state[22], double eps) {
    ero_t S;
    S.m = (int)state[0];
    memcpy(S.V, state + 1, sizeof(double) * 9);
    memcpy(S.A, state + 10, sizeof(double) * 9);
    memcpy(S.B, state + 19, sizeof(double) * 3);
    orthogonal_projection(xt, x0, n, b, &S, eps, NULL);
    state[0] = (double)S.m;
    memcpy(state + 1, S.V, sizeof(double) * 9);
    memcpy(state + 10, S.A, sizeof(double) * 9);
    memcpy(state + 19, S.B, sizeof(double) * 3);
}

typedef struct { double rho; uint64_t key; int64_t idx; } sort_item;

static int cmp_item(const void* a, const void* b) {
    const sort_item* p = (const sort_item*)a;
    const sort_item* q = (const sort_item*)b;
    if (p->rho < q->rho) return -1;
    if (p->rho > q->rho) return 1;
    if (p->key < q->key) return -1;
    if (p->key > q->key) return 1;
    return 0;
}

static int same_plane(const orc_halfspace* a, const orc_halfspace* b) {
    return a->n[0] == b->n[0] && a->n[1] == b->n[1] && a->n[2] == b->n[2] && a->d == b->d;
}

/* Algorithm 2 for one vertex; returns 1 if the vertex halted. */
static int project_vertex(const orc_params* prm, double w, const double x[3], const orc_halfspace* C,
                          int64_t nC, const double y_in[3], double y_out[3], int* violated,
                          flags_t* fl) {
    *violated = 0;
    if (w == 0.0) { y_out[0] = y_out[1] = y_out[2] = 0.0; return 0; }   /* static: no move */
    double xp[3] = {x[0] + y_in[0], x[1] + y_in[1], x[2] + y_in[2]};   /* x' */
    int halted = 0;
    if (nC > 0) {
        /* initial rho, sort ascending, drop exact duplicates */
        sort_item* it = (sort_item*)malloc(sizeof(sort_item) * (size_t)nC);
        for (int64_t k = 0; k < nC; ++k) {
            double dx[3] = {xp[0] - x[0], xp[1] - x[1], xp[2] - x[2]};
            it[k].rho = dot3(dx, C[k].n) + C[k].d;
            it[k].key = C[k].key;
            it[k].idx = k;
        }
        qsort(it, (size_t)nC, sizeof(sort_item), cmp_item);
        int64_t nk = 0;
        for (int64_t k = 0; k < nC; ++k) {
            int dup = 0;
            for (int64_t j = 0; j < nk && !dup; ++j)
                if (it[j].rho == it[k].rho && same_plane(&C[it[j].idx], &C[it[k].idx])) dup = 1;
            if (!dup) it[nk++] = it[k];
        }
        /* near-equal initial rho among violated half-spaces: their order may flip,
         * which matters unless the two planes are (nearly) the same plane */
        for (int64_t k = 1; k < nk; ++k) {
            if (it[k].rho < 0.0 && it[k - 1].rho < 0.0) {
                double sc = fabs(it[k].rho) + fabs(it[k - 1].rho);
                const orc_halfspace* a = &C[it[k].idx];
                const orc_halfspace* b = &C[it[k - 1].idx];
                double dn[3] = {a->n[0] - b->n[0], a->n[1] - b->n[1], a->n[2] - b->n[2]};
                int differ = norm3(dn) > 1e-7 || fabs(a->d - b->d) > 1e-7 * (fabs(a->d) + fabs(b->d)) + 1e-15;
                if (decide(fl, 0, differ && it[k].rho - it[k - 1].rho <= REL_RHO * sc, 1)) {
                    sort_item t = it[k];
                    it[k] = it[k - 1];
                    it[k - 1] = t;
                }
            }
        }
        if (nk > 0 && it[0].rho < 0.0) *violated = 1;

        halted = 1;
        for (int pass = 0; pass < prm->max_passes; ++pass) {
            double xt[3] = {xp[0], xp[1], xp[2]};
            double x0[3] = {xp[0], xp[1], xp[2]};
            int nviol = 0;
            ero_t S;
            S.m = 0;
            for (int64_t q = 0; q < nk; ++q) {
                const orc_halfspace* c = &C[it[q].idx];
                double dx[3] = {xt[0] - x[0], xt[1] - x[1], xt[2] - x[2]};
                double rho = dot3(dx, c->n) + c->d;
                double sc = norm3(dx) + fabs(c->d);
                if (decide(fl, rho >= 0.0, sc > 0.0 && fabs(rho) <= REL_RHO * sc, 0)) continue;
                double b = dot3(c->n, x) - c->d;
                nviol++;
                orthogonal_projection(xt, x0, c->n, b, &S, prm->eps_plesnik, fl);
                double D[3] = {xt[0] - x[0], xt[1] - x[1], xt[2] - x[2]};
                double nd = norm3(D);
                if (nd > prm->eps_retract) {
                    double f = (nd - prm->eps_retract) / nd;
                    for (int k = 0; k < 3; ++k) xt[k] = x[k] + f * D[k];
                } else {
                    memcpy(xt, x, sizeof(double) * 3);
                }
            }
            if (nviol == 0) { halted = 0; break; }
            memcpy(xp, xt, sizeof(double) * 3);
        }
        if (halted) memcpy(xp, x, sizeof(double) * 3);
        free(it);
    }
    /* r-ball clamp (Alg. 4) */
    double y[3] = {xp[0] - x[0], xp[1] - x[1], xp[2] - x[2]};
    double ny = norm3(y);
    if (ny > prm->r) {
        double f = prm->r / ny;
        for (int k = 0; k < 3; ++k) y[k] *= f;
    }
    memcpy(y_out, y, sizeof(double) * 3);
    return halted;
}

int orc_project_one(const orc_params* prm, double inv_mass, const double x[3],
                    const orc_halfspace* hs, int64_t n_hs, const double y_in[3],
                    double y_out[3], int* fragile) {
    flags_t fl = {0, 0, 0};
    int violated;
    int h = project_vertex(prm, inv_mass, x, hs, n_hs, y_in, y_out, &violated, &fl);
    if (fragile) *fragile = fl.fragile;
    return h;
}

void orc_project(const orc_mesh* m, const orc_params* prm,
                 const int64_t* offsets, const orc_halfspace* hs,
                 const double* y_in, double* y_out, int8_t* halted, int8_t* fragile,
                 int64_t stats[4]) {
    int64_t n_viol = 0, n_halt = 0, n_frag = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_viol, n_halt, n_frag)
    for (int32_t v = 0; v < m->n_verts; ++v) {
        flags_t fl = {0, 0, 0};
        int violated;
        int h = project_vertex(prm, m->inv_mass[v], m->x + 3 * (size_t)v, hs + offsets[v],
                               offsets[v + 1] - offsets[v], y_in + 3 * (size_t)v,
                               y_out + 3 * (size_t)v, &violated, &fl);
        if (halted) halted[v] = (int8_t)h;
        if (fragile) fragile[v] = (int8_t)fl.fragile;
        n_viol += violated;
        n_halt += h;
        n_frag += fl.fragile;
    }
    if (stats) { stats[0] = n_viol; stats[1] = n_halt; stats[2] = n_frag; stats[3] = 0; }
}

int orc_project_branches(const orc_params* prm, double inv_mass, const double x[3],
                         const orc_halfspace* hs, int64_t n_hs, const double y_in[3],
                         double* y_outs, int8_t* halts, int cap, int* complete) {
    /* Breadth-first walk of the tree of near-threshold decisions: a node fixes
     * the outcomes of its first `depth` decisions by `mask` (the rest default);
     * its children flip one later decision each. */
    typedef struct { uint64_t mask; int depth; } node_t;
    node_t* q = (node_t*)malloc(sizeof(node_t) * (size_t)(cap > 0 ? cap : 1));
    int head = 0, tail = 0, n_out = 0, full = 1;
    if (cap > 0) q[tail++] = (node_t){0, 0};
    while (head < tail) {
        node_t nd = q[head++];
        flags_t fl = {0, 0, nd.mask};
        int violated;
        double y[3];
        int h = project_vertex(prm, inv_mass, x, hs, n_hs, y_in, y, &violated, &fl);
        memcpy(y_outs + 3 * (size_t)n_out, y, sizeof(double) * 3);
        halts[n_out] = (int8_t)h;
        n_out++;
        const int nd_max = fl.n_dec < 64 ? fl.n_dec : 64;
        if (fl.n_dec > 64) full = 0;
        for (int i = nd.depth; i < nd_max; ++i) {
            if (tail >= cap) { full = 0; break; }
            q[tail++] = (node_t){nd.mask | ((uint64_t)1 << i), i + 1};
        }
    }
    free(q);
    if (complete) *complete = full;
    return n_out;
}
