/*
 * oracle_xpbd.c -- the plain XPBD substep around the CCFR calls (App. D,
 * Algorithm 4), FP64.
 *
 * TEST INFRASTRUCTURE ONLY (see ccfr_oracle.h).
 *
 * Reading of Algorithm 4 (no response, friction or early exit):
 *
 *   x~ = x + dt v + dt^2 g          (static / pinned vertices keep x)
 *   lambda = 0
 *   for it in 1..iters:
 *       candidates and regions at the anchor x           (broad + narrow phase)
 *       p = x~                                           ("initialize solve")
 *       one Gauss-Seidel pass over the stretch constraints, colour by colour,
 *         lambda carried over from the previous iterations
 *       applyResponse per vertex (with prm->response; oracle_response.c)
 *       y* = projectOntoConvexRegion(p - x), clamped to |y*| <= r
 *       x = x + y*
 *       evaluateConvergence (only with early_exit): stop once no dynamic
 *         vertex's step falls short of its expected advancement by more
 *         than conv_tol, max_v (|p_v - x_v| - |y*_v|) <= conv_tol
 *   v = (x - x_old) / dt
 *
 * Reading of the convergence check: the paper runs more iterations while
 * "the current step size falls short of the expected advancement"; the
 * expected advancement of an iteration is taken as the proposal displacement
 * p - x that the XPBD constraints ask for, the current step as y* after the
 * projection and the clamp, and the loop ends once every dynamic vertex's step
 * comes within conv_tol of its proposal.
 * Reading of the halting statistics: a run is a sequence of consecutive
 * iterations of one substep in which the same vertex halts; the step reports
 * the longest run and how many halts extended a run to length 2 or to 3 and
 * more.
 *
 * The stretch constraint of an edge (i, j) with rest length L is the XPBD
 * distance constraint C = |p_i - p_j| - L with compliance alpha (Macklin et al.
 * 2016): dlambda = (-C - alpha~ lambda) / (w_i + w_j + alpha~), alpha~ =
 * alpha / dt^2, p_i += w_i dlambda n, p_j -= w_j dlambda n.  Edges are coloured
 * greedily in index order so that a colour class shares no vertex; within a
 * class the order does not matter.
 */
#include "ccfr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t orc_color_edges(int32_t n_verts, int32_t n_edges, const int32_t* edges, int32_t* color) {
    /* colour(e) = the smallest colour not yet taken by an earlier edge sharing a
     * vertex with e; used[v] is the bitmask of colours taken at v */
    uint64_t* used = (uint64_t*)calloc((size_t)n_verts + 1, sizeof(uint64_t));
    int32_t n_colors = 0;
    for (int32_t e = 0; e < n_edges; ++e) {
        int32_t a = edges[2 * e], b = edges[2 * e + 1];
        uint64_t taken = used[a] | used[b];
        int32_t c = 0;
        while (c < 64 && ((taken >> c) & 1u)) ++c;
        if (c == 64) { free(used); return -1; }
        color[e] = c;
        used[a] |= (uint64_t)1 << c;
        used[b] |= (uint64_t)1 << c;
        if (c + 1 > n_colors) n_colors = c + 1;
    }
    free(used);
    return n_colors;
}

static void stretch_pass(int32_t n_edges, const int32_t* edges, const double* w, const double* rest,
                         const int32_t* color, int32_t n_colors, double* p, double* lambda,
                         double alpha_t) {
    for (int32_t c = 0; c < n_colors; ++c) {
        for (int32_t e = 0; e < n_edges; ++e) {
            if (color[e] != c) continue;
            int32_t i = edges[2 * e], j = edges[2 * e + 1];
            double W = w[i] + w[j];
            if (W == 0.0) continue;
            double dv[3] = {p[3 * i] - p[3 * j], p[3 * i + 1] - p[3 * j + 1], p[3 * i + 2] - p[3 * j + 2]};
            double len = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
            if (len == 0.0) continue;
            double C = len - rest[e];
            double dl = (-C - alpha_t * lambda[e]) / (W + alpha_t);
            for (int k = 0; k < 3; ++k) {
                double nk = dv[k] / len;
                p[3 * i + k] += w[i] * dl * nk;
                p[3 * j + k] -= w[j] * dl * nk;
            }
            lambda[e] += dl;
        }
    }
}

void orc_xpbd_step(int32_t n_verts, int32_t n_tris, int32_t n_edges,
                   const int32_t* tris, const int32_t* edges, const double* inv_mass,
                   const double* rest_len, const int32_t* color, int32_t n_colors,
                   double* x, double* v, const orc_params* prm, const orc_step_params* sp,
                   int64_t counters[12], double* trace) {
    const size_t N3 = 3 * (size_t)n_verts;
    double* x_old = (double*)malloc(sizeof(double) * N3);
    double* xt = (double*)malloc(sizeof(double) * N3);
    double* p = (double*)malloc(sizeof(double) * N3);
    double* y = (double*)malloc(sizeof(double) * N3);
    double* ys = (double*)malloc(sizeof(double) * N3);
    double* lambda = (double*)calloc((size_t)n_edges + 1, sizeof(double));
    int64_t* offsets = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n_verts + 1));
    int8_t* halted = (int8_t*)malloc((size_t)n_verts + 1);
    int32_t* run = (int32_t*)calloc((size_t)n_verts + 1, sizeof(int32_t));   /* consecutive halts */
    int64_t iters_run = 0, max_run = 0, runs2 = 0, runs3 = 0;
    memcpy(x_old, x, sizeof(double) * N3);
    const double dt = sp->dt;
    for (int32_t i = 0; i < n_verts; ++i)
        for (int k = 0; k < 3; ++k)
            xt[3 * i + k] = inv_mass[i] > 0.0 ? x[3 * i + k] + dt * v[3 * i + k] + dt * dt * sp->g[k]
                                              : x[3 * i + k];
    const double alpha_t = sp->alpha / (dt * dt);
    orc_mesh m = {n_verts, n_tris, n_edges, 0, x, inv_mass, tris, edges};

    for (int32_t it = 0; it < sp->iters; ++it) {
        /* broad phase at the anchor */
        int64_t cnt[4];
        orc_candidates(&m, prm, NULL, 0, NULL, 0, NULL, 0, NULL, 0, cnt);
        int32_t* vf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * cnt[0] + 2));
        int32_t* ee = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * cnt[1] + 2));
        int32_t* vv = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * cnt[2] + 2));
        int32_t* ve = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * cnt[3] + 2));
        orc_candidates(&m, prm, vf, cnt[0], ee, cnt[1], vv, cnt[2], ve, cnt[3], cnt);
        /* narrow phase */
        int64_t rstats[4];
        int64_t H = orc_regions(&m, prm, vf, cnt[0], ee, cnt[1], vv, cnt[2], ve, cnt[3], offsets, NULL, 0, rstats);
        orc_halfspace* hs = (orc_halfspace*)malloc(sizeof(orc_halfspace) * (size_t)(H + 1));
        orc_regions(&m, prm, vf, cnt[0], ee, cnt[1], vv, cnt[2], ve, cnt[3], offsets, hs, H, rstats);
        /* XPBD constraints from the prediction */
        memcpy(p, xt, sizeof(double) * N3);
        stretch_pass(n_edges, edges, inv_mass, rest_len, color, n_colors, p, lambda, alpha_t);
        /* response and friction (Sec. 3.3), then the projection of the
         * proposed displacement and the anchor update */
        for (size_t k = 0; k < N3; ++k) y[k] = p[k] - x[k];
        if (prm->response) {
            orc_response(&m, prm, offsets, hs, dt, y, ys);
            memcpy(y, ys, sizeof(double) * N3);
        }
        int64_t pstats[4];
        orc_project(&m, prm, offsets, hs, y, ys, halted, NULL, pstats);
        for (size_t k = 0; k < N3; ++k) x[k] += ys[k];
        if (trace) memcpy(trace + (size_t)it * N3, x, sizeof(double) * N3);
        iters_run++;
        double shortfall = 0.0;
        for (int32_t i = 0; i < n_verts; ++i) {
            if (inv_mass[i] == 0.0) continue;
            const double* a = y + 3 * (size_t)i;
            const double* b = ys + 3 * (size_t)i;
            double sf = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) - sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
            if (sf > shortfall) shortfall = sf;
            if (halted[i]) {
                run[i]++;
                if (run[i] > max_run) max_run = run[i];
                if (run[i] == 2) runs2++;
                if (run[i] >= 3) runs3++;
            } else {
                run[i] = 0;
            }
        }
        if (counters) {
            counters[0] += cnt[0]; counters[1] += cnt[1]; counters[2] += cnt[2] + cnt[3];
            counters[3] += H; counters[4] += pstats[0]; counters[5] += pstats[1];
            counters[6] += pstats[2]; counters[7] += rstats[0];
        }
        free(vf); free(ee); free(vv); free(ve); free(hs);
        if (sp->early_exit && shortfall <= sp->conv_tol) break;
    }
    if (counters) {
        counters[8] += iters_run;
        if (max_run > counters[9]) counters[9] = max_run;
        counters[10] += runs2;
        counters[11] += runs3;
    }
    free(halted); free(run);
    for (size_t k = 0; k < N3; ++k) v[k] = (x[k] - x_old[k]) / dt;
    free(x_old); free(xt); free(p); free(y); free(ys); free(lambda); free(offsets);
}
