/*
 * ccfr_oracle.h -- FP64 CPU oracle of the Convex Collision-Free Regions (CCFR)
 * hot path: candidate primitive pairs, per-vertex half-space regions, the
 * per-vertex projection onto a region, and the plain XPBD step around them.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, deliberately literal CPU
 * implementation written from the paper (Kikuchi & Kanai, "Convex Collision-Free
 * Regions"): Eq. 1-3 (Sec. 3.1), the numerical treatment of Sec. 3.2, and
 * Algorithms 1-4 (Appendices A-D).  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header, table or
 * helper with the HIP library, and the library never calls it.
 *
 * Precision: every geometric and projection quantity is FP64.  Inputs that the
 * GPU path receives in FP32 (positions, inverse masses) are passed here as the
 * same FP32 values widened exactly to FP64.  The one exception is the broad-phase
 * box test, which the candidate contract defines in FP32 (see oracle_candidates.c).
 *
 * Conventions: positions are [N][3] row-major, triangles [T][3], edges [E][2]
 * with a < b.  Every output array is caller-allocated; functions that produce
 * variable-length lists take a capacity, write at most that many entries and
 * return the full count, so a caller can size a second call.
 */
#ifndef CCFR_ORACLE_H
#define CCFR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Collision parameters (metres).  Sec. 3.1 (search radius r), Sec. 3.2
 * (retraction epsilon), App. A (ERO-line tolerance), App. B (pass budget),
 * Sec. 4.1 (box padding r + xi/2 + delta/2). */
typedef struct {
    double r;            /* search radius = per-iteration displacement bound      */
    double xi;           /* offset: minimum separation                             */
    double delta;        /* repulsion range (only pads the boxes here)             */
    double guard;        /* extra box padding keeping the FP32 box test conservative */
    double eps_retract;  /* retraction margin of Alg. 2                            */
    double eps_plesnik;  /* tolerance of Alg. 1                                     */
    int32_t max_passes;  /* n_maxIterations of Alg. 2                               */
    int32_t response;    /* 1: applyResponse (Sec. 3.3) between the XPBD constraints and the projection */
    double resp_compliance; /* alpha = 1/k of the response constraint                */
    double vis_width;    /* delta_v of the visibility weights (0: every weight is 1) */
    double mu_s, mu_k;   /* static and kinetic friction coefficients                 */
} orc_params;

/* Read-only view of one (possibly concatenated) mesh. */
typedef struct {
    int32_t n_verts, n_tris, n_edges, pad_;
    const double*  x;         /* [N][3] current (anchor) positions                   */
    const double*  inv_mass;  /* [N]    inverse masses, 0 = static / pinned           */
    const int32_t* tris;      /* [T][3]                                                */
    const int32_t* edges;     /* [E][2]                                                */
} orc_mesh;

/* One half-space of a vertex region: the vertex displacement y is admissible
 * iff n . y + d >= 0 (Alg. 2's rho).  phi is the pair's separation measure
 * (Alg. 3), key identifies the primitive pair (kind << 62 | a << 31 | b). */
typedef struct {
    double n[3];
    double d;
    double phi;
    double share;      /* the vertex side's share s of the pair's gap: d = s phi */
    uint64_t key;
    int32_t fragile;   /* 1 if a decision behind this entry sat near a threshold */
    int32_t pad_;
} orc_halfspace;

enum { ORC_KIND_VE = 0, ORC_KIND_VF = 1, ORC_KIND_EE = 2, ORC_KIND_VV = 3 };

/* ---- closest points (App. C: closestPointOnFace / closestPointOnEdge) ---- */
/* Closest point q on triangle (a, b, c) to p, with barycentrics bary (q = sum bary_i v_i).
 * Returns 0, or -1 if the triangle is degenerate (zero area). */
int orc_closest_point_triangle(const double p[3], const double a[3], const double b[3],
                               const double c[3], double q[3], double bary[3]);
/* Closest points p = (1-s) a + s b and q = (1-t) c + t d between two segments.
 * Returns 0, 1 if the segments were treated as parallel, -1 if one is degenerate. */
int orc_closest_points_segments(const double a[3], const double b[3], const double c[3],
                                const double d[3], double* s, double* t);
/* Closest point (1-t) a + t b on segment ab to p; -1 for a zero-length segment. */
int orc_closest_point_segment(const double p[3], const double a[3], const double b[3], double* t);

/* ---- candidates (Sec. 4.1 broad phase; contract: FP32 padded boxes) ---- */
float orc_box_pad(const orc_params* prm);
/* All candidate pairs, by brute force over every primitive pair, each list in
 * ascending lexicographic order.  counts[0..3] receive |VF|, |EE|, |VV|, |VE|
 * (VE: free particle, edge). */
void orc_candidates(const orc_mesh* m, const orc_params* prm,
                    int32_t* vf, int64_t cap_vf, int32_t* ee, int64_t cap_ee,
                    int32_t* vv, int64_t cap_vv, int32_t* ve, int64_t cap_ve, int64_t counts[4]);
/* Partners of one primitive, by brute force (ascending). */
int64_t orc_vf_tris_of_vertex(const orc_mesh* m, const orc_params* prm, int32_t v,
                              int32_t* out, int64_t cap);
int64_t orc_vf_verts_of_tri(const orc_mesh* m, const orc_params* prm, int32_t t,
                            int32_t* out, int64_t cap);
int64_t orc_ee_partners_of_edge(const orc_mesh* m, const orc_params* prm, int32_t e,
                                int32_t* out, int64_t cap);
int64_t orc_vv_partners_of_vertex(const orc_mesh* m, const orc_params* prm, int32_t v,
                                  int32_t* out, int64_t cap);
int64_t orc_ve_edges_of_vertex(const orc_mesh* m, const orc_params* prm, int32_t v, int32_t* out, int64_t cap);
int64_t orc_ve_verts_of_edge(const orc_mesh* m, const orc_params* prm, int32_t e, int32_t* out, int64_t cap);

/* ---- regions (Alg. 3 per vertex) ---- */
/* Regions of every vertex from the candidate lists.  offsets has N+1 entries.
 * Returns the total number of half-spaces H (entries written: min(H, cap)).
 * stats[0] receives the number of degenerate pairs skipped. */
int64_t orc_regions(const orc_mesh* m, const orc_params* prm,
                    const int32_t* vf, int64_t n_vf, const int32_t* ee, int64_t n_ee,
                    const int32_t* vv, int64_t n_vv, const int32_t* ve, int64_t n_ve,
                    int64_t* offsets, orc_halfspace* hs, int64_t cap, int64_t stats[4]);
/* Region of one vertex, its passive sets found by brute force. */
int64_t orc_vertex_region(const orc_mesh* m, const orc_params* prm, int32_t v,
                          orc_halfspace* hs, int64_t cap);

/* ---- projection (Alg. 2 with Alg. 1, the retraction of Sec. 3.2, the r-ball
 *      clamp of Alg. 4) ---- */
/* Per vertex v: region hs[offsets[v] .. offsets[v+1]), proposed displacement
 * y_in[v] = x' - x.  Writes y_out[v] = x* - x, halted[v] (1 = fallback to x),
 * fragile[v] (1 = some decision sat within the margin of its threshold).
 * stats: [0] vertices with a violated half-space, [1] halted, [2] fragile,
 * [3] Alg. 1 calls. */
void orc_project(const orc_mesh* m, const orc_params* prm,
                 const int64_t* offsets, const orc_halfspace* hs,
                 const double* y_in, double* y_out, int8_t* halted, int8_t* fragile,
                 int64_t stats[4]);
/* Same for a single vertex with an explicit half-space list (no mesh). */
int orc_project_one(const orc_params* prm, double inv_mass, const double x[3],
                    const orc_halfspace* hs, int64_t n_hs, const double y_in[3],
                    double y_out[3], int* fragile);
/* Every result the projection of one vertex can take when its near-threshold
 * decisions (those that make a vertex fragile) go either way: one run per
 * branch of the decision tree, at most cap runs.  Writes y_outs [n][3] and
 * halts [n], returns n; *complete = 0 if the tree had more than cap branches
 * (or a branch more than 64 decisions). */
int orc_project_branches(const orc_params* prm, double inv_mass, const double x[3],
                         const orc_halfspace* hs, int64_t n_hs, const double y_in[3],
                         double* y_outs, int8_t* halts, int cap, int* complete);
/* Counts of fragility flags raised so far, by rule: [0] sign of rho, [1] order of
 * two violated half-spaces, [2] comparison with eps_plesnik. */
void orc_fragile_reasons(int64_t out[3], int reset);
/* Alg. 1 on its own: adds plane (n, b) to the ERO state and updates xt.
 * state = { m, V[3][3], A[3][3], B[3] } packed as 1 + 9 + 9 + 3 doubles. */
void orc_orthogonal_projection(double xt[3], const double x0[3], const double n[3], double b,
                               double state[22], double eps);

/* ---- response and friction (Sec. 3.3, applyResponse of Alg. 4) ---- */
/* One vertex: its region (built at the anchor) and proposed displacement
 * y_in; returns the displacement after the response and friction of its
 * active contacts.  dt is the substep's time step. */
void orc_apply_response(const orc_params* prm, double inv_mass, const orc_halfspace* hs, int64_t n_hs,
                        double dt, const double y_in[3], double y_out[3]);
/* Every vertex (offsets/hs as for orc_project). */
void orc_response(const orc_mesh* m, const orc_params* prm, const int64_t* offsets, const orc_halfspace* hs,
                  double dt, const double* y_in, double* y_out);

/* ---- plain XPBD step (Alg. 4) ---- */
typedef struct {
    double dt;
    double g[3];
    int32_t iters;
    int32_t n_colors;      /* filled by orc_color_edges */
    double alpha;          /* stretch compliance */
    int32_t early_exit;    /* 1: evaluateConvergence ends the iterations (the reading in oracle_xpbd.c) */
    int32_t pad_;
    double conv_tol;       /* largest shortfall |p - x| - |y*| that counts as converged */
} orc_step_params;

/* Greedy edge colouring in edge-index order (vertex-disjoint colour classes). */
int32_t orc_color_edges(int32_t n_verts, int32_t n_edges, const int32_t* edges, int32_t* color);
/* One substep in place on x, v ([N][3], FP64).  rest_len [E].  color [E].
 * counters (nullable, summed over iterations): [0] VF, [1] EE, [2] VV candidates,
 * [3] half-spaces, [4] violating vertices, [5] halted vertices, [6] fragile
 * vertices, [7] degenerate pairs, [8] iterations run; [9] the longest run of
 * consecutive iterations in which one vertex halted (maximum over steps),
 * [10] halts that extended a run to 2, [11] halts that extended a run to 3 or
 * more.  trace (nullable, [iters][N][3]) receives the
 * anchor after every iteration. */
void orc_xpbd_step(int32_t n_verts, int32_t n_tris, int32_t n_edges,
                   const int32_t* tris, const int32_t* edges, const double* inv_mass,
                   const double* rest_len, const int32_t* color, int32_t n_colors,
                   double* x, double* v, const orc_params* prm, const orc_step_params* sp,
                   int64_t counters[12], double* trace);

/* ---- checks (independent of the routines above) ---- */
/* Exact signs of orientation determinants (Shewchuk's floating-point filter
 * with an exact expansion-arithmetic fallback): orient3d is the sign of
 * (b - a) . ((c - a) x (d - a)), orient2d of the 2-D (b - a) x (c - a). */
int orc_orient3d_sign(const double* a, const double* b, const double* c, const double* d);
int orc_orient2d_sign(const double* a, const double* b, const double* c);
/* Number of (edge, triangle) pairs sharing no vertex whose closed segment meets
 * the closed triangle, decided with the exact predicates (a coplanar segment
 * that touches the triangle counts; a triangle of zero area is skipped): any
 * such pair means two triangles interpenetrate or touch. */
int64_t orc_count_edge_tri_intersections(int32_t n_verts, const double* x, int32_t n_tris,
                                         const int32_t* tris, int32_t n_edges,
                                         const int32_t* edges);
/* Minimum distance over non-adjacent VF, EE, free-particle VV and VE pairs closer
 * than `reach` (returns reach if none), skipping pairs whose vertices all have
 * zero inverse mass; out_counts[k] counts pairs of kind k (0 VF, 1 EE, 2 VV,
 * 3 free particle - edge)
 * closer than `below`. */
double orc_min_separation(int32_t n_verts, const double* x, const double* inv_mass, int32_t n_tris,
                          const int32_t* tris, int32_t n_edges, const int32_t* edges, double reach,
                          double below, int64_t out_counts[4]);

/* The same check through a uniform grid (for large meshes): same pairs and
 * results as orc_min_separation. */
double orc_min_separation_grid(int32_t n_verts, const double* x, const double* inv_mass, int32_t n_tris,
                               const int32_t* tris, int32_t n_edges, const int32_t* edges, double reach,
                               double below, int64_t out_counts[4]);
/* Certified sampled check of the straight-line motion from x0 to x1 (one
 * iteration's anchor update): conservative advancement in t with the Lipschitz
 * bound 2 max |x1 - x0| of every pair distance.  Returns the smallest sampled
 * minimum distance (capped at reach); *certified = 1 when every distance stays
 * above floor_dist along the whole motion. */
double orc_motion_check(int32_t n_verts, const double* x0, const double* x1, const double* inv_mass,
                        int32_t n_tris, const int32_t* tris, int32_t n_edges, const int32_t* edges,
                        double floor_dist, double reach, int64_t max_samples, int32_t* certified,
                        int64_t* n_samples, double* t_min);

int orc_num_threads(void);
/* Threads of the OpenMP loops from now on (n > 0). */
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
