/*
 * ccfr.h -- C ABI of the MI355X (gfx950) implementation of the data-parallel hot
 * path of Convex Collision-Free Regions (Kikuchi & Kanai, "Convex Collision-Free
 * Regions"): per solver iteration,
 *
 *   ccfr_build_candidates       broad phase: primitive pairs whose padded boxes
 *                               overlap (Sec. 4.1)
 *   ccfr_build_regions          narrow phase: every vertex's convex region as
 *                               half-spaces on its displacement (Eq. 1-3, Alg. 3)
 *   ccfr_project_displacements  projection of proposed displacements onto the
 *                               regions (Alg. 2 with Alg. 1, Sec. 3.2) and the
 *                               r-ball clamp (Alg. 4)
 *   ccfr_xpbd_step              the plain XPBD substep that calls the three
 *                               (Alg. 4, without response or friction)
 *
 * plus batched entry points that run many independent meshes in one set of
 * launches per step.
 *
 * General rules
 *  - Every function returns a ccfr_status (0 = OK, negative = error) and never
 *    throws.  Argument errors are detected before anything is enqueued and
 *    leave outputs untouched.
 *  - Array arguments named `*_dev` or documented as "device" are device
 *    pointers (for example torch tensor data pointers) owned by the caller,
 *    contiguous, float32 or int32 as stated.  Host arrays are read during the
 *    call only.
 *  - All device work is enqueued on the given HIP stream and returns without
 *    waiting.  Errors found on the device (capacity overflow, non-finite input)
 *    set sticky bits in the context's status word, read by ccfr_sync_status,
 *    the only call that waits for the stream.  Outputs of a call whose status
 *    bits are set are undefined.
 *  - A context may be used from one host thread at a time; calls that share a
 *    context must be issued on one stream or otherwise ordered by the caller.
 *  - Units are metres and seconds.  Positions are [N][3] float32, packed.
 */
#ifndef CCFR_H
#define CCFR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* ccfr_stream;   /* hipStream_t; NULL = the null stream */

typedef enum {
    CCFR_OK = 0,
    CCFR_ERR_INVALID_ARG = -1,   /* bad pointer, size or parameter                      */
    CCFR_ERR_CAPACITY = -2,      /* a device list outgrew its buffer (see ccfr_status_info) */
    CCFR_ERR_HIP = -3,           /* a HIP runtime call failed                            */
    CCFR_ERR_NONFINITE = -4,     /* a position or displacement was NaN or infinite       */
    CCFR_ERR_DEGENERATE = -5,    /* reserved: degenerate primitives are skipped and counted */
    CCFR_ERR_NOT_READY = -6,     /* batch slot or graph not in a usable state           */
    CCFR_ERR_NO_MEMORY = -7      /* a device allocation failed                          */
} ccfr_status;

/* Collision parameters of one mesh (Sec. 3.1-3.3, Sec. 4.1, App. A-B). */
typedef struct {
    float r;            /* search radius; pairs are kept while phi < 2r, and no vertex
                           moves more than r per iteration (Alg. 4 clamp)              */
    float xi;           /* offset: minimum separation (phi = distance - xi)             */
    float delta;        /* repulsion range (Sec. 3.3): widens the boxes (Sec. 4.1) and,
                           with CCFR_FLAG_RESPONSE, is the range of the soft response  */
    float guard;        /* extra box padding keeping the FP32 box test conservative     */
    float eps_retract;  /* retraction margin of Alg. 2 (Sec. 3.2), e.g. 1e-6 m          */
    float eps_plesnik;  /* tolerance of Alg. 1, e.g. 1e-6                                */
    int32_t max_passes; /* pass budget of Alg. 2 (its n_maxIterations), >= 1            */
    int32_t flags;      /* CCFR_FLAG_RESPONSE or 0                                       */
    /* soft response and friction (Sec. 3.3), used with CCFR_FLAG_RESPONSE only */
    float resp_compliance; /* alpha = 1/k of the response constraint, >= 0           */
    float vis_width;    /* delta_v of the visibility weights (0: every weight is 1)     */
    float mu_s, mu_k;   /* static and kinetic friction coefficients, >= 0              */
} ccfr_params;

/* ccfr_params.flags: run applyResponse of Alg. 4 (the soft response with
 * visibility weights and friction of Sec. 3.3) between the XPBD constraints and
 * the projection of every iteration.  Needs 0 < delta <= 2r (the response acts
 * on the pairs of the vertex's region). */
#define CCFR_FLAG_RESPONSE 1

/* One half-space of a vertex region (Alg. 2's constraint tuple): a displacement
 * y of the vertex is admissible iff n . y + d >= 0.  phi is the pair's
 * separation measure (distance - xi), share the vertex side's share s of it
 * (d = s phi, Eq. 2), key = kind << 62 | a << 31 | b names the primitive pair
 * (kind 0 = particle-edge (free particle a, edge b), 1 = vertex-face (vertex a,
 * triangle b), 2 = edge-edge (edges a < b), 3 = point-point (particles a < b)).
 * 32 bytes. */
typedef struct {
    float n[3];
    float d;
    float phi;
    float share;
    uint64_t key;
} ccfr_halfspace;

/* Candidate pair lists (Sec. 4.1, Alg. 3 inputs, and the point interactions
 * of Sec. 4.2).  Pointers are device memory.  counts_dev[0..3] hold |VF|, |EE|,
 * |VV|, |VE| on the device after the build; a count above its capacity means
 * the list overflowed (CCFR_ERR_CAPACITY). */
typedef struct {
    int32_t* vf;          /* [cap_vf][2]: (vertex, triangle), vertex not in triangle  */
    int32_t* ee;          /* [cap_ee][2]: (e, e') with e < e', sharing no vertex       */
    int32_t* vv;          /* [cap_vv][2]: free particles (i, j), i < j                 */
    int32_t* counts_dev;  /* [4]                                                       */
    int64_t cap_vf, cap_ee, cap_vv;
    int32_t* ve;          /* [cap_ve][2]: (free particle, edge)                        */
    int64_t cap_ve;
} ccfr_candidates;

/* Per-vertex regions in CSR form.  Pointers are device memory: the half-spaces
 * of vertex v are hs[offsets[v] .. offsets[v+1]), in no particular order. */
typedef struct {
    int32_t n_verts;
    int32_t pad_;
    int32_t* offsets;     /* [n_verts + 1] */
    ccfr_halfspace* hs;   /* [cap]         */
    int64_t cap;
} ccfr_regions;

/* XPBD substep parameters (Alg. 4). */
typedef struct {
    float dt;
    float gravity[3];
    int32_t iters;       /* solver iterations; each runs candidates, regions, one
                            stretch pass and the projection                        */
    float alpha;         /* stretch compliance (XPBD distance constraints)         */
    ccfr_params collision;
    int32_t early_exit;  /* 0: exactly `iters` iterations.  1: the convergence
                            check of Alg. 4 ends them early: after an iteration
                            whose every dynamic vertex's step |y*| came within
                            conv_tol of its proposal |p - x| (the expected
                            advancement: nothing clamped or projected away),
                            the remaining iterations are skipped on the device */
    float conv_tol;      /* metres, >= 0 (early_exit only)                          */
} ccfr_step_params;

/* Device-side status and counters, copied out by ccfr_sync_status. */
typedef struct {
    uint32_t status_bits;   /* sticky: 1 VF, 2 EE, 4 VV, 128 VE, 8 half-spaces, 16
                               large primitives, 32 contacts overflowed; 64
                               non-finite                                           */
    int32_t last_counts[3]; /* |VF|, |EE|, |VV| of the last candidate build          */
    int32_t last_contacts;  /* pairs with phi < 2r in the last region build          */
    int32_t last_halfspaces;/* half-spaces in the last region build                  */
    int64_t need[6];        /* largest sizes seen since the last reset: VF, EE, VV,
                               contacts, half-spaces, large primitives               */
    int64_t totals[10];     /* accumulated since the last reset: [0..2] VF, EE, VV
                               pairs, [3] half-spaces, [4] violating vertices, [5]
                               halted vertices, [6] degenerate pairs, [7] projected
                               vertices, [8] contacts (pairs with phi < 2r), [9]
                               region builds                                        */
    int64_t candidate_builds; /* candidate builds closed since the last reset (the
                               pair totals are summed over these)                   */
    int64_t iterations_run; /* solver iterations of substeps run since the last
                               reset (fewer than iters x substeps with early_exit)  */
    int64_t halt_runs[2];   /* halts that made a vertex halt in 2, and in 3 or more,
                               consecutive iterations of one substep                */
    int32_t max_halt_run;   /* longest such run of one vertex (Sec. 4.3 reports at
                               most 2 consecutive halts)                            */
    int32_t last_ve;        /* |VE| of the last candidate build                       */
    int64_t need_ve;        /* largest |VE| seen since the last reset                 */
    int64_t total_ve;       /* VE pairs accumulated since the last reset              */
} ccfr_status_info;

typedef struct ccfr_ctx ccfr_ctx;
typedef struct ccfr_mesh ccfr_mesh;
typedef struct ccfr_batch ccfr_batch;

/* Static text for a status code. */
const char* ccfr_status_string(int code);

/* Context on HIP device `device`: owns the workspace (grid, candidate lists,
 * regions, scratch) and the device status word.  Capacities grow on demand
 * through ccfr_reserve; the initial sizes come from the first mesh used. */
int ccfr_create(ccfr_ctx** out, int device);
void ccfr_destroy(ccfr_ctx* ctx);

/* Device copy of one mesh (host arrays in, copied during the call):
 *  tris [n_tris][3], edges [n_edges][2] (a < b; NULL: derived from the
 *  triangles, unique and sorted), inv_mass [n_verts] (0 = static or pinned),
 *  rest_x [n_verts][3] (NULL: no stretch constraints).  Builds the stretch rest
 *  lengths, the greedy edge colouring used by the Gauss-Seidel pass, the list of
 *  free particles (vertices in no edge and no triangle) and the grid cell size.
 *  Vertex, triangle and (derived) edge counts are at most 2^30; more, an index
 *  out of range or an edge (a, a) is CCFR_ERR_INVALID_ARG. */
int ccfr_mesh_create(ccfr_ctx* ctx, int32_t n_verts, const int32_t* tris, int32_t n_tris,
                     const int32_t* edges, int32_t n_edges, const float* inv_mass,
                     const float* rest_x, ccfr_mesh** out);
void ccfr_mesh_destroy(ccfr_mesh* mesh);
/* Edge count after derivation, and a copy of the (possibly derived) edges. */
int ccfr_mesh_edges(const ccfr_mesh* mesh, int32_t* n_edges, int32_t* edges_host /* nullable */);
/* Device pointer to the mesh's inverse masses [n_verts] (float32). */
const float* ccfr_mesh_inv_mass_dev(const ccfr_mesh* mesh);

/* Grow the workspace so that lists of the given sizes fit (0 keeps a size).
 * Waits for the context's previous work.  Invalidates captured step graphs. */
int ccfr_reserve(ccfr_ctx* ctx, int64_t vf, int64_t ee, int64_t vv, int64_t ve, int64_t contacts,
                 int64_t halfspaces, ccfr_stream stream);

/* Broad phase (Sec. 4.1): every vertex-face, edge-edge, particle-particle and
 * particle-edge pair whose padded FP32 boxes overlap, with pad = fl32(r + xi/2 + delta/2 + guard)
 * and per axis lo = fl32(min - pad), hi = fl32(max + pad); pairs whose vertices
 * all have zero inverse mass are skipped.  x_anchor_dev: [n_verts][3] device
 * (may be NULL for a mesh with no vertices).  A primitive with a non-finite
 * coordinate is left out and raises the non-finite status bit.
 * On return `out` views the context's lists, valid until the next build on ctx. */
int ccfr_build_candidates(ccfr_ctx* ctx, const ccfr_mesh* mesh, const float* x_anchor_dev,
                          const ccfr_params* params, ccfr_candidates* out, ccfr_stream stream);

/* Narrow phase (Alg. 3 with Eq. 1-3): for each candidate pair, the closest points,
 * phi = distance - xi, and, while phi < 2r, the half-space (n, s phi) for every
 * vertex of the pair with non-zero inverse mass, n pointing away from the other
 * primitive and s the side's share w_side / (w_A + w_B) of barycentric-weighted
 * inverse masses.  `cands` may be the context's lists or caller-owned device
 * lists.  On return `out` views the context's regions, valid until the next build. */
int ccfr_build_regions(ccfr_ctx* ctx, const ccfr_mesh* mesh, const float* x_anchor_dev,
                       const ccfr_candidates* cands, const ccfr_params* params,
                       ccfr_regions* out, ccfr_stream stream);

/* Projection (Alg. 2 calling Alg. 1, with the epsilon retraction and halt
 * fallback of Sec. 3.2, then the clamp |y| <= r of Alg. 4), per vertex v with
 * proposed displacement y_in[v] = x'_v - x_v:
 *   half-spaces sorted by rho = n . y_in + d ascending (ties by key), exact
 *   duplicates dropped; up to max_passes passes of Alg. 1 over the violated
 *   ones; a pass with no violation returns its start point; otherwise y = 0 and
 *   halted[v] = 1.  Vertices with zero inverse mass get y = 0.
 * regions: device CSR (the context's or caller-owned; hs 16-byte aligned).  inv_mass_dev [N],
 * y_in_dev, y_out_dev [N][3] device (y_out may alias y_in); halted_dev [N] uint8
 * device or NULL (all pointers may be NULL when regions->n_verts is 0).  A
 * proposal with a non-finite component gives y = 0, halted = 1 and raises the
 * non-finite status bit.  The per-vertex arithmetic runs in FP64 registers. */
int ccfr_project_displacements(ccfr_ctx* ctx, const ccfr_regions* regions, const float* inv_mass_dev,
                               const float* y_in_dev, const ccfr_params* params, float* y_out_dev,
                               uint8_t* halted_dev, ccfr_stream stream);

/* applyResponse of Alg. 4 (Sec. 3.3) per vertex v with proposed displacement
 * y_in[v] and its region (built at the anchor): the contacts whose gap beyond
 * the offset at the proposal, d_c = (n_c . y + d_c) / share_c, is below delta
 * get the XPBD update of the response constraint max(0, delta - d_c) with
 * compliance resp_compliance / (w_c dt^2), w_c the product of the visibility
 * factors 1 - S((d_c - d_j) / vis_width) over the vertex's other active
 * contacts (S the cubic smoothstep); the vertex takes its share of each
 * correction, innermost contact first, each followed by friction on the
 * tangential part t of the displacement (removed if |t| < mu_s times the
 * correction, else shortened by mu_k times it).  Arguments as in
 * ccfr_project_displacements, plus dt > 0; params->flags must hold
 * CCFR_FLAG_RESPONSE (else y_out = y_in).  y_out may alias y_in. */
int ccfr_apply_response(ccfr_ctx* ctx, const ccfr_regions* regions, const float* inv_mass_dev,
                        const float* y_in_dev, const ccfr_params* params, float dt, float* y_out_dev,
                        ccfr_stream stream);

/* ccfr_project_displacements for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, no context, and no allocation of
 * any kind.  Its scratch (device counters, the list of deferred vertices, sort
 * keys of large regions) is one file-scope device array of about 56 MiB that
 * every GPU the library runs on holds until the process ends, found with
 * hipGetSymbolAddress on the first call on each device.
 *  - Limits: regions->n_verts <= 2^20 and regions->cap <= 2^22 half-spaces;
 *    larger calls return CCFR_ERR_CAPACITY before anything is enqueued.
 *  - Arguments as in ccfr_project_displacements; status_dev (nullable, device
 *    uint32) receives the call's device status bits (64 = a non-finite
 *    proposal, which gets y = 0 and halted = 1), written on `stream` after the
 *    projection.
 *  - Every call on one GPU shares that GPU's array: calls ordered on one
 *    stream are safe, calls that overlap on one GPU (several streams or host
 *    threads) race. */
int ccfr_project_displacements_noalloc(const ccfr_regions* regions, const float* inv_mass_dev,
                                       const float* y_in_dev, const ccfr_params* params, float* y_out_dev,
                                       uint8_t* halted_dev, uint32_t* status_dev, ccfr_stream stream);

/* One substep (Alg. 4), in place on x_dev and v_dev ([n_verts][3] device):
 *   x~ = x + dt v + dt^2 g for dynamic vertices; lambda = 0;
 *   per iteration: candidates and regions at the anchor x; p = x~; one
 *   Gauss-Seidel pass of XPBD distance constraints over the edge colours
 *   (lambda kept across iterations); with CCFR_FLAG_RESPONSE the response and
 *   friction of ccfr_apply_response on p; x += project(p - x); with
 *   sp->early_exit, the convergence check (see ccfr_step_params);
 *   finally v = (x - x_start) / dt.
 * The first call for a (mesh, x, v, parameters) combination records a HIP graph
 * of the whole substep; later calls replay it.  A mesh with no vertices is a
 * no-op (x_dev and v_dev may then be NULL). */
int ccfr_xpbd_step(ccfr_ctx* ctx, const ccfr_mesh* mesh, float* x_dev, float* v_dev,
                   const ccfr_step_params* sp, ccfr_stream stream);

/* The same substep, launched directly (never recorded), that also copies the
 * anchor after every iteration into trace_dev ([iters][n_verts][3] float32,
 * device, caller-owned): the straight-line motion of each iteration is
 * trace[i-1] -> trace[i] (from x_dev's entry value for i = 0), which is what the
 * paper's claim of no remaining violation (Sec. 4.3) is checked on.  Results
 * are bitwise those of ccfr_xpbd_step. */
int ccfr_xpbd_step_traced(ccfr_ctx* ctx, const ccfr_mesh* mesh, float* x_dev, float* v_dev,
                          const ccfr_step_params* sp, float* trace_dev, ccfr_stream stream);

/* Waits for `stream`, copies the status word and counters into *info (nullable)
 * and returns CCFR_ERR_CAPACITY / CCFR_ERR_NONFINITE if the matching sticky bits
 * are set, else CCFR_OK.  reset != 0 clears the whole device record: the bits,
 * need[], totals[] and also the list lengths behind ccfr_candidates.counts_dev,
 * so read the lists of a standalone build before resetting. */
int ccfr_sync_status(ccfr_ctx* ctx, ccfr_stream stream, ccfr_status_info* info, int reset);

/* ---- stage timing (measurement) ----
 * With profiling enabled, every substep runs as individual launches (not as the
 * recorded graph) and records HIP events around its stages on its stream:
 *   0 grid build (counter reset, binning, bucket scan, scatter)
 *   1 pair emission (the broad-phase query kernel alone)
 *   2 contacts (narrow phase: closest points, the contact list; per-vertex
 *     counts for CSR regions)
 *   3 region fill (CSR regions: offset scan and half-space scatter; inside a
 *     substep with per-vertex slots: the slot fill)
 *   4 stretch pass (the iteration's closing kernel and the colours launched
 *     on their own; with per-vertex slots the reset of p and the first colour
 *     run in the previous projection, the next three colours inside stages 2,
 *     3 and this one, and the last two inside stage 5)
 *   5 projection
 * Disabling profiling returns to the recorded graph. */
int ccfr_profile_enable(ccfr_ctx* ctx, int enable);
/* Waits for `stream`, then writes per stage the milliseconds summed over the
 * iterations of the most recent substep (ms[6]) and how often each stage ran
 * (launches[6], nullable: the iterations, or for stages 0 and 1 the candidate
 * builds). */
int ccfr_profile_read(ccfr_ctx* ctx, ccfr_stream stream, float* ms, int32_t* launches);

/* ---- tuning ----
 * Knobs that change speed only: the candidate set is fixed by the box test, so
 * every setting gives the same pairs, regions and displacements.
 *   cell_scale  grid cell size as a multiple of the default, 1.2 x the typical
 *               edge length + 2 pad (the cell never drops below 2.02 pad);
 *               in [0.25, 4], default 1.
 *   pair_split  lanes per broad-phase query: 1 (the whole 3 x 3 x 3 stencil),
 *               3 (one z layer each) or 9 (one row each); default 1.
 *   pair_reuse  solver iterations of a substep (ccfr_xpbd_step, ccfr_batch_step)
 *               that share one candidate build, 1..4 (0 reads as 1); default 1.
 *               A build serving k iterations widens the box of every primitive
 *               with a moving vertex by k - 1 times the most a vertex can move in
 *               one iteration (r, from the clamp of Alg. 4, plus the FP32
 *               rounding of the position update), so its list holds every pair
 *               whose boxes overlap at any of those iterations.  The narrow
 *               phase still keeps exactly the pairs with phi < 2r at the current
 *               positions, so regions and results are those of a build per
 *               iteration, bit for bit; the lists are longer.
 *   pair_skin   0 (default): builds grouped by pair_reuse.  s in 1..4: builds
 *               that follow the motion instead (pair_reuse is then unused):
 *               every build widens the boxes of primitives with a moving
 *               vertex by at least s r, and from the second iteration of a
 *               substep on, the device sums the largest coordinate move of each
 *               projection since the last build and builds again only once the
 *               sum may exceed the widening (every pair whose boxes overlap now
 *               had widened boxes overlapping at the build).  Results are again
 *               those of a build per iteration, bit for bit.
 * Setting them invalidates recorded step graphs (they are recorded again). */
typedef struct {
    float cell_scale;
    int32_t pair_split;
    int32_t pair_reuse;
    int32_t pair_skin;
    int32_t broad_phase; /* 0 (default): the multi-level hash grid; 1: a linear
                            bounding-volume hierarchy over the padded boxes of the
                            targets (the analogue of the paper's AABB tree, Sec.
                            4.1), rebuilt with every candidate build; the same pairs */
    int32_t direct_regions; /* substeps with per-vertex slot regions: 0 (default)
                            the narrow phase compacts the pairs in range into a
                            contact list and a fill launch writes their
                            half-spaces; 1 the narrow phase writes them into the
                            slots itself (one launch and the list fewer, but its
                            wavefronts wait on the writes: faster when most
                            candidate pairs are in range).  The same regions. */
} ccfr_tuning;
int ccfr_set_tuning(ccfr_ctx* ctx, const ccfr_tuning* tuning);
int ccfr_get_tuning(const ccfr_ctx* ctx, ccfr_tuning* tuning);

/* ---- batches: many independent meshes stepped together ---- */
/* The paper steps one scene at a time and defines no batching: these entry
 * points run the substep of Alg. 4 (with Alg. 2-3 inside) over many unrelated
 * meshes per launch.  Meshes are concatenated in a device pool; every vertex
 * carries its slot id, which selects its mesh's collision parameters and keeps
 * primitives of different slots from ever forming a pair, so each mesh evolves
 * exactly as it would alone (same candidates, regions and projection).
 *
 * A batch holds up to `max_slots` (<= 65535) meshes within `max_verts`,
 * `max_tris` and `max_edges` in total, and two copies of the pool (the second
 * receives survivors when removed slots are compacted, and the step's entry
 * snapshot).  It borrows `ctx`'s workspace: do not use `ctx` for other work
 * while a batch step may still run, and destroy the batch before `ctx`.
 * Capacity overflow of the workspace lists is reported by ccfr_sync_status on
 * `ctx` as for single meshes: call ccfr_reserve with the reported needs, then
 * ccfr_batch_rollback and step again. */
int ccfr_batch_create(ccfr_ctx* ctx, int32_t max_slots, int64_t max_verts, int64_t max_tris,
                      int64_t max_edges, ccfr_batch** out);
void ccfr_batch_destroy(ccfr_batch* b);
/* Upper bound on the device bytes a mesh of these sizes adds to a batch (both
 * pools plus its share of the workspace at default list sizes); -1 on negative
 * sizes.  A server admits requests while the sum stays within its budget. */
int64_t ccfr_batch_footprint(int32_t n_verts, int32_t n_tris, int32_t n_edges);
/* Admit a mesh: host arrays as in ccfr_mesh_create, plus initial x and v
 * ([n_verts][3] float32, finite) and its step parameters.  The collision part
 * of `sp` is per mesh; dt, gravity, iters and alpha must equal those of the
 * meshes already resident and early_exit must be 0 (a batch runs its meshes'
 * iterations together; else CCFR_ERR_INVALID_ARG).  The response
 * (CCFR_FLAG_RESPONSE) is per mesh too.  *slot receives the
 * lowest free slot id.  CCFR_ERR_CAPACITY if no slot or pool space is free;
 * nothing changes then.  Copies are made on `stream`, and the call waits for
 * them. */
int ccfr_batch_add(ccfr_batch* b, int32_t n_verts, const int32_t* tris, int32_t n_tris,
                   const int32_t* edges, int32_t n_edges, const float* inv_mass,
                   const float* rest_x, const float* x, const float* v,
                   const ccfr_step_params* sp, int32_t* slot, ccfr_stream stream);
/* Release a slot (CCFR_ERR_INVALID_ARG if not resident).  Its pool space is
 * reclaimed by compaction at the next add or step. */
int ccfr_batch_remove(ccfr_batch* b, int32_t slot, ccfr_stream stream);
/* One substep of every resident mesh, enqueued on `stream` (a recorded graph,
 * re-recorded whenever the resident set or the workspace changes).  It first
 * snapshots x and v of every mesh for ccfr_batch_rollback. */
int ccfr_batch_step(ccfr_batch* b, ccfr_stream stream);
/* Restore x and v of every resident mesh to what they were when the last
 * ccfr_batch_step began.  CCFR_ERR_NOT_READY if no step ran since the last
 * add or remove. */
int ccfr_batch_rollback(ccfr_batch* b, ccfr_stream stream);
/* Copy a slot's positions / velocities ([n][3] float32; either may be NULL) to
 * host memory; waits for `stream`. */
int ccfr_batch_read(ccfr_batch* b, int32_t slot, float* x_host, float* v_host, ccfr_stream stream);
/* Number of resident meshes and their total vertex count. */
int ccfr_batch_stats(const ccfr_batch* b, int32_t* n_resident, int64_t* n_verts);

#ifdef __cplusplus
}
#endif
#endif
