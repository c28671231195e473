// ccfr_host.h -- host-side state shared by the single-mesh and batch entry
// points: contexts (workspace, counters, recorded graphs), device meshes, and
// the step plan that the substep sequencer runs.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "ccfr_internal.h"

namespace ccfr {
namespace host {

// Largest vertex, triangle or edge count of a mesh: pair records keep a
// primitive index in 30 bits.
constexpr int32_t kMaxPrims = 1 << 30;

inline int ceil_log2(long long v) {
    int k = 0;
    while ((1LL << k) < v) ++k;
    return k;
}

template <class T>
hipError_t dev_alloc(T** p, long long count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    return hipMalloc((void**)p, sizeof(T) * (size_t)count);
}

template <class T>
void dev_free(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

// Topology prepared on the host from the caller's arrays: edges (given or
// derived), greedy colouring in edge-index order, edges sorted by colour with
// their rest lengths, free particles, and the edge length the grid is sized for.
struct MeshHost {
    int32_t n_verts = 0, n_tris = 0, n_edges = 0;
    std::vector<int32_t> tris, edges;          // edges: [E][2], a < b
    std::vector<int32_t> color_begin;          // [n_colors + 1]
    std::vector<int32_t> edges_sorted;         // [E][2] by (colour, index)
    std::vector<float> rest_sorted;            // [E]
    std::vector<int32_t> free_list;
    std::vector<uint8_t> vflags;               // per vertex: VF_FREE, VF_COLOR0
    float typ_len = 0.f;
    bool has_stretch = false;
};

// Builds a MeshHost; returns a ccfr_status.
int prepare_mesh(int32_t n_verts, const int32_t* tris, int32_t n_tris, const int32_t* edges, int32_t n_edges,
                 const float* inv_mass, const float* rest_x, MeshHost* out);

}  // namespace host
}  // namespace ccfr

struct ccfr_mesh {
    ccfr_ctx* ctx = nullptr;
    int32_t n_verts = 0, n_tris = 0, n_edges = 0, n_free = 0;
    int32_t* tris_d = nullptr;
    int32_t* edges_d = nullptr;
    float* inv_mass_d = nullptr;
    int32_t* free_list_d = nullptr;
    uint8_t* vflags_d = nullptr;
    // stretch constraints, edges sorted by colour; one segment per colour
    bool has_stretch = false;
    int32_t* edges_sorted_d = nullptr;
    float* rest_sorted_d = nullptr;
    float* lambda_d = nullptr;
    int2* segs_d = nullptr;             // (first edge, 0) per colour
    // two or more colours: the last one's multipliers alternate between
    // lambda_d and lambda_alt_d; last_edge_d maps a vertex to its edge there
    float* lambda_alt_d = nullptr;
    int2* last_edge_d = nullptr;
    int2* prev_edge_d = nullptr;        // three or more colours: the same for the one before the last
    std::vector<int32_t> color_begin;   // n_colors + 1
    float typ_len = 0.f;                // edge length the grid cell is sized for
    std::vector<int32_t> edges_h;
};

struct StepGraph {
    bool valid = false;
    const void* owner = nullptr;
    float* x = nullptr;
    float* v = nullptr;
    ccfr_step_params sp{};
    long long generation = -1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct ccfr_ctx {
    int device = 0;
    hipStream_t capture_stream = nullptr;
    ccfr::DevCounters* counters_d = nullptr;
    long long generation = 0;   // bumped whenever a workspace buffer moves
    bool use_graphs = true;
    bool csr_in_step = false;   // substeps build CSR regions instead of slots (measurement option)
    float cell_scale = 1.0f;    // grid cell size relative to the default
    int pair_split = 1;         // lanes per broad-phase query (1, 3 or 9)
    int pair_reuse = 1;         // solver iterations per candidate build inside a substep
    int pair_skin = 0;          // > 0: builds widened by pair_skin r, rebuilt when the motion needs it
    int broad_phase = 0;        // 0: multi-level hash grid, 1: bounding-volume hierarchy
    int direct_regions = 0;     // substeps: the narrow phase writes the slots itself (no contact list)
    long long tune_generation = 0;

    // bounding-volume hierarchy (broad_phase 1), sized for cap_lbvh leaves
    ccfr::LbvhWs lbvh{};
    long long cap_lbvh = 0;
    unsigned char* lbvh_sort_temp = nullptr;

    // grid
    long long cap_buckets = 0;
    long long cap_targets = 0;
    int32_t* cnt = nullptr;
    int32_t* start = nullptr;
    int32_t* rank = nullptr;
    int32_t* key = nullptr;
    ccfr::GridEntry* entries = nullptr;
    ccfr::GridEntry* staged = nullptr;
    uint32_t* level_mask = nullptr;
    int32_t cap_meshes = 0;
    int32_t* scan_tmp = nullptr;
    long long cap_scan_tmp = 0;

    // candidate lists
    int32_t* vf = nullptr;
    int32_t* ee = nullptr;
    int32_t* vv = nullptr;
    int32_t* ve = nullptr;
    long long cap_vf = 0, cap_ee = 0, cap_vv = 0, cap_ve = 0;

    // regions
    ccfr::Contact* contacts = nullptr;
    long long cap_contacts = 0;
    long long cap_verts = 0;
    int32_t* vcount = nullptr;
    int32_t* offsets = nullptr;
    int32_t* slow_list = nullptr;
    ccfr_halfspace* hs = nullptr;
    double* sort_key = nullptr;
    int32_t* sort_idx = nullptr;
    long long cap_hs = 0;

    // substep
    float* x_pred = nullptr;
    float* x_start = nullptr;
    float* p = nullptr;
    float* y_def = nullptr;      // proposals the fast projection hands to the slow one
    uint8_t* halt_run = nullptr; // per vertex: consecutive halts within the current substep
    long long cap_step = 0;

    StepGraph graph;

    // stage timing: events[iteration][stage][begin/end]
    bool profiling = false;
    int prof_iters = 0;        // events allocated for this many iterations
    int prof_last_iters = 0;   // iterations of the last profiled step
    int prof_last_reuse = 1;   // iterations per candidate build in that step
    std::vector<hipEvent_t> prof_events;
};

#define HIP_OK(call)                                              \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return CCFR_ERR_HIP;                \
    } while (0)

#define HIP_ALLOC(call)                                           \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return CCFR_ERR_NO_MEMORY;          \
    } while (0)

namespace ccfr {
namespace host {

constexpr int kStages = 6;

// Everything the substep sequencer needs, for one mesh or a batch of them.
struct StepPlan {
    Scene sc;                        // sc.x is the anchor, updated in place
    float* x = nullptr;
    float* v = nullptr;
    int n_meshes = 1;                // level masks to reset
    // stretch pass: colour c runs the segments [col_first[c], col_first[c] + col_nseg[c])
    // of segs (first edge, exclusive prefix of segment lengths), col_total[c] edges
    bool has_stretch = false;
    const int32_t* edges_sorted = nullptr;
    const float* rest_sorted = nullptr;
    float* lambda = nullptr;
    // the last colour runs inside the projection when both are set (two or
    // more colours): vertex -> its edge in that colour, and the second array
    // its multipliers alternate with
    const int2* last_edge = nullptr;
    const int2* prev_edge = nullptr;    // three or more colours: the one before the last is folded too
    float* lambda_alt = nullptr;
    long long n_edges = 0;
    const int2* segs = nullptr;
    std::vector<int32_t> col_first, col_nseg, col_total;
    float dt = 0.f, gx = 0.f, gy = 0.f, gz = 0.f, alpha_t = 0.f;
    int iters = 0;
    // builds that adapt to the motion: the least widening (pad_wide - pad) of
    // any mesh's moving boxes; 0 = fixed grouping of iterations
    double skin = 0.0;
    // nullable: [iters][N][3] receives the anchor after every iteration
    float* trace = nullptr;
    // evaluateConvergence: end the iterations once the largest shortfall of a
    // projection is at most conv_tol
    bool early_exit = false;
    float conv_tol = 0.f;
    // a batch: some resident mesh asks for the response (a single mesh reads
    // its own parameters)
    bool response_any = false;
};

void drop_graph(ccfr_ctx* ctx);
int ensure_grid(ccfr_ctx* ctx, long long T, long long E, long long F, long long N);
int ensure_meshes(ccfr_ctx* ctx, int n_meshes);
int ensure_pairs(ccfr_ctx* ctx, long long vf, long long ee, long long vv);
int ensure_regions(ccfr_ctx* ctx, long long n_verts, long long contacts, long long hs);
int ensure_step(ccfr_ctx* ctx, long long n_verts);
int ensure_sizes(ccfr_ctx* ctx, long long n_verts, long long n_tris, long long n_edges, long long n_free,
                 int n_meshes);
bool params_ok(const ccfr_params* p);
bool step_params_ok(const ccfr_step_params* sp);
MeshParams mesh_params(const ccfr_params* p, float typ_len, int salt, float cell_scale, int skin_iters = 0,
                       int skin_mult = 0);
// The widening a context's tuning asks of the boxes of a substep's builds:
// iterations covered beyond the first (fixed grouping) or multiples of r
// (builds that adapt to the motion); at most one of them is non-zero.
inline int ctx_skin_iters(const ccfr_ctx* c) { return c->pair_skin > 0 ? 0 : c->pair_reuse - 1; }
inline int ctx_skin_mult(const ccfr_ctx* c) { return c->pair_skin; }
int ensure_prof_events(ccfr_ctx* ctx, int iters);
void enqueue_step(ccfr_ctx* ctx, const StepPlan& plan, hipStream_t s);
// Records the plan as a graph into *g (replacing it) and launches it on s.
int launch_recorded(ccfr_ctx* ctx, StepGraph& g, const StepPlan& plan, const void* owner,
                    const ccfr_step_params* sp, bool same, hipStream_t s);

}  // namespace host
}  // namespace ccfr
