// ccfr_api.hip -- host side of the C ABI declared in include/ccfr.h: contexts,
// device meshes, workspace growth, the per-call entry points and the recorded
// HIP graph of the XPBD substep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "ccfr_internal.h"

using namespace ccfr;

namespace {

int ceil_log2(long long v) {
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

}  // namespace

struct ccfr_mesh {
    ccfr_ctx* ctx = nullptr;
    int32_t n_verts = 0, n_tris = 0, n_edges = 0, n_free = 0;
    int32_t* tris_d = nullptr;
    int32_t* edges_d = nullptr;
    float* inv_mass_d = nullptr;
    int32_t* free_list_d = nullptr;
    uint8_t* is_free_d = nullptr;
    // stretch constraints, edges sorted by colour
    bool has_stretch = false;
    int32_t* edges_sorted_d = nullptr;
    float* rest_sorted_d = nullptr;
    float* lambda_d = nullptr;
    std::vector<int32_t> color_begin;   // n_colors + 1
    float typ_len = 0.f;                // edge length the grid cell is sized for
    std::vector<int32_t> edges_h;
};

struct StepGraph {
    bool valid = false;
    const ccfr_mesh* mesh = nullptr;
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
    DevCounters* counters_d = nullptr;
    long long generation = 0;   // bumped whenever a workspace buffer moves
    bool use_graphs = true;
    bool narrow_fp32 = false;   // narrow-phase arithmetic in FP32 (measurement option)

    // grid
    int log2s = 0;
    long long cap_targets = 0;
    int32_t* cnt = nullptr;
    int32_t* start = nullptr;
    int32_t* rank = nullptr;
    int32_t* key = nullptr;
    GridEntry* entries = nullptr;
    uint32_t* level_mask = nullptr;
    int32_t cap_meshes = 0;
    int32_t* scan_tmp = nullptr;
    long long cap_scan_tmp = 0;

    // candidate lists
    int32_t* vf = nullptr;
    int32_t* ee = nullptr;
    int32_t* vv = nullptr;
    long long cap_vf = 0, cap_ee = 0, cap_vv = 0;

    // regions
    Contact* contacts = nullptr;
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
    long long cap_step = 0;

    StepGraph graph;

    // stage timing: events[iteration][stage][begin/end]
    bool profiling = false;
    int prof_iters = 0;        // events allocated for this many iterations
    int prof_last_iters = 0;   // iterations of the last profiled step
    std::vector<hipEvent_t> prof_events;
};

constexpr int kStages = 6;

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

namespace {

void drop_graph(ccfr_ctx* ctx) {
    if (ctx->graph.exec) (void)hipGraphExecDestroy(ctx->graph.exec);
    if (ctx->graph.graph) (void)hipGraphDestroy(ctx->graph.graph);
    ctx->graph = StepGraph{};
}

// Grows the grid for `targets` binned primitives.
int ensure_grid(ccfr_ctx* ctx, long long targets) {
    const int log2s = std::max(6, ceil_log2(std::max(64LL, targets)));
    if (log2s > ctx->log2s) {
        dev_free(ctx->cnt);
        dev_free(ctx->start);
        const long long S3 = 3LL << log2s;
        HIP_ALLOC(dev_alloc(&ctx->cnt, S3));
        HIP_ALLOC(dev_alloc(&ctx->start, S3 + 1));
        HIP_OK(hipMemset(ctx->cnt, 0, sizeof(int32_t) * (size_t)S3));
        ctx->log2s = log2s;
        const long long ntmp = (S3 + 1023) / 1024 + 2;
        if (ntmp > ctx->cap_scan_tmp) {
            dev_free(ctx->scan_tmp);
            HIP_ALLOC(dev_alloc(&ctx->scan_tmp, ntmp));
            ctx->cap_scan_tmp = ntmp;
        }
        ctx->generation++;
    }
    if (targets > ctx->cap_targets) {
        dev_free(ctx->rank);
        dev_free(ctx->key);
        dev_free(ctx->entries);
        HIP_ALLOC(dev_alloc(&ctx->rank, targets));
        HIP_ALLOC(dev_alloc(&ctx->key, targets));
        HIP_ALLOC(dev_alloc(&ctx->entries, targets));
        ctx->cap_targets = targets;
        ctx->generation++;
    }
    return CCFR_OK;
}

int ensure_meshes(ccfr_ctx* ctx, int n_meshes) {
    if (n_meshes > ctx->cap_meshes) {
        dev_free(ctx->level_mask);
        const int cap = std::max(n_meshes, 16);
        HIP_ALLOC(dev_alloc(&ctx->level_mask, cap));
        HIP_OK(hipMemset(ctx->level_mask, 0, sizeof(uint32_t) * (size_t)cap));
        ctx->cap_meshes = cap;
        ctx->generation++;
    }
    return CCFR_OK;
}

int ensure_pairs(ccfr_ctx* ctx, long long vf, long long ee, long long vv) {
    if (vf > ctx->cap_vf) {
        dev_free(ctx->vf);
        HIP_ALLOC(dev_alloc(&ctx->vf, 2 * vf));
        ctx->cap_vf = vf;
        ctx->generation++;
    }
    if (ee > ctx->cap_ee) {
        dev_free(ctx->ee);
        HIP_ALLOC(dev_alloc(&ctx->ee, 2 * ee));
        ctx->cap_ee = ee;
        ctx->generation++;
    }
    if (vv > ctx->cap_vv) {
        dev_free(ctx->vv);
        HIP_ALLOC(dev_alloc(&ctx->vv, 2 * vv));
        ctx->cap_vv = vv;
        ctx->generation++;
    }
    return CCFR_OK;
}

int ensure_regions(ccfr_ctx* ctx, long long n_verts, long long contacts, long long hs) {
    if (n_verts > ctx->cap_verts) {
        dev_free(ctx->vcount);
        dev_free(ctx->offsets);
        dev_free(ctx->slow_list);
        HIP_ALLOC(dev_alloc(&ctx->vcount, n_verts));
        HIP_ALLOC(dev_alloc(&ctx->offsets, n_verts + 1));
        HIP_ALLOC(dev_alloc(&ctx->slow_list, n_verts));
        HIP_OK(hipMemset(ctx->vcount, 0, sizeof(int32_t) * (size_t)n_verts));
        const long long ntmp = (n_verts + 1023) / 1024 + 2;
        if (ntmp > ctx->cap_scan_tmp) {
            dev_free(ctx->scan_tmp);
            HIP_ALLOC(dev_alloc(&ctx->scan_tmp, ntmp));
            ctx->cap_scan_tmp = ntmp;
        }
        ctx->cap_verts = n_verts;
        ctx->generation++;
    }
    if (contacts > ctx->cap_contacts) {
        dev_free(ctx->contacts);
        HIP_ALLOC(dev_alloc(&ctx->contacts, contacts));
        ctx->cap_contacts = contacts;
        ctx->generation++;
    }
    if (hs > ctx->cap_hs) {
        dev_free(ctx->hs);
        dev_free(ctx->sort_key);
        dev_free(ctx->sort_idx);
        HIP_ALLOC(dev_alloc(&ctx->hs, hs));
        HIP_ALLOC(dev_alloc(&ctx->sort_key, hs));
        HIP_ALLOC(dev_alloc(&ctx->sort_idx, hs));
        ctx->cap_hs = hs;
        ctx->generation++;
    }
    return CCFR_OK;
}

int ensure_step(ccfr_ctx* ctx, long long n_verts) {
    if (n_verts > ctx->cap_step) {
        dev_free(ctx->x_pred);
        dev_free(ctx->x_start);
        dev_free(ctx->p);
        HIP_ALLOC(dev_alloc(&ctx->x_pred, 3 * n_verts));
        HIP_ALLOC(dev_alloc(&ctx->x_start, 3 * n_verts));
        HIP_ALLOC(dev_alloc(&ctx->p, 3 * n_verts));
        ctx->cap_step = n_verts;
        ctx->generation++;
    }
    return CCFR_OK;
}

// Default sizes from the mesh; later growth follows the observed needs.
int ensure_for_mesh(ccfr_ctx* ctx, const ccfr_mesh* m) {
    int rc = ensure_grid(ctx, (long long)m->n_tris + m->n_edges + m->n_free);
    if (rc) return rc;
    rc = ensure_meshes(ctx, 1);
    if (rc) return rc;
    const long long vf = 8LL * m->n_verts + 4096, ee = 8LL * m->n_edges + 4096, vv = 16LL * m->n_free + 4096;
    rc = ensure_pairs(ctx, vf, ee, vv);
    if (rc) return rc;
    return ensure_regions(ctx, m->n_verts, (vf + ee + vv) / 2, 2 * (vf + ee + vv));
}

bool params_ok(const ccfr_params* p) {
    return p && std::isfinite(p->r) && p->r > 0.f && std::isfinite(p->xi) && p->xi >= 0.f &&
           std::isfinite(p->delta) && p->delta >= 0.f && std::isfinite(p->guard) && p->guard >= 0.f &&
           std::isfinite(p->eps_retract) && p->eps_retract >= 0.f && std::isfinite(p->eps_plesnik) &&
           p->eps_plesnik >= 0.f && p->max_passes >= 1;
}

// Per-mesh device parameters: the box pad (one FP32 rounding of an FP64 sum) and
// a grid cell large enough that typical primitives span at most two cells.
MeshParams mesh_params(const ccfr_params* p, float typ_len, int salt) {
    MeshParams m{};
    m.r = p->r;
    m.xi = p->xi;
    m.pad = (float)((double)p->r + 0.5 * (double)p->xi + 0.5 * (double)p->delta + (double)p->guard);
    m.two_r = 2.0f * p->r;
    m.eps_retract = p->eps_retract;
    m.eps_plesnik = p->eps_plesnik;
    const double h = std::max(2.02 * (double)m.pad, 1.2 * (double)typ_len + 2.0 * (double)m.pad);
    m.h = (float)h;
    m.inv_h = (float)(1.0 / h);
    m.max_passes = p->max_passes;
    m.mesh_salt = salt;
    return m;
}

Scene make_scene(const ccfr_mesh* m, const float* x, const ccfr_params* p) {
    Scene sc{};
    sc.narrow_fp32 = m->ctx->narrow_fp32 ? 1 : 0;
    sc.n_verts = m->n_verts;
    sc.n_tris = m->n_tris;
    sc.n_edges = m->n_edges;
    sc.n_free = m->n_free;
    sc.x = x;
    sc.inv_mass = m->inv_mass_d;
    sc.tris = m->tris_d;
    sc.edges = m->edges_d;
    sc.free_list = m->free_list_d;
    sc.is_free = m->is_free_d;
    sc.prm.table = nullptr;
    sc.prm.vmesh = nullptr;
    sc.prm.one = mesh_params(p, m->typ_len, 0);
    return sc;
}

GridWs grid_ws(ccfr_ctx* ctx) {
    GridWs g{};
    g.log2s = ctx->log2s;
    g.cnt = ctx->cnt;
    g.start = ctx->start;
    g.rank = ctx->rank;
    g.key = ctx->key;
    g.entries = ctx->entries;
    g.level_mask = ctx->level_mask;
    g.n_meshes = 1;
    g.scan_tmp = ctx->scan_tmp;
    return g;
}

// Event marks of stage `stage` in iteration `it` (no-op unless profiling).
struct Marks {
    ccfr_ctx* ctx;
    int it;
    hipStream_t s;
    void mark(int stage, int end) const {
        if (!ctx->profiling || it < 0 || it >= ctx->prof_iters) return;
        (void)hipEventRecord(ctx->prof_events[((size_t)it * kStages + stage) * 2 + end], s);
    }
};

// broad phase into the context's lists
void enqueue_candidates(ccfr_ctx* ctx, const Scene& sc, hipStream_t s, const Marks& mk) {
    GridWs g = grid_ws(ctx);
    mk.mark(0, 0);
    launch_reset_build(ctx->counters_d, g.level_mask, g.n_meshes, s);
    launch_grid_count(sc, g, ctx->counters_d, s);
    launch_scan(g.cnt, g.start, g.cnt, 3 << g.log2s, g.scan_tmp, s);
    launch_grid_scatter(sc, g, s);
    mk.mark(0, 1);
    PairLists pl{ctx->vf, ctx->ee, ctx->vv, ctx->cap_vf, ctx->cap_ee, ctx->cap_vv};
    mk.mark(1, 0);
    launch_pairs(sc, g, pl, ctx->counters_d, s);
    mk.mark(1, 1);
    launch_finalize_pairs(g, pl, ctx->counters_d, s);
}

void enqueue_regions(ccfr_ctx* ctx, const Scene& sc, const int32_t* vf, const int32_t* ee, const int32_t* vv,
                     const int32_t* counts, long long cap_vf, long long cap_ee, long long cap_vv, hipStream_t s,
                     const Marks& mk) {
    mk.mark(2, 0);
    launch_contacts(sc, vf, ee, vv, counts, cap_vf, cap_ee, cap_vv, ctx->contacts, ctx->cap_contacts, ctx->vcount,
                    ctx->counters_d, s);
    mk.mark(2, 1);
    mk.mark(3, 0);
    launch_scan(ctx->vcount, ctx->offsets, nullptr, sc.n_verts, ctx->scan_tmp, s);
    launch_fill(sc, ctx->contacts, ctx->cap_contacts, ctx->offsets, ctx->vcount, ctx->hs, ctx->cap_hs,
                ctx->counters_d, s);
    mk.mark(3, 1);
}

int32_t* counts_ptr(ccfr_ctx* ctx) { return &ctx->counters_d->n_vf; }

void enqueue_step(ccfr_ctx* ctx, const ccfr_mesh* m, float* x, float* v, const ccfr_step_params* sp,
                  hipStream_t s) {
    const Scene sc = make_scene(m, x, &sp->collision);
    const int n = m->n_verts;
    launch_predict(n, x, v, m->inv_mass_d, sp->dt, sp->gravity[0], sp->gravity[1], sp->gravity[2], ctx->x_pred,
                   ctx->x_start, s);
    if (m->has_stretch) launch_fill_zero(m->lambda_d, m->n_edges, s);
    const float alpha_t = sp->alpha / (sp->dt * sp->dt);
    for (int it = 0; it < sp->iters; ++it) {
        const Marks mk{ctx, it, s};
        enqueue_candidates(ctx, sc, s, mk);
        enqueue_regions(ctx, sc, ctx->vf, ctx->ee, ctx->vv, counts_ptr(ctx), ctx->cap_vf, ctx->cap_ee,
                        ctx->cap_vv, s, mk);
        mk.mark(4, 0);
        launch_copy(ctx->x_pred, ctx->p, 3LL * n, s);
        if (m->has_stretch) {
            const int nc = (int)m->color_begin.size() - 1;
            for (int c = 0; c < nc; ++c)
                launch_stretch_color(m->edges_sorted_d, m->rest_sorted_d, m->color_begin[c],
                                     m->color_begin[c + 1] - m->color_begin[c], m->inv_mass_d, ctx->p, m->lambda_d,
                                     alpha_t, s);
        }
        mk.mark(4, 1);
        ProjectArgs pa{};
        pa.n_verts = n;
        pa.offsets = ctx->offsets;
        pa.hs = ctx->hs;
        pa.cap_hs = ctx->cap_hs;
        pa.inv_mass = m->inv_mass_d;
        pa.y_in = nullptr;
        pa.p = ctx->p;
        pa.x_anchor = x;
        pa.y_out = nullptr;
        pa.halted = nullptr;
        pa.sort_key = ctx->sort_key;
        pa.sort_idx = ctx->sort_idx;
        pa.slow_list = ctx->slow_list;
        pa.prm = sc.prm;
        mk.mark(5, 0);
        launch_project(pa, ctx->counters_d, s);
        mk.mark(5, 1);
    }
    launch_update_velocity(n, x, ctx->x_start, 1.0f / sp->dt, v, s);
}

}  // namespace

extern "C" {

const char* ccfr_status_string(int code) {
    switch (code) {
        case CCFR_OK: return "ok";
        case CCFR_ERR_INVALID_ARG: return "invalid argument";
        case CCFR_ERR_CAPACITY: return "a device list outgrew its buffer";
        case CCFR_ERR_HIP: return "HIP runtime error";
        case CCFR_ERR_NONFINITE: return "non-finite position or displacement";
        case CCFR_ERR_DEGENERATE: return "degenerate primitive";
        case CCFR_ERR_NOT_READY: return "not ready";
        case CCFR_ERR_NO_MEMORY: return "device allocation failed";
        default: return "unknown status";
    }
}

int ccfr_create(ccfr_ctx** out, int device) {
    if (!out) return CCFR_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    HIP_OK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return CCFR_ERR_INVALID_ARG;
    HIP_OK(hipSetDevice(device));
    ccfr_ctx* ctx = new (std::nothrow) ccfr_ctx();
    if (!ctx) return CCFR_ERR_NO_MEMORY;
    ctx->device = device;
    const char* ng = std::getenv("CCFR_NO_GRAPHS");
    ctx->use_graphs = !(ng && ng[0] == '1');
    const char* nf = std::getenv("CCFR_NARROW_FP32");
    ctx->narrow_fp32 = nf && nf[0] == '1';
    if (dev_alloc(&ctx->counters_d, 1) != hipSuccess ||
        hipMemset(ctx->counters_d, 0, sizeof(DevCounters)) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        ccfr_destroy(ctx);
        return CCFR_ERR_HIP;
    }
    *out = ctx;
    return CCFR_OK;
}

void ccfr_destroy(ccfr_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    drop_graph(ctx);
    dev_free(ctx->counters_d);
    dev_free(ctx->cnt); dev_free(ctx->start); dev_free(ctx->rank); dev_free(ctx->key);
    dev_free(ctx->entries); dev_free(ctx->level_mask); dev_free(ctx->scan_tmp);
    dev_free(ctx->vf); dev_free(ctx->ee); dev_free(ctx->vv);
    dev_free(ctx->contacts); dev_free(ctx->vcount); dev_free(ctx->offsets); dev_free(ctx->slow_list);
    dev_free(ctx->hs);
    dev_free(ctx->sort_key); dev_free(ctx->sort_idx);
    dev_free(ctx->x_pred); dev_free(ctx->x_start); dev_free(ctx->p);
    for (hipEvent_t e : ctx->prof_events) (void)hipEventDestroy(e);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
}

int ccfr_mesh_create(ccfr_ctx* ctx, int32_t n_verts, const int32_t* tris, int32_t n_tris, const int32_t* edges,
                     int32_t n_edges, const float* inv_mass, const float* rest_x, ccfr_mesh** out) {
    if (!ctx || !out || n_verts < 0 || n_tris < 0 || n_edges < 0 || !inv_mass) return CCFR_ERR_INVALID_ARG;
    if (n_tris > 0 && !tris) return CCFR_ERR_INVALID_ARG;
    *out = nullptr;
    for (long long i = 0; i < 3LL * n_tris; ++i)
        if (tris[i] < 0 || tris[i] >= n_verts) return CCFR_ERR_INVALID_ARG;
    for (int32_t i = 0; i < n_verts; ++i)
        if (!(inv_mass[i] >= 0.f) || !std::isfinite(inv_mass[i])) return CCFR_ERR_INVALID_ARG;
    // edges: given, or the unique sorted edges of the triangles
    std::vector<int32_t> E;
    if (edges) {
        E.assign(edges, edges + 2LL * n_edges);
        for (int32_t e = 0; e < n_edges; ++e) {
            const int32_t a = E[2 * e], b = E[2 * e + 1];
            if (a < 0 || b < 0 || a >= n_verts || b >= n_verts || a == b) return CCFR_ERR_INVALID_ARG;
        }
    } else {
        std::vector<long long> keys;
        keys.reserve(3LL * n_tris);
        for (int32_t t = 0; t < n_tris; ++t)
            for (int k = 0; k < 3; ++k) {
                const long long a = tris[3 * t + k], b = tris[3 * t + (k + 1) % 3];
                keys.push_back(std::min(a, b) * (1LL << 32) + std::max(a, b));
            }
        std::sort(keys.begin(), keys.end());
        keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
        for (long long k : keys) {
            E.push_back((int32_t)(k >> 32));
            E.push_back((int32_t)(k & 0xffffffffLL));
        }
        n_edges = (int32_t)(E.size() / 2);
    }
    ccfr_mesh* m = new (std::nothrow) ccfr_mesh();
    if (!m) return CCFR_ERR_NO_MEMORY;
    m->ctx = ctx;
    m->n_verts = n_verts;
    m->n_tris = n_tris;
    m->n_edges = n_edges;
    m->edges_h = E;
    // free particles
    std::vector<uint8_t> is_free(n_verts, 1);
    for (long long i = 0; i < 3LL * n_tris; ++i) is_free[tris[i]] = 0;
    for (int32_t v : E) is_free[v] = 0;
    std::vector<int32_t> free_list;
    for (int32_t v = 0; v < n_verts; ++v)
        if (is_free[v]) free_list.push_back(v);
    m->n_free = (int32_t)free_list.size();
    // edge length the grid is sized for: the longest edge not longer than 8x the median
    if (n_edges > 0) {
        std::vector<float> len(n_edges);
        const float* px = rest_x;
        for (int32_t e = 0; e < n_edges && px; ++e) {
            const int32_t a = E[2 * e], b = E[2 * e + 1];
            double d2 = 0;
            for (int k = 0; k < 3; ++k) {
                const double d = (double)px[3 * a + k] - (double)px[3 * b + k];
                d2 += d * d;
            }
            len[e] = (float)std::sqrt(d2);
        }
        if (px) {
            std::vector<float> sorted = len;
            std::nth_element(sorted.begin(), sorted.begin() + n_edges / 2, sorted.end());
            const float med = sorted[n_edges / 2];
            float typ = 0.f;
            for (float l : len)
                if (l <= 8.f * med) typ = std::max(typ, l);
            m->typ_len = typ;
        }
    }
    // greedy colouring in edge-index order, then edges sorted by (colour, index)
    std::vector<int32_t> color(n_edges, 0);
    std::vector<uint64_t> used(n_verts, 0);
    int n_colors = 0;
    bool color_ok = true;
    for (int32_t e = 0; e < n_edges; ++e) {
        const int32_t a = E[2 * e], b = E[2 * e + 1];
        const uint64_t taken = used[a] | used[b];
        int c = 0;
        while (c < 64 && ((taken >> c) & 1ull)) ++c;
        if (c == 64) { color_ok = false; break; }
        color[e] = c;
        used[a] |= 1ull << c;
        used[b] |= 1ull << c;
        n_colors = std::max(n_colors, c + 1);
    }
    if (!color_ok) { delete m; return CCFR_ERR_INVALID_ARG; }
    m->color_begin.assign(n_colors + 1, 0);
    for (int32_t e = 0; e < n_edges; ++e) m->color_begin[color[e] + 1]++;
    for (int c = 0; c < n_colors; ++c) m->color_begin[c + 1] += m->color_begin[c];
    std::vector<int32_t> es(2LL * n_edges);
    std::vector<float> rs(n_edges, 0.f);
    {
        std::vector<int32_t> cur(m->color_begin.begin(), m->color_begin.end() - 1);
        for (int32_t e = 0; e < n_edges; ++e) {
            const int32_t pos = cur[color[e]]++;
            es[2 * pos] = E[2 * e];
            es[2 * pos + 1] = E[2 * e + 1];
            if (rest_x) {
                double d2 = 0;
                for (int k = 0; k < 3; ++k) {
                    const double d = (double)rest_x[3 * E[2 * e] + k] - (double)rest_x[3 * E[2 * e + 1] + k];
                    d2 += d * d;
                }
                rs[pos] = (float)std::sqrt(d2);
            }
        }
    }
    m->has_stretch = rest_x != nullptr && n_edges > 0;
    hipError_t e = hipSuccess;
    auto put = [&](auto** dst, const auto* src, long long count) {
        if (e != hipSuccess) return;
        e = dev_alloc(dst, count);
        if (e == hipSuccess && count > 0)
            e = hipMemcpy((void*)*dst, (const void*)src, sizeof(**dst) * (size_t)count, hipMemcpyHostToDevice);
    };
    put(&m->tris_d, tris, 3LL * n_tris);
    put(&m->edges_d, E.data(), 2LL * n_edges);
    put(&m->inv_mass_d, inv_mass, n_verts);
    put(&m->free_list_d, free_list.data(), (long long)free_list.size());
    put(&m->is_free_d, is_free.data(), n_verts);
    put(&m->edges_sorted_d, es.data(), 2LL * n_edges);
    put(&m->rest_sorted_d, rs.data(), n_edges);
    if (e == hipSuccess) e = dev_alloc(&m->lambda_d, std::max<long long>(n_edges, 1));
    if (e != hipSuccess) {
        ccfr_mesh_destroy(m);
        return CCFR_ERR_NO_MEMORY;
    }
    int rc = ensure_for_mesh(ctx, m);
    if (rc) {
        ccfr_mesh_destroy(m);
        return rc;
    }
    *out = m;
    return CCFR_OK;
}

void ccfr_mesh_destroy(ccfr_mesh* m) {
    if (!m) return;
    if (m->ctx && m->ctx->graph.mesh == m) drop_graph(m->ctx);
    dev_free(m->tris_d); dev_free(m->edges_d); dev_free(m->inv_mass_d); dev_free(m->free_list_d);
    dev_free(m->is_free_d); dev_free(m->edges_sorted_d); dev_free(m->rest_sorted_d); dev_free(m->lambda_d);
    delete m;
}

int ccfr_mesh_edges(const ccfr_mesh* m, int32_t* n_edges, int32_t* edges_host) {
    if (!m || !n_edges) return CCFR_ERR_INVALID_ARG;
    *n_edges = m->n_edges;
    if (edges_host) std::memcpy(edges_host, m->edges_h.data(), sizeof(int32_t) * m->edges_h.size());
    return CCFR_OK;
}

const float* ccfr_mesh_inv_mass_dev(const ccfr_mesh* m) { return m ? m->inv_mass_d : nullptr; }

int ccfr_reserve(ccfr_ctx* ctx, int64_t vf, int64_t ee, int64_t vv, int64_t contacts, int64_t halfspaces,
                 ccfr_stream stream) {
    if (!ctx || vf < 0 || ee < 0 || vv < 0 || contacts < 0 || halfspaces < 0) return CCFR_ERR_INVALID_ARG;
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    if (ctx->vcount) HIP_OK(hipMemset(ctx->vcount, 0, sizeof(int32_t) * (size_t)ctx->cap_verts));
    const long long gen = ctx->generation;
    int rc = ensure_pairs(ctx, vf, ee, vv);
    if (rc) return rc;
    rc = ensure_regions(ctx, 0, contacts, halfspaces);
    if (rc) return rc;
    if (ctx->generation != gen) drop_graph(ctx);
    return CCFR_OK;
}

int ccfr_build_candidates(ccfr_ctx* ctx, const ccfr_mesh* mesh, const float* x_anchor_dev, const ccfr_params* params,
                          ccfr_candidates* out, ccfr_stream stream) {
    if (!ctx || !mesh || !x_anchor_dev || !out || !params_ok(params)) return CCFR_ERR_INVALID_ARG;
    if (mesh->ctx != ctx) return CCFR_ERR_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    const Scene sc = make_scene(mesh, x_anchor_dev, params);
    enqueue_candidates(ctx, sc, s, Marks{ctx, -1, s});
    HIP_OK(hipGetLastError());
    out->vf = ctx->vf;
    out->ee = ctx->ee;
    out->vv = ctx->vv;
    out->counts_dev = counts_ptr(ctx);
    out->cap_vf = ctx->cap_vf;
    out->cap_ee = ctx->cap_ee;
    out->cap_vv = ctx->cap_vv;
    return CCFR_OK;
}

int ccfr_build_regions(ccfr_ctx* ctx, const ccfr_mesh* mesh, const float* x_anchor_dev, const ccfr_candidates* c,
                       const ccfr_params* params, ccfr_regions* out, ccfr_stream stream) {
    if (!ctx || !mesh || !x_anchor_dev || !c || !out || !params_ok(params)) return CCFR_ERR_INVALID_ARG;
    if (!c->counts_dev || c->cap_vf < 0 || c->cap_ee < 0 || c->cap_vv < 0) return CCFR_ERR_INVALID_ARG;
    if ((c->cap_vf > 0 && !c->vf) || (c->cap_ee > 0 && !c->ee) || (c->cap_vv > 0 && !c->vv))
        return CCFR_ERR_INVALID_ARG;
    if (mesh->ctx != ctx) return CCFR_ERR_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    const Scene sc = make_scene(mesh, x_anchor_dev, params);
    enqueue_regions(ctx, sc, c->vf, c->ee, c->vv, c->counts_dev, c->cap_vf, c->cap_ee, c->cap_vv, s,
                    Marks{ctx, -1, s});
    HIP_OK(hipGetLastError());
    out->n_verts = mesh->n_verts;
    out->pad_ = 0;
    out->offsets = ctx->offsets;
    out->hs = ctx->hs;
    out->cap = ctx->cap_hs;
    return CCFR_OK;
}

int ccfr_project_displacements(ccfr_ctx* ctx, const ccfr_regions* regions, const float* inv_mass_dev,
                               const float* y_in_dev, const ccfr_params* params, float* y_out_dev,
                               uint8_t* halted_dev, ccfr_stream stream) {
    if (!ctx || !regions || !inv_mass_dev || !y_in_dev || !y_out_dev || !params_ok(params)) return CCFR_ERR_INVALID_ARG;
    if (regions->n_verts < 0 || !regions->offsets || (regions->cap > 0 && !regions->hs) || regions->cap < 0)
        return CCFR_ERR_INVALID_ARG;
    // scratch for the sort and the list of violating vertices must cover the call
    if (regions->cap > ctx->cap_hs || regions->n_verts > ctx->cap_verts) {
        HIP_OK(hipStreamSynchronize((hipStream_t)stream));
        const long long gen = ctx->generation;
        int rc = ensure_regions(ctx, regions->n_verts, 0, regions->cap);
        if (rc) return rc;
        if (gen != ctx->generation) drop_graph(ctx);
    }
    ProjectArgs pa{};
    pa.n_verts = regions->n_verts;
    pa.offsets = regions->offsets;
    pa.hs = regions->hs;
    pa.cap_hs = regions->cap;
    pa.inv_mass = inv_mass_dev;
    pa.y_in = y_in_dev;
    pa.p = nullptr;
    pa.x_anchor = nullptr;
    pa.y_out = y_out_dev;
    pa.halted = halted_dev;
    pa.sort_key = ctx->sort_key;
    pa.sort_idx = ctx->sort_idx;
    pa.slow_list = ctx->slow_list;
    pa.prm.table = nullptr;
    pa.prm.vmesh = nullptr;
    pa.prm.one = mesh_params(params, 0.f, 0);
    launch_project(pa, ctx->counters_d, (hipStream_t)stream);
    HIP_OK(hipGetLastError());
    return CCFR_OK;
}

int ccfr_xpbd_step(ccfr_ctx* ctx, const ccfr_mesh* mesh, float* x_dev, float* v_dev, const ccfr_step_params* sp,
                   ccfr_stream stream) {
    if (!ctx || !mesh || !x_dev || !v_dev || !sp || !params_ok(&sp->collision)) return CCFR_ERR_INVALID_ARG;
    if (!(sp->dt > 0.f) || !std::isfinite(sp->dt) || sp->iters < 0 || !std::isfinite(sp->alpha) || sp->alpha < 0.f)
        return CCFR_ERR_INVALID_ARG;
    if (mesh->ctx != ctx) return CCFR_ERR_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    const long long gen0 = ctx->generation;
    int rc = ensure_step(ctx, mesh->n_verts);
    if (rc) return rc;
    rc = ensure_for_mesh(ctx, mesh);
    if (rc) return rc;
    if (ctx->generation != gen0) drop_graph(ctx);
    if (ctx->profiling && sp->iters > ctx->prof_iters) {
        drop_graph(ctx);
        const size_t need = (size_t)sp->iters * kStages * 2;
        while (ctx->prof_events.size() < need) {
            hipEvent_t e = nullptr;
            HIP_OK(hipEventCreate(&e));
            ctx->prof_events.push_back(e);
        }
        ctx->prof_iters = sp->iters;
    }
    if (ctx->profiling) ctx->prof_last_iters = sp->iters;
    // profiled steps run eagerly: the stage events bracket the launches on `s`
    if (!ctx->use_graphs || ctx->profiling) {
        enqueue_step(ctx, mesh, x_dev, v_dev, sp, s);
        HIP_OK(hipGetLastError());
        return CCFR_OK;
    }
    StepGraph& G = ctx->graph;
    const bool same = G.valid && G.mesh == mesh && G.x == x_dev && G.v == v_dev &&
                      std::memcmp(&G.sp, sp, sizeof(*sp)) == 0 && G.generation == ctx->generation;
    if (!same) {
        drop_graph(ctx);
        HIP_OK(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        enqueue_step(ctx, mesh, x_dev, v_dev, sp, ctx->capture_stream);
        hipGraph_t graph = nullptr;
        HIP_OK(hipStreamEndCapture(ctx->capture_stream, &graph));
        hipGraphExec_t exec = nullptr;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return CCFR_ERR_HIP;
        }
        G.valid = true;
        G.mesh = mesh;
        G.x = x_dev;
        G.v = v_dev;
        G.sp = *sp;
        G.generation = ctx->generation;
        G.graph = graph;
        G.exec = exec;
    }
    HIP_OK(hipGraphLaunch(G.exec, s));
    return CCFR_OK;
}

int ccfr_sync_status(ccfr_ctx* ctx, ccfr_stream stream, ccfr_status_info* info, int reset) {
    if (!ctx) return CCFR_ERR_INVALID_ARG;
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    DevCounters h{};
    HIP_OK(hipMemcpy(&h, ctx->counters_d, sizeof(h), hipMemcpyDeviceToHost));
    if (info) {
        info->status_bits = h.status;
        info->last_counts[0] = h.n_vf;
        info->last_counts[1] = h.n_ee;
        info->last_counts[2] = h.n_vv;
        info->last_contacts = h.n_contacts;
        info->last_halfspaces = h.last_hs;
        for (int k = 0; k < 6; ++k) info->need[k] = h.need[k];
        for (int k = 0; k < 10; ++k) info->totals[k] = h.totals[k];
    }
    // an overflowed contact list leaves per-vertex counts behind: clear them
    if ((h.status & ST_CONTACTS) && ctx->vcount)
        HIP_OK(hipMemset(ctx->vcount, 0, sizeof(int32_t) * (size_t)ctx->cap_verts));
    if (reset) {
        DevCounters z{};
        HIP_OK(hipMemcpy(ctx->counters_d, &z, sizeof(z), hipMemcpyHostToDevice));
    }
    if (h.status & ST_NONFINITE) return CCFR_ERR_NONFINITE;
    if (h.status & (ST_VF | ST_EE | ST_VV | ST_HS | ST_LARGE | ST_CONTACTS)) return CCFR_ERR_CAPACITY;
    return CCFR_OK;
}

int ccfr_profile_enable(ccfr_ctx* ctx, int enable) {
    if (!ctx) return CCFR_ERR_INVALID_ARG;
    if ((enable != 0) != ctx->profiling) {
        drop_graph(ctx);
        ctx->profiling = enable != 0;
    }
    return CCFR_OK;
}

int ccfr_profile_read(ccfr_ctx* ctx, ccfr_stream stream, float* ms, int32_t* launches) {
    if (!ctx || !ms) return CCFR_ERR_INVALID_ARG;
    if (!ctx->profiling) return CCFR_ERR_NOT_READY;
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    const int iters = ctx->prof_last_iters;
    for (int st = 0; st < kStages; ++st) {
        float total = 0.f;
        for (int it = 0; it < std::min(iters, ctx->prof_iters); ++it) {
            float t = 0.f;
            const size_t k = ((size_t)it * kStages + st) * 2;
            if (hipEventElapsedTime(&t, ctx->prof_events[k], ctx->prof_events[k + 1]) != hipSuccess)
                return CCFR_ERR_NOT_READY;
            total += t;
        }
        ms[st] = total;
        if (launches) launches[st] = std::min(iters, ctx->prof_iters);
    }
    return CCFR_OK;
}

}  // extern "C"
