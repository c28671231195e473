// ccfr_batch.hip -- many independent meshes stepped by one set of launches.
//
// Resident meshes are concatenated in a dense device pool: positions,
// velocities, inverse masses, mesh ids (the slot number, per vertex), free
// particle flags, triangles, edges in mesh order (global vertex ids), edges
// sorted by colour per mesh with their rest lengths, and free particles.  The
// kernels of the single-mesh path run over the whole pool; each vertex finds
// its mesh's parameters (r, xi, grid cell, ...) in a per-slot table, grid
// buckets are salted by slot, and grid entries carry the slot, so primitives of
// different meshes never form a pair.  The stretch pass merges colour c of
// every mesh into one launch over a segment table (one segment per mesh).
//
// Admission appends a mesh at the end of the pool.  Removal only marks the
// slot; the next step first compacts the survivors into the second pool in one
// launch (rebasing vertex ids) and swaps the pools.  The step is recorded as a
// HIP graph per layout and replayed until the set of meshes changes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "ccfr_host.h"

using namespace ccfr;
using namespace ccfr::host;

namespace {

struct Pool {
    float* x = nullptr;
    float* v = nullptr;
    float* w = nullptr;
    uint16_t* vmesh = nullptr;
    uint8_t* vflags = nullptr;
    int32_t* tris = nullptr;
    int32_t* edges = nullptr;
    int32_t* edges_sorted = nullptr;
    float* rest_sorted = nullptr;
    int32_t* free_list = nullptr;
};

struct BatchMesh {
    int32_t slot = -1;
    int32_t n_verts = 0, n_tris = 0, n_edges = 0, n_free = 0;
    long long v0 = 0, t0 = 0, e0 = 0, f0 = 0;
    std::vector<int32_t> color_begin;
    bool removed = false;
};

// Source and destination ranges of one surviving mesh during compaction.
struct Move {
    long long nv0, ov0, nv;
    long long nt0, ot0, nt;
    long long ne0, oe0, ne;
    long long nf0, of0, nf;
};

__device__ __forceinline__ int find_move(const Move* mv, int n, long long i, int cls) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const long long start = cls == 0 ? mv[mid].nv0 : cls == 1 ? mv[mid].nt0 : cls == 2 ? mv[mid].ne0 : mv[mid].nf0;
        if (start <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Copies every surviving mesh to its new place, rebasing vertex ids.
__global__ void k_compact(Pool src, Pool dst, const Move* mv, int n_moves, long long nv, long long nt, long long ne,
                          long long nf) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nv) {
        const Move& m = mv[find_move(mv, n_moves, i, 0)];
        const long long j = m.ov0 + (i - m.nv0);
        for (int k = 0; k < 3; ++k) {
            dst.x[3 * i + k] = src.x[3 * j + k];
            dst.v[3 * i + k] = src.v[3 * j + k];
        }
        dst.w[i] = src.w[j];
        dst.vmesh[i] = src.vmesh[j];
        dst.vflags[i] = src.vflags[j];
    }
    if (i < nt) {
        const Move& m = mv[find_move(mv, n_moves, i, 1)];
        const long long j = m.ot0 + (i - m.nt0);
        const int32_t d = (int32_t)(m.nv0 - m.ov0);
        for (int k = 0; k < 3; ++k) dst.tris[3 * i + k] = src.tris[3 * j + k] + d;
    }
    if (i < ne) {
        const Move& m = mv[find_move(mv, n_moves, i, 2)];
        const long long j = m.oe0 + (i - m.ne0);
        const int32_t d = (int32_t)(m.nv0 - m.ov0);
        for (int k = 0; k < 2; ++k) {
            dst.edges[2 * i + k] = src.edges[2 * j + k] + d;
            dst.edges_sorted[2 * i + k] = src.edges_sorted[2 * j + k] + d;
        }
        dst.rest_sorted[i] = src.rest_sorted[j];
    }
    if (i < nf) {
        const Move& m = mv[find_move(mv, n_moves, i, 3)];
        const long long j = m.of0 + (i - m.nf0);
        dst.free_list[i] = src.free_list[j] + (int32_t)(m.nv0 - m.ov0);
    }
}

__global__ void k_fill_u16(uint16_t* p, long long n, uint16_t value) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

}  // namespace

struct ccfr_batch {
    ccfr_ctx* ctx = nullptr;
    int32_t max_slots = 0;
    long long max_verts = 0, max_tris = 0, max_edges = 0;
    Pool pool[2];
    int cur = 0;
    float* lambda = nullptr;
    float* lambda_alt = nullptr;          // the last stretch colour's multipliers alternate
    int2* last_edge = nullptr;            // vertex -> (its edge in the last colour, partner)
    int2* prev_edge = nullptr;            // the same for the colour before the last
    MeshParams* table_d = nullptr;
    std::vector<MeshParams> table_h;
    std::vector<ccfr_params> coll_h;      // per slot: collision parameters
    std::vector<float> typ_h;             // per slot: edge length the cell is sized for
    long long tune_generation = -1;
    Move* moves_d = nullptr;
    int2* segs_d = nullptr;
    long long cap_segs = 0;
    std::vector<BatchMesh> meshes;        // pool order
    std::vector<uint8_t> slot_busy;
    long long used_v = 0, used_t = 0, used_e = 0, used_f = 0;
    bool has_sp = false;
    ccfr_step_params sp{};                // shared by all resident meshes
    bool dirty = true;
    bool compact_pending = false;
    bool snap_valid = false;              // spare pool x, v hold the last step's entry state
    StepPlan plan;
    StepGraph graph;
};

namespace {

void free_pool(Pool& p) {
    dev_free(p.x); dev_free(p.v); dev_free(p.w); dev_free(p.vmesh); dev_free(p.vflags);
    dev_free(p.tris); dev_free(p.edges); dev_free(p.edges_sorted); dev_free(p.rest_sorted); dev_free(p.free_list);
}

int alloc_pool(Pool& p, long long nv, long long nt, long long ne) {
    HIP_ALLOC(dev_alloc(&p.x, 3 * nv));
    HIP_ALLOC(dev_alloc(&p.v, 3 * nv));
    HIP_ALLOC(dev_alloc(&p.w, nv));
    HIP_ALLOC(dev_alloc(&p.vmesh, nv));
    HIP_ALLOC(dev_alloc(&p.vflags, nv));
    HIP_ALLOC(dev_alloc(&p.tris, 3 * nt));
    HIP_ALLOC(dev_alloc(&p.edges, 2 * ne));
    HIP_ALLOC(dev_alloc(&p.edges_sorted, 2 * ne));
    HIP_ALLOC(dev_alloc(&p.rest_sorted, ne));
    HIP_ALLOC(dev_alloc(&p.free_list, nv));
    return CCFR_OK;
}

int slot_salt(int slot) { return (int)(0x9E3779B1u * (uint32_t)(slot + 1)); }

// Parameters of every resident slot again, after a tuning change.
int refresh_table(ccfr_batch* b, hipStream_t s) {
    for (int k = 0; k < b->max_slots; ++k)
        if (b->slot_busy[k]) b->table_h[k] = mesh_params(&b->coll_h[k], b->typ_h[k], slot_salt(k), b->ctx->cell_scale,
                                  ctx_skin_iters(b->ctx), ctx_skin_mult(b->ctx));
    HIP_OK(hipMemcpyAsync(b->table_d, b->table_h.data(), sizeof(MeshParams) * b->table_h.size(),
                          hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    b->tune_generation = b->ctx->tune_generation;
    b->dirty = true;
    return CCFR_OK;
}

void drop_batch_graph(ccfr_batch* b) {
    if (b->graph.exec) (void)hipGraphExecDestroy(b->graph.exec);
    if (b->graph.graph) (void)hipGraphDestroy(b->graph.graph);
    b->graph = StepGraph{};
}

bool same_step(const ccfr_step_params& a, const ccfr_step_params& b) {
    return a.dt == b.dt && a.gravity[0] == b.gravity[0] && a.gravity[1] == b.gravity[1] &&
           a.gravity[2] == b.gravity[2] && a.iters == b.iters && a.alpha == b.alpha;
}

// Compacts the survivors of removed slots into the other pool.
int compact(ccfr_batch* b, hipStream_t s) {
    std::vector<Move> mv;
    std::vector<BatchMesh> keep;
    long long v = 0, t = 0, e = 0, f = 0;
    for (const BatchMesh& m : b->meshes) {
        if (m.removed) continue;
        Move r{v, m.v0, m.n_verts, t, m.t0, m.n_tris, e, m.e0, m.n_edges, f, m.f0, m.n_free};
        mv.push_back(r);
        BatchMesh k = m;
        k.v0 = v; k.t0 = t; k.e0 = e; k.f0 = f;
        keep.push_back(k);
        v += m.n_verts; t += m.n_tris; e += m.n_edges; f += m.n_free;
    }
    if (!mv.empty()) {
        HIP_OK(hipMemcpyAsync(b->moves_d, mv.data(), sizeof(Move) * mv.size(), hipMemcpyHostToDevice, s));
        const long long n = std::max(std::max(v, t), std::max(e, f));
        if (n > 0)
            hipLaunchKernelGGL(k_compact, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b->pool[b->cur],
                               b->pool[1 - b->cur], b->moves_d, (int)mv.size(), v, t, e, f);
        HIP_OK(hipGetLastError());
        // the move table is read by the launch above: wait before it can change
        HIP_OK(hipStreamSynchronize(s));
        b->cur = 1 - b->cur;
    }
    b->meshes = keep;
    b->used_v = v; b->used_t = t; b->used_e = e; b->used_f = f;
    b->compact_pending = false;
    b->dirty = true;
    return CCFR_OK;
}

// Rebuilds the step plan (scene over the pool, merged colour segments).
int rebuild_plan(ccfr_batch* b, hipStream_t s) {
    ccfr_ctx* ctx = b->ctx;
    const Pool& P = b->pool[b->cur];
    StepPlan& pl = b->plan;
    pl = StepPlan{};
    Scene& sc = pl.sc;
    sc.n_verts = (int32_t)b->used_v;
    sc.n_tris = (int32_t)b->used_t;
    sc.n_edges = (int32_t)b->used_e;
    sc.n_free = (int32_t)b->used_f;
    sc.x = P.x;
    sc.inv_mass = P.w;
    sc.tris = P.tris;
    sc.edges = P.edges;
    sc.free_list = P.free_list;
    sc.vflags = P.vflags;
    sc.prm.table = b->table_d;
    sc.prm.vmesh = P.vmesh;
    pl.x = P.x;
    pl.v = P.v;
    pl.n_meshes = b->max_slots;
    for (int k = 0; k < b->max_slots; ++k)
        if (b->slot_busy[k] && b->table_h[k].response) pl.response_any = true;
    // builds that adapt to the motion: the least widening over the resident meshes
    if (ctx_skin_mult(ctx) > 0) {
        double skin = 0.0;
        for (int k = 0; k < b->max_slots; ++k)
            if (b->slot_busy[k]) {
                const double w = (double)b->table_h[k].pad_wide - (double)b->table_h[k].pad;
                skin = skin > 0.0 ? std::min(skin, w) : w;
            }
        pl.skin = skin;
    }
    // colour c of every mesh: one segment each
    int n_colors = 0;
    for (const BatchMesh& m : b->meshes) n_colors = std::max(n_colors, (int)m.color_begin.size() - 1);
    std::vector<int2> segs;
    for (int c = 0; c < n_colors; ++c) {
        const int first = (int)segs.size();
        int total = 0;
        for (const BatchMesh& m : b->meshes) {
            if ((int)m.color_begin.size() - 1 <= c) continue;
            const int cnt = m.color_begin[c + 1] - m.color_begin[c];
            if (cnt <= 0) continue;
            segs.push_back(make_int2((int)(m.e0 + m.color_begin[c]), total));
            total += cnt;
        }
        pl.col_first.push_back(first);
        pl.col_nseg.push_back((int)segs.size() - first);
        pl.col_total.push_back(total);
    }
    if ((long long)segs.size() > b->cap_segs) {
        HIP_OK(hipStreamSynchronize(s));
        dev_free(b->segs_d);
        b->cap_segs = std::max<long long>((long long)segs.size(), 2 * b->cap_segs + 64);
        HIP_ALLOC(dev_alloc(&b->segs_d, b->cap_segs));
    }
    if (!segs.empty()) {
        HIP_OK(hipMemcpyAsync(b->segs_d, segs.data(), sizeof(int2) * segs.size(), hipMemcpyHostToDevice, s));
        if (n_colors >= 2)
            launch_last_colour_map(P.edges_sorted, b->segs_d + pl.col_first[n_colors - 1], pl.col_nseg[n_colors - 1],
                                   pl.col_total[n_colors - 1], (int32_t)b->used_v, b->last_edge, s);
        if (n_colors >= 3)
            launch_last_colour_map(P.edges_sorted, b->segs_d + pl.col_first[n_colors - 2], pl.col_nseg[n_colors - 2],
                                   pl.col_total[n_colors - 2], (int32_t)b->used_v, b->prev_edge, s);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(s));
    }
    pl.has_stretch = !segs.empty();
    pl.edges_sorted = P.edges_sorted;
    pl.rest_sorted = P.rest_sorted;
    pl.lambda = b->lambda;
    if (n_colors >= 2) {
        pl.lambda_alt = b->lambda_alt;
        pl.last_edge = b->last_edge;
    }
    if (n_colors >= 3) pl.prev_edge = b->prev_edge;
    pl.n_edges = b->used_e;
    pl.segs = b->segs_d;
    pl.dt = b->sp.dt;
    pl.gx = b->sp.gravity[0];
    pl.gy = b->sp.gravity[1];
    pl.gz = b->sp.gravity[2];
    pl.alpha_t = b->sp.alpha / (b->sp.dt * b->sp.dt);
    pl.iters = b->sp.iters;
    drop_batch_graph(b);
    b->dirty = false;
    return CCFR_OK;
}

}  // namespace

extern "C" {

int64_t ccfr_batch_footprint(int32_t n_verts, int32_t n_tris, int32_t n_edges) {
    if (n_verts < 0 || n_tris < 0 || n_edges < 0) return -1;
    const long long N = n_verts, T = n_tris, E = n_edges;
    // free particles: vertices no edge or triangle can reach (an estimate)
    const long long F = std::max(0LL, N - 2 * E - 3 * T);
    // two pools: x, v (12 B each), w (4), mesh id (2), free flag (1), free
    // list entry (4) per vertex; 12 B per triangle; 20 B per edge (edge, sorted
    // edge, rest length); plus lambda twice (8 B per edge) and the last stretch
    // colours' vertex maps (16 B per vertex)
    long long bytes = 2 * (35 * N + 12 * T + 20 * E) + 8 * E + 16 * N;
    // workspace at the default list sizes: substep buffers (36 B per vertex),
    // region CSR (12), grid entry twice (sorted and staged) + rank + key (104
    // per binned primitive or vertex) and at most 8 bucket counters and 8
    // offsets (4 B each) per entry,
    // 8 B per candidate pair slot (vertex-face, edge-edge, particle-particle
    // and particle-edge lists at their default sizes),
    // 48 B per contact slot (half the pair slots) and 44 B per half-space slot
    // (twice the pair slots: record, sort key, sort index)
    const long long pairs = 8 * N + 8 * E + 24 * F;
    bytes += 48 * N + 168 * (T + E + F + N) + 8 * pairs + 48 * (pairs / 2) + 44 * (2 * pairs);
    return bytes;
}

int ccfr_batch_create(ccfr_ctx* ctx, int32_t max_slots, int64_t max_verts, int64_t max_tris, int64_t max_edges,
                      ccfr_batch** out) {
    if (!ctx || !out || max_slots <= 0 || max_slots > 65535 || max_verts <= 0 || max_tris < 0 || max_edges < 0 ||
        max_verts > (1LL << 30) || max_tris > (1LL << 30) || max_edges > (1LL << 30))
        return CCFR_ERR_INVALID_ARG;
    *out = nullptr;
    HIP_OK(hipSetDevice(ctx->device));
    ccfr_batch* b = new (std::nothrow) ccfr_batch();
    if (!b) return CCFR_ERR_NO_MEMORY;
    b->ctx = ctx;
    b->max_slots = max_slots;
    b->max_verts = max_verts;
    b->max_tris = max_tris;
    b->max_edges = max_edges;
    b->slot_busy.assign(max_slots, 0);
    b->table_h.assign(max_slots, MeshParams{});
    b->coll_h.assign(max_slots, ccfr_params{});
    b->typ_h.assign(max_slots, 0.f);
    b->tune_generation = ctx->tune_generation;
    int rc = CCFR_OK;
    for (int k = 0; k < 2 && rc == CCFR_OK; ++k) rc = alloc_pool(b->pool[k], max_verts, max_tris, max_edges);
    if (rc == CCFR_OK && (dev_alloc(&b->lambda, std::max<long long>(max_edges, 1)) != hipSuccess ||
                          dev_alloc(&b->lambda_alt, std::max<long long>(max_edges, 1)) != hipSuccess ||
                          dev_alloc(&b->last_edge, max_verts) != hipSuccess ||
                          dev_alloc(&b->prev_edge, max_verts) != hipSuccess ||
                          dev_alloc(&b->table_d, max_slots) != hipSuccess ||
                          dev_alloc(&b->moves_d, max_slots) != hipSuccess))
        rc = CCFR_ERR_NO_MEMORY;
    if (rc == CCFR_OK) rc = ensure_step(ctx, max_verts);
    // the grid holds every primitive and vertex the pool can hold (any vertex
    // may be a free particle); list sizes start from the meshes' topology
    if (rc == CCFR_OK) rc = ensure_grid(ctx, max_tris, max_edges, max_verts, max_verts);
    if (rc == CCFR_OK) rc = ensure_sizes(ctx, max_verts, max_tris, max_edges, 0, max_slots);
    if (rc != CCFR_OK) {
        ccfr_batch_destroy(b);
        return rc;
    }
    *out = b;
    return CCFR_OK;
}

void ccfr_batch_destroy(ccfr_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    (void)hipDeviceSynchronize();
    drop_batch_graph(b);
    free_pool(b->pool[0]);
    free_pool(b->pool[1]);
    dev_free(b->lambda);
    dev_free(b->lambda_alt);
    dev_free(b->last_edge);
    dev_free(b->prev_edge);
    dev_free(b->table_d);
    dev_free(b->moves_d);
    dev_free(b->segs_d);
    delete b;
}

int ccfr_batch_add(ccfr_batch* b, int32_t n_verts, const int32_t* tris, int32_t n_tris, const int32_t* edges,
                   int32_t n_edges, const float* inv_mass, const float* rest_x, const float* x, const float* v,
                   const ccfr_step_params* sp, int32_t* slot, ccfr_stream stream) {
    if (!b || !x || !v || !slot || !step_params_ok(sp)) return CCFR_ERR_INVALID_ARG;
    if (sp->early_exit) return CCFR_ERR_INVALID_ARG;     // a batch runs its meshes' iterations together
    if (b->has_sp && !b->meshes.empty() && !same_step(b->sp, *sp)) return CCFR_ERR_INVALID_ARG;
    for (long long i = 0; i < 3LL * n_verts; ++i)
        if (!std::isfinite(x[i]) || !std::isfinite(v[i])) return CCFR_ERR_INVALID_ARG;
    MeshHost h;
    int rc = prepare_mesh(n_verts, tris, n_tris, edges, n_edges, inv_mass, rest_x, &h);
    if (rc) return rc;
    const hipStream_t s = (hipStream_t)stream;
    if (b->compact_pending) {
        rc = compact(b, s);
        if (rc) return rc;
    }
    int sl = -1;
    for (int k = 0; k < b->max_slots; ++k)
        if (!b->slot_busy[k]) { sl = k; break; }
    const long long nf = (long long)h.free_list.size();
    if (sl < 0 || b->used_v + h.n_verts > b->max_verts || b->used_t + h.n_tris > b->max_tris ||
        b->used_e + h.n_edges > b->max_edges || b->used_f + nf > b->max_verts)
        return CCFR_ERR_CAPACITY;
    BatchMesh m;
    m.slot = sl;
    m.n_verts = h.n_verts; m.n_tris = h.n_tris; m.n_edges = h.n_edges; m.n_free = (int32_t)nf;
    m.v0 = b->used_v; m.t0 = b->used_t; m.e0 = b->used_e; m.f0 = b->used_f;
    m.color_begin = h.color_begin;
    // rebase vertex ids to the pool
    const int32_t off = (int32_t)m.v0;
    for (int32_t& q : h.tris) q += off;
    for (int32_t& q : h.edges) q += off;
    for (int32_t& q : h.edges_sorted) q += off;
    for (int32_t& q : h.free_list) q += off;
    Pool& P = b->pool[b->cur];
    HIP_OK(hipMemcpyAsync(P.x + 3 * m.v0, x, sizeof(float) * 3 * h.n_verts, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(P.v + 3 * m.v0, v, sizeof(float) * 3 * h.n_verts, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(P.w + m.v0, inv_mass, sizeof(float) * h.n_verts, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(P.vflags + m.v0, h.vflags.data(), h.n_verts, hipMemcpyHostToDevice, s));
    if (h.n_tris)
        HIP_OK(hipMemcpyAsync(P.tris + 3 * m.t0, h.tris.data(), sizeof(int32_t) * 3 * h.n_tris, hipMemcpyHostToDevice, s));
    if (h.n_edges) {
        HIP_OK(hipMemcpyAsync(P.edges + 2 * m.e0, h.edges.data(), sizeof(int32_t) * 2 * h.n_edges,
                              hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(P.edges_sorted + 2 * m.e0, h.edges_sorted.data(), sizeof(int32_t) * 2 * h.n_edges,
                              hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(P.rest_sorted + m.e0, h.rest_sorted.data(), sizeof(float) * h.n_edges,
                              hipMemcpyHostToDevice, s));
    }
    if (nf)
        HIP_OK(hipMemcpyAsync(P.free_list + m.f0, h.free_list.data(), sizeof(int32_t) * nf, hipMemcpyHostToDevice, s));
    if (h.n_verts)
        hipLaunchKernelGGL(k_fill_u16, dim3((unsigned)((h.n_verts + 255) / 256)), dim3(256), 0, s, P.vmesh + m.v0,
                           (long long)h.n_verts, (uint16_t)sl);
    // a mesh's stretch constraints are off when it has no rest shape
    if (!h.has_stretch) m.color_begin.assign(1, 0);
    b->coll_h[sl] = sp->collision;
    b->typ_h[sl] = h.typ_len;
    b->table_h[sl] = mesh_params(&sp->collision, h.typ_len, slot_salt(sl), b->ctx->cell_scale,
                                  ctx_skin_iters(b->ctx), ctx_skin_mult(b->ctx));
    HIP_OK(hipMemcpyAsync(b->table_d + sl, &b->table_h[sl], sizeof(MeshParams), hipMemcpyHostToDevice, s));
    // pageable sources: the copies must finish before the host vectors go away
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipGetLastError());
    b->slot_busy[sl] = 1;
    b->meshes.push_back(m);
    b->used_v += h.n_verts; b->used_t += h.n_tris; b->used_e += h.n_edges; b->used_f += nf;
    b->sp = *sp;
    b->has_sp = true;
    b->dirty = true;
    b->snap_valid = false;
    *slot = sl;
    return CCFR_OK;
}

int ccfr_batch_remove(ccfr_batch* b, int32_t slot, ccfr_stream stream) {
    (void)stream;
    if (!b || slot < 0 || slot >= b->max_slots || !b->slot_busy[slot]) return CCFR_ERR_INVALID_ARG;
    for (BatchMesh& m : b->meshes)
        if (m.slot == slot && !m.removed) m.removed = true;
    b->slot_busy[slot] = 0;
    b->compact_pending = true;
    b->dirty = true;
    b->snap_valid = false;
    return CCFR_OK;
}

int ccfr_batch_step(ccfr_batch* b, ccfr_stream stream) {
    if (!b) return CCFR_ERR_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    ccfr_ctx* ctx = b->ctx;
    int rc;
    if (b->compact_pending) {
        rc = compact(b, s);
        if (rc) return rc;
    }
    if (b->meshes.empty()) return CCFR_OK;
    const long long gen0 = ctx->generation;
    rc = ensure_step(ctx, b->max_verts);
    if (rc) return rc;
    rc = ensure_grid(ctx, b->max_tris, b->max_edges, b->max_verts, b->max_verts);
    if (rc) return rc;
    rc = ensure_sizes(ctx, b->max_verts, b->max_tris, b->max_edges, 0, b->max_slots);
    if (rc) return rc;
    if (ctx->generation != gen0) drop_graph(ctx);
    if (b->tune_generation != ctx->tune_generation) {
        rc = refresh_table(b, s);
        if (rc) return rc;
    }
    if (b->dirty) {
        rc = rebuild_plan(b, s);
        if (rc) return rc;
    }
    rc = ensure_prof_events(ctx, b->sp.iters);
    if (rc) return rc;
    if (ctx->profiling) {
        ctx->prof_last_iters = b->sp.iters;
        ctx->prof_last_reuse = ctx->pair_skin > 0 ? 1 : ctx->pair_reuse;
    }
    {
        const Pool& P = b->pool[b->cur];
        const Pool& Q = b->pool[1 - b->cur];
        launch_copy(P.x, Q.x, 3 * b->used_v, s);
        launch_copy(P.v, Q.v, 3 * b->used_v, s);
        HIP_OK(hipGetLastError());
        b->snap_valid = true;
    }
    // the hierarchy's radix sort clears its scratch with memset operations,
    // which are not recorded into graphs here: those steps run directly
    if (!ctx->use_graphs || ctx->profiling || ctx->broad_phase == 1) {
        enqueue_step(ctx, b->plan, s);
        HIP_OK(hipGetLastError());
        return CCFR_OK;
    }
    const bool same = b->graph.valid && b->graph.generation == ctx->generation;
    return launch_recorded(ctx, b->graph, b->plan, b, &b->sp, same, s);
}

int ccfr_batch_rollback(ccfr_batch* b, ccfr_stream stream) {
    if (!b) return CCFR_ERR_INVALID_ARG;
    if (!b->snap_valid || b->compact_pending) return CCFR_ERR_NOT_READY;
    const hipStream_t s = (hipStream_t)stream;
    const Pool& P = b->pool[b->cur];
    const Pool& Q = b->pool[1 - b->cur];
    launch_copy(Q.x, P.x, 3 * b->used_v, s);
    launch_copy(Q.v, P.v, 3 * b->used_v, s);
    HIP_OK(hipGetLastError());
    return CCFR_OK;
}

int ccfr_batch_read(ccfr_batch* b, int32_t slot, float* x_host, float* v_host, ccfr_stream stream) {
    if (!b || slot < 0 || slot >= b->max_slots || !b->slot_busy[slot]) return CCFR_ERR_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    for (const BatchMesh& m : b->meshes) {
        if (m.slot != slot || m.removed) continue;
        HIP_OK(hipStreamSynchronize(s));
        const Pool& P = b->pool[b->cur];
        if (x_host) HIP_OK(hipMemcpy(x_host, P.x + 3 * m.v0, sizeof(float) * 3 * m.n_verts, hipMemcpyDeviceToHost));
        if (v_host) HIP_OK(hipMemcpy(v_host, P.v + 3 * m.v0, sizeof(float) * 3 * m.n_verts, hipMemcpyDeviceToHost));
        return CCFR_OK;
    }
    return CCFR_ERR_INVALID_ARG;
}

int ccfr_batch_stats(const ccfr_batch* b, int32_t* n_resident, int64_t* n_verts) {
    if (!b) return CCFR_ERR_INVALID_ARG;
    int32_t n = 0;
    long long nv = 0;
    for (const BatchMesh& m : b->meshes)
        if (!m.removed) { ++n; nv += m.n_verts; }
    if (n_resident) *n_resident = n;
    if (n_verts) *n_verts = nv;
    return CCFR_OK;
}

}  // extern "C"
