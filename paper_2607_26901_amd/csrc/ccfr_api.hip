// ccfr_api.hip -- host side of the C ABI declared in include/ccfr.h: contexts,
// device meshes, workspace growth, the per-call entry points and the recorded
// HIP graph of the XPBD substep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "ccfr_host.h"

using namespace ccfr;

using namespace ccfr::host;

namespace ccfr {
namespace host {

void drop_graph(ccfr_ctx* ctx) {
    if (ctx->graph.exec) (void)hipGraphExecDestroy(ctx->graph.exec);
    if (ctx->graph.graph) (void)hipGraphDestroy(ctx->graph.graph);
    ctx->graph = StepGraph{};
}

// Bucket table size (log2) for `entries` binned entries of one kind.
int grid_log2s(long long entries) { return std::max(6, ceil_log2(std::max(64LL, entries))); }

// Bucket tables (see TB_*) for these counts: four buckets per entry for the
// level-0 tables, so that few occupied cells share a bucket (the target tables
// are looked up by the queries, and the vertex table orders them: a crowded one
// would interleave distant blocks in one wavefront); the tables of the coarser
// levels get an eighth of their level-0 table, since few entries are binned
// above level 0 when the cell size follows the typical edge.
void grid_layout(long long T, long long E, long long F, long long N, int32_t log2k[TB_COUNT],
                 int32_t off[TB_COUNT + 1]) {
    log2k[TB_TRI0] = grid_log2s(4 * T);
    log2k[TB_TRIC] = std::max(6, log2k[TB_TRI0] - 3);
    log2k[TB_EDGE0] = grid_log2s(4 * E);
    log2k[TB_EDGEC] = std::max(6, log2k[TB_EDGE0] - 3);
    log2k[TB_PART] = grid_log2s(4 * F);
    log2k[TB_VERT] = grid_log2s(4 * N);
    off[0] = 0;
    for (int k = 0; k < TB_COUNT; ++k) off[k + 1] = off[k] + (1 << log2k[k]);
}

// Grows the grid for T triangles, E edges, F free particles and N vertices.
int ensure_grid(ccfr_ctx* ctx, long long T, long long E, long long F, long long N) {
    int32_t log2k[TB_COUNT], off[TB_COUNT + 1];
    grid_layout(T, E, F, N, log2k, off);
    const long long buckets = off[TB_COUNT];
    if (buckets > ctx->cap_buckets) {
        dev_free(ctx->cnt);
        dev_free(ctx->start);
        HIP_ALLOC(dev_alloc(&ctx->cnt, buckets));
        HIP_ALLOC(dev_alloc(&ctx->start, buckets + 1));
        HIP_OK(hipMemset(ctx->cnt, 0, sizeof(int32_t) * (size_t)buckets));
        ctx->cap_buckets = buckets;
        const long long ntmp = (buckets + 1023) / 1024 + 2;
        if (ntmp > ctx->cap_scan_tmp) {
            dev_free(ctx->scan_tmp);
            HIP_ALLOC(dev_alloc(&ctx->scan_tmp, ntmp));
            ctx->cap_scan_tmp = ntmp;
        }
        ctx->generation++;
    }
    const long long leaves = T + E + F;
    if (ctx->broad_phase == 1 && leaves > ctx->cap_lbvh) {
        LbvhWs& w = ctx->lbvh;
        dev_free(w.leaf_lo); dev_free(w.leaf_hi); dev_free(w.leaf_meta); dev_free(w.keys_in); dev_free(w.keys_out);
        dev_free(w.idx_in); dev_free(w.idx_out); dev_free(w.leaf_parent); dev_free(w.child);
        dev_free(w.node_parent); dev_free(w.node_flag); dev_free(w.node_lo); dev_free(w.node_hi);
        dev_free(ctx->lbvh_sort_temp);
        const long long L = std::max(leaves, 2LL);
        HIP_ALLOC(dev_alloc(&w.leaf_lo, 3 * L));
        HIP_ALLOC(dev_alloc(&w.leaf_hi, 3 * L));
        HIP_ALLOC(dev_alloc(&w.leaf_meta, L));
        HIP_ALLOC(dev_alloc(&w.keys_in, L));
        HIP_ALLOC(dev_alloc(&w.keys_out, L));
        HIP_ALLOC(dev_alloc(&w.idx_in, L));
        HIP_ALLOC(dev_alloc(&w.idx_out, L));
        HIP_ALLOC(dev_alloc(&w.leaf_parent, L));
        HIP_ALLOC(dev_alloc(&w.child, 2 * L));
        HIP_ALLOC(dev_alloc(&w.node_parent, L));
        HIP_ALLOC(dev_alloc(&w.node_flag, L));
        HIP_ALLOC(dev_alloc(&w.node_lo, 3 * L));
        HIP_ALLOC(dev_alloc(&w.node_hi, 3 * L));
        w.sort_temp_bytes = std::max<size_t>(lbvh_sort_temp_bytes((int)L), 16);
        HIP_ALLOC(dev_alloc(&ctx->lbvh_sort_temp, (long long)w.sort_temp_bytes));
        w.sort_temp = ctx->lbvh_sort_temp;
        ctx->cap_lbvh = L;
        ctx->generation++;
    }
    const long long targets = T + E + F + N;
    if (targets > ctx->cap_targets) {
        dev_free(ctx->rank);
        dev_free(ctx->key);
        dev_free(ctx->entries);
        dev_free(ctx->staged);
        HIP_ALLOC(dev_alloc(&ctx->rank, targets));
        HIP_ALLOC(dev_alloc(&ctx->key, targets));
        HIP_ALLOC(dev_alloc(&ctx->entries, targets));
        HIP_ALLOC(dev_alloc(&ctx->staged, targets));
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

int ensure_pairs(ccfr_ctx* ctx, long long vf, long long ee, long long vv, long long ve) {
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
    if (ve > ctx->cap_ve) {
        dev_free(ctx->ve);
        HIP_ALLOC(dev_alloc(&ctx->ve, 2 * ve));
        ctx->cap_ve = ve;
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
        HIP_ALLOC(dev_alloc(&ctx->slow_list, 2 * n_verts));
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
        dev_free(ctx->y_def);
        dev_free(ctx->halt_run);
        HIP_ALLOC(dev_alloc(&ctx->x_pred, 3 * n_verts));
        HIP_ALLOC(dev_alloc(&ctx->x_start, 3 * n_verts));
        HIP_ALLOC(dev_alloc(&ctx->p, 3 * n_verts));
        HIP_ALLOC(dev_alloc(&ctx->y_def, 3 * n_verts));
        HIP_ALLOC(dev_alloc(&ctx->halt_run, n_verts));
        ctx->cap_step = n_verts;
        ctx->generation++;
    }
    return CCFR_OK;
}

// Default list sizes for a scene of these sizes; later growth follows the
// observed needs (ccfr_reserve).
int ensure_sizes(ccfr_ctx* ctx, long long n_verts, long long n_tris, long long n_edges, long long n_free,
                 int n_meshes) {
    int rc = ensure_grid(ctx, n_tris, n_edges, n_free, n_verts);
    if (rc) return rc;
    rc = ensure_meshes(ctx, n_meshes);
    if (rc) return rc;
    const long long vf = 8LL * n_verts + 4096, ee = 8LL * n_edges + 4096, vv = 16LL * n_free + 4096;
    const long long ve = 8LL * n_free + 4096;
    rc = ensure_pairs(ctx, vf, ee, vv, ve);
    if (rc) return rc;
    return ensure_regions(ctx, n_verts, (vf + ee + vv + ve) / 2, 2 * (vf + ee + vv + ve));
}

bool params_ok(const ccfr_params* p) {
    if (!(p && std::isfinite(p->r) && p->r > 0.f && std::isfinite(p->xi) && p->xi >= 0.f &&
          std::isfinite(p->delta) && p->delta >= 0.f && std::isfinite(p->guard) && p->guard >= 0.f &&
          std::isfinite(p->eps_retract) && p->eps_retract >= 0.f && std::isfinite(p->eps_plesnik) &&
          p->eps_plesnik >= 0.f && p->max_passes >= 1))
        return false;
    if (p->flags & ~CCFR_FLAG_RESPONSE) return false;
    if (p->flags & CCFR_FLAG_RESPONSE)
        return p->delta > 0.f && p->delta <= 2.0f * p->r && std::isfinite(p->resp_compliance) &&
               p->resp_compliance >= 0.f && std::isfinite(p->vis_width) && p->vis_width >= 0.f &&
               std::isfinite(p->mu_s) && p->mu_s >= 0.f && std::isfinite(p->mu_k) && p->mu_k >= 0.f;
    return true;
}

bool step_params_ok(const ccfr_step_params* sp) {
    return sp && params_ok(&sp->collision) && sp->dt > 0.f && std::isfinite(sp->dt) && sp->iters >= 0 &&
           (sp->early_exit == 0 || sp->early_exit == 1) && std::isfinite(sp->conv_tol) && sp->conv_tol >= 0.f &&
           std::isfinite(sp->alpha) && sp->alpha >= 0.f && std::isfinite(sp->gravity[0]) &&
           std::isfinite(sp->gravity[1]) && std::isfinite(sp->gravity[2]);
}

// Per-mesh device parameters: the box pad (one FP32 rounding of an FP64 sum) and
// a grid cell large enough that typical primitives span at most two cells.  A
// build that serves skin_iters more iterations widens moving boxes by about
// skin_iters r per side, one that adapts to the motion by skin_mult r (pad_wide:
// the FP32 sum rounded up one step, so that pad_wide - pad >= skin_mult r); the
// cell is sized for that width (with slack for the rounding term), so that a
// particle's box still fits one cell.
MeshParams mesh_params(const ccfr_params* p, float typ_len, int salt, float cell_scale, int skin_iters,
                       int skin_mult) {
    MeshParams m{};
    m.r = p->r;
    m.xi = p->xi;
    m.pad = (float)((double)p->r + 0.5 * (double)p->xi + 0.5 * (double)p->delta + (double)p->guard);
    m.two_r = 2.0f * p->r;
    m.eps_retract = p->eps_retract;
    m.eps_plesnik = p->eps_plesnik;
    m.pad_wide = m.pad;
    if (skin_mult > 0) {
        const double want = (double)skin_mult * (double)p->r;
        m.pad_wide = (float)((double)m.pad + want);
        while ((double)m.pad_wide - (double)m.pad < want)
            m.pad_wide = std::nextafter(m.pad_wide, std::numeric_limits<float>::infinity());
    }
    const double wide = (double)m.pad + 1.25 * std::max(skin_iters, skin_mult) * (double)p->r;
    const double h = std::max(2.02 * wide, (double)cell_scale * (1.2 * (double)typ_len + 2.0 * wide));
    m.h = (float)h;
    m.inv_h = (float)(1.0 / h);
    m.max_passes = p->max_passes;
    m.mesh_salt = salt;
    m.response = (p->flags & CCFR_FLAG_RESPONSE) ? 1 : 0;
    m.delta = p->delta;
    m.resp_compliance = p->resp_compliance;
    m.vis_width = p->vis_width;
    m.mu_s = p->mu_s;
    m.mu_k = p->mu_k;
    return m;
}

namespace {

Scene make_scene(const ccfr_mesh* m, const float* x, const ccfr_params* p, int skin_iters = 0,
                 int skin_mult = 0) {
    Scene sc{};
    sc.n_verts = m->n_verts;
    sc.n_tris = m->n_tris;
    sc.n_edges = m->n_edges;
    sc.n_free = m->n_free;
    sc.x = x;
    sc.inv_mass = m->inv_mass_d;
    sc.tris = m->tris_d;
    sc.edges = m->edges_d;
    sc.free_list = m->free_list_d;
    sc.vflags = m->vflags_d;
    sc.prm.table = nullptr;
    sc.prm.vmesh = nullptr;
    sc.prm.one = mesh_params(p, m->typ_len, 0, m->ctx->cell_scale, skin_iters, skin_mult);
    return sc;
}

// The table is sized for the entries of the grid build at hand (not the allocation), so the
// scan and the bucket range follow the meshes actually present.
GridWs grid_ws(ccfr_ctx* ctx, const Scene& sc, int n_meshes) {
    GridWs g{};
    grid_layout(sc.n_tris, sc.n_edges, sc.n_free, sc.n_verts, g.log2k, g.off);
    g.cnt = ctx->cnt;
    g.start = ctx->start;
    g.rank = ctx->rank;
    g.key = ctx->key;
    g.entries = ctx->entries;
    g.staged = ctx->staged;
    g.level_mask = ctx->level_mask;
    g.n_meshes = n_meshes;
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

// The context's candidate lists.
PairLists ctx_lists(const ccfr_ctx* ctx) {
    return PairLists{ctx->vf, ctx->ee, ctx->vv, ctx->ve, ctx->cap_vf, ctx->cap_ee, ctx->cap_vv, ctx->cap_ve};
}

// broad phase into the context's lists; `standalone` brackets it with its own
// counter reset and build close (inside a substep the neighbouring kernels do both)
void enqueue_candidates(ccfr_ctx* ctx, const Scene& sc, int n_meshes, hipStream_t s, const Marks& mk,
                        bool standalone) {
    GridWs g = grid_ws(ctx, sc, n_meshes);
    mk.mark(0, 0);
    if (standalone) launch_reset_build(ctx->counters_d, g.level_mask, g.n_meshes, s);
    if (ctx->broad_phase == 1) {
        // the hierarchy: build (stage 0), then the queries (stage 1)
        launch_lbvh_build(sc, ctx->lbvh, ctx->counters_d, s);
        mk.mark(0, 1);
        const PairLists pl = ctx_lists(ctx);
        mk.mark(1, 0);
        launch_lbvh_query(sc, ctx->lbvh, pl, ctx->counters_d, s);
        mk.mark(1, 1);
        if (standalone) launch_finalize_pairs(g, pl, ctx->counters_d, s);
        return;
    }
    launch_grid_count(sc, g, ctx->counters_d, s);
    launch_scan(g.cnt, g.start, g.cnt, g.off[TB_COUNT], g.scan_tmp, s,
                sc.build_gated ? &ctx->counters_d->rebuild : nullptr, sc.skip);
    launch_grid_scatter(sc, g, ctx->counters_d, s);
    mk.mark(0, 1);
    const PairLists pl = ctx_lists(ctx);
    mk.mark(1, 0);
    launch_pairs(sc, g, pl, ctx->counters_d, ctx->pair_split, s);
    mk.mark(1, 1);
    if (standalone) launch_finalize_pairs(g, pl, ctx->counters_d, s);
}

// Slots per vertex when a substep's regions go into per-vertex slots (the
// context's half-space buffer divided evenly), or 0 for CSR regions.
int32_t step_slot_stride(const ccfr_ctx* ctx, int n_verts) {
    if (ctx->csr_in_step || n_verts <= 0) return 0;
    return (int32_t)std::max<long long>(1, std::min<long long>(ctx->cap_hs / n_verts, 1LL << 20));
}

// narrow phase into the context's regions; inside a substep (`in_step`) both
// builds are closed by launch_close_iteration, and with slot_stride > 0 the
// half-spaces go into per-vertex slots (no count scan): from the contact list
// by a fill launch, or with the direct_regions knob straight from the narrow
// phase (no contact list, one launch fewer)
void enqueue_regions(ccfr_ctx* ctx, const Scene& sc, const PairLists& pl, const int32_t* counts, hipStream_t s,
                     const Marks& mk, bool in_step, int32_t slot_stride = 0,
                     const ColourJob* job_contacts = nullptr, const ColourJob* job_fill = nullptr) {
    const bool slots = in_step && slot_stride > 0;
    const bool direct = slots && ctx->direct_regions;
    mk.mark(2, 0);
    launch_contacts(sc, pl, counts, ctx->contacts, ctx->cap_contacts, slots && !direct ? nullptr : ctx->vcount,
                    ctx->counters_d, s, direct ? ctx->hs : nullptr, direct ? slot_stride : 0, job_contacts);
    mk.mark(2, 1);
    mk.mark(3, 0);
    if (slots) {
        if (!direct)
            launch_fill_slots(sc, ctx->contacts, ctx->cap_contacts, ctx->vcount, ctx->hs, slot_stride,
                              ctx->counters_d, s, job_fill);
        mk.mark(3, 1);
        return;
    }
    launch_scan(ctx->vcount, ctx->offsets, nullptr, sc.n_verts, ctx->scan_tmp, s);
    launch_fill(sc, ctx->contacts, ctx->cap_contacts, ctx->offsets, ctx->vcount, ctx->hs, ctx->cap_hs,
                ctx->counters_d, !in_step, s);
    mk.mark(3, 1);
}

int32_t* counts_ptr(ccfr_ctx* ctx) { return &ctx->counters_d->n_vf; }

}  // namespace

int ensure_prof_events(ccfr_ctx* ctx, int iters) {
    if (!ctx->profiling || iters <= ctx->prof_iters) return CCFR_OK;
    drop_graph(ctx);
    const size_t need = (size_t)iters * kStages * 2;
    while (ctx->prof_events.size() < need) {
        hipEvent_t e = nullptr;
        HIP_OK(hipEventCreate(&e));
        ctx->prof_events.push_back(e);
    }
    ctx->prof_iters = iters;
    return CCFR_OK;
}

// The substep of Alg. 4 (without response, friction or early exit).
void enqueue_step(ccfr_ctx* ctx, const StepPlan& plan, hipStream_t s) {
    // with the convergence check every kernel of an iteration returns at once
    // once the substep's iterations have ended
    const uint32_t* skip = plan.early_exit ? &ctx->counters_d->converged : nullptr;
    Scene sc = plan.sc;
    sc.skip = skip;
    const int n = sc.n_verts;
    launch_predict(n, plan.x, plan.v, sc.inv_mass, plan.dt, plan.gx, plan.gy, plan.gz, ctx->x_pred, ctx->x_start, s,
                   ctx->halt_run, ctx->counters_d, plan.early_exit ? 0 : plan.iters);
    if (plan.has_stretch) launch_fill_zero(plan.lambda, plan.n_edges, s);
    // counters and level masks start clear; each iteration's close clears them
    // for the next one
    launch_reset_build(ctx->counters_d, ctx->level_mask, plan.n_meshes, s);
    // Fixed grouping: a candidate build serves `reuse` consecutive iterations
    // (the last group of the substep may be shorter); its boxes are widened for
    // the iterations after the first.  Adaptive (plan.skin > 0): every build's
    // moving boxes are widened by the skin, and from the second iteration on a
    // decision kernel asks for a new build only once the summed anchor moves
    // since the last one may exceed it; the stage's kernels run every iteration
    // and return at once when no build is asked for.
    const bool adaptive = plan.skin > 0.0;
    const int reuse = adaptive ? 1 : std::max(1, ctx->pair_reuse);
    const PairCaps caps = ctx_lists(ctx).caps();
    const int32_t slots = step_slot_stride(ctx, n);
    // The stretch pass: the first colour runs with p's reset to the
    // prediction, the last one (of two or more) inside the projection's fast
    // kernel, which reads its result, and with three or more colours the one
    // before the last too.  With per-vertex slots the pass runs in
    // blocks of kernels already on the path, since none of them reads p: the
    // next iteration's reset and first colour in extra blocks of the slow
    // projection (the first iteration's in a launch of their own), the second,
    // third and fourth colours in the first blocks of the narrow phase, the
    // slot fill (when there is one) and the closing kernel; further colours
    // get launches of their own.
    StretchColor0 c0{};
    if (plan.has_stretch && !plan.col_total.empty())
        c0 = StretchColor0{plan.edges_sorted, plan.rest_sorted, plan.segs + plan.col_first[0], plan.col_nseg[0],
                           plan.col_total[0], sc.inv_mass, plan.lambda, plan.alpha_t, sc.vflags};
    const int n_col = (int)plan.col_total.size();
    // with the response (Sec. 3.3), which acts on the whole pass's result, no
    // stretch colour is folded into the projection; in a batch the response
    // kernel runs when any mesh asks for it and passes the others' vertices by
    const bool response = sc.prm.table ? plan.response_any : sc.prm.one.response != 0;
    const bool fold = plan.has_stretch && n_col >= 2 && plan.last_edge && plan.lambda_alt && !response;
    const bool fold2 = fold && n_col >= 3 && plan.prev_edge;
    const int n_launched = n_col - (fold2 ? 2 : fold ? 1 : 0);     // colours before the folded ones
    const bool hosted = fold && slots > 0;
    const RestartJob restart{ctx->x_pred, ctx->p, 3LL * n, c0};
    auto colour_job = [&](int c) {
        ColourJob j{};
        if (hosted && c >= 1 && c < n_launched)
            j = ColourJob{plan.edges_sorted, plan.rest_sorted, plan.segs + plan.col_first[c], plan.col_nseg[c],
                          plan.col_total[c], sc.inv_mass, ctx->p, plan.lambda, plan.alpha_t};
        return j;
    };
    const bool direct = slots > 0 && ctx->direct_regions;     // no slot fill launch to host a colour
    const ColourJob job_contacts = colour_job(1), job_fill = direct ? ColourJob{} : colour_job(2),
                    job_close = colour_job(direct ? 2 : 3);
    const int first_launched = direct ? 3 : 4;                   // first colour with a launch of its own
    if (hosted)
        launch_close_iteration(ctx->x_pred, ctx->p, 3LL * n, ctx->counters_d, ctx->level_mask, plan.n_meshes, n,
                               ctx->offsets, caps, direct ? -1 : ctx->cap_contacts, ctx->cap_hs, false, s, slots, &c0, false);
    for (int it = 0; it < plan.iters; ++it) {
        const Marks mk{ctx, it, s};
        const int first = it - it % reuse;
        const int group = std::min(reuse, plan.iters - first);
        if (plan.early_exit) launch_decide_converged(ctx->counters_d, plan.conv_tol, it == 0 ? 1 : 0, s);
        if (adaptive) {
            if (it > 0) launch_decide_build(ctx->counters_d, ctx->level_mask, plan.n_meshes, plan.skin, caps, s, skip);
            Scene sb = sc;
            sb.skin_wide = 1;
            sb.build_gated = 1;
            enqueue_candidates(ctx, sb, plan.n_meshes, s, mk, false);
        } else if (it == first) {
            Scene sb = sc;
            sb.skin_iters = group - 1;
            enqueue_candidates(ctx, sb, plan.n_meshes, s, mk, false);
        } else {
            for (int st = 0; st < 2; ++st) {      // no build: empty stage marks
                mk.mark(st, 0);
                mk.mark(st, 1);
            }
        }
        enqueue_regions(ctx, sc, ctx_lists(ctx), counts_ptr(ctx), s, mk, true, slots, &job_contacts, &job_fill);
        mk.mark(4, 0);
        const bool close_pairs = adaptive ? it == plan.iters - 1 : it == first + group - 1;
        if (hosted)
            launch_close_iteration(nullptr, nullptr, 0, ctx->counters_d, ctx->level_mask, plan.n_meshes, n,
                                   ctx->offsets, caps, direct ? -1 : ctx->cap_contacts, ctx->cap_hs, close_pairs, s, slots, nullptr,
                                   true, &job_close, skip);
        else
            launch_close_iteration(ctx->x_pred, ctx->p, 3LL * n, ctx->counters_d, ctx->level_mask, plan.n_meshes, n,
                                   ctx->offsets, caps, direct ? -1 : ctx->cap_contacts, ctx->cap_hs, close_pairs, s, slots, &c0,
                                   true, nullptr, skip);
        if (plan.has_stretch)
            for (int c = hosted ? first_launched : 1; c < n_launched; ++c)
                launch_stretch_segments(plan.edges_sorted, plan.rest_sorted, plan.segs + plan.col_first[c],
                                        plan.col_nseg[c], plan.col_total[c], sc.inv_mass, ctx->p, plan.lambda,
                                        plan.alpha_t, s, skip);
        if (response) {
            ResponseArgs ra{};
            ra.n_verts = n;
            ra.offsets = ctx->offsets;
            ra.hs = ctx->hs;
            ra.slot_counts = ctx->vcount;
            ra.slot_stride = slots;
            ra.inv_mass = sc.inv_mass;
            ra.x_anchor = plan.x;
            ra.p = ctx->p;
            ra.dt = plan.dt;
            ra.prm = sc.prm;
            ra.skip = skip;
            ra.list = ctx->slow_list;         // free until the projection lists its vertices
            ra.c = ctx->counters_d;
            launch_response(ra, s);
        }
        mk.mark(4, 1);
        ProjectArgs pa{};
        pa.n_verts = n;
        pa.offsets = ctx->offsets;
        pa.hs = ctx->hs;
        pa.cap_hs = ctx->cap_hs;
        pa.inv_mass = sc.inv_mass;
        pa.y_in = nullptr;
        pa.p = ctx->p;
        pa.x_anchor = plan.x;
        pa.y_out = nullptr;
        pa.halted = nullptr;
        pa.sort_key = ctx->sort_key;
        pa.sort_idx = ctx->sort_idx;
        pa.slow_list = ctx->slow_list;
        pa.motion_max = adaptive ? &ctx->counters_d->maxima[0][kMaxMotion] : nullptr;
        pa.slot_counts = ctx->vcount;
        pa.slot_stride = slots;
        pa.prm = sc.prm;
        pa.skip = skip;
        pa.shortfall_max = plan.early_exit ? &ctx->counters_d->maxima[0][kMaxShortfall] : nullptr;
        pa.halt_run = ctx->halt_run;
        if (fold)   // the multipliers of the folded colour alternate between two arrays
            pa.sl = StretchLast{plan.last_edge, fold2 ? plan.prev_edge : nullptr, plan.rest_sorted,
                                (it & 1) ? plan.lambda_alt : plan.lambda, (it & 1) ? plan.lambda : plan.lambda_alt,
                                plan.alpha_t, ctx->y_def};
        if (hosted && it + 1 < plan.iters) pa.next = restart;
        mk.mark(5, 0);
        launch_project(pa, ctx->counters_d, false, s);
        mk.mark(5, 1);
        if (plan.trace) launch_copy(plan.x, plan.trace + (size_t)it * 3 * (size_t)n, 3LL * n, s);
    }
    launch_update_velocity(n, plan.x, ctx->x_start, 1.0f / plan.dt, plan.v, s);
}

int launch_recorded(ccfr_ctx* ctx, StepGraph& G, const StepPlan& plan, const void* owner,
                    const ccfr_step_params* sp, bool same, hipStream_t s) {
    if (!same) {
        if (G.exec) (void)hipGraphExecDestroy(G.exec);
        if (G.graph) (void)hipGraphDestroy(G.graph);
        G = StepGraph{};
        HIP_OK(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        enqueue_step(ctx, plan, ctx->capture_stream);
        hipGraph_t graph = nullptr;
        HIP_OK(hipStreamEndCapture(ctx->capture_stream, &graph));
        hipGraphExec_t exec = nullptr;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return CCFR_ERR_HIP;
        }
        G.valid = true;
        G.owner = owner;
        G.x = plan.x;
        G.v = plan.v;
        G.sp = *sp;
        G.generation = ctx->generation;
        G.graph = graph;
        G.exec = exec;
    }
    HIP_OK(hipGraphLaunch(G.exec, s));
    return CCFR_OK;
}

int prepare_mesh(int32_t n_verts, const int32_t* tris, int32_t n_tris, const int32_t* edges, int32_t n_edges,
                 const float* inv_mass, const float* rest_x, MeshHost* out) {
    if (n_verts < 0 || n_tris < 0 || n_edges < 0 || !inv_mass || !out) return CCFR_ERR_INVALID_ARG;
    // pair records keep a primitive index in 30 bits
    if (n_verts > kMaxPrims || n_tris > kMaxPrims || n_edges > kMaxPrims) return CCFR_ERR_INVALID_ARG;
    if (n_tris > 0 && !tris) return CCFR_ERR_INVALID_ARG;
    for (long long i = 0; i < 3LL * n_tris; ++i)
        if (tris[i] < 0 || tris[i] >= n_verts) return CCFR_ERR_INVALID_ARG;
    for (int32_t i = 0; i < n_verts; ++i)
        if (!(inv_mass[i] >= 0.f) || !std::isfinite(inv_mass[i])) return CCFR_ERR_INVALID_ARG;
    MeshHost& m = *out;
    m = MeshHost{};
    m.n_verts = n_verts;
    m.n_tris = n_tris;
    m.tris.assign(tris ? tris : nullptr, tris ? tris + 3LL * n_tris : nullptr);
    std::vector<int32_t>& E = m.edges;
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
        if ((long long)(E.size() / 2) > kMaxPrims) return CCFR_ERR_INVALID_ARG;
        n_edges = (int32_t)(E.size() / 2);
    }
    m.n_edges = n_edges;
    // free particles: vertices in no edge and no triangle
    m.vflags.assign(n_verts, VF_FREE);
    for (int32_t v : m.tris) m.vflags[v] = 0;
    for (int32_t v : E) m.vflags[v] = 0;
    for (int32_t v = 0; v < n_verts; ++v)
        if (m.vflags[v] & VF_FREE) m.free_list.push_back(v);
    // edge length the grid is sized for: the longest edge not longer than 8x the
    // median over all binned primitives, free particles counting as length 0 (a
    // particle system with a few long wall edges gets cells sized by the pad)
    if (n_edges > 0 && rest_x) {
        std::vector<float> len(n_edges);
        for (int32_t e = 0; e < n_edges; ++e) {
            double d2 = 0;
            for (int k = 0; k < 3; ++k) {
                const double d = (double)rest_x[3 * E[2 * e] + k] - (double)rest_x[3 * E[2 * e + 1] + k];
                d2 += d * d;
            }
            len[e] = (float)std::sqrt(d2);
        }
        std::vector<float> sorted = len;
        sorted.resize(len.size() + m.free_list.size(), 0.f);
        const size_t mid = sorted.size() / 2;
        std::nth_element(sorted.begin(), sorted.begin() + mid, sorted.end());
        const float med = sorted[mid];
        for (float l : len)
            if (l <= 8.f * med) m.typ_len = std::max(m.typ_len, l);
    }
    // greedy colouring in edge-index order, then edges sorted by (colour, index)
    std::vector<int32_t> color(n_edges, 0);
    std::vector<uint64_t> used(n_verts, 0);
    int n_colors = 0;
    for (int32_t e = 0; e < n_edges; ++e) {
        const int32_t a = E[2 * e], b = E[2 * e + 1];
        const uint64_t taken = used[a] | used[b];
        int c = 0;
        while (c < 64 && ((taken >> c) & 1ull)) ++c;
        if (c == 64) return CCFR_ERR_INVALID_ARG;   // a vertex with more than 32 edges
        color[e] = c;
        used[a] |= 1ull << c;
        used[b] |= 1ull << c;
        n_colors = std::max(n_colors, c + 1);
    }
    m.color_begin.assign(n_colors + 1, 0);
    for (int32_t e = 0; e < n_edges; ++e) m.color_begin[color[e] + 1]++;
    for (int c = 0; c < n_colors; ++c) m.color_begin[c + 1] += m.color_begin[c];
    m.edges_sorted.assign(2LL * n_edges, 0);
    m.rest_sorted.assign(n_edges, 0.f);
    std::vector<int32_t> cur(m.color_begin.begin(), m.color_begin.end() - 1);
    for (int32_t e = 0; e < n_edges; ++e) {
        const int32_t pos = cur[color[e]]++;
        m.edges_sorted[2 * pos] = E[2 * e];
        m.edges_sorted[2 * pos + 1] = E[2 * e + 1];
        if (rest_x) {
            double d2 = 0;
            for (int k = 0; k < 3; ++k) {
                const double d = (double)rest_x[3 * E[2 * e] + k] - (double)rest_x[3 * E[2 * e + 1] + k];
                d2 += d * d;
            }
            m.rest_sorted[pos] = (float)std::sqrt(d2);
        }
    }
    m.has_stretch = rest_x != nullptr && n_edges > 0;
    if (m.has_stretch)
        for (int32_t e = m.color_begin[0]; e < m.color_begin[1]; ++e) {
            m.vflags[m.edges_sorted[2 * e]] |= VF_COLOR0;
            m.vflags[m.edges_sorted[2 * e + 1]] |= VF_COLOR0;
        }
    return CCFR_OK;
}

}  // namespace host
}  // namespace ccfr

namespace {

StepPlan mesh_plan(ccfr_ctx* ctx, const ccfr_mesh* m, float* x, float* v, const ccfr_step_params* sp) {
    StepPlan plan;
    plan.sc = make_scene(m, x, &sp->collision, ctx_skin_iters(ctx), ctx_skin_mult(ctx));
    if (ctx_skin_mult(ctx) > 0) plan.skin = (double)plan.sc.prm.one.pad_wide - (double)plan.sc.prm.one.pad;
    plan.x = x;
    plan.v = v;
    plan.n_meshes = 1;
    plan.has_stretch = m->has_stretch;
    plan.edges_sorted = m->edges_sorted_d;
    plan.rest_sorted = m->rest_sorted_d;
    plan.lambda = m->lambda_d;
    plan.lambda_alt = m->lambda_alt_d;
    plan.last_edge = m->last_edge_d;
    plan.prev_edge = m->prev_edge_d;
    plan.n_edges = m->n_edges;
    plan.segs = m->segs_d;
    const int nc = (int)m->color_begin.size() - 1;
    for (int c = 0; c < nc; ++c) {
        plan.col_first.push_back(c);
        plan.col_nseg.push_back(1);
        plan.col_total.push_back(m->color_begin[c + 1] - m->color_begin[c]);
    }
    plan.dt = sp->dt;
    plan.gx = sp->gravity[0];
    plan.gy = sp->gravity[1];
    plan.gz = sp->gravity[2];
    plan.alpha_t = sp->alpha / (sp->dt * sp->dt);
    plan.iters = sp->iters;
    plan.early_exit = sp->early_exit != 0;
    plan.conv_tol = sp->conv_tol;
    (void)ctx;
    return plan;
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
    const char* cs = std::getenv("CCFR_CSR_IN_STEP");
    ctx->csr_in_step = cs && cs[0] == '1';
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
    dev_free(ctx->entries); dev_free(ctx->staged); dev_free(ctx->level_mask); dev_free(ctx->scan_tmp);
    dev_free(ctx->vf); dev_free(ctx->ee); dev_free(ctx->vv); dev_free(ctx->ve);
    dev_free(ctx->contacts); dev_free(ctx->vcount); dev_free(ctx->offsets); dev_free(ctx->slow_list);
    dev_free(ctx->hs);
    dev_free(ctx->sort_key); dev_free(ctx->sort_idx);
    dev_free(ctx->x_pred); dev_free(ctx->x_start); dev_free(ctx->p); dev_free(ctx->y_def); dev_free(ctx->halt_run);
    {
        LbvhWs& w = ctx->lbvh;
        dev_free(w.leaf_lo); dev_free(w.leaf_hi); dev_free(w.leaf_meta); dev_free(w.keys_in); dev_free(w.keys_out);
        dev_free(w.idx_in); dev_free(w.idx_out); dev_free(w.leaf_parent); dev_free(w.child);
        dev_free(w.node_parent); dev_free(w.node_flag); dev_free(w.node_lo); dev_free(w.node_hi);
        dev_free(ctx->lbvh_sort_temp);
    }
    for (hipEvent_t e : ctx->prof_events) (void)hipEventDestroy(e);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
}

int ccfr_mesh_create(ccfr_ctx* ctx, int32_t n_verts, const int32_t* tris, int32_t n_tris, const int32_t* edges,
                     int32_t n_edges, const float* inv_mass, const float* rest_x, ccfr_mesh** out) {
    if (!ctx || !out) return CCFR_ERR_INVALID_ARG;
    *out = nullptr;
    MeshHost h;
    int rc = prepare_mesh(n_verts, tris, n_tris, edges, n_edges, inv_mass, rest_x, &h);
    if (rc) return rc;
    HIP_OK(hipSetDevice(ctx->device));
    ccfr_mesh* m = new (std::nothrow) ccfr_mesh();
    if (!m) return CCFR_ERR_NO_MEMORY;
    m->ctx = ctx;
    m->n_verts = h.n_verts;
    m->n_tris = h.n_tris;
    m->n_edges = h.n_edges;
    m->n_free = (int32_t)h.free_list.size();
    m->edges_h = h.edges;
    m->typ_len = h.typ_len;
    m->color_begin = h.color_begin;
    m->has_stretch = h.has_stretch;
    std::vector<int2> segs;
    for (size_t c = 0; c + 1 < h.color_begin.size(); ++c) segs.push_back(make_int2(h.color_begin[c], 0));
    hipError_t e = hipSuccess;
    auto put = [&](auto** dst, const auto* src, long long count) {
        if (e != hipSuccess) return;
        e = dev_alloc(dst, count);
        if (e == hipSuccess && count > 0)
            e = hipMemcpy((void*)*dst, (const void*)src, sizeof(**dst) * (size_t)count, hipMemcpyHostToDevice);
    };
    put(&m->tris_d, h.tris.data(), 3LL * h.n_tris);
    put(&m->edges_d, h.edges.data(), 2LL * h.n_edges);
    put(&m->inv_mass_d, inv_mass, h.n_verts);
    put(&m->free_list_d, h.free_list.data(), (long long)h.free_list.size());
    put(&m->vflags_d, h.vflags.data(), h.n_verts);
    put(&m->edges_sorted_d, h.edges_sorted.data(), 2LL * h.n_edges);
    put(&m->rest_sorted_d, h.rest_sorted.data(), h.n_edges);
    put(&m->segs_d, segs.data(), (long long)segs.size());
    if (e == hipSuccess) e = dev_alloc(&m->lambda_d, std::max<long long>(h.n_edges, 1));
    // the map of the last stretch colour, run inside the projection
    const int nc = (int)h.color_begin.size() - 1;
    if (e == hipSuccess && h.has_stretch && nc >= 2) {
        e = dev_alloc(&m->lambda_alt_d, h.n_edges);
        if (e == hipSuccess) e = dev_alloc(&m->last_edge_d, h.n_verts);
        if (e == hipSuccess && nc >= 3) e = dev_alloc(&m->prev_edge_d, h.n_verts);
        if (e == hipSuccess) {
            launch_last_colour_map(m->edges_sorted_d, m->segs_d + (nc - 1), 1,
                                   h.color_begin[nc] - h.color_begin[nc - 1], h.n_verts, m->last_edge_d, nullptr);
            if (nc >= 3)
                launch_last_colour_map(m->edges_sorted_d, m->segs_d + (nc - 2), 1,
                                       h.color_begin[nc - 1] - h.color_begin[nc - 2], h.n_verts, m->prev_edge_d,
                                       nullptr);
            e = hipDeviceSynchronize();
        }
    }
    if (e != hipSuccess) {
        ccfr_mesh_destroy(m);
        return CCFR_ERR_NO_MEMORY;
    }
    rc = ensure_sizes(ctx, m->n_verts, m->n_tris, m->n_edges, m->n_free, 1);
    if (rc) {
        ccfr_mesh_destroy(m);
        return rc;
    }
    *out = m;
    return CCFR_OK;
}

void ccfr_mesh_destroy(ccfr_mesh* m) {
    if (!m) return;
    if (m->ctx && m->ctx->graph.owner == m) drop_graph(m->ctx);
    dev_free(m->tris_d); dev_free(m->edges_d); dev_free(m->inv_mass_d); dev_free(m->free_list_d);
    dev_free(m->vflags_d); dev_free(m->edges_sorted_d); dev_free(m->rest_sorted_d); dev_free(m->lambda_d);
    dev_free(m->segs_d); dev_free(m->lambda_alt_d); dev_free(m->last_edge_d); dev_free(m->prev_edge_d);
    delete m;
}

int ccfr_mesh_edges(const ccfr_mesh* m, int32_t* n_edges, int32_t* edges_host) {
    if (!m || !n_edges) return CCFR_ERR_INVALID_ARG;
    *n_edges = m->n_edges;
    if (edges_host) std::memcpy(edges_host, m->edges_h.data(), sizeof(int32_t) * m->edges_h.size());
    return CCFR_OK;
}

const float* ccfr_mesh_inv_mass_dev(const ccfr_mesh* m) { return m ? m->inv_mass_d : nullptr; }

int ccfr_reserve(ccfr_ctx* ctx, int64_t vf, int64_t ee, int64_t vv, int64_t ve, int64_t contacts,
                 int64_t halfspaces, ccfr_stream stream) {
    if (!ctx || vf < 0 || ee < 0 || vv < 0 || ve < 0 || contacts < 0 || halfspaces < 0) return CCFR_ERR_INVALID_ARG;
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    if (ctx->vcount) HIP_OK(hipMemset(ctx->vcount, 0, sizeof(int32_t) * (size_t)ctx->cap_verts));
    const long long gen = ctx->generation;
    int rc = ensure_pairs(ctx, vf, ee, vv, ve);
    if (rc) return rc;
    rc = ensure_regions(ctx, 0, contacts, halfspaces);
    if (rc) return rc;
    if (ctx->generation != gen) drop_graph(ctx);
    return CCFR_OK;
}

int ccfr_build_candidates(ccfr_ctx* ctx, const ccfr_mesh* mesh, const float* x_anchor_dev, const ccfr_params* params,
                          ccfr_candidates* out, ccfr_stream stream) {
    if (!ctx || !mesh || !out || !params_ok(params)) return CCFR_ERR_INVALID_ARG;
    if (!x_anchor_dev && mesh->n_verts > 0) return CCFR_ERR_INVALID_ARG;
    if (mesh->ctx != ctx) return CCFR_ERR_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    const Scene sc = make_scene(mesh, x_anchor_dev, params);
    enqueue_candidates(ctx, sc, 1, s, Marks{ctx, -1, s}, true);
    HIP_OK(hipGetLastError());
    out->vf = ctx->vf;
    out->ee = ctx->ee;
    out->vv = ctx->vv;
    out->counts_dev = counts_ptr(ctx);
    out->cap_vf = ctx->cap_vf;
    out->cap_ee = ctx->cap_ee;
    out->cap_vv = ctx->cap_vv;
    out->ve = ctx->ve;
    out->cap_ve = ctx->cap_ve;
    return CCFR_OK;
}

int ccfr_build_regions(ccfr_ctx* ctx, const ccfr_mesh* mesh, const float* x_anchor_dev, const ccfr_candidates* c,
                       const ccfr_params* params, ccfr_regions* out, ccfr_stream stream) {
    if (!ctx || !mesh || !c || !out || !params_ok(params)) return CCFR_ERR_INVALID_ARG;
    if (!x_anchor_dev && mesh->n_verts > 0) return CCFR_ERR_INVALID_ARG;
    if (!c->counts_dev || c->cap_vf < 0 || c->cap_ee < 0 || c->cap_vv < 0 || c->cap_ve < 0)
        return CCFR_ERR_INVALID_ARG;
    if ((c->cap_vf > 0 && !c->vf) || (c->cap_ee > 0 && !c->ee) || (c->cap_vv > 0 && !c->vv) ||
        (c->cap_ve > 0 && !c->ve))
        return CCFR_ERR_INVALID_ARG;
    if (mesh->ctx != ctx) return CCFR_ERR_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    const Scene sc = make_scene(mesh, x_anchor_dev, params);
    const PairLists pl{c->vf, c->ee, c->vv, c->ve, c->cap_vf, c->cap_ee, c->cap_vv, c->cap_ve};
    enqueue_regions(ctx, sc, pl, c->counts_dev, s, Marks{ctx, -1, s}, false);
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
    if (!ctx || !regions || !params_ok(params)) return CCFR_ERR_INVALID_ARG;
    if ((!inv_mass_dev || !y_in_dev || !y_out_dev) && regions->n_verts > 0) return CCFR_ERR_INVALID_ARG;
    if (regions->n_verts < 0 || !regions->offsets || (regions->cap > 0 && !regions->hs) || regions->cap < 0)
        return CCFR_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(regions->hs) % 16 != 0) return CCFR_ERR_INVALID_ARG;   // 16-byte plane loads
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
    pa.prm.one = mesh_params(params, 0.f, 0, 1.0f);
    launch_project(pa, ctx->counters_d, true, (hipStream_t)stream);
    HIP_OK(hipGetLastError());
    return CCFR_OK;
}

int ccfr_apply_response(ccfr_ctx* ctx, const ccfr_regions* regions, const float* inv_mass_dev,
                        const float* y_in_dev, const ccfr_params* params, float dt, float* y_out_dev,
                        ccfr_stream stream) {
    if (!ctx || !regions || !params_ok(params) || !(dt > 0.f) || !std::isfinite(dt)) return CCFR_ERR_INVALID_ARG;
    if ((!inv_mass_dev || !y_in_dev || !y_out_dev) && regions->n_verts > 0) return CCFR_ERR_INVALID_ARG;
    if (regions->n_verts < 0 || !regions->offsets || (regions->cap > 0 && !regions->hs) || regions->cap < 0)
        return CCFR_ERR_INVALID_ARG;
    // the list of vertices with large regions needs room for every vertex
    if (regions->n_verts > ctx->cap_verts) {
        HIP_OK(hipStreamSynchronize((hipStream_t)stream));
        const long long gen = ctx->generation;
        int rc = ensure_regions(ctx, regions->n_verts, 0, 0);
        if (rc) return rc;
        if (gen != ctx->generation) drop_graph(ctx);
    }
    ResponseArgs ra{};
    ra.n_verts = regions->n_verts;
    ra.list = ctx->slow_list;
    ra.c = ctx->counters_d;
    ra.offsets = regions->offsets;
    ra.hs = regions->hs;
    ra.inv_mass = inv_mass_dev;
    ra.y_in = y_in_dev;
    ra.y_out = y_out_dev;
    ra.dt = dt;
    ra.prm.table = nullptr;
    ra.prm.vmesh = nullptr;
    ra.prm.one = mesh_params(params, 0.f, 0, 1.0f);
    launch_response(ra, (hipStream_t)stream);
    HIP_OK(hipGetLastError());
    return CCFR_OK;
}

int ccfr_xpbd_step(ccfr_ctx* ctx, const ccfr_mesh* mesh, float* x_dev, float* v_dev, const ccfr_step_params* sp,
                   ccfr_stream stream) {
    if (!ctx || !mesh || !step_params_ok(sp)) return CCFR_ERR_INVALID_ARG;
    if ((!x_dev || !v_dev) && mesh->n_verts > 0) return CCFR_ERR_INVALID_ARG;
    if (mesh->ctx != ctx) return CCFR_ERR_INVALID_ARG;
    if (mesh->n_verts == 0) return CCFR_OK;     // nothing moves
    const hipStream_t s = (hipStream_t)stream;
    const long long gen0 = ctx->generation;
    int rc = ensure_step(ctx, mesh->n_verts);
    if (rc) return rc;
    rc = ensure_sizes(ctx, mesh->n_verts, mesh->n_tris, mesh->n_edges, mesh->n_free, 1);
    if (rc) return rc;
    if (ctx->generation != gen0) drop_graph(ctx);
    rc = ensure_prof_events(ctx, sp->iters);
    if (rc) return rc;
    const StepPlan plan = mesh_plan(ctx, mesh, x_dev, v_dev, sp);
    if (ctx->profiling) {
        ctx->prof_last_iters = sp->iters;
        ctx->prof_last_reuse = ctx->pair_skin > 0 ? 1 : ctx->pair_reuse;
    }
    // profiled steps run eagerly: the stage events bracket the launches on `s`
    // the hierarchy's radix sort clears its scratch with memset operations,
    // which are not recorded into graphs here: those steps run directly
    if (!ctx->use_graphs || ctx->profiling || ctx->broad_phase == 1) {
        enqueue_step(ctx, plan, s);
        HIP_OK(hipGetLastError());
        return CCFR_OK;
    }
    const StepGraph& G = ctx->graph;
    const bool same = G.valid && G.owner == mesh && G.x == x_dev && G.v == v_dev &&
                      std::memcmp(&G.sp, sp, sizeof(*sp)) == 0 && G.generation == ctx->generation;
    return launch_recorded(ctx, ctx->graph, plan, mesh, sp, same, s);
}

int ccfr_xpbd_step_traced(ccfr_ctx* ctx, const ccfr_mesh* mesh, float* x_dev, float* v_dev,
                          const ccfr_step_params* sp, float* trace_dev, ccfr_stream stream) {
    if (!ctx || !mesh || !step_params_ok(sp)) return CCFR_ERR_INVALID_ARG;
    if ((!x_dev || !v_dev || !trace_dev) && mesh->n_verts > 0 && sp->iters > 0) return CCFR_ERR_INVALID_ARG;
    if (mesh->ctx != ctx) return CCFR_ERR_INVALID_ARG;
    if (mesh->n_verts == 0) return CCFR_OK;
    const hipStream_t s = (hipStream_t)stream;
    const long long gen0 = ctx->generation;
    int rc = ensure_step(ctx, mesh->n_verts);
    if (rc) return rc;
    rc = ensure_sizes(ctx, mesh->n_verts, mesh->n_tris, mesh->n_edges, mesh->n_free, 1);
    if (rc) return rc;
    if (ctx->generation != gen0) drop_graph(ctx);
    rc = ensure_prof_events(ctx, sp->iters);
    if (rc) return rc;
    StepPlan plan = mesh_plan(ctx, mesh, x_dev, v_dev, sp);
    plan.trace = trace_dev;
    enqueue_step(ctx, plan, s);      // launched directly, never recorded
    HIP_OK(hipGetLastError());
    return CCFR_OK;
}

int ccfr_sync_status(ccfr_ctx* ctx, ccfr_stream stream, ccfr_status_info* info, int reset) {
    if (!ctx) return CCFR_ERR_INVALID_ARG;
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    DevCounters h{};
    HIP_OK(hipMemcpy(&h, ctx->counters_d, sizeof(h), hipMemcpyDeviceToHost));
    if (info) {
        info->status_bits = h.status;
        for (int k = 0; k < 3; ++k) info->last_counts[k] = h.last_pairs[k];
        info->last_ve = h.last_pairs[3];
        info->last_contacts = h.last_nc;
        info->last_halfspaces = h.last_hs;
        for (int k = 0; k < 6; ++k) info->need[k] = h.need[k];
        for (int k = 0; k < 10; ++k) info->totals[k] = h.totals[k];
        info->candidate_builds = h.builds;
        info->iterations_run = h.iters_run;
        info->halt_runs[0] = h.halt_runs[0];
        info->halt_runs[1] = h.halt_runs[1];
        info->max_halt_run = h.max_halt_run;
        info->need_ve = h.need[6];
        info->total_ve = h.totals[10];
        const int slot_of[3] = {4, 5, 7};
        for (int w = 0; w < 3; ++w)
            for (int k = 0; k < 64; ++k) info->totals[slot_of[w]] += h.spread[w][k];
    }
    // an overflowed contact list leaves per-vertex counts behind: clear them
    if ((h.status & ST_CONTACTS) && ctx->vcount)
        HIP_OK(hipMemset(ctx->vcount, 0, sizeof(int32_t) * (size_t)ctx->cap_verts));
    if (reset) {
        DevCounters z{};
        HIP_OK(hipMemcpy(ctx->counters_d, &z, sizeof(z), hipMemcpyHostToDevice));
    }
    if (h.status & ST_NONFINITE) return CCFR_ERR_NONFINITE;
    if (h.status & (ST_VF | ST_EE | ST_VV | ST_VE | ST_HS | ST_LARGE | ST_CONTACTS)) return CCFR_ERR_CAPACITY;
    return CCFR_OK;
}

int ccfr_set_tuning(ccfr_ctx* ctx, const ccfr_tuning* t) {
    if (!ctx || !t || !std::isfinite(t->cell_scale) || t->cell_scale < 0.25f || t->cell_scale > 4.0f ||
        (t->pair_split != 1 && t->pair_split != 3 && t->pair_split != 9) || t->pair_reuse < 0 || t->pair_reuse > 4 ||
        t->pair_skin < 0 || t->pair_skin > 4 || (t->broad_phase != 0 && t->broad_phase != 1) ||
        (t->direct_regions != 0 && t->direct_regions != 1))
        return CCFR_ERR_INVALID_ARG;
    const int reuse = std::max(1, (int)t->pair_reuse);
    if (t->cell_scale != ctx->cell_scale || t->pair_split != ctx->pair_split || reuse != ctx->pair_reuse ||
        t->pair_skin != ctx->pair_skin || t->broad_phase != ctx->broad_phase ||
        t->direct_regions != ctx->direct_regions) {
        ctx->cell_scale = t->cell_scale;
        ctx->pair_split = t->pair_split;
        ctx->pair_reuse = reuse;
        ctx->pair_skin = t->pair_skin;
        ctx->broad_phase = t->broad_phase;
        ctx->direct_regions = t->direct_regions;
        ctx->tune_generation++;
        ctx->generation++;          // recorded graphs carry the old settings
        drop_graph(ctx);
    }
    return CCFR_OK;
}

int ccfr_get_tuning(const ccfr_ctx* ctx, ccfr_tuning* t) {
    if (!ctx || !t) return CCFR_ERR_INVALID_ARG;
    *t = ccfr_tuning{};
    t->cell_scale = ctx->cell_scale;
    t->pair_split = ctx->pair_split;
    t->pair_reuse = ctx->pair_reuse;
    t->pair_skin = ctx->pair_skin;
    t->broad_phase = ctx->broad_phase;
    t->direct_regions = ctx->direct_regions;
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
        // stages 0 and 1 run once per candidate build
        const int reuse = st < 2 ? std::max(1, ctx->prof_last_reuse) : 1;
        if (launches) launches[st] = (std::min(iters, ctx->prof_iters) + reuse - 1) / reuse;
    }
    return CCFR_OK;
}

}  // extern "C"
