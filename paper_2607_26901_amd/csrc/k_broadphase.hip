// k_broadphase.hip -- candidate primitive pairs (Sec. 4.1 broad phase) on gfx950.
//
// Contract (exact in FP32): pad = fl32(r + xi/2 + delta/2 + guard); a primitive's
// box is lo = fl32(min_v x_v - pad), hi = fl32(max_v x_v + pad) per axis; two
// primitives are a candidate pair iff their boxes overlap on all three axes.
// Pair kinds: vertex-face (vertex not in the triangle), edge-edge (no shared
// vertex, e < e'), free particle pairs (i < j), free particle and edge; pairs
// whose vertices all have zero inverse mass are skipped, and primitives of
// different meshes never pair.
// The grid below only decides which pairs are tested; the set is decided by the
// box test alone.
//
// Multi-level hash grid.  Level l has cells of size h 2^l (h per mesh).  Every
// target (triangle, edge, free particle) is binned once, at the finest level
// where its box spans at most two cells per axis, in the cell of its box's lower
// corner.  A query whose box spans at most two cells at level l finds every
// overlapping target of that level in the 3 x 3 x 3 cells [c(lo) - 1, c(hi)];
// it scans the levels, at or above its own, that its mesh occupies (a bitmask
// kept per mesh).  Pairs of two edges binned at different levels are found only
// by the finer one; pairs at the same level by the lower index.  Uneven sizes
// (a 4 m ground quad under 8 mm cloth triangles, large obstacles under fine
// hair) therefore cost a few extra buckets, not a brute-force list.
//
// The coarser levels of triangles and of edges have bucket tables of their own
// (few entries live there; sharing the level-0 tables would fill their buckets
// with level-0 entries that every coarse lookup reads and rejects).
//
// Vertices are binned too, in a table of their own, only to order the queries: the
// pair kernel takes vertex and edge queries in bucket order, in which the 64
// buckets of a 4 x 4 x 4 block of cells are consecutive, so the lanes of a
// wavefront (and the workgroups of one XCD, see xcd_block) read the same
// neighbouring buckets and the entries come from L1 / L2 instead of HBM.
//
// Pipeline per build:
//   reset        counters and the per-mesh level masks
//   grid_count   one thread per target and per vertex: box, level, bucket, rank
//                inside the bucket (atomic)
//   scan         exclusive prefix of the per-(kind, bucket) counts
//   grid_scatter the entries (48 B each: box, index, flags, vertices; written
//                in primitive order by grid_count) moved to their sorted slots
//   pairs        one thread per query (vertex entries, then edge entries, in
//                sorted order); each lane keeps the pairs it finds in its own
//                LDS slice (a register counts them), a wavefront writes its
//                slices out when one is nearly full, and what is left at the
//                end goes out with one atomic per block and list
#include "ccfr_internal.h"
#include "pair_emit.h"

#include <algorithm>

namespace ccfr {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxLevel = 24;
constexpr int KIND_VX = 4;     // vertex entries (query order only)

// Workgroup b runs on XCD b % 8; give each XCD a contiguous run of logical
// blocks so that spatially adjacent queries share one L2.
__device__ __forceinline__ int xcd_block(int b, int n) {
    const int per = n >> 3, rem = n & 7;
    const int x = b & 7, k = b >> 3;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + k;
}

__device__ __forceinline__ void load3(const float* x, int v, float o[3]) {
    o[0] = x[3 * v + 0];
    o[1] = x[3 * v + 1];
    o[2] = x[3 * v + 2];
}

__device__ __forceinline__ bool finite3(const float o[3]) {
    return isfinite(o[0]) && isfinite(o[1]) && isfinite(o[2]);
}

// Box overlap, evaluated without branches (every comparison, then one and).
__device__ __forceinline__ bool overlap(const float alo[3], const float ahi[3], const float blo[3],
                                        const float bhi[3]) {
    return (alo[0] <= bhi[0]) & (blo[0] <= ahi[0]) & (alo[1] <= bhi[1]) & (blo[1] <= ahi[1]) &
           (alo[2] <= bhi[2]) & (blo[2] <= ahi[2]);
}

// The primitive behind grid slot t: triangles, edges, free particles, then vertices.
struct Target {
    int kind;      // KIND_VF (triangle), KIND_EE (edge), KIND_VV (particle), KIND_VX (vertex)
    int idx;
    int nv;
    int v[3];
};

__device__ __forceinline__ Target target_of(const Scene& sc, int t) {
    Target g;
    if (t < sc.n_tris) {
        g.kind = KIND_VF; g.idx = t; g.nv = 3;
        g.v[0] = sc.tris[3 * t]; g.v[1] = sc.tris[3 * t + 1]; g.v[2] = sc.tris[3 * t + 2];
    } else if (t < sc.n_tris + sc.n_edges) {
        const int e = t - sc.n_tris;
        g.kind = KIND_EE; g.idx = e; g.nv = 2;
        g.v[0] = sc.edges[2 * e]; g.v[1] = sc.edges[2 * e + 1]; g.v[2] = g.v[1];
    } else if (t < sc.n_tris + sc.n_edges + sc.n_free) {
        const int p = sc.free_list[t - sc.n_tris - sc.n_edges];
        g.kind = KIND_VV; g.idx = p; g.nv = 1;
        g.v[0] = g.v[1] = g.v[2] = p;
    } else {
        const int p = t - sc.n_tris - sc.n_edges - sc.n_free;
        g.kind = KIND_VX; g.idx = p; g.nv = 1;
        g.v[0] = g.v[1] = g.v[2] = p;
    }
    return g;
}

// How far a box must reach beyond `pad` so that a list built now holds every
// pair whose pad-boxes overlap within the next `k` iterations.  A vertex moves
// by the projected displacement, |y| <= r (per coordinate, after its rounding
// to FP32, r (1 + 2^-23)), plus the rounding of x + y (at most 2^-24 |x + y|);
// the bound below takes each term with ample slack.  The FP32 sum pad + reach
// is rounded up by one step so that it is never below the exact sum.
__device__ __forceinline__ float skin_pad(float pad, float r, int k, float maxabs) {
    const float kf = (float)k;
    const float reach = kf * (r * (1.0f + 0x1p-18f) + (maxabs + (kf + 1.0f) * 2.0f * r) * 0x1p-21f);
    return __int_as_float(__float_as_int(pad + reach) + 1);    // positive and finite: one step up
}

// Box of a target and its static flag; false if a coordinate is not finite.
// The box of a target with a moving vertex is widened: by skin_pad when
// sc.skin_iters > 0, to pad_wide when sc.skin_wide is set.
__device__ __forceinline__ bool target_box(const Scene& sc, const Target& g, const MeshParams& P, float lo[3],
                                           float hi[3], bool* is_static) {
    float pad = P.pad;
    float p[3];
    load3(sc.x, g.v[0], p);
    bool fin = finite3(p);
    float mn[3] = {p[0], p[1], p[2]}, mx[3] = {p[0], p[1], p[2]};
    bool st = sc.inv_mass[g.v[0]] == 0.0f;
    for (int i = 1; i < g.nv; ++i) {
        load3(sc.x, g.v[i], p);
        fin = fin && finite3(p);
        st = st && (sc.inv_mass[g.v[i]] == 0.0f);
        for (int k = 0; k < 3; ++k) {
            mn[k] = fminf(mn[k], p[k]);
            mx[k] = fmaxf(mx[k], p[k]);
        }
    }
    if (sc.skin_iters > 0 && !st) {
        float m = 0.0f;
        for (int k = 0; k < 3; ++k) m = fmaxf(m, fmaxf(fabsf(mn[k]), fabsf(mx[k])));
        pad = skin_pad(pad, P.r, sc.skin_iters, m);
    } else if (sc.skin_wide && !st) {
        pad = P.pad_wide;
    }
    for (int k = 0; k < 3; ++k) {
        lo[k] = __fsub_rn(mn[k], pad);
        hi[k] = __fadd_rn(mx[k], pad);
    }
    *is_static = st;
    return fin;
}

// Finest level at which the box spans at most two cells per axis (-1: none).
__device__ __forceinline__ int box_level(const float lo[3], const float hi[3], float inv_h, int clo[3]) {
    for (int l = 0; l <= kMaxLevel; ++l) {
        const float inv = ldexpf(inv_h, -l);
        bool fits = true;
        for (int k = 0; k < 3; ++k) {
            clo[k] = cell_coord(lo[k], inv);
            fits = fits && (cell_coord(hi[k], inv) - clo[k] <= 1);
        }
        if (fits) return l;
    }
    return -1;
}

// Order of cell c against the query's own cell o (the cell its entry is binned
// in): -1, 0, +1, lexicographic in (z, y, x).  Two entries of one level whose
// boxes overlap each lie in the other's query stencil, so the pair is taken
// only by the query whose own cell comes first, or, in one cell, by the lower
// index: every such pair is tested once instead of twice.
__device__ __forceinline__ int cell_order(int cx, int cy, int cz, const int o[3]) {
    if (cz != o[2]) return cz < o[2] ? -1 : 1;
    if (cy != o[1]) return cy < o[1] ? -1 : 1;
    if (cx != o[0]) return cx < o[0] ? -1 : 1;
    return 0;
}

__device__ __forceinline__ int level_salt(int mesh_salt, int level) {
    return mesh_salt ^ (int)((uint32_t)(level + 1) * 0x9E3779B9u);
}

__device__ __forceinline__ uint32_t make_flags(bool st, int level, int mesh) {
    return (st ? 1u : 0u) | ((uint32_t)level << 1) | ((uint32_t)mesh << 8);
}

__device__ __forceinline__ bool entry_ok(const GridEntry& e, int mesh, int level, bool q_static) {
    // same mesh, binned at the level being scanned, not a static-static pair
    return ((e.flags >> 8) == (uint32_t)mesh) & (((e.flags >> 1) & 31u) == (uint32_t)level) &
           !(q_static & ((e.flags & 1u) != 0u));
}

// Sets bit `level` of the mesh's level mask.  The lanes of a wavefront that share
// a mesh OR their bits together first, and a bit already visible costs no atomic.
__device__ __forceinline__ void mark_level(uint32_t* level_mask, int mesh, uint32_t bits) {
    const unsigned long long active = __ballot(true);
    const int lead = __ffsll((long long)active) - 1;
    const int m0 = __shfl(mesh, lead);
    const bool uniform = __ballot(mesh != m0) == 0ull;
    if (uniform) {
        const int lane = __lane_id();
        for (int off = 1; off < warpSize; off <<= 1) {
            const uint32_t o = __shfl_xor(bits, off);
            if ((active >> (lane ^ off)) & 1ull) bits |= o;     // only lanes still running
        }
        if (lane == lead && bits && (level_mask[mesh] & bits) != bits) atomicOr(&level_mask[mesh], bits);
    } else if (bits && (level_mask[mesh] & bits) != bits) {
        atomicOr(&level_mask[mesh], bits);
    }
}

__global__ void k_reset_build(DevCounters* c, uint32_t* level_mask, int n_meshes) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        reset_build_counters(c);
        c->rebuild = 1u;            // the first build of a substep or a standalone build
        c->motion_acc = 0.0;
        c->converged = 0u;          // a substep's iterations run until its convergence check ends them
    }
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < n_meshes; m += gridDim.x * blockDim.x)
        level_mask[m] = 0u;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < 64; k += gridDim.x * blockDim.x) {
        c->maxima[k][kMaxMotion] = 0u;
        c->maxima[k][kMaxShortfall] = 0u;
    }
}

// Level and lower-corner cell of an entry (vertex entries: level 0, their box
// is narrower than a cell); -1 if it is not binned.
__device__ __forceinline__ int entry_level(const Target& tg, const float lo[3], const float hi[3], float inv_h,
                                           int clo[3]) {
    if (tg.kind == KIND_VX) {
        for (int k = 0; k < 3; ++k) clo[k] = cell_coord(lo[k], inv_h);
        return 0;
    }
    return box_level(lo, hi, inv_h, clo);
}

__global__ __launch_bounds__(kBlock) void k_grid_count(Scene sc, GridWs g, DevCounters* c) {
    if (sc.skip && *sc.skip) return;             // the substep's iterations have ended
    if (sc.build_gated && !c->rebuild) return;   // the lists of an earlier build still hold
    const int n_all = sc.n_tris + sc.n_edges + sc.n_free + sc.n_verts;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_all) return;
    const Target tg = target_of(sc, t);
    const int mesh = sc.prm.mesh_of(tg.v[0]);
    const MeshParams P = sc.prm.get(mesh);
    float lo[3], hi[3];
    bool st;
    int clo[3];
    int level = -2;
    if (!target_box(sc, tg, P, lo, hi, &st)) {
        atomicOr(&c->status, ST_NONFINITE);
    } else {
        level = entry_level(tg, lo, hi, P.inv_h, clo);
        // a box wider than h 2^24 is not binned; nor is a particle box wider
        // than a cell (particle pairs are looked up on the finest level only),
        // which takes coordinates so large that their FP32 spacing nears the pad
        if (tg.kind == KIND_VV && level > 0) level = -1;
        if (level < 0) atomicOr(&c->status, ST_LARGE);
    }
    // every lane still in the kernel takes part in the wave-wide OR
    mark_level(g.level_mask, mesh, (level < 0 || tg.kind == KIND_VX) ? 0u : (1u << level));
    if (level < 0) {
        g.key[t] = -1;
        return;
    }
    const int key = g.bucket(table_of(tg.kind - 1, level), clo[0], clo[1], clo[2], level_salt(P.mesh_salt, level));
    g.key[t] = key;
    g.rank[t] = atomicAdd(&g.cnt[key], 1);
    // the entry itself, in primitive order; the scatter only moves it
    GridEntry e;
    for (int k = 0; k < 3; ++k) {
        e.lo[k] = lo[k];
        e.hi[k] = hi[k];
        e.v[k] = tg.v[k];
    }
    e.idx = tg.idx;
    e.flags = make_flags(st, level, mesh);
    e.pad = 0;
    g.staged[t] = e;
}

__global__ __launch_bounds__(kBlock) void k_grid_scatter(Scene sc, GridWs g, const DevCounters* c) {
    if (sc.skip && *sc.skip) return;
    if (sc.build_gated && !c->rebuild) return;
    const int n_all = sc.n_tris + sc.n_edges + sc.n_free + sc.n_verts;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_all) return;
    const int key = g.key[t];
    if (key < 0) return;
    g.entries[g.start[key] + g.rank[t]] = g.staged[t];
}

// Found pairs are staged in per-lane LDS slices (pair_emit.h).
static_assert(kBlock == kEmitBlock, "the pair kernel stages pairs in blocks of kEmitBlock lanes");
constexpr int kRound = 4;      // entries read per round of a bucket walk

// Called by the active lanes before a round that may append up to kRound pairs each.
__device__ __forceinline__ void lane_room(LaneBuf& lb, const PairLists& pl, DevCounters* c) {
    lane_room_for(lb, pl, c, kRound);
}

// Cells of the stencil [clo - 1, chi] that work item `part` of `split` walks:
// all (split 1), one z layer (split 3) or one (z, y) row (split 9).
__device__ __forceinline__ bool part_range(int split, int part, const int clo[3], const int chi[3], int r0[3],
                                           int r1[3]) {
    for (int k = 0; k < 3; ++k) {
        r0[k] = clo[k] - 1;
        r1[k] = chi[k];
    }
    if (split >= 3) {
        r0[2] += split == 3 ? part : part / 3;
        if (r0[2] > r1[2]) return false;
        r1[2] = r0[2];
    }
    if (split == 9) {
        r0[1] += part % 3;
        if (r0[1] > r1[1]) return false;
        r1[1] = r0[1];
    }
    return true;
}

// Bucket range in table `table` of cell k (0..8, row-major in y then x) of one
// z layer of a stencil [r0, r1]; ord is the cell's order against the query's own cell when
// the half shell applies (`half`), else 1; an empty range is returned for a
// cell outside the stencil or before the own cell.
__device__ __forceinline__ void cell_range(const GridWs& g, int table, int salt, int k, int cz, const int r0[3],
                                           const int r1[3], const int own[3], bool half, int& s0, int& s1,
                                           int& ord) {
    const int cx = r0[0] + k % 3, cy = r0[1] + k / 3;
    s0 = s1 = 0;
    ord = -1;
    if (cx > r1[0] || cy > r1[1]) return;
    ord = half ? cell_order(cx, cy, cz, own) : 1;
    if (ord < 0) return;
    const int b = g.bucket(table, cx, cy, cz, salt);
    s0 = g.start[b];
    s1 = g.start[b + 1];
}

// Bucket ranges in table `table` of the nine cells of z layer cz of a stencil
// [r0, r1] (row-major in y then x), all looked up at once so that their loads
// are in flight together; a cell outside the stencil, or before the query's
// own cell when the half shell applies (`half`), gets an empty range.  Returns
// the position of the own cell in the layer, or -1.
struct Layer {
    int s0[9], s1[9];
    // moves cell k + 1 to position k (constant indices: the ranges stay in registers)
    __device__ __forceinline__ void shift() {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            s0[k] = s0[k + 1];
            s1[k] = s1[k + 1];
        }
    }
};

__device__ __forceinline__ int layer_ranges(const GridWs& g, int table, int salt, int cz, const int r0[3],
                                            const int r1[3], const int own[3], bool half, Layer& L) {
    const uint32_t hz = hash_z(cz, salt);
    int k_own = -1;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
        const int cy = r0[1] + ky;
        const uint32_t hy = hash_y(cy, hz);
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            const int cx = r0[0] + kx;
            const int k = 3 * ky + kx;
            bool in = (cx <= r1[0]) & (cy <= r1[1]);
            if (half) {
                const int o = cell_order(cx, cy, cz, own);
                in = in & (o >= 0);
                if (in & (o == 0)) k_own = k;
            }
            L.s0[k] = L.s1[k] = 0;
            if (in) {
                const int b = g.bucket_hy(table, cx, cy, cz, hy);
                L.s0[k] = g.start[b];
                L.s1[k] = g.start[b + 1];
            }
        }
    }
    return k_own;
}

// ---- entry tests of one cell's bucket ----

struct GlobalSrc {
    const GridEntry* e;
    __device__ __forceinline__ GridEntry get(int i) const { return e[i]; }
};

// Vertex query v against the triangle entries [i0, i1) of one cell.
template <class Src>
__device__ __forceinline__ void scan_vf(Src src, int i0, int i1, const GridEntry& me, int v, int mesh, int l,
                                        bool q_static, LaneBuf& lb, const PairLists& pl, DevCounters* c) {
    for (int i = i0; i < i1; i += kRound) {
        lane_room(lb, pl, c);
        GridEntry e[kRound];
#pragma unroll
        for (int u = 0; u < kRound; ++u) e[u] = src.get(min(i + u, i1 - 1));
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
            const bool hit = (i + u < i1) & entry_ok(e[u], mesh, l, q_static) & overlap(me.lo, me.hi, e[u].lo, e[u].hi) &
                             (e[u].v[0] != v) & (e[u].v[1] != v) & (e[u].v[2] != v);
            lane_put(lb, e[u].idx, hit);
        }
    }
}

// Free particle v against the particle entries [i0, i1) of one cell (level 0,
// half shell with the cell's order `ord`).
template <class Src>
__device__ __forceinline__ void scan_vv(Src src, int i0, int i1, int ord, const GridEntry& me, int v, int mesh,
                                        bool q_static, LaneBuf& lb, const PairLists& pl, DevCounters* c) {
    for (int i = i0; i < i1; i += kRound) {
        lane_room(lb, pl, c);
        GridEntry e[kRound];
#pragma unroll
        for (int u = 0; u < kRound; ++u) e[u] = src.get(min(i + u, i1 - 1));
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
            const bool hit = (i + u < i1) & ((ord > 0) | (e[u].idx > v)) & entry_ok(e[u], mesh, 0, q_static) &
                             overlap(me.lo, me.hi, e[u].lo, e[u].hi);
            lane_put_vv(lb, e[u].idx, hit);
        }
    }
}

// Free particle v against the edge entries [i0, i1) of one cell of level l (a
// free particle is in no edge, so no shared vertex is possible).
template <class Src>
__device__ __forceinline__ void scan_ve(Src src, int i0, int i1, const GridEntry& me, int mesh, int l, bool q_static,
                                        LaneBuf& lb, const PairLists& pl, DevCounters* c) {
    for (int i = i0; i < i1; i += kRound) {
        lane_room(lb, pl, c);
        GridEntry e[kRound];
#pragma unroll
        for (int u = 0; u < kRound; ++u) e[u] = src.get(min(i + u, i1 - 1));
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
            const bool hit = (i + u < i1) & entry_ok(e[u], mesh, l, q_static) & overlap(me.lo, me.hi, e[u].lo, e[u].hi);
            lane_put_ve(lb, e[u].idx, hit);
        }
    }
}

// Edge query eq = (a, bb) of level lq against the edge entries [i0, i1) of one
// cell of level l (half shell with the cell's order `ord` when l == lq).
template <class Src>
__device__ __forceinline__ void scan_ee(Src src, int i0, int i1, int ord, const GridEntry& me, int eq, int a, int bb,
                                        int mesh, int l, bool q_static, LaneBuf& lb, const PairLists& pl,
                                        DevCounters* c) {
    for (int i = i0; i < i1; i += kRound) {
        lane_room(lb, pl, c);
        GridEntry e[kRound];
#pragma unroll
        for (int u = 0; u < kRound; ++u) e[u] = src.get(min(i + u, i1 - 1));
#pragma unroll
        for (int u = 0; u < kRound; ++u) {
            const bool hit = (i + u < i1) & ((ord > 0) | (e[u].idx > eq)) & entry_ok(e[u], mesh, l, q_static) &
                             overlap(me.lo, me.hi, e[u].lo, e[u].hi) & (e[u].v[0] != a) & (e[u].v[0] != bb) &
                             (e[u].v[1] != a) & (e[u].v[1] != bb);
            lane_put(lb, e[u].idx, hit);
        }
    }
}

// ---- per-lane walks of one level's stencil through global memory ----

__device__ __forceinline__ void stencil_cells(const GridEntry& me, float inv, int clo[3], int chi[3]) {
    for (int k = 0; k < 3; ++k) {
        clo[k] = cell_coord(me.lo[k], inv);
        chi[k] = cell_coord(me.hi[k], inv);
    }
}

__device__ void walk_vf_global(const GridWs& g, const GridEntry& me, int v, int mesh, int l, int salt, bool q_static,
                               const int clo[3], const int r0[3], const int r1[3], LaneBuf& lb,
                               const PairLists& pl, DevCounters* c) {
    const GlobalSrc src{g.entries};
    const int tb = table_of(0, l);
    for (int cz = r0[2]; cz <= r1[2]; ++cz) {
        Layer L;
        layer_ranges(g, tb, salt, cz, r0, r1, clo, false, L);
#pragma unroll 1
        for (int k = 0; k < 9; ++k) {
            const int s0 = L.s0[0], s1 = L.s1[0];
            L.shift();
            scan_vf(src, s0, s1, me, v, mesh, l, q_static, lb, pl, c);
        }
    }
}

__device__ void walk_ve_global(const GridWs& g, const GridEntry& me, int mesh, int l, int salt, bool q_static,
                               const int clo[3], const int r0[3], const int r1[3], LaneBuf& lb,
                               const PairLists& pl, DevCounters* c) {
    const GlobalSrc src{g.entries};
    const int tb = table_of(1, l);
    for (int cz = r0[2]; cz <= r1[2]; ++cz) {
        Layer L;
        layer_ranges(g, tb, salt, cz, r0, r1, clo, false, L);
#pragma unroll 1
        for (int k = 0; k < 9; ++k) {
            const int s0 = L.s0[0], s1 = L.s1[0];
            L.shift();
            scan_ve(src, s0, s1, me, mesh, l, q_static, lb, pl, c);
        }
    }
}

__device__ void walk_vv_global(const GridWs& g, const GridEntry& me, int v, int mesh, int salt, bool q_static,
                               const int clo[3], const int r0[3], const int r1[3], LaneBuf& lb,
                               const PairLists& pl, DevCounters* c) {
    const GlobalSrc src{g.entries};
    for (int cz = r0[2]; cz <= r1[2]; ++cz)
        for (int k = 0; k < 9; ++k) {
            int u0, u1, ord;
            cell_range(g, TB_PART, salt, k, cz, r0, r1, clo, true, u0, u1, ord);
            scan_vv(src, u0, u1, ord, me, v, mesh, q_static, lb, pl, c);
        }
}

__device__ void walk_ee_global(const GridWs& g, const GridEntry& me, int eq, int a, int bb, int mesh, int lq, int l,
                               int salt, bool q_static, const int clo[3], const int r0[3], const int r1[3],
                               LaneBuf& lb, const PairLists& pl, DevCounters* c) {
    const GlobalSrc src{g.entries};
    const bool half = l == lq;
    const int tb = table_of(1, l);
    for (int cz = r0[2]; cz <= r1[2]; ++cz) {
        Layer L;
        const int k_own = layer_ranges(g, tb, salt, cz, r0, r1, clo, half, L);
#pragma unroll 1
        for (int k = 0; k < 9; ++k) {
            const int s0 = L.s0[0], s1 = L.s1[0];
            L.shift();
            scan_ee(src, s0, s1, k == k_own ? 0 : 1, me, eq, a, bb, mesh, l, q_static, lb, pl, c);
        }
    }
}

// Work item = (query, part of its stencil) with `split` lanes per query; every
// lane walks its stencil through global memory.  A wavefront takes 64
// consecutive items of one kind: vertex items (vertex-face and particle pairs)
// or edge items.  The vertex wavefronts are spread evenly among the edge
// wavefronts over the whole grid (Bresenham), so that every XCD, and every SIMD,
// gets both kinds in proportion instead of some taking all the heavier vertex
// queries.
__global__ __launch_bounds__(kBlock) void k_pairs(Scene sc, GridWs g, PairLists pl, DevCounters* c, int split,
                                                  long long vwaves, long long waves) {
    if (sc.skip && *sc.skip) return;
    if (sc.build_gated && !c->rebuild) return;
    __shared__ int32_t lane_pairs[kLaneCap][kEmitBlock];
    LaneBuf lb{(LDS_PTR int32_t*)&lane_pairs[0][threadIdx.x], 0, 0, 0, true, 0};
    const long long w = (long long)xcd_block(blockIdx.x, gridDim.x) * kEmitWaves + threadIdx.x / 64;
    const long long vw = w * vwaves / waves;                 // vertex wavefronts before w
    const bool vwave = (w + 1) * vwaves / waves > vw;
    const long long item = (vwave ? vw : w - vw) * 64 + __lane_id();
    const int q = (int)(item / split);
    const int part = (int)(item - (long long)q * split);
    const int v0 = g.start[g.off[TB_VERT]], nv_q = g.start[g.off[TB_VERT + 1]] - v0;     // binned vertices
    const int e0 = g.start[g.off[TB_EDGE0]], ne_q = g.start[g.off[TB_EDGEC + 1]] - e0;   // binned edges
    if (w >= waves) {
        // past the last wavefront: no query
    } else if (vwave && q < nv_q) {
        // ---- vertex query: vertex-face pairs, and for a free particle its
        //      particle pairs and particle-edge pairs
        const GridEntry me = g.entries[v0 + q];
        const int v = me.idx;
        lb.self = v;
        const int mesh = (int)(me.flags >> 8);
        const MeshParams P = sc.prm.get(mesh);
        const bool q_static = (me.flags & 1u) != 0u;
        const bool q_free = (sc.vflags[v] & VF_FREE) != 0;
        uint32_t levels = g.level_mask[mesh];
        while (levels) {
            const int l = __ffs((int)levels) - 1;
            levels &= levels - 1u;
            const int salt = level_salt(P.mesh_salt, l);
            int clo[3], chi[3], r0[3], r1[3];
            stencil_cells(me, ldexpf(P.inv_h, -l), clo, chi);
            if (!part_range(split, part, clo, chi, r0, r1)) continue;
            walk_vf_global(g, me, v, mesh, l, salt, q_static, clo, r0, r1, lb, pl, c);
            if (q_free) {
                walk_ve_global(g, me, mesh, l, salt, q_static, clo, r0, r1, lb, pl, c);
                if (l == 0) walk_vv_global(g, me, v, mesh, salt, q_static, clo, r0, r1, lb, pl, c);
            }
        }
    } else if (!vwave && q < ne_q) {
        // ---- edge query: edge-edge pairs
        lb.vert = false;
        const GridEntry me = g.entries[e0 + q];
        const int eq = me.idx;
        lb.self = eq;
        const int a = me.v[0], bb = me.v[1];
        const int mesh = (int)(me.flags >> 8);
        const int lq = (int)((me.flags >> 1) & 31u);
        const MeshParams P = sc.prm.get(mesh);
        const bool q_static = (me.flags & 1u) != 0u;
        uint32_t levels = g.level_mask[mesh] & ~((1u << lq) - 1u);
        while (levels) {
            const int l = __ffs((int)levels) - 1;
            levels &= levels - 1u;
            const int salt = level_salt(P.mesh_salt, l);
            int clo[3], chi[3], r0[3], r1[3];
            stencil_cells(me, ldexpf(P.inv_h, -l), clo, chi);
            if (!part_range(split, part, clo, chi, r0, r1)) continue;
            walk_ee_global(g, me, eq, a, bb, mesh, lq, l, salt, q_static, clo, r0, r1, lb, pl, c);
        }
    }
    block_flush(lb, pl, c);
}

__global__ void k_finalize_pairs(PairLists pl, DevCounters* c) {
    if (threadIdx.x == 0) finalize_pairs_body(c, pl.caps());
}

}  // namespace

void launch_reset_build(DevCounters* c, uint32_t* level_mask, int n_meshes, hipStream_t s) {
    const int blocks = std::max(1, std::min(64, (n_meshes + 255) / 256));
    hipLaunchKernelGGL(k_reset_build, dim3(blocks), dim3(256), 0, s, c, level_mask, n_meshes);
}

void launch_grid_count(const Scene& sc, GridWs& g, DevCounters* c, hipStream_t s) {
    const int n = sc.n_tris + sc.n_edges + sc.n_free + sc.n_verts;
    if (n == 0) return;
    hipLaunchKernelGGL(k_grid_count, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, sc, g, c);
}

void launch_grid_scatter(const Scene& sc, GridWs& g, DevCounters* c, hipStream_t s) {
    const int n = sc.n_tris + sc.n_edges + sc.n_free + sc.n_verts;
    if (n == 0) return;
    hipLaunchKernelGGL(k_grid_scatter, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, sc, g, c);
}

void launch_pairs(const Scene& sc, const GridWs& g, PairLists pl, DevCounters* c, int split, hipStream_t s) {
    const long long n = (long long)sc.n_verts + sc.n_edges;
    if (n <= 0) return;
    if (split != 3 && split != 9) split = 1;
    while (split > 1 && n * split > (1LL << 31) - kBlock) split /= 3;
    // wavefronts of vertex items and of edge items (the binned counts are known
    // on the device only: the items cover every vertex and every edge)
    const long long vwaves = ((long long)sc.n_verts * split + 63) / 64;
    const long long waves = vwaves + ((long long)sc.n_edges * split + 63) / 64;
    hipLaunchKernelGGL(k_pairs, dim3((unsigned)((waves + kEmitWaves - 1) / kEmitWaves)), dim3(kBlock), 0, s, sc, g, pl, c,
                       split, vwaves, waves);
}

void launch_finalize_pairs(const GridWs& g, PairLists pl, DevCounters* c, hipStream_t s) {
    (void)g;
    hipLaunchKernelGGL(k_finalize_pairs, dim3(1), dim3(64), 0, s, pl, c);
}

}  // namespace ccfr
