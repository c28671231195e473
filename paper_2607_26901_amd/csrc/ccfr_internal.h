// ccfr_internal.h -- shared device-side definitions of the gfx950 CCFR library.
//
// Layout on the device (one "scene" = one or more concatenated meshes):
//   x        float [N][3]   anchor positions (packed, 12 B per vertex)
//   inv_mass float [N]
//   tris     int   [T][3],  edges int [E][2]
//   vmesh    u16   [N]      mesh id of every vertex (nullptr: all mesh 0)
//   MeshParams table [M]    per-mesh collision parameters and grid cell size
//
// Broad phase: a multi-level spatial hash grid.  Every target primitive
// (triangle, edge, free particle) is binned once, at the finest level where its
// box spans at most two cells, by the cell of its box's lower corner; a query
// scans the 3x3x3 cells (at most) its own box can reach on each occupied level.
// The bucket of a cell keeps the low two bits of each cell coordinate verbatim
// and hashes the rest, so the <= 27 cells a query scans on one level always land
// in distinct buckets and no target is seen twice by one query.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ccfr.h"

namespace ccfr {

// pair kinds (the top bits of a half-space key): particle-edge, vertex-face,
// edge-edge, particle-particle
enum : int { KIND_VE = 0, KIND_VF = 1, KIND_EE = 2, KIND_VV = 3 };

// Per-vertex flags: a free particle (in no edge and no triangle); an endpoint
// of an edge of the first stretch colour (the pass starts in the iteration's
// closing kernel, which then leaves such a vertex to its edge)
enum : uint8_t { VF_FREE = 1, VF_COLOR0 = 2 };

// status bits (sticky)
enum : uint32_t {
    ST_VF = 1u, ST_EE = 2u, ST_VV = 4u, ST_HS = 8u, ST_LARGE = 16u, ST_CONTACTS = 32u,
    ST_NONFINITE = 64u, ST_VE = 128u,
};

struct MeshParams {
    float r, xi, pad, two_r;
    float eps_retract, eps_plesnik, h, inv_h;   // h: grid cell size of this mesh
    int32_t max_passes, mesh_salt;
    float pad_wide;     // box pad of moving primitives in builds widened by a fixed skin
    int32_t response;   // 1: soft response and friction before the projection (Sec. 3.3)
    float delta, resp_compliance, vis_width, mu_s, mu_k;
    int32_t pad2[3];
};

// Device counters shared by all kernels of a context.
struct DevCounters {
    uint32_t status;
    int32_t n_vf, n_ee, n_vv, n_ve;    // pair counts of the current build (in this order: the
                                       // candidate lists' counts_dev points at n_vf)
    int32_t n_large_t, n_large_e;      // large primitives of the current build
    int32_t n_contacts;                // pairs inside the range
    int32_t n_viol;                    // deferred vertices with small regions (slow list front)
    int32_t last_hs;
    int32_t n_viol_b;                  // deferred vertices with larger regions (slow list back)
    int32_t last_nc;                   // contacts of the last closed region build
    int32_t last_pairs[4];             // VF, EE, VV, VE of the last closed candidate build
    // substeps whose candidate builds adapt to the motion: whether this
    // iteration builds (the last projection's largest coordinate move is in
    // maxima), and the moves summed since the last build
    uint32_t rebuild, pad1;
    double motion_acc;
    // region builds into per-vertex slots: half-spaces written, and the largest
    // number any vertex received (beyond its slots they are dropped)
    int32_t n_hs, max_slot;
    long long builds;                  // candidate builds closed
    // the convergence check of a substep (evaluateConvergence of Alg. 4, with
    // early exit): whether the substep's iterations have ended (the last
    // projection's largest shortfall is in maxima), and the iterations run
    uint32_t converged, pad2;
    long long iters_run;
    // consecutive halts of one vertex within a substep: the longest run seen,
    // and the halts that extended a run to 2 or to 3 and more
    int32_t max_halt_run, pad3;
    long long halt_runs[2];
    int32_t n_resp;                    // vertices whose response a wavefront takes (list)
    int32_t n_viol_m;                  // deferred vertices with mid-size regions (second half of the slow list)
    long long need[7];                 // max sizes seen: vf, ee, vv, contacts, hs, large, ve
    long long totals[11];              // vf, ee, vv, hs, violating, halted, degenerate, projected,
                                       // contacts, region builds, ve
    // per-vertex tallies of the projection (violating, halted, projected),
    // spread over 64 slots by block so that the atomics do not queue on one
    // address; the host adds them into totals[4], [5], [7]
    long long spread[3][64];
    // the last projection's largest coordinate move (word kMaxMotion) and
    // largest shortfall |p - x| - |y*| (word kMaxShortfall), FP32 bits rounded
    // up, spread over 64 slots a cache line apart by block: the wavefronts of
    // a launch would otherwise queue on one address.  The decision kernels
    // take the maxima and clear the slots.
    uint32_t maxima[64][32];
};

constexpr int kMaxMotion = 0, kMaxShortfall = 1;

// Capacities of the four candidate lists.
struct PairCaps {
    int64_t vf, ee, vv, ve;
};

// End of a candidate build (one thread): overflow bits, largest sizes, totals.
__device__ __forceinline__ void finalize_pairs_body(DevCounters* c, const PairCaps& caps) {
    const long long nvf = c->n_vf, nee = c->n_ee, nvv = c->n_vv, nve = c->n_ve;
    uint32_t st = 0;
    if (nvf > caps.vf) st |= ST_VF;
    if (nee > caps.ee) st |= ST_EE;
    if (nvv > caps.vv) st |= ST_VV;
    if (nve > caps.ve) st |= ST_VE;
    if (st) c->status |= st;
    c->need[0] = max(c->need[0], nvf);
    c->need[1] = max(c->need[1], nee);
    c->need[2] = max(c->need[2], nvv);
    c->need[6] = max(c->need[6], nve);
    c->totals[0] += nvf;
    c->totals[1] += nee;
    c->totals[2] += nvv;
    c->totals[10] += nve;
    c->last_pairs[0] = (int32_t)nvf;
    c->last_pairs[1] = (int32_t)nee;
    c->last_pairs[2] = (int32_t)nvv;
    c->last_pairs[3] = (int32_t)nve;
    c->builds += 1;
}

// End of a region build (one thread): overflow bits, largest sizes, totals.
__device__ __forceinline__ void finalize_regions_body(DevCounters* c, int32_t n_verts, const int32_t* offsets,
                                                      int64_t cap_contacts, int64_t cap_hs) {
    const long long H = offsets[n_verts];
    const long long nc = c->n_contacts;
    uint32_t st = 0;
    if (nc > cap_contacts) st |= ST_CONTACTS;
    if (H > cap_hs) st |= ST_HS;
    if (st) c->status |= st;
    c->need[3] = max(c->need[3], nc);
    c->need[4] = max(c->need[4], H);
    c->totals[3] += H;
    c->totals[8] += nc;
    c->totals[9] += 1;
    c->last_hs = (int32_t)H;
    c->last_nc = (int32_t)nc;
}

// Per-build counters back to zero (one thread); level masks are cleared apart.
__device__ __forceinline__ void reset_region_counters(DevCounters* c) {
    c->n_contacts = 0;
    c->n_viol = 0;
    c->n_viol_b = 0;
    c->n_viol_m = 0;
    c->n_hs = 0;
    c->max_slot = 0;
}

// End of a region build into per-vertex slots of `stride` entries (one thread):
// a vertex that received more half-spaces than its slots sets the overflow bit,
// and the need is reported as the half-space buffer that would hold them all.
// cap_contacts: the contact list's room (-1 when the narrow phase wrote the
// slots itself and stored no list).
__device__ __forceinline__ void finalize_slot_regions_body(DevCounters* c, int32_t n_verts, int32_t stride,
                                                           int64_t cap_contacts) {
    const long long H = c->n_hs;
    const long long nc = c->n_contacts;
    if (c->max_slot > stride) c->status |= ST_HS;
    if (cap_contacts >= 0 && nc > cap_contacts) c->status |= ST_CONTACTS;
    c->need[3] = max(c->need[3], nc);
    c->need[4] = max(c->need[4], (long long)c->max_slot * (long long)n_verts);
    c->totals[3] += H;
    c->totals[8] += nc;
    c->totals[9] += 1;
    c->last_hs = (int32_t)H;
    c->last_nc = (int32_t)nc;
}

__device__ __forceinline__ void reset_build_counters(DevCounters* c) {
    c->n_vf = c->n_ee = c->n_vv = c->n_ve = 0;
    c->n_large_t = c->n_large_e = 0;
    reset_region_counters(c);
}

__device__ __forceinline__ void spread_add(DevCounters* c, int which, unsigned long long n) {
    atomicAdd((unsigned long long*)&c->spread[which][blockIdx.x & 63], n);
}

// Maximum of one word of the 64 maxima slots, which it clears; called by the
// 64 lanes of one wavefront, after the launches that wrote the slots.
__device__ __forceinline__ uint32_t take_maximum(DevCounters* c, int word) {
    const int lane = threadIdx.x & 63;
    uint32_t m = c->maxima[lane][word];
    c->maxima[lane][word] = 0u;
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    return m;
}

// One binned entry of the grid: its padded box, index, flags and vertices (48 B).
struct GridEntry {
    float lo[3];
    int32_t idx;
    float hi[3];
    uint32_t flags;   // bit 0: all vertices static; bits 1..5: level; bits 8..23: mesh id
    int32_t v[3];     // the primitive's vertices (an edge repeats its second, a point its only one)
    int32_t pad;
};

// A pair inside the interaction range, between the two passes of the region
// build: normal (side A away from side B), phi, side A's share, the pair.
struct alignas(16) Contact {
    float n[3];
    float phi;
    float dA, dB;      // d = s phi of side A and of side B
    int32_t a;         // kind << 30 | first primitive
    int32_t b;         // second primitive
    // the vertices that receive a half-space, side A first (one for a vertex or
    // particle, two for an edge), then side B; -1 for a static vertex or none
    int32_t rv[4];
    float sA, sB;      // the shares s of side A and side B (Eq. 2)
    int32_t pad[2];
};

struct ParamSrc {
    const MeshParams* table;   // device table, or nullptr for the single mesh `one`
    const uint16_t* vmesh;     // per-vertex mesh id, or nullptr
    MeshParams one;
    __device__ __forceinline__ int mesh_of(int v) const { return vmesh ? (int)vmesh[v] : 0; }
    __device__ __forceinline__ MeshParams get(int m) const { return table ? table[m] : one; }
};

__device__ __forceinline__ uint32_t mix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x7feb352dU;
    h ^= h >> 15;
    h *= 0x846ca68bU;
    h ^= h >> 16;
    return h;
}

// Bucket of cell (cx, cy, cz) of mesh `salt` in a table of 2^log2s buckets
// (log2s >= 6): the 64 cells of a 4 x 4 x 4 block share the high bits, a hash
// of the block; the hash is taken in three steps (z, then y, then x) so that a
// walk over neighbouring cells can share the first two.
__device__ __forceinline__ uint32_t hash_z(int cz, int salt) {
    return mix32((uint32_t)(cz >> 2) * 0xC2B2AE3Du ^ (uint32_t)salt);
}
__device__ __forceinline__ uint32_t hash_y(int cy, uint32_t hz) { return mix32((uint32_t)(cy >> 2) * 0x85EBCA77u ^ hz); }
__device__ __forceinline__ uint32_t bucket_x(int cx, int cy, int cz, uint32_t hy, int log2s) {
    const uint32_t low = (uint32_t)(cx & 3) | ((uint32_t)(cy & 3) << 2) | ((uint32_t)(cz & 3) << 4);
    const uint32_t h = mix32((uint32_t)(cx >> 2) * 0x9E3779B1u ^ hy);
    return low | ((h & ((1u << (log2s - 6)) - 1u)) << 6);
}
__device__ __forceinline__ uint32_t cell_bucket(int cx, int cy, int cz, int salt, int log2s) {
    return bucket_x(cx, cy, cz, hash_y(cy, hash_z(cz, salt)), log2s);
}

// Grid cell of coordinate v (cell size 1 / inv_h).  The cells are shifted by
// half a cell so that a plane through the origin (the usual ground) lies inside
// a cell row at every level instead of on a cell boundary, which would put
// every box resting on it across two cell rows.  The map is monotone in v,
// which is all the stencil argument needs.
__device__ __forceinline__ int cell_coord(float v, float inv_h) {
    float c = floorf(v * inv_h + 0.5f);
    c = fminf(fmaxf(c, -1.0e9f), 1.0e9f);
    return (int)c;
}

// ---- launchers (defined in the .hip files) ----
struct Scene {
    int32_t n_verts, n_tris, n_edges, n_free;
    const float* x;
    const float* inv_mass;
    const int32_t* tris;
    const int32_t* edges;
    const int32_t* free_list;   // [n_free] free particles (vertices in no edge / triangle)
    const uint8_t* vflags;      // [n_verts] VF_FREE | VF_COLOR0
    int32_t skin_iters;         // candidate builds: further iterations the lists must cover
    int32_t skin_wide;          // candidate builds: moving boxes padded by MeshParams::pad_wide
    int32_t build_gated;        // candidate builds: run only when DevCounters::rebuild is set
    const uint32_t* skip;       // nullable: kernels return at once when *skip != 0 (the
                                // substep's iterations ended at the convergence check)
    ParamSrc prm;
};

// Bucket tables, stored one after the other: triangles of level 0, triangles
// of the coarser levels, edges of level 0, edges of the coarser levels, free
// particles (level 0 only), vertices (query order only, level 0).  Splitting
// off the coarser levels keeps their few entries from sharing buckets with the
// many of level 0: a lookup at a coarse level then meets (nearly) only entries
// of its own level.
enum : int { TB_TRI0 = 0, TB_TRIC = 1, TB_EDGE0 = 2, TB_EDGEC = 3, TB_PART = 4, TB_VERT = 5, TB_COUNT = 6 };

// Table of an entry kind (0 triangles, 1 edges, 2 particles, 3 vertices) at a level.
__device__ __forceinline__ int table_of(int kind0, int level) {
    return kind0 == 0 ? (level ? TB_TRIC : TB_TRI0) : kind0 == 1 ? (level ? TB_EDGEC : TB_EDGE0)
                                                    : (kind0 == 2 ? TB_PART : TB_VERT);
}

struct GridWs {
    // table t has 2^log2k[t] buckets starting at bucket off[t]; off[TB_COUNT] = all buckets
    int32_t log2k[TB_COUNT];
    int32_t off[TB_COUNT + 1];
    int32_t* cnt;               // [off[TB_COUNT]] counts, zero between builds
    int32_t* start;             // [off[TB_COUNT] + 1] exclusive prefix
    int32_t* rank;              // [T + E + F + N] rank of each entry inside its bucket
    int32_t* key;               // [T + E + F + N] global bucket, -1 = not binned
    GridEntry* entries;         // [T + E + F + N] sorted in table order
    GridEntry* staged;          // [T + E + F + N] the same entries in primitive order
    uint32_t* level_mask;       // [n_meshes] grid levels occupied by each mesh
    int32_t n_meshes;
    int32_t* scan_tmp;          // block partials of the scan
    __device__ __forceinline__ int bucket(int table, int cx, int cy, int cz, int salt) const {
        return off[table] + (int)cell_bucket(cx, cy, cz, salt, log2k[table]);
    }
    // the same with the z and y steps of the hash already taken (hy)
    __device__ __forceinline__ int bucket_hy(int table, int cx, int cy, int cz, uint32_t hy) const {
        return off[table] + (int)bucket_x(cx, cy, cz, hy, log2k[table]);
    }
};

// The candidate lists: (vertex, triangle), (edge, edge), (particle, particle)
// and (particle, edge) pairs.
struct PairLists {
    int32_t* vf; int32_t* ee; int32_t* vv; int32_t* ve;
    int64_t cap_vf, cap_ee, cap_vv, cap_ve;
    __host__ __device__ PairCaps caps() const { return PairCaps{cap_vf, cap_ee, cap_vv, cap_ve}; }
};

// The hierarchy broad phase (k_lbvh.hip): buffers for L = T + E + F leaves.
struct LbvhWs {
    float* leaf_lo;          // [L][3] padded boxes, in target order
    float* leaf_hi;          // [L][3]
    uint32_t* leaf_meta;     // [L] bit 0 static, bits 8.. mesh id; ~0 = not binned
    uint64_t* keys_in;       // [L] Morton codes, target order
    uint64_t* keys_out;      // [L] sorted
    int32_t* idx_in;         // [L] target indices
    int32_t* idx_out;        // [L] target of each sorted position
    int32_t* leaf_parent;    // [L] by sorted position
    int32_t* child;          // [L - 1][2] children (bit 31: a leaf's sorted position)
    int32_t* node_parent;    // [L - 1]
    int32_t* node_flag;      // [L - 1] refit arrivals
    float* node_lo;          // [L - 1][3]
    float* node_hi;          // [L - 1][3]
    void* sort_temp;
    size_t sort_temp_bytes;
};
size_t lbvh_sort_temp_bytes(int n);
// Build the hierarchy over the targets of `sc`; then emit every candidate pair
// into pl (counts in c->n_vf, n_ee, n_vv, n_ve; list overflow as for the grid).
void launch_lbvh_build(const Scene& sc, LbvhWs& w, DevCounters* c, hipStream_t s);
void launch_lbvh_query(const Scene& sc, const LbvhWs& w, PairLists pl, DevCounters* c, hipStream_t s);

void launch_reset_build(DevCounters* c, uint32_t* level_mask, int n_meshes, hipStream_t s);
void launch_grid_count(const Scene& sc, GridWs& g, DevCounters* c, hipStream_t s);
// run_flag (nullable): the scan does nothing when *run_flag is 0; skip
// (nullable): nor when *skip is not 0
void launch_scan(const int32_t* in, int32_t* out, int32_t* zero_in, int n, int32_t* tmp, hipStream_t s,
                 const uint32_t* run_flag = nullptr, const uint32_t* skip = nullptr);
void launch_grid_scatter(const Scene& sc, GridWs& g, DevCounters* c, hipStream_t s);
void launch_pairs(const Scene& sc, const GridWs& g, PairLists pl, DevCounters* c, int split, hipStream_t s);
void launch_finalize_pairs(const GridWs& g, PairLists pl, DevCounters* c, hipStream_t s);

// The narrow phase over the candidate pairs (counts: the four list lengths,
// VF, EE, VV, VE, on the device).  slot_stride == 0: the kept pairs go into
// the contact list and vcount counts each vertex's half-spaces for the CSR;
// slot_stride > 0: their half-spaces go straight into per-vertex slots,
// slot_hs[v * slot_stride + k] for the k-th one vertex v receives, vcount[v]
// counting them (no contact list)
struct ColourJob;
void launch_contacts(const Scene& sc, const PairLists& pl, const int32_t* counts, Contact* contacts,
                     int64_t cap_contacts, int32_t* vcount, DevCounters* c, hipStream_t s,
                     ccfr_halfspace* slot_hs = nullptr, int32_t slot_stride = 0, const ColourJob* job = nullptr);
// The contact list's half-spaces into per-vertex slots: slot_hs[v * slot_stride + k]
// for the k-th one vertex v receives (vcount[v] counts them)
void launch_fill_slots(const Scene& sc, const Contact* contacts, int64_t cap_contacts, int32_t* vcount,
                       ccfr_halfspace* slot_hs, int32_t slot_stride, DevCounters* c, hipStream_t s,
                       const ColourJob* job = nullptr);
// finalize: close the region build (overflow bits, totals) in a launch of its own
void launch_fill(const Scene& sc, const Contact* contacts, int64_t cap_contacts, const int32_t* offsets,
                 int32_t* vcount, ccfr_halfspace* hs, int64_t cap_hs, DevCounters* c, bool finalize,
                 hipStream_t s);

// The first colour of the stretch pass, run by the iteration's closing kernel
// (total == 0: none).
struct StretchColor0 {
    const int32_t* edges_sorted;
    const float* rest_sorted;
    const int2* segs;
    int32_t nseg, total;
    const float* inv_mass;
    float* lambda_sorted;
    float alpha_t;
    const uint8_t* vflags;
};
// Edge t of a colour class whose edges lie in nseg segments of the
// colour-sorted edge array, segs[k] = (first edge, exclusive prefix of segment
// lengths): binary search for its segment.
__device__ __forceinline__ int colour_edge(const int2* segs, int nseg, int t) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].y <= t) lo = mid;
        else hi = mid - 1;
    }
    return segs[lo].x + (t - segs[lo].y);
}

// One XPBD distance-constraint update of edge e (Macklin et al. 2016): reads
// the endpoints from `src`, writes them to `dst` (the same array inside the
// pass; the first colour reads the prediction and writes p, so both endpoints
// are always written), and accumulates the edge's multiplier.
__device__ __forceinline__ void stretch_edge(int e, const int32_t* edges, const float* rest, const float* w,
                                             const float* src, float* dst, float* lambda, float alpha_t,
                                             bool always_write) {
    const int i = edges[2 * e], j = edges[2 * e + 1];
    const float wi = w[i], wj = w[j];
    const float W = wi + wj;
    float pi[3], pj[3], d[3];
    for (int c = 0; c < 3; ++c) {
        pi[c] = src[3 * i + c];
        pj[c] = src[3 * j + c];
        d[c] = pi[c] - pj[c];
    }
    const float len = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (W == 0.0f || len == 0.0f) {
        if (always_write)
            for (int c = 0; c < 3; ++c) {
                dst[3 * i + c] = pi[c];
                dst[3 * j + c] = pj[c];
            }
        return;
    }
    const float C = len - rest[e];
    const float lam = lambda[e];
    const float dl = (-C - alpha_t * lam) / (W + alpha_t);
    const float s = dl / len;
    for (int c = 0; c < 3; ++c) {
        dst[3 * i + c] = pi[c] + wi * s * d[c];
        dst[3 * j + c] = pj[c] - wj * s * d[c];
    }
    lambda[e] = lam + dl;
}

// A colour class of the stretch pass (edges as in colour_edge, total == 0:
// none) run by the first blocks of a kernel that precedes the next colour and
// touches neither p nor the multipliers: one thread per edge.
struct ColourJob {
    const int32_t* edges_sorted;
    const float* rest_sorted;
    const int2* segs;
    int32_t nseg, total;
    const float* inv_mass;
    float* p;
    float* lambda_sorted;
    float alpha_t;
};
inline int colour_job_blocks(const ColourJob& j, int block) {
    return j.total > 0 && j.nseg > 0 ? (int)((j.total + block - 1) / block) : 0;
}
__device__ __forceinline__ void run_colour_job(const ColourJob& j, int t) {
    if (t < j.total)
        stretch_edge(colour_edge(j.segs, j.nseg, t), j.edges_sorted, j.rest_sorted, j.inv_mass, j.p, j.p,
                     j.lambda_sorted, j.alpha_t, false);
}

// The start of an iteration's stretch pass: p = x_pred (n3 entries), and the
// first colour (c0.total edges) on it: an endpoint of such an edge gets its p
// from the edge's update, every other vertex a copy.  Entry i of the grid.
__device__ __forceinline__ void restart_pass(const float* x_pred, float* p, long long n3, const StretchColor0& c0,
                                             long long i) {
    if (i < n3 && !(c0.total > 0 && (c0.vflags[i / 3] & VF_COLOR0))) p[i] = x_pred[i];
    if (i < c0.total)
        stretch_edge(colour_edge(c0.segs, c0.nseg, (int)i), c0.edges_sorted, c0.rest_sorted, c0.inv_mass, x_pred, p,
                     c0.lambda_sorted, c0.alpha_t, true);
}
// restart_pass run by extra blocks of another kernel (n3 == 0: none).  The
// host kernel may hold few wavefronts per SIMD, so each thread copies
// kRestartWide entries (block q covers kRestartWide * block consecutive ones,
// every load coalesced, all loads issued before the stores) and takes one
// edge of colour 0.
constexpr int kRestartWide = 4;
struct RestartJob {
    const float* x_pred;
    float* p;
    long long n3;
    StretchColor0 c0;
};
inline int restart_job_blocks(const RestartJob& r, int block) {
    if (r.n3 <= 0) return 0;
    const long long span = (long long)kRestartWide * block;
    const long long copy_blocks = (r.n3 + span - 1) / span;
    const long long edge_blocks = ((long long)r.c0.total + block - 1) / block;
    return (int)(copy_blocks > edge_blocks ? copy_blocks : edge_blocks);
}
__device__ __forceinline__ void restart_pass_wide(const RestartJob& r, long long q, int t, int block) {
    const long long i0 = q * kRestartWide * block + t;
    float xv[kRestartWide];
    uint8_t fl[kRestartWide];
#pragma unroll
    for (int j = 0; j < kRestartWide; ++j) {
        const long long i = i0 + (long long)j * block;
        xv[j] = i < r.n3 ? r.x_pred[i] : 0.0f;
        fl[j] = (i < r.n3 && r.c0.total > 0) ? r.c0.vflags[i / 3] : (uint8_t)0;
    }
#pragma unroll
    for (int j = 0; j < kRestartWide; ++j) {
        const long long i = i0 + (long long)j * block;
        if (i < r.n3 && !(fl[j] & VF_COLOR0)) r.p[i] = xv[j];
    }
    const long long e = q * block + t;
    if (e < r.c0.total)
        stretch_edge(colour_edge(r.c0.segs, r.c0.nseg, (int)e), r.c0.edges_sorted, r.c0.rest_sorted, r.c0.inv_mass,
                     r.x_pred, r.p, r.c0.lambda_sorted, r.c0.alpha_t, true);
}

// The last colour of the stretch pass, folded into the projection that reads
// its result (last_edge == nullptr: none): last_edge[v] = (v's edge e in that
// colour, with bit 31 set when v is its second endpoint; the other endpoint),
// or (0, -1) for a vertex in no such edge.  The projection takes as v's
// proposal the position the edge's update gives it, computed from p as the
// colour's own launch would, and the edge's first endpoint writes the new
// multiplier to lambda_out (both endpoints read lambda_in, so the two arrays
// alternate between iterations).  The fast kernel hands the displacement of a
// vertex it defers to the slow one in y_def (3 floats per vertex).
// With prev_edge (the same kind of map for the colour before the last), that
// colour is folded in as well: each vertex recomputes its own and its
// last-colour partner's positions after it.
struct StretchLast {
    const int2* last_edge;
    const int2* prev_edge;
    const float* rest_sorted;
    const float* lambda_in;
    float* lambda_out;
    float alpha_t;
    float* y_def;
};
struct ProjectArgs {
    int32_t n_verts;
    const int32_t* offsets;
    const ccfr_halfspace* hs;
    int64_t cap_hs;
    const float* inv_mass;
    const float* y_in;       // displacement in (or nullptr: use p - x)
    const float* p;          // proposal positions (when y_in == nullptr)
    float* x_anchor;         // anchor, updated in place when y_out == nullptr
    float* y_out;
    uint8_t* halted;
    double* sort_key;        // [cap_hs] scratch of regions larger than a wavefront sorts
    int32_t* sort_idx;       // [cap_hs]
    int32_t* slow_list;      // [2 n_verts] vertices with a violated half-space: small regions from
                             // the front, large ones from the back of the first half, mid-size
                             // ones in the second half
    uint32_t* motion_max;    // nullable: slot words (32 apart) of the largest coordinate move of
                             // an anchor update (FP32 bits); a block writes slot blockIdx & 63
    // regions in per-vertex slots (slot_stride > 0, offsets unused): vertex v's
    // half-spaces are hs[v * slot_stride ...] and slot_counts[v] of them; the
    // projection sets each count back to zero once it has read it
    int32_t* slot_counts;
    int32_t slot_stride;
    ParamSrc prm;
    StretchLast sl;
    RestartJob next;         // the next iteration's stretch start, in extra blocks of the slow kernel
    const uint32_t* skip;    // nullable: return at once when *skip != 0
    uint32_t* shortfall_max; // nullable: slot words (as motion_max) of the largest
                             // |proposal| - |result| (FP32 bits, rounded up)
    uint8_t* halt_run;       // nullable: per-vertex consecutive halts, updated with every result
};
// zero_counters: clear the slow-list counters first (the substep clears them
// in launch_close_iteration instead)
void launch_project(const ProjectArgs& a, DevCounters* c, bool zero_counters, hipStream_t s);

// applyResponse of Alg. 4 (Sec. 3.3) per vertex on its region: proposals read
// from y_in (or p - x_anchor when y_in is null), results written to y_out (or
// into p, as the new proposal, when y_out is null).
struct ResponseArgs {
    int32_t n_verts;
    const int32_t* offsets;          // CSR regions (slot_stride == 0)
    const ccfr_halfspace* hs;
    const int32_t* slot_counts;      // per-vertex slots (slot_stride > 0)
    int32_t slot_stride;
    const float* inv_mass;
    const float* y_in;
    const float* x_anchor;
    float* p;
    float* y_out;
    float dt;
    ParamSrc prm;
    const uint32_t* skip;
    int32_t* list;                   // [n_verts] scratch: vertices with large regions
    DevCounters* c;                  // its length (n_resp)
};
// One lane per vertex; a vertex with more than 32 half-spaces is listed and
// taken by a wavefront in a second launch, and a third clears the list.
void launch_response(const ResponseArgs& a, hipStream_t s);

// halt_run (nullable): per-vertex consecutive-halt counts, cleared for the
// substep; iters_add: iterations the substep runs for certain (added to the
// counters' iterations run; 0 when its convergence check counts them)
void launch_predict(int n, const float* x, const float* v, const float* inv_mass, float dt,
                    float gx, float gy, float gz, float* x_pred, float* x_start, hipStream_t s,
                    uint8_t* halt_run = nullptr, DevCounters* c = nullptr, int iters_add = 0);
void launch_fill_zero(float* p, int64_t n, hipStream_t s);
void launch_copy(const float* src, float* dst, int64_t n, hipStream_t s);
// Between the region build and the stretch pass of a substep iteration: close
// the region build and, unless the next iteration reuses the lists, the
// candidate build (overflow bits, totals), clear the per-build counters (and
// then the level masks) for the next build, and copy the prediction into p.
// slot_stride > 0: the region build went into per-vertex slots (offsets unused)
void launch_close_iteration(const float* x_pred, float* p, int64_t n3, DevCounters* c, uint32_t* level_mask,
                            int n_meshes, int32_t n_verts, const int32_t* offsets, PairCaps caps,
                            int64_t cap_contacts, int64_t cap_hs, bool close_pairs, hipStream_t s,
                            int32_t slot_stride = 0, const StretchColor0* c0 = nullptr, bool finalize = true,
                            const ColourJob* job = nullptr, const uint32_t* skip = nullptr);
// Before the candidate stage of an iteration in a substep whose builds adapt to
// the motion: adds the last projection's largest move to the moves summed
// since the last build; if the sum may exceed `skin` (the least widening of
// any mesh's moving boxes), closes the last build and asks for a new one
// (DevCounters::rebuild), else the stage's kernels leave the lists as they are.
void launch_decide_build(DevCounters* c, uint32_t* level_mask, int n_meshes, double skin, PairCaps caps,
                         hipStream_t s, const uint32_t* skip = nullptr);
// evaluateConvergence of Alg. 4 (one thread): at the start of iteration
// `first == 0`, the substep's iterations end (DevCounters::converged) once the
// last projection's largest shortfall is at most tol; counts the iterations run.
void launch_decide_converged(DevCounters* c, float tol, int first, hipStream_t s);
void launch_stretch_segments(const int32_t* edges_sorted, const float* rest_sorted, const int2* segs, int32_t nseg,
                             int32_t total, const float* inv_mass, float* p, float* lambda_sorted, float alpha_t,
                             hipStream_t s, const uint32_t* skip = nullptr);
// last_edge[v] for the colour class (edges as in a stretch colour: nseg
// segments, total edges) as StretchLast reads it; n_verts entries.
void launch_last_colour_map(const int32_t* edges_sorted, const int2* segs, int32_t nseg, int32_t total,
                            int32_t n_verts, int2* last_edge, hipStream_t s);
void launch_update_velocity(int n, const float* x, const float* x_start, float inv_dt, float* v,
                            hipStream_t s);

}  // namespace ccfr
