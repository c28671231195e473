// k_lbvh.hip -- the broad phase as a linear bounding-volume hierarchy over the
// padded boxes of every target primitive (triangles, edges, free particles):
// the GPU analogue of the paper's AABB tree (Sec. 4.1), behind the same
// candidate contract as the hash grid (k_broadphase.hip): a pair is emitted
// iff the FP32 boxes of the grid's target_box definition overlap, so both
// broad phases give the same lists after sorting.
//
// Per build (all kernels return at once when a gated build is not due):
//   leaves    one thread per target: its box (the grid's definition, widened
//             the same way for shared builds), a 63-bit Morton code of its
//             centre quantised by the mesh's grid cell, its index
//   sort      the (code, index) pairs by code (hipCUB radix sort)
//   hierarchy one thread per internal node: its key range and split from the
//             longest common prefix of neighbouring sorted codes (Karras,
//             "Maximizing Parallelism in the Construction of BVHs, Octrees
//             and k-d Trees", HPG 2012), equal codes ordered by index
//   refit     one thread per leaf walks towards the root; the second child to
//             arrive at a node merges both boxes (an atomic per node)
//   query     one thread per vertex and per edge: a stack walk of the tree
//             with the query's own padded box; at a leaf the contract's box
//             test and pair rules decide (vertex-face: vertex not in the
//             triangle; edge-edge: the higher edge index, no shared vertex;
//             particle-particle: both free, the higher index; particle-edge:
//             a free particle's query; never two static primitives, never
//             two meshes); found pairs are staged in per-lane LDS slices
//             (pair_emit.h) and written out a wavefront or a block at a time.
#include <hipcub/hipcub.hpp>

#include "ccfr_internal.h"
#include "pair_emit.h"

namespace ccfr {

namespace {

constexpr int kBlock = 256;
constexpr int kStack = 64;
static_assert(kBlock == kEmitBlock, "the query kernel stages pairs in blocks of kEmitBlock lanes");

__device__ __forceinline__ void load3(const float* x, int v, float o[3]) {
    o[0] = x[3 * v + 0];
    o[1] = x[3 * v + 1];
    o[2] = x[3 * v + 2];
}

// Target t: triangles, edges, free particles (the grid's order).
struct Leaf {
    int kind, idx, nv;
    int v[3];
};

__device__ __forceinline__ Leaf leaf_of(const Scene& sc, int t) {
    Leaf g;
    if (t < sc.n_tris) {
        g.kind = KIND_VF; g.idx = t; g.nv = 3;
        g.v[0] = sc.tris[3 * t]; g.v[1] = sc.tris[3 * t + 1]; g.v[2] = sc.tris[3 * t + 2];
    } else if (t < sc.n_tris + sc.n_edges) {
        const int e = t - sc.n_tris;
        g.kind = KIND_EE; g.idx = e; g.nv = 2;
        g.v[0] = sc.edges[2 * e]; g.v[1] = sc.edges[2 * e + 1]; g.v[2] = g.v[1];
    } else {
        const int p = sc.free_list[t - sc.n_tris - sc.n_edges];
        g.kind = KIND_VV; g.idx = p; g.nv = 1;
        g.v[0] = g.v[1] = g.v[2] = p;
    }
    return g;
}

// The padded box of a primitive with vertices v[0..nv), widened as the grid
// widens the boxes of builds shared by several iterations (the same FP32
// operations, so the same box).
__device__ __forceinline__ float skin_pad(float pad, float r, int k, float maxabs) {
    const float kf = (float)k;
    const float reach = kf * (r * (1.0f + 0x1p-18f) + (maxabs + (kf + 1.0f) * 2.0f * r) * 0x1p-21f);
    return __int_as_float(__float_as_int(pad + reach) + 1);
}

__device__ __forceinline__ bool prim_box(const Scene& sc, const int* v, int nv, const MeshParams& P, float lo[3],
                                         float hi[3], bool* is_static) {
    float pad = P.pad;
    float p[3];
    load3(sc.x, v[0], p);
    bool fin = isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]);
    float mn[3] = {p[0], p[1], p[2]}, mx[3] = {p[0], p[1], p[2]};
    bool st = sc.inv_mass[v[0]] == 0.0f;
    for (int i = 1; i < nv; ++i) {
        load3(sc.x, v[i], p);
        fin = fin && isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]);
        st = st && (sc.inv_mass[v[i]] == 0.0f);
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

__device__ __forceinline__ bool overlap(const float alo[3], const float ahi[3], const float blo[3],
                                        const float bhi[3]) {
    return (alo[0] <= bhi[0]) & (blo[0] <= ahi[0]) & (alo[1] <= bhi[1]) & (blo[1] <= ahi[1]) &
           (alo[2] <= bhi[2]) & (blo[2] <= ahi[2]);
}

// 21 bits of x spread to every third bit
__device__ __forceinline__ uint64_t spread3(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint64_t morton_of(const float lo[3], const float hi[3], float inv_h) {
    uint64_t c[3];
    for (int k = 0; k < 3; ++k) {
        float q = floorf(0.5f * (lo[k] + hi[k]) * inv_h) + 1048576.0f;
        q = fminf(fmaxf(q, 0.0f), 2097151.0f);
        c[k] = (uint64_t)q;
    }
    return spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
}

// Leaf boxes and Morton codes.  Non-finite or unused leaves sort last.
__global__ __launch_bounds__(kBlock) void k_lbvh_leaves(Scene sc, LbvhWs w, DevCounters* c) {
    if (sc.skip && *sc.skip) return;
    if (sc.build_gated && !c->rebuild) return;
    const int n = sc.n_tris + sc.n_edges + sc.n_free;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    const Leaf g = leaf_of(sc, t);
    const int mesh = sc.prm.mesh_of(g.v[0]);
    const MeshParams P = sc.prm.get(mesh);
    float lo[3], hi[3];
    bool st;
    uint64_t code = ~0ull;
    uint32_t meta = 0xffffffffu;
    if (prim_box(sc, g.v, g.nv, P, lo, hi, &st)) {
        code = morton_of(lo, hi, P.inv_h) >> 1;             // 62 bits, below the invalid code
        meta = (st ? 1u : 0u) | ((uint32_t)mesh << 8);
    } else {
        atomicOr(&c->status, ST_NONFINITE);
        for (int k = 0; k < 3; ++k) {
            lo[k] = 1.0f;                                   // an empty box: overlaps nothing
            hi[k] = -1.0f;
        }
    }
    for (int k = 0; k < 3; ++k) {
        w.leaf_lo[3 * t + k] = lo[k];
        w.leaf_hi[3 * t + k] = hi[k];
    }
    w.leaf_meta[t] = meta;
    w.keys_in[t] = code;
    w.idx_in[t] = t;
}

// longest common prefix of sorted entries i and j (equal codes: by index)
__device__ __forceinline__ int delta_of(const uint64_t* keys, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    const uint64_t a = keys[i], b = keys[j];
    if (a != b) return __clzll((long long)(a ^ b));
    return 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

// Internal node i of n - 1 (children: bit 31 set = leaf position)
__global__ __launch_bounds__(kBlock) void k_lbvh_hierarchy(Scene sc, LbvhWs w, int n, DevCounters* c) {
    if (sc.skip && *sc.skip) return;
    if (sc.build_gated && !c->rebuild) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n - 1) return;
    const uint64_t* K = w.keys_out;
    const int d = (delta_of(K, n, i, i + 1) - delta_of(K, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta_of(K, n, i, i - d);
    int lmax = 2;
    while (delta_of(K, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta_of(K, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = delta_of(K, n, i, j);
    int s = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (delta_of(K, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int gamma = i + s * d + min(d, 0);
    const int left = min(i, j) == gamma ? (int)(0x80000000u | (uint32_t)gamma) : gamma;
    const int right = max(i, j) == gamma + 1 ? (int)(0x80000000u | (uint32_t)(gamma + 1)) : gamma + 1;
    w.child[2 * i] = left;
    w.child[2 * i + 1] = right;
    if (left < 0) w.leaf_parent[left & 0x7fffffff] = i;
    else w.node_parent[left] = i;
    if (right < 0) w.leaf_parent[right & 0x7fffffff] = i;
    else w.node_parent[right] = i;
    w.node_flag[i] = 0;
    if (i == 0) w.node_parent[0] = -1;
}

__device__ __forceinline__ void child_box(const LbvhWs& w, int ch, float lo[3], float hi[3]) {
    if (ch < 0) {
        const int t = w.idx_out[ch & 0x7fffffff];
        for (int k = 0; k < 3; ++k) {
            lo[k] = w.leaf_lo[3 * t + k];
            hi[k] = w.leaf_hi[3 * t + k];
        }
    } else {
        for (int k = 0; k < 3; ++k) {
            lo[k] = __hip_atomic_load(&w.node_lo[3 * ch + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            hi[k] = __hip_atomic_load(&w.node_hi[3 * ch + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Bottom-up boxes: each leaf climbs; the second arrival at a node merges its
// two children and climbs on, the first stops (each node is merged once).
__global__ __launch_bounds__(kBlock) void k_lbvh_refit(Scene sc, LbvhWs w, int n, DevCounters* c) {
    if (sc.skip && *sc.skip) return;
    if (sc.build_gated && !c->rebuild) return;
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= n || n < 2) return;
    int node = w.leaf_parent[q];
    while (node >= 0) {
        __threadfence();
        const int prev = atomicAdd(&w.node_flag[node], 1);
        if (prev == 0) return;                      // the other child is still on its way
        __threadfence();
        float alo[3], ahi[3], blo[3], bhi[3];
        child_box(w, w.child[2 * node], alo, ahi);
        child_box(w, w.child[2 * node + 1], blo, bhi);
        for (int k = 0; k < 3; ++k) {
            __hip_atomic_store(&w.node_lo[3 * node + k], fminf(alo[k], blo[k]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&w.node_hi[3 * node + k], fmaxf(ahi[k], bhi[k]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        node = w.node_parent[node];
    }
}

// A child's box in the query (the refit has completed: plain loads)
__device__ __forceinline__ void child_box_q(const LbvhWs& w, int ch, float lo[3], float hi[3]) {
    if (ch < 0) {
        const int t = w.idx_out[ch & 0x7fffffff];
        for (int k = 0; k < 3; ++k) {
            lo[k] = w.leaf_lo[3 * t + k];
            hi[k] = w.leaf_hi[3 * t + k];
        }
    } else {
        for (int k = 0; k < 3; ++k) {
            lo[k] = w.node_lo[3 * ch + k];
            hi[k] = w.node_hi[3 * ch + k];
        }
    }
}

// One thread per query: vertices (vertex-face pairs; for a free particle also
// particle-particle and particle-edge pairs), then edges (edge-edge pairs).
__global__ __launch_bounds__(kBlock) void k_lbvh_query(Scene sc, LbvhWs w, int n, PairLists pl, DevCounters* c) {
    if (sc.skip && *sc.skip) return;
    if (sc.build_gated && !c->rebuild) return;
    const int q = blockIdx.x * kBlock + threadIdx.x;
    const int nq = sc.n_verts + sc.n_edges;
    bool active = q < nq && n > 0;
    int qv[2] = {0, 0};
    bool is_edge = false, q_static = false, q_free = false;
    int mesh = 0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    if (active) {
        if (q < sc.n_verts) {
            qv[0] = qv[1] = q;
            q_free = sc.vflags && (sc.vflags[q] & VF_FREE);
        } else {
            is_edge = true;
            qv[0] = sc.edges[2 * (q - sc.n_verts)];
            qv[1] = sc.edges[2 * (q - sc.n_verts) + 1];
        }
        mesh = sc.prm.mesh_of(qv[0]);
        const MeshParams P = sc.prm.get(mesh);
        active = prim_box(sc, qv, is_edge ? 2 : 1, P, lo, hi, &q_static);
        if (!active) atomicOr(&c->status, ST_NONFINITE);
    }
    const int qe = is_edge ? q - sc.n_verts : -1;
    __shared__ int32_t lane_pairs[kLaneCap][kEmitBlock];
    LaneBuf lb{(LDS_PTR int32_t*)&lane_pairs[0][threadIdx.x], 0, 0, 0, !is_edge, is_edge ? qe : qv[0]};
    int stack[kStack];
    int sp = 0;
    int node = n > 1 ? 0 : (int)0x80000000u;       // a single leaf is its own root
    bool done = !active;
    while (true) {
        lane_room_for(lb, pl, c, 1);                 // every lane of the wavefront, done or not
        if (!done) {
            float blo[3], bhi[3];
            if (node < 0) {
                // a leaf: the contract's box test and the pair rules
                const int t = w.idx_out[node & 0x7fffffff];
                for (int k = 0; k < 3; ++k) {
                    blo[k] = w.leaf_lo[3 * t + k];
                    bhi[k] = w.leaf_hi[3 * t + k];
                }
                const uint32_t meta = w.leaf_meta[t];
                const bool ok = meta != 0xffffffffu && (meta >> 8) == (uint32_t)mesh &&
                                !(q_static && (meta & 1u)) && overlap(lo, hi, blo, bhi);
                if (ok) {
                    if (t < sc.n_tris) {
                        if (!is_edge) {
                            const int a = sc.tris[3 * t], b = sc.tris[3 * t + 1], d = sc.tris[3 * t + 2];
                            lane_put(lb, t, a != qv[0] && b != qv[0] && d != qv[0]);
                        }
                    } else if (t < sc.n_tris + sc.n_edges) {
                        const int e = t - sc.n_tris;
                        if (is_edge && e > qe) {
                            const int a = sc.edges[2 * e], b = sc.edges[2 * e + 1];
                            lane_put(lb, e, a != qv[0] && a != qv[1] && b != qv[0] && b != qv[1]);
                        } else if (!is_edge && q_free) {
                            lane_put_ve(lb, e, true);        // a free particle is in no edge
                        }
                    } else if (!is_edge && q_free) {
                        const int p = sc.free_list[t - sc.n_tris - sc.n_edges];
                        lane_put_vv(lb, p, p > qv[0]);
                    }
                }
                node = sp > 0 ? stack[--sp] : 0x7fffffff;
            } else {
                const int l = w.child[2 * node], r = w.child[2 * node + 1];
                float llo[3], lhi[3], rlo[3], rhi[3];
                child_box_q(w, l, llo, lhi);
                child_box_q(w, r, rlo, rhi);
                const bool ol = overlap(lo, hi, llo, lhi), orr = overlap(lo, hi, rlo, rhi);
                if (ol && orr) {
                    if (sp < kStack) stack[sp++] = r;
                    else atomicOr(&c->status, ST_LARGE);       // too deep: reported, never silent
                    node = l;
                } else if (ol) {
                    node = l;
                } else if (orr) {
                    node = r;
                } else {
                    node = sp > 0 ? stack[--sp] : 0x7fffffff;
                }
            }
            if (node == 0x7fffffff) done = true;
        }
        if (__ballot(!done) == 0ull) break;
    }
    block_flush(lb, pl, c);
}

inline int blocks_for(long long n) { return (int)std::max<long long>(1, (n + kBlock - 1) / kBlock); }

}  // namespace

size_t lbvh_sort_temp_bytes(int n) {
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                              (const int32_t*)nullptr, (int32_t*)nullptr, n, 0, 64);
    return bytes;
}

void launch_lbvh_build(const Scene& sc, LbvhWs& w, DevCounters* c, hipStream_t s) {
    const int n = sc.n_tris + sc.n_edges + sc.n_free;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_lbvh_leaves, dim3(blocks_for(n)), dim3(kBlock), 0, s, sc, w, c);
    size_t bytes = w.sort_temp_bytes;
    (void)hipcub::DeviceRadixSort::SortPairs(w.sort_temp, bytes, w.keys_in, w.keys_out, w.idx_in, w.idx_out, n, 0,
                                              64, s);
    if (n > 1) {
        hipLaunchKernelGGL(k_lbvh_hierarchy, dim3(blocks_for(n - 1)), dim3(kBlock), 0, s, sc, w, n, c);
        hipLaunchKernelGGL(k_lbvh_refit, dim3(blocks_for(n)), dim3(kBlock), 0, s, sc, w, n, c);
    }
}

void launch_lbvh_query(const Scene& sc, const LbvhWs& w, PairLists pl, DevCounters* c, hipStream_t s) {
    const int n = sc.n_tris + sc.n_edges + sc.n_free;
    hipLaunchKernelGGL(k_lbvh_query, dim3(blocks_for((long long)sc.n_verts + sc.n_edges)), dim3(kBlock), 0, s, sc,
                       w, n, pl, c);
}

}  // namespace ccfr
