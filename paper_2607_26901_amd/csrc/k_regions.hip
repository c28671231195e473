// k_regions.hip -- per-vertex convex regions (Alg. 3 with Eq. 1-3) on gfx950.
//
// Work is per candidate pair rather than per vertex: the pair's closest points
// are computed once and its half-space is scattered to every vertex of the pair
// with non-zero inverse mass.  This yields exactly the union of Alg. 3's three
// per-vertex loops (VF for the vertex, EE for both edges' endpoints, FV for the
// face's vertices), because all of them evaluate the same closest points of the
// same pair; the point interactions of Sec. 4.2 (particle-particle, and a free
// particle against an edge: the particle on one side, the edge's endpoints
// with their barycentric share on the other) are built the same way.  Two
// passes build the CSR:
//
//   contacts  per pair: closest points in pair-local coordinates (one vertex
//             subtracted first), phi = |x_A - x_B| - xi, kept while phi < 2r;
//             kept pairs are compacted into 64 B Contact records (normal, phi,
//             the two sides' d = s phi and shares s, the receiving vertices)
//             and every receiving vertex's count is incremented.  The arithmetic runs in FP64 registers by default
//             (FP32 in, FP32 out): near-parallel edges make the FP32 closest
//             points lose digits as 1/sin^2 of their angle, and CDNA's FP64
//             rate keeps this memory-bound kernel's cost unchanged.
//   scan      counts -> offsets
//   fill      per contact: (n, s_A phi) to side A's vertices, (-n, s_B phi) to
//             side B's, each at offsets[v] + (atomic decrement of its count),
//             which also returns the counts to zero for the next build
//
// Inside a substep the regions go into per-vertex slots instead: every kept
// pair's half-spaces go into the next free slot of each receiving vertex (one
// atomic each), either from the contact list by a fill launch or, with the
// direct_regions knob, straight from the narrow phase (no contact list).
//
// Readings of the printed Alg. 3: d = s (|n| - xi); for the face side of a
// vertex-face pair the normal points from the vertex towards the face and the
// share is w_f / (w_f + w_q); effective inverse masses are sum_i bary_i w_i,
// and a pair with w_A + w_B = 0 gives no half-space; parallel edges
// (|d1 x d2|^2 <= 1e-10 |d1|^2 |d2|^2) take the midpoint of their overlap;
// zero-area triangles, zero-length edges and coincident closest points are
// skipped and counted.
#include "ccfr_internal.h"

namespace ccfr {

namespace {

constexpr int kBlock = 256;

template <class R>
__device__ __forceinline__ void ld3(const float* x, int v, R o[3]) {
    o[0] = (R)x[3 * v]; o[1] = (R)x[3 * v + 1]; o[2] = (R)x[3 * v + 2];
}
template <class R>
__device__ __forceinline__ R dot3(const R a[3], const R b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
template <class R>
__device__ __forceinline__ R clamp01(R v) {
    return v < R(0) ? R(0) : (v > R(1) ? R(1) : v);
}

// Closest point of triangle (a, b, c) to the origin (the query vertex has been
// subtracted): Voronoi-region walk.  Returns false for a zero-area triangle.
template <class R>
__device__ bool closest_on_triangle(const R a[3], const R b[3], const R c[3], R q[3], R bary[3]) {
    R ab[3], ac[3], n[3];
    for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; ac[k] = c[k] - a[k]; }
    n[0] = ab[1] * ac[2] - ab[2] * ac[1];
    n[1] = ab[2] * ac[0] - ab[0] * ac[2];
    n[2] = ab[0] * ac[1] - ab[1] * ac[0];
    if (dot3(n, n) <= R(1e-12) * dot3(ab, ab) * dot3(ac, ac)) return false;
    // p = origin: ap = -a, bp = -b, cp = -c
    const R d1 = -dot3(ab, a), d2 = -dot3(ac, a);
    const R d3 = -dot3(ab, b), d4 = -dot3(ac, b);
    const R d5 = -dot3(ab, c), d6 = -dot3(ac, c);
    R u, v, w;   // barycentrics of a, b, c
    if (d1 <= R(0) && d2 <= R(0)) { u = 1; v = 0; w = 0; }
    else if (d3 >= R(0) && d4 <= d3) { u = 0; v = 1; w = 0; }
    else if (d6 >= R(0) && d5 <= d6) { u = 0; v = 0; w = 1; }
    else {
        const R vc = d1 * d4 - d3 * d2;
        const R vb = d5 * d2 - d1 * d6;
        const R va = d3 * d6 - d5 * d4;
        if (vc <= R(0) && d1 >= R(0) && d3 <= R(0)) {
            v = d1 / (d1 - d3); u = R(1) - v; w = 0;
        } else if (vb <= R(0) && d2 >= R(0) && d6 <= R(0)) {
            w = d2 / (d2 - d6); u = R(1) - w; v = 0;
        } else if (va <= R(0) && (d4 - d3) >= R(0) && (d5 - d6) >= R(0)) {
            w = (d4 - d3) / ((d4 - d3) + (d5 - d6)); v = R(1) - w; u = 0;
        } else {
            const R den = R(1) / (va + vb + vc);
            v = vb * den; w = vc * den; u = R(1) - v - w;
        }
    }
    bary[0] = u; bary[1] = v; bary[2] = w;
    for (int k = 0; k < 3; ++k) q[k] = u * a[k] + v * b[k] + w * c[k];
    return true;
}

// Closest points p = a + s (b - a), q = c + t (d - c) of two segments.
// Returns 0, 1 (parallel rule used) or -1 (zero-length segment).
template <class R>
__device__ int closest_on_segments(const R a[3], const R b[3], const R c[3], const R d[3], R* s_out, R* t_out) {
    R d1[3], d2[3], r[3], cr[3];
    for (int k = 0; k < 3; ++k) { d1[k] = b[k] - a[k]; d2[k] = d[k] - c[k]; r[k] = a[k] - c[k]; }
    const R A = dot3(d1, d1), E = dot3(d2, d2);
    if (A <= R(0) || E <= R(0)) return -1;
    const R F = dot3(d2, r), C = dot3(d1, r), B = dot3(d1, d2);
    cr[0] = d1[1] * d2[2] - d1[2] * d2[1];
    cr[1] = d1[2] * d2[0] - d1[0] * d2[2];
    cr[2] = d1[0] * d2[1] - d1[1] * d2[0];
    R s, t;
    if (dot3(cr, cr) <= R(1e-10) * A * E) {
        R ca[3], da[3];
        for (int k = 0; k < 3; ++k) { ca[k] = c[k] - a[k]; da[k] = d[k] - a[k]; }
        const R tc = dot3(ca, d1) / A, td = dot3(da, d1) / A;
        const R lo = tc < td ? tc : td, hi = tc < td ? td : tc;
        const R olo = lo > R(0) ? lo : R(0), ohi = hi < R(1) ? hi : R(1);
        s = olo <= ohi ? R(0.5) * (olo + ohi) : (hi < R(0) ? R(0) : R(1));
        R pc[3];
        for (int k = 0; k < 3; ++k) pc[k] = a[k] + s * d1[k] - c[k];
        t = clamp01(dot3(pc, d2) / E);
        *s_out = s; *t_out = t;
        return 1;
    }
    const R den = A * E - B * B;
    s = clamp01((B * F - C * E) / den);
    t = (B * s + F) / E;
    if (t < R(0)) { t = 0; s = clamp01(-C / A); }
    else if (t > R(1)) { t = 1; s = clamp01((B - C) / A); }
    *s_out = s; *t_out = t;
    return 0;
}

// Appends the contacts of the whole block with one atomic: every thread of the
// block must call it (the rounds of k_contacts are uniform across the block).
constexpr int kWavesPerBlock = kBlock / 64;

__device__ __forceinline__ void block_append(Contact* list, int32_t* counter, int64_t cap, const Contact& rec,
                                             bool pred, int* wave_cnt, int* block_base) {
    const unsigned long long mask = __ballot(pred);
    const int lane = __lane_id();
    const int wave = threadIdx.x / 64;
    if (lane == 0) wave_cnt[wave] = __popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) {
            const int t = wave_cnt[w];
            wave_cnt[w] = acc;
            acc += t;
        }
        *block_base = acc ? atomicAdd(counter, acc) : 0;
    }
    __syncthreads();
    if (pred) {
        const long long idx = (long long)*block_base + wave_cnt[wave] + __popcll(mask & ((1ull << lane) - 1ull));
        if (idx < cap) list[idx] = rec;
    }
    __syncthreads();
}

// Evaluate pair i of the concatenated lists [VF | EE | VV | VE].  On success fills
// the contact (normal from side B towards side A) and the vertices of both sides.
struct PairVerts {
    int nA, nB;
    int a[2], b[3];
    float wa[2], wb[3];   // their inverse masses (filled for pairs in range)
};

template <class R>
__device__ bool eval_pair(const Scene& sc, int kind, int pa, int pb, Contact* rec, PairVerts* pv,
                          bool* degenerate) {
    *degenerate = false;
    R nvec[3];
    R wA, wB;
    int mesh;
    // geometry first: the inverse masses are read only for the few pairs in range
    R bary[3], s = R(0), t = R(0);
    if (kind == KIND_VF) {
        const int v = pa, tr = pb;
        const int t0 = sc.tris[3 * tr], t1 = sc.tris[3 * tr + 1], t2 = sc.tris[3 * tr + 2];
        mesh = sc.prm.mesh_of(v);
        R p[3], A[3], B[3], Cc[3];
        ld3(sc.x, v, p); ld3(sc.x, t0, A); ld3(sc.x, t1, B); ld3(sc.x, t2, Cc);
        for (int k = 0; k < 3; ++k) { A[k] -= p[k]; B[k] -= p[k]; Cc[k] -= p[k]; }
        R q[3];
        if (!closest_on_triangle(A, B, Cc, q, bary)) { *degenerate = true; return false; }
        for (int k = 0; k < 3; ++k) nvec[k] = -q[k];
        pv->nA = 1; pv->a[0] = v;
        pv->nB = 3; pv->b[0] = t0; pv->b[1] = t1; pv->b[2] = t2;
    } else if (kind == KIND_EE) {
        const int e = pa, f = pb;   // e < f
        const int e0 = sc.edges[2 * e], e1 = sc.edges[2 * e + 1];
        const int f0 = sc.edges[2 * f], f1 = sc.edges[2 * f + 1];
        mesh = sc.prm.mesh_of(e0);
        R A[3], B[3], Cc[3], D[3];
        ld3(sc.x, e0, A); ld3(sc.x, e1, B); ld3(sc.x, f0, Cc); ld3(sc.x, f1, D);
        for (int k = 0; k < 3; ++k) { B[k] -= A[k]; Cc[k] -= A[k]; D[k] -= A[k]; A[k] = R(0); }
        if (closest_on_segments(A, B, Cc, D, &s, &t) < 0) { *degenerate = true; return false; }
        for (int k = 0; k < 3; ++k) {
            const R pp = s * B[k];
            const R qq = Cc[k] + t * (D[k] - Cc[k]);
            nvec[k] = pp - qq;
        }
        pv->nA = 2; pv->a[0] = e0; pv->a[1] = e1;
        pv->nB = 2; pv->b[0] = f0; pv->b[1] = f1;
    } else if (kind == KIND_VE) {
        // particle p against edge (e0, e1): the closest point e0 + t (e1 - e0),
        // t clamped to [0, 1], in coordinates relative to p
        const int p = pa, e = pb;
        const int e0 = sc.edges[2 * e], e1 = sc.edges[2 * e + 1];
        mesh = sc.prm.mesh_of(p);
        R P0[3], A[3], B[3];
        ld3(sc.x, p, P0); ld3(sc.x, e0, A); ld3(sc.x, e1, B);
        R ab[3];
        for (int k = 0; k < 3; ++k) { A[k] -= P0[k]; B[k] -= P0[k]; ab[k] = B[k] - A[k]; }
        const R L = dot3(ab, ab);
        if (!(L > R(0))) { *degenerate = true; return false; }
        t = clamp01(-dot3(A, ab) / L);
        for (int k = 0; k < 3; ++k) nvec[k] = -(A[k] + t * ab[k]);
        pv->nA = 1; pv->a[0] = p;
        pv->nB = 2; pv->b[0] = e0; pv->b[1] = e1;
    } else {
        const int i = pa, j = pb;
        mesh = sc.prm.mesh_of(i);
        R A[3], B[3];
        ld3(sc.x, i, A); ld3(sc.x, j, B);
        for (int k = 0; k < 3; ++k) nvec[k] = A[k] - B[k];
        pv->nA = 1; pv->a[0] = i;
        pv->nB = 1; pv->b[0] = j;
    }
    const MeshParams P = sc.prm.get(mesh);
    const R D = sqrt(dot3(nvec, nvec));
    const R phi = D - (R)P.xi;
    if (!(phi < (R)P.two_r)) return false;
    if (D == R(0)) { *degenerate = true; return false; }
    // all five inverse masses at once (unused slots repeat a vertex of the pair)
    pv->wa[0] = sc.inv_mass[pv->a[0]];
    pv->wa[1] = sc.inv_mass[pv->nA > 1 ? pv->a[1] : pv->a[0]];
    pv->wb[0] = sc.inv_mass[pv->b[0]];
    pv->wb[1] = sc.inv_mass[pv->nB > 1 ? pv->b[1] : pv->b[0]];
    pv->wb[2] = sc.inv_mass[pv->nB > 2 ? pv->b[2] : pv->b[0]];
    if (kind == KIND_VF) {
        wA = (R)pv->wa[0];
        wB = bary[0] * (R)pv->wb[0] + bary[1] * (R)pv->wb[1] + bary[2] * (R)pv->wb[2];
    } else if (kind == KIND_EE) {
        wA = (R(1) - s) * (R)pv->wa[0] + s * (R)pv->wa[1];
        wB = (R(1) - t) * (R)pv->wb[0] + t * (R)pv->wb[1];
    } else if (kind == KIND_VE) {
        wA = (R)pv->wa[0];
        wB = (R(1) - t) * (R)pv->wb[0] + t * (R)pv->wb[1];
    } else {
        wA = (R)pv->wa[0];
        wB = (R)pv->wb[0];
    }
    const R wsum = wA + wB;
    if (wsum == R(0)) return false;
    const R inv = R(1) / D;
    for (int k = 0; k < 3; ++k) rec->n[k] = (float)(nvec[k] * inv);
    rec->phi = (float)phi;
    // d = s phi, formed in the working precision and stored
    rec->dA = (float)(wA / wsum * phi);
    rec->dB = (float)(wB / wsum * phi);
    rec->sA = (float)(wA / wsum);
    rec->sB = (float)(wB / wsum);
    rec->pad[0] = rec->pad[1] = 0;
    rec->a = pa | (kind << 30);
    rec->b = pb;
    return true;
}

// A contact's half-spaces into per-vertex slots: every receiving vertex claims
// its next slot of `stride` with one atomic on its count; a vertex that
// receives more than its slots keeps the first ones it got (the largest count
// is reported and the step is repeated with more room).  Counts the
// half-spaces written and the largest slot claimed.
__device__ __forceinline__ void put_slots(const Contact& rec, int32_t* counts, ccfr_halfspace* hs, int32_t stride,
                                          int& n_hs, int& top) {
    const int kind = (int)((uint32_t)rec.a >> 30);
    const int pa = rec.a & 0x3fffffff, pb = rec.b;
    const int nA = kind == KIND_EE ? 2 : 1;     // receiving vertices of side A come first
    int slot[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) slot[k] = rec.rv[k] >= 0 ? atomicAdd(&counts[rec.rv[k]], 1) : 0;
    ccfr_halfspace h;
    h.phi = rec.phi;
    h.key = ((uint64_t)kind << 62) | ((uint64_t)(uint32_t)pa << 31) | (uint64_t)(uint32_t)pb;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (rec.rv[k] < 0) continue;
        const float sg = k < nA ? 1.0f : -1.0f;
        h.n[0] = sg * rec.n[0]; h.n[1] = sg * rec.n[1]; h.n[2] = sg * rec.n[2];
        h.d = k < nA ? rec.dA : rec.dB;
        h.share = k < nA ? rec.sA : rec.sB;
        top = max(top, slot[k] + 1);
        if (slot[k] < stride) {
            hs[(long long)rec.rv[k] * stride + slot[k]] = h;
            ++n_hs;
        }
    }
}

// Block sums of the slot writes (half-spaces written, largest slot, pairs
// kept) added to the counters with one atomic each.  Every thread of the
// block calls it.
__device__ __forceinline__ void flush_slot_counts(DevCounters* c, int n_hs, int top, int n_kept) {
    for (int off = 32; off > 0; off >>= 1) {
        n_hs += __shfl_xor(n_hs, off);
        top = max(top, __shfl_xor(top, off));
        n_kept += __shfl_xor(n_kept, off);
    }
    __shared__ int red[kBlock / 64][3];
    const int wave = threadIdx.x / 64;
    if (__lane_id() == 0) {
        red[wave][0] = n_hs;
        red[wave][1] = top;
        red[wave][2] = n_kept;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int b = 0, t = 0, k = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            b += red[w][0];
            t = max(t, red[w][1]);
            k += red[w][2];
        }
        if (b) atomicAdd(&c->n_hs, b);
        if (t > 0) atomicMax(&c->max_slot, t);
        if (k) atomicAdd(&c->n_contacts, k);
    }
}

template <class R>
__global__ __launch_bounds__(kBlock, 5) void k_contacts(Scene sc, PairLists pl, const int32_t* counts,
                                                     Contact* contacts, int64_t cap_contacts,
                                                     int32_t* vcount, ccfr_halfspace* slot_hs, int32_t slot_stride,
                                                     DevCounters* c, ColourJob job, int job_blocks) {
    if (sc.skip && *sc.skip) return;              // the substep's iterations have ended
    // the first job_blocks blocks run a stretch colour (the pairs read no p)
    if ((int)blockIdx.x < job_blocks) {
        run_colour_job(job, blockIdx.x * kBlock + threadIdx.x);
        return;
    }
    const long long nvf = min((long long)counts[0], (long long)pl.cap_vf);
    const long long nee = min((long long)counts[1], (long long)pl.cap_ee);
    const long long nvv = min((long long)counts[2], (long long)pl.cap_vv);
    const long long nve = min((long long)counts[3], (long long)pl.cap_ve);
    const long long total = nvf + nee + nvv + nve;
    __shared__ int wave_cnt[kWavesPerBlock];
    __shared__ int block_base;
    const bool slots = slot_stride > 0;      // half-spaces straight into per-vertex slots
    int n_degenerate = 0, n_hs = 0, top = 0, n_kept = 0;
    // grid-stride: every thread of the block runs the same number of rounds so
    // that the block-level append sees all of them together
    const long long stride = (long long)(gridDim.x - job_blocks) * kBlock;
    const long long rounds = (total + stride - 1) / stride;
    const long long i0 = (long long)(blockIdx.x - job_blocks) * kBlock + threadIdx.x;
    for (long long rd = 0; rd < rounds; ++rd) {
        const long long i = i0 + rd * stride;
        bool keep = false;
        Contact rec;
        PairVerts pv;
        if (i < total) {
            int kind, pa, pb;
            if (i < nvf) {
                kind = KIND_VF; pa = pl.vf[2 * i]; pb = pl.vf[2 * i + 1];
            } else if (i < nvf + nee) {
                const long long j = i - nvf;
                kind = KIND_EE; pa = pl.ee[2 * j]; pb = pl.ee[2 * j + 1];
            } else if (i < nvf + nee + nvv) {
                const long long j = i - nvf - nee;
                kind = KIND_VV; pa = pl.vv[2 * j]; pb = pl.vv[2 * j + 1];
            } else {
                const long long j = i - nvf - nee - nvv;
                kind = KIND_VE; pa = pl.ve[2 * j]; pb = pl.ve[2 * j + 1];
            }
            bool deg;
            keep = eval_pair<R>(sc, kind, pa, pb, &rec, &pv, &deg);
            if (keep) {
                // the receiving vertices, so that the fill reads no topology or
                // masses: side A's (two for an edge-edge pair, else one), then
                // side B's (three for a face, two for an edge, one for a particle)
                const int a1 = kind == KIND_EE ? pv.a[1] : pv.b[0];
                const float wa1 = kind == KIND_EE ? pv.wa[1] : pv.wb[0];
                const int b0 = kind == KIND_EE ? pv.b[0] : pv.b[1];
                const float wb0 = kind == KIND_EE ? pv.wb[0] : pv.wb[1];
                const int b1 = kind == KIND_EE ? pv.b[1] : pv.b[2];
                const float wb1 = kind == KIND_EE ? pv.wb[1] : pv.wb[2];
                rec.rv[0] = pv.wa[0] > 0.f ? pv.a[0] : -1;
                rec.rv[1] = wa1 > 0.f ? a1 : -1;
                rec.rv[2] = kind != KIND_VV && wb0 > 0.f ? b0 : -1;
                rec.rv[3] = (kind == KIND_VF || kind == KIND_EE) && wb1 > 0.f ? b1 : -1;
            }
            n_degenerate += deg ? 1 : 0;
            if (keep && slots) {
                put_slots(rec, vcount, slot_hs, slot_stride, n_hs, top);
                ++n_kept;
            } else if (keep && vcount) {
                for (int k = 0; k < pv.nA; ++k)
                    if (pv.wa[k] > 0.f) atomicAdd(&vcount[pv.a[k]], 1);
                for (int k = 0; k < pv.nB; ++k)
                    if (pv.wb[k] > 0.f) atomicAdd(&vcount[pv.b[k]], 1);
            }
        }
        if (!slots) block_append(contacts, &c->n_contacts, cap_contacts, rec, keep, wave_cnt, &block_base);
    }
    if (slots) flush_slot_counts(c, n_hs, top, n_kept);
    if (n_degenerate) atomicAdd((unsigned long long*)&c->totals[6], (unsigned long long)n_degenerate);
}

// Inside a substep, unless the narrow phase writes the slots itself: the
// contact list is built as for the CSR (without per-vertex counts), then every
// contact claims the next slot of each receiving vertex (put_slots), so no
// count scan is needed.
__global__ __launch_bounds__(kBlock) void k_fill_slots(Scene sc, const Contact* contacts, int64_t cap_contacts,
                                                       int32_t* counts, ccfr_halfspace* hs, int32_t stride,
                                                       DevCounters* c, ColourJob job, int job_blocks) {
    if (sc.skip && *sc.skip) return;
    if ((int)blockIdx.x < job_blocks) {
        run_colour_job(job, blockIdx.x * kBlock + threadIdx.x);
        return;
    }
    const long long n = min((long long)c->n_contacts, (long long)cap_contacts);
    const long long stride_g = (long long)(gridDim.x - job_blocks) * kBlock;
    int n_hs = 0, top = 0;
    for (long long i = (long long)(blockIdx.x - job_blocks) * kBlock + threadIdx.x; i < n; i += stride_g)
        put_slots(contacts[i], counts, hs, stride, n_hs, top);
    flush_slot_counts(c, n_hs, top, 0);
}

__global__ __launch_bounds__(kBlock) void k_fill(Scene sc, const Contact* contacts, int64_t cap_contacts,
                                                 const int32_t* offsets, int32_t* vcount, ccfr_halfspace* hs,
                                                 int64_t cap_hs, DevCounters* c) {
    if (sc.skip && *sc.skip) return;
    const long long n = min((long long)c->n_contacts, (long long)cap_contacts);
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const Contact rec = contacts[i];
        const int kind = (int)((uint32_t)rec.a >> 30);
        const int pa = rec.a & 0x3fffffff, pb = rec.b;
        const int nA = kind == KIND_EE ? 2 : 1;     // receiving vertices of side A come first
        ccfr_halfspace h;
        h.phi = rec.phi;
        h.key = ((uint64_t)kind << 62) | ((uint64_t)(uint32_t)pa << 31) | (uint64_t)(uint32_t)pb;
        for (int k = 0; k < 4; ++k) {
            const int v = rec.rv[k];
            if (v < 0) continue;
            const float sg = k < nA ? 1.0f : -1.0f;
            const long long pos = (long long)offsets[v] + atomicSub(&vcount[v], 1) - 1;
            h.n[0] = sg * rec.n[0]; h.n[1] = sg * rec.n[1]; h.n[2] = sg * rec.n[2];
            h.d = k < nA ? rec.dA : rec.dB;
            h.share = k < nA ? rec.sA : rec.sB;
            if (pos < cap_hs) hs[pos] = h;
        }
    }
}

__global__ void k_finalize_regions(int32_t n_verts, const int32_t* offsets, int64_t cap_contacts,
                                   int64_t cap_hs, DevCounters* c) {
    if (threadIdx.x == 0) finalize_regions_body(c, n_verts, offsets, cap_contacts, cap_hs);
}

int grid_for(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    return (int)b;
}

}  // namespace

void launch_contacts(const Scene& sc, const PairLists& pl, const int32_t* counts, Contact* contacts,
                     int64_t cap_contacts, int32_t* vcount, DevCounters* c, hipStream_t s, ccfr_halfspace* slot_hs,
                     int32_t slot_stride, const ColourJob* job) {
    ColourJob hosted{};
    if (job) hosted = *job;
    const int jb = colour_job_blocks(hosted, kBlock);
    const int blocks = grid_for(pl.cap_vf + pl.cap_ee + pl.cap_vv + pl.cap_ve) + jb;
    hipLaunchKernelGGL(k_contacts<double>, dim3(blocks), dim3(kBlock), 0, s, sc, pl, counts, contacts, cap_contacts,
                       vcount, slot_stride > 0 ? slot_hs : nullptr, slot_stride > 0 ? slot_stride : 0, c, hosted,
                       jb);
}

void launch_fill_slots(const Scene& sc, const Contact* contacts, int64_t cap_contacts, int32_t* vcount,
                       ccfr_halfspace* slot_hs, int32_t slot_stride, DevCounters* c, hipStream_t s,
                       const ColourJob* job) {
    ColourJob hosted{};
    if (job) hosted = *job;
    const int jb = colour_job_blocks(hosted, kBlock);
    // grid-stride over the contacts: a sixteenth of the capacity's blocks
    hipLaunchKernelGGL(k_fill_slots, dim3(grid_for(cap_contacts / 16) + jb), dim3(kBlock), 0, s, sc, contacts,
                       cap_contacts, vcount, slot_hs, slot_stride, c, hosted, jb);
}

void launch_fill(const Scene& sc, const Contact* contacts, int64_t cap_contacts, const int32_t* offsets,
                 int32_t* vcount, ccfr_halfspace* hs, int64_t cap_hs, DevCounters* c, bool finalize,
                 hipStream_t s) {
    const int blocks = grid_for(cap_contacts);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kBlock), 0, s, sc, contacts, cap_contacts, offsets, vcount, hs,
                       cap_hs, c);
    if (finalize)
        hipLaunchKernelGGL(k_finalize_regions, dim3(1), dim3(64), 0, s, sc.n_verts, offsets, cap_contacts, cap_hs,
                           c);
}

}  // namespace ccfr
