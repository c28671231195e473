// k_response.hip -- applyResponse of Alg. 4: the soft response with
// visibility weights and friction of Sec. 3.3, per vertex on its region,
// between the XPBD constraints and the projection.
//
// The response energy k/2 w_c max(0, delta - d_c)^2 is the XPBD constraint
// C_c = max(0, delta - d_c) with compliance alpha = 1/k.  Constraints are
// owned per vertex (Sec. 3.4), so each vertex is handled on its own, with no
// colouring:
//   d_c = (n_c . y + d_c) / s_c     the pair's gap beyond the offset at the
//                                   proposal y when both sides advance in
//                                   proportion to their shares s (d = s phi)
//   active while d_c < delta; weight w_c = prod over the vertex's other
//   active contacts of 1 - S((d_c - d_j) / delta_v), S the cubic smoothstep
//   innermost contact first (ascending d_c, ties by key): the vertex takes its
//   share of the correction, dn = w (s_c delta - rho_c) / (w + alpha / (w_c dt^2)),
//   along n_c, then friction (Macklin et al. 2014) on the tangential part t
//   of the displacement: removed if |t| < mu_s dn, else shortened by mu_k dn.
// The multiplier starts at zero every iteration (the constraint set is
// rebuilt by every iteration's narrow phase).  The gaps are taken at the
// proposal, so the order and the weights are known before any update.  Only
// contacts within delta_v of the innermost one can have a weight above zero
// (the innermost one's factor for the others is 1 - S(1) = 0), and the factors
// of a contact come from the contacts before it in the order.  Arithmetic in
// FP64 registers from the FP32 region and proposal.
//
// Regions of up to kLaneK half-spaces: one lane, the relevant contacts sorted
// in registers (up to kRel of them).  Larger regions, and regions with more
// relevant contacts, are listed and taken by a wavefront each: the relevant
// contacts sorted in LDS, their weights formed in parallel, then applied in
// order.  (Without a
// list, or beyond the wavefront's 256 entries, one lane walks the region in
// order, finding each next contact by a scan.)
#include "ccfr_internal.h"

namespace ccfr {
namespace {

constexpr int kBlock = 256;
constexpr int kLaneK = 8;          // regions up to this size by one lane
constexpr int kRel = 8;            // relevant contacts a lane sorts in registers
constexpr int kChunks = 4;         // entries per lane of the wavefront path (256 per wavefront)

__device__ __forceinline__ double smoothstep(double t) {
    if (t <= 0.0) return 0.0;
    if (t >= 1.0) return 1.0;
    return t * t * (3.0 - 2.0 * t);
}

struct Plane {
    double n[3];
    double d, share;
    uint64_t key;
};

__device__ __forceinline__ Plane plane_at(const ccfr_halfspace* H, int k) {
    const ccfr_halfspace h = H[k];
    Plane p;
    p.n[0] = h.n[0]; p.n[1] = h.n[1]; p.n[2] = h.n[2];
    p.d = h.d;
    p.share = h.share;
    p.key = h.key;
    return p;
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// gap beyond the offset at the proposal y0, or +inf when the entry does not count
__device__ __forceinline__ double gap_of(const Plane& p, const double y0[3]) {
    if (!(p.share > 0.0)) return __longlong_as_double(0x7ff0000000000000ll);
    return (dot3(p.n, y0) + p.d) / p.share;
}

// Whether a contact at gap d may have a weight above zero: active, and, with
// delta_v > 0, closer than delta_v to the innermost gap d_min (the ratio is
// formed as in the weight, so a contact left out has weight 0).
__device__ __forceinline__ bool relevant(double d, double d_min, double delta, double dv) {
    return d < delta && (dv == 0.0 || (d - d_min) / dv < 1.0);
}

// One contact's update of y: its share of the XPBD correction of the response
// constraint with weight wc, then friction on the tangential part.
__device__ __forceinline__ void apply_contact(const MeshParams& P, double w, double dt, const Plane& p, double wc,
                                              double y[3]) {
    const double delta = P.delta;
    const double rho = dot3(p.n, y) + p.d;
    const double cv = p.share * delta - rho;
    if (!(cv > 0.0)) return;
    const double at = (double)P.resp_compliance / (wc * dt * dt);
    const double dn = w * cv / (w + at);
    for (int k = 0; k < 3; ++k) y[k] += dn * p.n[k];
    if (P.mu_s > 0.0f || P.mu_k > 0.0f) {
        const double yn = dot3(p.n, y);
        const double t[3] = {y[0] - yn * p.n[0], y[1] - yn * p.n[1], y[2] - yn * p.n[2]};
        const double lt = sqrt(dot3(t, t));
        double f = 0.0;
        if (lt < (double)P.mu_s * dn) f = 1.0;
        else if (lt > 0.0) f = fmin((double)P.mu_k * dn / lt, 1.0);
        for (int k = 0; k < 3; ++k) y[k] -= f * t[k];
    }
}

struct Vertex {
    MeshParams P;
    float yf[3];          // the proposal
    double w;
    int K;
    const ccfr_halfspace* H;
    bool idle;            // nothing to do: the proposal is the result
};

__device__ __forceinline__ Vertex vertex_of(const ResponseArgs& a, int v) {
    Vertex x;
    x.P = a.prm.get(a.prm.mesh_of(v));
    for (int k = 0; k < 3; ++k) x.yf[k] = a.y_in ? a.y_in[3 * v + k] : a.p[3 * v + k] - a.x_anchor[3 * v + k];
    x.w = a.inv_mass[v];
    if (a.slot_stride > 0) {
        x.K = min(a.slot_counts[v], a.slot_stride);
        x.H = a.hs + (long long)v * a.slot_stride;
    } else {
        x.K = a.offsets[v + 1] - a.offsets[v];
        x.H = a.hs + a.offsets[v];
    }
    x.idle = !(x.w > 0.0) || !x.P.response || x.K == 0 || !(x.P.delta > 0.0f) ||
             !(isfinite(x.yf[0]) && isfinite(x.yf[1]) && isfinite(x.yf[2]));
    return x;
}

__device__ __forceinline__ void write_out(const ResponseArgs& a, int v, const double y[3]) {
    if (a.y_out) {
        for (int k = 0; k < 3; ++k) a.y_out[3 * v + k] = (float)y[k];
    } else {
        for (int k = 0; k < 3; ++k) a.p[3 * v + k] = a.x_anchor[3 * v + k] + (float)y[k];
    }
}

// The ordered walk over a region: the next active contact in (gap, key) order
// is found again for every step.
__device__ void ordered_walk(const Vertex& x, double dt, const double y0[3], double y[3]) {
    const double delta = x.P.delta, dv = x.P.vis_width;
    double last_d = -__longlong_as_double(0x7ff0000000000000ll);
    uint64_t last_key = 0;
    bool first = true;
    for (;;) {
        int c = -1;
        double dc = 0.0;
        uint64_t kc = 0;
        for (int k = 0; k < x.K; ++k) {
            const Plane p = plane_at(x.H, k);
            const double d = gap_of(p, y0);
            if (!(d < delta)) continue;
            const bool after = first || d > last_d || (d == last_d && p.key > last_key);
            const bool before_best = c < 0 || d < dc || (d == dc && p.key < kc);
            if (after && before_best) {
                c = k;
                dc = d;
                kc = p.key;
            }
        }
        if (c < 0) break;
        first = false;
        last_d = dc;
        last_key = kc;
        double wc = 1.0;
        if (dv > 0.0)
            for (int j = 0; j < x.K; ++j) {
                if (j == c) continue;
                const double dj = gap_of(plane_at(x.H, j), y0);
                if (dj < delta) wc *= 1.0 - smoothstep((dc - dj) / dv);
            }
        if (!(wc > 0.0)) continue;
        apply_contact(x.P, x.w, dt, plane_at(x.H, c), wc, y);
    }
}

__global__ __launch_bounds__(kBlock) void k_response(ResponseArgs a) {
    if (a.skip && *a.skip) return;
    const int v = blockIdx.x * kBlock + threadIdx.x;
    const bool in = v < a.n_verts;
    Vertex x{};
    if (in) x = vertex_of(a, v);
    // large regions go to the wavefront launch (one atomic per wavefront)
    const bool can_list = a.list && a.c;
    const bool listed = in && !x.idle && x.K > kLaneK && can_list;
    const unsigned long long m = __ballot(listed);
    if (m) {
        const int lead = __ffsll((long long)m) - 1;
        int base = 0;
        if (__lane_id() == lead) base = atomicAdd(&a.c->n_resp, __popcll(m));
        base = __shfl(base, lead);
        if (listed) a.list[base + __popcll(m & ((1ull << __lane_id()) - 1ull))] = v;
    }
    if (!in || listed) return;
    if (x.idle) {
        if (a.y_out)
            for (int k = 0; k < 3; ++k) a.y_out[3 * v + k] = x.yf[k];
        return;
    }
    const double y0[3] = {x.yf[0], x.yf[1], x.yf[2]};
    const double delta = x.P.delta, dv = x.P.vis_width, dt = a.dt;
    double y[3] = {y0[0], y0[1], y0[2]};
    double d_min = __longlong_as_double(0x7ff0000000000000ll);
    for (int k = 0; k < x.K; ++k) {
        const double d = gap_of(plane_at(x.H, k), y0);
        if (d < delta) d_min = fmin(d_min, d);
    }
    // the relevant contacts, sorted by (gap, key) in registers (constant
    // indices keep the arrays there)
    double rd[kRel];
    uint64_t rk[kRel];
    int ri[kRel];
    int n_rel = 0;
    bool overflow = false;
    for (int k = 0; k < x.K; ++k) {
        const Plane p = plane_at(x.H, k);
        const double d = gap_of(p, y0);
        if (!relevant(d, d_min, delta, dv)) continue;
        if (n_rel == kRel) {
            overflow = true;
            break;
        }
        int pos = n_rel;
#pragma unroll
        for (int q = kRel - 1; q >= 0; --q)
            if (q < n_rel && (rd[q] > d || (rd[q] == d && rk[q] > p.key))) pos = q;
#pragma unroll
        for (int q = kRel - 1; q > 0; --q)
            if (q > pos && q <= n_rel) {
                rd[q] = rd[q - 1];
                rk[q] = rk[q - 1];
                ri[q] = ri[q - 1];
            }
#pragma unroll
        for (int q = 0; q < kRel; ++q)
            if (q == pos) {
                rd[q] = d;
                rk[q] = p.key;
                ri[q] = k;
            }
        ++n_rel;
    }
    // more relevant contacts than the registers hold: listed for the
    // wavefront launch too (a lane's ordered walk would hold its whole
    // wavefront for the region's K x relevant gap evaluations)
    const unsigned long long mo = __ballot(overflow && can_list);
    if (mo) {
        const int lead = __ffsll((long long)mo) - 1;
        int base = 0;
        if (__lane_id() == lead) base = atomicAdd(&a.c->n_resp, __popcll(mo));
        base = __shfl(base, lead);
        if (overflow) {
            a.list[base + __popcll(mo & ((1ull << __lane_id()) - 1ull))] = v;
            return;
        }
    }
    if (overflow) {
        ordered_walk(x, dt, y0, y);
    } else {
#pragma unroll
        for (int c = 0; c < kRel; ++c) {
            if (c >= n_rel) break;
            // the factors of the contacts before it (equal gaps give 1)
            double wc = 1.0;
            if (dv > 0.0)
#pragma unroll
                for (int j = 0; j < kRel; ++j)
                    if (j < c) wc *= 1.0 - smoothstep((rd[c] - rd[j]) / dv);
            if (!(wc > 0.0)) continue;
            apply_contact(x.P, x.w, dt, plane_at(x.H, ri[c]), wc, y);
        }
    }
    write_out(a, v, y);
}

__device__ __forceinline__ double wave_min(double x) {
    for (int off = 32; off > 0; off >>= 1) x = fmin(x, __shfl_xor(x, off));
    return x;
}

__device__ __forceinline__ double wave_prod(double x) {
    for (int off = 32; off > 0; off >>= 1) x *= __shfl_xor(x, off);
    return x;
}

// A wavefront's LDS for one listed vertex: its relevant contacts in (gap,
// key) order with their region index and weight.
struct RespLds {
    double g[64 * kChunks];
    uint64_t key[64 * kChunks];
    double w[64 * kChunks];
    int16_t idx[64 * kChunks];
};

// Orders the LDS writes and reads of one wavefront.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// One listed vertex by one wavefront (every lane runs it; y is the same on
// all).  The gaps are taken at the proposal, so the order of the relevant
// contacts and every weight are known before any update: the lanes compact
// the relevant contacts into LDS, sort them by (gap, key) with a bitonic
// network, form each contact's weight from the contacts before it (in that
// order, as the lane path does), and then apply them one after the other.
__device__ void response_wave_vertex(const ResponseArgs& a, int v, RespLds* L) {
    const int lane = __lane_id();
    const Vertex x = vertex_of(a, v);
    const double y0[3] = {x.yf[0], x.yf[1], x.yf[2]};
    const double delta = x.P.delta, dv = x.P.vis_width, dt = a.dt;
    double y[3] = {y0[0], y0[1], y0[2]};
    if (x.K > 64 * kChunks) {
        // beyond the wavefront's LDS: one lane walks the region
        if (lane == 0) {
            ordered_walk(x, dt, y0, y);
            write_out(a, v, y);
        }
        return;
    }
    double g[kChunks];
    uint64_t key[kChunks];
    double d_min = __longlong_as_double(0x7ff0000000000000ll);
#pragma unroll
    for (int ch = 0; ch < kChunks; ++ch) {
        const int j = ch * 64 + lane;
        g[ch] = __longlong_as_double(0x7ff0000000000000ll);
        key[ch] = ~0ull;
        if (j < x.K) {
            const Plane p = plane_at(x.H, j);
            g[ch] = gap_of(p, y0);
            key[ch] = p.key;
            if (g[ch] < delta) d_min = fmin(d_min, g[ch]);
        }
    }
    d_min = wave_min(d_min);
    // the relevant contacts, compacted in region order
    int n_rel = 0;
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int ch = 0; ch < kChunks; ++ch) {
        const bool r = ch * 64 + lane < x.K && relevant(g[ch], d_min, delta, dv);
        const unsigned long long m = __ballot(r);
        if (r) {
            const int q = n_rel + __popcll(m & below);
            L->g[q] = g[ch];
            L->key[q] = key[ch];
            L->idx[q] = (int16_t)(ch * 64 + lane);
        }
        n_rel += __popcll(m);
    }
    if (n_rel > 0) {
        int np = 1;
        while (np < n_rel) np <<= 1;
        for (int q = n_rel + lane; q < np; q += 64) {
            L->g[q] = __longlong_as_double(0x7ff0000000000000ll);   // +inf: sorts last
            L->key[q] = ~0ull;
            L->idx[q] = 0;
        }
        wave_sync();
        for (int size = 2; size <= np; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = lane; t < (np >> 1); t += 64) {
                    const int p = 2 * t - (t & (stride - 1));
                    const int q = p + stride;
                    const bool up = (p & size) == 0;
                    const double gp = L->g[p], gq = L->g[q];
                    const uint64_t kp = L->key[p], kq = L->key[q];
                    const bool q_first = gq < gp || (gq == gp && kq < kp);
                    if (up ? q_first : !q_first) {
                        L->g[p] = gq; L->g[q] = gp;
                        L->key[p] = kq; L->key[q] = kp;
                        const int16_t ti = L->idx[p]; L->idx[p] = L->idx[q]; L->idx[q] = ti;
                    }
                }
                wave_sync();
            }
        }
        // each contact's weight: the factors of the contacts before it
        for (int c = lane; c < n_rel; c += 64) {
            double wc = 1.0;
            if (dv > 0.0) {
                const double gc = L->g[c];
                for (int j = 0; j < c; ++j) wc *= 1.0 - smoothstep((gc - L->g[j]) / dv);
            }
            L->w[c] = wc;
        }
        wave_sync();
        for (int c = 0; c < n_rel; ++c) {
            const double wc = L->w[c];
            if (wc > 0.0) apply_contact(x.P, x.w, dt, plane_at(x.H, L->idx[c]), wc, y);
        }
    }
    if (lane == 0) write_out(a, v, y);
    wave_sync();   // the LDS is reused by the wavefront's next vertex
}

__global__ __launch_bounds__(kBlock) void k_response_waves(ResponseArgs a, int waves) {
    if (a.skip && *a.skip) return;
    __shared__ RespLds lds[kBlock / 64];
    const int n = a.c->n_resp;
    for (int i = blockIdx.x * (kBlock / 64) + threadIdx.x / 64; i < n; i += waves)
        response_wave_vertex(a, a.list[i], &lds[threadIdx.x / 64]);
}

__global__ void k_response_clear(DevCounters* c, const uint32_t* skip) {
    if (skip && *skip) return;
    if (threadIdx.x == 0) c->n_resp = 0;
}

}  // namespace

void launch_response(const ResponseArgs& a, hipStream_t s) {
    if (a.n_verts <= 0) return;
    hipLaunchKernelGGL(k_response, dim3((a.n_verts + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
    if (!a.list || !a.c) return;
    // the list's length is known on the device only: a wavefront per 64
    // vertices, at most 4096, which take the listed vertices in turn
    const int blocks = std::max(1, std::min(1024, (a.n_verts + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_response_waves, dim3(blocks), dim3(kBlock), 0, s, a, blocks * (kBlock / 64));
    hipLaunchKernelGGL(k_response_clear, dim3(1), dim3(64), 0, s, a.c, a.skip);
}

}  // namespace ccfr
