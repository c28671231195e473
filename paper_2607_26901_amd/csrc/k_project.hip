// k_project.hip -- projection of proposed displacements onto the vertex regions
// (Alg. 2 calling Alg. 1, the retraction and halt fallback of Sec. 3.2, and the
// r-ball clamp of Alg. 4) on gfx950.
//
// Region data stays FP32 in HBM; the arithmetic of the
// projection runs in FP64 registers, working in displacement coordinates (the
// anchor is the origin, so a constraint n . x' >= b with b = n . x - d reads
// n . y + d >= 0).  This removes the cancellation of world coordinates, which
// is what makes the sign tests of Alg. 2 fragile in single precision (the
// paper's Sec. 5 names single-precision robustness as open).
//
// Fast kernel (every vertex): a vertex none of whose half-spaces is violated by
// its proposal returns it unchanged (Alg. 2 with no violation in its first
// pass); a vertex with exactly one violated half-space whose projection leaves
// every other one satisfied returns that projection (the first two passes of
// Alg. 2, which need no sort in that case).  All other vertices are compacted
// into lists for the slow kernel: their half-spaces are sorted by initial rho
// ascending, ties by key (by one lane in registers up to 8; up to 32 by one
// lane, (rho, index) in registers and the records gathered in sorted order,
// when the listed vertices outnumber the wavefronts, else by a wavefront; by
// a wavefront in LDS up to 256 and in a scratch range parallel to the region
// beyond), exact duplicates (bitwise-equal n and d) are dropped, then up to
// max_passes passes of Alg. 1 over the violated ones, each followed by the
// retraction by eps; a pass without violation returns its start point, and
// otherwise the vertex halts at y = 0.  Every path takes the same arithmetic
// in the same order, so a vertex's result does not depend on the path.
//
// Readings of the paper taken here: Alg. 1's entry j = m is the new plane, and
// the stored plane is that plane; Alg. 1 returns its input once three planes
// are stored; max_passes is the literal loop count; the clamp also applies
// without half-spaces, and zero inverse mass gives y = 0.
#include "ccfr_internal.h"

#include <algorithm>

namespace ccfr {

namespace {

constexpr int kBlock = 256;
constexpr int kSmall = 8;      // regions up to this size stay in registers
constexpr int kMid = 32;       // up to this size a violated region is projected by one lane
constexpr int kScan = 32;      // up to this size the fast kernel checks for a violation
constexpr int kWave = 256;     // up to this size a wavefront sorts them in LDS

struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 mk(double a, double b, double c) { return d3{a, b, c}; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ d3 operator*(double s, d3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ double norm(d3 a) { return sqrt(dot(a, a)); }

// Plesnik state of Alg. 1: up to three stored planes (A, B) and ERO directions V.
struct Ero {
    int m;
    d3 V0, V1, V2;
    d3 A0, A1, A2;
    double B0, B1, B2;
};

// Alg. 1: add plane n . y = b, move yt to the orthogonal projection of y0 onto
// the intersection of all stored planes.
__device__ void orthogonal_projection(d3& yt, const d3 y0, const d3 n, const double b, Ero& S,
                                      const double eps) {
    if (S.m == 0) {
        const d3 v0 = n;
        const double beta0 = dot(n, v0);
        if (fabs(beta0) < eps) return;
        yt = yt + ((b - dot(n, yt)) / beta0) * v0;
        S.V0 = v0; S.A0 = n; S.B0 = b; S.m = 1;
        return;
    }
    if (S.m == 3) return;
    const int m = S.m;
    const d3 n0 = S.A0;
    const double b0 = S.B0;
    const d3 Vlast = (m == 1) ? S.V0 : S.V1;
    const d3 dn = n - n0;
    const double beta_u = dot(dn, Vlast);
    const double alpha_u = b - dot(n, yt);
    if (fabs(beta_u) < eps) return;
    const d3 u = yt + (alpha_u / beta_u) * Vlast;
    d3 w = y0 + n;
    {   // j = 1: plane A1 if stored, else the new one; direction V0
        const d3 n1 = (m > 1) ? S.A1 : n;
        const double b1 = (m > 1) ? S.B1 : b;
        const d3 dn1 = n1 - n0;
        const double beta_w = dot(dn1, S.V0);
        if (fabs(beta_w) > eps) w = w + ((b1 - b0 - dot(dn1, w)) / beta_w) * S.V0;
    }
    if (m == 2) {   // j = 2: the new plane; direction V1
        const double beta_w = dot(dn, S.V1);
        if (fabs(beta_w) > eps) w = w + ((b - b0 - dot(dn, w)) / beta_w) * S.V1;
    }
    const d3 vnew = w - u;
    if (norm(vnew) > eps) {
        const double beta_new = dot(n0, vnew);
        if (fabs(beta_new) < eps) {
            yt = u;
        } else {
            yt = u + ((b0 - dot(n0, u)) / beta_new) * vnew;
        }
        if (m == 1) { S.V1 = vnew; S.A1 = n; S.B1 = b; }
        else { S.V2 = vnew; S.A2 = n; S.B2 = b; }
        S.m = m + 1;
    }
}

__device__ __forceinline__ d3 load_n(const ccfr_halfspace& h) { return mk(h.n[0], h.n[1], h.n[2]); }

__device__ __forceinline__ bool same_plane(const ccfr_halfspace& a, const ccfr_halfspace& b) {
    return a.n[0] == b.n[0] && a.n[1] == b.n[1] && a.n[2] == b.n[2] && a.d == b.d;
}

__device__ __forceinline__ double rho_of(const ccfr_halfspace& h, const d3 y) {
    return dot(load_n(h), y) + (double)h.d;
}

// Orders one wavefront's global-memory writes before its later reads (all of
// its lanes run together; the workgroup's L1 serves them all).
__device__ __forceinline__ void scratch_sync() {
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int orig_index(int i) { return i < 0 ? -1 - i : i; }

// Alg. 2 for a region larger than a wavefront's LDS holds, by the 64 lanes of
// one wavefront in the scratch range parallel to the region (skey, sidx).
// (rho, index) pairs are sorted by (rho, key) with a bitonic network in the
// form whose comparators all put the smaller element first (each merge opens
// with a comparison of mirrored positions), so entries beyond K, taken as
// +inf, never move and the range needs no padding; exact duplicates after the
// first of their rho run get a negative index; the passes advance by ballots
// over 64 sorted entries at a time, visiting exactly the half-spaces the
// sequential pass of run_passes would, in the same order, with the same
// arithmetic (its scalar tail once three planes are stored included).
// Returns true (on every lane) if the vertex halted.
__device__ bool project_slow(const ccfr_halfspace* H, int K, const d3 yprop, const MeshParams& P,
                             double* skey, int32_t* sidx, d3& yres) {
    const int lane = __lane_id();
    for (int j = lane; j < K; j += 64) {
        skey[j] = rho_of(H[j], yprop);
        sidx[j] = j;
    }
    scratch_sync();
    int Kp = 1;
    while (Kp < K) Kp <<= 1;
    for (int size = 2; size <= Kp; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < (Kp >> 1); t += 64) {
                const int p = 2 * t - (t & (stride - 1));              // bit `stride` of p is clear
                const int q = stride == (size >> 1) ? (p ^ (size - 1)) : (p | stride);
                if (q >= K) continue;
                const double rp = skey[p], rq = skey[q];
                bool sw = rq < rp;
                const int ip = sidx[p], iq = sidx[q];
                if (rq == rp) sw = H[iq].key < H[ip].key;
                if (sw) {
                    skey[p] = rq; skey[q] = rp;
                    sidx[p] = iq; sidx[q] = ip;
                }
            }
            scratch_sync();
        }
    }
    // exact duplicates share rho, so they sit in one run; 64 entries per lane
    // at a time are checked against the earlier entries of their run, then marked
    for (int seg = 0; seg < K; seg += 64 * 64) {
        uint64_t dropm = 0ull;
        for (int k = 0; k < 64; ++k) {
            const int q = seg + 64 * k + lane;
            if (q >= K) break;
            if (q == 0 || skey[q - 1] != skey[q]) continue;
            const ccfr_halfspace hq = H[orig_index(sidx[q])];
            for (int r = q - 1; r >= 0 && skey[r] == skey[q]; --r)
                if (same_plane(H[orig_index(sidx[r])], hq)) {
                    dropm |= 1ull << k;
                    break;
                }
        }
        scratch_sync();
        for (int k = 0; k < 64; ++k)
            if ((dropm >> k) & 1ull) {
                const int q = seg + 64 * k + lane;
                sidx[q] = -1 - sidx[q];
            }
        scratch_sync();
    }
    const double eps_r = (double)P.eps_retract;
    const double eps_p = (double)P.eps_plesnik;
    d3 yp = yprop;
    for (int pass = 0; pass < P.max_passes; ++pass) {
        d3 yt = yp;
        const d3 y0 = yp;
        Ero S;
        S.m = 0;
        int nviol = 0;
        int from = 0;
        while (true) {
            // lowest violated entry at or after `from`, at the current point
            int hit = -1;
            for (int base = from & ~63; base < K; base += 64) {
                const int q = base + lane;
                bool viol = false;
                if (q >= from && q < K) {
                    const int idx = sidx[q];
                    viol = idx >= 0 && rho_of(H[idx], yt) < 0.0;
                }
                const unsigned long long m = __ballot(viol);
                if (m) {
                    hit = base + __ffsll((long long)m) - 1;
                    break;
                }
            }
            if (hit < 0) break;
            const ccfr_halfspace h = H[sidx[hit]];
            ++nviol;
            orthogonal_projection(yt, y0, load_n(h), -(double)h.d, S, eps_p);
            const double nd = norm(yt);
            yt = (nd > eps_r) ? ((nd - eps_r) / nd) * yt : mk(0.0, 0.0, 0.0);
            from = hit + 1;
            if (S.m == 3) {
                // the rest of the pass on the scalar length, as in run_passes
                double lam = norm(yt);
                const d3 u = lam > 0.0 ? (1.0 / lam) * yt : mk(0.0, 0.0, 0.0);
                while (true) {
                    int hit2 = -1;
                    for (int base = from & ~63; base < K; base += 64) {
                        const int q = base + lane;
                        bool viol = false;
                        if (q >= from && q < K) {
                            const int idx = sidx[q];
                            if (idx >= 0) {
                                const ccfr_halfspace hq = H[idx];
                                const double au = dot(load_n(hq), u);
                                viol = lam * au + (double)hq.d < 0.0;
                            }
                        }
                        const unsigned long long m = __ballot(viol);
                        if (m) {
                            hit2 = base + __ffsll((long long)m) - 1;
                            break;
                        }
                    }
                    if (hit2 < 0) break;
                    ++nviol;
                    lam = lam > eps_r ? lam - eps_r : 0.0;
                    from = hit2 + 1;
                }
                yt = lam * u;
                break;
            }
        }
        if (nviol == 0) {
            yres = yp;
            return false;
        }
        yp = yt;
    }
    yres = mk(0.0, 0.0, 0.0);
    return true;
}

// ---- shared per-vertex plumbing ----

// One endpoint's side of an edge's XPBD distance update (Macklin et al.
// 2016) in a folded colour: x is the vertex, m its map entry (edge, with bit 31
// set when x is the second endpoint; partner), px and po the positions of x
// and its partner before the colour.  The arithmetic is that of a colour
// launch, so both endpoints take the same step; the first one stores the
// multiplier when write_lambda.
__device__ __forceinline__ void edge_side(const ProjectArgs& a, int2 m, int x, const float px[3], const float po[3],
                                          float out[3], bool write_lambda) {
    for (int k = 0; k < 3; ++k) out[k] = px[k];
    if (m.y < 0) return;
    const bool second = m.x < 0;
    const int e = m.x & 0x7fffffff;
    const int i = second ? m.y : x, j = second ? x : m.y;
    const float wi = a.inv_mass[i], wj = a.inv_mass[j];
    const float W = wi + wj;
    float pi[3], pj[3], d[3];
    for (int k = 0; k < 3; ++k) {
        pi[k] = second ? po[k] : px[k];
        pj[k] = second ? px[k] : po[k];
        d[k] = pi[k] - pj[k];
    }
    const float len = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const float lam = a.sl.lambda_in[e];
    if (W == 0.0f || len == 0.0f) {
        if (write_lambda && !second) a.sl.lambda_out[e] = lam;
        return;
    }
    const float C = len - a.sl.rest_sorted[e];
    const float dl = (-C - a.sl.alpha_t * lam) / (W + a.sl.alpha_t);
    const float s = dl / len;
    if (!second) {
        for (int k = 0; k < 3; ++k) out[k] = pi[k] + wi * s * d[k];
        if (write_lambda) a.sl.lambda_out[e] = lam + dl;
    } else {
        for (int k = 0; k < 3; ++k) out[k] = pj[k] - wj * s * d[k];
    }
}

// Vertex v's position after the folded colours: the last one, and, with
// prev_edge, the one before it.  p is not written during the projection, so
// v's update of an edge and its partner's agree.  With two colours v needs
// its own and its last-colour partner's positions after the earlier colour;
// both come out of the same instructions (a loop that is not unrolled), so
// that v and the partner, each computing both, use the same values.
__device__ __forceinline__ void folded_position(const ProjectArgs& a, int v, float pv[3], bool write_lambda) {
    const int2 m = a.sl.last_edge[v];
    const int b = m.y >= 0 ? m.y : v;
    float q0[3], q1[3];
    if (a.sl.prev_edge) {
#pragma unroll 1
        for (int r = 0; r < 2; ++r) {
            const int x = r == 0 ? v : b;
            const int2 mp = a.sl.prev_edge[x];
            float px[3], po[3], out[3];
            for (int k = 0; k < 3; ++k) {
                px[k] = a.p[3 * x + k];
                po[k] = a.p[3 * (mp.y >= 0 ? mp.y : x) + k];
            }
            edge_side(a, mp, x, px, po, out, write_lambda && r == 0);
            for (int k = 0; k < 3; ++k) {
                if (r == 0) q0[k] = out[k];
                else q1[k] = out[k];
            }
        }
    } else {
        for (int k = 0; k < 3; ++k) {
            q0[k] = a.p[3 * v + k];
            q1[k] = a.p[3 * b + k];
        }
    }
    edge_side(a, m, v, q0, q1, pv, write_lambda);
}

__device__ __forceinline__ d3 load_prop(const ProjectArgs& a, int v) {
    float yf[3];
    if (a.y_in) {
        yf[0] = a.y_in[3 * v]; yf[1] = a.y_in[3 * v + 1]; yf[2] = a.y_in[3 * v + 2];
    } else {
        if (a.sl.last_edge) {
            // a deferred vertex: the fast kernel left its displacement
            for (int k = 0; k < 3; ++k) yf[k] = a.sl.y_def[3 * v + k];
        } else {
            for (int k = 0; k < 3; ++k) yf[k] = a.p[3 * v + k] - a.x_anchor[3 * v + k];
        }
    }
    return mk(yf[0], yf[1], yf[2]);
}

// The first read of every vertex's proposal (zero for a pinned vertex); with
// the folded colour it also stores the colour's multipliers, for pinned
// endpoints too.
__device__ __forceinline__ d3 load_prop_first(const ProjectArgs& a, int v) {
    if (a.y_in || !a.sl.last_edge) return a.inv_mass[v] > 0.0f ? load_prop(a, v) : mk(0.0, 0.0, 0.0);
    float pv[3];
    folded_position(a, v, pv, true);
    if (!(a.inv_mass[v] > 0.0f)) return mk(0.0, 0.0, 0.0);
    float yf[3];
    for (int k = 0; k < 3; ++k) yf[k] = pv[k] - a.x_anchor[3 * v + k];
    return mk(yf[0], yf[1], yf[2]);
}

// Writes the clamped displacement (or adds it to the anchor) and returns the
// largest coordinate move of the anchor, exact in FP64 and rounded up to FP32
// (0 when the anchor is not updated).  With a.shortfall_max, sf takes the
// larger of itself and the vertex's shortfall nprop - |y| (nprop = |proposal|,
// 0 for a vertex that does not count); with a.halt_run, the vertex's run of
// consecutive halts grows or ends, and runs of 2 and more are tallied.
__device__ __forceinline__ float write_result(const ProjectArgs& a, DevCounters* c, int v, d3 y, double r,
                                              bool halted, double nprop, float& sf) {
    const double ny = norm(y);
    if (ny > r) y = (r / ny) * y;                      // r-ball clamp
    if (a.shortfall_max && nprop > 0.0) {
        const double f = nprop - fmin(ny, r);
        float ff = (float)f;
        if ((double)ff < f) ff = __int_as_float(__float_as_int(ff) + 1);
        sf = fmaxf(sf, ff);
    }
    if (a.halt_run) {
        const int prev = a.halt_run[v];
        const int run = halted ? min(prev + 1, 255) : 0;
        if (run != prev) a.halt_run[v] = (uint8_t)run;
        if (run >= 2) {
            atomicAdd((unsigned long long*)&c->halt_runs[run >= 3 ? 1 : 0], 1ull);
            atomicMax(&c->max_halt_run, run);
        }
    }
    float move = 0.0f;
    if (a.y_out) {
        a.y_out[3 * v] = (float)y.x;
        a.y_out[3 * v + 1] = (float)y.y;
        a.y_out[3 * v + 2] = (float)y.z;
    } else {
        const float y3[3] = {(float)y.x, (float)y.y, (float)y.z};
        double m = 0.0;
        for (int k = 0; k < 3; ++k) {
            const float o = a.x_anchor[3 * v + k];
            const float n = o + y3[k];
            a.x_anchor[3 * v + k] = n;
            m = fmax(m, fabs((double)n - (double)o));    // the difference of two floats: exact
        }
        move = (float)m;
        if ((double)move < m) move = __int_as_float(__float_as_int(move) + 1);
    }
    if (a.halted) a.halted[v] = halted ? 1 : 0;
    return move;
}

__device__ __forceinline__ float wave_max(float x) {
    for (int off = 32; off > 0; off >>= 1) x = fmaxf(x, __shfl_xor(x, off));
    return x;
}

// A wavefront's maximum into its block's slot of a launch-wide maximum of
// non-negative floats (which order like their bit patterns).  A slot only
// grows during a launch, so a wavefront whose value the slot already holds or
// exceeds writes nothing.
__device__ __forceinline__ void max_into(uint32_t* slots, float m) {
    if (__lane_id() != 0 || !(m > 0.0f)) return;
    uint32_t* word = slots + 32 * (blockIdx.x & 63);
    const uint32_t bits = __float_as_uint(m);
    if (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < bits) atomicMax(word, bits);
}

// Largest shortfall of a wavefront's vertices into the launch-wide maximum.
__device__ __forceinline__ void record_shortfall(const ProjectArgs& a, float sf) {
    if (!a.shortfall_max) return;
    max_into(a.shortfall_max, wave_max(sf));
}

// Largest move of a wavefront's lanes into the device maximum.
__device__ __forceinline__ void record_motion(const ProjectArgs& a, float move) {
    if (!a.motion_max) return;
    max_into(a.motion_max, wave_max(move));
}

// The vertex's CSR range, clipped to the half-space buffer (an offset outside
// it yields an empty region, never an access outside the buffer); or its slots.
__device__ __forceinline__ void slots_consumed(const ProjectArgs& a, int v) {
    if (a.slot_stride > 0) a.slot_counts[v] = 0;     // clear for the next region build
}

__device__ __forceinline__ int region_size(const ProjectArgs& a, int v, long long* o0) {
    if (a.slot_stride > 0) {
        *o0 = (long long)v * a.slot_stride;
        return min(a.slot_counts[v], a.slot_stride);
    }
    const long long lo = a.offsets[v];
    const long long o1 = min((long long)a.offsets[v + 1], (long long)a.cap_hs);
    *o0 = (lo < 0 || lo > a.cap_hs) ? 0 : lo;
    return (lo >= 0 && o1 > lo) ? (int)(o1 - lo) : 0;
}

// Alg. 2's passes over a sorted, de-duplicated sequence: entry q of K gives a
// plane (n, d) or is skipped (get is asked for 0, 1, ..., K - 1 in order in
// every pass).  Once Alg. 1 holds three planes it returns its input for the
// rest of the pass, so every further violation only retracts: yt = lam u
// keeps its direction and loses eps in length, and rho of an entry is
// lam (n . u) + d.  The rest of the pass runs on the scalar lam (the result
// differs from rescaling yt step by step by rounding only); every path of the
// projection takes this same step, so a vertex's result does not depend on
// which path takes it.  Returns true if the vertex halted.
template <class Get>
__device__ __forceinline__ bool run_passes(int K, const Get& get, const d3 yprop, const MeshParams& P, d3& yres) {
    const double eps_r = (double)P.eps_retract;
    const double eps_p = (double)P.eps_plesnik;
    d3 yp = yprop;
    for (int pass = 0; pass < P.max_passes; ++pass) {
        d3 yt = yp;
        const d3 y0 = yp;
        Ero S;
        S.m = 0;
        int nviol = 0;
        for (int q = 0; q < K; ++q) {
            d3 n;
            double d;
            if (!get(q, n, d)) continue;
            if (dot(n, yt) + d >= 0.0) continue;
            ++nviol;
            orthogonal_projection(yt, y0, n, -d, S, eps_p);
            const double nd = norm(yt);
            yt = (nd > eps_r) ? ((nd - eps_r) / nd) * yt : mk(0.0, 0.0, 0.0);
            if (S.m == 3) {
                double lam = norm(yt);
                const d3 u = lam > 0.0 ? (1.0 / lam) * yt : mk(0.0, 0.0, 0.0);
                for (int q2 = q + 1; q2 < K; ++q2) {
                    if (!get(q2, n, d)) continue;
                    const double au = dot(n, u);
                    if (lam * au + d < 0.0) {
                        ++nviol;
                        lam = lam > eps_r ? lam - eps_r : 0.0;
                    }
                }
                yt = lam * u;
                break;
            }
        }
        if (nviol == 0) {
            yres = yp;
            return false;
        }
        yp = yt;
    }
    yres = mk(0.0, 0.0, 0.0);
    return true;
}

// ---- fast path: every vertex; the ones with a violated half-space go to a list ----

__device__ __forceinline__ float4 load_plane(const ccfr_halfspace* h) {
    return *reinterpret_cast<const float4*>(h);          // n[3], d: the first 16 bytes
}

__device__ __forceinline__ double rho_at(const float4 r, const d3 y) {
    return dot(mk(r.x, r.y, r.z), y) + (double)r.w;
}

// One violated half-space: it is first in Alg. 2's sorted order, so the first
// pass projects onto it (Alg. 1 with no stored plane), retracts, and re-checks
// every other half-space at the new point; if none is violated there, the
// second pass finds nothing and returns that point.  Evaluated here with the
// same arithmetic as the passes, this gives Alg. 2's result without the sort;
// returns false when the shortcut does not apply.
__device__ __forceinline__ bool one_plane_regs(const float4 (&R)[kSmall], int K, const float4 hv, const d3 yprop,
                                               const MeshParams& P, d3& yres) {
    if (P.max_passes < 2) return false;
    const d3 n = mk(hv.x, hv.y, hv.z);
    const double beta0 = dot(n, n);
    if (fabs(beta0) < (double)P.eps_plesnik) return false;
    d3 yt = yprop + ((-(double)hv.w - dot(n, yprop)) / beta0) * n;
    const double nd = norm(yt);
    const double eps_r = (double)P.eps_retract;
    yt = (nd > eps_r) ? ((nd - eps_r) / nd) * yt : mk(0.0, 0.0, 0.0);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < kSmall; ++k)
        if (k < K) ok = ok && !(rho_at(R[k], yt) < 0.0);
    if (ok) yres = yt;
    return ok;
}

// Regions of at most kSmall half-spaces are read into registers (independent
// loads, 16 bytes each); up to kScan the lane only checks for a violated one
// (none: done); larger ones go to the wavefront path unexamined, so that no
// lane walks a long region while the rest of its wavefront waits.
__global__ __launch_bounds__(kBlock) void k_project_fast(ProjectArgs a, DevCounters* c) {
    if (a.skip && *a.skip) return;                 // the substep's iterations have ended
    const int v = blockIdx.x * kBlock + threadIdx.x;
    const bool active = v < a.n_verts;
    bool violated = false, deferred = false, big = false, mid = false, moved = false, bad = false;
    float move = 0.0f, sf = 0.0f;
    d3 ykeep = mk(0.0, 0.0, 0.0);
    if (active) {
        const d3 yprop = load_prop_first(a, v);
        ykeep = yprop;
        bad = !(isfinite(yprop.x) && isfinite(yprop.y) && isfinite(yprop.z));
        if (bad) {
            // a non-finite proposal is not moved and raises the status bit
            move = write_result(a, c, v, mk(0.0, 0.0, 0.0), 0.0, true, 0.0, sf);
        } else if (a.inv_mass[v] > 0.0f) {
            moved = true;
            const MeshParams P = a.prm.get(a.prm.mesh_of(v));
            long long o0;
            const int K = region_size(a, v, &o0);
            const ccfr_halfspace* H = a.hs + o0;
            big = K > kSmall;
            if (K > kScan) {
                deferred = true;                 // checked and counted by the wavefront path
            } else if (big) {
                // a mid-size region: no violated half-space finishes it here
                // (Alg. 2's first pass returns the proposal); else the
                // wavefront path takes it (and counts it)
                bool any = false;
                for (int k0 = 0; k0 < K; k0 += 4) {
                    float4 R4[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) R4[k] = k0 + k < K ? load_plane(H + k0 + k) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                    for (int k = 0; k < 4; ++k) any = any || (k0 + k < K && rho_at(R4[k], yprop) < 0.0);
                }
                deferred = any;
                mid = any && K <= kMid;          // one lane of the slow kernel takes it
                if (!deferred) move = write_result(a, c, v, yprop, (double)P.r, false, norm(yprop), sf);
            } else {
                float4 R[kSmall];
#pragma unroll
                for (int k = 0; k < kSmall; ++k)
                    R[k] = k < K ? load_plane(H + k) : make_float4(0.f, 0.f, 0.f, 0.f);
                int n_viol = 0;
                float4 hv = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int k = 0; k < kSmall; ++k) {
                    const bool vk = k < K && rho_at(R[k], yprop) < 0.0;
                    n_viol += vk ? 1 : 0;
                    if (vk) hv = R[k];
                }
                violated = n_viol > 0;
                d3 y = yprop;
                if (n_viol == 1) deferred = !one_plane_regs(R, K, hv, yprop, P, y);
                else deferred = n_viol > 1;
                if (!deferred) move = write_result(a, c, v, y, (double)P.r, false, norm(yprop), sf);
            }
        } else {
            move = write_result(a, c, v, mk(0.0, 0.0, 0.0), 0.0, false, 0.0, sf);
        }
    }
    if (active && !deferred) slots_consumed(a, v);
    if (deferred && a.sl.last_edge && !a.y_in)
    {
        a.sl.y_def[3 * v] = (float)ykeep.x;         // exact: the values came from floats
        a.sl.y_def[3 * v + 1] = (float)ykeep.y;
        a.sl.y_def[3 * v + 2] = (float)ykeep.z;
    }
    record_motion(a, move);
    record_shortfall(a, sf);
    // vertices that need the full Alg. 2 go to the slow lists, one atomic per
    // block and list: small regions from the front of the first half, large
    // ones from its back, mid-size ones into the second half (the slow kernel
    // counts the violating vertices of the two latter lists).
    const unsigned long long md = __ballot(deferred && !big);
    const unsigned long long mb = __ballot(deferred && big && !mid);
    const unsigned long long mi = __ballot(mid);
    const unsigned long long mv = __ballot(violated);
    const unsigned long long mm = __ballot(moved);
    const int lane = __lane_id();
    if (__ballot(bad) && lane == 0) atomicOr(&c->status, ST_NONFINITE);
    const int wave = threadIdx.x / 64;
    constexpr int kW = kBlock / 64;
    __shared__ int pre[kW][3];
    __shared__ int tally[kW][2];
    __shared__ int bases[3];
    if (lane == 0) {
        pre[wave][0] = __popcll(md);
        pre[wave][1] = __popcll(mb);
        pre[wave][2] = __popcll(mi);
        tally[wave][0] = __popcll(mv);
        tally[wave][1] = __popcll(mm);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc[3] = {0, 0, 0}, nv = 0, nm = 0;
        for (int w = 0; w < kW; ++w) {
            for (int l = 0; l < 3; ++l) {
                const int t = pre[w][l];
                pre[w][l] = acc[l];
                acc[l] += t;
            }
            nv += tally[w][0];
            nm += tally[w][1];
        }
        bases[0] = acc[0] ? atomicAdd(&c->n_viol, acc[0]) : 0;
        bases[1] = acc[1] ? atomicAdd(&c->n_viol_b, acc[1]) : 0;
        bases[2] = acc[2] ? atomicAdd(&c->n_viol_m, acc[2]) : 0;
        if (nv) spread_add(c, 0, (unsigned long long)nv);
        if (nm) spread_add(c, 2, (unsigned long long)nm);
    }
    __syncthreads();
    const unsigned long long lt = (1ull << lane) - 1ull;
    if (deferred && !big) a.slow_list[bases[0] + pre[wave][0] + __popcll(md & lt)] = v;
    if (deferred && big && !mid) a.slow_list[a.n_verts - 1 - (bases[1] + pre[wave][1] + __popcll(mb & lt))] = v;
    if (mid) a.slow_list[a.n_verts + bases[2] + pre[wave][2] + __popcll(mi & lt)] = v;
}

// ---- slow path: one lane per listed vertex; bigger regions cooperatively ----


__device__ __forceinline__ bool before(double ra, uint64_t ka, double rb, uint64_t kb) {
    return ra < rb || (ra == rb && ka < kb);
}

// compare-exchange of slots i < j of the register sort
#define CE(i, j)                                                                   \
    if (before(rho[j], key[j], rho[i], key[i])) {                                  \
        double tr = rho[i]; rho[i] = rho[j]; rho[j] = tr;                           \
        uint64_t tk = key[i]; key[i] = key[j]; key[j] = tk;                         \
        float4 tn = R[i]; R[i] = R[j]; R[j] = tn;                                   \
    }

// A region of at most 8 half-spaces projected by one lane: the records in
// registers (every index a constant after unrolling), sorted by (rho, key)
// with Batcher's odd-even merge sort, exact duplicates after the first of
// their rho run dropped, then Alg. 2's passes.
__device__ bool project_small(const ccfr_halfspace* H, int K, const d3 yprop, const MeshParams& P, d3& yres) {
    float4 R[kSmall];
    uint64_t key[kSmall];
    double rho[kSmall];
#pragma unroll
    for (int j = 0; j < kSmall; ++j) {
        if (j < K) {
            const ccfr_halfspace h = H[j];
            R[j] = make_float4(h.n[0], h.n[1], h.n[2], h.d);
            key[j] = h.key;
            rho[j] = dot(load_n(h), yprop) + (double)h.d;
        } else {
            R[j] = make_float4(0.f, 0.f, 0.f, 0.f);
            key[j] = ~0ull;
            rho[j] = __longlong_as_double(0x7ff0000000000000ll);   // +inf: sorts last
        }
    }
    // Batcher's odd-even merge sort of 8 by (rho, key)
    CE(0, 1) CE(2, 3) CE(4, 5) CE(6, 7)
    CE(0, 2) CE(1, 3) CE(4, 6) CE(5, 7)
    CE(1, 2) CE(5, 6)
    CE(0, 4) CE(1, 5) CE(2, 6) CE(3, 7)
    CE(2, 4) CE(3, 5)
    CE(1, 2) CE(3, 4) CE(5, 6)
    // exact duplicates (same rho, bitwise-equal n and d) after the first are dropped
    bool drop[kSmall];
#pragma unroll
    for (int j = 0; j < kSmall; ++j) {
        drop[j] = false;
#pragma unroll
        for (int i = 0; i < j; ++i)
            drop[j] = drop[j] || (rho[i] == rho[j] && R[i].x == R[j].x && R[i].y == R[j].y && R[i].z == R[j].z &&
                                  R[i].w == R[j].w);
    }
    auto get = [&](int q, d3& n, double& d) -> bool {
        bool ok = false;
#pragma unroll
        for (int j = 0; j < kSmall; ++j)
            if (j == q) {
                ok = !drop[j];
                n = mk(R[j].x, R[j].y, R[j].z);
                d = (double)R[j].w;
            }
        return ok;
    };
    return run_passes(K, get, yprop, P, yres);
}
#undef CE

// A region of kSmall < K <= kMid half-spaces projected by one lane.  Only
// (rho, index) pairs go through the sorting network (a bitonic one, every
// index a constant after unrolling); the keys that break ties of rho are read
// from memory when a tie occurs.  The sorted indices go to the lane's column
// of LDS (entry q at col[q * kBlock], so that the lanes of a wavefront read
// neighbouring bytes), and the passes gather each record from the region in
// sorted order, the next one loaded while the current one is evaluated.  Keys
// are unique within a region, so the order is that of the other paths;
// duplicates and passes as in project_small.
__device__ __forceinline__ uint64_t key_at(const ccfr_halfspace* H, int K, int q) {
    return q < K ? H[q].key : ~0ull;
}

#define CEI(i, j)                                                                            \
    {                                                                                        \
        bool sw = rho[j] < rho[i];                                                           \
        if (rho[j] == rho[i]) sw = key_at(H, K, idx[j]) < key_at(H, K, idx[i]);              \
        if (sw) {                                                                            \
            const double tr = rho[i]; rho[i] = rho[j]; rho[j] = tr;                          \
            const int ti = idx[i]; idx[i] = idx[j]; idx[j] = ti;                             \
        }                                                                                    \
    }

__device__ bool project_mid(const ccfr_halfspace* H, int K, const d3 yprop, const MeshParams& P, d3& yres,
                            uint8_t* col) {
    double rho[kMid];
    int idx[kMid];
#pragma unroll
    for (int j = 0; j < kMid; ++j) {
        idx[j] = j;
        rho[j] = j < K ? rho_at(load_plane(H + j), yprop) : __longlong_as_double(0x7ff0000000000000ll);
    }
#pragma unroll
    for (int size = 2; size <= kMid; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
            for (int i = 0; i < kMid; ++i) {
                const int j = i ^ stride;
                if (j > i) {
                    if ((i & size) == 0) CEI(i, j) else CEI(j, i)
                }
            }
        }
    }
    // (a NaN rho can leave padding before K: the index is clamped)
#pragma unroll
    for (int j = 0; j < kMid; ++j) col[j * kBlock] = (uint8_t)min(idx[j], K - 1);
    auto rec = [&](int q) { return load_plane(H + col[q * kBlock]); };
    // an exact duplicate shares its rho with the entries before it in its run
    // of equal rho (the order is sorted), and is compared with those only
    uint32_t drop = 0u;
    int run = 0;                               // first entry of the current run
#pragma unroll
    for (int j = 1; j < kMid; ++j) {
        if (j < K) {
            if (rho[j - 1] != rho[j]) {
                run = j;
            } else {
                const float4 rj = rec(j);
                for (int i = run; i < j; ++i) {
                    const float4 ri = rec(i);
                    if (ri.x == rj.x && ri.y == rj.y && ri.z == rj.z && ri.w == rj.w) {
                        drop |= 1u << j;
                        break;
                    }
                }
            }
        }
    }
    // run_passes asks for entries 0, 1, ..., K - 1 in order in every pass
    float4 nxt = make_float4(0.f, 0.f, 0.f, 0.f);
    auto get = [&](int q, d3& n, double& d) -> bool {
        const float4 cur = q == 0 ? rec(0) : nxt;
        if (q + 1 < K) nxt = rec(q + 1);
        n = mk(cur.x, cur.y, cur.z);
        d = (double)cur.w;
        return ((drop >> q) & 1u) == 0u;
    };
    return run_passes(K, get, yprop, P, yres);
}
#undef CEI

struct WaveLds {
    float4 rec[kWave];
    uint64_t key[kWave];
    double rho[kWave];
    int16_t idx[kWave];
};

// Orders the LDS writes and reads of one wavefront (its lanes run together, so
// completing the wavefront's own LDS operations is all a barrier has to do).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

constexpr int kChunks = kWave / 64;   // sorted entries held per lane

__device__ __forceinline__ float lane_value(float x, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}

// Lane `src`'s copy of a wave-uniform chunk's record: every chunk is read out
// of that lane and the chunk picked afterwards, so that R is only ever indexed
// by constants (a runtime index would move it to scratch memory).
__device__ __forceinline__ float4 take(const float4 (&R)[kChunks], int chunk, int src) {
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        const float4 t = make_float4(lane_value(R[c].x, src), lane_value(R[c].y, src), lane_value(R[c].z, src),
                                     lane_value(R[c].w, src));
        if (chunk == c) r = t;
    }
    return r;
}

// One vertex of list B by one wavefront: its half-spaces are sorted in LDS by a
// bitonic network, then held in registers in sorted order (lane l keeps entries
// l, l + 64, ...; dropped duplicates and padding read as never violated).  Each
// pass of Alg. 2 advances by ballots: every lane evaluates rho at the current
// point for its entries at or after the last hit, the lowest violated one is
// the next hit, and all lanes apply the same Alg. 1 update and retraction to
// their (identical) copies of the state.  This visits exactly the half-spaces
// the sequential pass of run_passes would, in the same order, with the same
// arithmetic, its scalar tail once three planes are stored included.
// Returns the anchor's largest coordinate move (on lane 0; 0 elsewhere).
__device__ __forceinline__ float project_wave_vertex(const ProjectArgs& a, DevCounters* c, WaveLds* L, int v,
                                                     float& sf) {
    const int lane = __lane_id();
    long long o0;
    const int K = region_size(a, v, &o0);
    const MeshParams P = a.prm.get(a.prm.mesh_of(v));
    const d3 yprop = load_prop(a, v);
    d3 y = yprop;
    bool halted = false;
    const ccfr_halfspace* H = a.hs + o0;
    if (K > kWave) {
        // beyond LDS: the wavefront sorts in the scratch range parallel to the region
        bool any = false;
        for (int j = lane; j < K; j += 64) any = any || rho_at(load_plane(H + j), yprop) < 0.0;
        if (__ballot(any)) {
            if (lane == 0) spread_add(c, 0, 1ull);
            halted = project_slow(H, K, yprop, P, a.sort_key + o0, a.sort_idx + o0, y);
        }
    } else {
        int Kp = 1;
        while (Kp < K) Kp <<= 1;
        bool any = false;
        for (int j = lane; j < Kp; j += 64) {
            if (j < K) {
                const ccfr_halfspace h = H[j];
                L->rec[j] = make_float4(h.n[0], h.n[1], h.n[2], h.d);
                L->key[j] = h.key;
                const double r = dot(load_n(h), yprop) + (double)h.d;
                L->rho[j] = r;
                any = any || r < 0.0;
            } else {
                L->key[j] = ~0ull;
                L->rho[j] = __longlong_as_double(0x7ff0000000000000ll);   // +inf: sorts last
            }
            L->idx[j] = (int16_t)j;
        }
        // no violation: the first pass returns the proposal (no sort needed)
        if (__ballot(any)) {
            if (lane == 0) spread_add(c, 0, 1ull);
            wave_sync();
            for (int size = 2; size <= Kp; size <<= 1) {
                for (int stride = size >> 1; stride > 0; stride >>= 1) {
                    for (int t = lane; t < (Kp >> 1); t += 64) {
                        const int p = 2 * t - (t & (stride - 1));
                        const int q = p + stride;
                        const bool up = (p & size) == 0;
                        const bool swap = up ? before(L->rho[q], L->key[q], L->rho[p], L->key[p])
                                             : before(L->rho[p], L->key[p], L->rho[q], L->key[q]);
                        if (swap) {
                            const double tr = L->rho[p]; L->rho[p] = L->rho[q]; L->rho[q] = tr;
                            const uint64_t tk = L->key[p]; L->key[p] = L->key[q]; L->key[q] = tk;
                            const int16_t ti = L->idx[p]; L->idx[p] = L->idx[q]; L->idx[q] = ti;
                        }
                    }
                    wave_sync();
                }
            }
            // sorted records into registers; exact duplicates after the first of
            // their rho run, and the padding, get d = +inf (never violated)
            float4 R[kChunks];
#pragma unroll
            for (int ch = 0; ch < kChunks; ++ch) {
                const int q = ch * 64 + lane;
                R[ch] = make_float4(0.f, 0.f, 0.f, __builtin_inff());
                if (q < K) {
                    const float4 rq = L->rec[L->idx[q]];
                    bool dup = false;
                    for (int r = q - 1; r >= 0 && L->rho[r] == L->rho[q] && !dup; --r) {
                        const float4 rr = L->rec[L->idx[r]];
                        dup = rr.x == rq.x && rr.y == rq.y && rr.z == rq.z && rr.w == rq.w;
                    }
                    if (!dup) R[ch] = rq;
                }
            }
            const int n_chunks = (K + 63) >> 6;
            const double eps_r = (double)P.eps_retract;
            const double eps_p = (double)P.eps_plesnik;
            d3 yp = yprop;
            halted = true;
            for (int pass = 0; pass < P.max_passes; ++pass) {
                d3 yt = yp;
                const d3 y0 = yp;
                Ero S;
                S.m = 0;
                int nviol = 0;
                int from = 0;
                while (true) {
                    // lowest violated sorted entry at or after `from`, at the current point
                    int hit = -1;
#pragma unroll
                    for (int ch = 0; ch < kChunks; ++ch) {
                        if (hit < 0 && ch < n_chunks && ch * 64 + 63 >= from) {
                            const int q = ch * 64 + lane;
                            const bool viol = q >= from && rho_at(R[ch], yt) < 0.0;
                            const unsigned long long m = __ballot(viol);
                            if (m) hit = ch * 64 + __ffsll((long long)m) - 1;
                        }
                    }
                    if (hit < 0) break;
                    const float4 rr = take(R, hit >> 6, hit & 63);
                    ++nviol;
                    orthogonal_projection(yt, y0, mk(rr.x, rr.y, rr.z), -(double)rr.w, S, eps_p);
                    const double nd = norm(yt);
                    yt = (nd > eps_r) ? ((nd - eps_r) / nd) * yt : mk(0.0, 0.0, 0.0);
                    from = hit + 1;
                    if (S.m == 3) {
                        // Alg. 1 holds three planes and returns its input from now
                        // on, so every further violation of this pass only
                        // retracts: yt keeps its direction u and loses eps in
                        // length.  With yt = lam u, rho of entry q is
                        // lam (n_q . u) + d_q, and the rest of the pass runs on
                        // the scalar lam (the same steps, without a square root
                        // and a division per violation).
                        double lam = norm(yt);
                        const d3 u = lam > 0.0 ? (1.0 / lam) * yt : mk(0.0, 0.0, 0.0);
                        double au[kChunks];
#pragma unroll
                        for (int ch = 0; ch < kChunks; ++ch) au[ch] = dot(mk(R[ch].x, R[ch].y, R[ch].z), u);
                        while (true) {
                            int hit2 = -1;
#pragma unroll
                            for (int ch = 0; ch < kChunks; ++ch) {
                                if (hit2 < 0 && ch < n_chunks && ch * 64 + 63 >= from) {
                                    const int q = ch * 64 + lane;
                                    const bool viol = q >= from && lam * au[ch] + (double)R[ch].w < 0.0;
                                    const unsigned long long m = __ballot(viol);
                                    if (m) hit2 = ch * 64 + __ffsll((long long)m) - 1;
                                }
                            }
                            if (hit2 < 0) break;
                            ++nviol;
                            lam = lam > eps_r ? lam - eps_r : 0.0;
                            from = hit2 + 1;
                        }
                        yt = lam * u;
                        break;
                    }
                }
                if (nviol == 0) {
                    y = yp;
                    halted = false;
                    break;
                }
                yp = yt;
            }
            if (halted) y = mk(0.0, 0.0, 0.0);
        }
        wave_sync();   // the LDS slice is reused by the wavefront's next vertex
    }
    float move = 0.0f;
    if (lane == 0) {
        move = write_result(a, c, v, y, (double)P.r, halted, norm(yprop), sf);
        if (halted) spread_add(c, 1, 1ull);
        slots_consumed(a, v);
    }
    return move;
}

// One lane per listed vertex, the sort and the passes in registers, over list
// A (regions of at most kSmall half-spaces) and then the n_m entries of the
// mid-size list (kSmall < K <= kMid; none when the wavefronts take it);
// block lb of the lane path's nb.
__device__ __forceinline__ void project_lane_lists(const ProjectArgs& a, DevCounters* c, int n_a, int n_m, int lb,
                                                   int nb, uint8_t* col) {
    float move = 0.0f, sf = 0.0f;
    const int n_list = n_a + n_m;
    for (int i0 = lb * kBlock; i0 < n_list; i0 += nb * kBlock) {
        const int i = i0 + threadIdx.x;
        bool halted = false;
        const bool mid = i >= n_a && i < n_list;
        if (i < n_list) {
            const int v = mid ? a.slow_list[a.n_verts + (i - n_a)] : a.slow_list[i];
            long long o0;
            const int K = region_size(a, v, &o0);
            const MeshParams P = a.prm.get(a.prm.mesh_of(v));
            d3 y;
            const d3 yp = load_prop(a, v);
            halted = mid ? project_mid(a.hs + o0, K, yp, P, y, col) : project_small(a.hs + o0, K, yp, P, y);
            move = fmaxf(move, write_result(a, c, v, y, (double)P.r, halted, norm(yp), sf));
            slots_consumed(a, v);
        }
        const unsigned long long mh = __ballot(halted);
        if (__lane_id() == 0 && mh) spread_add(c, 1, (unsigned long long)__popcll(mh));
        // every vertex of the mid-size list has a violated half-space
        const unsigned long long ml = __ballot(mid);
        if (__lane_id() == 0 && ml) spread_add(c, 0, (unsigned long long)__popcll(ml));
    }
    record_motion(a, move);
    record_shortfall(a, sf);
}

// The three slow lists in one launch.  Blocks [0, wave_blocks) run list B
// (regions above kMid half-spaces), one vertex per wavefront, first, since
// their vertices take the longest; the next lane_blocks run list A (K <=
// kSmall) and then the mid-size list (kSmall < K <= kMid), one lane per
// vertex, the sort and the passes in registers.
__global__ __launch_bounds__(kBlock) void k_project_slow(ProjectArgs a, DevCounters* c, int wave_blocks,
                                                         int lane_blocks) {
    if (a.skip && *a.skip) return;
    __shared__ WaveLds lds[kBlock / 64];
    const int b = (int)blockIdx.x;
    if (b >= wave_blocks + lane_blocks) {
        // the next iteration's stretch start: the slow path reads no p
        restart_pass_wide(a.next, b - wave_blocks - lane_blocks, threadIdx.x, kBlock);
        return;
    }
    // The mid-size list goes to the wavefronts too when they are enough for
    // every listed vertex of both lists (a wavefront per vertex finishes one
    // sooner than a lane does); when they are not, the lanes take it after
    // list A, 64 vertices per wavefront.  The choice is the same for every block.
    const int n_b = c->n_viol_b, n_m = c->n_viol_m;
    const int workers = wave_blocks * (kBlock / 64);
    const bool mid_by_waves = (long long)n_b + n_m <= workers;
    if (b < wave_blocks) {
        const int wave = threadIdx.x / 64;
        const int n_list = n_b + (mid_by_waves ? n_m : 0);
        WaveLds* L = &lds[wave];
        float move = 0.0f, sf = 0.0f;
        for (int i = b * (kBlock / 64) + wave; i < n_list; i += workers) {
            const int v = i < n_b ? a.slow_list[a.n_verts - 1 - i] : a.slow_list[a.n_verts + (i - n_b)];
            move = fmaxf(move, project_wave_vertex(a, c, L, v, sf));
        }
        record_motion(a, move);
        record_shortfall(a, sf);
        return;
    }
    // the lane path uses the wavefronts' LDS for the sorted indices
    static_assert(sizeof(lds) >= (size_t)kMid * kBlock, "LDS of a block holds the sorted indices");
    uint8_t* col = reinterpret_cast<uint8_t*>(lds) + threadIdx.x;
    project_lane_lists(a, c, c->n_viol, mid_by_waves ? 0 : n_m, b - wave_blocks, lane_blocks, col);
}

__global__ void k_zero_viol(DevCounters* c) {
    if (threadIdx.x == 0) {
        c->n_viol = 0;
        c->n_viol_b = 0;
        c->n_viol_m = 0;
    }
}

}  // namespace

void launch_project(const ProjectArgs& a, DevCounters* c, bool zero_counters, hipStream_t s) {
    if (a.n_verts <= 0) return;
    if (zero_counters) hipLaunchKernelGGL(k_zero_viol, dim3(1), dim3(64), 0, s, c);
    hipLaunchKernelGGL(k_project_fast, dim3((a.n_verts + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a, c);
    // list sizes are known on the device only: enough blocks for a few
    // thousand wavefront vertices and a grid-stride over the lane list
    const int lane_blocks = std::max(1, std::min(1024, (a.n_verts + kBlock - 1) / kBlock));
    const int wave_blocks = std::max(1, std::min(1024, (a.n_verts + kBlock / 64 - 1) / (kBlock / 64)));
    const int restart_blocks = restart_job_blocks(a.next, kBlock);
    hipLaunchKernelGGL(k_project_slow, dim3(wave_blocks + lane_blocks + restart_blocks), dim3(kBlock), 0, s, a, c,
                       wave_blocks, lane_blocks);
}

}  // namespace ccfr
