// pair_emit.h -- staging of found candidate pairs in LDS for the broad-phase
// kernels (the hash grid's pair kernel and the hierarchy's query kernel).
//
// A block of kEmitBlock threads, one query per lane.  Every lane owns a slice of
// kLaneCap entries of the block's array lane_pairs[slot][thread] and counts
// its entries in a register, so an append is one LDS store.  An entry holds
// only the partner of the pair, the other primitive being the lane's own query:
// a vertex query's partners are triangles (vertex-face list), particles (the
// particle list; tagged by bit 31) and edges (the particle-edge list; tagged by
// bit 30); an edge query's are edges (edge-edge list, stored as (min, max)).
// A wavefront whose lanes might overflow writes its slices out with one atomic
// per list; what is left at the end of the block goes out with one atomic per
// list for the whole block.  Appending each pair with its own atomic on the
// list's counter serialises every wavefront of the launch on four words.
#pragma once

#include "ccfr_internal.h"

namespace ccfr {

#define LDS_PTR __attribute__((address_space(3)))

constexpr int kEmitBlock = 256;                // threads per block of a kernel that emits
constexpr int kEmitWaves = kEmitBlock / 64;
constexpr int kLaneCap = 32;                   // pairs per lane slice

struct LaneBuf {
    LDS_PTR int32_t* slot0;    // &lane_pairs[0][thread]; slot s at slot0[s * kEmitBlock]: a partner
    int fill;                  // entries in the slice
    int n_vv;                  // of them particle partners (top bit set)
    int n_ve;                  // of them edge partners of a particle (bit 30 set)
    bool vert;                 // vertex query: pairs (self, triangle); edge query: edge pairs (min, max)
    int self;                  // the query: vertex or edge
};

__device__ __forceinline__ void lane_put(LaneBuf& lb, int partner, bool pred) {
    if (pred) {
        lb.slot0[lb.fill * kEmitBlock] = partner;
        ++lb.fill;
    }
}

__device__ __forceinline__ void lane_put_vv(LaneBuf& lb, int partner, bool pred) {
    if (pred) {
        lb.slot0[lb.fill * kEmitBlock] = partner | (int)0x80000000;
        ++lb.fill;
        ++lb.n_vv;
    }
}

__device__ __forceinline__ void lane_put_ve(LaneBuf& lb, int partner, bool pred) {
    if (pred) {
        lb.slot0[lb.fill * kEmitBlock] = partner | 0x40000000;
        ++lb.fill;
        ++lb.n_ve;
    }
}

// Exclusive prefix (over the lanes below this one) and total of `n`
// (0..kLaneCap) among the active lanes for which `mine` holds; lanes outside
// take no part.
__device__ __forceinline__ void wave_prefix(int n, bool mine, int& pre, int& tot) {
    const unsigned long long below = (1ull << __lane_id()) - 1ull;
    pre = tot = 0;
#pragma unroll
    for (int bit = 0; (1 << bit) <= kLaneCap; ++bit) {
        const unsigned long long m = __ballot(mine && ((n >> bit) & 1));
        pre += __popcll(m & below) << bit;
        tot += __popcll(m) << bit;
    }
}

// Writes a lane's slice: its first-list pairs (vertex-face or edge-edge) from
// position `at`, its particle pairs from `at_vv`, its particle-edge pairs from
// `at_ve`.
__device__ __forceinline__ void lane_write(const LaneBuf& lb, const PairLists& pl, long long at, long long at_vv,
                                           long long at_ve) {
    int32_t* list = lb.vert ? pl.vf : pl.ee;
    const int64_t cap = lb.vert ? pl.cap_vf : pl.cap_ee;
    for (int s = 0; s < lb.fill; ++s) {
        const int pr = lb.slot0[s * kEmitBlock];
        if (pr < 0) {
            const int q = pr & 0x7fffffff;
            if (at_vv < pl.cap_vv) {
                pl.vv[2 * at_vv + 0] = min(lb.self, q);
                pl.vv[2 * at_vv + 1] = max(lb.self, q);
            }
            ++at_vv;
        } else if (pr & 0x40000000) {
            if (at_ve < pl.cap_ve) {
                pl.ve[2 * at_ve + 0] = lb.self;
                pl.ve[2 * at_ve + 1] = pr & 0x3fffffff;
            }
            ++at_ve;
        } else {
            if (at < cap) {
                list[2 * at + 0] = lb.vert ? lb.self : min(lb.self, pr);
                list[2 * at + 1] = lb.vert ? pr : max(lb.self, pr);
            }
            ++at;
        }
    }
}

// The slice counts' prefix and total per list among the active lanes.
struct KindPrefix {
    int pv, tv, pe, te, pp, tp, px, tx;
    __device__ __forceinline__ explicit KindPrefix(const LaneBuf& lb) {
        const int main = lb.fill - lb.n_vv - lb.n_ve;
        wave_prefix(main, lb.vert, pv, tv);
        wave_prefix(main, !lb.vert, pe, te);
        wave_prefix(lb.n_vv, true, pp, tp);
        wave_prefix(lb.n_ve, true, px, tx);
    }
};

// The active lanes of a wavefront write their slices out.
__device__ __forceinline__ void lane_flush(LaneBuf& lb, const PairLists& pl, DevCounters* c) {
    const KindPrefix kp(lb);
    const int lead = __ffsll((long long)__ballot(true)) - 1;
    int bv = 0, be = 0, bp = 0, bx = 0;
    if (__lane_id() == lead) {
        if (kp.tv) bv = atomicAdd(&c->n_vf, kp.tv);
        if (kp.te) be = atomicAdd(&c->n_ee, kp.te);
        if (kp.tp) bp = atomicAdd(&c->n_vv, kp.tp);
        if (kp.tx) bx = atomicAdd(&c->n_ve, kp.tx);
    }
    bv = __shfl(bv, lead);
    be = __shfl(be, lead);
    bp = __shfl(bp, lead);
    bx = __shfl(bx, lead);
    lane_write(lb, pl, lb.vert ? (long long)bv + kp.pv : (long long)be + kp.pe, (long long)bp + kp.pp,
               (long long)bx + kp.px);
    lb.fill = 0;
    lb.n_vv = 0;
    lb.n_ve = 0;
}

// Called by the active lanes before a round that may append up to `round`
// pairs each: a wavefront with a lane that might overflow writes its slices out.
__device__ __forceinline__ void lane_room_for(LaneBuf& lb, const PairLists& pl, DevCounters* c, int round) {
    if (__ballot(lb.fill > kLaneCap - round) != 0ull) lane_flush(lb, pl, c);
}

// The block is done: what is left in the lane slices goes out with one atomic
// per list for the whole block.  Every thread of the block calls it.
__device__ __forceinline__ void block_flush(LaneBuf& lb, const PairLists& pl, DevCounters* c) {
    __shared__ int wsum[kEmitWaves][4];
    __shared__ int base[kEmitWaves][4];
    const int wave = threadIdx.x / 64;
    const KindPrefix kp(lb);
    if (__lane_id() == 0) {
        wsum[wave][0] = kp.tv;
        wsum[wave][1] = kp.te;
        wsum[wave][2] = kp.tp;
        wsum[wave][3] = kp.tx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t* counters[4] = {&c->n_vf, &c->n_ee, &c->n_vv, &c->n_ve};
        for (int k = 0; k < 4; ++k) {
            int acc = 0;
            for (int w = 0; w < kEmitWaves; ++w) {
                base[w][k] = acc;
                acc += wsum[w][k];
            }
            const int b0 = acc ? atomicAdd(counters[k], acc) : 0;
            for (int w = 0; w < kEmitWaves; ++w) base[w][k] += b0;
        }
    }
    __syncthreads();
    lane_write(lb, pl, lb.vert ? (long long)base[wave][0] + kp.pv : (long long)base[wave][1] + kp.pe,
               (long long)base[wave][2] + kp.pp, (long long)base[wave][3] + kp.px);
}

}  // namespace ccfr
