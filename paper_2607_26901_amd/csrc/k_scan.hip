// k_scan.hip -- exclusive prefix sum of int32 counts (grid buckets, per-vertex
// half-space counts) on gfx950 in two launches: per-block totals, then a
// per-block rescan whose base every block sums itself from the totals before
// it (a few hundred totals for millions of counts, read from L2).  Each thread
// takes 16 consecutive counts with 16-byte loads and stores.  out has n + 1
// entries, out[n] = total.  If zero_in is given, the input is cleared as it is
// read, so count arrays are zero again for the next build without a separate
// memset.  The arrays are allocation bases (16-byte aligned).
#include "ccfr_internal.h"

namespace ccfr {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;

// inclusive scan of one value per thread across the block
__device__ __forceinline__ int block_inclusive(int v, int* lds_waves) {
    const int lane = __lane_id();
    const int wave = threadIdx.x / warpSize;
    for (int off = 1; off < warpSize; off <<= 1) {
        const int t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    if (lane == warpSize - 1) lds_waves[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int k = 0; k < kThreads / warpSize; ++k) {
            const int t = lds_waves[k];
            lds_waves[k] = acc;
            acc += t;
        }
    }
    __syncthreads();
    v += lds_waves[wave];
    __syncthreads();
    return v;
}

// A thread's kItems counts from `base` (zeros past n).
__device__ __forceinline__ void load_items(const int32_t* in, long long base, int n, int v[kItems]) {
    if (base + kItems <= n) {
        const int4* q = reinterpret_cast<const int4*>(in + base);
#pragma unroll
        for (int j = 0; j < kItems / 4; ++j) {
            const int4 t = q[j];
            v[4 * j] = t.x; v[4 * j + 1] = t.y; v[4 * j + 2] = t.z; v[4 * j + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) v[k] = base + k < n ? in[base + k] : 0;
    }
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const int32_t* in, int n, int32_t* partial,
                                                          const uint32_t* run_flag, const uint32_t* skip) {
    if ((run_flag && !*run_flag) || (skip && *skip)) return;
    __shared__ int lds[kThreads / 64 + 1];
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kItems;
    int v[kItems];
    load_items(in, base, n, v);
    int s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) s += v[k];
    const int inc = block_inclusive(s, lds);
    if (threadIdx.x == kThreads - 1) partial[blockIdx.x] = inc;
}

// Sum of partial[0, b) by the whole block.
__device__ __forceinline__ int block_base(const int32_t* partial, int b, int* lds_waves) {
    int s = 0;
    for (int i = threadIdx.x; i < b; i += kThreads) s += partial[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    const int wave = threadIdx.x / warpSize;
    if (__lane_id() == 0) lds_waves[wave] = s;
    __syncthreads();
    int t = 0;
    for (int k = 0; k < kThreads / warpSize; ++k) t += lds_waves[k];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(kThreads) void k_scan_down(const int32_t* in, int32_t* out, int32_t* zero_in, int n,
                                                        const int32_t* partial, int nb, const uint32_t* run_flag,
                                                        const uint32_t* skip) {
    if ((run_flag && !*run_flag) || (skip && *skip)) return;
    __shared__ int lds[kThreads / 64 + 1];
    const int block_base_v = block_base(partial, blockIdx.x, lds);
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kItems;
    int vals[kItems];
    load_items(in, base, n, vals);
    int s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) s += vals[k];
    const int inc = block_inclusive(s, lds);
    int run = block_base_v + inc - s;
    int o[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        o[k] = run;
        run += vals[k];
    }
    if (base + kItems <= n) {
        int4* q = reinterpret_cast<int4*>(out + base);
#pragma unroll
        for (int j = 0; j < kItems / 4; ++j) q[j] = make_int4(o[4 * j], o[4 * j + 1], o[4 * j + 2], o[4 * j + 3]);
        if (zero_in) {
            int4* z = reinterpret_cast<int4*>(zero_in + base);
#pragma unroll
            for (int j = 0; j < kItems / 4; ++j) z[j] = make_int4(0, 0, 0, 0);
        }
    } else {
        for (int k = 0; k < kItems; ++k)
            if (base + k < n) {
                out[base + k] = o[k];
                if (zero_in) zero_in[base + k] = 0;
            }
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == kThreads - 1) out[n] = run;
}

}  // namespace

// tmp must hold ceil(n / 4096) ints
void launch_scan(const int32_t* in, int32_t* out, int32_t* zero_in, int n, int32_t* tmp, hipStream_t s,
                 const uint32_t* run_flag, const uint32_t* skip) {
    const int nb = n > 0 ? (n + kTile - 1) / kTile : 1;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kThreads), 0, s, in, n, tmp, run_flag, skip);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kThreads), 0, s, in, out, zero_in, n, tmp, nb, run_flag, skip);
}

}  // namespace ccfr
