// k_scan.hip -- exclusive prefix sum of int32 counts (grid buckets, per-vertex
// half-space counts) on gfx950: per-block totals, a one-block scan of the
// totals, and a per-block rescan that adds its base.  out has n + 1 entries,
// out[n] = total.  If zero_in is given, the input is cleared as it is read, so
// count arrays are zero again for the next build without a separate memset.
#include "ccfr_internal.h"

namespace ccfr {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 4;
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

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const int32_t* in, int n, int32_t* partial) {
    __shared__ int lds[kThreads / 64 + 1];
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kItems;
    int s = 0;
    for (int k = 0; k < kItems; ++k)
        if (base + k < n) s += in[base + k];
    const int inc = block_inclusive(s, lds);
    if (threadIdx.x == kThreads - 1) partial[blockIdx.x] = inc;
}

__global__ __launch_bounds__(kThreads) void k_scan_partials(int32_t* partial, int nb) {
    __shared__ int lds[kThreads / 64 + 1];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nb; b0 += kThreads) {
        const int i = b0 + threadIdx.x;
        const int v = i < nb ? partial[i] : 0;
        const int inc = block_inclusive(v, lds);
        const int c0 = carry;
        if (i < nb) partial[i] = c0 + inc - v;
        __syncthreads();
        if (threadIdx.x == kThreads - 1) carry = c0 + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[nb] = carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_down(const int32_t* in, int32_t* out, int32_t* zero_in, int n,
                                                        const int32_t* partial, int nb) {
    __shared__ int lds[kThreads / 64 + 1];
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kItems;
    int vals[kItems];
    int s = 0;
    for (int k = 0; k < kItems; ++k) {
        vals[k] = (base + k < n) ? in[base + k] : 0;
        s += vals[k];
    }
    const int inc = block_inclusive(s, lds);
    int run = partial[blockIdx.x] + inc - s;
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) {
            out[base + k] = run;
            if (zero_in) zero_in[base + k] = 0;
        }
        run += vals[k];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = partial[nb];
}

}  // namespace

// tmp must hold ceil(n / 1024) + 1 ints
void launch_scan(const int32_t* in, int32_t* out, int32_t* zero_in, int n, int32_t* tmp, hipStream_t s) {
    const int nb = n > 0 ? (n + kTile - 1) / kTile : 1;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kThreads), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kThreads), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kThreads), 0, s, in, out, zero_in, n, tmp, nb);
}

}  // namespace ccfr
