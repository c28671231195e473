// k_xpbd.hip -- the plain XPBD substep around the CCFR calls (Alg. 4, no
// response or friction): prediction, one Gauss-Seidel pass of XPBD distance
// constraints per solver iteration (Macklin et al. 2016), velocity update.
//
// The stretch pass runs colour by colour: the edges are stored sorted by a
// greedy colouring (edge-index order) whose classes share no vertex, so one
// launch per colour updates its edges in parallel with the same result as the
// sequential pass in colour order.
#include <algorithm>

#include "ccfr_internal.h"

namespace ccfr {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_predict(int n, const float* x, const float* v, const float* w,
                                                    float dt, float gx, float gy, float gz, float* xp,
                                                    float* xs, uint8_t* halt_run, DevCounters* c, int iters_add) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i == 0 && c && iters_add) c->iters_run += iters_add;     // a fixed iteration count
    if (i >= n) return;
    if (halt_run) halt_run[i] = 0;
    const float g[3] = {gx, gy, gz};
    const bool dyn = w[i] > 0.0f;
    for (int k = 0; k < 3; ++k) {
        const float xi = x[3 * i + k];
        xs[3 * i + k] = xi;
        xp[3 * i + k] = dyn ? xi + dt * v[3 * i + k] + dt * dt * g[k] : xi;
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(float* p, long long n) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void k_copy(const float* src, float* dst, long long n) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// End of an iteration's builds (finalize): closes the region build, and the
// candidate build too when no later iteration reuses its lists (close_pairs),
// then clears what the next build counts.  The stretch pass starts here
// (restart_pass on n3 entries and c0), or, when it started earlier, the first
// job_blocks blocks run one of its colours.
__global__ __launch_bounds__(kBlock) void k_close_iteration(const float* x_pred, float* p, long long n3,
                                                            DevCounters* c, uint32_t* level_mask, int n_meshes,
                                                            int32_t n_verts, const int32_t* offsets,
                                                            PairCaps caps, int64_t cap_contacts, int64_t cap_hs,
                                                            int close_pairs, int32_t slot_stride,
                                                            StretchColor0 c0, int finalize, ColourJob job,
                                                            int job_blocks, const uint32_t* skip) {
    if (skip && *skip) return;
    if ((int)blockIdx.x < job_blocks) {
        run_colour_job(job, blockIdx.x * kBlock + threadIdx.x);
        return;
    }
    const long long i = (long long)(blockIdx.x - job_blocks) * kBlock + threadIdx.x;
    const long long n_threads = (long long)(gridDim.x - job_blocks) * kBlock;
    if (i == 0 && finalize) {
        if (close_pairs) finalize_pairs_body(c, caps);
        if (slot_stride > 0) finalize_slot_regions_body(c, n_verts, slot_stride, cap_contacts);
        else finalize_regions_body(c, n_verts, offsets, cap_contacts, cap_hs);
        if (close_pairs) reset_build_counters(c);
        else reset_region_counters(c);
    }
    if (close_pairs && finalize)
        for (long long m = i; m < n_meshes; m += n_threads) level_mask[m] = 0u;
    restart_pass(x_pred, p, n3, c0, i);
}

// One block.  The first wavefront takes the last projection's largest move,
// thread 0 decides (only it reads and writes the motion fields); the block
// then clears the level masks of a build to come.
__global__ __launch_bounds__(kBlock) void k_decide_build(DevCounters* c, uint32_t* level_mask, int n_meshes,
                                                         double skin, PairCaps caps, const uint32_t* skip) {
    if (skip && *skip) return;
    __shared__ int go;
    uint32_t moved = 0u;
    if (threadIdx.x < 64) moved = take_maximum(c, kMaxMotion);
    if (threadIdx.x == 0) {
        const double acc = c->motion_acc + (double)__uint_as_float(moved);
        // the sum is rounded: compare with a relative margin far above its error
        const bool rebuild = acc * (1.0 + 1e-12) > skin;
        if (rebuild) {
            finalize_pairs_body(c, caps);
            c->n_vf = c->n_ee = c->n_vv = 0;
            c->n_large_t = c->n_large_e = 0;
        }
        c->motion_acc = rebuild ? 0.0 : acc;
        c->rebuild = rebuild ? 1u : 0u;
        go = rebuild ? 1 : 0;
    }
    __syncthreads();
    if (go)
        for (int m = threadIdx.x; m < n_meshes; m += kBlock) level_mask[m] = 0u;
}

// evaluateConvergence (Alg. 4), one wavefront: the iterations of the substep
// end once no dynamic vertex's last step fell short of its proposal by more
// than tol (reading of the check: the expected advancement of an iteration is
// the proposal p - x, the step taken is the projected and clamped y*).
__global__ void k_decide_converged(DevCounters* c, float tol, int first) {
    if (blockIdx.x != 0 || threadIdx.x >= 64) return;
    const uint32_t shortfall = take_maximum(c, kMaxShortfall);
    if (threadIdx.x != 0) return;
    if (first) c->converged = 0u;
    else if (!c->converged && __uint_as_float(shortfall) <= tol) c->converged = 1u;
    if (!c->converged) c->iters_run += 1;
}

// Colour class of the stretch pass (edges as in colour_edge), one thread per edge.
__global__ __launch_bounds__(kBlock) void k_stretch(const int32_t* edges, const float* rest, const int2* segs,
                                                    int nseg, int total, const float* w, float* p, float* lambda,
                                                    float alpha_t, const uint32_t* skip) {
    if (skip && *skip) return;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= total) return;
    stretch_edge(colour_edge(segs, nseg, t), edges, rest, w, p, p, lambda, alpha_t, false);
}

__global__ __launch_bounds__(kBlock) void k_fill_no_edge(int2* a, int n) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = make_int2(0, -1);
}

// The endpoints of a colour class's edges point at their edge and each other.
__global__ __launch_bounds__(kBlock) void k_last_colour_map(const int32_t* edges, const int2* segs, int nseg,
                                                            int total, int n_verts, int2* last_edge) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= total) return;
    const int e = colour_edge(segs, nseg, t);
    const int i = edges[2 * e], j = edges[2 * e + 1];
    if (i < 0 || i >= n_verts || j < 0 || j >= n_verts) return;
    last_edge[i] = make_int2(e, j);
    last_edge[j] = make_int2((int)(0x80000000u | (uint32_t)e), i);
}

__global__ __launch_bounds__(kBlock) void k_update_velocity(int n, const float* x, const float* xs, float inv_dt,
                                                            float* v) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < 3; ++k) v[3 * i + k] = (x[3 * i + k] - xs[3 * i + k]) * inv_dt;
}

inline int blocks_for(long long n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

void launch_predict(int n, const float* x, const float* v, const float* inv_mass, float dt, float gx, float gy,
                    float gz, float* x_pred, float* x_start, hipStream_t s, uint8_t* halt_run, DevCounters* c,
                    int iters_add) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_predict, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, x, v, inv_mass, dt, gx, gy, gz,
                       x_pred, x_start, halt_run, c, iters_add);
}

void launch_fill_zero(float* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, (long long)n);
}

void launch_copy(const float* src, float* dst, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3(blocks_for(n)), dim3(kBlock), 0, s, src, dst, (long long)n);
}

void launch_close_iteration(const float* x_pred, float* p, int64_t n3, DevCounters* c, uint32_t* level_mask,
                            int n_meshes, int32_t n_verts, const int32_t* offsets, PairCaps caps,
                            int64_t cap_contacts, int64_t cap_hs, bool close_pairs, hipStream_t s,
                            int32_t slot_stride, const StretchColor0* c0, bool finalize, const ColourJob* job,
                            const uint32_t* skip) {
    StretchColor0 first{};
    if (c0 && c0->total > 0 && c0->nseg > 0) first = *c0;
    ColourJob hosted{};
    if (job) hosted = *job;
    const int jb = colour_job_blocks(hosted, kBlock);
    const long long n = std::max<long long>(
        std::max<long long>(std::max<long long>(n3, finalize ? n_meshes : 0), first.total), 1);
    hipLaunchKernelGGL(k_close_iteration, dim3(blocks_for(n) + jb), dim3(kBlock), 0, s, x_pred, p, (long long)n3, c,
                       level_mask, n_meshes, n_verts, offsets, caps, cap_contacts, cap_hs, close_pairs ? 1 : 0,
                       slot_stride, first, finalize ? 1 : 0, hosted, jb, skip);
}

void launch_decide_build(DevCounters* c, uint32_t* level_mask, int n_meshes, double skin, PairCaps caps,
                         hipStream_t s, const uint32_t* skip) {
    hipLaunchKernelGGL(k_decide_build, dim3(1), dim3(kBlock), 0, s, c, level_mask, n_meshes, skin, caps, skip);
}

void launch_decide_converged(DevCounters* c, float tol, int first, hipStream_t s) {
    hipLaunchKernelGGL(k_decide_converged, dim3(1), dim3(64), 0, s, c, tol, first);
}

void launch_stretch_segments(const int32_t* edges_sorted, const float* rest_sorted, const int2* segs, int32_t nseg,
                             int32_t total, const float* inv_mass, float* p, float* lambda_sorted, float alpha_t,
                             hipStream_t s, const uint32_t* skip) {
    if (total <= 0 || nseg <= 0) return;
    hipLaunchKernelGGL(k_stretch, dim3(blocks_for(total)), dim3(kBlock), 0, s, edges_sorted, rest_sorted, segs, nseg,
                       total, inv_mass, p, lambda_sorted, alpha_t, skip);
}

void launch_last_colour_map(const int32_t* edges_sorted, const int2* segs, int32_t nseg, int32_t total,
                            int32_t n_verts, int2* last_edge, hipStream_t s) {
    if (n_verts <= 0) return;
    hipLaunchKernelGGL(k_fill_no_edge, dim3(blocks_for(n_verts)), dim3(kBlock), 0, s, last_edge, n_verts);
    if (total <= 0 || nseg <= 0) return;
    hipLaunchKernelGGL(k_last_colour_map, dim3(blocks_for(total)), dim3(kBlock), 0, s, edges_sorted, segs, nseg,
                       total, n_verts, last_edge);
}

void launch_update_velocity(int n, const float* x, const float* x_start, float inv_dt, float* v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_update_velocity, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, x, x_start, inv_dt, v);
}

}  // namespace ccfr
