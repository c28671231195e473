// ccfr_noalloc.hip -- ccfr_project_displacements for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc): the same projection kernels, with their
// scratch (the device counters, the list of vertices deferred to the slow
// path, and the sort keys of regions larger than a wavefront sorts) in one
// file-scope device array instead of a context's workspace.
//
// The array lives in every GPU the library runs on until the process ends.
// Host code never passes the array's name to a kernel: its address on the
// current device is looked up once per device with hipGetSymbolAddress and
// kept, and that address is what the kernels receive.  Every call on a GPU
// shares that GPU's array, so calls that overlap on one GPU (different
// streams, or host threads) race; calls ordered on one stream do not.
#include <mutex>

#include "ccfr_host.h"
#include "ccfr_internal.h"

namespace ccfr {
namespace {

constexpr long long kNaMaxVerts = 1LL << 20;   // vertices per call
constexpr long long kNaMaxHs = 1LL << 22;      // half-spaces (regions->cap) per call
constexpr size_t kNaCounters = (sizeof(DevCounters) + 255) / 256 * 256;
constexpr size_t kNaSlowList = kNaCounters;                                  // int32 [2 kNaMaxVerts]
constexpr size_t kNaSortKey = kNaSlowList + 8 * (size_t)kNaMaxVerts;         // double [kNaMaxHs]
constexpr size_t kNaSortIdx = kNaSortKey + 8 * (size_t)kNaMaxHs;             // int32 [kNaMaxHs]
constexpr size_t kNaBytes = kNaSortIdx + 4 * (size_t)kNaMaxHs;
constexpr int kNaDevices = 64;

__device__ __align__(256) unsigned char scratch[kNaBytes];

std::mutex g_na_mutex;
unsigned char* g_na_ptr[kNaDevices] = {};

// Address of `scratch` on the current device (looked up once per device).
hipError_t scratch_on_current_device(unsigned char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNaDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_na_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_na_ptr[dev];
    return hipSuccess;
}

// The counters start each call at zero (a fill kernel, not a memset node, so
// that the call may be recorded into a graph).
__global__ void k_na_zero(uint32_t* words, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) words[i] = 0u;
}

__global__ void k_na_status(const DevCounters* c, uint32_t* status_dev) {
    if (threadIdx.x == 0) *status_dev = c->status;
}

}  // namespace
}  // namespace ccfr

using namespace ccfr;
using namespace ccfr::host;

extern "C" int ccfr_project_displacements_noalloc(const ccfr_regions* regions, const float* inv_mass_dev,
                                                  const float* y_in_dev, const ccfr_params* params,
                                                  float* y_out_dev, uint8_t* halted_dev, uint32_t* status_dev,
                                                  ccfr_stream stream) {
    if (!regions || !params_ok(params)) return CCFR_ERR_INVALID_ARG;
    if ((!inv_mass_dev || !y_in_dev || !y_out_dev) && regions->n_verts > 0) return CCFR_ERR_INVALID_ARG;
    if (regions->n_verts < 0 || !regions->offsets || (regions->cap > 0 && !regions->hs) || regions->cap < 0)
        return CCFR_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(regions->hs) % 16 != 0) return CCFR_ERR_INVALID_ARG;
    if (regions->n_verts > kNaMaxVerts || regions->cap > kNaMaxHs) return CCFR_ERR_CAPACITY;
    unsigned char* base = nullptr;
    if (scratch_on_current_device(&base) != hipSuccess) return CCFR_ERR_HIP;
    const hipStream_t s = (hipStream_t)stream;
    DevCounters* c = reinterpret_cast<DevCounters*>(base);
    hipLaunchKernelGGL(k_na_zero, dim3(1), dim3(256), 0, s, reinterpret_cast<uint32_t*>(base),
                       (int)(sizeof(DevCounters) / 4));
    ProjectArgs pa{};
    pa.n_verts = regions->n_verts;
    pa.offsets = regions->offsets;
    pa.hs = regions->hs;
    pa.cap_hs = regions->cap;
    pa.inv_mass = inv_mass_dev;
    pa.y_in = y_in_dev;
    pa.p = nullptr;
    pa.x_anchor = nullptr;
    pa.y_out = y_out_dev;
    pa.halted = halted_dev;
    pa.sort_key = reinterpret_cast<double*>(base + kNaSortKey);
    pa.sort_idx = reinterpret_cast<int32_t*>(base + kNaSortIdx);
    pa.slow_list = reinterpret_cast<int32_t*>(base + kNaSlowList);
    pa.prm.table = nullptr;
    pa.prm.vmesh = nullptr;
    pa.prm.one = mesh_params(params, 0.f, 0, 1.0f);
    launch_project(pa, c, false, s);
    if (status_dev) hipLaunchKernelGGL(k_na_status, dim3(1), dim3(64), 0, s, c, status_dev);
    return hipGetLastError() == hipSuccess ? CCFR_OK : CCFR_ERR_HIP;
}
