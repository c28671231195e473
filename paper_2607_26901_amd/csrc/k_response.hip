// k_response.hip -- applyResponse of Alg. 4: the soft response with
// visibility weights and friction of Sec. 3.3, per vertex on its region,
// between the XPBD constraints and the projection.
//
// The response energy k/2 w_c max(0, delta - d_c)^2 is the XPBD constraint
// C_c = max(0, delta - d_c) with compliance alpha = 1/k.  Constraints are
// owned per vertex (Sec. 3.4), so one thread handles one vertex with no
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
// rebuilt by every iteration's narrow phase).  The active contacts are found
// again for every step of the ordered walk instead of being stored, so the
// kernel keeps no per-vertex list; regions are small.  Arithmetic in FP64
// registers from the FP32 region and proposal.
#include "ccfr_internal.h"

namespace ccfr {
namespace {

constexpr int kBlock = 256;

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

__global__ __launch_bounds__(kBlock) void k_response(ResponseArgs a) {
    if (a.skip && *a.skip) return;
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= a.n_verts) return;
    const MeshParams P = a.prm.get(a.prm.mesh_of(v));
    float yf[3];
    for (int k = 0; k < 3; ++k) yf[k] = a.y_in ? a.y_in[3 * v + k] : a.p[3 * v + k] - a.x_anchor[3 * v + k];
    const double w = a.inv_mass[v];
    int K = 0;
    const ccfr_halfspace* H = nullptr;
    if (a.slot_stride > 0) {
        K = min(a.slot_counts[v], a.slot_stride);
        H = a.hs + (long long)v * a.slot_stride;
    } else {
        K = a.offsets[v + 1] - a.offsets[v];
        H = a.hs + a.offsets[v];
    }
    if (!(w > 0.0) || !P.response || K == 0 || !(P.delta > 0.0f) ||
        !(isfinite(yf[0]) && isfinite(yf[1]) && isfinite(yf[2]))) {
        if (a.y_out)
            for (int k = 0; k < 3; ++k) a.y_out[3 * v + k] = yf[k];
        return;
    }
    const double y0[3] = {yf[0], yf[1], yf[2]};
    const double delta = P.delta, dv = P.vis_width, dt = a.dt;
    double y[3] = {y0[0], y0[1], y0[2]};
    double last_d = -__longlong_as_double(0x7ff0000000000000ll);
    uint64_t last_key = 0;
    bool first = true;
    for (;;) {
        // the next active contact in (gap, key) order
        int c = -1;
        double dc = 0.0;
        uint64_t kc = 0;
        for (int k = 0; k < K; ++k) {
            const Plane p = plane_at(H, k);
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
        // its visibility weight over the other active contacts
        double wc = 1.0;
        if (dv > 0.0)
            for (int j = 0; j < K; ++j) {
                if (j == c) continue;
                const double dj = gap_of(plane_at(H, j), y0);
                if (dj < delta) wc *= 1.0 - smoothstep((dc - dj) / dv);
            }
        if (!(wc > 0.0)) continue;
        const Plane p = plane_at(H, c);
        const double rho = dot3(p.n, y) + p.d;
        const double cv = p.share * delta - rho;
        if (!(cv > 0.0)) continue;
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
    if (a.y_out) {
        for (int k = 0; k < 3; ++k) a.y_out[3 * v + k] = (float)y[k];
    } else {
        for (int k = 0; k < 3; ++k) a.p[3 * v + k] = a.x_anchor[3 * v + k] + (float)y[k];
    }
}

}  // namespace

void launch_response(const ResponseArgs& a, hipStream_t s) {
    if (a.n_verts <= 0) return;
    hipLaunchKernelGGL(k_response, dim3((a.n_verts + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}

}  // namespace ccfr
