// k_project.hip -- projection of proposed displacements onto the vertex regions
// (Alg. 2 calling Alg. 1, the retraction and halt fallback of Sec. 3.2, and the
// r-ball clamp of Alg. 4) on gfx950.
//
// One lane per vertex.  Region data stays FP32 in HBM; the arithmetic of the
// projection runs in FP64 registers, working in displacement coordinates (the
// anchor is the origin, so a constraint n . x' >= b with b = n . x - d reads
// n . y + d >= 0).  This removes the cancellation of world coordinates, which
// is what makes the sign tests of Alg. 2 fragile in single precision (the
// paper's Sec. 5 names single-precision robustness as open).
//
// Fast path: a vertex none of whose half-spaces is violated by its proposal
// returns it unchanged (Alg. 2 with no violation in its first pass), clamped.
// Slow path (violating vertices): the half-spaces are sorted by their initial
// rho ascending, ties by key, into a scratch range parallel to the vertex's CSR
// range; exact duplicates (bitwise-equal n and d) are dropped; then up to
// max_passes passes of Alg. 1 over the violated ones, each followed by the
// retraction by eps; a pass without violation returns its start point, and
// otherwise the vertex halts at y = 0.
//
// Readings: A12 (Alg. 1's entry j = m is the new plane, and the stored plane is
// that plane), A14 (Alg. 1 returns its input once three planes are stored), A15
// (max_passes is the literal loop count), A16 (the clamp also applies without
// half-spaces; zero inverse mass gives y = 0).
#include "ccfr_internal.h"

namespace ccfr {

namespace {

constexpr int kBlock = 256;

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

// Alg. 2 for a vertex with at least one violated half-space.  Returns true if it halted.
__device__ bool project_slow(const ccfr_halfspace* H, int K, const d3 yprop, const MeshParams& P,
                             double* skey, int32_t* sidx, d3& yres) {
    // sort by (initial rho, key) ascending: insertion sort into the scratch range
    for (int i = 0; i < K; ++i) {
        const ccfr_halfspace hi = H[i];
        const double rho = dot(load_n(hi), yprop) + (double)hi.d;
        int j = i;
        while (j > 0) {
            const double pr = skey[j - 1];
            const int pi = sidx[j - 1];
            if (pr < rho || (pr == rho && H[pi].key < hi.key)) break;
            skey[j] = pr;
            sidx[j] = pi;
            --j;
        }
        skey[j] = rho;
        sidx[j] = i;
    }
    // drop exact duplicates: they share rho, so they sit in the same run
    for (int q = 1; q < K; ++q) {
        const ccfr_halfspace hq = H[sidx[q]];
        for (int r = q - 1; r >= 0 && skey[r] == skey[q]; --r) {
            if (sidx[r] >= 0 && same_plane(H[sidx[r]], hq)) {
                sidx[q] = -1 - sidx[q];   // keep the index recoverable, mark dropped
                break;
            }
        }
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
        for (int q = 0; q < K; ++q) {
            const int idx = sidx[q];
            if (idx < 0) continue;
            const ccfr_halfspace h = H[idx];
            const d3 n = load_n(h);
            const double d = (double)h.d;
            if (dot(n, yt) + d >= 0.0) continue;
            ++nviol;
            orthogonal_projection(yt, y0, n, -d, S, eps_p);
            const double nd = norm(yt);
            yt = (nd > eps_r) ? ((nd - eps_r) / nd) * yt : mk(0.0, 0.0, 0.0);
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

__global__ __launch_bounds__(kBlock) void k_project(ProjectArgs a, DevCounters* c) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    const bool active = v < a.n_verts;
    bool violated = false, halted = false, moved = false;
    if (active) {
        const float w = a.inv_mass[v];
        float yf[3];
        if (a.y_in) {
            yf[0] = a.y_in[3 * v]; yf[1] = a.y_in[3 * v + 1]; yf[2] = a.y_in[3 * v + 2];
        } else {
            for (int k = 0; k < 3; ++k) yf[k] = a.p[3 * v + k] - a.x_anchor[3 * v + k];
        }
        d3 y = mk(0.0, 0.0, 0.0);
        if (w > 0.0f) {
            moved = true;
            const MeshParams P = a.prm.get(a.prm.mesh_of(v));
            const d3 yprop = mk(yf[0], yf[1], yf[2]);
            const long long o0 = a.offsets[v];
            const long long o1 = min((long long)a.offsets[v + 1], (long long)a.cap_hs);
            const int K = o1 > o0 ? (int)(o1 - o0) : 0;
            const ccfr_halfspace* H = a.hs + o0;
            for (int k = 0; k < K && !violated; ++k) {
                const ccfr_halfspace h = H[k];
                violated = dot(load_n(h), yprop) + (double)h.d < 0.0;
            }
            if (!violated) {
                y = yprop;
            } else {
                halted = project_slow(H, K, yprop, P, a.sort_key + o0, a.sort_idx + o0, y);
            }
            const double ny = norm(y);
            const double r = (double)P.r;
            if (ny > r) y = (r / ny) * y;
        }
        if (a.y_out) {
            a.y_out[3 * v] = (float)y.x;
            a.y_out[3 * v + 1] = (float)y.y;
            a.y_out[3 * v + 2] = (float)y.z;
        } else {
            a.x_anchor[3 * v] += (float)y.x;
            a.x_anchor[3 * v + 1] += (float)y.y;
            a.x_anchor[3 * v + 2] += (float)y.z;
        }
        if (a.halted) a.halted[v] = halted ? 1 : 0;
    }
    // one atomic per wave for the counters
    const unsigned long long mv = __ballot(violated);
    const unsigned long long mh = __ballot(halted);
    const unsigned long long mm = __ballot(moved);
    if (__lane_id() == 0) {
        if (mv) atomicAdd((unsigned long long*)&c->totals[4], (unsigned long long)__popcll(mv));
        if (mh) atomicAdd((unsigned long long*)&c->totals[5], (unsigned long long)__popcll(mh));
        if (mm) atomicAdd((unsigned long long*)&c->totals[7], (unsigned long long)__popcll(mm));
    }
}

}  // namespace

void launch_project(const ProjectArgs& a, DevCounters* c, hipStream_t s) {
    if (a.n_verts <= 0) return;
    hipLaunchKernelGGL(k_project, dim3((a.n_verts + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a, c);
}

}  // namespace ccfr
