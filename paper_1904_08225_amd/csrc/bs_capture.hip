// bs_capture.hip -- the initial surfel set of a node (paper Sec. 3.1): its
// visible surface captured from the eight corners of its bounding box.
//
// The paper rasterizes the node into position / normal / colour buffers from
// eight orthographic views (each box corner looking at the centre) and turns
// every covered pixel into a candidate surfel.  Here the node is a set of
// analytic primitives and every pixel's candidate is the first surface its
// ray meets -- the visibility a rasterizer resolves at the pixel centre --
// computed by a ray cast over all primitives:
//   1. capture_kernel: one thread per pixel of every view (views on
//      blockIdx.y); the primitives are staged through LDS in chunks; the
//      nearest hit (lowest primitive index on equal t) goes to a G-buffer
//      (position + covered flag, normal + colour), and each workgroup counts
//      its covered pixels;
//   2. capture_scan_kernel: one workgroup turns the counts into offsets;
//   3. capture_scatter_kernel: covered pixels are written in view, row,
//      column order (ballot ranks within the workgroup).
// Arithmetic: binary32 with the operation order below (no contraction,
// correctly rounded division and square root); the sphere and cylinder roots
// start from the ray's closest approach to the centre / axis, which keeps
// the far ray origin from cancelling the discriminant.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <cmath>

#include "bs_internal.h"

namespace bs {
namespace {

constexpr int kCapBlock = 256;
constexpr int kPrimChunk = 128;  // primitives staged in LDS at a time

struct View {
    float d[3], u[3], w[3], c[3], s;
    int ok;
};
struct Views {
    View v[8];
};

struct PrimLds {
    int kind;
    float c[3], r[9], p[3];
    uint32_t rgb;
};

__device__ __forceinline__ float dot3(float a0, float a1, float a2, float b0, float b1, float b2) {
    return (a0 * b0 + a1 * b1) + a2 * b2;
}

// First hit t > 0 of the local ray o + t d with one primitive; local normal.
__device__ __forceinline__ bool hit_prim(const PrimLds& P, const float o[3], const float d[3], float& t_out,
                                         float nl[3]) {
    if (P.kind == 0) {  // sphere
        const float r = P.p[0];
        const float a = dot3(d[0], d[1], d[2], d[0], d[1], d[2]);
        const float t0 = -dot3(o[0], o[1], o[2], d[0], d[1], d[2]) / a;
        const float p0 = o[0] + t0 * d[0], p1 = o[1] + t0 * d[1], p2 = o[2] + t0 * d[2];
        const float h2 = r * r - dot3(p0, p1, p2, p0, p1, p2);
        if (h2 < 0.f) return false;
        const float t = t0 - sqrtf(h2 / a);
        if (!(t > 0.f)) return false;
        nl[0] = (o[0] + t * d[0]) / r;
        nl[1] = (o[1] + t * d[1]) / r;
        nl[2] = (o[2] + t * d[2]) / r;
        t_out = t;
        return true;
    }
    if (P.kind == 1) {  // box: slabs
        float tn = -INFINITY, tf = INFINITY;
        int axis = -1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float h = P.p[k];
            if (d[k] == 0.f) {
                if (o[k] < -h || o[k] > h) return false;
                continue;
            }
            const float t1 = (-h - o[k]) / d[k];
            const float t2 = (h - o[k]) / d[k];
            const float lo = t1 < t2 ? t1 : t2;
            const float hi = t1 < t2 ? t2 : t1;
            if (lo > tn) {
                tn = lo;
                axis = k;
            }
            if (hi < tf) tf = hi;
        }
        if (axis < 0 || !(tn <= tf) || !(tn > 0.f)) return false;
        nl[0] = nl[1] = nl[2] = 0.f;
        const float sg = d[axis] > 0.f ? -1.f : 1.f;
        if (axis == 0) nl[0] = sg;
        else if (axis == 1) nl[1] = sg;
        else nl[2] = sg;
        t_out = tn;
        return true;
    }
    if (P.kind == 2) {  // cylinder along local z: lateral surface, two caps
        const float r = P.p[0], h = P.p[1];
        float best = INFINITY;
        int side = -1;
        const float a = d[0] * d[0] + d[1] * d[1];
        if (a > 0.f) {
            const float t0 = -(o[0] * d[0] + o[1] * d[1]) / a;
            const float x0 = o[0] + t0 * d[0];
            const float y0 = o[1] + t0 * d[1];
            const float h2 = r * r - (x0 * x0 + y0 * y0);
            if (h2 >= 0.f) {
                const float t = t0 - sqrtf(h2 / a);
                const float z = o[2] + t * d[2];
                if (t > 0.f && z >= -h && z <= h) {
                    best = t;
                    side = 0;
                }
            }
        }
        if (d[2] != 0.f) {
#pragma unroll
            for (int cap = 0; cap < 2; ++cap) {
                const float zc = cap ? h : -h;
                const float t = (zc - o[2]) / d[2];
                const float x = o[0] + t * d[0];
                const float y = o[1] + t * d[1];
                if (t > 0.f && (x * x + y * y) <= r * r && t < best) {
                    best = t;
                    side = 1 + cap;
                }
            }
        }
        if (side < 0) return false;
        if (side == 0) {
            nl[0] = (o[0] + best * d[0]) / r;
            nl[1] = (o[1] + best * d[1]) / r;
            nl[2] = 0.f;
        } else {
            nl[0] = 0.f;
            nl[1] = 0.f;
            nl[2] = side == 2 ? 1.f : -1.f;
        }
        t_out = best;
        return true;
    }
    return false;
}

__global__ void __launch_bounds__(kCapBlock)
    capture_kernel(const bs_primitive* __restrict__ prims, int count, Views views, int R, float4* __restrict__ gpos,
                   uint4* __restrict__ gnrm, uint32_t* __restrict__ block_counts) {
    __shared__ PrimLds sp[kPrimChunk];
    __shared__ uint32_t s_cnt;
    const int view = blockIdx.y;
    const View V = views.v[view];
    const int64_t per_view = int64_t(R) * R;
    const int64_t pix = int64_t(blockIdx.x) * kCapBlock + threadIdx.x;
    const bool in = V.ok && pix < per_view;
    const int j = int(pix / R), i = int(pix % R);
    const float s = V.s, s2 = 2.f * s;
    const float fa = float(2 * i + 1) / float(R) - 1.f;
    const float fb = float(2 * j + 1) / float(R) - 1.f;
    const float a = fa * s, b = fb * s;
    float o[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) o[k] = ((V.c[k] + a * V.u[k]) + b * V.w[k]) - s2 * V.d[k];
    float tbest = INFINITY;
    float nb[3] = {0.f, 0.f, 0.f};
    uint32_t rgb = 0;
    if (threadIdx.x == 0) s_cnt = 0;
    for (int base = 0; base < count; base += kPrimChunk) {
        __syncthreads();
        for (int q = threadIdx.x; q < kPrimChunk && base + q < count; q += kCapBlock) {
            const bs_primitive& g = prims[base + q];
            PrimLds& L = sp[q];
            L.kind = g.kind;
            for (int k = 0; k < 3; ++k) {
                L.c[k] = g.center[k];
                L.p[k] = g.prm[k];
            }
            for (int k = 0; k < 9; ++k) L.r[k] = g.rot[k];
            L.rgb = uint32_t(g.rgb[0]) | (uint32_t(g.rgb[1]) << 8) | (uint32_t(g.rgb[2]) << 16);
        }
        __syncthreads();
        const int nq = count - base < kPrimChunk ? count - base : kPrimChunk;
        if (in) {
            for (int q = 0; q < nq; ++q) {
                const PrimLds& P = sp[q];
                const float oc0 = o[0] - P.c[0], oc1 = o[1] - P.c[1], oc2 = o[2] - P.c[2];
                const float ol[3] = {(P.r[0] * oc0 + P.r[3] * oc1) + P.r[6] * oc2,
                                     (P.r[1] * oc0 + P.r[4] * oc1) + P.r[7] * oc2,
                                     (P.r[2] * oc0 + P.r[5] * oc1) + P.r[8] * oc2};
                const float dl[3] = {(P.r[0] * V.d[0] + P.r[3] * V.d[1]) + P.r[6] * V.d[2],
                                     (P.r[1] * V.d[0] + P.r[4] * V.d[1]) + P.r[7] * V.d[2],
                                     (P.r[2] * V.d[0] + P.r[5] * V.d[1]) + P.r[8] * V.d[2]};
                float t, nl[3];
                if (hit_prim(P, ol, dl, t, nl) && t < tbest) {
                    tbest = t;
                    nb[0] = (P.r[0] * nl[0] + P.r[1] * nl[1]) + P.r[2] * nl[2];
                    nb[1] = (P.r[3] * nl[0] + P.r[4] * nl[1]) + P.r[5] * nl[2];
                    nb[2] = (P.r[6] * nl[0] + P.r[7] * nl[1]) + P.r[8] * nl[2];
                    rgb = P.rgb;
                }
            }
        }
    }
    const bool hit = in && tbest < INFINITY;
    if (in) {
        const int64_t g = int64_t(view) * per_view + pix;
        gpos[g] = make_float4(o[0] + tbest * V.d[0], o[1] + tbest * V.d[1], o[2] + tbest * V.d[2], hit ? 1.f : 0.f);
        gnrm[g] = make_uint4(__float_as_uint(nb[0]), __float_as_uint(nb[1]), __float_as_uint(nb[2]), rgb);
    }
    const uint64_t m = __ballot(hit);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&s_cnt, uint32_t(__popcll(m)));
    __syncthreads();
    if (threadIdx.x == 0) block_counts[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = s_cnt;
}

// Exclusive scan of the per-workgroup counts by one workgroup of 1024
// threads; offsets[nb] = total, written to *count as well.
__global__ void __launch_bounds__(1024)
    capture_scan_kernel(const uint32_t* __restrict__ counts, int64_t nb, int64_t* __restrict__ offsets,
                        int64_t* __restrict__ total) {
    __shared__ int64_t s_part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t lo = int64_t(tid) * per, hi = lo + per < nb ? lo + per : nb;
    int64_t sum = 0;
    for (int64_t b = lo; b < hi; ++b) sum += counts[b];
    s_part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = tid >= off ? s_part[tid - off] : 0;
        __syncthreads();
        s_part[tid] += v;
        __syncthreads();
    }
    int64_t run = s_part[tid] - sum;
    for (int64_t b = lo; b < hi; ++b) {
        offsets[b] = run;
        run += counts[b];
    }
    if (tid == 1023) {
        offsets[nb] = s_part[1023];
        *total = s_part[1023];
    }
}

__global__ void __launch_bounds__(kCapBlock)
    capture_scatter_kernel(const float4* __restrict__ gpos, const uint4* __restrict__ gnrm, int R, int views_ok,
                           const int64_t* __restrict__ offsets, float* __restrict__ out_pts,
                           float* __restrict__ out_nrm, uint8_t* __restrict__ out_col) {
    __shared__ uint32_t s_w[kCapBlock / 64];
    const int view = blockIdx.y;
    const int64_t per_view = int64_t(R) * R;
    const int64_t pix = int64_t(blockIdx.x) * kCapBlock + threadIdx.x;
    const bool in = ((views_ok >> view) & 1) && pix < per_view;
    const int64_t g = int64_t(view) * per_view + pix;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    if (in) p = gpos[g];
    const bool hit = in && p.w != 0.f;
    const uint64_t m = __ballot(hit);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_w[wave] = uint32_t(__popcll(m));
    __syncthreads();
    int64_t at = offsets[int64_t(blockIdx.y) * gridDim.x + blockIdx.x];
    for (int w = 0; w < wave; ++w) at += s_w[w];
    at += __popcll(m & ((1ull << lane) - 1ull));
    if (hit) {
        const uint4 q = gnrm[g];
        out_pts[3 * at + 0] = p.x;
        out_pts[3 * at + 1] = p.y;
        out_pts[3 * at + 2] = p.z;
        if (out_nrm) {
            out_nrm[3 * at + 0] = __uint_as_float(q.x);
            out_nrm[3 * at + 1] = __uint_as_float(q.y);
            out_nrm[3 * at + 2] = __uint_as_float(q.z);
        }
        if (out_col) {
            out_col[3 * at + 0] = uint8_t(q.w);
            out_col[3 * at + 1] = uint8_t(q.w >> 8);
            out_col[3 * at + 2] = uint8_t(q.w >> 16);
        }
    }
}

float fdot3(const float* a, const float* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

// Camera of view v (corner bits x, y, z choose hi over lo), binary32.
View make_view(const float* lo, const float* hi, int v) {
    View V{};
    float e[3], dv[3];
    for (int a = 0; a < 3; ++a) {
        V.c[a] = 0.5f * (lo[a] + hi[a]);
        e[a] = hi[a] - lo[a];
        const float corner = ((v >> a) & 1) ? hi[a] : lo[a];
        dv[a] = V.c[a] - corner;
    }
    V.s = 0.5f * sqrtf(fdot3(e, e));
    const float L = sqrtf(fdot3(dv, dv));
    if (!(L > 0.f)) return V;
    for (int a = 0; a < 3; ++a) V.d[a] = dv[a] / L;
    float u[3] = {V.d[1], -V.d[0], 0.f};
    float lu = sqrtf(fdot3(u, u));
    if (!(lu >= 1e-6f)) {
        u[0] = -V.d[2];
        u[1] = 0.f;
        u[2] = V.d[0];
        lu = sqrtf(fdot3(u, u));
    }
    for (int a = 0; a < 3; ++a) V.u[a] = u[a] / lu;
    V.w[0] = V.u[1] * V.d[2] - V.u[2] * V.d[1];
    V.w[1] = V.u[2] * V.d[0] - V.u[0] * V.d[2];
    V.w[2] = V.u[0] * V.d[1] - V.u[1] * V.d[0];
    V.ok = 1;
    return V;
}

struct CapWs {
    float4* gpos;
    uint4* gnrm;
    uint32_t* counts;
    int64_t* offsets;
    size_t total;
};

CapWs cap_layout(int R, char* base) {
    CapWs w{};
    const size_t pix = size_t(8) * size_t(R) * size_t(R);
    const size_t nb = size_t(8) * ((size_t(R) * R + kCapBlock - 1) / kCapBlock);
    size_t off = 0;
    w.gpos = reinterpret_cast<float4*>(base + off);
    off += align_up(pix * sizeof(float4));
    w.gnrm = reinterpret_cast<uint4*>(base + off);
    off += align_up(pix * sizeof(uint4));
    w.counts = reinterpret_cast<uint32_t*>(base + off);
    off += align_up(nb * 4);
    w.offsets = reinterpret_cast<int64_t*>(base + off);
    off += align_up((nb + 1) * 8);
    w.total = off;
    return w;
}

constexpr int kMaxResolution = 8192;

}  // namespace
}  // namespace bs

using namespace bs;

extern "C" {

size_t bs_capture_workspace_size(int32_t resolution) {
    if (resolution < 1 || resolution > kMaxResolution) return 0;
    return cap_layout(resolution, nullptr).total;
}

int bs_capture(const bs_primitive* d_prims, int32_t count, const float* h_lo, const float* h_hi, int32_t resolution,
               float* d_out_points, float* d_out_normals, uint8_t* d_out_colors, int64_t* d_out_count,
               void* d_workspace, size_t workspace_bytes, void* stream) {
    static_assert(sizeof(bs_primitive) == 68, "primitive record");
    if (count < 0 || (count > 0 && !d_prims)) return set_error(BS_ERR_INVALID_ARG, "null or negative primitives");
    if (!h_lo || !h_hi || !d_out_points || !d_out_count) return set_error(BS_ERR_INVALID_ARG, "null argument");
    if (resolution < 1 || resolution > kMaxResolution)
        return set_error(BS_ERR_INVALID_ARG, "resolution %d outside 1..%d", resolution, kMaxResolution);
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(h_lo[a]) || !std::isfinite(h_hi[a]) || h_lo[a] > h_hi[a])
            return set_error(BS_ERR_INVALID_ARG, "bounding box must be finite with lo <= hi");
    const size_t need = bs_capture_workspace_size(resolution);
    if (!d_workspace || workspace_bytes < need)
        return set_error(BS_ERR_INVALID_ARG, "workspace %zu bytes < %zu needed", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
        return set_error(BS_ERR_INVALID_ARG, "workspace not %zu-byte aligned", kAlign);
    Views views{};
    int ok = 0;
    for (int v = 0; v < 8; ++v) {
        views.v[v] = make_view(h_lo, h_hi, v);
        ok |= views.v[v].ok << v;
    }
    const CapWs w = cap_layout(resolution, static_cast<char*>(d_workspace));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t per_view = int64_t(resolution) * resolution;
    const unsigned gx = unsigned((per_view + kCapBlock - 1) / kCapBlock);
    hipLaunchKernelGGL(capture_kernel, dim3(gx, 8), dim3(kCapBlock), 0, st, d_prims, count, views, resolution, w.gpos,
                       w.gnrm, w.counts);
    hipLaunchKernelGGL(capture_scan_kernel, dim3(1), dim3(1024), 0, st, w.counts, int64_t(gx) * 8, w.offsets,
                       d_out_count);
    hipLaunchKernelGGL(capture_scatter_kernel, dim3(gx, 8), dim3(kCapBlock), 0, st, w.gpos, w.gnrm, resolution, ok,
                       w.offsets, d_out_points, d_out_normals, d_out_colors);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "capture launch: %s", hipGetErrorString(e));
    return BS_OK;
}

}  // extern "C"
