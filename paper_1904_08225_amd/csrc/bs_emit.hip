// bs_emit.hip -- the ordered surfel buffer and the prefix-length estimate.
//
// An approximation is one contiguous vertex buffer of surfels whose order
// makes every prefix a level of detail (paper Sec. 3).  emit_kernel gathers
// the ordered candidates into 20-byte records (the per-surfel size Table 1
// implies): position as binary32, normal as an octahedral code (two snorm16,
// the map of Meyer et al. 2010), colour as RGBA8.  The paper does not state
// the packing; these are this library's readings.
//
// Sec. 4.1 estimates the prefix length for a surfel radius r as
// p(r) = p_m (r_m / r)^2, where r_m is the median, over the first p_m
// ordered surfels, of each one's distance to its nearest other surfel in
// that prefix.  median_nn_kernel computes r_m in one workgroup: the prefix
// in LDS, all pairs, a bitonic sort of the distances in LDS.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bs_internal.h"

namespace bs {
namespace {

constexpr int kEmitBlock = 256;
constexpr int kNnBlock = 1024;

__device__ __forceinline__ float sq_dist(float ax, float ay, float az, float bx, float by, float bz) {
    const float dx = ax - bx, dy = ay - by, dz = az - bz;
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float s = xx + yy;
    return s + zz;
}

__device__ __forceinline__ int16_t to_snorm16(float v) {
    const float c = fminf(fmaxf(v, -1.f), 1.f);
    return int16_t(int(rintf(c * 32767.f)));
}

// Octahedral code: p = (x, y) / (|x| + |y| + |z|), folded over the diagonals
// for z < 0; (0, 0) for a zero or non-finite normal.
__device__ __forceinline__ uint32_t oct_code(float x, float y, float z) {
    const float ax = fabsf(x), ay = fabsf(y), az = fabsf(z);
    const float s = ax + ay;
    const float l1 = s + az;
    if (!(l1 > 0.f) || !isfinite(l1)) return 0u;
    float px = x / l1, py = y / l1;
    if (z < 0.f) {
        const float qx = (1.f - fabsf(py)) * (px >= 0.f ? 1.f : -1.f);
        const float qy = (1.f - fabsf(px)) * (py >= 0.f ? 1.f : -1.f);
        px = qx;
        py = qy;
    }
    return uint32_t(uint16_t(to_snorm16(px))) | (uint32_t(uint16_t(to_snorm16(py))) << 16);
}

__global__ void __launch_bounds__(kEmitBlock)
    emit_kernel(const float* __restrict__ pts, const float* __restrict__ nrm, const uint8_t* __restrict__ col,
                int64_t n, const int32_t* __restrict__ order, int64_t k, uint32_t* __restrict__ out) {
    const int64_t t = int64_t(blockIdx.x) * kEmitBlock + threadIdx.x;
    if (t >= k) return;
    const int64_t i = order[t];
    uint32_t w[5];
    if (i < 0 || i >= n) {
        const uint32_t qnan = 0x7FC00000u;
        w[0] = w[1] = w[2] = qnan;
        w[3] = 0u;
        w[4] = 0u;
    } else {
        w[0] = __float_as_uint(pts[3 * i + 0]);
        w[1] = __float_as_uint(pts[3 * i + 1]);
        w[2] = __float_as_uint(pts[3 * i + 2]);
        w[3] = nrm ? oct_code(nrm[3 * i + 0], nrm[3 * i + 1], nrm[3 * i + 2]) : 0u;
        w[4] = col ? (uint32_t(col[3 * i]) | (uint32_t(col[3 * i + 1]) << 8) | (uint32_t(col[3 * i + 2]) << 16) |
                      0xFF000000u)
                   : 0xFFFFFFFFu;
    }
    uint32_t* r = out + 5 * t;
#pragma unroll
    for (int j = 0; j < 5; ++j) r[j] = w[j];
}

__global__ void __launch_bounds__(kNnBlock)
    median_nn_kernel(const float* __restrict__ pts, int64_t n, const int32_t* __restrict__ order, int pm, int pow2,
                     float* __restrict__ out_rm) {
    __shared__ float sx[kMaxPrefixPm], sy[kMaxPrefixPm], sz[kMaxPrefixPm];
    __shared__ float nn[kMaxPrefixPm];
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int a = tid; a < pm; a += kNnBlock) {
        const int64_t i = order[a];
        if (i < 0 || i >= n) {  // an entry of a non-finite ordering: no estimate
            s_bad = 1;
            sx[a] = sy[a] = sz[a] = 0.f;
        } else {
            sx[a] = pts[3 * i + 0];
            sy[a] = pts[3 * i + 1];
            sz[a] = pts[3 * i + 2];
        }
    }
    __syncthreads();
    for (int a = tid; a < pow2; a += kNnBlock) {
        float m = INFINITY;
        if (a < pm) {
            const float ax = sx[a], ay = sy[a], az = sz[a];
            for (int b = 0; b < pm; ++b) {
                const float d = sq_dist(ax, ay, az, sx[b], sy[b], sz[b]);
                m = (b != a && d < m) ? d : m;
            }
            m = sqrtf(m);
        }
        nn[a] = m;  // padding sorts last
    }
    __syncthreads();
    // bitonic sort of nn[0 .. pow2) ascending
    for (int size = 2; size <= pow2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int a = tid; a < pow2; a += kNnBlock) {
                const int b = a ^ stride;
                if (b > a) {
                    const bool up = (a & size) == 0;
                    const float va = nn[a], vb = nn[b];
                    if ((va > vb) == up) {
                        nn[a] = vb;
                        nn[b] = va;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (tid == 0)
        *out_rm = s_bad ? __builtin_nanf("") : ((pm & 1) ? nn[pm / 2] : 0.5f * (nn[pm / 2 - 1] + nn[pm / 2]));
}

// Each of the first p ordered surfels' distance to its nearest other surfel
// of the prefix (Sec. 3.3): one thread per prefix surfel, the prefix staged
// through LDS a tile at a time.  Any order entry outside [0, n) makes every
// output NaN.
constexpr int kPnnBlock = 256;

__global__ void __launch_bounds__(kPnnBlock)
    prefix_nn_kernel(const float* __restrict__ pts, int64_t n, const int32_t* __restrict__ order, int p,
                     float* __restrict__ out) {
    __shared__ float tx[kPnnBlock], ty[kPnnBlock], tz[kPnnBlock];
    __shared__ int s_bad;
    const int a = blockIdx.x * kPnnBlock + threadIdx.x;
    if (threadIdx.x == 0) s_bad = 0;
    float ax = 0.f, ay = 0.f, az = 0.f;
    if (a < p) {
        const int64_t i = order[a];
        if (i >= 0 && i < n) {
            ax = pts[3 * i + 0];
            ay = pts[3 * i + 1];
            az = pts[3 * i + 2];
        }
    }
    float m = INFINITY;
    for (int base = 0; base < p; base += kPnnBlock) {
        __syncthreads();
        const int b = base + threadIdx.x;
        if (b < p) {
            const int64_t i = order[b];
            if (i < 0 || i >= n) {
                s_bad = 1;
                tx[threadIdx.x] = ty[threadIdx.x] = tz[threadIdx.x] = 0.f;
            } else {
                tx[threadIdx.x] = pts[3 * i + 0];
                ty[threadIdx.x] = pts[3 * i + 1];
                tz[threadIdx.x] = pts[3 * i + 2];
            }
        }
        __syncthreads();
        const int cnt = p - base < kPnnBlock ? p - base : kPnnBlock;
        for (int j = 0; j < cnt; ++j) {
            const float d = sq_dist(ax, ay, az, tx[j], ty[j], tz[j]);
            m = (base + j != a && d < m) ? d : m;
        }
    }
    __syncthreads();
    if (a < p) out[a] = s_bad ? __builtin_nanf("") : sqrtf(m);
}

}  // namespace

hipError_t launch_prefix_nn(const float* pts, int64_t n, const int32_t* order, int p, float* out, hipStream_t st) {
    if (p < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(prefix_nn_kernel, dim3((p + kPnnBlock - 1) / kPnnBlock), dim3(kPnnBlock), 0, st, pts, n,
                       order, p, out);
    return hipGetLastError();
}

hipError_t launch_emit(const float* pts, const float* nrm, const uint8_t* col, int64_t n, const int32_t* order,
                       int64_t k, void* out, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    const int64_t blocks = (k + kEmitBlock - 1) / kEmitBlock;
    hipLaunchKernelGGL(emit_kernel, dim3(unsigned(blocks)), dim3(kEmitBlock), 0, st, pts, nrm, col, n, order, k,
                       static_cast<uint32_t*>(out));
    return hipGetLastError();
}

hipError_t launch_median_nn(const float* pts, int64_t n, const int32_t* order, int pm, float* out_rm,
                            hipStream_t st) {
    if (pm < 2 || pm > kMaxPrefixPm) return hipErrorInvalidValue;
    int pow2 = 1;
    while (pow2 < pm) pow2 <<= 1;
    hipLaunchKernelGGL(median_nn_kernel, dim3(1), dim3(kNnBlock), 0, st, pts, n, order, pm, pow2, out_rm);
    return hipGetLastError();
}

}  // namespace bs
