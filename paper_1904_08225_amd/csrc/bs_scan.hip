// bs_scan.hip -- resident full-scan greedy permutation kernels for gfx950.
//
// The greedy permutation of the paper (Sec. 3.2 progressive sampling,
// Sec. 3.3 greedy permutation): after choosing c_t, every remaining
// candidate's nearest-chosen squared distance becomes
// min(m_i, d2(p_i, p_{c_t})), and c_{t+1} is the remaining candidate with the
// largest m_i (lowest index on ties).
//
// Design (MI355X): the candidates and their m_i stay in VGPRs for the whole
// ordering (each thread owns `P` candidates, 16 bytes each, so one CU holds
// 16K candidates and 256 CUs hold 4M).  One fused pass per step updates m_i
// and tracks the thread's best (m_i, index) together with its coordinates;
// a 64-bit key  (bits(m) << 32) | (0x7FFFFFFF - index)  turns "largest m,
// then lowest index" into a plain unsigned maximum, reduced with DPP inside
// the wavefront and through LDS across wavefronts.  With several
// workgroups, each publishes its winner (key + coordinates) into a
// double-buffered record of tagged 64-bit words written and polled with
// relaxed device-scope atomics (one hop, no fences: every word carries the
// full step tag it belongs to), and every workgroup reduces all records.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bs_internal.h"

namespace bs {
namespace {

// Exchange record: five 64-bit words, each (step tag << 32) | 32-bit payload:
// key high, key low, x, y, z.  A reader accepts a record only when all five
// carry the current step's tag, so words of different steps (relaxed stores
// may become visible in any order) are never combined.
constexpr int kRecWords = 8;

// Squared distance with the fixed association ((dx*dx + dy*dy) + dz*dz).
__device__ __forceinline__ float dist2(float ax, float ay, float az, float bx, float by,
                                       float bz) {
    const float dx = ax - bx;
    const float dy = ay - by;
    const float dz = az - bz;
    const float xx = dx * dx;
    const float yy = dy * dy;
    const float zz = dz * dz;
    const float s = xx + yy;
    return s + zz;
}

// Selection key: larger m first, then lower index.  m >= +0 here, so its
// bit pattern orders like an unsigned integer.  0 means "no live candidate".
__device__ __forceinline__ uint64_t make_key(float m, uint32_t idx) {
    return (uint64_t(__float_as_uint(m)) << 32) | uint64_t(0x7FFFFFFFu - idx);
}
__device__ __forceinline__ uint32_t key_index(uint64_t key) {
    return 0x7FFFFFFFu - uint32_t(key & 0x7FFFFFFFull);
}
__device__ __forceinline__ float key_value(uint64_t key) {
    return __uint_as_float(uint32_t(key >> 32));
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_max_step(uint64_t v) {
    const int lo = int(uint32_t(v));
    const int hi = int(uint32_t(v >> 32));
    const uint32_t olo = uint32_t(__builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false));
    const uint32_t ohi = uint32_t(__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false));
    const uint64_t o = (uint64_t(ohi) << 32) | olo;
    return o > v ? o : v;
}

// Unsigned 64-bit maximum over the 64 lanes of a wavefront (uniform result).
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
    v = dpp_max_step<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = dpp_max_step<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = dpp_max_step<0x141, 0xF>(v);  // row_half_mirror
    v = dpp_max_step<0x140, 0xF>(v);  // row_mirror: every lane holds its row's max
    v = dpp_max_step<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_max_step<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3: lane 63 = max
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), 63));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), 63));
    return (uint64_t(hi) << 32) | lo;
}

__device__ __forceinline__ void st_dev(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_dev(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t ord_encode(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Candidates with non-finite coordinates make the whole result invalid.
__device__ void write_invalid(int32_t* order, float* radius, int k, int first, int stride) {
    for (int t = first; t < k; t += stride) {
        order[t] = -1;
        if (radius) radius[t] = __builtin_nanf("");
    }
}

__global__ void init_header_kernel(DevHeader* hdr) {
    // word layout: nonfinite, error, bbox min x,y,z (start at all-ones), bbox max x,y,z, pad
    const int tid = threadIdx.x;
    if (tid < 64) {
        uint32_t* w = reinterpret_cast<uint32_t*>(hdr);
        w[tid] = (tid >= 2 && tid < 5) ? 0xFFFFFFFFu : 0u;
    }
}

// A bounded wait gave up: the outputs are partly written, so all of them
// become order = -2, radius = NaN.  Nothing to do otherwise.
__global__ void finish_kernel(const DevHeader* __restrict__ hdr, int32_t* __restrict__ order,
                              float* __restrict__ radius, int k) {
    if (__hip_atomic_load(&hdr->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < k; t += gridDim.x * blockDim.x) {
        order[t] = -2;
        if (radius) radius[t] = __builtin_nanf("");
    }
}

__global__ void clear_slots_kernel(uint64_t* slots, int nslots) {
    for (int i = threadIdx.x; i < nslots; i += blockDim.x) st_dev(slots + i, 0);
}

__global__ void validate_kernel(const float* __restrict__ pts, int64_t n, DevHeader* hdr) {
    const int64_t total = 3 * n;
    uint32_t bad = 0;
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    uint32_t hi[3] = {0, 0, 0};
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        for (int a = 0; a < 3; ++a) {
            const float v = pts[3 * i + a];
            bad |= isfinite(v) ? 0u : 1u;
            const uint32_t e = ord_encode(v);
            lo[a] = min(lo[a], e);
            hi[a] = max(hi[a], e);
        }
    }
    (void)total;
    // wave, then workgroup reduction: one set of atomics per workgroup
    __shared__ uint32_t s_red[4][7];
    const int w = threadIdx.x >> 6;
    const bool any_bad = __any(bad);
    uint32_t v[6];
    for (int a = 0; a < 3; ++a) {
        uint32_t l = lo[a], h = hi[a];
        for (int off = 32; off > 0; off >>= 1) {
            l = min(l, uint32_t(__shfl_xor(int(l), off, 64)));
            h = max(h, uint32_t(__shfl_xor(int(h), off, 64)));
        }
        v[a] = l;
        v[3 + a] = h;
    }
    if ((threadIdx.x & 63) == 0) {
        for (int a = 0; a < 6; ++a) s_red[w][a] = v[a];
        s_red[w][6] = any_bad ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = int(blockDim.x) >> 6;
        for (int j = 1; j < nw; ++j) {
            for (int a = 0; a < 3; ++a) {
                v[a] = min(v[a], s_red[j][a]);
                v[3 + a] = max(v[3 + a], s_red[j][3 + a]);
            }
            s_red[0][6] |= s_red[j][6];
        }
        if (s_red[0][6]) atomicOr(&hdr->nonfinite, 1u);
        for (int a = 0; a < 3; ++a) {
            atomicMin(&hdr->bbox[a], v[a]);
            atomicMax(&hdr->bbox[3 + a], v[3 + a]);
        }
    }
}

// Persistent resident scan.  Workgroup g owns candidates
// [g*BLOCK*P, (g+1)*BLOCK*P); thread `tid` owns g*BLOCK*P + j*BLOCK + tid.
// It makes picks 0 .. k_stop-1 of a k-pick ordering.  With k_stop < k it
// hands the ordering over: m_out[i] receives every candidate's m after the
// updates of picks 0 .. k_stop-2 (-1 for chosen ones, pick k_stop-1
// included), and handoff[0], handoff[1] the last pick's index and the bits
// of its m (its update is left to the next kernel).
template <int BLOCK, int P, bool MULTI>
__global__ void __launch_bounds__(BLOCK)
    scan_kernel(const float* __restrict__ pts, int n, int k, int start,
                int32_t* __restrict__ order, float* __restrict__ radius,
                DevHeader* __restrict__ hdr, uint64_t* __restrict__ slots,
                uint64_t* __restrict__ ticks, int k_stop, float* __restrict__ m_out,
                uint32_t* __restrict__ handoff, uint32_t spin_limit) {
    constexpr int NW = BLOCK / 64;
    __shared__ uint64_t s_key[2][NW];
    __shared__ float s_pos[2][NW][4];
    __shared__ uint64_t s_part[2][NW];   // per-wavefront reduction of polled records
    __shared__ float s_ppos[2][NW][4];
    __shared__ int s_abort;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int G = MULTI ? int(gridDim.x) : 1;
    const int g = MULTI ? int(blockIdx.x) : 0;
    if (k <= 0) return;
    if (hdr->nonfinite) {
        write_invalid(order, radius, k, g * BLOCK + tid, G * BLOCK);
        return;
    }

    const int base = g * (BLOCK * P);
    float px[P], py[P], pz[P], m[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int i = base + j * BLOCK + tid;
        if (i < n) {
            px[j] = pts[3 * i + 0];
            py[j] = pts[3 * i + 1];
            pz[j] = pts[3 * i + 2];
            m[j] = INFINITY;
        } else {
            px[j] = py[j] = pz[j] = 0.f;
            m[j] = -1.f;  // padding: never selectable, and min() keeps it at -1
        }
    }

    int c = start;
    float cx = pts[3 * c + 0], cy = pts[3 * c + 1], cz = pts[3 * c + 2];
    {
        const int off = c - base;
        if (off >= 0 && off < BLOCK * P && (off % BLOCK) == tid) {
            const int jj = off / BLOCK;
#pragma unroll
            for (int j = 0; j < P; ++j)
                if (j == jj) m[j] = -1.f;
        }
    }
    if (g == 0 && tid == 0) {
        order[0] = c;
        if (radius) radius[0] = INFINITY;
        if (ticks) ticks[0] = wall_clock64();
    }
    if (tid == 0) s_abort = 0;
    __syncthreads();

    float cm = INFINITY;  // m of the latest pick
    for (int t = 1; t < k_stop; ++t) {
        const int buf = t & 1;
        // fused update + thread-local argmax
        float bv = -1.f, bx = 0.f, by = 0.f, bz = 0.f;
        int bj = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const float d = dist2(px[j], py[j], pz[j], cx, cy, cz);
            m[j] = fminf(m[j], d);
            const bool better = m[j] > bv;
            bv = better ? m[j] : bv;
            bj = better ? j : bj;
            bx = better ? px[j] : bx;
            by = better ? py[j] : by;
            bz = better ? pz[j] : bz;
        }
        const uint64_t key = bv >= 0.f ? make_key(bv, uint32_t(base + bj * BLOCK + tid)) : 0ull;
        const uint64_t wk = wave_max_u64(key);
        if (wk != 0 && key == wk) {
            s_key[buf][wave] = wk;
            s_pos[buf][wave][0] = bx;
            s_pos[buf][wave][1] = by;
            s_pos[buf][wave][2] = bz;
        }
        if (wk == 0 && lane == 0) s_key[buf][wave] = 0;
        __syncthreads();

        uint64_t best = 0;
        int bw = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint64_t kk = s_key[buf][w];
            if (kk > best) {
                best = kk;
                bw = w;
            }
        }
        float ncx = s_pos[buf][bw][0], ncy = s_pos[buf][bw][1], ncz = s_pos[buf][bw][2];

        if constexpr (MULTI) {
            // publish this workgroup's winner, then every wavefront polls up
            // to 64 records (one per lane) and reduces them
            const uint64_t tag = uint64_t(uint32_t(t)) << 32;
            if (tid == 0) {
                uint64_t* rec = slots + (size_t(buf) * G + g) * kRecWords;
                st_dev(rec + 0, tag | uint32_t(best >> 32));
                st_dev(rec + 1, tag | uint32_t(best));
                st_dev(rec + 2, tag | __float_as_uint(ncx));
                st_dev(rec + 3, tag | __float_as_uint(ncy));
                st_dev(rec + 4, tag | __float_as_uint(ncz));
            }
            if (wave * 64 < G) {
                const int r = tid;
                bool ok = r >= G;
                bool aborted = false;
                uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0;
                uint32_t spins = 0;
                const uint64_t* rec = slots + (size_t(buf) * G + (r < G ? r : 0)) * kRecWords;
                while (true) {
                    if (!ok) {
                        w0 = ld_dev(rec + 0);
                        w1 = ld_dev(rec + 1);
                        w2 = ld_dev(rec + 2);
                        w3 = ld_dev(rec + 3);
                        w4 = ld_dev(rec + 4);
                        ok = ((w0 & w1 & w2 & w3 & w4) >> 32) == uint64_t(uint32_t(t)) &&
                             ((w0 | w1 | w2 | w3 | w4) >> 32) == uint64_t(uint32_t(t));
                    }
                    if (__ballot(!ok) == 0) break;
                    if (++spins > spin_limit) {
                        aborted = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                const uint64_t kk = (r < G) ? ((w0 << 32) | (w1 & 0xFFFFFFFFull)) : 0ull;
                const uint64_t pk = wave_max_u64(kk);
                if (pk != 0 && kk == pk) {
                    s_ppos[buf][wave][0] = __uint_as_float(uint32_t(w2));
                    s_ppos[buf][wave][1] = __uint_as_float(uint32_t(w3));
                    s_ppos[buf][wave][2] = __uint_as_float(uint32_t(w4));
                }
                if (lane == 0) {
                    s_part[buf][wave] = pk;
                    if (aborted) {
                        s_abort = 1;
                        atomicOr(&hdr->error, 1u);
                    }
                }
            }
            __syncthreads();
            if (s_abort) return;
            best = 0;
            bw = 0;
            const int nparts = (G + 63) / 64;
            for (int w = 0; w < nparts; ++w) {
                const uint64_t kk = s_part[buf][w];
                if (kk > best) {
                    best = kk;
                    bw = w;
                }
            }
            ncx = s_ppos[buf][bw][0];
            ncy = s_ppos[buf][bw][1];
            ncz = s_ppos[buf][bw][2];
        }

        c = int(key_index(best));
        cm = key_value(best);
        cx = ncx;
        cy = ncy;
        cz = ncz;
        {
            const int off = c - base;
            if (off >= 0 && off < BLOCK * P && (off % BLOCK) == tid) {
                const int jj = off / BLOCK;
#pragma unroll
                for (int j = 0; j < P; ++j)
                    if (j == jj) m[j] = -1.f;
            }
        }
        if (g == 0 && tid == 0) {
            order[t] = c;
            if (radius) radius[t] = sqrtf(key_value(best));
            if (ticks) ticks[t] = wall_clock64();
        }
    }
    if (m_out) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int i = base + j * BLOCK + tid;
            if (i < n) m_out[i] = m[j];
        }
    }
    if (handoff && g == 0 && tid == 0) {
        handoff[0] = uint32_t(c);
        handoff[1] = __float_as_uint(cm);
    }
}

using ScanFn = void (*)(const float*, int, int, int, int32_t*, float*, DevHeader*, uint64_t*,
                       uint64_t*, int, float*, uint32_t*, uint32_t);

struct ScanEntry {
    int block, per_thread;
    ScanFn single, multi;
};

#define BS_SCAN_ENTRY(B, PP) \
    {B, PP, scan_kernel<B, PP, false>, scan_kernel<B, PP, true>}

const ScanEntry kScanTable[] = {
    BS_SCAN_ENTRY(1024, 1), BS_SCAN_ENTRY(1024, 2), BS_SCAN_ENTRY(1024, 4),
    BS_SCAN_ENTRY(1024, 8), BS_SCAN_ENTRY(1024, 12), BS_SCAN_ENTRY(1024, 16),
    BS_SCAN_ENTRY(512, 24), BS_SCAN_ENTRY(512, 32),
};

const ScanEntry* find_entry(int block, int pt) {
    for (const ScanEntry& e : kScanTable)
        if (e.block == block && e.per_thread == pt) return &e;
    return nullptr;
}

}  // namespace

bool scan_shape_supported(int block, int per_thread) {
    return find_entry(block, per_thread) != nullptr;
}

bool choose_scan_shape(int64_t n, int cus, int want_block, int want_pt, int want_groups,
                       ScanShape* out) {
    if (n < 1) return false;
    if (want_block > 0 || want_pt > 0) {
        const int b = want_block > 0 ? want_block : 1024;
        const int p = want_pt > 0 ? want_pt : 16;
        if (!scan_shape_supported(b, p)) return false;
        const int64_t cap = int64_t(b) * p;
        int64_t g = (n + cap - 1) / cap;
        if (want_groups > 0) {
            if (int64_t(want_groups) < g) return false;
            g = want_groups;
        }
        if (g > kMaxCoopGroups || g > b) return false;
        *out = ScanShape{b, p, int(g)};
        return true;
    }
    // Automatic: one workgroup while it holds n; otherwise the smallest
    // per-thread count whose cooperative grid fits one workgroup per CU.
    for (const ScanEntry& e : kScanTable) {
        if (e.block == 1024 && int64_t(e.block) * e.per_thread >= n) {
            if (want_groups > 1) break;
            *out = ScanShape{e.block, e.per_thread, 1};
            return true;
        }
    }
    for (const ScanEntry& e : kScanTable) {
        if (e.block != 1024) continue;
        const int64_t cap = int64_t(e.block) * e.per_thread;
        const int64_t g = (n + cap - 1) / cap;
        if (e.per_thread >= 4 && g <= cus && g <= e.block) {
            *out = ScanShape{e.block, e.per_thread, int(g)};
            return true;
        }
    }
    return false;
}

size_t scan_slot_bytes(int groups) { return align_up(size_t(2) * size_t(groups > 0 ? groups : 1) * kRecWords * 8); }

size_t scan_workspace_bytes(const ScanShape& s) { return align_up(sizeof(DevHeader)) + scan_slot_bytes(s.groups); }

hipError_t launch_init_header(DevHeader* hdr, hipStream_t st) {
    hipLaunchKernelGGL(init_header_kernel, dim3(1), dim3(64), 0, st, hdr);
    return hipGetLastError();
}

hipError_t launch_finish(const DevHeader* hdr, int32_t* order, float* radius, int k, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    int blocks = (k + 255) / 256;
    if (blocks > 256) blocks = 256;
    hipLaunchKernelGGL(finish_kernel, dim3(blocks), dim3(256), 0, st, hdr, order, radius, k);
    return hipGetLastError();
}

hipError_t launch_validate(const float* pts, int64_t n, DevHeader* hdr, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(validate_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, pts, n, hdr);
    return hipGetLastError();
}

hipError_t launch_scan(const ScanShape& s, const float* pts, int n, int k, int start,
                       int32_t* order, float* radius, DevHeader* hdr, void* scratch,
                       uint64_t* ticks, hipStream_t st, const LaunchOpts* ev, int k_stop,
                       float* m_out, uint32_t* handoff) {
    const ScanEntry* e = find_entry(s.block, s.per_thread);
    if (!e) return hipErrorInvalidValue;
    if (k_stop < 0 || k_stop > k) k_stop = k;
    uint64_t* slots = reinterpret_cast<uint64_t*>(scratch);
    uint32_t spin = spin_limit_of(ev);
    hipError_t err = hipSuccess;
    if (s.groups <= 1) {
        if (ev && ev->begin && (err = hipEventRecord(ev->begin, st)) != hipSuccess) return err;
        hipLaunchKernelGGL(e->single, dim3(1), dim3(s.block), 0, st, pts, n, k, start, order,
                           radius, hdr, slots, ticks, k_stop, m_out, handoff, spin);
    } else {
        // stale records from an earlier call must not carry matching tags
        hipLaunchKernelGGL(clear_slots_kernel, dim3(1), dim3(256), 0, st, slots, 2 * s.groups * kRecWords);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if (ev && ev->begin && (err = hipEventRecord(ev->begin, st)) != hipSuccess) return err;
        void* args[] = {(void*)&pts,   (void*)&n,     (void*)&k,      (void*)&start,
                        (void*)&order, (void*)&radius, (void*)&hdr,   (void*)&slots,
                        (void*)&ticks, (void*)&k_stop, (void*)&m_out, (void*)&handoff,
                        (void*)&spin};
        err = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(e->multi), dim3(s.groups),
                                         dim3(s.block), args, 0, st);
    }
    if (err == hipSuccess) err = hipGetLastError();
    if (err == hipSuccess && ev && ev->end) err = hipEventRecord(ev->end, st);
    // a cooperative wait may give up (a following kernel of a handoff checks
    // the error word itself and finishes the outputs)
    if (err == hipSuccess && s.groups > 1 && !handoff) err = launch_finish(hdr, order, radius, k, st);
    return err;
}

}  // namespace bs
