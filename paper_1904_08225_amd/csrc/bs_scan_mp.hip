// bs_scan_mp.hip -- cooperative full scan with several exact picks per step.
//
// The greedy step (paper Sec. 3.2 / 3.3) appends the remaining candidate
// with the largest m, then lowers every m to its distance to the pick.  The
// order can be read ahead exactly: among the remaining candidates
// q_1 > q_2 > ... by key (value bits of m above the complemented original
// index, unique), q_j is the pick after q_1 .. q_{j-1} iff none of them
// lowers it and every other remaining key lies below it before the step.
//
// Design (MI355X): the candidates, in Morton order, stay in VGPRs of 256
// cooperative workgroups for the whole ordering; each wavefront holds 1,024
// consecutive ones, a compact region with a bounding box.  Every workgroup
// is a bucket: it publishes its two best keys (with coordinates and sorted
// positions) and the value bits R of its third best, which bound all its
// other keys.  Every workgroup reads all records and makes the same
// selection: with tau the fixed point of "tau <- max R over the workgroups
// holding an entry above tau" (from the top workgroup's R), the entries
// above tau (and the top) are exactly the prefix that the sequential rule
// accepts up to distance conflicts -- every member exceeds R of every
// workgroup with a member, and everything else lies below every member.
// Members are ranked among themselves, the first `picks` kept, and the
// first one that an earlier member lowers ends the step.  The next step
// applies all accepted picks at once, m <- min(m, d2(., q_1), ...), equal to
// the sequential updates because min is exact and order-free; a wavefront
// whose box no pick's ball reaches (binary32 box lower bound >= m of the
// pick, which bounds every remaining m at its step) skips the update and
// keeps its cached three best keys.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bs_grid.h"
#include "bs_grid_device.h"
#include "bs_internal.h"

namespace bs {
namespace {

constexpr uint32_t kMpSpinLimit = 1u << 21;  // bounded wait (about a second), then give up
constexpr int kMpRecStride = 16;              // words per exchange record
constexpr int kMpWords = 13;  // e1 hi, lo, x, y, z, pos; e2 hi, lo, x, y, z, pos; R
constexpr int kMpMaxPicks = 32;
constexpr int kMpMaxGroups = 256;

__device__ __forceinline__ void st_rec(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_rec(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ void dpp_top3_step(uint64_t& a1, uint64_t& a2, uint64_t& a3) {
    uint64_t b[3];
    const uint64_t a[3] = {a1, a2, a3};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(a[q])), CTRL, ROWS, 0xF, false));
        const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(a[q] >> 32)), CTRL, ROWS, 0xF, false));
        b[q] = (uint64_t(hi) << 32) | lo;
    }
    // the three largest of two descending triples (keys are unique; 0 = none)
    const bool x = a1 > b[0];
    const uint64_t c1 = x ? a1 : b[0];
    const uint64_t p = x ? a2 : a1, q = x ? b[0] : b[1];
    const bool y = p > q;
    const uint64_t c2 = y ? p : q;
    const uint64_t r1 = x ? (y ? a3 : a2) : (y ? a2 : a1);
    const uint64_t r2 = x ? (y ? b[0] : b[1]) : (y ? b[1] : b[2]);
    a1 = c1;
    a2 = c2;
    a3 = r1 > r2 ? r1 : r2;
}

__device__ __forceinline__ void insert3(uint64_t kk, uint64_t& a1, uint64_t& a2, uint64_t& a3) {
    const bool g1 = kk > a1, g2 = kk > a2, g3 = kk > a3;
    a3 = g2 ? a2 : (g3 ? kk : a3);
    a2 = g1 ? a1 : (g2 ? kk : a2);
    a1 = g1 ? kk : a1;
}

__device__ __forceinline__ uint64_t rl64(uint64_t v, int l) {
    return (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), l))) << 32) |
           uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), l));
}

// Points: lane l of wavefront w in workgroup g holds sorted positions
// g*BLOCK*P + w*64*P + j*64 + l, j < P.
template <int BLOCK, int P>
__global__ void __launch_bounds__(BLOCK)
    scan_mp_kernel(const float4* __restrict__ xyzm, const uint32_t* __restrict__ ids,
                   const int32_t* __restrict__ start_pos, int n, int k, int start, int32_t* __restrict__ order,
                   float* __restrict__ radius, const DevHeader* __restrict__ hdr, uint32_t* __restrict__ err,
                   uint64_t* __restrict__ slots, uint64_t* __restrict__ ticks, int max_picks) {
    constexpr int NW = BLOCK / 64;
    static_assert(kMpMaxPicks * kMpMaxPicks <= BLOCK, "one pair per thread");
    __shared__ uint64_t s_w[NW][3];                // per wavefront: its three best keys (cached)
    __shared__ float4 s_wc[NW][2];                 // and x, y, z, sorted position of the best two
    __shared__ uint64_t s_ek[2 * kMpMaxGroups];    // entries: keys (2 per workgroup)
    __shared__ float4 s_ec[2 * kMpMaxGroups];      // entries: x, y, z, sorted position
    __shared__ uint32_t s_er[kMpMaxGroups];        // per workgroup: R
    __shared__ float4 s_pk[kMpMaxPicks];           // picks by rank: x, y, z, m
    __shared__ uint32_t s_pid[kMpMaxPicks];        // original index
    __shared__ int s_ppos[kMpMaxPicks];            // sorted position
    __shared__ uint32_t s_id[P * BLOCK];           // original index of each held candidate
    __shared__ float s_z[P * BLOCK];               // and its z
    __shared__ int s_kfail, s_abort;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int G = int(gridDim.x);
    const int g = int(blockIdx.x);
    if (k <= 0) return;
    if (hdr->nonfinite) {
        for (int t = g * BLOCK + tid; t < k; t += G * BLOCK) {
            order[t] = -1;
            if (radius) radius[t] = __builtin_nanf("");
        }
        return;
    }
    const int cap_picks = max_picks < kMpMaxPicks ? max_picks : kMpMaxPicks;
    const int wbase = g * BLOCK * P + wave * 64 * P;

    float px[P], py[P], m[P];  // z in LDS: 16 candidates a thread fit 128 registers
    float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int i = wbase + j * 64 + lane;
        if (i < n) {
            const float4 q = xyzm[i];
            px[j] = q.x;
            py[j] = q.y;
            s_z[j * BLOCK + tid] = q.z;
            m[j] = INFINITY;
            s_id[j * BLOCK + tid] = ids[i];
            lx = fminf(lx, q.x); ly = fminf(ly, q.y); lz = fminf(lz, q.z);
            hx = fmaxf(hx, q.x); hy = fmaxf(hy, q.y); hz = fmaxf(hz, q.z);
        } else {
            px[j] = py[j] = 0.f;
            s_z[j * BLOCK + tid] = 0.f;
            m[j] = -1.f;  // padding: never selectable, min() keeps it at -1
            s_id[j * BLOCK + tid] = 0;
        }
    }
    // this wavefront's box (uniform)
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        lx = fminf(lx, __shfl_xor(lx, d, 64)); ly = fminf(ly, __shfl_xor(ly, d, 64));
        lz = fminf(lz, __shfl_xor(lz, d, 64)); hx = fmaxf(hx, __shfl_xor(hx, d, 64));
        hy = fmaxf(hy, __shfl_xor(hy, d, 64)); hz = fmaxf(hz, __shfl_xor(hz, d, 64));
    }
    if (lane == 0) {
        s_w[wave][0] = s_w[wave][1] = s_w[wave][2] = 0ull;
        s_wc[wave][0] = s_wc[wave][1] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (tid == 0) {
        const int sp = *start_pos;
        const float4 c = xyzm[sp];
        s_pk[0] = make_float4(c.x, c.y, c.z, INFINITY);
        s_pid[0] = uint32_t(start);
        s_ppos[0] = sp;
        s_abort = 0;
        if (g == 0) {
            order[0] = start;
            if (radius) radius[0] = INFINITY;
            if (ticks) ticks[0] = wall_clock64();
        }
    }
    __syncthreads();

    int t = 1;  // picks made
    int K = 1;  // picks of the previous step, in s_pk by rank
    for (uint32_t step = 1;; ++step) {
        const int buf = step & 1;
        // 1. the previous step's picks: the ones whose ball reaches this
        // wavefront's box lower m; the ones it owns become chosen
        bool reach = false, own = false;
        if (lane < K) {
            const float4 q = s_pk[lane];
            reach = box_lower(lx, ly, lz, hx, hy, hz, q.x, q.y, q.z) < q.w;
            const int off = s_ppos[lane] - wbase;
            own = off >= 0 && off < 64 * P;
        }
        const uint32_t rm = uint32_t(__ballot(reach)), om = uint32_t(__ballot(own));
        if ((rm | om) != 0u || step == 1) {  // step 1 fills every wavefront's cache
            for (uint32_t mm = rm; mm; mm &= mm - 1) {
                const float4 q = s_pk[__builtin_ctz(mm)];
#pragma unroll
                for (int j = 0; j < P; ++j) m[j] = fminf(m[j], dist2(px[j], py[j], s_z[j * BLOCK + tid], q.x, q.y, q.z));
            }
            for (uint32_t mm = om; mm; mm &= mm - 1) {
                const int off = s_ppos[__builtin_ctz(mm)] - wbase;
#pragma unroll
                for (int j = 0; j < P; ++j)
                    if (off == j * 64 + lane) m[j] = -1.f;
            }
            uint64_t a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
            for (int j = 0; j < P; ++j) insert3(m[j] >= 0.f ? make_key(m[j], s_id[j * BLOCK + tid]) : 0ull, a1, a2, a3);
            dpp_top3_step<0xB1, 0xF>(a1, a2, a3);
            dpp_top3_step<0x4E, 0xF>(a1, a2, a3);
            dpp_top3_step<0x141, 0xF>(a1, a2, a3);
            dpp_top3_step<0x140, 0xF>(a1, a2, a3);
            dpp_top3_step<0x142, 0xA>(a1, a2, a3);
            dpp_top3_step<0x143, 0xC>(a1, a2, a3);
            const uint64_t w1 = rl64(a1, 63), w2 = rl64(a2, 63), w3 = rl64(a3, 63);
#pragma unroll
            for (int j = 0; j < P; ++j) {
                // keys are unique: compare the value first, the index only then
                const uint32_t vb = __float_as_uint(m[j]);
                const bool h1 = m[j] >= 0.f && vb == uint32_t(w1 >> 32) && w1 != 0;
                const bool h2 = m[j] >= 0.f && vb == uint32_t(w2 >> 32) && w2 != 0;
                if (h1 || h2) {
                    const uint64_t kk = make_key(m[j], s_id[j * BLOCK + tid]);
                    if (kk == w1 || kk == w2)
                        s_wc[wave][kk == w1 ? 0 : 1] =
                            make_float4(px[j], py[j], s_z[j * BLOCK + tid], __int_as_float(wbase + j * 64 + lane));
                }
            }
            if (lane == 0) {
                s_w[wave][0] = w1;
                s_w[wave][1] = w2;
                s_w[wave][2] = w3;
            }
        }
        __syncthreads();
        // 2. the workgroup's three best and the entries of its record
        uint64_t v1 = lane < NW ? s_w[lane][0] : 0ull, v2 = lane < NW ? s_w[lane][1] : 0ull,
                 v3 = lane < NW ? s_w[lane][2] : 0ull;
        dpp_top3_step<0xB1, 0xF>(v1, v2, v3);
        dpp_top3_step<0x4E, 0xF>(v1, v2, v3);
        dpp_top3_step<0x141, 0xF>(v1, v2, v3);
        dpp_top3_step<0x140, 0xF>(v1, v2, v3);  // every lane of row 0 holds the result
        const uint64_t e1 = rl64(v1, 0), e2 = rl64(v2, 0);
        const uint32_t rg = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v3 >> 32)), 0));
        // 3. publish this workgroup's record, read every record
        const uint64_t tag = uint64_t(step) << 32;
        if (tid == 0) {
            float4 x1 = make_float4(0.f, 0.f, 0.f, 0.f), x2 = x1;
            for (int w = 0; w < NW; ++w) {
                if (e1 != 0 && s_w[w][0] == e1) x1 = s_wc[w][0];
                if (e1 != 0 && s_w[w][1] == e1) x1 = s_wc[w][1];
                if (e2 != 0 && s_w[w][0] == e2) x2 = s_wc[w][0];
                if (e2 != 0 && s_w[w][1] == e2) x2 = s_wc[w][1];
            }
            uint64_t* rec = slots + (size_t(buf) * G + g) * kMpRecStride;
            st_rec(rec + 0, tag | uint32_t(e1 >> 32));
            st_rec(rec + 1, tag | uint32_t(e1));
            st_rec(rec + 2, tag | __float_as_uint(x1.x));
            st_rec(rec + 3, tag | __float_as_uint(x1.y));
            st_rec(rec + 4, tag | __float_as_uint(x1.z));
            st_rec(rec + 5, tag | __float_as_uint(x1.w));
            st_rec(rec + 6, tag | uint32_t(e2 >> 32));
            st_rec(rec + 7, tag | uint32_t(e2));
            st_rec(rec + 8, tag | __float_as_uint(x2.x));
            st_rec(rec + 9, tag | __float_as_uint(x2.y));
            st_rec(rec + 10, tag | __float_as_uint(x2.z));
            st_rec(rec + 11, tag | __float_as_uint(x2.w));
            st_rec(rec + 12, tag | rg);
        }
        if (wave * 64 < G) {
            const int r = tid;
            bool ok = r >= G;
            bool aborted = false;
            uint32_t w[kMpWords];  // low words; the high word of each is the step
#pragma unroll
            for (int q = 0; q < kMpWords; ++q) w[q] = 0;
            const uint64_t* rec = slots + (size_t(buf) * G + (r < G ? r : 0)) * kMpRecStride;
            uint32_t spins = 0;
            while (true) {
                if (!ok) {
                    uint32_t all_and = ~0u, all_or = 0;
#pragma unroll
                    for (int q = 0; q < kMpWords; ++q) {
                        const uint64_t v = ld_rec(rec + q);
                        w[q] = uint32_t(v);
                        all_and &= uint32_t(v >> 32);
                        all_or |= uint32_t(v >> 32);
                    }
                    ok = all_and == step && all_or == step;
                }
                if (__ballot(!ok) == 0) break;
                if (++spins > kMpSpinLimit) {
                    aborted = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (r < G) {
                s_ek[2 * r] = (uint64_t(w[0]) << 32) | w[1];
                s_ec[2 * r] = make_float4(__uint_as_float((w[2])), __uint_as_float((w[3])),
                                          __uint_as_float((w[4])), __uint_as_float((w[5])));
                s_ek[2 * r + 1] = (uint64_t(w[6]) << 32) | w[7];
                s_ec[2 * r + 1] = make_float4(__uint_as_float((w[8])), __uint_as_float((w[9])),
                                              __uint_as_float((w[10])), __uint_as_float((w[11])));
                s_er[r] = w[12];
            }
            if (aborted && lane == 0) {
                s_abort = 1;
                atomicOr(err, 1u);
            }
        }
        if (tid == 0) s_kfail = kMpMaxPicks;
        __syncthreads();
        if (s_abort) return;

        // 4. the accepted set: tau from the top workgroup's R up to its fixed
        // point; members ranked among themselves, the first `cap` published
        const int cap = min(cap_picks, k - t);
        const int ne = 2 * G;
        uint64_t top = 0;
        int topw = 0;
        for (int e = lane; e < ne; e += 64) {
            const uint64_t kk = s_ek[e];
            if (kk > top) {
                top = kk;
                topw = e >> 1;
            }
        }
        {
            uint64_t tk = top;
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) {
                const uint32_t lo = uint32_t(__shfl_xor(int(uint32_t(tk)), d, 64));
                const uint32_t hi = uint32_t(__shfl_xor(int(uint32_t(tk >> 32)), d, 64));
                const uint64_t o = (uint64_t(hi) << 32) | lo;
                tk = o > tk ? o : tk;
            }
            const int tl = __builtin_ctzll(__ballot(top == tk) | (1ull << 63));
            topw = __builtin_amdgcn_readlane(topw, tl);
            top = tk;
        }
        uint32_t tau = s_er[topw];
        for (int it = 0; it <= kMpMaxGroups; ++it) {  // tau strictly rises through R values: ends in time
            uint32_t mr = 0;
            for (int e = lane; e < ne; e += 64) {
                const uint64_t kk = s_ek[e];
                if (kk != 0 && uint32_t(kk >> 32) > tau) mr = max(mr, s_er[e >> 1]);
            }
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) mr = max(mr, uint32_t(__shfl_xor(int(mr), d, 64)));
            if (mr <= tau) break;
            tau = mr;
        }
        int na = 0;
        for (int e0 = 0; e0 < ne; e0 += 64) {
            const int e = e0 + lane;
            const uint64_t kk = e < ne ? s_ek[e] : 0ull;
            const bool mem = kk != 0 && (kk == top || uint32_t(kk >> 32) > tau);
            const uint64_t mm0 = __ballot(mem);
            const int pos = na + __popcll(mm0 & ((1ull << lane) - 1));
            na += __popcll(mm0);
            for (uint64_t mm = __ballot(mem && (pos % NW) == wave); mm; mm &= mm - 1) {
                const int lc = __builtin_ctzll(mm);
                const uint64_t kc = rl64(kk, lc);
                int rank = 0;
                for (int f0 = 0; f0 < ne; f0 += 64) {
                    const int f = f0 + lane;
                    const uint64_t kf = f < ne ? s_ek[f] : 0ull;
                    const bool mf = kf != 0 && (kf == top || uint32_t(kf >> 32) > tau);
                    rank += __popcll(__ballot(mf && kf > kc));
                }
                if (rank < cap && lane == 0) {
                    const float4 c = s_ec[e0 + lc];
                    s_pk[rank] = make_float4(c.x, c.y, c.z, key_value(kc));
                    s_pid[rank] = key_id(kc);
                    s_ppos[rank] = __float_as_int(c.w);
                }
            }
        }
        const int nr = min(na, cap);
        __syncthreads();
        // 5. distance conflicts: thread (j, i) tests member j against i < j
        {
            const int j = tid / kMpMaxPicks, i = tid % kMpMaxPicks;
            if (j < nr && i < j) {
                const float4 cj = s_pk[j], ci = s_pk[i];
                if (dist2(cj.x, cj.y, cj.z, ci.x, ci.y, ci.z) < cj.w) atomicMin(&s_kfail, j);
            }
        }
        __syncthreads();
        K = min(s_kfail, nr);
        if (g == 0 && tid < K) {
            order[t + tid] = int32_t(s_pid[tid]);
            if (radius) radius[t + tid] = sqrtf(s_pk[tid].w);
            if (ticks) ticks[t + tid] = wall_clock64();
        }
        t += K;
        if (t >= k || K <= 0) break;
    }
}

using ScanMpFn = void (*)(const float4*, const uint32_t*, const int32_t*, int, int, int, int32_t*, float*,
                          const DevHeader*, uint32_t*, uint64_t*, uint64_t*, int);

struct MpEntry {
    int per_thread;
    ScanMpFn fn;
};

const MpEntry kMpTable[] = {
    {4, scan_mp_kernel<1024, 4>},
    {8, scan_mp_kernel<1024, 8>},
    {12, scan_mp_kernel<1024, 12>},
    {16, scan_mp_kernel<1024, 16>},
};

__global__ void clear_mp_slots_kernel(uint64_t* slots, int nwords) {
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) st_rec(slots + i, 0);
}

}  // namespace

bool scan_several_supported(const ScanShape& s) {
    if (s.block != 1024 || s.groups <= 1 || s.groups > kMpMaxGroups) return false;
    for (const MpEntry& e : kMpTable)
        if (e.per_thread == s.per_thread) return true;
    return false;
}

hipError_t launch_scan_several(const ScanShape& s, const float* pts, int n, int k, int start, int32_t* order,
                               float* radius, void* ws, uint64_t* ticks, int picks, hipStream_t st,
                               const KernelEvents* ev) {
    ScanMpFn fn = nullptr;
    for (const MpEntry& e : kMpTable)
        if (e.per_thread == s.per_thread) fn = e.fn;
    if (!fn || !scan_several_supported(s)) return hipErrorInvalidValue;
    SortedPoints sp{};
    hipError_t e = launch_sorted_points(pts, n, start, ws, st, &sp);
    if (e != hipSuccess) return e;
    uint64_t* slots = static_cast<uint64_t*>(sp.slots);
    hipLaunchKernelGGL(clear_mp_slots_kernel, dim3(1), dim3(256), 0, st, slots, 2 * s.groups * kMpRecStride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && ev->begin && (e = hipEventRecord(ev->begin, st)) != hipSuccess) return e;
    const float4* xyzm = sp.xyzm;
    const uint32_t* ids = sp.ids;
    const int32_t* start_pos = sp.start_pos;
    const DevHeader* hdr = sp.hdr;
    uint32_t* err = &sp.hdr->error;
    void* args[] = {(void*)&xyzm,  (void*)&ids,   (void*)&start_pos, (void*)&n,     (void*)&k,
                    (void*)&start, (void*)&order, (void*)&radius,    (void*)&hdr,   (void*)&err,
                    (void*)&slots, (void*)&ticks, (void*)&picks};
    e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(fn), dim3(s.groups), dim3(s.block), args, 0, st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess && ev && ev->end) e = hipEventRecord(ev->end, st);
    return e;
}

}  // namespace bs
