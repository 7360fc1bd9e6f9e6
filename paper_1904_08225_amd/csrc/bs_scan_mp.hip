// bs_scan_mp.hip -- cooperative full scan with several exact picks per step.
//
// The greedy step (paper Sec. 3.2 / 3.3) appends the remaining candidate
// with the largest m, then lowers every m to its distance to the pick.  The
// order can be read ahead exactly: among the remaining candidates
// q_1 > q_2 > ... by key (value bits of m above the complemented original
// index, unique), q_j is the pick after q_1 .. q_{j-1} iff none of them
// lowers it and every other remaining key lies below it before the step.
//
// Design (MI355X): the candidates, in Morton order, stay in VGPRs of up to
// 256 cooperative workgroups for the whole ordering; each wavefront holds
// 64*P consecutive ones in P slabs of 64, split into two groups where the
// Morton codes first differ, each group and each slab with a box.  Each
// wavefront keeps a chain: c1, its best key; c2, its best key once c1's ball
// has lowered the others (the value in c2's key includes that update); and
// the bound of all its other values once both are taken.  Every workgroup
// is a bucket: it publishes its E best chain keys (four or five, with coordinates and
// sorted positions) and value bits R that bound every value it does not
// offer (the largest chain key it keeps back, and every wavefront's bound
// after its chain: a wavefront's published keys are a prefix of its chain).
// Every workgroup reads all records and makes the same selection: with tau
// the fixed point of "tau <- max R over the workgroups holding an entry
// above tau" (from the top workgroup's R), the entries
// above tau (and the top) are exactly the prefix that the sequential rule
// accepts up to distance conflicts -- every member exceeds R of every
// workgroup with a member, and everything else lies below every member.
// Members are ranked among themselves, the first `picks` kept, and the
// first one that an earlier member lowers ends the step (an earlier key of
// the same chain never does: the chain value is at most that distance).
// The next step applies all accepted picks at once, m <- min(m, d2(., q_1), ...), equal to
// the sequential updates because min is exact and order-free; a group or
// slab whose box no pick's ball reaches (binary32 box lower bound >= m of the
// pick, which bounds every remaining m at its step) skips the update, and a
// wavefront where neither chain key's m changed keeps its cached chain.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bs_grid.h"
#include "bs_grid_device.h"
#include "bs_internal.h"

namespace bs {
namespace {

// Entries a workgroup offers per step: more entries let more of them clear
// tau (a workgroup's bound R is its first key kept back), but the member set
// to rank and test grows with them.  Four suit the kernels of up to 256
// picks per step (many workgroups), five the 128-pick ones (few workgroups,
// so few entries in all): 26.6 ms against 27.7 (five) and 30.8 before (three)
// on the 4,194,304-candidate part to 262,144; 3.3 ms against 3.9 (four) and
// 5.0 (three) on the 16,384-candidate sphere and box with 16 workgroups.
template <int MAXPICKS>
constexpr int mp_entries() { return MAXPICKS > 128 ? 4 : 5; }
constexpr int kMpMaxEntries = 5;
// An exchange record: three packed words per entry, then R, each word with a
// 2-bit step tag above 62 payload bits; one 128-byte line per record.
constexpr int kMpEntryWords = 3;
template <int E>
constexpr int mp_words() { return kMpEntryWords * E + 1; }
constexpr int kMpRecStride = 16;  // words per exchange record
static_assert(mp_words<kMpMaxEntries>() <= kMpRecStride, "a record fits its line");
constexpr uint64_t kMpPayload = (uint64_t(1) << 62) - 1u;
constexpr uint32_t kMpMaxPos = 1u << 22;  // sorted positions fit 22 bits (n <= 2^22)
// Most picks per step: 256, or 128 for a kernel with fewer passes of one
// lane per pick in the reach test and wider conflict columns (a step's fixed
// cost is lower; with few workgroups, and so few entries, 128 never binds).
constexpr int kMpMaxPicks = 256;
constexpr int kMpMaxGroups = 256;

// A workgroup barrier ordering LDS only: within a step the workgroup's
// threads share nothing through global memory, so a barrier need not wait
// for the record and output stores still in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Wavefront maxima through DPP row operations (no LDS round trips): after
// the row steps every row holds its maximum, the two row broadcasts carry
// them to lane 63.  Lanes a step leaves unwritten read 0, the identity.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, dpp_u32<0xB1, 0xF>(v));
    v = max(v, dpp_u32<0x4E, 0xF>(v));
    v = max(v, dpp_u32<0x141, 0xF>(v));
    v = max(v, dpp_u32<0x140, 0xF>(v));
    v = max(v, dpp_u32<0x142, 0xA>(v));
    v = max(v, dpp_u32<0x143, 0xC>(v));
    return uint32_t(__builtin_amdgcn_readlane(int(v), 63));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_max_u64(uint64_t v) {
    const uint32_t lo = dpp_u32<CTRL, ROWS>(uint32_t(v)), hi = dpp_u32<CTRL, ROWS>(uint32_t(v >> 32));
    const uint64_t o = (uint64_t(hi) << 32) | lo;
    return o > v ? o : v;
}
// Sum over a row of 16 lanes, held by every lane of the row (swaps within
// pairs and quads, then the half-row and row mirrors: all permutations
// inside the row, so rows never mix and every source lane is active).
__device__ __forceinline__ int row_sum16(int v) {
    v += int(dpp_u32<0xB1, 0xF>(uint32_t(v)));
    v += int(dpp_u32<0x4E, 0xF>(uint32_t(v)));
    v += int(dpp_u32<0x141, 0xF>(uint32_t(v)));
    v += int(dpp_u32<0x140, 0xF>(uint32_t(v)));
    return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
    v = dpp_max_u64<0xB1, 0xF>(v);
    v = dpp_max_u64<0x4E, 0xF>(v);
    v = dpp_max_u64<0x141, 0xF>(v);
    v = dpp_max_u64<0x140, 0xF>(v);
    v = dpp_max_u64<0x142, 0xA>(v);
    v = dpp_max_u64<0x143, 0xC>(v);
    return (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), 63))) << 32) |
           uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), 63));
}

// A box the whole wavefront shares (held in scalar registers).
struct WaveBox {
    float lo[3], hi[3];
};
__device__ __forceinline__ float uniform_f32(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ float uniform_at(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ float wave_min_f32(float v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fminf(v, __shfl_xor(v, d, 64));
    return uniform_f32(v);
}
__device__ __forceinline__ float wave_max_f32(float v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    return uniform_f32(v);
}
// Binary32 lower bound of d2 from c to the box (+inf for an empty box).
__device__ __forceinline__ float wave_box_lower(const WaveBox& b, float cx, float cy, float cz) {
    return box_lower(b.lo[0], b.lo[1], b.lo[2], b.hi[0], b.hi[1], b.hi[2], cx, cy, cz);
}

// Set bits of a wavefront mask below this lane.
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return int(__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
}

// Entry e of the records (workgroup e / E, slot e % E),
// three packed words (payload bits only):
//   w0: value bits 0..30 of the key (m >= 0: the sign bit is 0), then the
//       31 bits of its complemented index;
//   w1: x, the sorted position (22 bits) from bit 32, z bits 0..7 from bit 54;
//   w2: y, z bits 8..31 from bit 32.
// Word mp_words<E>() - 1 of a workgroup's record is R.
template <int E>
__device__ __forceinline__ const uint64_t* rec_entry(const uint64_t* rw, int e) {
    return rw + (e / E) * mp_words<E>() + kMpEntryWords * (e % E);
}
template <int E>
__device__ __forceinline__ uint64_t rec_key(const uint64_t* rw, int e) {
    const uint64_t w0 = rec_entry<E>(rw, e)[0];
    return ((w0 & 0x7FFFFFFFull) << 32) | ((w0 >> 31) & 0x7FFFFFFFull);
}
// x, y, z and the sorted position (as the bits of w) of entry e.
template <int E>
__device__ __forceinline__ float4 rec_coords(const uint64_t* rw, int e) {
    const uint64_t* p = rec_entry<E>(rw, e);
    const uint64_t w1 = p[1], w2 = p[2];
    const uint32_t z = uint32_t((w1 >> 54) & 0xFFu) | (uint32_t(w2 >> 32) << 8);
    return make_float4(__uint_as_float(uint32_t(w1)), __uint_as_float(uint32_t(w2)), __uint_as_float(z),
                       __int_as_float(int((w1 >> 32) & (kMpMaxPos - 1u))));
}
template <int E>
__device__ __forceinline__ uint32_t rec_bound(const uint64_t* rw, int g) {
    return uint32_t(rw[g * mp_words<E>() + kMpEntryWords * E]);
}
// Word f of an entry from its key, coordinates and position (32-bit fields).
__device__ __forceinline__ uint64_t pack_entry_word(int f, uint32_t key_hi, uint32_t key_lo, uint32_t x, uint32_t y,
                                                    uint32_t z, uint32_t pos) {
    if (f == 0) return uint64_t(key_hi & 0x7FFFFFFFu) | (uint64_t(key_lo & 0x7FFFFFFFu) << 31);
    if (f == 1) return uint64_t(x) | (uint64_t(pos & (kMpMaxPos - 1u)) << 32) | (uint64_t(z & 0xFFu) << 54);
    return uint64_t(y) | (uint64_t(z >> 8) << 32);
}

__device__ __forceinline__ void st_rec(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_rec(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void insert3(uint64_t kk, uint64_t& a1, uint64_t& a2, uint64_t& a3) {
    const bool g1 = kk > a1, g2 = kk > a2, g3 = kk > a3;
    a3 = g2 ? a2 : (g3 ? kk : a3);
    a2 = g1 ? a1 : (g2 ? kk : a2);
    a1 = g1 ? kk : a1;
}

// The wavefront's largest key among per-slot values w (bits of the value
// plus one; 0 = none), given each lane's largest value vm, its slot jm and
// whether another slot of the lane ties it.  Usually one slot holds the
// largest value and only its original index is read; otherwise every slot
// with that value is compared by index (the lowest wins, as in the key).
// `value(j, 0)` recomputes slot j's w.  Returns key 0 when no slot is live.
struct BestKey {
    uint64_t key;
    int lane, slot;
};
template <int BLOCK, int P, class ValueFn>
__device__ __forceinline__ BestKey wave_best(uint32_t vm, int jm, bool tie, const uint32_t* ids, int lane,
                                             ValueFn value) {
    BestKey r{0ull, 0, 0};
    const uint32_t top = wave_max_u32(vm);
    if (top == 0u) return r;
    const uint64_t at = __ballot(vm == top);
    if (__popcll(at) == 1 && __ballot(vm == top && tie) == 0ull) {
        r.lane = __builtin_ctzll(at);
        r.slot = __builtin_amdgcn_readlane(jm, r.lane);
        r.key = (uint64_t(top - 1u) << 32) | (0x7FFFFFFFu - ids[r.slot * BLOCK + r.lane]);
        return r;
    }
    uint32_t bi = 0u;  // complemented index of this lane's best slot with the top value
    int bj = 0;
    // an opaque zero: the values are recomputed here rather than kept live
    // from the caller's loop (sixteen more registers)
    int z = 0;
    asm volatile("" : "+v"(z));
#pragma unroll
    for (int j = 0; j < P; ++j) {
        if (value(j, z) == top) {
            const uint32_t ni = 0x7FFFFFFFu - ids[j * BLOCK + lane];  // >= 1: indices are below 2^31 - 1
            bj = ni > bi ? j : bj;
            bi = ni > bi ? ni : bi;
        }
    }
    const uint32_t bl = wave_max_u32(bi);
    r.lane = __builtin_ctzll(__ballot(bi == bl));
    r.slot = __builtin_amdgcn_readlane(bj, r.lane);
    r.key = (uint64_t(top - 1u) << 32) | bl;
    return r;
}

// Points: lane l of wavefront w in workgroup g holds sorted positions
// g*BLOCK*P + w*64*P + j*64 + l, j < P.
template <int BLOCK, int P, int MAXPICKS>
__global__ void __launch_bounds__(BLOCK)
    scan_mp_kernel(const float4* __restrict__ xyzm, const uint32_t* __restrict__ ids,
                   const uint32_t* __restrict__ codes, const int32_t* __restrict__ start_pos, int n, int k, int start, int32_t* __restrict__ order,
                   float* __restrict__ radius, const DevHeader* __restrict__ hdr, uint32_t* __restrict__ err,
                   uint64_t* __restrict__ slots, uint64_t* __restrict__ ticks, int max_picks,
                   uint32_t spin_limit) {
    constexpr int NW = BLOCK / 64;
    constexpr int kMpEntries = mp_entries<MAXPICKS>();
    constexpr int kMpWords = mp_words<kMpEntries>();
    constexpr int kMpPickWords = MAXPICKS / 64;  // reach-test passes of 64 picks
    static_assert(MAXPICKS % 64 == 0 && MAXPICKS <= kMpMaxPicks && MAXPICKS <= BLOCK,
                  "passes of 64 picks; one emitting thread a pick");
    __shared__ __align__(16) uint64_t s_w[NW][2];  // per wavefront: its chain's two keys (cached)
    __shared__ uint32_t s_c3[NW];                  // and the bound after them (value bits)
    __shared__ uint32_t s_ent[6 * kMpEntries];     // the record's entry words, staged by rank
    __shared__ float4 s_wc[NW][2];                 // x, y, z, sorted position of each chain key
    __shared__ uint64_t s_rw[kMpMaxGroups * kMpWords];  // every workgroup's record (payload bits)
    __shared__ __align__(16) uint64_t s_mk[kMpEntries * kMpMaxGroups + 2];  // members: keys
    __shared__ int s_mi[kMpEntries * kMpMaxGroups];  // members: entry index
    __shared__ float4 s_pk[MAXPICKS];           // picks by rank: x, y, z, m
    __shared__ uint32_t s_pid[MAXPICKS];        // original index
    __shared__ int s_ppos[MAXPICKS];            // sorted position
    __shared__ uint32_t s_id[P * BLOCK];           // original index of each held candidate
    __shared__ float4 s_slo[NW][P], s_shi[NW][P];  // box of each slab of 64 (x, y, z; w unused)
    __shared__ float4 s_gb[NW][4];                 // boxes of the wavefront's two groups (lo, hi each)
    __shared__ int s_kfail, s_na, s_abort;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: addresses stay scalar
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
    const int cap_picks = max_picks < MAXPICKS ? max_picks : MAXPICKS;
    const int wbase = g * BLOCK * P + wave * 64 * P;

    float px[P], py[P], pz[P], m[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int i = wbase + j * 64 + lane;
        if (i < n) {
            const float4 q = xyzm[i];
            px[j] = q.x;
            py[j] = q.y;
            pz[j] = q.z;
            m[j] = INFINITY;
            s_id[j * BLOCK + tid] = ids[i];
        } else {
            px[j] = py[j] = pz[j] = 0.f;
            m[j] = -1.f;  // padding: never selectable, min() keeps it at -1
            s_id[j * BLOCK + tid] = 0;
        }
    }
    // The wavefront's candidates (positions p = j*64 + lane, Morton order)
    // form two groups, p < split and p >= split, split where the first and
    // last codes first differ: each group lies in one cell of the Morton tree,
    // so a wavefront across a large jump of the curve does not get one box
    // spanning both sides (which nearly every pick would reach).
    int split = 64 * P;
    {
        const int wn = min(64 * P, n - wbase);
        if (wn > 1) {
            const uint32_t c0 = codes[wbase], c1 = codes[wbase + wn - 1];
            if (c0 != c1) {
                const uint32_t bit = 1u << (31 - __builtin_clz(c0 ^ c1));
                int cnt = 0;
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const int i = wbase + j * 64 + lane;
                    cnt += __popcll(__ballot(i < n && (codes[i] & bit) == 0u));
                }
                split = __builtin_amdgcn_readfirstlane(cnt);  // sorted: the first cnt positions have the bit clear
            }
        }
    }
    // slabs of 64 positions holding group a / group b members (uniform)
    uint32_t slabs_a = 0u, slabs_b = 0u;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        if (j * 64 < split) slabs_a |= 1u << j;
        if ((j + 1) * 64 > split) slabs_b |= 1u << j;
    }
    slabs_a = __builtin_amdgcn_readfirstlane(slabs_a);
    slabs_b = __builtin_amdgcn_readfirstlane(slabs_b);
    // each slab's box (lane j of the reach test below tests slab j), from
    // the sorted points again so that the loop need not unroll
#pragma unroll 1
    for (int j = 0; j < P; ++j) {
        const int i = wbase + j * 64 + lane;
        const bool live = i < n;
        const float4 c = live ? xyzm[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float lx = wave_min_f32(live ? c.x : INFINITY), hx = wave_max_f32(live ? c.x : -INFINITY);
        const float ly = wave_min_f32(live ? c.y : INFINITY), hy = wave_max_f32(live ? c.y : -INFINITY);
        const float lz = wave_min_f32(live ? c.z : INFINITY), hz = wave_max_f32(live ? c.z : -INFINITY);
        if (lane == 0) {
            s_slo[wave][j] = make_float4(lx, ly, lz, 0.f);
            s_shi[wave][j] = make_float4(hx, hy, hz, 0.f);
        }
    }
    // boxes of the groups p < split, p >= split, in LDS (s_gb: lo, hi of
    // each), which keeps registers for the candidates
    {
        float lo[2][3], hi[2][3];
#pragma unroll
        for (int gi = 0; gi < 2; ++gi)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                lo[gi][d] = INFINITY;
                hi[gi][d] = -INFINITY;
            }
#pragma unroll
        for (int j = 0; j < P; ++j) {
            if (m[j] < 0.f) continue;  // padding
            const int gi = j * 64 + lane < split ? 0 : 1;
            const float c[3] = {px[j], py[j], pz[j]};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                lo[gi][d] = fminf(lo[gi][d], c[d]);
                hi[gi][d] = fmaxf(hi[gi][d], c[d]);
            }
        }
#pragma unroll
        for (int gi = 0; gi < 2; ++gi) {
            WaveBox b;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                b.lo[d] = wave_min_f32(lo[gi][d]);
                b.hi[d] = wave_max_f32(hi[gi][d]);
            }
            if (lane == 0) {
                s_gb[wave][2 * gi] = make_float4(b.lo[0], b.lo[1], b.lo[2], 0.f);
                s_gb[wave][2 * gi + 1] = make_float4(b.hi[0], b.hi[1], b.hi[2], 0.f);
            }
        }
    }
    if (lane == 0) {
        s_w[wave][0] = s_w[wave][1] = 0ull;
        s_c3[wave] = 0u;
        s_wc[wave][0] = s_wc[wave][1] = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
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
        // thread-derived values are recomputed every step from an opaque copy
        // of the thread index (a few VALU operations) instead of being kept
        // live across the loop next to the 64 registers of candidates, where
        // the compiler would spill them
        int tid_v = int(threadIdx.x);
        asm volatile("" : "+v"(tid_v));
        const int tid = tid_v, lane = tid_v & 63;
        const int buf = step & 1;
        // 1. the previous step's picks: the ones whose ball reaches a group's
        // box lower m in that group's slabs of 64; the ones it owns become chosen
        uint64_t ra[kMpPickWords], rb[kMpPickWords], om[kMpPickWords];  // picks 64 h .. 64 h + 63
        uint64_t any_reach = 0ull, any_own = 0ull;
#pragma unroll
        for (int h = 0; h < kMpPickWords; ++h) {
            const int qi = h * 64 + lane;
            bool reach_a = false, reach_b = false, own = false;
            if (qi < K) {
                const float4 q = s_pk[qi];
                const float4 alo = s_gb[wave][0], ahi = s_gb[wave][1], blo = s_gb[wave][2], bhi = s_gb[wave][3];
                reach_a = box_lower(alo.x, alo.y, alo.z, ahi.x, ahi.y, ahi.z, q.x, q.y, q.z) < q.w;
                reach_b = box_lower(blo.x, blo.y, blo.z, bhi.x, bhi.y, bhi.z, q.x, q.y, q.z) < q.w;
                const int off = s_ppos[qi] - wbase;
                own = off >= 0 && off < 64 * P;
            }
            ra[h] = __ballot(reach_a);
            rb[h] = __ballot(reach_b);
            om[h] = __ballot(own);
            any_reach |= ra[h] | rb[h];
            any_own |= om[h];
        }
        if ((any_reach | any_own) != 0ull || step == 1) {  // step 1 fills every cache
            // slots of this lane holding one of the wavefront's two chain
            // keys (their sorted positions are cached with them): only a
            // lowered m there can change the chain; any other m only drops,
            // which keeps both chain keys the largest and the bound an
            // upper bound
            uint32_t topm[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int cp = __float_as_int(s_wc[wave][e].w) - wbase;
                topm[e] = (cp >= 0 && cp < 64 * P && (cp & 63) == lane) ? 1u << (cp >> 6) : 0u;
            }
            uint32_t lowm = 0u;  // slots of this lane whose m dropped
#pragma unroll
            for (int h = 0; h < kMpPickWords; ++h)
                for (uint64_t mm = ra[h] | rb[h]; mm; mm &= mm - 1) {
                    const int bq = __builtin_ctzll(mm);
                    const float4 q = s_pk[h * 64 + bq];
                    // the slabs holding a group the pick reaches, then of those
                    // the ones whose own box it reaches (lane j tests slab j)
                    const uint32_t sg = (((ra[h] >> bq) & 1ull) ? slabs_a : 0u) | (((rb[h] >> bq) & 1ull) ? slabs_b : 0u);
                    bool hit = false;
                    if (lane < P && ((sg >> lane) & 1u)) {
                        const float4 lo = s_slo[wave][lane], hi = s_shi[wave][lane];
                        hit = box_lower(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, q.x, q.y, q.z) < q.w;
                    }
                    const uint32_t sm = uint32_t(__ballot(hit));
#pragma unroll
                    for (int j = 0; j < P; ++j) {
                        if (sm & (1u << j)) {
                            const float d = dist2(px[j], py[j], pz[j], q.x, q.y, q.z);
                            const bool lower = d < m[j];  // no NaN here: min without canonicalising
                            m[j] = lower ? d : m[j];
                            lowm |= lower ? 1u << j : 0u;
                        }
                    }
                }
#pragma unroll
            for (int h = 0; h < kMpPickWords; ++h)
                for (uint64_t mm = om[h]; mm; mm &= mm - 1) {
                    const int off = s_ppos[h * 64 + __builtin_ctzll(mm)] - wbase;
#pragma unroll
                    for (int j = 0; j < P; ++j)
                        if (off == j * 64 + lane) m[j] = -1.f;
                }
            // the cached chain stays exact unless the m of one of its keys
            // dropped or a pick (always one of them) was taken here: all of
            // it is rebuilt when a pick was taken here or c1's m dropped
            // (step 1 fills every cache), from c2 on when only c2's m did
            const bool redo1 = any_own != 0ull || step == 1 || __ballot((lowm & topm[0]) != 0u) != 0ull;
            if (redo1 || __ballot((lowm & topm[1]) != 0u) != 0ull) {
                const uint32_t* ids = s_id + (tid - lane);  // this wavefront's column of s_id
                uint64_t c1;
                float4 e1;
                if (redo1) {
                    // c1: per lane the largest value (bits + 1; 0 = none) and its slot
                    uint32_t vm = 0u;
                    int jm = 0;
                    bool tie = false;
#pragma unroll
                    for (int j = 0; j < P; ++j) {
                        const uint32_t w = m[j] >= 0.f ? __float_as_uint(m[j]) + 1u : 0u;
                        tie = w == vm ? true : (w > vm ? false : tie);
                        jm = w > vm ? j : jm;
                        vm = max(vm, w);
                    }
                    const BestKey b = wave_best<BLOCK, P>(vm, jm, tie, ids, lane, [&](int j, int zero) {
                        return m[j] >= 0.f ? (__float_as_uint(m[j]) | uint32_t(zero)) + 1u : 0u;
                    });
                    c1 = b.key;
                    e1 = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
                    if (c1 != 0ull) {
                        float x = px[0], y = py[0], z = pz[0];
#pragma unroll
                        for (int j = 1; j < P; ++j)
                            if (b.slot == j) {  // uniform
                                x = px[j];
                                y = py[j];
                                z = pz[j];
                            }
                        e1 = make_float4(uniform_at(x, b.lane), uniform_at(y, b.lane), uniform_at(z, b.lane),
                                         __int_as_float(wbase + b.slot * 64 + b.lane));
                    }
                } else {
                    c1 = s_w[wave][0];
                    e1 = s_wc[wave][0];
                }
                uint64_t c2 = 0ull;
                uint32_t c3 = 0u;
                float4 e2 = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
                if (c1 != 0ull) {
                    // c2: the best key once c1's ball has lowered the others.
                    // A slab whose box lies beyond that ball keeps its values
                    // (the box bound is at least c1's m, which bounds them all).
                    const int p1 = __float_as_int(e1.w) - wbase;
                    const int l1 = p1 & 63, j1 = p1 >> 6;
                    const float x1 = e1.x, y1 = e1.y, z1 = e1.z, r1 = key_value(c1);
                    bool hit = false;
                    if (lane < P) {
                        const float4 lo = s_slo[wave][lane], hi = s_shi[wave][lane];
                        hit = box_lower(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, x1, y1, z1) < r1;
                    }
                    const uint32_t sm1 = uint32_t(__ballot(hit));
                    auto value2 = [&](int j, int zero) {
                        float v = m[j];
                        if (sm1 & (1u << j)) {  // uniform
                            const float d = dist2(px[j], py[j], pz[j], __int_as_float(__float_as_int(x1) | zero), y1, z1);
                            v = d < v ? d : v;
                        }
                        const bool live = m[j] >= 0.f && !(lane == l1 && j == j1);
                        return live ? __float_as_uint(v) + 1u : 0u;
                    };
                    // per lane the largest and second largest of those values
                    uint32_t vm = 0u, t2 = 0u;
                    int jm = 0;
                    bool tie = false;
#pragma unroll
                    for (int j = 0; j < P; ++j) {
                        const uint32_t w = value2(j, 0);
                        t2 = max(t2, min(vm, w));
                        tie = w == vm ? true : (w > vm ? false : tie);
                        jm = w > vm ? j : jm;
                        vm = max(vm, w);
                        // one slot at a time: computing all sixteen values
                        // first would need more registers than remain
                        asm volatile("" : "+v"(vm), "+v"(jm), "+v"(t2));
                    }
                    const BestKey b = wave_best<BLOCK, P>(vm, jm, tie, ids, lane, value2);
                    c2 = b.key;
                    if (c2 != 0ull) {
                        float x = px[0], y = py[0], z = pz[0];
#pragma unroll
                        for (int j = 1; j < P; ++j)
                            if (b.slot == j) {
                                x = px[j];
                                y = py[j];
                                z = pz[j];
                            }
                        e2 = make_float4(uniform_at(x, b.lane), uniform_at(y, b.lane), uniform_at(z, b.lane),
                                         __int_as_float(wbase + b.slot * 64 + b.lane));
                        // c3: bound of every other value once c1 and c2 are
                        // taken -- the largest value after c1's update other
                        // than c2's (c2's ball can only lower them further)
                        const uint32_t top = wave_max_u32(lane == b.lane ? t2 : vm);
                        c3 = top ? top - 1u : 0u;
                    }
                }
                if (lane == 0) {
                    if (redo1) {
                        s_w[wave][0] = c1;
                        s_wc[wave][0] = e1;
                    }
                    s_w[wave][1] = c2;
                    s_c3[wave] = c3;
                    s_wc[wave][1] = e2;
                }
            }
        }
        lds_barrier();
        // 2. wavefront 0: the workgroup's E best chain keys become its
        // entries, with their data from the wavefronts that hold them, and R
        // bounds every value it does not offer; its record is one word a lane
        const uint64_t tag = uint64_t(step & 3u) << 62;
        if (wave == 0) {
            // chain key i of wavefront w on lane 2 w + i, ranked among all
            // listed keys by counting the larger ones (keys are unique, 0 =
            // none); ranks 0 .. E-1 are the entries
            constexpr int NK = 2 * NW;
            static_assert(NK % 2 == 0 && NK <= 64 && 6 * kMpEntries <= 64, "one key a lane");
            const int kw = lane >> 1, ki = lane & 1;
            const uint64_t kv = lane < NK ? s_w[kw][ki] : 0ull;
            const ulonglong2* sw2 = reinterpret_cast<const ulonglong2*>(&s_w[0][0]);
            int rank = 0;
#pragma unroll
            for (int c = 0; c < NK / 2; ++c) {
                const ulonglong2 b = sw2[c];
                rank += int(b.x > kv) + int(b.y > kv);
            }
            // R: the largest listed key kept back, and every wavefront's
            // bound after its two chain keys (a wavefront's entries are a
            // prefix of its chain, so its next listed key or that bound
            // caps the rest of it)
            const bool kept = kv != 0 && rank >= kMpEntries;
            uint32_t rv = kept ? uint32_t(kv >> 32) : 0u;
            if (lane < NW) rv = max(rv, s_c3[lane]);
            const uint32_t rg = wave_max_u32(rv);
            const int nz = __popcll(__ballot(kv != 0));
            if (kv != 0 && rank < kMpEntries) {
                const float4 c = s_wc[kw][ki];
                uint32_t* e = s_ent + 6 * rank;
                e[0] = uint32_t(kv >> 32);
                e[1] = uint32_t(kv);
                e[2] = __float_as_uint(c.x);
                e[3] = __float_as_uint(c.y);
                e[4] = __float_as_uint(c.z);
                e[5] = __float_as_uint(c.w);
            }
            __builtin_amdgcn_wave_barrier();  // LDS in program order within the wavefront
            // lane 3 e + f carries packed word f of entry e (zero past the
            // listed keys); lane 3 E carries R
            uint64_t wv = rg;
            if (lane < kMpEntryWords * kMpEntries) {
                const int e = lane / kMpEntryWords, f = lane - e * kMpEntryWords;
                const uint32_t* q = s_ent + 6 * e;
                wv = e < nz ? pack_entry_word(f, q[0], q[1], q[2], q[3], q[4], q[5]) : 0ull;
            }
            if (lane < kMpWords) st_rec(slots + (size_t(buf) * G + g) * kMpRecStride + lane, tag | wv);
        }
        // 3. every record, a few words a thread, into s_rw (kMpWords per
        // workgroup); a word is current once its high half is this step
        {
            constexpr int RW = (kMpMaxGroups * kMpWords + BLOCK - 1) / BLOCK;  // words a thread reads
            const int nw = G * kMpWords;
            const uint64_t* recs = slots + size_t(buf) * G * kMpRecStride;
            uint32_t spins = 0;
            bool aborted = false;
            while (true) {  // each wavefront polls its own words; one barrier after
                uint64_t v[RW];
#pragma unroll
                for (int c = 0; c < RW; ++c) {
                    const int i = min(tid + c * BLOCK, nw - 1);
                    const int r = i / kMpWords;
                    int off = r * kMpRecStride + (i - r * kMpWords);
                    // the 32-bit offset stays live across steps, the 64-bit
                    // address is formed here (two per offset would not fit)
                    asm volatile("" : "+v"(off));
                    v[c] = ld_rec(recs + off);
                }
                bool pending = false;
#pragma unroll
                for (int c = 0; c < RW; ++c) {
                    const int i = tid + c * BLOCK;
                    if (i < nw) {
                        if ((v[c] >> 62) == (step & 3u)) s_rw[i] = v[c] & kMpPayload;
                        else pending = true;
                    }
                }
                if (__ballot(pending) == 0) break;
                if (++spins > spin_limit) {
                    aborted = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (aborted && lane == 0) s_abort = 1;
        }
        if (tid == 0) {
            s_kfail = MAXPICKS;
            s_na = 0;
        }
        lds_barrier();
        if (s_abort) {  // a wait gave up: every workgroup's waits end the same way
            if (tid == 0) atomicOr(err, 1u);
            return;
        }

        // 4. the accepted set: the top entry, tau from the top workgroup's R
        // up to its fixed point (a workgroup holds an entry above tau iff its
        // first does), each found by every wavefront that lists members; the
        // members of workgroups 64 c .. 64 c + 63 listed in s_mk / s_mi by
        // wavefront c, at a base taken with one LDS atomic (their order there
        // is free: ranks come from the keys)
        const int cap = min(cap_picks, k - t);
        if (wave < ((G + 63) >> 6)) {
            uint64_t k1[kMpMaxGroups / 64];
            uint32_t rr[kMpMaxGroups / 64];
#pragma unroll
            for (int c = 0; c < kMpMaxGroups / 64; ++c) {
                const int w = c * 64 + lane;
                k1[c] = w < G ? rec_key<kMpEntries>(s_rw, kMpEntries * w) : 0ull;
                rr[c] = w < G ? rec_bound<kMpEntries>(s_rw, w) : 0u;
            }
            uint64_t top = 0;
            uint32_t topr = 0;
#pragma unroll
            for (int c = 0; c < kMpMaxGroups / 64; ++c) {
                topr = k1[c] > top ? rr[c] : topr;
                top = k1[c] > top ? k1[c] : top;
            }
            // the top key: its value bits by a 32-bit maximum, its index
            // bits only when values tie (keys are unique)
            const uint32_t tv = wave_max_u32(uint32_t(top >> 32));
            const bool atv = uint32_t(top >> 32) == tv;
            const uint64_t tied = __ballot(atv);
            int tl = __builtin_ctzll(tied);
            if (__popcll(tied) > 1) {
                const uint32_t tlo = wave_max_u32(atv ? uint32_t(top) : 0u);
                tl = __builtin_ctzll(__ballot(atv && uint32_t(top) == tlo));
            }
            const uint64_t tk = (uint64_t(tv) << 32) | uint32_t(__builtin_amdgcn_readlane(int(uint32_t(top)), tl));
            // R of the top workgroup, then tau up to its fixed point
            uint32_t tau = uint32_t(__builtin_amdgcn_readlane(int(topr), tl));
            for (int it = 0; it <= kMpMaxGroups; ++it) {  // at most two passes in exact arithmetic
                uint32_t mr = 0;
#pragma unroll
                for (int c = 0; c < kMpMaxGroups / 64; ++c) mr = uint32_t(k1[c] >> 32) > tau ? max(mr, rr[c]) : mr;
                mr = wave_max_u32(mr);
                if (mr <= tau) break;
                tau = mr;
            }
            const int w = wave * 64 + lane;
            uint64_t k1w = k1[0];
#pragma unroll
            for (int c = 1; c < kMpMaxGroups / 64; ++c) k1w = wave == c ? k1[c] : k1w;
            // entry e of workgroup w is a member when above tau (the first
            // also when it is the top key); the later entries of a
            // workgroup lie below its earlier ones
            uint64_t ke[kMpEntries];
            bool me[kMpEntries];
            uint64_t be[kMpEntries];
            ke[0] = k1w;
            me[0] = k1w != 0 && (k1w == tk || uint32_t(k1w >> 32) > tau);
#pragma unroll
            for (int e = 1; e < kMpEntries; ++e) {
                ke[e] = w < G ? rec_key<kMpEntries>(s_rw, kMpEntries * w + e) : 0ull;
                me[e] = ke[e] != 0 && uint32_t(ke[e] >> 32) > tau;
            }
            int cnt = 0;
#pragma unroll
            for (int e = 0; e < kMpEntries; ++e) {
                be[e] = __ballot(me[e]);
                cnt += __popcll(be[e]);
            }
            int base = 0;
            if (cnt != 0) {
                int old = 0;
                if (lane == 0) old = atomicAdd(&s_na, cnt);
                base = __builtin_amdgcn_readfirstlane(old);  // the whole wavefront is active: lane 0
            }
#pragma unroll
            for (int e = 0; e < kMpEntries; ++e) {
                if (me[e]) {
                    const int p = base + lanes_below(be[e]);
                    s_mk[p] = ke[e];
                    s_mi[p] = kMpEntries * w + e;
                }
                base += __popcll(be[e]);
            }
        }
        lds_barrier();
        const int na = s_na;
        // members ranked among themselves, the first `cap` published: a row
        // of 16 lanes ranks MR members, each lane counting over every 16th
        // pair of member keys (one load serves MR compares), the counts
        // summed across the row with DPP
        {
            constexpr int MR = 4;
            const int row = tid >> 4, part = tid & 15;
            const ulonglong2* mk2 = reinterpret_cast<const ulonglong2*>(s_mk);
            const int npairs = (na + 1) >> 1;  // the last pair's second key is ignored when na is odd
            for (int base = 0; base < na; base += (BLOCK / 16) * MR) {
                const int m0 = base + row * MR;
                if (m0 >= na) continue;  // whole rows drop out
                uint64_t kc[MR];
                int rk[MR];
#pragma unroll
                for (int r = 0; r < MR; ++r) {
                    kc[r] = m0 + r < na ? s_mk[m0 + r] : ~0ull;
                    rk[r] = 0;
                }
#pragma unroll 2
                for (int q = part; q < npairs; q += 16) {
                    const ulonglong2 kb = mk2[q];
                    const bool yok = 2 * q + 1 < na;
#pragma unroll
                    for (int r = 0; r < MR; ++r) rk[r] += int(kb.x > kc[r]) + int(yok && kb.y > kc[r]);
                }
#pragma unroll
                for (int r = 0; r < MR; ++r) rk[r] = row_sum16(rk[r]);
                int rank = rk[0];
#pragma unroll
                for (int r = 1; r < MR; ++r) rank = part == r ? rk[r] : rank;
                const int mi = m0 + part;
                if (part < MR && mi < na && rank < cap) {
                    const float4 c = rec_coords<kMpEntries>(s_rw, s_mi[mi]);
                    s_pk[rank] = make_float4(c.x, c.y, c.z, key_value(s_mk[mi]));
                    s_pid[rank] = key_id(s_mk[mi]);
                    s_ppos[rank] = __float_as_int(c.w);
                }
            }
        }
        const int nr = min(na, cap);
        lds_barrier();
        // 5. distance conflicts: member j is tested against the earlier
        // members i < j.  Columns are paired, c with nr - 1 - c, so that
        // every pair holds nr - 1 tests; TPP threads share a pair, each
        // taking every TPP-th test of column c, then of column nr - 1 - c.
        // Per wavefront the lowest lowered column of each kind comes from a
        // ballot (c grows with the lane, nr - 1 - c falls), and the lower
        // goes to LDS in one atomic
        {
            constexpr int TPP = BLOCK / (MAXPICKS / 2);  // threads per column pair
            static_assert(TPP >= 1 && (TPP & (TPP - 1)) == 0 && 64 % TPP == 0, "conflict tiling");
            const int c = tid / TPP, part = tid % TPP;  // c < MAXPICKS / 2
            bool low1 = false, low2 = false;
            if (c < (nr + 1) / 2) {
                const int j2 = nr - 1 - c;  // == c only for the middle column of an odd nr
                const float4 c1 = s_pk[c];
#pragma unroll 2
                for (int i = part; i < c; i += TPP) {
                    const float4 ci = s_pk[i];
                    if (dist2(c1.x, c1.y, c1.z, ci.x, ci.y, ci.z) < c1.w) low1 = true;
                }
                if (j2 > c) {
                    const float4 c2 = s_pk[j2];
#pragma unroll 2
                    for (int i = part; i < j2; i += TPP) {
                        const float4 ci = s_pk[i];
                        if (dist2(c2.x, c2.y, c2.z, ci.x, ci.y, ci.z) < c2.w) low2 = true;
                    }
                }
            }
            const uint64_t b1 = __ballot(low1), b2 = __ballot(low2);
            if (lane == 0 && (b1 | b2) != 0ull) {
                int f = MAXPICKS;
                if (b1) f = min(f, (wave * 64 + __builtin_ctzll(b1)) / TPP);
                if (b2) f = min(f, nr - 1 - (wave * 64 + 63 - __builtin_clzll(b2)) / TPP);
                atomicMin(&s_kfail, f);
            }
        }
        lds_barrier();
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

using ScanMpFn = void (*)(const float4*, const uint32_t*, const uint32_t*, const int32_t*, int, int, int, int32_t*, float*,
                          const DevHeader*, uint32_t*, uint64_t*, uint64_t*, int, uint32_t);

struct MpEntry {
    int block;
    int per_thread;
    ScanMpFn fn128, fn256;  // at most 128 / 256 picks per step
};

#define BS_MP_ENTRY(B, P) {B, P, scan_mp_kernel<B, P, 128>, scan_mp_kernel<B, P, 256>}
const MpEntry kMpTable[] = {
    BS_MP_ENTRY(1024, 1),  BS_MP_ENTRY(1024, 2),  BS_MP_ENTRY(1024, 4), BS_MP_ENTRY(1024, 8),
    BS_MP_ENTRY(1024, 12), BS_MP_ENTRY(1024, 16), BS_MP_ENTRY(512, 24), BS_MP_ENTRY(512, 32),
};
#undef BS_MP_ENTRY

__global__ void clear_mp_slots_kernel(uint64_t* slots, int nwords) {
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) st_rec(slots + i, 0);
}

}  // namespace

bool scan_several_supported(const ScanShape& s) {
    if (s.groups <= 1 || s.groups > kMpMaxGroups) return false;
    for (const MpEntry& e : kMpTable)
        if (e.block == s.block && e.per_thread == s.per_thread) return true;
    return false;
}

hipError_t launch_scan_several(const ScanShape& s, const float* pts, int n, int k, int start, int32_t* order,
                               float* radius, void* ws, uint64_t* ticks, int picks, hipStream_t st,
                               const LaunchOpts* ev) {
    ScanMpFn fn = nullptr;
    for (const MpEntry& e : kMpTable)
        if (e.block == s.block && e.per_thread == s.per_thread) fn = picks > 128 ? e.fn256 : e.fn128;
    if (!fn || !scan_several_supported(s)) return hipErrorInvalidValue;
    if (uint32_t(n) > kMpMaxPos) return hipErrorInvalidValue;  // positions are packed in 22 bits
    // both record buffers must fit the exchange area the workspace reserves
    if (size_t(2) * size_t(s.groups) * kMpRecStride * sizeof(uint64_t) > scan_slot_bytes(kMaxCoopGroups))
        return hipErrorInvalidValue;
    SortedPoints sp{};
    hipError_t e = launch_sorted_points(pts, n, start, ws, st, &sp);
    if (e != hipSuccess) return e;
    uint64_t* slots = static_cast<uint64_t*>(sp.slots);
    hipLaunchKernelGGL(clear_mp_slots_kernel, dim3(1), dim3(256), 0, st, slots, 2 * s.groups * kMpRecStride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && ev->begin && (e = hipEventRecord(ev->begin, st)) != hipSuccess) return e;
    const float4* xyzm = sp.xyzm;
    const uint32_t* ids = sp.ids;
    const uint32_t* codes = sp.codes;
    const int32_t* start_pos = sp.start_pos;
    const DevHeader* hdr = sp.hdr;
    uint32_t* err = &sp.hdr->error;
    uint32_t spin = spin_limit_of(ev);
    void* args[] = {(void*)&xyzm,  (void*)&ids,   (void*)&codes, (void*)&start_pos, (void*)&n,     (void*)&k,
                    (void*)&start, (void*)&order, (void*)&radius,    (void*)&hdr,   (void*)&err,
                    (void*)&slots, (void*)&ticks, (void*)&picks, (void*)&spin};
    e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(fn), dim3(s.groups), dim3(s.block), args, 0, st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess && ev && ev->end) e = hipEventRecord(ev->end, st);
    if (e == hipSuccess) e = launch_finish(sp.hdr, order, radius, k, st);
    return e;
}

}  // namespace bs
