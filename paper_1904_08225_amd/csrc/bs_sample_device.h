// bs_sample_device.h -- device code of the paper's randomized progressive
// sampler (Sec. 3.2) over the grid of one object, shared by the
// single-object kernel and the batched work-queue kernel.
//
// The sampler appends, round after round, the member of a random sample of
// the remaining candidates that lies farthest from every surfel chosen so
// far.  Its "distance to all chosen surfels" is each candidate's m (squared
// distance to the nearest chosen surfel), kept exact for every candidate the
// same way as the grid-pruned exact ordering keeps it: a pick lowers m only
// inside its reach, and a cell whose box lower bound is at least the largest
// m still held anywhere (the hierarchy's top key) cannot contain a candidate
// the pick lowers.  So a sample member's m is read from memory when it is
// drawn, and every later pick of the same round is folded into the sampled
// values in registers (min is exact and order-free).  Removals (picks, and
// sample members near the chosen surfels when asked) mark m = -1 and
// refresh their cell's best key, so the hierarchy's top key stays the exact
// farthest remaining candidate: a round whose draws all miss takes it.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "bs_grid.h"
#include "bs_grid_device.h"

namespace bs {

constexpr int kSampleMaxSlots = 256;  // sample slots per round (one per thread)
constexpr int kSampleAttempts = 16;   // draws a slot makes before it stays empty

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): the first output word
// for counter (c0, c1, c2, c3) and key (k0, k1).  Ten rounds; each multiplies
// words 0 and 2 by 0xD2511F53 and 0xCD9E8D57 into 64-bit products and mixes
// the halves with words 1 and 3 and the key, which grows by 0x9E3779B9 and
// 0xBB67AE85 between rounds.
__device__ __forceinline__ uint32_t philox_first(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return c0;
}

// Sampler parameters and per-object extras.
struct SampleSpec {
    uint32_t key0, key1;      // Philox key: low and high words of the object's seed
    int S;                    // sample slots per round (0 = the whole remaining set), <= kSampleMaxSlots
    int K;                    // rounds between growth steps of the picks per round (< 0: one pick)
    float vicinity;           // removal factor v (0 = no removal)
    int n;                    // candidates of the object
    const int32_t* pos_of;    // [n] sorted position of each original index
    const uint32_t* cellidx;  // [sorted] inclusive cell count: cell of position p = cellidx[p] - 1 - cell_base
    int cell_base;
    int32_t* count;           // optional: number of picks made
};

template <int NW>
struct SampleLds {
    uint64_t wkey[NW];
    float4 win;                     // x, y, z, sorted position of the chosen slot
    int wcnt[NW];
    int nrem;
    int2 rem[kSampleMaxSlots];      // removed sample members: (sorted position, cell)
};

// Workgroup maximum of a 64-bit key (uniform result); two barriers.
template <int NW>
__device__ __forceinline__ uint64_t block_max_key(uint64_t v, SampleLds<NW>& S) {
    const uint64_t wk = wave_max_key(v);
    if ((threadIdx.x & 63) == 0) S.wkey[threadIdx.x >> 6] = wk;
    __syncthreads();
    uint64_t best = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint64_t k = S.wkey[w];
        best = k > best ? k : best;
    }
    __syncthreads();
    return best;
}

// The whole sampler run of one object by one workgroup (picks 0 .. k-1).
template <int BLOCK, int MAXB>
__device__ inline void sample_object(const GridObject& o, const SampleSpec& sp, GridLds<BLOCK / 64, MAXB>& L,
                                     SampleLds<BLOCK / 64>& SL) {
    constexpr int NW = BLOCK / 64;
    constexpr int BPT = MAXB / BLOCK;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int k = o.k;
    const int NB = o.NB;
    const int nsb = (NB + 63) / 64;

    float blx[BPT], bly[BPT], blz[BPT], bhx[BPT], bhy[BPT], bhz[BPT];
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int b = j * BLOCK + tid;
        if (b < NB) {
            const float4 lo = o.bstat[2 * b], hi = o.bstat[2 * b + 1];
            blx[j] = lo.x; bly[j] = lo.y; blz[j] = lo.z;
            bhx[j] = hi.x; bhy[j] = hi.y; bhz[j] = hi.z;
            const uint4 d0 = o.bdyn[2 * b], d1 = o.bdyn[2 * b + 1];
            L.bkey[b] = (uint64_t(d0.y) << 32) | d0.x;
            L.bwin[b] = make_float4(__uint_as_float(d1.x), __uint_as_float(d1.y), __uint_as_float(d1.z),
                                    __int_as_float(int(d0.z)));
            L.bcell[b] = int(d0.w);
        } else {
            blx[j] = bly[j] = blz[j] = INFINITY;
            bhx[j] = bhy[j] = bhz[j] = -INFINITY;
            L.bkey[b] = 0;
        }
    }
    float slx = INFINITY, sly = INFINITY, slz = INFINITY, shx = -INFINITY, shy = -INFINITY, shz = -INFINITY;
    if (lane < nsb) {
        const float4 lo = o.sbstat[2 * lane], hi = o.sbstat[2 * lane + 1];
        slx = lo.x; sly = lo.y; slz = lo.z;
        shx = hi.x; shy = hi.y; shz = hi.z;
    }

    int c_pos = o.start_pos, c_cell = o.start_cell;
    const float4 sp0 = o.xyzm[c_pos];
    float cx = sp0.x, cy = sp0.y, cz = sp0.z;
    if (tid == 0) {
        o.order[0] = int32_t(o.start_id);
        if (o.radius) o.radius[0] = INFINITY;
        if (o.ticks) o.ticks[0] = wall_clock64();
    }
    __syncthreads();

    uint64_t sbk = 0;
    int sbb = 0;
    for (int sb = 0; sb < nsb; ++sb) {
        uint64_t kk;
        int bb;
        superblock_best(L, sb, kk, bb);
        if (lane == sb) {
            sbk = kk;
            sbb = bb;
        }
    }

    // One pass of the update of pick (or removal) c: cells that may hold a
    // candidate with m > d2(p, c), i.e. box lower bound < mc (the largest m
    // left), plus c's own cell; UPD = false only marks c removed.  Then the
    // touched superblocks' bests.  Returns the top key left.
    auto pass = [&](auto upd_tag, float mc) -> uint64_t {
        constexpr bool UPD = decltype(upd_tag)::value;
        const int cb = c_cell >> 6;
        const bool stouch = lane < nsb &&
                            (lane == (cb >> 6) || box_lower(slx, sly, slz, shx, shy, shz, cx, cy, cz) < mc);
        const uint64_t smask = __ballot(stouch);
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int sb = j * NW + wave;
            uint64_t msk = 0;
            if ((smask >> sb) & 1ull) {
                const int b = j * BLOCK + tid;
                const bool touch =
                    b == cb || box_lower(blx[j], bly[j], blz[j], bhx[j], bhy[j], bhz[j], cx, cy, cz) < mc;
                msk = __ballot(touch);
            }
            if (lane == 0) L.mask[sb] = msk;
        }
        __syncthreads();
        const uint64_t mword = lane < nsb ? L.mask[lane] : 0ull;
        const uint64_t nz = __ballot(mword != 0);
        int rank = 0;
        for (uint64_t zs = nz; zs;) {
            const int mi = __builtin_ctzll(zs);
            zs &= zs - 1;
            const uint32_t mlo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(mword)), mi));
            const uint32_t mhi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(mword >> 32)), mi));
            for (uint64_t mk = (uint64_t(mhi) << 32) | mlo; mk;) {
                const int b = mi * 64 + __builtin_ctzll(mk);
                mk &= mk - 1;
                if (rank % NW == wave)
                    process_block<GridLds<NW, MAXB>, UPD>(o, L, b, c_pos, c_cell, cx, cy, cz, mc, 0);
                ++rank;
            }
        }
        __syncthreads();
        for (uint64_t zs = nz; zs;) {
            const int mi = __builtin_ctzll(zs);
            zs &= zs - 1;
            uint64_t kk;
            int bb;
            superblock_best(L, mi, kk, bb);
            if (lane == mi) {
                sbk = kk;
                sbb = bb;
            }
        }
        return wave_max_key(sbk);
    };
    using Upd = std::integral_constant<bool, true>;    // a pick: distances drop, it is marked
    using Mark = std::integral_constant<bool, false>;  // a removal: only marked

    // the start's update (every candidate's m is +inf before it)
    uint64_t top = pass(Upd{}, INFINITY);

    const int S = sp.S;
    const bool has_slot = tid < S;
    int t = 1;
    int remaining = sp.n - 1;
    uint32_t round = 0;
    // this thread's sample slot
    bool live = false;
    float val = 0.f, px = 0.f, py = 0.f, pz = 0.f;
    int ppos = 0;
    uint32_t pid = 0;
    while (t < k && remaining > 0) {
        // --- a new round: draw the sample
        bool whole = S == 0;
        if (!whole) {
            live = false;
            if (has_slot) {
                for (uint32_t a = 0; a < uint32_t(kSampleAttempts); ++a) {
                    const uint32_t u = philox_first(round, uint32_t(tid), a, 0u, sp.key0, sp.key1);
                    const uint32_t idx = uint32_t((uint64_t(u) * uint64_t(uint32_t(sp.n))) >> 32);
                    const int pos = sp.pos_of[idx];
                    const float4 p = o.xyzm[pos];
                    if (p.w >= 0.f) {
                        live = true;
                        val = p.w;
                        px = p.x;
                        py = p.y;
                        pz = p.z;
                        ppos = pos;
                        pid = idx;
                        break;
                    }
                }
            }
            const uint64_t anyk = block_max_key(live ? 1ull : 0ull, SL);
            whole = anyk == 0;  // every draw missed: the farthest remaining candidate
        }
        int q = sp.K < 0 ? 1 : 1 + int(round / uint32_t(sp.K));
        if (whole && S > 0) q = 1;
        float d_first = 0.f;
        for (int p = 0; p < q && t < k && remaining > 0; ++p) {
            uint64_t best;
            if (whole) {
                best = top;
                if (best == 0) {  // nothing left (cannot happen while remaining > 0)
                    remaining = 0;
                    break;
                }
                const int wl = __builtin_ctzll(__ballot(sbk == best) | (1ull << 63));
                const int bb = __builtin_amdgcn_readlane(sbb, wl);
                const float4 win = L.bwin[bb];
                c_cell = L.bcell[bb];
                c_pos = __float_as_int(win.w);
                cx = win.x;
                cy = win.y;
                cz = win.z;
            } else {
                best = block_max_key(live ? make_key(val, pid) : 0ull, SL);
                if (best == 0) break;  // the sample is used up
                if (live && make_key(val, pid) == best)
                    SL.win = make_float4(px, py, pz, __int_as_float(ppos));
                __syncthreads();
                const float4 win = SL.win;
                c_pos = __float_as_int(win.w);
                c_cell = int(sp.cellidx[c_pos]) - 1 - sp.cell_base;
                cx = win.x;
                cy = win.y;
                cz = win.z;
                __syncthreads();
            }
            const float mv = key_value(best);
            if (p == 0) d_first = mv;
            if (tid == 0) {
                o.order[t] = int32_t(key_id(best));
                if (o.radius) o.radius[t] = sqrtf(mv);
                if (o.ticks) o.ticks[t] = wall_clock64();
            }
            ++t;
            --remaining;
            // fold the pick into the sampled values (the same min as the update)
            if (live) {
                if (pid == key_id(best)) live = false;
                else val = fminf(val, dist2(px, py, pz, cx, cy, cz));
            }
            top = pass(Upd{}, key_value(top));
        }
        // --- removal of sample members near the chosen surfels
        if (sp.vicinity > 0.f && !whole) {
            const float thr = (sp.vicinity * sp.vicinity) * d_first;
            if (tid == 0) SL.nrem = 0;
            __syncthreads();
            bool rm = live && val < thr;
            if (rm) {
                const int at = atomicAdd(&SL.nrem, 1);
                SL.rem[at] = make_int2(ppos, int(pid));
            }
            __syncthreads();
            const int nr = SL.nrem;
            // a candidate named by two slots is listed twice: removed once
            for (int r = 0; r < nr; ++r) {
                const int2 e = SL.rem[r];
                bool dup = false;
                for (int r2 = 0; r2 < r; ++r2) dup |= SL.rem[r2].y == e.y;
                if (dup) continue;
                c_pos = e.x;
                c_cell = int(sp.cellidx[c_pos]) - 1 - sp.cell_base;
                const float4 pc = o.xyzm[c_pos];
                cx = pc.x;
                cy = pc.y;
                cz = pc.z;
                __syncthreads();
                top = pass(Mark{}, -1.f);
                --remaining;
            }
            if (rm) live = false;
        }
        ++round;
    }
    if (tid == 0 && sp.count) *sp.count = t;
    for (int u = t + tid; u < k; u += BLOCK) {
        o.order[u] = -3;
        if (o.radius) o.radius[u] = __builtin_nanf("");
    }
}

}  // namespace bs
