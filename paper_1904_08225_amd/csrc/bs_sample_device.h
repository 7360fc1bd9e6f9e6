// bs_sample_device.h -- device code of the paper's randomized progressive
// sampler (Sec. 3.2) over the grid of one object, shared by the
// single-object kernel and the batched work-queue kernel.
//
// The sampler appends, round after round, the member of a random sample of
// the remaining candidates that lies farthest from every surfel chosen so
// far.  Its "distance to all chosen surfels" is each candidate's m (squared
// distance to the nearest chosen surfel), kept exact for every candidate the
// same way as the grid-pruned exact ordering keeps it: a pick lowers m only
// inside its reach, and a superblock, block or cell whose box lower bound
// from the pick is at least the largest m it holds (its best key's value)
// cannot contain a candidate the pick lowers.  So a sample member's m is
// read from memory when it is
// drawn, and every later pick of the same round is folded into the sampled
// values in registers (min is exact and order-free).  Removals (picks, and
// sample members near the chosen surfels when asked) mark m = -1 and
// refresh their cell's best key, so the hierarchy's top key stays the exact
// farthest remaining candidate: a round whose draws all miss takes it.
// Nothing in a round reads the m held in memory after its draws (its later
// picks come from the sampled values in registers), so the round's picks
// are applied to memory together, in one grid pass of up to 32 picks: every
// m becomes the minimum over all of them, as after one pass per pick.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "bs_grid.h"
#include "bs_grid_device.h"
#include "bs_grid_multi.h"

namespace bs {

constexpr int kSampleMaxSlots = 256;  // sample slots per round (one per thread)
constexpr int kSampleAttempts = 16;   // draws a slot makes before it stays empty
constexpr int kSamplePassPicks = 32;  // picks applied by one grid pass (bits of a 32-bit mask)

// A workgroup barrier ordering LDS only.  __syncthreads() also waits for the
// wavefront's global stores in flight (the picks just emitted, say), which
// a barrier that only hands LDS data to the other wavefronts need not do.
// Global data one wavefront writes and another reads is still ordered by a
// __syncthreads() between the two.
__device__ __forceinline__ void barrier_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

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
    int wcnt[NW];
    int nrem;
    int2 rem[kSampleMaxSlots];      // removed sample members: (sorted position, cell)
    float4 pk[kSamplePassPicks];    // picks not yet applied to memory: x, y, z (w unused)
    int pkpos[kSamplePassPicks];    // their sorted positions
    int pkcell[kSamplePassPicks];   // their cells
    uint32_t hmask[NW][64];         // per wavefront: the picks reaching each hit cell of its block
    // a pick's selection from the sample (two alternating sets, so that one
    // barrier per pick suffices): each wavefront's best sampled key, its
    // x, y, z and sorted position, and its cell
    uint64_t skey[2][NW];
    float4 swin[2][NW];
    int scell[2][NW];
};

// One wavefront applies the picks in pm (bits of SL.pk) to every candidate of
// block b they can reach -- a cell is hit by pick j when it is the pick's
// cell or its box lower bound from the pick lies below the cell's largest m
// (its best key's value: no member with a smaller m can drop) -- marks the
// picks taken, and rewrites the hit cells' best keys and the block's best in
// LDS.  The hit cells each get an aligned group of lanes, as in
// process_block.  Wave-local: no barrier.
// Cell records of one block as one wavefront holds them (lane = cell).
struct SampleCells {
    float4 lo, hi;  // cell box, first member / member count
    uint4 d0, d1;   // best key, its position; its coordinates
};

__device__ __forceinline__ SampleCells sample_cells_load(const GridObject& o, int b) {
    const int cell = b * 64 + int(threadIdx.x & 63);
    const int ci = cell < o.C ? cell : o.C - 1;
    SampleCells r;
    r.lo = o.cstat[2 * ci];
    r.hi = o.cstat[2 * ci + 1];
    r.d0 = o.cdyn[2 * ci];
    r.d1 = o.cdyn[2 * ci + 1];
    return r;
}

template <int NW, int MAXB>
__device__ inline void sample_block_update(const GridObject& o, GridLds<NW, MAXB>& L, SampleLds<NW>& SL, int b,
                                           uint32_t pm, const SampleCells& rec) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    WaveScratch& W = L.ws[wave];
    const int cell = b * 64 + lane;
    const bool valid = cell < o.C;
    const float4 lo = rec.lo, hi = rec.hi;
    const uint4 d0 = rec.d0, d1 = rec.d1;
    uint64_t ckey = valid ? ((uint64_t(d0.y) << 32) | d0.x) : 0ull;
    float4 cwin = make_float4(__uint_as_float(d1.x), __uint_as_float(d1.y), __uint_as_float(d1.z),
                              __int_as_float(int(d0.z)));
    const float cmax = key_value(ckey);  // 0 when no member is left
    uint32_t cm = 0u;
    for (uint32_t mm = pm; mm; mm &= mm - 1) {
        const int j = __builtin_ctz(mm);
        const float4 q = SL.pk[j];
        const bool h = valid && (cell == SL.pkcell[j] ||
                                 box_lower(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, q.x, q.y, q.z) < cmax);
        cm |= h ? (1u << j) : 0u;
    }
    const bool hit = cm != 0u;
    const uint64_t hm = __ballot(hit);
    const int nh = __popcll(hm);
    if (nh == 0) return;  // nothing in reach: the block's best is unchanged
    // lanes -> (hit cell r, sub-lane s)
    const int rank = __popcll(hm & ((1ull << lane) - 1));
    if (hit) {
        W.tab[rank] = make_int2(__float_as_int(lo.w), __float_as_int(hi.w));
        SL.hmask[wave][rank] = cm;
    }
    int steps = 0;
    while ((1 << steps) < nh) ++steps;
    const int gshift = 6 - steps;
    const int G = 1 << gshift;
    const int r = lane >> gshift;
    wave_lds_sync();
    const int2 my = W.tab[r < nh ? r : 0];
    const uint32_t rm = r < nh ? SL.hmask[wave][r] : 0u;
    const int start = my.x;
    const int count = r < nh ? my.y : 0;
    const int s = lane & (G - 1);
    const bool single = __popc(rm) == 1;
    const int j0 = __builtin_ctz(rm | 0x80000000u) & (kSamplePassPicks - 1);
    const float4 q0 = SL.pk[j0];
    const int qpos0 = SL.pkpos[j0];
    uint64_t lk = 0, l2 = 0;
    float4 lw = make_float4(0.f, 0.f, 0.f, 0.f);
    const int per = count > s ? (count - s + G - 1) >> gshift : 0;
    const int maxper = __builtin_amdgcn_readfirstlane(int(wave_max_key(uint64_t(per) << 32) >> 32));
    constexpr int U = NW >= 16 ? 2 : 4;  // member loads in flight per lane
    if (maxper <= 1)
        member_batches_mp<1>(o, SL, start, count, s, G, rm, single, q0.x, q0.y, q0.z, qpos0, lk, l2, lw);
    else
        member_batches_mp<U>(o, SL, start, count, s, G, rm, single, q0.x, q0.y, q0.z, qpos0, lk, l2, lw);
    // each hit cell's new best, then the block's
    const uint64_t gm = group_max_u64(lk, gshift);
    if (s == G - 1 && r < nh) W.gkey[r] = gm;
    wave_lds_sync();
    if (r < nh && lk != 0 && lk == W.gkey[r]) W.gwin[r] = lw;
    wave_lds_sync();
    if (hit) {
        ckey = W.gkey[rank];
        cwin = W.gwin[rank];
        o.cdyn[2 * cell + 0] = make_uint4(uint32_t(ckey), uint32_t(ckey >> 32), uint32_t(__float_as_int(cwin.w)), 0u);
        o.cdyn[2 * cell + 1] = make_uint4(__float_as_uint(cwin.x), __float_as_uint(cwin.y),
                                          __float_as_uint(cwin.z), 0u);
    }
    const uint64_t bk = wave_max_key(ckey);
    if (bk != 0 && ckey == bk) {
        L.bwin[b] = cwin;
        L.bcell[b] = cell;
    }
    if (lane == 0) L.bkey[b] = bk;
    wave_lds_sync();
}

// Workgroup maximum of a 64-bit key (uniform result); two barriers.
template <int NW>
__device__ __forceinline__ uint64_t block_max_key(uint64_t v, SampleLds<NW>& S) {
    const uint64_t wk = wave_max_key(v);
    if ((threadIdx.x & 63) == 0) S.wkey[threadIdx.x >> 6] = wk;
    barrier_lds();
    uint64_t best = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint64_t k = S.wkey[w];
        best = k > best ? k : best;
    }
    barrier_lds();
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

    // One pass applying the np picks held in SL.pk: superblocks, then
    // blocks, then cells, each tested against the picks that reach the level
    // above, a pick reaching a box when the box's lower bound from it lies
    // below the largest m held in the box (its best key's value), or when it
    // lies in the box; then the touched superblocks' bests.  Returns the top
    // key left.
    auto pass_set = [&](int np) -> uint64_t {
        barrier_lds();  // the picks' LDS entries are written
        uint32_t sm = 0u;  // lane = superblock: the picks that may reach it
        if (lane < nsb) {
            const float smax = key_value(sbk);
            for (int j = 0; j < np; ++j) {
                const float4 q = SL.pk[j];
                const bool r = lane == (SL.pkcell[j] >> 12) ||  // its own superblock (64 blocks of 64 cells)
                               box_lower(slx, sly, slz, shx, shy, shz, q.x, q.y, q.z) < smax;
                sm |= r ? (1u << j) : 0u;
            }
        }
        const uint64_t smask = __ballot(sm != 0u);
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int sb = j * NW + wave;
            uint64_t msk = 0;
            if ((smask >> sb) & 1ull) {
                const int b = j * BLOCK + tid;
                const uint32_t bm = uint32_t(__builtin_amdgcn_readlane(int(sm), sb));
                const float bmax = key_value(L.bkey[b]);
                bool touch = false;
                for (uint32_t mm = bm; mm; mm &= mm - 1) {
                    const int jj = __builtin_ctz(mm);
                    const float4 q = SL.pk[jj];
                    touch = touch || b == (SL.pkcell[jj] >> 6) ||
                            box_lower(blx[j], bly[j], blz[j], bhx[j], bhy[j], bhz[j], q.x, q.y, q.z) < bmax;
                }
                msk = __ballot(touch);
            }
            if (lane == 0) L.mask[sb] = msk;
        }
        barrier_lds();
        const uint64_t mword = lane < nsb ? L.mask[lane] : 0ull;
        const uint64_t nz = __ballot(mword != 0);
        // this wavefront's blocks (ranks wave, wave + NW, ...): the next
        // one's cell records load while the current one is updated
        int rank = 0, pb = -1;
        uint32_t ppm = 0u;
        SampleCells cur;
        for (uint64_t zs = nz; zs;) {
            const int mi = __builtin_ctzll(zs);
            zs &= zs - 1;
            const uint32_t mlo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(mword)), mi));
            const uint32_t mhi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(mword >> 32)), mi));
            const uint32_t bm = uint32_t(__builtin_amdgcn_readlane(int(sm), mi));
            for (uint64_t mk = (uint64_t(mhi) << 32) | mlo; mk;) {
                const int b = mi * 64 + __builtin_ctzll(mk);
                mk &= mk - 1;
                if (rank % NW == wave) {
                    const SampleCells nxt = sample_cells_load(o, b);
                    if (pb >= 0) sample_block_update<NW, MAXB>(o, L, SL, pb, ppm, cur);
                    cur = nxt;
                    pb = b;
                    ppm = bm;
                }
                ++rank;
            }
        }
        if (pb >= 0) sample_block_update<NW, MAXB>(o, L, SL, pb, ppm, cur);
        __syncthreads();  // also orders the member and cell stores for later passes and draws
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

    // the start's update (every candidate's m is +inf before it)
    uint64_t top = pass(Upd{}, INFINITY);

    const int S = sp.S;
    const bool has_slot = tid < S;
    const int slot_waves = (S + 63) / 64;  // wavefronts holding sample slots (S <= kSampleMaxSlots)
    int t = 1;
    int remaining = sp.n - 1;
    uint32_t round = 0;
    // this thread's sample slot
    bool live = false;
    float val = 0.f, px = 0.f, py = 0.f, pz = 0.f;
    int ppos = 0, pcell = 0;
    uint32_t pid = 0;
    uint32_t sel = 0;  // selections from the sample so far (alternate LDS sets)
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
                        pcell = int(sp.cellidx[pos]) - 1 - sp.cell_base;
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
        int np = 0;  // picks of this round not yet applied to memory
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
                // the largest sampled key: per wavefront holding slots, then
                // over those wavefronts' entries (lanes holding the same key
                // hold the same candidate, so any of them may write its data);
                // the other wavefronts only read the result
                const int par = int(sel & 1u);
                ++sel;
                if (wave < slot_waves) {
                    const uint64_t mine = live ? make_key(val, pid) : 0ull;
                    const uint64_t wk = wave_max_key(mine);
                    if (lane == 0) SL.skey[par][wave] = wk;
                    if (wk != 0 && mine == wk) {
                        SL.swin[par][wave] = make_float4(px, py, pz, __int_as_float(ppos));
                        SL.scell[par][wave] = pcell;
                    }
                }
                barrier_lds();  // the emitted picks' stores need not complete here
                best = 0;
                int bw = 0;
#pragma unroll
                for (int w = 0; w < kSampleMaxSlots / 64 && w < NW; ++w) {
                    const uint64_t kw = w < slot_waves ? SL.skey[par][w] : 0ull;
                    bw = kw > best ? w : bw;
                    best = kw > best ? kw : best;
                }
                if (best == 0) break;  // the sample is used up
                const float4 win = SL.swin[par][bw];
                c_pos = __float_as_int(win.w);
                c_cell = SL.scell[par][bw];
                cx = win.x;
                cy = win.y;
                cz = win.z;
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
            if (tid == 0) {
                SL.pk[np] = make_float4(cx, cy, cz, 0.f);
                SL.pkpos[np] = c_pos;
                SL.pkcell[np] = c_cell;
            }
            ++np;
            // a pick taken from the top key needs memory up to date for the
            // next one (the whole remaining set as the sample)
            if (whole || np == kSamplePassPicks) {
                top = pass_set(np);
                np = 0;
            }
        }
        if (np > 0) top = pass_set(np);
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
