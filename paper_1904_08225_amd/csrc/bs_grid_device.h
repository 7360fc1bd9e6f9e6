// bs_grid_device.h -- device code of the uniform-grid radius-pruned ordering,
// shared by the single-object kernel and the batched work-queue kernel.
//
// The ordering loop (grid_order_object) is described in bs_grid.hip.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bs_grid.h"

namespace bs {

constexpr int kMortonBits = 10;  // per axis
constexpr int kMaxBlocksAny = 4096;  // upper bound of blocks (64 cells each) per object

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

// Lower bound of d2(p, c) over p in the box [lo, hi] (see file comment).
__device__ __forceinline__ float box_lower(float lx, float ly, float lz, float hx, float hy,
                                           float hz, float cx, float cy, float cz) {
    const float gx = cx < lx ? lx - cx : (cx > hx ? cx - hx : 0.f);
    const float gy = cy < ly ? ly - cy : (cy > hy ? cy - hy : 0.f);
    const float gz = cz < lz ? lz - cz : (cz > hz ? cz - hz : 0.f);
    const float xx = gx * gx;
    const float yy = gy * gy;
    const float zz = gz * gz;
    const float s = xx + yy;
    return s + zz;
}

// A load whose address every lane shares, kept on the vector memory path
// (the address goes through a vector register): a persistent kernel reads
// such data for one work item after another, and memory may be rewritten
// between items.
template <class T>
__device__ __forceinline__ T load_vec(const T* p) {
    int z = 0;
    asm volatile("" : "+v"(z));
    return p[z];
}

__device__ __forceinline__ uint64_t make_key(float m, uint32_t id) {
    return (uint64_t(__float_as_uint(m)) << 32) | uint64_t(0x7FFFFFFFu - id);
}
__device__ __forceinline__ uint32_t key_id(uint64_t key) {
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

template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_max_u32(uint32_t v) {
    const uint32_t o = uint32_t(__builtin_amdgcn_update_dpp(int(v), int(v), CTRL, ROWS, 0xF, false));
    return o > v ? o : v;
}

// Wave-uniform maximum of 64-bit keys: reduce the high words with 32-bit
// DPP steps, then take the low word of the unique lane holding that high
// word (or reduce the low words of the tied lanes).
__device__ __forceinline__ uint64_t wave_max_key(uint64_t v) {
    uint32_t h = uint32_t(v >> 32);
    h = dpp_max_u32<0xB1, 0xF>(h);
    h = dpp_max_u32<0x4E, 0xF>(h);
    h = dpp_max_u32<0x141, 0xF>(h);
    h = dpp_max_u32<0x140, 0xF>(h);
    h = dpp_max_u32<0x142, 0xA>(h);
    h = dpp_max_u32<0x143, 0xC>(h);
    const uint32_t H = uint32_t(__builtin_amdgcn_readlane(int(h), 63));
    const uint64_t tied = __ballot(uint32_t(v >> 32) == H);
    uint32_t lo;
    if (__popcll(tied) == 1) {
        lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), __builtin_ctzll(tied)));
    } else {
        uint32_t l = uint32_t(v >> 32) == H ? uint32_t(v) : 0u;
        l = dpp_max_u32<0xB1, 0xF>(l);
        l = dpp_max_u32<0x4E, 0xF>(l);
        l = dpp_max_u32<0x141, 0xF>(l);
        l = dpp_max_u32<0x140, 0xF>(l);
        l = dpp_max_u32<0x142, 0xA>(l);
        l = dpp_max_u32<0x143, 0xC>(l);
        lo = uint32_t(__builtin_amdgcn_readlane(int(l), 63));
    }
    return (uint64_t(H) << 32) | lo;
}

__device__ __forceinline__ float ord_decode(uint32_t e) {
    const uint32_t u = (e & 0x80000000u) ? (e & 0x7FFFFFFFu) : ~e;
    return __uint_as_float(u);
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// ---------------------------------------------------------------- ordering

// Per-wavefront scratch for one block: hit-cell table and per-cell bests.
struct WaveScratch {
    int2 tab[64];        // (start, count) of the r-th hit cell
    uint64_t gkey[64];   // its new best key
    float4 gwin[64];     // x, y, z, sorted position of that best
};

// LDS state of one object's ordering: per-block best key, its coordinates
// and sorted position, its cell, the per-step touched-block masks, and the
// wavefront scratch.
template <int NW, int MAXB>
struct GridLds {
    static constexpr int kMaxBlocks = MAXB;
    uint64_t mask[MAXB / 64];
    uint64_t bkey[MAXB];
    float4 bwin[MAXB];
    int bcell[MAXB];
    WaveScratch ws[NW];
};

// LDS writes by some lanes become visible to reads by other lanes of the
// same wavefront once they have completed; also a compiler memory barrier.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Max over aligned groups of 2^steps lanes: afterwards the last lane of each
// group holds the group's maximum (steps = 6: lane 63 holds the wave max).
// `steps` must be wave-uniform.
__device__ __forceinline__ uint64_t group_max_u64(uint64_t v, int steps) {
    if (steps >= 1) v = dpp_max_step<0xB1, 0xF>(v);
    if (steps >= 2) v = dpp_max_step<0x4E, 0xF>(v);
    if (steps >= 3) v = dpp_max_step<0x141, 0xF>(v);
    if (steps >= 4) v = dpp_max_step<0x140, 0xF>(v);
    if (steps >= 5) v = dpp_max_step<0x142, 0xA>(v);
    if (steps >= 6) v = dpp_max_step<0x143, 0xC>(v);
    return v;
}

constexpr int kUnroll = 8;  // members per lane in flight

// Update members start + s, start + s + G, ... (< start + count) of one cell
// with the pick, U of them in flight per lane; track the lane's best key.
// UPD = false only marks the candidate at c_pos as taken (a removal that is
// not a pick) and recomputes the best key; no distance changes.
template <int U, bool UPD = true>
__device__ __forceinline__ void member_batches(float4* __restrict__ xyzm,
                                               const uint32_t* __restrict__ ids, int start,
                                               int count, int s, int G, int c_pos, float cx,
                                               float cy, float cz, uint64_t& lk, float4& lw) {
    for (int q0 = s; q0 < count; q0 += G * U) {
        int pos[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + u * G;
            ok[u] = q < count;
            pos[u] = start + (ok[u] ? q : 0);
        }
        float4 p[U];
        uint32_t id[U];
#pragma unroll
        for (int u = 0; u < U; ++u) p[u] = xyzm[pos[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) id[u] = ids[pos[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool pick = ok[u] && pos[u] == c_pos;
            const bool live = ok[u] && !pick && p[u].w >= 0.f;
            const float d = dist2(p[u].x, p[u].y, p[u].z, cx, cy, cz);
            const bool dec = UPD && live && d < p[u].w;
            const float m = dec ? d : p[u].w;
            if (dec || (pick && p[u].w != -1.f)) xyzm[pos[u]].w = pick ? -1.f : d;
            const uint64_t kk = live ? make_key(m, id[u]) : 0ull;
            const bool better = kk > lk;
            lk = better ? kk : lk;
            lw = better ? make_float4(p[u].x, p[u].y, p[u].z, __int_as_float(pos[u])) : lw;
        }
    }
}

// One wavefront updates every candidate of block b that the pick can reach
// and rewrites the block's best into LDS.  The nh hit cells each get an
// aligned group of 64 / 2^ceil(log2 nh) lanes.  Wave-local: no barrier.
// Loads are issued unconditionally (clamped to a valid address) so that a
// batch of them is in flight together.
template <class Lds, bool UPD = true>
__device__ inline void process_block(const GridObject& o, Lds& L, int b, int c_pos, int c_cell,
                              float cx, float cy, float cz, float mc, int prof_t) {
    (void)prof_t;
    const int lane = threadIdx.x & 63;
    WaveScratch& W = L.ws[threadIdx.x >> 6];
    float4* __restrict__ xyzm = o.xyzm;
    const uint32_t* __restrict__ ids = o.ids;
    const int cell = b * 64 + lane;
    const bool valid = cell < o.C;
    const int ci = valid ? cell : o.C - 1;
    const float4 lo = o.cstat[2 * ci], hi = o.cstat[2 * ci + 1];
    const uint4 d0 = o.cdyn[2 * ci], d1 = o.cdyn[2 * ci + 1];
    uint64_t ckey = valid ? ((uint64_t(d0.y) << 32) | d0.x) : 0ull;
    float4 cwin = make_float4(__uint_as_float(d1.x), __uint_as_float(d1.y), __uint_as_float(d1.z),
                              __int_as_float(int(d0.z)));
    const bool hit = valid && (cell == c_cell ||
                               box_lower(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, cx, cy, cz) < mc);
    const uint64_t hm = __ballot(hit);
    const int nh = __popcll(hm);
    if (nh == 0) return;  // nothing in reach: the block's best is unchanged

    // lanes -> (hit cell r, sub-lane s)
    int start, count, G, gshift, r;
    if (nh == 1) {
        const int h = __builtin_ctzll(hm);
        start = __builtin_amdgcn_readlane(__float_as_int(lo.w), h);
        count = __builtin_amdgcn_readlane(__float_as_int(hi.w), h);
        gshift = 6;
        G = 64;
        r = 0;
    } else {
        const int rank = __popcll(hm & ((1ull << lane) - 1));
        if (hit) W.tab[rank] = make_int2(__float_as_int(lo.w), __float_as_int(hi.w));
        int steps = 0;
        while ((1 << steps) < nh) ++steps;
        gshift = 6 - steps;
        G = 1 << gshift;
        r = lane >> gshift;
        wave_lds_sync();
        const int2 my = W.tab[r < nh ? r : 0];
        start = my.x;
        count = r < nh ? my.y : 0;
    }
    const int s = lane & (G - 1);

    uint64_t lk = 0;
    float4 lw = make_float4(0.f, 0.f, 0.f, 0.f);
    // members each lane walks; few (late steps): short batches, else deep ones
    const int per = count > s ? (count - s + G - 1) >> gshift : 0;
    const int maxper = __builtin_amdgcn_readfirstlane(int(wave_max_key(uint64_t(per) << 32) >> 32));
    if (maxper <= 2)
        member_batches<2, UPD>(xyzm, ids, start, count, s, G, c_pos, cx, cy, cz, lk, lw);
    else
        member_batches<kUnroll, UPD>(xyzm, ids, start, count, s, G, c_pos, cx, cy, cz, lk, lw);

    if (nh == 1) {
        // block best = max(new best of the hit cell, best of the other cells)
        const int h = __builtin_ctzll(hm);
        const uint64_t wk = wave_max_key(lk);
        const uint64_t ok = wave_max_key(hit ? 0ull : ckey);
        if (wk != 0) {
            const int wl = __builtin_ctzll(__ballot(lk == wk));
            const float4 w = make_float4(
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lw.x), wl)),
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lw.y), wl)),
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lw.z), wl)),
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lw.w), wl)));
            if (lane == h) cwin = w;
        }
        if (lane == h) {
            ckey = wk;
            o.cdyn[2 * cell + 0] = make_uint4(uint32_t(ckey), uint32_t(ckey >> 32),
                                              uint32_t(__float_as_int(cwin.w)), 0u);
            o.cdyn[2 * cell + 1] = make_uint4(__float_as_uint(cwin.x), __float_as_uint(cwin.y),
                                              __float_as_uint(cwin.z), 0u);
        }
        const uint64_t bk = wk > ok ? wk : ok;
        if (bk != 0 && ckey == bk) {
            L.bwin[b] = cwin;
            L.bcell[b] = cell;
        }
        if (lane == 0) L.bkey[b] = bk;
    } else {
        const uint64_t gm = group_max_u64(lk, gshift);
        if (s == G - 1 && r < nh) W.gkey[r] = gm;
        wave_lds_sync();
        if (r < nh && lk != 0 && lk == W.gkey[r]) W.gwin[r] = lw;
        wave_lds_sync();
        if (hit) {
            const int rank = __popcll(hm & ((1ull << lane) - 1));
            ckey = W.gkey[rank];
            cwin = W.gwin[rank];
            o.cdyn[2 * cell + 0] = make_uint4(uint32_t(ckey), uint32_t(ckey >> 32),
                                              uint32_t(__float_as_int(cwin.w)), 0u);
            o.cdyn[2 * cell + 1] = make_uint4(__float_as_uint(cwin.x), __float_as_uint(cwin.y),
                                              __float_as_uint(cwin.z), 0u);
        }
        const uint64_t bk = wave_max_key(ckey);
        if (bk != 0 && ckey == bk) {
            L.bwin[b] = cwin;
            L.bcell[b] = cell;
        }
        if (lane == 0) L.bkey[b] = bk;
    }
    wave_lds_sync();
}

// Best block of superblock sb (64 consecutive blocks), computed by one
// wavefront from LDS: (key, block).
template <class Lds>
__device__ __forceinline__ void superblock_best(Lds& L, int sb, uint64_t& key, int& blk) {
    const int lane = threadIdx.x & 63;
    const uint64_t v = L.bkey[sb * 64 + lane];
    key = wave_max_key(v);
    blk = sb * 64 + __builtin_ctzll(__ballot(v == key) | (1ull << 63));
}

// Whole ordering of one object by one workgroup (steps 1 .. k-1).
template <int BLOCK, int MAXB>
__device__ inline void grid_order_object(const GridObject& o, GridLds<BLOCK / 64, MAXB>& L) {
    constexpr int NW = BLOCK / 64;
    constexpr int BPT = MAXB / BLOCK;  // block boxes held per thread
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
            L.bwin[b] = make_float4(__uint_as_float(d1.x), __uint_as_float(d1.y),
                                    __uint_as_float(d1.z), __int_as_float(int(d0.z)));
            L.bcell[b] = int(d0.w);
        } else {
            blx[j] = bly[j] = blz[j] = INFINITY;  // empty box: never touched
            bhx[j] = bhy[j] = bhz[j] = -INFINITY;
            L.bkey[b] = 0;
        }
    }

    // superblock boxes (64 blocks each): lane s of every wavefront holds box s
    float slx = INFINITY, sly = INFINITY, slz = INFINITY, shx = -INFINITY, shy = -INFINITY,
          shz = -INFINITY;
    if (lane < nsb) {
        const float4 lo = o.sbstat[2 * lane], hi = o.sbstat[2 * lane + 1];
        slx = lo.x; sly = lo.y; slz = lo.z;
        shx = hi.x; shy = hi.y; shz = hi.z;
    }

    int c_pos = o.start_pos, c_cell = o.start_cell;
    const float4 sp = o.xyzm[c_pos];
    float cx = sp.x, cy = sp.y, cz = sp.z;
    float mc = INFINITY;
    if (tid == 0) {
        o.order[0] = int32_t(o.start_id);
        if (o.radius) o.radius[0] = INFINITY;
        if (o.ticks) o.ticks[0] = wall_clock64();
    }
    __syncthreads();

    // superblock bests, kept redundantly by every wavefront: lane j holds superblock j
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

    for (int t = 1; t < k; ++t) {
        const int prof_t = t;
        (void)prof_t;
        // blocks that may hold a candidate whose m can drop, or the pick:
        // superblock boxes first (one per lane), then the blocks of touched ones
        const int cb = c_cell >> 6;
        const bool stouch = lane < nsb && (lane == (cb >> 6) ||
                                           box_lower(slx, sly, slz, shx, shy, shz, cx, cy, cz) < mc);
        const uint64_t smask = __ballot(stouch);
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int sb = j * NW + wave;  // superblock of this wavefront's blocks (uniform)
            uint64_t m = 0;
            if ((smask >> sb) & 1ull) {
                const int b = j * BLOCK + tid;
                const bool touch = b == cb ||
                    box_lower(blx[j], bly[j], blz[j], bhx[j], bhy[j], bhz[j], cx, cy, cz) < mc;
                m = __ballot(touch);
            }
            if (lane == 0) L.mask[sb] = m;
        }
        __syncthreads();

        // wavefront w takes the touched blocks of rank w, w + NW, ...
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
                if (rank % NW == wave) process_block(o, L, b, c_pos, c_cell, cx, cy, cz, mc, t);
                ++rank;
            }
        }
        __syncthreads();

        // refresh the touched superblocks, then the argmax over superblocks
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
        const uint64_t best = wave_max_key(sbk);
        const int wl = __builtin_ctzll(__ballot(sbk == best) | (1ull << 63));
        const int bb = __builtin_amdgcn_readlane(sbb, wl);
        const float4 win = L.bwin[bb];
        c_cell = L.bcell[bb];
        c_pos = __float_as_int(win.w);
        cx = win.x;
        cy = win.y;
        cz = win.z;
        mc = key_value(best);
        if (tid == 0) {
            o.order[t] = int32_t(key_id(best));
            if (o.radius) o.radius[t] = sqrtf(mc);
            if (o.ticks) o.ticks[t] = wall_clock64();
        }
    }
}

}  // namespace bs
