// bs_grid_multi.h -- grid-pruned ordering with several exact picks per round.
//
// The greedy step (paper Sec. 3.2 / 3.3) appends the remaining candidate
// with the largest m_i, then lowers every m_i to d2(p_i, pick).  Updates
// only lower values, so the sequential order can be read ahead exactly:
// let q_1 > q_2 > ... be the remaining candidates by key at the start of a
// round (key = value bits : complemented index, unique).  q_1 is the next
// pick.  q_j (j > 1) is the pick after q_1 .. q_{j-1} iff
//   (i)  none of q_1 .. q_{j-1} lowers it: d2(q_j, q_i) >= m(q_j) for all
//        i < j (then min(m, d2) = m, its key is unchanged), and
//   (ii) every remaining candidate other than q_j has a key below q_j's
//        before the round (then after the round too, since keys only drop).
// (ii) is checked with bounds: every superblock offers two entries, the best
// keys of its two best blocks, and keeps a bound R on all its other keys.
// The candidates are the entries by descending key; q_j is accepted while
// (i) holds and its value exceeds R of every superblock with an entry among
// q_1 .. q_{j-1} (an entry of a superblock none of q_1 .. q_{j-1} came from
// lies below q_j by the order itself); the walk stops at the first failure.
// Every wavefront ranks a share of the candidates (two ballots per
// candidate) and tests it against the higher-ranked ones; the accepted count
// is the lowest failing rank.  The round then applies all accepted picks at once:
// m_i <- min(m_i, d2(p_i, q_1), ..., d2(p_i, q_K)), which equals the
// sequential updates because min is exact and order-free; a candidate or box
// is skipped for pick q_j when its binary32 box lower bound is >= m(q_j),
// which bounds its value at step j (see bs_grid.hip), or >= the largest m
// the box held before the round (its best key's value): either way no m in
// it can drop.
//
// Levels: cells keep their best key, its position/coordinates and their
// exact second key (cdyn); blocks of 64 cells keep best key, coordinates,
// cell and second-value bound in LDS; superblocks of SBS = 2^s blocks (at
// most 64 superblocks, one per lane) keep their two entries, their blocks
// and the bound R in LDS.
#pragma once
#pragma clang fp contract(off)

#include "bs_grid_device.h"

namespace bs {

constexpr int kMaxPicks = 32;  // picks per round (<= 32: pick masks are 32-bit)

// Per-wavefront scratch of the wavefront-per-block path.
struct WaveScratchMP {
    int2 tab[64];        // (start, count) of the r-th hit cell
    uint32_t tabm[64];   // picks that can reach it
    uint64_t g1[64];     // its new best key
    uint64_t g2[64];     // its new second key
    float4 gwin[64];     // x, y, z, sorted position of that best
};

// Workgroup-wide lists of the cell-parallel path (rounds touching few
// blocks); they share LDS with the per-wavefront scratch, so wider
// workgroups have room for longer lists.
template <int NW>
struct HitCaps {
    static constexpr int cells = NW >= 16 ? 768 : 256;   // hit cells per round
    static constexpr int blocks = NW >= 16 ? 128 : 64;   // touched blocks per round
};

struct CellResult {
    uint64_t g1, g2;  // new best and second key of the cell
    float4 win;       // x, y, z, sorted position of the best
};

// A touched block with hit cells: its hit cells (a range of the cell list)
// and the best of its other cells.
struct HitBlock {
    uint64_t n1;      // best key among the cells not hit (0: none)
    float4 n1win;     // its coordinates and position
    uint32_t n1sec;   // value bits of that cell's second key
    uint32_t n2;      // largest value among the other cells not hit
    int n1cell, first, cnt, b;
};

template <int NW>
union ScratchMP {
    WaveScratchMP ws[NW];
    struct {
        int4 hc[HitCaps<NW>::cells];     // cell, first member, member count, pick mask
        CellResult cr[HitCaps<NW>::cells];
        HitBlock hb[HitCaps<NW>::blocks];
    } lists;
};

template <int NW, int MAXB>
struct GridLdsMP {
    static constexpr int kMaxBlocks = MAXB;
    uint64_t mask[MAXB / 64];
    uint64_t bkey[MAXB];
    uint32_t bsec[MAXB];   // value bits bounding every other key of the block
    float4 bwin[MAXB];
    int bcell[MAXB];
    uint64_t sbkey[64];    // superblock entries: best key of its best block
    uint64_t sbkey2[64];   //   and of its second best block (0: none)
    uint32_t sbsec[64];    // value bits bounding every key of the superblock but the two entries
    int sbblk[64], sbblk2[64];  // the blocks of the two entries
    float4 sblo[64], sbhi[64];  // superblock boxes
    uint32_t spm[64];      // picks (by rank) reaching each superblock
    float4 pk[kMaxPicks];  // picks of the round by rank: x, y, z, m
    int pkpos[kMaxPicks];
    int pkcell[kMaxPicks];
    uint32_t pkid[kMaxPicks];  // their original indices
    int kfail;             // selection: lowest rank that cannot follow the ranks before it
    int tlist[HitCaps<NW>::blocks];  // touched blocks by rank (rounds touching few blocks)
    static constexpr int kHitCells = HitCaps<NW>::cells;
    static constexpr int kHitBlocks = HitCaps<NW>::blocks;
    int hcount, hbcount, overflow;
    ScratchMP<NW> u;
};

// One DPP step of a top-2 merge of 64-bit keys (0 = none).  Lanes whose
// source is outside the enabled rows read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ void dpp_top2_step(uint64_t& a1, uint64_t& a2) {
    const uint32_t b1l = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(a1)), CTRL, ROWS, 0xF, false));
    const uint32_t b1h = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(a1 >> 32)), CTRL, ROWS, 0xF, false));
    const uint32_t b2l = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(a2)), CTRL, ROWS, 0xF, false));
    const uint32_t b2h = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(a2 >> 32)), CTRL, ROWS, 0xF, false));
    const uint64_t b1 = (uint64_t(b1h) << 32) | b1l;
    const uint64_t b2 = (uint64_t(b2h) << 32) | b2l;
    const uint64_t hi = a1 > b1 ? a1 : b1;
    const uint64_t lo = a1 > b1 ? b1 : a1;
    const uint64_t s = a2 > b2 ? a2 : b2;
    a1 = hi;
    a2 = lo > s ? lo : s;
}

// Top-2 over aligned groups of 2^steps lanes; the last lane of each group
// holds the result.  The partners of every step hold disjoint lane sets, so
// merging two top-2 lists is exact.  `steps` must be wave-uniform.
__device__ __forceinline__ void group_top2(uint64_t& a1, uint64_t& a2, int steps) {
    if (steps >= 1) dpp_top2_step<0xB1, 0xF>(a1, a2);
    if (steps >= 2) dpp_top2_step<0x4E, 0xF>(a1, a2);
    if (steps >= 3) dpp_top2_step<0x141, 0xF>(a1, a2);
    if (steps >= 4) dpp_top2_step<0x140, 0xF>(a1, a2);
    if (steps >= 5) dpp_top2_step<0x142, 0xA>(a1, a2);
    if (steps >= 6) dpp_top2_step<0x143, 0xC>(a1, a2);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = dpp_max_u32<0xB1, 0xF>(v);
    v = dpp_max_u32<0x4E, 0xF>(v);
    v = dpp_max_u32<0x141, 0xF>(v);
    v = dpp_max_u32<0x140, 0xF>(v);
    v = dpp_max_u32<0x142, 0xA>(v);
    v = dpp_max_u32<0x143, 0xC>(v);
    return uint32_t(__builtin_amdgcn_readlane(int(v), 63));
}

__device__ __forceinline__ float rl(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Members start + s, start + s + G, ... of one cell, U loads in flight per
// lane, against the picks in `pm` (one pick in registers when `single`).
template <int U, class Lds>
__device__ __forceinline__ void member_batches_mp(const GridObject& o, const Lds& L, int start,
                                                  int count, int s, int G, uint32_t pm, bool single,
                                                  float qx, float qy, float qz, int qpos,
                                                  uint64_t& a1, uint64_t& a2, float4& lw) {
    float4* __restrict__ xyzm = o.xyzm;
    const uint32_t* __restrict__ ids = o.ids;
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
        float dmin[U];
        bool pick[U];
        if (single) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                dmin[u] = dist2(p[u].x, p[u].y, p[u].z, qx, qy, qz);
                pick[u] = pos[u] == qpos;
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                dmin[u] = INFINITY;
                pick[u] = false;
            }
            for (uint32_t mm = pm; mm; mm &= mm - 1) {
                const int j = __builtin_ctz(mm);
                const float4 q = L.pk[j];
                const int qp = L.pkpos[j];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    dmin[u] = fminf(dmin[u], dist2(p[u].x, p[u].y, p[u].z, q.x, q.y, q.z));
                    pick[u] = pick[u] || pos[u] == qp;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool pk = ok[u] && pick[u];
            const bool live = ok[u] && !pk && p[u].w >= 0.f;
            const bool dec = live && dmin[u] < p[u].w;
            const float m = dec ? dmin[u] : p[u].w;
            if (dec || (pk && p[u].w != -1.f)) xyzm[pos[u]].w = pk ? -1.f : dmin[u];
            const uint64_t kk = live ? make_key(m, id[u]) : 0ull;
            const bool b1 = kk > a1;
            a2 = b1 ? a1 : (kk > a2 ? kk : a2);
            a1 = b1 ? kk : a1;
            lw = b1 ? make_float4(p[u].x, p[u].y, p[u].z, __int_as_float(pos[u])) : lw;
        }
    }
}

// Cell records of one block as one wavefront holds them (lane = cell).
struct BlockRec {
    float4 lo, hi;  // cell box + first member / member count
    uint4 d0, d1;   // cell best key, position, second key, coordinates
};

__device__ __forceinline__ BlockRec load_block(const GridObject& o, int b) {
    const int lane = threadIdx.x & 63;
    const int cell = b * 64 + lane;
    const int ci = cell < o.C ? cell : o.C - 1;
    BlockRec r;
    r.lo = o.cstat[2 * ci];
    r.hi = o.cstat[2 * ci + 1];
    r.d0 = o.cdyn[2 * ci];
    r.d1 = o.cdyn[2 * ci + 1];
    return r;
}

// Touched blocks of this wavefront (rank % NW == wave) in mask order.
struct BlockIter {
    uint64_t zs;  // mask words still to visit
    uint64_t mk;  // bits left in the current word
    int mi;       // current word
    int rank;     // touched blocks seen so far
};

__device__ __forceinline__ int next_block(BlockIter& it, uint64_t mword, int wave, int nw) {
    while (true) {
        while (it.mk == 0) {
            if (it.zs == 0) return -1;
            it.mi = __builtin_ctzll(it.zs);
            it.zs &= it.zs - 1;
            const uint32_t mlo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(mword)), it.mi));
            const uint32_t mhi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(mword >> 32)), it.mi));
            it.mk = (uint64_t(mhi) << 32) | mlo;
        }
        const int b = it.mi * 64 + __builtin_ctzll(it.mk);
        it.mk &= it.mk - 1;
        const int r = it.rank++;
        if (r % nw == wave) return b;
    }
}

// One wavefront updates the members of block b that any of the K picks can
// reach and rewrites the cell records and the block's LDS entry.  Picks are
// held by lanes 0..K-1 (px, py, pz, pm, pcell) of every wavefront.
template <int UMAX, class Lds>
__device__ inline int process_block_mp(const GridObject& o, Lds& L, int b, const BlockRec& rec,
                                        int K, float px, float py, float pz, float pm, int ppos,
                                        int pcell, uint64_t* acc) {
    (void)acc;
    const int lane = threadIdx.x & 63;
    WaveScratchMP& W = L.u.ws[threadIdx.x >> 6];
    const int cell = b * 64 + lane;
    const bool valid = cell < o.C;
    const float4 lo = rec.lo, hi = rec.hi;
    const uint4 d0 = rec.d0, d1 = rec.d1;
    const float4 blo = load_vec(o.bstat + 2 * b), bhi = load_vec(o.bstat + 2 * b + 1);
    uint64_t ckey = valid ? ((uint64_t(d0.y) << 32) | d0.x) : 0ull;
    uint64_t csec = valid ? ((uint64_t(d1.w) << 32) | d0.w) : 0ull;
    float4 cwin = make_float4(__uint_as_float(d1.x), __uint_as_float(d1.y), __uint_as_float(d1.z),
                              __int_as_float(int(d0.z)));
    // picks that can reach the block (lane j tests pick j)
    const bool bt = lane < K && ((pcell >> 6) == b ||
                                 box_lower(blo.x, blo.y, blo.z, bhi.x, bhi.y, bhi.z, px, py, pz) < pm);
    uint32_t bm = uint32_t(__ballot(bt));
    // per cell: which of those picks reach it
    const float cmax = __uint_as_float(d0.y);  // no member's m exceeds the cell's best key's value
    uint32_t cm = 0, um = 0;
    for (uint32_t mm = bm; mm; mm &= mm - 1) {
        const int j = __builtin_ctz(mm);
        const float qx = rl(px, j), qy = rl(py, j), qz = rl(pz, j), qm = rl(pm, j);
        const int qc = __builtin_amdgcn_readlane(pcell, j);
        const bool h = valid && (cell == qc ||
                                 box_lower(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, qx, qy, qz) < fminf(qm, cmax));
        cm |= h ? (1u << j) : 0u;
        um |= __ballot(h) ? (1u << j) : 0u;
    }
    const bool hit = cm != 0;
    const uint64_t hm = __ballot(hit);
    const int nh = __popcll(hm);
    if (nh == 0) return 0;  // nothing in reach: the block's entry is unchanged

    int start, count, G, gshift, r;
    uint32_t gm;
    if (nh == 1) {
        const int h = __builtin_ctzll(hm);
        start = __builtin_amdgcn_readlane(__float_as_int(lo.w), h);
        count = __builtin_amdgcn_readlane(__float_as_int(hi.w), h);
        gm = uint32_t(__builtin_amdgcn_readlane(int(cm), h));
        gshift = 6;
        G = 64;
        r = 0;
    } else {
        const int rank = __popcll(hm & ((1ull << lane) - 1));
        if (hit) {
            W.tab[rank] = make_int2(__float_as_int(lo.w), __float_as_int(hi.w));
            W.tabm[rank] = cm;
        }
        int steps = 0;
        while ((1 << steps) < nh) ++steps;
        gshift = 6 - steps;
        G = 1 << gshift;
        r = lane >> gshift;
        wave_lds_sync();
        const int rr = r < nh ? r : 0;
        const int2 my = W.tab[rr];
        gm = W.tabm[rr];
        start = my.x;
        count = r < nh ? my.y : 0;
    }
    const int s = lane & (G - 1);
    const bool single = __popc(um) == 1;
    const int j0 = __builtin_ctz(um | 0x80000000u);
    const float qx = rl(px, j0), qy = rl(py, j0), qz = rl(pz, j0);
    const int qpos = __builtin_amdgcn_readlane(ppos, j0);

    uint64_t a1 = 0, a2 = 0;
    float4 lw = make_float4(0.f, 0.f, 0.f, 0.f);
    const int per = count > s ? (count - s + G - 1) >> gshift : 0;
    const int maxper = __builtin_amdgcn_readfirstlane(int(wave_max_key(uint64_t(per) << 32) >> 32));
    if (maxper <= 2)
        member_batches_mp<2>(o, L, start, count, s, G, gm, single, qx, qy, qz, qpos, a1, a2, lw);
    else
        member_batches_mp<UMAX>(o, L, start, count, s, G, gm, single, qx, qy, qz, qpos, a1, a2, lw);

    // per hit cell: best key, second key, and the coordinates of the best
    // (published by the one lane whose own best is it: keys are unique)
    const uint64_t own = a1;
    group_top2(a1, a2, gshift);
    if (s == G - 1 && r < nh) {
        W.g1[r] = a1;
        W.g2[r] = a2;
    }
    wave_lds_sync();
    if (r < nh && own != 0 && own == W.g1[r]) W.gwin[r] = lw;
    wave_lds_sync();
    if (hit) {
        const int rank = __popcll(hm & ((1ull << lane) - 1));
        ckey = W.g1[rank];
        csec = W.g2[rank];
        cwin = W.gwin[rank];
        o.cdyn[2 * cell + 0] = make_uint4(uint32_t(ckey), uint32_t(ckey >> 32),
                                          uint32_t(__float_as_int(cwin.w)), uint32_t(csec));
        o.cdyn[2 * cell + 1] = make_uint4(__float_as_uint(cwin.x), __float_as_uint(cwin.y),
                                          __float_as_uint(cwin.z), uint32_t(csec >> 32));
    }
    // block: best over cells; bound = max(second of the best cell, other cells' values)
    const uint64_t bk = wave_max_key(ckey);
    const int wl = __builtin_ctzll(__ballot(ckey == bk) | (1ull << 63));
    const uint32_t sv = wave_max_u32(lane == wl ? uint32_t(csec >> 32) : uint32_t(ckey >> 32));
    if (bk != 0 && lane == wl) {
        L.bwin[b] = cwin;
        L.bcell[b] = cell;
    }
    if (lane == 0) {
        L.bkey[b] = bk;
        L.bsec[b] = sv;
    }
    wave_lds_sync();
    return nh;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0xB1, 0xF, 0xF, false));
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x4E, 0xF, 0xF, false));
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x141, 0xF, 0xF, false));
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x140, 0xF, 0xF, false));
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x142, 0xA, 0xF, false));
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x143, 0xC, 0xF, false));
    return uint32_t(__builtin_amdgcn_readlane(int(v), 63));
}

// Cell-parallel path, phase 1 (one wavefront per touched block): find the
// block's hit cells, append them to the workgroup's cell list and record
// the best of the cells that no pick reaches.  Reads only.
template <class Lds>
__device__ inline void collect_block(const GridObject& o, Lds& L, int b, const BlockRec& rec, int K,
                                     float px, float py, float pz, float pm, int pcell) {
    const int lane = threadIdx.x & 63;
    const int cell = b * 64 + lane;
    const bool valid = cell < o.C;
    const float4 lo = rec.lo, hi = rec.hi;
    const uint4 d0 = rec.d0, d1 = rec.d1;
    const float4 blo = load_vec(o.bstat + 2 * b), bhi = load_vec(o.bstat + 2 * b + 1);
    const bool bt = lane < K && ((pcell >> 6) == b ||
                                 box_lower(blo.x, blo.y, blo.z, bhi.x, bhi.y, bhi.z, px, py, pz) < pm);
    const float cmax = __uint_as_float(d0.y);  // no member's m exceeds the cell's best key's value
    uint32_t cm = 0;
    for (uint32_t mm = uint32_t(__ballot(bt)); mm; mm &= mm - 1) {
        const int j = __builtin_ctz(mm);
        const float qx = rl(px, j), qy = rl(py, j), qz = rl(pz, j), qm = rl(pm, j);
        const int qc = __builtin_amdgcn_readlane(pcell, j);
        const bool h = valid && (cell == qc ||
                                 box_lower(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, qx, qy, qz) < fminf(qm, cmax));
        cm |= h ? (1u << j) : 0u;
    }
    const bool hit = cm != 0;
    const uint64_t hm = __ballot(hit);
    const int nh = __popcll(hm);
    if (nh == 0) return;
    int base = 0, hbi = 0;
    if (lane == 0) {
        base = atomicAdd(&L.hcount, nh);
        hbi = atomicAdd(&L.hbcount, 1);
    }
    base = __builtin_amdgcn_readfirstlane(base);
    hbi = __builtin_amdgcn_readfirstlane(hbi);
    if (base + nh > Lds::kHitCells || hbi >= Lds::kHitBlocks) {
        if (lane == 0) L.overflow = 1;
        return;
    }
    if (hit) {
        const int rank = __popcll(hm & ((1ull << lane) - 1));
        L.u.lists.hc[base + rank] = make_int4(cell, __float_as_int(lo.w), __float_as_int(hi.w), int(cm));
    }
    // best, its second value, and the next value among the cells not hit
    const uint64_t ckey = valid ? ((uint64_t(d0.y) << 32) | d0.x) : 0ull;
    const uint64_t nk = hit ? 0ull : ckey;
    const uint64_t n1 = wave_max_key(nk);
    const int wl = __builtin_ctzll(__ballot(n1 != 0 && nk == n1) | (1ull << 63));
    const uint32_t n2 = wave_max_u32(lane != wl ? uint32_t(nk >> 32) : 0u);
    HitBlock& hb = L.u.lists.hb[hbi];
    if (lane == wl) {
        hb.n1win = make_float4(__uint_as_float(d1.x), __uint_as_float(d1.y), __uint_as_float(d1.z),
                               __int_as_float(int(d0.z)));
        hb.n1sec = d1.w;
        hb.n1cell = cell;
    }
    if (lane == 0) {
        hb.n1 = n1;
        hb.n2 = n2;
        hb.first = base;
        hb.cnt = nh;
        hb.b = b;
    }
}

// Phase 2: the hit cells of the round spread over every lane of the
// workgroup (aligned groups of G lanes per cell); each group updates its
// cell's members, writes the cell record and the cell's result to LDS.
template <int NW, int UMAX, class Lds>
__device__ inline void update_cells(const GridObject& o, Lds& L) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int H = L.hcount;
    int per_wave = (H + NW - 1) / NW;  // cells per wavefront and pass
    int gsteps = 0;                    // log2 of cells per wavefront per pass
    while ((1 << gsteps) < per_wave && gsteps < 6) ++gsteps;
    const int gshift = 6 - gsteps;
    const int G = 1 << gshift;
    const int cpw = 1 << gsteps;
    const int passes = (H + NW * cpw - 1) / (NW * cpw);
    const int s = lane & (G - 1);
    for (int p = 0; p < passes; ++p) {
        const int c = (p * NW + wave) * cpw + (lane >> gshift);
        const bool has = c < H;
        const int4 e = has ? L.u.lists.hc[c] : make_int4(0, 0, 0, 0);
        const uint32_t pmask = uint32_t(e.w);
        const bool single = __popc(pmask) == 1;
        const int j0 = __builtin_ctz(pmask | 0x80000000u) & (kMaxPicks - 1);
        const float4 q = L.pk[j0];
        const int qpos = L.pkpos[j0];
        uint64_t a1 = 0, a2 = 0;
        float4 lw = make_float4(0.f, 0.f, 0.f, 0.f);
        const int count = has ? e.z : 0;
        const int per = count > s ? (count - s + G - 1) >> gshift : 0;
        const int maxper = __builtin_amdgcn_readfirstlane(int(wave_max_key(uint64_t(per) << 32) >> 32));
        if (maxper <= 1)
            member_batches_mp<1>(o, L, e.y, count, s, G, pmask, single, q.x, q.y, q.z, qpos, a1, a2, lw);
        else
            member_batches_mp<UMAX>(o, L, e.y, count, s, G, pmask, single, q.x, q.y, q.z, qpos, a1, a2,
                                    lw);
        const uint64_t own = a1;
        group_top2(a1, a2, gshift);
        CellResult* const cr = L.u.lists.cr;
        if (has && s == G - 1) {
            cr[c].g1 = a1;
            cr[c].g2 = a2;
        }
        wave_lds_sync();
        if (has && own != 0 && own == cr[c].g1) cr[c].win = lw;
        wave_lds_sync();
        if (has && s == G - 1) {
            const float4 w = cr[c].win;
            const int cell = e.x;
            o.cdyn[2 * cell + 0] = make_uint4(uint32_t(a1), uint32_t(a1 >> 32),
                                              uint32_t(__float_as_int(w.w)), uint32_t(a2));
            o.cdyn[2 * cell + 1] = make_uint4(__float_as_uint(w.x), __float_as_uint(w.y),
                                              __float_as_uint(w.z), uint32_t(a2 >> 32));
        }
    }
}

// Phase 3: every block with hit cells gets its new LDS entry from its hit
// cells' results and the best of its other cells.
template <int NW, class Lds>
__device__ inline void finish_blocks(Lds& L) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int HB = L.hbcount;
    for (int i = wave; i < HB; i += NW) {
        const HitBlock hb = L.u.lists.hb[i];
        const bool in = lane < hb.cnt;
        uint64_t k1 = 0, k2 = 0;
        float4 w = make_float4(0.f, 0.f, 0.f, 0.f);
        int cell = 0;
        if (in) {
            const CellResult r = L.u.lists.cr[hb.first + lane];
            k1 = r.g1;
            k2 = r.g2;
            w = r.win;
            cell = L.u.lists.hc[hb.first + lane].x;
        }
        const uint64_t m = wave_max_key(k1);
        const uint64_t bk = m > hb.n1 ? m : hb.n1;
        uint32_t wsec, others;
        float4 bw;
        int bc;
        if (bk == 0) {
            wsec = 0;
            others = 0;
            bw = w;
            bc = 0;
        } else if (bk == hb.n1) {  // a cell no pick reached keeps the block's best
            wsec = hb.n1sec;
            others = max(hb.n2, wave_max_u32(uint32_t(k1 >> 32)));
            bw = hb.n1win;
            bc = hb.n1cell;
        } else {
            const int wl = __builtin_ctzll(__ballot(k1 == bk) | (1ull << 63));
            wsec = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(k2 >> 32)), wl));
            others = max(max(uint32_t(hb.n1 >> 32), hb.n2),
                         wave_max_u32(lane != wl ? uint32_t(k1 >> 32) : 0u));
            bw = make_float4(rl(w.x, wl), rl(w.y, wl), rl(w.z, wl), rl(w.w, wl));
            bc = __builtin_amdgcn_readlane(cell, wl);
        }
        if (lane == 0) {
            L.bkey[hb.b] = bk;
            L.bsec[hb.b] = max(wsec, others);
            if (bk != 0) {
                L.bwin[hb.b] = bw;
                L.bcell[hb.b] = bc;
            }
        }
    }
}

// The two best blocks of superblock sb (blocks sb*SBS .. sb*SBS + SBS - 1,
// SBS <= 64) and the value bound R of every other key (the two blocks'
// second bounds, the other blocks' best values), from LDS, into the
// superblock entry.  One wavefront.
template <class Lds>
__device__ __forceinline__ void superblock_refresh(Lds& L, int sb, int sbshift, int NB) {
    const int lane = threadIdx.x & 63;
    const int b = (sb << sbshift) + lane;
    const bool in = lane < (1 << sbshift) && b < NB;
    const uint64_t v = in ? L.bkey[b] : 0ull;
    const uint32_t sec = in ? L.bsec[b] : 0u;
    // top two keys of the superblock in one merge (keys are unique)
    uint64_t a1 = v, a2 = 0;
    group_top2(a1, a2, 6);
    const uint64_t w1 = (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(a1 >> 32)), 63))) << 32) |
                        uint32_t(__builtin_amdgcn_readlane(int(uint32_t(a1)), 63));
    const uint64_t w2 = (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(a2 >> 32)), 63))) << 32) |
                        uint32_t(__builtin_amdgcn_readlane(int(uint32_t(a2)), 63));
    const int l1 = w1 != 0 ? __builtin_ctzll(__ballot(v == w1)) : -1;
    const int l2 = w2 != 0 ? __builtin_ctzll(__ballot(v == w2)) : -1;
    const uint32_t rest = wave_max_u32((lane == l1 || lane == l2) ? sec : uint32_t(v >> 32));
    if (lane == 0) {
        L.sbkey[sb] = w1;
        L.sbkey2[sb] = w2;
        L.sbsec[sb] = rest;
        L.sbblk[sb] = (sb << sbshift) + (l1 > 0 ? l1 : 0);
        L.sbblk2[sb] = (sb << sbshift) + (l2 > 0 ? l2 : 0);
    }
}

// Whole ordering of one object by one workgroup, several picks per round.
//
// A round: (1) every wavefront tests its block boxes against the picks that
// reach the superblocks they lie in -> touched-block masks; (2) few touched
// blocks: collect hit cells, update them with all lanes, rebuild the blocks'
// LDS entries; many: one wavefront per touched block; (3) refresh the
// touched superblocks; (4) every wavefront ranks and tests its share of the
// candidates for the next round and publishes them by rank through LDS.
template <int BLOCK, int MAXB>
__device__ inline void grid_order_object_mp(const GridObject& o, GridLdsMP<BLOCK / 64, MAXB>& L) {
    constexpr int NW = BLOCK / 64;
    constexpr int UMAX = BLOCK >= 1024 ? 2 : 4;  // member loads in flight per lane
    constexpr bool PREFETCH = BLOCK < 1024;      // next block's records during this one
    constexpr int BPT = MAXB / BLOCK;            // block boxes held per thread
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int k = o.k;
    const int NB = o.NB;
    int sbshift = 0;
    while ((64 << sbshift) < NB) ++sbshift;
    const int nsb = (NB + (1 << sbshift) - 1) >> sbshift;
    const int nwords = (NB + 63) >> 6;

    float blx[BPT], bly[BPT], blz[BPT], bhx[BPT], bhy[BPT], bhz[BPT];
    // block entries start from the grid build (best key, its coordinates and
    // cell, and a bound on the block's other keys): a block that no pick ever
    // reaches keeps them
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int b = j * BLOCK + tid;
        if (b < NB) {
            const float4 lo = o.bstat[2 * b], hi = o.bstat[2 * b + 1];
            blx[j] = lo.x; bly[j] = lo.y; blz[j] = lo.z;
            bhx[j] = hi.x; bhy[j] = hi.y; bhz[j] = hi.z;
            const uint4 d0 = o.bdyn[2 * b], d1 = o.bdyn[2 * b + 1];
            const uint64_t key = (uint64_t(d0.y) << 32) | d0.x;
            L.bkey[b] = key;
            L.bsec[b] = d1.w;
            L.bwin[b] = make_float4(__uint_as_float(d1.x), __uint_as_float(d1.y), __uint_as_float(d1.z),
                                    __int_as_float(int(d0.z)));
            L.bcell[b] = int(d0.w);
        } else {
            blx[j] = bly[j] = blz[j] = INFINITY;  // empty box: never touched
            bhx[j] = bhy[j] = bhz[j] = -INFINITY;
            L.bkey[b] = 0;
            L.bsec[b] = 0;
        }
    }
    if (wave == 0) {
        float slx = INFINITY, sly = INFINITY, slz = INFINITY, shx = -INFINITY, shy = -INFINITY,
              shz = -INFINITY;
        if (lane < nsb) {
            const int b0 = lane << sbshift;
            const int b1 = min(NB, b0 + (1 << sbshift));
            for (int b = b0; b < b1; ++b) {
                const float4 lo = o.bstat[2 * b], hi = o.bstat[2 * b + 1];
                slx = fminf(slx, lo.x); sly = fminf(sly, lo.y); slz = fminf(slz, lo.z);
                shx = fmaxf(shx, hi.x); shy = fmaxf(shy, hi.y); shz = fmaxf(shz, hi.z);
            }
        }
        L.sblo[lane] = make_float4(slx, sly, slz, 0.f);
        L.sbhi[lane] = make_float4(shx, shy, shz, 0.f);
        L.spm[lane] = lane < nsb ? 1u : 0u;  // the start may reach every superblock
        if (lane == 0) {
            // the start pick: pick 0, or the last pick of a leading scan
            // (already emitted; its update is this kernel's first round)
            const float4 sp = load_vec(o.xyzm + o.start_pos);
            if (o.t0 == 0) {
                o.order[0] = int32_t(o.start_id);
                if (o.radius) o.radius[0] = INFINITY;
                if (o.ticks) o.ticks[0] = wall_clock64();
            }
            L.pk[0] = make_float4(sp.x, sp.y, sp.z, o.start_m);
            L.pkpos[0] = o.start_pos;
            L.pkcell[0] = o.start_cell;
            L.pkid[0] = o.start_id;
            L.hcount = 0;
            L.hbcount = 0;
            L.overflow = 0;
        }
    }
    __syncthreads();
    for (int sb = wave; sb < nsb; sb += NW) superblock_refresh(L, sb, sbshift, NB);
    __syncthreads();

    int t = o.t0 + 1;  // picks emitted once this round's picks are
    int K = 1;         // picks of this round (ranks 0 .. K-1 of the LDS pick arrays)
    int round_no = 0;
    while (true) {
        // ---- the round's picks: lane j of every wavefront holds pick j
        float px = 0.f, py = 0.f, pz = 0.f, pm = 0.f;
        int ppos = 0, pcell = 0;
        if (lane < K) {
            const float4 q = L.pk[lane];
            px = q.x; py = q.y; pz = q.z; pm = q.w;
            ppos = L.pkpos[lane];
            pcell = L.pkcell[lane];
        }
        if (round_no > 0 && wave == 0 && lane < K) {  // emit them (the start pick was emitted before)
            o.order[t - K + lane] = int32_t(L.pkid[lane]);
            if (o.radius) o.radius[t - K + lane] = sqrtf(pm);
            if (o.ticks) o.ticks[t - K + lane] = wall_clock64();
        }
        const uint32_t kmask = K >= 32 ? 0xFFFFFFFFu : ((1u << K) - 1u);

        // ---- touched blocks: this wavefront's block boxes against the picks
        // that reach the superblocks they lie in
#pragma unroll
        for (int jb = 0; jb < BPT; ++jb) {
            const int b = jb * BLOCK + tid;
            const int sb = min(b >> sbshift, 63);
            const uint32_t mine = b < NB ? (L.spm[sb] & kmask) : 0u;
            uint32_t wm = 0;
            for (int j = 0; j < K; ++j) wm |= __ballot((mine >> j) & 1u) ? (1u << j) : 0u;
            // no m in the block exceeds its best key's value (0 past NB)
            const float bmax = key_value(L.bkey[b]);
            bool touch = false;
            for (uint32_t mm = wm; mm; mm &= mm - 1) {
                const int j = __builtin_ctz(mm);
                const float qx = rl(px, j), qy = rl(py, j), qz = rl(pz, j), qm = rl(pm, j);
                const int qb = __builtin_amdgcn_readlane(pcell, j) >> 6;
                touch = touch || (((mine >> j) & 1u) &&
                                  (b == qb || box_lower(blx[jb], bly[jb], blz[jb], bhx[jb], bhy[jb],
                                                        bhz[jb], qx, qy, qz) < fminf(qm, bmax)));
            }
            const uint64_t m = __ballot(touch);
            if (lane == 0) L.mask[jb * NW + wave] = m;
        }
        __syncthreads();

        const uint64_t mword = lane < nwords ? L.mask[lane] : 0ull;
        const uint32_t pc = uint32_t(__popcll(mword));
        const int touched = int(wave_sum_u32(pc));
        int nblk = 0, nhit = 0, ncells = 0;
        (void)nblk; (void)nhit; (void)ncells;
        uint64_t pacc[3] = {0, 0, 0};
        bool per_block = touched > L.kHitBlocks;
        int mycount = 0;  // touched blocks of this wavefront (few-block rounds)
        if (!per_block) {
            // this wavefront's touched blocks (ranks wave, wave + NW, ...) into tlist
            uint32_t ex = pc;  // exclusive prefix of the popcounts over lanes
            {
                uint32_t v = pc;
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t o2 = uint32_t(__shfl_up(int(v), d, 64));
                    if (lane >= d) v += o2;
                }
                ex = v - pc;
            }
            int r = int(ex);
            for (uint64_t mk = mword; mk; mk &= mk - 1, ++r)
                if (r % NW == wave) L.tlist[r] = lane * 64 + __builtin_ctzll(mk);
            wave_lds_sync();
            mycount = touched > wave ? (touched - wave + NW - 1) / NW : 0;

            // ---- collect hit cells, update them with all lanes, rebuild blocks
            BlockRec cur, nxt;
            if (PREFETCH && mycount > 0) cur = load_block(o, L.tlist[wave]);
            for (int i = 0; i < mycount; ++i) {
                const int b = L.tlist[wave + i * NW];
                if (PREFETCH && i + 1 < mycount) nxt = load_block(o, L.tlist[wave + (i + 1) * NW]);
                if (!PREFETCH) cur = load_block(o, b);
                collect_block(o, L, b, cur, K, px, py, pz, pm, pcell);
                if (PREFETCH) cur = nxt;
            }
            __syncthreads();
            per_block = L.overflow != 0;  // too many hit cells: redo the round per block
            if (!per_block) {
                update_cells<NW, UMAX>(o, L);
                __syncthreads();
                finish_blocks<NW>(L);
            }
        }
        if (per_block) {
            // ---- wavefront w updates the touched blocks of rank w, w + NW, ...
            const uint64_t nz = __ballot(mword != 0);
            BlockIter it{nz, 0ull, 0, 0};
            int b = next_block(it, mword, wave, NW);
            BlockRec cur;
            if (PREFETCH && b >= 0) cur = load_block(o, b);
            while (b >= 0) {  // the next block's records load while this one is processed
                const int nb = next_block(it, mword, wave, NW);
                BlockRec nxt;
                if (PREFETCH && nb >= 0) nxt = load_block(o, nb);
                if (!PREFETCH) cur = load_block(o, b);
                const int nh = process_block_mp<UMAX>(o, L, b, cur, K, px, py, pz, pm, ppos, pcell, pacc);
                ++nblk;
                nhit += nh > 0 ? 1 : 0;
                ncells += nh;
                b = nb;
                if (PREFETCH) cur = nxt;
            }
        }
        __syncthreads();

        // ---- refresh the touched superblocks, spread over the wavefronts;
        // clear the selection's LDS state (nothing reads it before the barrier)
        {
            bool st = false;
            if (lane < nsb) {
                const int b0 = lane << sbshift;
                const int nb = 1 << sbshift;
                if (nb >= 64) {
                    st = L.mask[b0 >> 6] != 0;
                } else {
                    const uint64_t w = L.mask[b0 >> 6] >> (b0 & 63);
                    st = (w & ((1ull << nb) - 1)) != 0;
                }
            }
            int r2 = 0;
            for (uint64_t ts = __ballot(st); ts; ts &= ts - 1) {
                const int sb = __builtin_ctzll(ts);
                if (r2 % NW == wave) superblock_refresh(L, sb, sbshift, NB);
                ++r2;
            }
            if (wave == NW - 1) {
                L.spm[lane] = 0u;
                if (lane == 0) {
                    L.kfail = kMaxPicks;
                    L.hcount = 0;
                    L.hbcount = 0;
                    L.overflow = 0;
                }
            }
        }
        __syncthreads();
        if (t >= k) break;

        // ---- next picks.  Candidates: the entries (lane = superblock, slot 1
        // or 2) above the top superblock's bound, and the top entry itself.
        // Every wavefront ranks every NW-th candidate; a candidate of rank r
        // fails when some higher-ranked candidate lowers it or comes from a
        // superblock whose bound R reaches its value.
        const int cap = min(min(o.max_picks, kMaxPicks), k - t);
        const bool inl = lane < nsb;
        const uint64_t e1 = inl ? L.sbkey[lane] : 0ull;
        const uint64_t e2 = inl ? L.sbkey2[lane] : 0ull;
        const uint32_t rb = inl ? L.sbsec[lane] : 0u;
        const uint64_t top = wave_max_key(e1);
        const int tl = __builtin_ctzll(__ballot(e1 == top) | (1ull << 63));
        const uint32_t trb = uint32_t(__builtin_amdgcn_readlane(int(rb), tl));
        const bool c1 = e1 != 0 && (lane == tl || uint32_t(e1 >> 32) > trb);
        const bool c2 = e2 != 0 && uint32_t(e2 >> 32) > trb;
        const uint64_t m1 = __ballot(c1), m2 = __ballot(c2);
        const int nc = __popcll(m1) + __popcll(m2);
        float4 w1 = make_float4(0.f, 0.f, 0.f, 0.f), w2 = w1;
        int cl1 = 0, cl2 = 0;
        if (c1) {
            const int bb = L.sbblk[lane];
            w1 = L.bwin[bb];
            cl1 = L.bcell[bb];
        }
        if (c2) {
            const int bb = L.sbblk2[lane];
            w2 = L.bwin[bb];
            cl2 = L.bcell[bb];
        }
        const float4 slo = L.sblo[lane], shi = L.sbhi[lane];
        const uint64_t lt = (1ull << lane) - 1ull;
        const int i1 = __popcll(m1 & lt) + __popcll(m2 & lt);  // position of slot 1 in lane order
        const int i2 = i1 + (c1 ? 1 : 0);
        const uint64_t my1 = __ballot(c1 && (i1 % NW) == wave);
        const uint64_t my2 = __ballot(c2 && (i2 % NW) == wave);
#pragma unroll
        for (int slot = 0; slot < 2; ++slot) {
            const uint64_t ek = slot == 0 ? e1 : e2;
            const float4 wk = slot == 0 ? w1 : w2;
            const int ck = slot == 0 ? cl1 : cl2;
            for (uint64_t mm = slot == 0 ? my1 : my2; mm; mm &= mm - 1) {
                const int lc = __builtin_ctzll(mm);
                const uint32_t klo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(ek)), lc));
                const uint32_t khi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(ek >> 32)), lc));
                const uint64_t kc = (uint64_t(khi) << 32) | klo;
                const bool g1 = c1 && e1 > kc, g2 = c2 && e2 > kc;
                const int rank = __popcll(__ballot(g1)) + __popcll(__ballot(g2));
                if (rank >= cap) continue;
                const float cx = rl(wk.x, lc), cy = rl(wk.y, lc), cz = rl(wk.z, lc);
                const int cpos = __builtin_amdgcn_readlane(__float_as_int(wk.w), lc);
                const int ccell = __builtin_amdgcn_readlane(ck, lc);
                const float cm = key_value(kc);
                const bool f = (g1 && (dist2(w1.x, w1.y, w1.z, cx, cy, cz) < cm || khi <= rb)) ||
                               (g2 && (dist2(w2.x, w2.y, w2.z, cx, cy, cz) < cm || khi <= rb));
                const bool fail = __ballot(f) != 0;
                const int csb = (ccell >> 6) >> sbshift;
                const bool reach = inl && (lane == csb ||
                                           box_lower(slo.x, slo.y, slo.z, shi.x, shi.y, shi.z, cx, cy, cz) <
                                               fminf(cm, key_value(e1)));
                if (reach) atomicOr(&L.spm[lane], 1u << rank);
                if (lane == 0) {
                    if (fail) atomicMin(&L.kfail, rank);
                    L.pk[rank] = make_float4(cx, cy, cz, cm);
                    L.pkpos[rank] = cpos;
                    L.pkcell[rank] = ccell;
                    L.pkid[rank] = key_id(kc);
                }
            }
        }
        ++round_no;
        __syncthreads();
        K = min(min(L.kfail, nc), cap);
        if (K <= 0) break;  // cannot happen while t < k <= n; keeps the loop finite
        t += K;
    }
}

}  // namespace bs
