// bs_grid.hip -- uniform-grid radius-pruned greedy permutation for gfx950.
//
// Same ordering as the resident full scan (paper Sec. 3.2 / 3.3: append the
// remaining candidate farthest from its nearest chosen surfel), but a step
// only touches candidates that can change.  After picking c with squared
// covering radius mc (every remaining m_i <= mc), m_i can only drop when
// d2(p_i, c) < m_i <= mc.  Candidates are grouped into cubic grid cells (a
// Morton-sorted uniform grid whose level is chosen on the device for a
// target mean occupancy) and cells into blocks of B consecutive cells.  For
// a cell (or block) with exact member box [lo, hi], the box lower bound
//     L = ((gx*gx + gy*gy) + gz*gz),  gx = lo.x - c.x if c.x < lo.x,
//                                         c.x - hi.x if c.x > hi.x, else 0
// evaluated in binary32 is <= d2(p, c) for every member p, because each
// binary32 operation is monotone in its arguments; so L >= mc proves that
// no member changes and the cell is skipped, with no tolerance.
//
// Per object, one workgroup runs the whole ordering.  Block maxima and block
// boxes live in LDS; cell records (box, start, count, current best key and
// its coordinates) and the Morton-sorted candidates (x, y, z, m) live in
// HBM.  A step: test all block boxes (LDS) -> load the touched blocks' cell
// records (round trip 1) -> one wavefront per hit cell loads and updates its
// members and reduces the cell's best (round trip 2) -> recompute touched
// block maxima -> argmax over blocks (LDS).
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <math.h>
#include <stdint.h>

#include "bs_grid.h"
#include "bs_internal.h"

namespace bs {
namespace {

constexpr int kMortonBits = 10;  // per axis
constexpr int kMaxBlocks = 1024; // blocks of 64 cells per object (LDS-resident maxima)

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

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
    v = dpp_max_step<0xB1, 0xF>(v);
    v = dpp_max_step<0x4E, 0xF>(v);
    v = dpp_max_step<0x141, 0xF>(v);
    v = dpp_max_step<0x140, 0xF>(v);
    v = dpp_max_step<0x142, 0xA>(v);
    v = dpp_max_step<0x143, 0xC>(v);
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), 63));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), 63));
    return (uint64_t(hi) << 32) | lo;
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

// ------------------------------------------------------------ preprocessing

__global__ void init_grid_header_kernel(GridHeader* gh) {
    if (threadIdx.x < 64) reinterpret_cast<uint32_t*>(gh)[threadIdx.x] = 0u;
}

__global__ void morton_kernel(const float* __restrict__ pts, int n, const DevHeader* hdr,
                              uint32_t* __restrict__ codes, uint32_t* __restrict__ vals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float lx = ord_decode(hdr->bbox[0]), ly = ord_decode(hdr->bbox[1]),
                lz = ord_decode(hdr->bbox[2]);
    const float hx = ord_decode(hdr->bbox[3]), hy = ord_decode(hdr->bbox[4]),
                hz = ord_decode(hdr->bbox[5]);
    float ext = fmaxf(hx - lx, fmaxf(hy - ly, hz - lz));
    const float scale = (ext > 0.f && isfinite(ext)) ? float(1 << kMortonBits) / ext : 0.f;
    uint32_t q[3];
    const float lo[3] = {lx, ly, lz};
    for (int a = 0; a < 3; ++a) {
        float f = (pts[3 * i + a] - lo[a]) * scale;
        int v = isfinite(f) ? int(f) : 0;
        v = v < 0 ? 0 : (v > (1 << kMortonBits) - 1 ? (1 << kMortonBits) - 1 : v);
        q[a] = uint32_t(v);
    }
    codes[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
    vals[i] = uint32_t(i);
}

// hist[l] = number of adjacent sorted pairs whose cells first differ at level l
__global__ void level_hist_kernel(const uint32_t* __restrict__ codes, int n, GridHeader* gh) {
    __shared__ uint32_t h[kMortonBits + 1];
    if (threadIdx.x <= kMortonBits) h[threadIdx.x] = 0;
    __syncthreads();
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x + 1; i < n; i += stride) {
        const uint32_t d = codes[i] ^ codes[i - 1];
        if (d) {
            const int b = 31 - __clz(d);            // highest differing bit
            const int l = kMortonBits - b / 3;       // first level that separates them
            atomicAdd(&h[l], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x <= kMortonBits && h[threadIdx.x]) atomicAdd(&gh->hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void choose_level_kernel(int n, GridHeader* gh, float target) {
    if (threadIdx.x != 0) return;
    const double cap = fmin(fmax(1.0, double(n) / double(target)), double(64 * kMaxBlocks));
    int level = 0;
    uint32_t cells = 1, acc = 1;
    for (int l = 1; l <= kMortonBits; ++l) {
        acc += gh->hist[l];
        if (double(acc) <= cap) {
            level = l;
            cells = acc;
        }
    }
    gh->level = level;
    gh->C = int(cells);
    gh->B = 64;
    gh->NB = int((cells + 63) / 64);
}

__global__ void cell_flag_kernel(const uint32_t* __restrict__ codes, int n, const GridHeader* gh,
                                 uint32_t* __restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = 3 * (kMortonBits - gh->level);
    flags[i] = (i == 0 || (codes[i] >> s) != (codes[i - 1] >> s)) ? 1u : 0u;
}

__global__ void gather_kernel(const float* __restrict__ pts, const uint32_t* __restrict__ ids,
                              const uint32_t* __restrict__ flags,
                              const uint32_t* __restrict__ cellidx, int n, int start,
                              GridHeader* gh, float4* __restrict__ xyzm,
                              int32_t* __restrict__ cstart) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t id = ids[i];
    xyzm[i] = make_float4(pts[3 * id + 0], pts[3 * id + 1], pts[3 * id + 2], INFINITY);
    const int cell = int(cellidx[i]) - 1;
    if (flags[i]) cstart[cell] = i;
    if (int(id) == start) {
        gh->start_pos = i;
        gh->start_cell = cell;
    }
}

// One thread per cell: exact member box, start/count, initial best (all m = +inf:
// the lowest original index wins).
__global__ void cell_build_kernel(const int32_t* __restrict__ cstart, int n,
                                  const GridHeader* gh, const float4* __restrict__ xyzm,
                                  const uint32_t* __restrict__ ids, float4* __restrict__ cstat,
                                  uint4* __restrict__ cdyn) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int C = gh->C;
    if (c >= C) return;
    const int s = cstart[c];
    const int e = (c + 1 < C) ? cstart[c + 1] : n;
    float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY,
          hz = -INFINITY;
    uint32_t best_id = 0xFFFFFFFFu;
    int best_pos = s;
    for (int i = s; i < e; ++i) {
        const float4 p = xyzm[i];
        lx = fminf(lx, p.x);
        ly = fminf(ly, p.y);
        lz = fminf(lz, p.z);
        hx = fmaxf(hx, p.x);
        hy = fmaxf(hy, p.y);
        hz = fmaxf(hz, p.z);
        if (ids[i] < best_id) {
            best_id = ids[i];
            best_pos = i;
        }
    }
    cstat[2 * c + 0] = make_float4(lx, ly, lz, __int_as_float(s));
    cstat[2 * c + 1] = make_float4(hx, hy, hz, __int_as_float(e - s));
    const uint64_t key = make_key(INFINITY, best_id);
    const float4 w = xyzm[best_pos];
    cdyn[2 * c + 0] = make_uint4(uint32_t(key), uint32_t(key >> 32), uint32_t(best_pos), 0u);
    cdyn[2 * c + 1] = make_uint4(__float_as_uint(w.x), __float_as_uint(w.y), __float_as_uint(w.z), 0u);
}

// One thread per block: union box and best over its cells.
__global__ void block_build_kernel(const GridHeader* gh, const float4* __restrict__ cstat,
                                   const uint4* __restrict__ cdyn, float4* __restrict__ bstat,
                                   uint4* __restrict__ bdyn) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= gh->NB) return;
    const int C = gh->C, B = gh->B;
    float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY,
          hz = -INFINITY;
    uint64_t best = 0;
    int bc = b * B;
    for (int c = b * B; c < C && c < (b + 1) * B; ++c) {
        const float4 lo = cstat[2 * c], hi = cstat[2 * c + 1];
        lx = fminf(lx, lo.x);
        ly = fminf(ly, lo.y);
        lz = fminf(lz, lo.z);
        hx = fmaxf(hx, hi.x);
        hy = fmaxf(hy, hi.y);
        hz = fmaxf(hz, hi.z);
        const uint4 d = cdyn[2 * c];
        const uint64_t key = (uint64_t(d.y) << 32) | d.x;
        if (key > best) {
            best = key;
            bc = c;
        }
    }
    bstat[2 * b + 0] = make_float4(lx, ly, lz, 0.f);
    bstat[2 * b + 1] = make_float4(hx, hy, hz, 0.f);
    const uint4 d0 = cdyn[2 * bc], d1 = cdyn[2 * bc + 1];
    bdyn[2 * b + 0] = make_uint4(d0.x, d0.y, d0.z, uint32_t(bc));
    bdyn[2 * b + 1] = d1;
}

}  // namespace

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
template <int NW>
struct GridLds {
    uint64_t mask[kMaxBlocks / 64];
    uint64_t bkey[kMaxBlocks];
    float4 bwin[kMaxBlocks];
    int bcell[kMaxBlocks];
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

#ifdef BS_PHASE_PROF
#define BS_PROF(slot) \
    do { if (o.ticks && threadIdx.x == 0) o.ticks[size_t(prof_t) * 16 + (slot)] = wall_clock64(); } while (0)
#else
#define BS_PROF(slot) do { } while (0)
#endif

// One wavefront updates every candidate of block b that the pick can reach
// and rewrites the block's best into LDS.  The nh hit cells each get an
// aligned group of 64 / 2^ceil(log2 nh) lanes.  Wave-local: no barrier.
// Loads are issued unconditionally (clamped to a valid address) so that a
// batch of them is in flight together.
template <int NW>
__device__ void process_block(const GridObject& o, GridLds<NW>& L, int b, int c_pos, int c_cell,
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
    BS_PROF(8);
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
    for (int q0 = s; q0 < count; q0 += G * kUnroll) {
        int pos[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int q = q0 + u * G;
            ok[u] = q < count;
            pos[u] = start + (ok[u] ? q : 0);
        }
        float4 p[kUnroll];
        uint32_t id[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) p[u] = xyzm[pos[u]];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) id[u] = ids[pos[u]];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const bool pick = ok[u] && pos[u] == c_pos;
            const bool live = ok[u] && !pick && p[u].w >= 0.f;
            const float d = dist2(p[u].x, p[u].y, p[u].z, cx, cy, cz);
            const bool dec = live && d < p[u].w;
            const float m = dec ? d : p[u].w;
            if (dec || (pick && p[u].w != -1.f)) xyzm[pos[u]].w = pick ? -1.f : d;
            const uint64_t kk = live ? make_key(m, id[u]) : 0ull;
            const bool better = kk > lk;
            lk = better ? kk : lk;
            lw = better ? make_float4(p[u].x, p[u].y, p[u].z, __int_as_float(pos[u])) : lw;
        }
    }
    BS_PROF(9);

    if (nh == 1) {
        const int h = __builtin_ctzll(hm);
        const uint64_t wk = wave_max_u64(lk);
        const int wl = __builtin_ctzll(__ballot(lk == wk) | (1ull << 63));
        const float wx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lw.x), wl));
        const float wy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lw.y), wl));
        const float wz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lw.z), wl));
        const float wp = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lw.w), wl));
        if (lane == h) {
            ckey = wk;
            cwin = make_float4(wx, wy, wz, wp);
        }
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
        }
    }
    if (hit) {
        o.cdyn[2 * cell + 0] = make_uint4(uint32_t(ckey), uint32_t(ckey >> 32),
                                          uint32_t(__float_as_int(cwin.w)), 0u);
        o.cdyn[2 * cell + 1] = make_uint4(__float_as_uint(cwin.x), __float_as_uint(cwin.y),
                                          __float_as_uint(cwin.z), 0u);
    }
    const uint64_t bk = wave_max_u64(ckey);
    if (bk != 0 && ckey == bk) {
        L.bwin[b] = cwin;
        L.bcell[b] = cell;
    }
    if (lane == 0) L.bkey[b] = bk;
    wave_lds_sync();
    BS_PROF(10);
}

// Best block of superblock sb (64 consecutive blocks), computed by one
// wavefront from LDS: (key, block).
template <int NW>
__device__ __forceinline__ void superblock_best(GridLds<NW>& L, int sb, uint64_t& key, int& blk) {
    const int lane = threadIdx.x & 63;
    const uint64_t v = L.bkey[sb * 64 + lane];
    key = wave_max_u64(v);
    blk = sb * 64 + __builtin_ctzll(__ballot(v == key) | (1ull << 63));
}

// Whole ordering of one object by one workgroup (steps 1 .. k-1).
template <int BLOCK>
__device__ void grid_order_object(const GridObject& o, GridLds<BLOCK / 64>& L) {
    constexpr int NW = BLOCK / 64;
    constexpr int BPT = kMaxBlocks / BLOCK;  // block boxes held per thread
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

    int c_pos = o.start_pos, c_cell = o.start_cell;
    const float4 sp = o.xyzm[c_pos];
    float cx = sp.x, cy = sp.y, cz = sp.z;
    float mc = INFINITY;
    if (tid == 0) {
        o.order[0] = int32_t(o.start_id);
        if (o.radius) o.radius[0] = INFINITY;
#ifndef BS_PHASE_PROF
        if (o.ticks) o.ticks[0] = wall_clock64();
#endif
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
        BS_PROF(0);
        // blocks that may hold a candidate whose m can drop, or the pick
        const int cb = c_cell >> 6;
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int b = j * BLOCK + tid;
            const bool touch =
                b == cb || box_lower(blx[j], bly[j], blz[j], bhx[j], bhy[j], bhz[j], cx, cy, cz) < mc;
            const uint64_t m = __ballot(touch);
            if (lane == 0) L.mask[j * NW + wave] = m;
        }
        BS_PROF(1);
        __syncthreads();
        BS_PROF(2);

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
        BS_PROF(3);
        __syncthreads();
        BS_PROF(4);

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
        BS_PROF(5);
        const uint64_t best = wave_max_u64(sbk);
        const int wl = __builtin_ctzll(__ballot(sbk == best) | (1ull << 63));
        const int bb = __builtin_amdgcn_readlane(sbb, wl);
        const float4 win = L.bwin[bb];
        c_cell = L.bcell[bb];
        c_pos = __float_as_int(win.w);
        cx = win.x;
        cy = win.y;
        cz = win.z;
        mc = key_value(best);
        BS_PROF(6);
        if (tid == 0) {
            o.order[t] = int32_t(key_id(best));
            if (o.radius) o.radius[t] = sqrtf(mc);
#ifndef BS_PHASE_PROF
            if (o.ticks) o.ticks[t] = wall_clock64();
#endif
        }
    }
}

namespace {

template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) grid_single_kernel(GridObject o, const DevHeader* hdr,
                                                            const GridHeader* gh) {
    __shared__ GridLds<BLOCK / 64> L;
    GridObject obj = o;
    if (o.k <= 0) return;
    if (hdr->nonfinite) {
        for (int t = threadIdx.x; t < o.k; t += BLOCK) {
            o.order[t] = -1;
            if (o.radius) o.radius[t] = __builtin_nanf("");
        }
        return;
    }
    obj.C = gh->C;
    obj.B = gh->B;
    obj.NB = gh->NB;
    obj.start_pos = gh->start_pos;
    obj.start_cell = gh->start_cell;
    grid_order_object<BLOCK>(obj, L);
}

}  // namespace

// ------------------------------------------------------------ host side

GridLayout grid_layout(int64_t n, int block) {
    GridLayout g;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(bytes);
        return at;
    };
    const size_t N = size_t(n);
    const size_t maxC = N;  // level choice keeps C <= max(1, n / target) <= n
    g.dev_header = take(sizeof(DevHeader));
    g.grid_header = take(sizeof(GridHeader));
    g.codes = take(N * 4);
    g.vals = take(N * 4);
    g.codes_sorted = take(N * 4);
    g.ids = take(N * 4);
    g.flags = take(N * 4);
    g.cellidx = take(N * 4);
    g.cstart = take(maxC * 4);
    g.xyzm = take(N * 16);
    g.cstat = take(maxC * 32);
    g.cdyn = take(maxC * 32);
    g.bstat = take(size_t(kMaxBlocks) * 32);
    g.bdyn = take(size_t(kMaxBlocks) * 32);
    size_t sort_bytes = 0, scan_bytes = 0;
    hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                       (const uint32_t*)nullptr, (uint32_t*)nullptr, int(n), 0,
                                       3 * kMortonBits);
    hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                     int(n));
    g.temp = take(sort_bytes > scan_bytes ? sort_bytes : scan_bytes);
    g.temp_bytes = sort_bytes > scan_bytes ? sort_bytes : scan_bytes;
    g.total = off;
    return g;
}

int grid_block_size(int64_t n) { return n > (int64_t(1) << 16) ? 1024 : 256; }

hipError_t launch_grid(const float* pts, int n, int k, int start, int32_t* order, float* radius,
                       void* ws, float target, int block, uint64_t* ticks, hipStream_t st) {
    const GridLayout g = grid_layout(n, block);
    char* base = static_cast<char*>(ws);
    DevHeader* hdr = reinterpret_cast<DevHeader*>(base + g.dev_header);
    GridHeader* gh = reinterpret_cast<GridHeader*>(base + g.grid_header);
    uint32_t* codes = reinterpret_cast<uint32_t*>(base + g.codes);
    uint32_t* vals = reinterpret_cast<uint32_t*>(base + g.vals);
    uint32_t* codes_s = reinterpret_cast<uint32_t*>(base + g.codes_sorted);
    uint32_t* ids = reinterpret_cast<uint32_t*>(base + g.ids);
    uint32_t* flags = reinterpret_cast<uint32_t*>(base + g.flags);
    uint32_t* cellidx = reinterpret_cast<uint32_t*>(base + g.cellidx);
    int32_t* cstart = reinterpret_cast<int32_t*>(base + g.cstart);
    float4* xyzm = reinterpret_cast<float4*>(base + g.xyzm);
    float4* cstat = reinterpret_cast<float4*>(base + g.cstat);
    uint4* cdyn = reinterpret_cast<uint4*>(base + g.cdyn);
    float4* bstat = reinterpret_cast<float4*>(base + g.bstat);
    uint4* bdyn = reinterpret_cast<uint4*>(base + g.bdyn);
    void* temp = base + g.temp;

    hipError_t e = launch_init_header(hdr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(init_grid_header_kernel, dim3(1), dim3(64), 0, st, gh);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_validate(pts, n, hdr, st)) != hipSuccess) return e;
    const int tb = 256;
    const int nblk = (n + tb - 1) / tb;
    hipLaunchKernelGGL(morton_kernel, dim3(nblk), dim3(tb), 0, st, pts, n, hdr, codes, vals);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    size_t tbytes = g.temp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(temp, tbytes, codes, codes_s, vals, ids, n, 0,
                                           3 * kMortonBits, st);
    if (e != hipSuccess) return e;
    const int hblk = nblk < 1024 ? nblk : 1024;
    hipLaunchKernelGGL(level_hist_kernel, dim3(hblk), dim3(tb), 0, st, codes_s, n, gh);
    hipLaunchKernelGGL(choose_level_kernel, dim3(1), dim3(64), 0, st, n, gh, target);
    hipLaunchKernelGGL(cell_flag_kernel, dim3(nblk), dim3(tb), 0, st, codes_s, n, gh, flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    tbytes = g.temp_bytes;
    e = hipcub::DeviceScan::InclusiveSum(temp, tbytes, flags, cellidx, n, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gather_kernel, dim3(nblk), dim3(tb), 0, st, pts, ids, flags, cellidx, n, start,
                       gh, xyzm, cstart);
    hipLaunchKernelGGL(cell_build_kernel, dim3(nblk), dim3(tb), 0, st, cstart, n, gh, xyzm, ids, cstat,
                       cdyn);
    hipLaunchKernelGGL(block_build_kernel, dim3((kMaxBlocks + tb - 1) / tb), dim3(tb), 0, st, gh, cstat,
                       cdyn, bstat, bdyn);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    GridObject o{};
    o.k = k;
    o.start_id = uint32_t(start);
    o.xyzm = xyzm;
    o.ids = ids;
    o.cstat = cstat;
    o.cdyn = cdyn;
    o.bstat = bstat;
    o.bdyn = bdyn;
    o.order = order;
    o.radius = radius;
    o.ticks = ticks;
    if (block == 1024)
        hipLaunchKernelGGL(grid_single_kernel<1024>, dim3(1), dim3(1024), 0, st, o, hdr, gh);
    else
        hipLaunchKernelGGL(grid_single_kernel<256>, dim3(1), dim3(256), 0, st, o, hdr, gh);
    return hipGetLastError();
}

}  // namespace bs
