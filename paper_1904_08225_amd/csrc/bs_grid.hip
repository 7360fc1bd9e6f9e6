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
#include <math.h>
#include <stdint.h>

#include "bs_grid.h"
#include "bs_grid_device.h"
#include "bs_grid_multi.h"
#include "bs_internal.h"
#include "bs_sample_device.h"

namespace bs {
namespace {

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

// Cells are the runs of sorted codes sharing their top `level` bits (one
// bit at a time: each step halves a cell along one axis, so the cell count
// can follow the target closely).  hist[p] = number of adjacent sorted pairs
// whose codes first differ within the top p bits (p = 1 .. 3 * kMortonBits).
__global__ void level_hist_kernel(const uint32_t* __restrict__ codes, int n, GridHeader* gh) {
    constexpr int kBits = 3 * kMortonBits;
    __shared__ uint32_t h[kBits + 1];
    if (threadIdx.x <= kBits) h[threadIdx.x] = 0;
    __syncthreads();
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x + 1; i < n; i += stride) {
        const uint32_t d = codes[i] ^ codes[i - 1];
        if (d) {
            const int b = 31 - __clz(d);  // highest differing bit (< kBits)
            atomicAdd(&h[kBits - b], 1u); // first prefix length that separates them
        }
    }
    __syncthreads();
    if (threadIdx.x <= kBits && h[threadIdx.x]) atomicAdd(&gh->hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void choose_level_kernel(int n, GridHeader* gh, float target, int max_blocks) {
    if (threadIdx.x != 0) return;
    const double cap = fmin(fmax(1.0, double(n) / double(target)), double(64 * max_blocks));
    int level = 0;
    uint32_t cells = 1, acc = 1;
    for (int l = 1; l <= 3 * kMortonBits; ++l) {
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
    const int s = 3 * kMortonBits - gh->level;
    flags[i] = (i == 0 || (codes[i] >> s) != (codes[i - 1] >> s)) ? 1u : 0u;
}

// m_in: NULL (every m = +inf) or each candidate's m left by a leading scan,
// whose last pick (gh->lead_id) is then the start.
__global__ void gather_kernel(const float* __restrict__ pts, const uint32_t* __restrict__ ids,
                              const uint32_t* __restrict__ flags,
                              const uint32_t* __restrict__ cellidx, int n, int start,
                              GridHeader* gh, float4* __restrict__ xyzm,
                              int32_t* __restrict__ cstart, const float* __restrict__ m_in) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t id = ids[i];
    if (m_in) start = int(gh->lead_id);
    xyzm[i] = make_float4(pts[3 * id + 0], pts[3 * id + 1], pts[3 * id + 2], m_in ? m_in[id] : INFINITY);
    const int cell = int(cellidx[i]) - 1;
    if (flags[i]) cstart[cell] = i;
    if (int(id) == start) {
        gh->start_pos = i;
        gh->start_cell = cell;
    }
}

// Candidates in Morton order for the sorted full scan: x, y, z, m = +inf.
__global__ void sorted_gather_kernel(const float* __restrict__ pts, const uint32_t* __restrict__ ids, int n,
                                     int start, GridHeader* gh, float4* __restrict__ xyzm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t id = ids[i];
    xyzm[i] = make_float4(pts[3 * id + 0], pts[3 * id + 1], pts[3 * id + 2], INFINITY);
    if (int(id) == start) gh->start_pos = i;
}

// One thread per cell: exact member box, start/count, best and second key
// of the members' m (chosen candidates, m = -1, have none).
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
    uint64_t key = 0, sec = 0;
    int best_pos = s;
    for (int i = s; i < e; ++i) {
        const float4 p = xyzm[i];
        lx = fminf(lx, p.x);
        ly = fminf(ly, p.y);
        lz = fminf(lz, p.z);
        hx = fmaxf(hx, p.x);
        hy = fmaxf(hy, p.y);
        hz = fmaxf(hz, p.z);
        const uint64_t kk = p.w >= 0.f ? make_key(p.w, ids[i]) : 0ull;
        if (kk > key) {
            sec = key;
            key = kk;
            best_pos = i;
        } else if (kk > sec) {
            sec = kk;
        }
    }
    cstat[2 * c + 0] = make_float4(lx, ly, lz, __int_as_float(s));
    cstat[2 * c + 1] = make_float4(hx, hy, hz, __int_as_float(e - s));
    const float4 w = xyzm[best_pos];
    // second key slot (w words): the cell's second key
    cdyn[2 * c + 0] = make_uint4(uint32_t(key), uint32_t(key >> 32), uint32_t(best_pos), uint32_t(sec));
    cdyn[2 * c + 1] = make_uint4(__float_as_uint(w.x), __float_as_uint(w.y), __float_as_uint(w.z),
                                 uint32_t(sec >> 32));
}

// One thread per block: union box, best over its cells, and in the last word
// the value bits of a bound on the block's other keys (the best cell's second
// key and the other cells' best keys).
__global__ void block_build_kernel(const GridHeader* gh, const float4* __restrict__ cstat,
                                   const uint4* __restrict__ cdyn, float4* __restrict__ bstat,
                                   uint4* __restrict__ bdyn) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= gh->NB) return;
    const int C = gh->C, B = gh->B;
    float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY,
          hz = -INFINITY;
    uint64_t best = 0;
    uint32_t other = 0;  // value bits of the best key among the cells that are not the best cell
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
            if (best) other = max(other, uint32_t(best >> 32));
            best = key;
            bc = c;
        } else {
            other = max(other, d.y);
        }
    }
    bstat[2 * b + 0] = make_float4(lx, ly, lz, 0.f);
    bstat[2 * b + 1] = make_float4(hx, hy, hz, 0.f);
    const uint4 d0 = cdyn[2 * bc], d1 = cdyn[2 * bc + 1];
    bdyn[2 * b + 0] = make_uint4(d0.x, d0.y, d0.z, uint32_t(bc));
    bdyn[2 * b + 1] = make_uint4(d1.x, d1.y, d1.z, max(other, d1.w));
}

// One thread per superblock (64 consecutive blocks): union box.
__global__ void superblock_build_kernel(const GridHeader* gh, const float4* __restrict__ bstat,
                                        float4* __restrict__ sbstat) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int NB = gh->NB;
    if (s * 64 >= NB) return;
    float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY,
          hz = -INFINITY;
    for (int b = s * 64; b < NB && b < (s + 1) * 64; ++b) {
        const float4 lo = bstat[2 * b], hi = bstat[2 * b + 1];
        lx = fminf(lx, lo.x);
        ly = fminf(ly, lo.y);
        lz = fminf(lz, lo.z);
        hx = fmaxf(hx, hi.x);
        hy = fmaxf(hy, hi.y);
        hz = fmaxf(hz, hi.z);
    }
    sbstat[2 * s + 0] = make_float4(lx, ly, lz, 0.f);
    sbstat[2 * s + 1] = make_float4(hx, hy, hz, 0.f);
}

}  // namespace

namespace {

template <int BLOCK, int MAXB>
__global__ void __launch_bounds__(BLOCK) grid_single_kernel(GridObject o, const DevHeader* hdr,
                                                            const GridHeader* gh) {
    __shared__ GridLds<BLOCK / 64, MAXB> L;
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
    grid_order_object<BLOCK, MAXB>(obj, L);
}

template <int BLOCK, int MAXB>
__global__ void __launch_bounds__(BLOCK) grid_multi_kernel(GridObject o, const DevHeader* hdr,
                                                           const GridHeader* gh) {
    __shared__ GridLdsMP<BLOCK / 64, MAXB> L;
    GridObject obj = o;
    if (o.k <= 0) return;
    if (hdr->nonfinite) {
        for (int t = threadIdx.x; t < o.k; t += BLOCK) {
            o.order[t] = -1;
            if (o.radius) o.radius[t] = __builtin_nanf("");
        }
        return;
    }
    if (hdr->error) return;  // a leading scan gave up: its state is incomplete
    obj.C = gh->C;
    obj.B = gh->B;
    obj.NB = gh->NB;
    obj.start_pos = gh->start_pos;
    obj.start_cell = gh->start_cell;
    if (o.t0 > 0) {
        obj.start_id = gh->lead_id;
        obj.start_m = __uint_as_float(gh->lead_m);
    }
    grid_order_object_mp<BLOCK, MAXB>(obj, L);
}

// pos_of[id] = sorted position of candidate id
__global__ void position_kernel(const uint32_t* __restrict__ ids, int n, int32_t* __restrict__ pos_of) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pos_of[ids[i]] = i;
}

// The paper's randomized sampler (Sec. 3.2) on one object's grid.
template <int BLOCK, int MAXB>
__global__ void __launch_bounds__(BLOCK) sample_single_kernel(GridObject o, SampleSpec sp, const DevHeader* hdr,
                                                              const GridHeader* gh) {
    __shared__ GridLds<BLOCK / 64, MAXB> L;
    __shared__ SampleLds<BLOCK / 64> SL;
    GridObject obj = o;
    if (o.k <= 0) return;
    if (hdr->nonfinite) {
        for (int t = threadIdx.x; t < o.k; t += BLOCK) {
            o.order[t] = -1;
            if (o.radius) o.radius[t] = __builtin_nanf("");
        }
        if (threadIdx.x == 0 && sp.count) *sp.count = 0;
        return;
    }
    obj.C = gh->C;
    obj.B = gh->B;
    obj.NB = gh->NB;
    obj.start_pos = gh->start_pos;
    obj.start_cell = gh->start_cell;
    sample_object<BLOCK, MAXB>(obj, sp, L, SL);
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
    g.bstat = take(size_t(kMaxBlocksAny) * 32);
    g.bdyn = take(size_t(kMaxBlocksAny) * 32);
    g.sbstat = take(size_t(kMaxBlocksAny / 64) * 32);
    g.lead_slots = take(scan_slot_bytes(kMaxCoopGroups));
    const size_t sort_bytes = sort_temp_bytes(sort_tile_count(n)), scan_bytes = scan_temp_bytes(n);
    g.temp = take(sort_bytes > scan_bytes ? sort_bytes : scan_bytes);
    g.temp_bytes = sort_bytes > scan_bytes ? sort_bytes : scan_bytes;
    g.total = off;
    return g;
}

hipError_t launch_sorted_points(const float* pts, int n, int start, void* ws, hipStream_t st, SortedPoints* out) {
    const GridLayout g = grid_layout(n, 1024);
    char* base = static_cast<char*>(ws);
    DevHeader* hdr = reinterpret_cast<DevHeader*>(base + g.dev_header);
    GridHeader* gh = reinterpret_cast<GridHeader*>(base + g.grid_header);
    uint32_t* codes = reinterpret_cast<uint32_t*>(base + g.codes);
    uint32_t* vals = reinterpret_cast<uint32_t*>(base + g.vals);
    uint32_t* codes_s = reinterpret_cast<uint32_t*>(base + g.codes_sorted);
    uint32_t* ids = reinterpret_cast<uint32_t*>(base + g.ids);
    float4* xyzm = reinterpret_cast<float4*>(base + g.xyzm);
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
    static_assert(3 * kMortonBits == 30, "the sort orders 30-bit codes");
    e = sort_codes_u32(codes, codes_s, vals, ids, n, temp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sorted_gather_kernel, dim3(nblk), dim3(tb), 0, st, pts, ids, n, start, gh, xyzm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    out->hdr = hdr;
    out->xyzm = xyzm;
    out->ids = ids;
    out->codes = codes_s;
    out->start_pos = &gh->start_pos;
    out->slots = base + g.lead_slots;
    return hipSuccess;
}

hipError_t launch_morton_order(const float* pts, int n, int32_t* out_perm, void* ws, hipStream_t st) {
    SortedPoints sp{};
    hipError_t e = launch_sorted_points(pts, n, 0, ws, st, &sp);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out_perm, sp.ids, size_t(n) * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
    return e;
}

int grid_block_size(int64_t n) { return n > (int64_t(1) << 16) ? 512 : 256; }

int grid_max_blocks(int block, int picks) {
    if (picks > 1 && block == 1024) return 2048;
    return block == 512 ? 4096 : 1024;
}

namespace {

// Pieces of one object's grid workspace.
struct GridPieces {
    DevHeader* hdr;
    GridHeader* gh;
    uint32_t *codes, *vals, *codes_s, *ids, *flags, *cellidx;
    int32_t* cstart;
    float4 *xyzm, *cstat, *bstat, *sbstat;
    uint4 *cdyn, *bdyn;
    void* temp;
    char* lead_slots;
};

GridPieces grid_pieces(int n, int block, void* ws) {
    const GridLayout g = grid_layout(n, block);
    char* base = static_cast<char*>(ws);
    GridPieces q;
    q.hdr = reinterpret_cast<DevHeader*>(base + g.dev_header);
    q.gh = reinterpret_cast<GridHeader*>(base + g.grid_header);
    q.codes = reinterpret_cast<uint32_t*>(base + g.codes);
    q.vals = reinterpret_cast<uint32_t*>(base + g.vals);
    q.codes_s = reinterpret_cast<uint32_t*>(base + g.codes_sorted);
    q.ids = reinterpret_cast<uint32_t*>(base + g.ids);
    q.flags = reinterpret_cast<uint32_t*>(base + g.flags);
    q.cellidx = reinterpret_cast<uint32_t*>(base + g.cellidx);
    q.cstart = reinterpret_cast<int32_t*>(base + g.cstart);
    q.xyzm = reinterpret_cast<float4*>(base + g.xyzm);
    q.cstat = reinterpret_cast<float4*>(base + g.cstat);
    q.cdyn = reinterpret_cast<uint4*>(base + g.cdyn);
    q.bstat = reinterpret_cast<float4*>(base + g.bstat);
    q.bdyn = reinterpret_cast<uint4*>(base + g.bdyn);
    q.sbstat = reinterpret_cast<float4*>(base + g.sbstat);
    q.temp = base + g.temp;
    q.lead_slots = base + g.lead_slots;
    return q;
}

// First half of the grid build: header, validation, Morton codes and their
// sort, the cell level, cell flags and cell indices.
hipError_t grid_build_sort(const float* pts, int n, const GridPieces& q, float target,
                           int max_blocks, hipStream_t st) {
    hipError_t e = launch_init_header(q.hdr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(init_grid_header_kernel, dim3(1), dim3(64), 0, st, q.gh);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_validate(pts, n, q.hdr, st)) != hipSuccess) return e;
    const int tb = 256;
    const int nblk = (n + tb - 1) / tb;
    hipLaunchKernelGGL(morton_kernel, dim3(nblk), dim3(tb), 0, st, pts, n, q.hdr, q.codes, q.vals);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = sort_codes_u32(q.codes, q.codes_s, q.vals, q.ids, n, q.temp, st);
    if (e != hipSuccess) return e;
    const int hblk = nblk < 1024 ? nblk : 1024;
    hipLaunchKernelGGL(level_hist_kernel, dim3(hblk), dim3(tb), 0, st, q.codes_s, n, q.gh);
    hipLaunchKernelGGL(choose_level_kernel, dim3(1), dim3(64), 0, st, n, q.gh, target, max_blocks);
    hipLaunchKernelGGL(cell_flag_kernel, dim3(nblk), dim3(tb), 0, st, q.codes_s, n, q.gh, q.flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return inclusive_scan_u32(q.flags, q.cellidx, n, q.temp, st);
}

// Second half: the sorted candidates (with m from a leading scan, or +inf),
// cell records, blocks and superblocks.
hipError_t grid_build_cells(const float* pts, int n, int start, const GridPieces& q, const float* m_lead,
                            hipStream_t st) {
    const int tb = 256;
    const int nblk = (n + tb - 1) / tb;
    hipLaunchKernelGGL(gather_kernel, dim3(nblk), dim3(tb), 0, st, pts, q.ids, q.flags, q.cellidx, n, start,
                       q.gh, q.xyzm, q.cstart, m_lead);
    hipLaunchKernelGGL(cell_build_kernel, dim3(nblk), dim3(tb), 0, st, q.cstart, n, q.gh, q.xyzm, q.ids, q.cstat,
                       q.cdyn);
    hipLaunchKernelGGL(block_build_kernel, dim3((kMaxBlocksAny + tb - 1) / tb), dim3(tb), 0, st, q.gh, q.cstat,
                       q.cdyn, q.bstat, q.bdyn);
    hipLaunchKernelGGL(superblock_build_kernel, dim3(1), dim3(64), 0, st, q.gh, q.bstat, q.sbstat);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_grid_sample(const float* pts, int n, int k, int start, uint64_t seed, int S, int K,
                              float vicinity, int32_t* order, float* radius, int32_t* count, void* ws,
                              float target, uint64_t* ticks, hipStream_t st, const LaunchOpts* ev) {
    constexpr int kBlock = 1024, kMaxB = 1024;
    const GridLayout g = grid_layout(n, kBlock);
    const GridPieces q = grid_pieces(n, kBlock, ws);
    hipError_t e = grid_build_sort(pts, n, q, target, kMaxB, st);
    if (e != hipSuccess) return e;
    if ((e = grid_build_cells(pts, n, start, q, nullptr, st)) != hipSuccess) return e;
    // the unsorted Morton values are dead after the sort: each candidate's sorted position
    int32_t* pos_of = reinterpret_cast<int32_t*>(q.vals);
    hipLaunchKernelGGL(position_kernel, dim3((n + 255) / 256), dim3(256), 0, st, q.ids, n, pos_of);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    GridObject o{};
    o.k = k;
    o.start_id = uint32_t(start);
    o.xyzm = q.xyzm;
    o.ids = q.ids;
    o.cstat = q.cstat;
    o.cdyn = q.cdyn;
    o.bstat = q.bstat;
    o.bdyn = q.bdyn;
    o.sbstat = q.sbstat;
    o.order = order;
    o.radius = radius;
    o.ticks = ticks;
    o.max_picks = 1;
    o.t0 = 0;
    o.start_m = INFINITY;
    SampleSpec sp{};
    sp.key0 = uint32_t(seed);
    sp.key1 = uint32_t(seed >> 32);
    sp.S = S;
    sp.K = K;
    sp.vicinity = vicinity;
    sp.n = n;
    sp.pos_of = pos_of;
    sp.cellidx = q.cellidx;
    sp.cell_base = 0;
    sp.count = count;
    if (ev && ev->begin && (e = hipEventRecord(ev->begin, st)) != hipSuccess) return e;
    hipLaunchKernelGGL((sample_single_kernel<kBlock, kMaxB>), dim3(1), dim3(kBlock), 0, st, o, sp, q.hdr, q.gh);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && ev->end) e = hipEventRecord(ev->end, st);
    return e;
}

hipError_t launch_grid(const float* pts, int n, int k, int start, int32_t* order, float* radius,
                       void* ws, float target, int block, int picks, uint64_t* ticks,
                       hipStream_t st, const LaunchOpts* ev, int lead, const ScanShape* lead_shape) {
    if (picks <= 1 || !lead_shape || lead < 2) lead = 0;
    if (lead > k) lead = k;
    const GridLayout g = grid_layout(n, block);
    const GridPieces q = grid_pieces(n, block, ws);
    DevHeader* hdr = q.hdr;
    GridHeader* gh = q.gh;
    float4* xyzm = q.xyzm;
    uint32_t* ids = q.ids;
    float4* cstat = q.cstat;
    uint4* cdyn = q.cdyn;
    float4* bstat = q.bstat;
    uint4* bdyn = q.bdyn;
    float4* sbstat = q.sbstat;

    hipError_t e = grid_build_sort(pts, n, q, target, grid_max_blocks(block, picks), st);
    if (e != hipSuccess) return e;
    float* m_lead = nullptr;
    if (lead >= 2) {
        // picks 0 .. lead-1 by the cooperative full scan; its m values land in
        // the (now unused) unsorted Morton codes, its last pick in the header
        m_lead = reinterpret_cast<float*>(q.codes);
        LaunchOpts lo;  // the events bracket the grid kernel; the wait limit applies here
        lo.spin_limit = ev ? ev->spin_limit : 0;
        e = launch_scan(*lead_shape, pts, n, k, start, order, radius, hdr, q.lead_slots, ticks, st, &lo, lead,
                        m_lead, &gh->lead_id);
        if (e != hipSuccess) return e;
    }
    if ((e = grid_build_cells(pts, n, start, q, m_lead, st)) != hipSuccess) return e;

    GridObject o{};
    o.k = k;
    o.start_id = uint32_t(start);
    o.xyzm = xyzm;
    o.ids = ids;
    o.cstat = cstat;
    o.cdyn = cdyn;
    o.bstat = bstat;
    o.bdyn = bdyn;
    o.sbstat = sbstat;
    o.order = order;
    o.radius = radius;
    o.ticks = ticks;
    o.max_picks = picks < kMaxPicks ? picks : kMaxPicks;
    o.t0 = lead >= 2 ? lead - 1 : 0;
    o.start_m = INFINITY;
    if (ev && ev->begin && (e = hipEventRecord(ev->begin, st)) != hipSuccess) return e;
    if (picks > 1) {
        if (block == 512)
            hipLaunchKernelGGL((grid_multi_kernel<512, 4096>), dim3(1), dim3(512), 0, st, o, hdr, gh);
        else if (block == 1024)
            hipLaunchKernelGGL((grid_multi_kernel<1024, 2048>), dim3(1), dim3(1024), 0, st, o, hdr, gh);
        else
            hipLaunchKernelGGL((grid_multi_kernel<256, 1024>), dim3(1), dim3(256), 0, st, o, hdr, gh);
    } else if (block == 512)
        hipLaunchKernelGGL((grid_single_kernel<512, 4096>), dim3(1), dim3(512), 0, st, o, hdr, gh);
    else if (block == 1024)
        hipLaunchKernelGGL((grid_single_kernel<1024, 1024>), dim3(1), dim3(1024), 0, st, o, hdr, gh);
    else
        hipLaunchKernelGGL((grid_single_kernel<256, 1024>), dim3(1), dim3(256), 0, st, o, hdr, gh);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && ev->end && (e = hipEventRecord(ev->end, st)) != hipSuccess) return e;
    if (lead >= 2) e = launch_finish(hdr, order, radius, k, st);
    return e;
}

}  // namespace bs
