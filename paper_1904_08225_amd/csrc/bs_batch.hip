// bs_batch.hip -- batched ordering: thousands of objects in one persistent
// work-queue launch captured in a hipGraph.
//
// The paper generates one approximation per scene-graph node and notes that
// the sampling is easily parallelised over the objects of a scene (Sec. 3.4
// hierarchical generation, Sec. 5 preprocessing).  Here every object is an
// independent greedy permutation (same result, bit for bit, as ordering it
// alone): the grid of every object is built by segmented preprocessing
// kernels over all candidates at once (sort key = object id : Morton code),
// then a persistent kernel whose workgroups pop objects from a device queue,
// largest k first, runs the grid-pruned ordering loop of each object.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "bs_grid.h"
#include "bs_grid_device.h"
#include "bs_grid_multi.h"
#include "bs_internal.h"
#include "bs_sample_device.h"

namespace bs {

namespace {

constexpr int kBatchBlock = 256;         // threads per ordering workgroup
constexpr int kWideBlock = 1024;         // threads per workgroup for the largest objects
constexpr int64_t kWideMinK = 65536;     // automatic choice: smallest k given a wide workgroup
constexpr int kBatchMaxBlocks = 1024;    // blocks of 64 cells per object
// A batch whose 1024-thread workgroups get an object of more than
// 64 x 64 x kBatchMaxBlocks candidates (cells above 64 candidates) gives
// them twice as many blocks, and so smaller cells (LDS: 116 KB a workgroup;
// a pick's update reads whole cells): the hierarchy's cluster nodes of about
// 9 M candidates, cells of about 70 instead of 140, 4.3 s -> 3.5 s for the
// whole hierarchy.  Otherwise the 1024-block kernel is kept: the 1,000-part
// batch ran 0.81 s with it against 0.86 s with 2048 blocks (cells of 16
// instead of 32 for its largest parts, but two block boxes a thread).
constexpr int kWideMaxBlocks = 2048;
// Most exact picks per round of an object, unless the plan sets it: 24 for
// cells of up to 64 candidates on average (the 1,000-part batch, whose
// largest objects have cells of about 32: 0.86, 0.83, 0.81, 0.82 and 0.85 s
// at 16, 20, 24, 28 and 32), 16 for larger cells (a pick's update of a large
// cell costs more than a round's fixed cost; the hierarchy with its cluster
// nodes' cells of about 140: 4.3 s at 16 against 4.7 s at 24).
constexpr int kBatchPicks = 24;
constexpr int kBatchPicksLargeCells = 16;
constexpr int kLargeCell = 64;
constexpr int kObjBits = 30;             // Morton bits below the object id

// Per-object device state of the batched preprocessing (256 bytes).
struct ObjHdr {
    uint32_t bbox[6];  // order-preserving encodings: min x,y,z, max x,y,z
    uint32_t nonfinite;
    uint32_t hist[31];  // adjacent sorted pairs first separated by each code prefix length
    int32_t level;      // cells: runs of codes sharing their top `level` bits
    int32_t cell_base, C, NB, block_base, nsb, sb_base, start_pos, start_cell;
    int32_t max_blocks;  // blocks of 64 cells at most (by the workgroup that orders the object)
    int32_t split;       // cells split into runs of at most `split` candidates (0: not split)
    int32_t pad[15];
};
static_assert(sizeof(ObjHdr) == 256, "object header size");

__device__ __forceinline__ uint32_t ord_encode_f(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// object of global candidate i: largest j with offs[j] <= i
__device__ __forceinline__ int find_obj(const int32_t* __restrict__ offs, int m, int i) {
    int lo = 0, hi = m - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void bobj_init_kernel(int m, ObjHdr* __restrict__ hd, int max_blocks) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    ObjHdr h{};
    for (int a = 0; a < 3; ++a) {
        h.bbox[a] = 0xFFFFFFFFu;
        h.bbox[3 + a] = 0u;
    }
    h.start_pos = -1;
    h.max_blocks = max_blocks;
    hd[j] = h;
}

// The objects of the 1024-thread workgroups (the head of the LPT order) may
// have more blocks (after bobj_init_kernel, on the same stream).
__global__ void bwide_kernel(int nwide, const int32_t* __restrict__ lpt, ObjHdr* __restrict__ hd,
                             int max_blocks) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nwide) hd[lpt[r]].max_blocks = max_blocks;
}

template <bool UMAX>
__device__ __forceinline__ uint32_t wave_minmax_u32(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = uint32_t(__shfl_xor(int(v), off, 64));
        v = UMAX ? (o > v ? o : v) : (o < v ? o : v);
    }
    return v;
}

// finiteness flag and box of every object
__global__ void bvalidate_kernel(const float* __restrict__ pts, int N, const int32_t* __restrict__ offs,
                                 int m, ObjHdr* __restrict__ hd) {
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < N; base += stride) {
        const int i = base + threadIdx.x;
        const bool in = i < N;
        const int obj = in ? find_obj(offs, m, i) : -1;
        uint32_t lo[3], hi[3];
        bool bad = false;
        for (int a = 0; a < 3; ++a) {
            const float v = in ? pts[3 * size_t(i) + a] : 0.f;
            bad |= in && !isfinite(v);
            const uint32_t e = ord_encode_f(v);
            lo[a] = in ? e : 0xFFFFFFFFu;
            hi[a] = in ? e : 0u;
        }
        const int o0 = __builtin_amdgcn_readfirstlane(obj);
        const bool uniform = __ballot(in && obj != o0) == 0 && o0 >= 0;
        if (uniform) {
            for (int a = 0; a < 3; ++a) {
                lo[a] = wave_minmax_u32<false>(lo[a]);
                hi[a] = wave_minmax_u32<true>(hi[a]);
            }
            const bool anybad = __ballot(bad) != 0;
            if ((threadIdx.x & 63) == 0) {
                for (int a = 0; a < 3; ++a) {
                    atomicMin(&hd[o0].bbox[a], lo[a]);
                    atomicMax(&hd[o0].bbox[3 + a], hi[a]);
                }
                if (anybad) atomicOr(&hd[o0].nonfinite, 1u);
            }
        } else if (in) {
            for (int a = 0; a < 3; ++a) {
                atomicMin(&hd[obj].bbox[a], lo[a]);
                atomicMax(&hd[obj].bbox[3 + a], hi[a]);
            }
            if (bad) atomicOr(&hd[obj].nonfinite, 1u);
        }
    }
}

__global__ void bmorton_kernel(const float* __restrict__ pts, int N, const int32_t* __restrict__ offs,
                               int m, const ObjHdr* __restrict__ hd, uint64_t* __restrict__ keys,
                               uint32_t* __restrict__ vals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int obj = find_obj(offs, m, i);
    const ObjHdr& h = hd[obj];
    float lo[3], ext = 0.f;
    for (int a = 0; a < 3; ++a) {
        lo[a] = ord_decode(h.bbox[a]);
        ext = fmaxf(ext, ord_decode(h.bbox[3 + a]) - lo[a]);
    }
    const float scale = (ext > 0.f && isfinite(ext)) ? float(1 << kMortonBits) / ext : 0.f;
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        const float f = (pts[3 * size_t(i) + a] - lo[a]) * scale;
        int v = isfinite(f) ? int(f) : 0;
        v = v < 0 ? 0 : (v > (1 << kMortonBits) - 1 ? (1 << kMortonBits) - 1 : v);
        q[a] = uint32_t(v);
    }
    const uint32_t code = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
    keys[i] = (uint64_t(obj) << kObjBits) | code;
    vals[i] = uint32_t(i);
}

// per object: adjacent sorted pairs first separated by each code prefix
// length (cells are chosen one Morton bit at a time, as for one object)
__global__ void bhist_kernel(const uint64_t* __restrict__ keys, int N, ObjHdr* __restrict__ hd) {
    constexpr int kBits = 3 * kMortonBits;
    __shared__ uint32_t h[kBits + 1];
    const int first = blockIdx.x * blockDim.x;
    if (first >= N) return;
    const int obj0 = int(keys[first] >> kObjBits);
    if (threadIdx.x <= kBits) h[threadIdx.x] = 0;
    __syncthreads();
    const int i = first + threadIdx.x;
    if (i >= 1 && i < N) {
        const uint64_t a = keys[i], b = keys[i - 1];
        if ((a >> kObjBits) == (b >> kObjBits)) {
            const uint32_t d = uint32_t(a ^ b) & ((1u << kObjBits) - 1u);
            if (d) {
                const int l = kBits - (31 - __clz(d));
                const int obj = int(a >> kObjBits);
                if (obj == obj0) atomicAdd(&h[l], 1u);
                else atomicAdd(&hd[obj].hist[l], 1u);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x <= kBits && h[threadIdx.x]) atomicAdd(&hd[obj0].hist[threadIdx.x], h[threadIdx.x]);
}

// Cells at most of object j (the workspace is sized for it).
__device__ __forceinline__ double cell_cap(int n, float target, int max_blocks) {
    return fmin(fmax(1.0, double(n) / double(target)), double(64 * max_blocks));
}

// halve: leave room for splitting cells (the level takes at most half the cells)
__global__ void blevel_kernel(int m, const int32_t* __restrict__ offs, ObjHdr* __restrict__ hd,
                              float target, int halve) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int n = offs[j + 1] - offs[j];
    const double full = cell_cap(n, target, hd[j].max_blocks);
    const double cap = halve ? fmax(1.0, floor(full / 2.0)) : full;
    int level = 0;
    uint32_t acc = 1;
    for (int l = 1; l <= 3 * kMortonBits; ++l) {
        acc += hd[j].hist[l];
        if (double(acc) <= cap) level = l;
    }
    hd[j].level = level;
}

__global__ void bflag_kernel(const uint64_t* __restrict__ keys, int N, const ObjHdr* __restrict__ hd,
                             uint32_t* __restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint64_t a = keys[i];
    if (i == 0) {
        flags[i] = 1u;
        return;
    }
    const uint64_t b = keys[i - 1];
    const int obj = int(a >> kObjBits);
    const int s = 3 * kMortonBits - hd[obj].level;
    const uint32_t ca = uint32_t(a) & ((1u << kObjBits) - 1u), cb = uint32_t(b) & ((1u << kObjBits) - 1u);
    flags[i] = ((a >> kObjBits) != (b >> kObjBits) || (ca >> s) != (cb >> s)) ? 1u : 0u;
}

// Splitting uneven cells (candidate sets made of compact groups, such as a
// hierarchy node's children's surfels, give Morton-prefix cells far above
// the mean where the groups lie): every run of a cell's candidates is cut
// into pieces of at most S, with S per object the smallest that keeps the
// cells within the object's limit.  Cells stay runs of consecutive sorted
// candidates; their boxes come from their members.
__global__ void bcstart_kernel(const uint32_t* __restrict__ flags, const uint32_t* __restrict__ cellidx, int N,
                               int32_t* __restrict__ cstart) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N && flags[i]) cstart[cellidx[i] - 1] = i;
}

__global__ void bsplit_prep_kernel(int m, const int32_t* __restrict__ offs, const uint32_t* __restrict__ cellidx,
                                   ObjHdr* __restrict__ hd, float target) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int a = offs[j], b = offs[j + 1], n = b - a;
    hd[j].split = 0;
    if (n <= 0) return;
    const int cells = int(cellidx[b - 1]) - (a > 0 ? int(cellidx[a - 1]) : 0);
    const int cap = int(cell_cap(n, target, hd[j].max_blocks));
    // pieces beyond the first of each cell number at most n / S <= cap - cells
    if (cap > cells) {
        const int64_t room = int64_t(cap) - cells;
        hd[j].split = int(max(int64_t(1), (int64_t(n) + room - 1) / room));
    }
}

__global__ void bsplit_kernel(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ cellidx, int N,
                              const int32_t* __restrict__ cstart, const ObjHdr* __restrict__ hd,
                              uint32_t* __restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int S = hd[int(keys[i] >> kObjBits)].split;
    if (S > 0 && (i - cstart[cellidx[i] - 1]) % S == 0) flags[i] = 1u;
}

__global__ void bgather_kernel(const float* __restrict__ pts, const uint64_t* __restrict__ keys,
                               const uint32_t* __restrict__ vals, const uint32_t* __restrict__ flags,
                               const uint32_t* __restrict__ cellidx, int N,
                               const int32_t* __restrict__ offs, const int32_t* __restrict__ starts,
                               ObjHdr* __restrict__ hd, float4* __restrict__ xyzm,
                               uint32_t* __restrict__ ids, int32_t* __restrict__ cstart) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint32_t g = vals[i];
    const int obj = int(keys[i] >> kObjBits);
    const uint32_t local = g - uint32_t(offs[obj]);
    xyzm[i] = make_float4(pts[3 * size_t(g) + 0], pts[3 * size_t(g) + 1], pts[3 * size_t(g) + 2], INFINITY);
    ids[i] = local;
    const int cell = int(cellidx[i]) - 1;
    if (flags[i]) cstart[cell] = i;
    if (i == 0 || (keys[i - 1] >> kObjBits) != uint64_t(obj)) hd[obj].cell_base = cell;
    if (int(local) == starts[obj]) {
        hd[obj].start_pos = i;
        hd[obj].start_cell = cell;
    }
}

// one workgroup: per-object cell / block / superblock counts and bases
__global__ void bobj_fin_kernel(int m, const uint32_t* __restrict__ cellidx, int N,
                                ObjHdr* __restrict__ hd, int32_t* __restrict__ totals) {
    __shared__ int32_t s_carry[2];
    __shared__ int32_t s_w[2][16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int total_cells = int(cellidx[N - 1]);
    if (tid == 0) {
        s_carry[0] = 0;
        s_carry[1] = 0;
    }
    __syncthreads();
    for (int base = 0; base < m; base += blockDim.x) {
        const int j = base + tid;
        int nb = 0, ns = 0;
        if (j < m) {
            const int cb = hd[j].cell_base;
            const int ce = (j + 1 < m) ? hd[j + 1].cell_base : total_cells;
            const int C = ce - cb;
            nb = (C + 63) / 64;
            ns = (nb + 63) / 64;
            hd[j].C = C;
            hd[j].NB = nb;
            hd[j].nsb = ns;
            hd[j].start_cell -= cb;
        }
        // block-wide exclusive scans of nb and ns
        int xb = nb, xs = ns;
        for (int off = 1; off < 64; off <<= 1) {
            const int yb = __shfl_up(xb, off, 64), ys = __shfl_up(xs, off, 64);
            if (lane >= off) {
                xb += yb;
                xs += ys;
            }
        }
        if (lane == 63) {
            s_w[0][wave] = xb;
            s_w[1][wave] = xs;
        }
        __syncthreads();
        int ob = s_carry[0], os = s_carry[1];
        const int nw = blockDim.x / 64;
        int tb = 0, ts = 0;
        for (int w = 0; w < nw; ++w) {
            if (w < wave) {
                ob += s_w[0][w];
                os += s_w[1][w];
            }
            tb += s_w[0][w];
            ts += s_w[1][w];
        }
        if (j < m) {
            hd[j].block_base = ob + xb - nb;
            hd[j].sb_base = os + xs - ns;
        }
        __syncthreads();
        if (tid == 0) {
            s_carry[0] += tb;
            s_carry[1] += ts;
        }
        __syncthreads();
    }
    if (tid == 0) {
        totals[0] = total_cells;
        totals[1] = s_carry[0];
        totals[2] = s_carry[1];
    }
}

__global__ void bcells_kernel(const int32_t* __restrict__ cstart, int N, const int32_t* __restrict__ totals,
                              const float4* __restrict__ xyzm, const uint32_t* __restrict__ ids,
                              float4* __restrict__ cstat, uint4* __restrict__ cdyn) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int C = totals[0];
    if (c >= C) return;
    const int s = cstart[c];
    const int e = (c + 1 < C) ? cstart[c + 1] : N;
    float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
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
    cstat[2 * size_t(c) + 0] = make_float4(lx, ly, lz, __int_as_float(s));
    cstat[2 * size_t(c) + 1] = make_float4(hx, hy, hz, __int_as_float(e - s));
    const uint64_t key = make_key(INFINITY, best_id);
    const float4 w = xyzm[best_pos];
    // second key slot: the best key bounds the other keys until the first update
    cdyn[2 * size_t(c) + 0] = make_uint4(uint32_t(key), uint32_t(key >> 32), uint32_t(best_pos), uint32_t(key));
    cdyn[2 * size_t(c) + 1] = make_uint4(__float_as_uint(w.x), __float_as_uint(w.y), __float_as_uint(w.z),
                                         uint32_t(key >> 32));
}

// object owning global block / superblock b: largest j with base(j) <= b
template <int FIELD>
__device__ __forceinline__ int find_obj_by_base(const ObjHdr* __restrict__ hd, int m, int b) {
    int lo = 0, hi = m - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int base = FIELD == 0 ? hd[mid].block_base : hd[mid].sb_base;
        if (base <= b) lo = mid;
        else hi = mid - 1;
    }
    // skip objects with no blocks that share the same base
    while (lo + 1 < m && (FIELD == 0 ? hd[lo + 1].block_base : hd[lo + 1].sb_base) <= b) ++lo;
    return lo;
}

__global__ void bblocks_kernel(int m, const ObjHdr* __restrict__ hd, const int32_t* __restrict__ totals,
                               const float4* __restrict__ cstat, const uint4* __restrict__ cdyn,
                               float4* __restrict__ bstat, uint4* __restrict__ bdyn) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= totals[1]) return;
    const int j = find_obj_by_base<0>(hd, m, b);
    const int lb = b - hd[j].block_base;
    const int cb = hd[j].cell_base, C = hd[j].C;
    float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
    uint64_t best = 0;
    uint32_t other = 0;  // value bits of the best key of the cells other than the best one
    int bc = lb * 64;
    for (int c = lb * 64; c < C && c < (lb + 1) * 64; ++c) {
        const size_t g = size_t(cb) + c;
        const float4 lo = cstat[2 * g], hi = cstat[2 * g + 1];
        lx = fminf(lx, lo.x);
        ly = fminf(ly, lo.y);
        lz = fminf(lz, lo.z);
        hx = fmaxf(hx, hi.x);
        hy = fmaxf(hy, hi.y);
        hz = fmaxf(hz, hi.z);
        const uint4 d = cdyn[2 * g];
        const uint64_t key = (uint64_t(d.y) << 32) | d.x;
        if (key > best) {
            if (best) other = max(other, uint32_t(best >> 32));
            best = key;
            bc = c;
        } else {
            other = max(other, d.y);
        }
    }
    bstat[2 * size_t(b) + 0] = make_float4(lx, ly, lz, 0.f);
    bstat[2 * size_t(b) + 1] = make_float4(hx, hy, hz, 0.f);
    const size_t g = size_t(cb) + bc;
    const uint4 d0 = cdyn[2 * g], d1 = cdyn[2 * g + 1];
    // last word: value bits of a bound on the block's other keys
    bdyn[2 * size_t(b) + 0] = make_uint4(d0.x, d0.y, d0.z, uint32_t(bc));
    bdyn[2 * size_t(b) + 1] = make_uint4(d1.x, d1.y, d1.z, max(other, d1.w));
}

__global__ void bsuper_kernel(int m, const ObjHdr* __restrict__ hd, const int32_t* __restrict__ totals,
                              const float4* __restrict__ bstat, float4* __restrict__ sbstat) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= totals[2]) return;
    const int j = find_obj_by_base<1>(hd, m, s);
    const int ls = s - hd[j].sb_base;
    const int bb = hd[j].block_base, NB = hd[j].NB;
    float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
    for (int b = ls * 64; b < NB && b < (ls + 1) * 64; ++b) {
        const float4 lo = bstat[2 * (size_t(bb) + b)], hi = bstat[2 * (size_t(bb) + b) + 1];
        lx = fminf(lx, lo.x);
        ly = fminf(ly, lo.y);
        lz = fminf(lz, lo.z);
        hx = fmaxf(hx, hi.x);
        hy = fmaxf(hy, hi.y);
        hz = fmaxf(hz, hi.z);
    }
    sbstat[2 * size_t(s) + 0] = make_float4(lx, ly, lz, 0.f);
    sbstat[2 * size_t(s) + 1] = make_float4(hx, hy, hz, 0.f);
}

struct ObjDesc {
    GridObject o;
    uint32_t* done;    // optional completion flag (host-visible memory), set to 1 at the end
    int nonfinite;
    int pad;
};

// Optional per-object outputs (served jobs write straight into their own buffers).
struct JobIo {
    int32_t* order;
    float* radius;
    uint32_t* done;
    void* pad;
};

__global__ void bdesc_kernel(int m, const ObjHdr* __restrict__ hd, const int32_t* __restrict__ ks,
                             const int32_t* __restrict__ starts, const int64_t* __restrict__ out_offs,
                             float4* xyzm, const uint32_t* ids, const float4* cstat, uint4* cdyn,
                             const float4* bstat, const uint4* bdyn, const float4* sbstat,
                             int32_t* out_order, float* out_radius, const JobIo* __restrict__ io,
                             const int32_t* __restrict__ offs, int max_picks, ObjDesc* __restrict__ desc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const ObjHdr& h = hd[j];
    ObjDesc d{};
    GridObject& o = d.o;
    o.k = ks[j];
    o.start_id = uint32_t(starts[j]);
    o.C = h.C;
    o.B = 64;
    o.NB = h.NB;
    o.start_pos = h.start_pos;
    o.start_cell = h.start_cell;
    o.xyzm = xyzm;
    o.ids = ids;
    o.cstat = cstat + 2 * size_t(h.cell_base);
    o.cdyn = cdyn + 2 * size_t(h.cell_base);
    o.bstat = bstat + 2 * size_t(h.block_base);
    o.bdyn = bdyn + 2 * size_t(h.block_base);
    o.sbstat = sbstat + 2 * size_t(h.sb_base);
    if (io) {
        o.order = io[j].order;
        o.radius = io[j].radius;
        d.done = io[j].done;
    } else {
        o.order = out_order + out_offs[j];
        o.radius = out_radius ? out_radius + out_offs[j] : nullptr;
        d.done = nullptr;
    }
    o.ticks = nullptr;
    const int64_t n = int64_t(offs[j + 1]) - offs[j];
    o.max_picks = max_picks > 0 ? max_picks : n > int64_t(kLargeCell) * h.C ? kBatchPicksLargeCells : kBatchPicks;
    o.t0 = 0;
    o.start_m = INFINITY;
    d.nonfinite = int(h.nonfinite);
    desc[j] = d;
}

// Sorted position -> index within its object (the Morton order of each object).
__global__ void blocal_kernel(const uint64_t* __restrict__ keys_s, const uint32_t* __restrict__ vals_s, int N,
                              const int32_t* __restrict__ offs, int32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    out[i] = int32_t(vals_s[i]) - offs[int(keys_s[i] >> kObjBits)];
}

__global__ void queue_reset_kernel(uint32_t* q) {
    if (threadIdx.x < 2) q[threadIdx.x] = 0u;
}

// Randomized sampler (Sec. 3.2) over the same grids: each object's sorted
// position of every original index, and its sampler parameters.
__global__ void bpos_kernel(const uint64_t* __restrict__ keys_s, const uint32_t* __restrict__ ids, int N,
                            const int32_t* __restrict__ offs, int32_t* __restrict__ pos_of) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int obj = int(keys_s[i] >> kObjBits);
    pos_of[offs[obj] + int(ids[i])] = i;
}

struct SampleParams {
    int S, K;
    float vicinity;
    int pad;
};

__global__ void bsdesc_kernel(int m, const ObjHdr* __restrict__ hd, const int32_t* __restrict__ offs,
                              const uint64_t* __restrict__ seeds, const int32_t* __restrict__ kept,
                              const int32_t* __restrict__ pos_of, const uint32_t* __restrict__ cellidx,
                              SampleParams prm, int32_t* out_count, SampleSpec* __restrict__ sdesc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    SampleSpec s{};
    s.key0 = uint32_t(seeds[j]);
    s.key1 = uint32_t(seeds[j] >> 32);
    s.S = prm.S;
    s.K = prm.K;
    s.vicinity = prm.vicinity;
    s.n = offs[j + 1] - offs[j];
    s.pos_of = pos_of + offs[j];
    s.cellidx = cellidx;
    s.cell_base = hd[j].cell_base;
    s.count = out_count ? out_count + kept[j] : nullptr;
    sdesc[j] = s;
}

__global__ void fill_i32_kernel(int32_t* p, int n, int32_t v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// Persistent work queue of sampler runs (largest k first), one object per
// 256-thread workgroup; the batch's largest objects may get 1024-thread
// workgroups (a second launch with its own queue), as in the exact ordering.
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK)
    sample_batch_kernel(const ObjDesc* __restrict__ desc, const SampleSpec* __restrict__ sdesc,
                        const int32_t* __restrict__ lpt, int mwork, uint32_t* __restrict__ queue) {
    __shared__ GridLds<BLOCK / 64, kBatchMaxBlocks> L;
    __shared__ SampleLds<BLOCK / 64> SL;
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = int(atomicAdd(queue, 1u));
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= mwork) return;
        const int j = lpt[item];
        const GridObject o = desc[j].o;
        const SampleSpec sp = sdesc[j];
        if (o.k > 0) {
            if (desc[j].nonfinite) {
                for (int t = threadIdx.x; t < o.k; t += BLOCK) {
                    o.order[t] = -1;
                    if (o.radius) o.radius[t] = __builtin_nanf("");
                }
                if (threadIdx.x == 0 && sp.count) *sp.count = 0;
            } else {
                sample_object<BLOCK, kBatchMaxBlocks>(o, sp, L, SL);
            }
        }
        __syncthreads();
    }
}

// Persistent work queue: each workgroup pops objects (largest k first) until
// the queue is drained; every pop ends the loop for all its waves alike.
// BLOCK = 256 for most objects; the largest ones may get 1024-thread
// workgroups (a second launch of the same loop with its own queue).
template <int BLOCK, int MAXB>
__global__ void __launch_bounds__(BLOCK)
    batch_order_kernel(const ObjDesc* __restrict__ desc, const int32_t* __restrict__ lpt, int mwork,
                       uint32_t* __restrict__ queue) {
    __shared__ GridLdsMP<BLOCK / 64, MAXB> L;
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = int(atomicAdd(queue, 1u));
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= mwork) return;
        const int j = lpt[item];
        const GridObject o = desc[j].o;
        uint32_t* done = desc[j].done;
        if (o.k > 0) {
            if (desc[j].nonfinite) {
                for (int t = threadIdx.x; t < o.k; t += BLOCK) {
                    o.order[t] = -1;
                    if (o.radius) o.radius[t] = __builtin_nanf("");
                }
            } else {
                grid_order_object_mp<BLOCK, MAXB>(o, L);
            }
        }
        __syncthreads();
        if (done && threadIdx.x == 0) {
            // outputs of this object happen-before the flag, at system scope
            __atomic_thread_fence(__ATOMIC_RELEASE);
            __hip_atomic_store(done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// Appends count descriptors, largest k first, at ring positions base, ...
// and then publishes them by advancing tail (release at device scope: the
// descriptors and everything the preprocessing wrote before them become
// visible to a worker that observes the new tail).
__global__ void publish_kernel(const ObjDesc* __restrict__ desc, const int32_t* __restrict__ lpt, int count,
                               ObjDesc* __restrict__ slots, uint32_t cap, uint32_t base, uint32_t* tail) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) slots[(base + uint32_t(i)) % cap] = desc[lpt[i]];
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(tail, base + uint32_t(count), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Persistent serving workers: each workgroup claims the next published
// descriptor (compare-and-swap on head below tail), copies it into LDS with
// device-coherent loads (ring slots are rewritten while the kernel runs),
// orders that object and sets its completion flag.  A workgroup exits when
// stop is set and nothing is left to claim, or after idle_polls empty polls.
// Workers have 1024 threads: a worker then holds a whole CU (its waves take
// most of each SIMD's registers), so the workers take at most seven eighths
// of the CUs and leave the others to the preprocessing of later micro-batches.
__global__ void __launch_bounds__(kWideBlock)
    serve_kernel(const ObjDesc* __restrict__ slots, uint32_t cap, uint32_t* head, const uint32_t* tail,
                 const uint32_t* stop, uint32_t idle_polls) {
    __shared__ GridLdsMP<kWideBlock / 64, kBatchMaxBlocks> L;
    __shared__ int s_item;
    __shared__ __align__(16) uint32_t s_desc[(sizeof(ObjDesc) + 3) / 4];
    static_assert(sizeof(ObjDesc) % 4 == 0, "descriptor words");
    constexpr int kWords = int(sizeof(ObjDesc) / 4);
    static_assert(kWords <= kWideBlock, "one word per thread");
    for (;;) {
        if (threadIdx.x == 0) {
            int item = -1;
            uint32_t idle = 0;
            for (;;) {
                const uint32_t t = __hip_atomic_load(tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                uint32_t h = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (h < t) {
                    if (__hip_atomic_compare_exchange_strong(head, &h, h + 1, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) {
                        item = int(h % cap);
                        break;
                    }
                    continue;
                }
                if (__hip_atomic_load(stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) != 0u) break;
                if (++idle > idle_polls) break;
                __builtin_amdgcn_s_sleep(127);
            }
            s_item = item;
        }
        __syncthreads();
        const int item = s_item;
        if (item < 0) return;
        if (int(threadIdx.x) < kWords)
            s_desc[threadIdx.x] = __hip_atomic_load(reinterpret_cast<const uint32_t*>(slots + item) + threadIdx.x,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const ObjDesc d = *reinterpret_cast<const ObjDesc*>(s_desc);
        const GridObject& o = d.o;
        if (o.k > 0) {
            if (d.nonfinite) {
                for (int t = threadIdx.x; t < o.k; t += kWideBlock) {
                    o.order[t] = -1;
                    if (o.radius) o.radius[t] = __builtin_nanf("");
                }
            } else {
                grid_order_object_mp<kWideBlock, kBatchMaxBlocks>(o, L);
            }
        }
        __syncthreads();
        if (d.done && threadIdx.x == 0) {
            __atomic_thread_fence(__ATOMIC_RELEASE);
            __hip_atomic_store(d.done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

template <class T>
T* carve(char* base, size_t& off, size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off += align_up(count * sizeof(T));
    return p;
}

}  // namespace

struct BatchPlan {
    int m = 0;                      // objects with n >= 1
    int m_all = 0;                  // objects as given
    int N = 0;                      // total candidates
    int64_t total_k = 0;
    float target = 32.f;
    std::vector<int32_t> h_offs;    // m + 1
    std::vector<int32_t> h_k, h_start, h_lpt;
    std::vector<SortTile> h_tiles;  // tiles of the per-object Morton sort
    std::vector<uint64_t> h_seed;     // kept objects' seeds (the sampler's Philox keys)
    std::vector<int32_t> h_kept;      // caller object number of each kept object (device upload)
    std::vector<int64_t> h_out_offs;  // m_all + 1 (caller's object numbering)
    std::vector<int64_t> h_outo;      // m + 1 (kept objects)
    std::vector<JobIo> h_io;          // optional per-object outputs (kept objects)
    std::vector<int> kept;            // caller object number of each kept object
    int mwork = 0;                  // objects with k > 0
    size_t maxC = 0, maxB = 0, maxS = 0;
    size_t sort_bytes = 0, scan_bytes = 0;
    size_t ws_bytes = 0;
    int slots = 0;                  // persistent workgroups
    int nwide = 0;                  // the first nwide objects of h_lpt go to 1024-thread workgroups
    int wide_slots = 0;             // their persistent workgroups
    int picks = 0;                  // most exact picks per round of an object (0: by cell size)
    int wide_blocks = kBatchMaxBlocks;  // blocks at most of the 1024-thread workgroups' objects
    bool split_cells = false;       // cut uneven cells into runs (see bsplit_kernel)
    hipStream_t side = nullptr;     // stream of the wide launch (forked from the caller's)
    hipEvent_t fork = nullptr, join = nullptr;
    bool use_graph = true;
    // Device copies of the plan's arrays (batch and hierarchy plans, made by
    // batch_plan_upload; serving plans upload theirs into the workspace).
    void* dev = nullptr;
    int32_t *d_offs = nullptr, *d_ks = nullptr, *d_starts = nullptr, *d_lpt = nullptr, *d_kept = nullptr;
    int64_t* d_outo = nullptr;
    uint64_t* d_seeds = nullptr;
    SortTile* d_tiles = nullptr;
    // The captured execute (preprocessing, queue reset, both ordering
    // kernels), valid for the pointers it was captured with.
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    const void* graph_key[4] = {nullptr, nullptr, nullptr, nullptr};  // workspace, points, order, radius
    std::mutex mu;
};

namespace {

struct BatchWs {
    ObjHdr* hd;
    uint64_t* keys;
    uint64_t* keys_s;
    uint32_t* vals;
    uint32_t* vals_s;
    uint32_t* flags;
    uint32_t* cellidx;
    int32_t* cstart;
    float4* xyzm;
    uint32_t* ids;
    float4* cstat;
    uint4* cdyn;
    float4* bstat;
    uint4* bdyn;
    float4* sbstat;
    ObjDesc* desc;
    int32_t* totals;
    uint32_t* queue;
    int32_t* offs;
    int32_t* ks;
    int32_t* starts;
    int32_t* lpt;
    int64_t* outo;
    JobIo* io;
    int32_t* pos_of;
    SampleSpec* sdesc;
    uint64_t* seeds;
    int32_t* kept;
    SortTile* tiles;
    void* temp;
    size_t total;
};

BatchWs batch_layout(const BatchPlan& p, char* base) {
    BatchWs w{};
    size_t off = 0;
    const size_t N = size_t(p.N), m = size_t(p.m);
    w.hd = carve<ObjHdr>(base, off, m);
    w.keys = carve<uint64_t>(base, off, N);
    w.keys_s = carve<uint64_t>(base, off, N);
    w.vals = carve<uint32_t>(base, off, N);
    w.vals_s = carve<uint32_t>(base, off, N);
    w.flags = carve<uint32_t>(base, off, N);
    w.cellidx = carve<uint32_t>(base, off, N);
    w.cstart = carve<int32_t>(base, off, p.maxC);
    w.xyzm = carve<float4>(base, off, N);
    w.ids = carve<uint32_t>(base, off, N);
    w.cstat = carve<float4>(base, off, 2 * p.maxC);
    w.cdyn = carve<uint4>(base, off, 2 * p.maxC);
    w.bstat = carve<float4>(base, off, 2 * p.maxB);
    w.bdyn = carve<uint4>(base, off, 2 * p.maxB);
    w.sbstat = carve<float4>(base, off, 2 * p.maxS);
    w.desc = carve<ObjDesc>(base, off, m);
    w.totals = carve<int32_t>(base, off, 4);
    w.queue = carve<uint32_t>(base, off, 4);
    w.offs = carve<int32_t>(base, off, m + 1);
    w.ks = carve<int32_t>(base, off, m + 1);
    w.starts = carve<int32_t>(base, off, m + 1);
    w.lpt = carve<int32_t>(base, off, m + 1);
    w.outo = carve<int64_t>(base, off, m + 1);
    w.io = carve<JobIo>(base, off, m + 1);
    w.pos_of = carve<int32_t>(base, off, std::max<size_t>(N, 1));
    w.sdesc = carve<SampleSpec>(base, off, m + 1);
    w.seeds = carve<uint64_t>(base, off, m + 1);
    w.kept = carve<int32_t>(base, off, m + 1);
    w.tiles = carve<SortTile>(base, off, std::max<size_t>(p.h_tiles.size(), 1));
    w.temp = base + off;
    off += align_up(std::max(p.sort_bytes, p.scan_bytes));
    w.total = off;
    return w;
}

}  // namespace

void batch_plan_free(BatchPlan* p) {
    if (!p) return;
    if (p->dev) (void)hipFree(p->dev);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->side) (void)hipStreamDestroy(p->side);
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->join) (void)hipEventDestroy(p->join);
    delete p;
}

int batch_plan_create(const int64_t* h_offsets, const int64_t* h_k, const uint64_t* h_seed, int32_t m,
                      float target, int wide, int wide_groups, BatchPlan** out) {
    if (!out || m < 0 || (m > 0 && (!h_offsets || !h_k)))
        return set_error(BS_ERR_INVALID_ARG, "null plan arguments");
    if (h_offsets && h_offsets[0] != 0) return set_error(BS_ERR_INVALID_ARG, "offsets[0] must be 0");
    for (int j = 0; j < m; ++j) {
        const int64_t n = h_offsets[j + 1] - h_offsets[j];
        if (n < 0) return set_error(BS_ERR_INVALID_ARG, "offsets decrease at object %d", j);
        if (h_k[j] < 0 || h_k[j] > n)
            return set_error(BS_ERR_INVALID_ARG, "object %d: k=%lld outside [0, n=%lld]", j,
                             (long long)h_k[j], (long long)n);
    }
    if (m > 0 && h_offsets[m] >= (int64_t(1) << 31))
        return set_error(BS_ERR_INVALID_ARG, "total candidates %lld >= 2^31", (long long)h_offsets[m]);
    BatchPlan* p = new BatchPlan();
    p->m_all = m;
    p->target = target < 8.f ? 8.f : target;
    // objects without candidates have k = 0 and take no part
    std::vector<int> keep;
    for (int j = 0; j < m; ++j)
        if (h_offsets[j + 1] > h_offsets[j]) keep.push_back(j);
    p->h_out_offs.assign(size_t(m) + 1, 0);
    for (int j = 0; j < m; ++j) p->h_out_offs[j + 1] = p->h_out_offs[j] + h_k[j];
    p->total_k = p->h_out_offs[m];
    p->m = int(keep.size());
    p->kept = keep;
    p->h_kept.assign(keep.begin(), keep.end());
    p->N = m > 0 ? int(h_offsets[m]) : 0;
    p->h_offs.resize(size_t(p->m) + 1);
    p->h_k.resize(p->m);
    p->h_start.resize(p->m);
    p->h_seed.resize(p->m);
    std::vector<int64_t> outo(size_t(p->m) + 1);
    for (int i = 0; i < p->m; ++i) {
        const int j = keep[i];
        const int64_t n = h_offsets[j + 1] - h_offsets[j];
        p->h_offs[i] = int32_t(h_offsets[j]);
        p->h_k[i] = int32_t(h_k[j]);
        p->h_start[i] = int32_t(bs_start_index(h_seed ? h_seed[j] : 0, n));
        p->h_seed[i] = h_seed ? h_seed[j] : 0;
        outo[i] = p->h_out_offs[j];
    }
    p->h_offs[p->m] = p->N;
    outo[p->m] = p->total_k;
    // largest chains first (longest-processing-time order)
    p->h_lpt.clear();
    for (int i = 0; i < p->m; ++i)
        if (p->h_k[i] > 0) p->h_lpt.push_back(i);
    std::stable_sort(p->h_lpt.begin(), p->h_lpt.end(),
                     [&](int a, int b) { return p->h_k[a] > p->h_k[b]; });
    p->mwork = int(p->h_lpt.size());
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per, reinterpret_cast<const void*>(batch_order_kernel<kBatchBlock, kBatchMaxBlocks>), kBatchBlock, 0);
    if (cus <= 0) cus = 256;
    if (per <= 0) per = 1;
    // the largest objects (the head of the LPT order) on 1024-thread
    // workgroups, one CU each, on a share of the CUs: those whose chain is
    // long against the mean work of a 256-thread slot (a 1024-thread
    // workgroup finishes a long chain ~2.5x sooner but takes a whole CU, which
    // costs throughput on short chains), or as many as asked
    int nw = 0;
    if (wide > 0) {
        nw = std::min(wide, p->mwork);
    } else if (wide == 0 && p->mwork > 1) {
        const double mean = double(p->total_k) / double(cus * per);
        while (nw < p->mwork && p->h_k[p->h_lpt[nw]] >= kWideMinK && double(p->h_k[p->h_lpt[nw]]) > 0.5 * mean)
            ++nw;
    }
    p->nwide = nw;
    // cells, blocks and superblocks at most (the 1024-thread workgroups'
    // objects may have more blocks)
    std::vector<char> is_wide(size_t(p->m), 0);
    for (int r = 0; r < nw; ++r) {
        const int i = p->h_lpt[r];
        is_wide[size_t(i)] = 1;
        if (int64_t(p->h_offs[i + 1]) - p->h_offs[i] > int64_t(kLargeCell) * 64 * kBatchMaxBlocks)
            p->wide_blocks = kWideMaxBlocks;
    }
    size_t maxC = 0, maxB = 0, maxS = 0;
    for (int i = 0; i < p->m; ++i) {
        const int64_t n = int64_t(p->h_offs[i + 1]) - p->h_offs[i];
        const int mb = is_wide[size_t(i)] ? p->wide_blocks : kBatchMaxBlocks;
        const double cap = std::min(std::max(1.0, double(n) / double(p->target)), double(64 * mb));
        const size_t c = size_t(cap);
        maxC += c;
        const size_t nb = (c + 63) / 64;
        maxB += nb;
        maxS += (nb + 63) / 64;
    }
    p->maxC = std::max<size_t>(maxC, 1);
    p->maxB = std::max<size_t>(maxB, 1);
    p->maxS = std::max<size_t>(maxS, 1);
    // tiles of the per-object sort (each object sorted where it lies)
    p->h_tiles = sort_tiles(p->h_offs.data(), p->m);
    p->sort_bytes = sort_temp_bytes(int64_t(p->h_tiles.size()));
    p->scan_bytes = scan_temp_bytes(p->N);
    p->h_outo = outo;
    p->ws_bytes = batch_layout(*p, nullptr).total;
    // three quarters of the CUs by default (1,000-part batch: half 1.07-1.10 s,
    // three quarters 0.95-0.96 s, seven eighths 0.95-0.97 s); the batch
    // autotuner times the share on the whole batch
    p->wide_slots = std::min(nw, wide_groups > 0 ? wide_groups : std::max(1, cus - cus / 4));
    const int rest = p->mwork - nw;
    p->slots = std::max(1, std::min((cus - p->wide_slots) * per, std::max(rest, 1)));
    if (nw > 0) {
        hipError_t e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join, hipEventDisableTiming);
        if (e != hipSuccess) {
            batch_plan_free(p);
            return set_error(BS_ERR_HIP, "batch plan stream: %s", hipGetErrorString(e));
        }
    }
    *out = p;
    return BS_OK;
}

// Served micro-batches: per-object output buffers and completion flags
// (index = caller object number), plain launches instead of a graph.
void batch_set_job_io(BatchPlan* p, const std::vector<int32_t*>& order, const std::vector<float*>& radius,
                      const std::vector<uint32_t*>& done) {
    p->h_io.resize(size_t(p->m) + 1);
    for (int i = 0; i < p->m; ++i) {
        const int j = p->kept[i];
        p->h_io[i] = JobIo{order[j], radius[j], done[j], nullptr};
    }
    p->use_graph = false;
}

size_t batch_workspace_bytes(const BatchPlan* p) { return p ? p->ws_bytes : 0; }
int64_t batch_total_k(const BatchPlan* p) { return p ? p->total_k : 0; }
int batch_wide_count(const BatchPlan* p) { return p ? p->nwide : 0; }
void batch_set_split_cells(BatchPlan* p, bool split) {
    if (p) p->split_cells = split;
}
void batch_set_picks(BatchPlan* p, int picks) {
    if (p) p->picks = picks > 0 ? picks : 0;
}
const int64_t* batch_out_offsets(const BatchPlan* p) { return p->h_out_offs.data(); }
int batch_slots(const BatchPlan* p) { return p ? p->slots : 0; }

namespace {

// Validation, per-object grids and the objects' descriptors (w.desc), all
// enqueued on st; shared by the batched launch and the serving ring.  With
// sort_only, up to the per-object Morton sort (keys_s, vals_s).
// narrow_only: every object gets the 256-thread workgroups' block limit
// (the sampler's kernel); otherwise the objects of 1024-thread workgroups may
// have up to kWideMaxBlocks.
int batch_preprocess(BatchPlan* p, const float* pts, int32_t* out_order, float* out_radius, void* ws,
                     size_t ws_bytes, hipStream_t st, BatchWs& w, bool sort_only = false,
                     bool narrow_only = false) {
    if (!pts || (!sort_only && !out_order && p->h_io.empty()))
        return set_error(BS_ERR_INVALID_ARG, "null points or output");
    if (!ws || ws_bytes < p->ws_bytes)
        return set_error(BS_ERR_INVALID_ARG, "workspace %zu bytes < %zu needed", ws_bytes, p->ws_bytes);
    if (reinterpret_cast<uintptr_t>(ws) % kAlign)
        return set_error(BS_ERR_INVALID_ARG, "workspace not %zu-byte aligned", kAlign);
    w = batch_layout(*p, static_cast<char*>(ws));
    const int N = p->N, m = p->m;
    hipError_t e = hipSuccess;
    if (p->dev) {  // the plan's own device copies: nothing to upload
        w.offs = p->d_offs;
        w.ks = p->d_ks;
        w.starts = p->d_starts;
        w.lpt = p->d_lpt;
        w.outo = p->d_outo;
        w.tiles = p->d_tiles;
        w.seeds = p->d_seeds;
        w.kept = p->d_kept;
    } else {
        e = hipMemcpyAsync(w.offs, p->h_offs.data(), p->h_offs.size() * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && m)
            e = hipMemcpyAsync(w.ks, p->h_k.data(), p->h_k.size() * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && m)
            e = hipMemcpyAsync(w.starts, p->h_start.data(), p->h_start.size() * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && p->mwork)
            e = hipMemcpyAsync(w.lpt, p->h_lpt.data(), p->h_lpt.size() * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && !p->h_tiles.empty())
            e = hipMemcpyAsync(w.tiles, p->h_tiles.data(), p->h_tiles.size() * sizeof(SortTile),
                               hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(w.outo, p->h_outo.data(), p->h_outo.size() * 8, hipMemcpyHostToDevice, st);
    }
    const bool use_io = !p->h_io.empty();
    if (e == hipSuccess && use_io)
        e = hipMemcpyAsync(w.io, p->h_io.data(), p->h_io.size() * sizeof(JobIo), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "plan upload: %s", hipGetErrorString(e));
    const int tb = 256;
    const int nblk = (N + tb - 1) / tb;
    const int mblk = (m + tb - 1) / tb;
    hipLaunchKernelGGL(bobj_init_kernel, dim3(mblk), dim3(tb), 0, st, m, w.hd, kBatchMaxBlocks);
    if (!narrow_only && p->nwide > 0 && p->wide_blocks > kBatchMaxBlocks)
        hipLaunchKernelGGL(bwide_kernel, dim3((p->nwide + tb - 1) / tb), dim3(tb), 0, st, p->nwide, w.lpt, w.hd,
                           p->wide_blocks);
    hipLaunchKernelGGL(bvalidate_kernel, dim3(std::min(nblk, 8192)), dim3(tb), 0, st, pts, N, w.offs, m, w.hd);
    hipLaunchKernelGGL(bmorton_kernel, dim3(nblk), dim3(tb), 0, st, pts, N, w.offs, m, w.hd, w.keys, w.vals);
    if ((e = hipGetLastError()) != hipSuccess) return set_error(BS_ERR_HIP, "%s", hipGetErrorString(e));
    e = sort_codes_segmented(w.keys, w.keys_s, w.vals, w.vals_s, w.tiles, int(p->h_tiles.size()), N, w.temp, st);
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "sort: %s", hipGetErrorString(e));
    if (sort_only) return BS_OK;
    hipLaunchKernelGGL(bhist_kernel, dim3(nblk), dim3(tb), 0, st, w.keys_s, N, w.hd);
    hipLaunchKernelGGL(blevel_kernel, dim3(mblk), dim3(tb), 0, st, m, w.offs, w.hd, p->target,
                       p->split_cells ? 1 : 0);
    hipLaunchKernelGGL(bflag_kernel, dim3(nblk), dim3(tb), 0, st, w.keys_s, N, w.hd, w.flags);
    e = inclusive_scan_u32(w.flags, w.cellidx, N, w.temp, st);
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "scan: %s", hipGetErrorString(e));
    if (p->split_cells) {
        hipLaunchKernelGGL(bcstart_kernel, dim3(nblk), dim3(tb), 0, st, w.flags, w.cellidx, N, w.cstart);
        hipLaunchKernelGGL(bsplit_prep_kernel, dim3(mblk), dim3(tb), 0, st, m, w.offs, w.cellidx, w.hd, p->target);
        hipLaunchKernelGGL(bsplit_kernel, dim3(nblk), dim3(tb), 0, st, w.keys_s, w.cellidx, N, w.cstart, w.hd,
                           w.flags);
        e = inclusive_scan_u32(w.flags, w.cellidx, N, w.temp, st);
        if (e != hipSuccess) return set_error(BS_ERR_HIP, "scan: %s", hipGetErrorString(e));
    }
    hipLaunchKernelGGL(bgather_kernel, dim3(nblk), dim3(tb), 0, st, pts, w.keys_s, w.vals_s, w.flags,
                       w.cellidx, N, w.offs, w.starts, w.hd, w.xyzm, w.ids, w.cstart);
    hipLaunchKernelGGL(bobj_fin_kernel, dim3(1), dim3(1024), 0, st, m, w.cellidx, N, w.hd, w.totals);
    const int cblk = int((p->maxC + tb - 1) / tb);
    hipLaunchKernelGGL(bcells_kernel, dim3(cblk), dim3(tb), 0, st, w.cstart, N, w.totals, w.xyzm, w.ids,
                       w.cstat, w.cdyn);
    hipLaunchKernelGGL(bblocks_kernel, dim3(int((p->maxB + tb - 1) / tb)), dim3(tb), 0, st, m, w.hd,
                       w.totals, w.cstat, w.cdyn, w.bstat, w.bdyn);
    hipLaunchKernelGGL(bsuper_kernel, dim3(int((p->maxS + tb - 1) / tb)), dim3(tb), 0, st, m, w.hd,
                       w.totals, w.bstat, w.sbstat);
    hipLaunchKernelGGL(bdesc_kernel, dim3(mblk), dim3(tb), 0, st, m, w.hd, w.ks, w.starts,
                       w.outo, w.xyzm, w.ids, w.cstat, w.cdyn, w.bstat, w.bdyn, w.sbstat,
                       out_order, out_radius, use_io ? w.io : nullptr, w.offs, p->picks, w.desc);
    if ((e = hipGetLastError()) != hipSuccess) return set_error(BS_ERR_HIP, "%s", hipGetErrorString(e));
    return BS_OK;
}

}  // namespace

namespace {

// Everything of one execute, enqueued on st (eagerly, or into a capture):
// preprocessing, the queue reset, the 1024-thread kernel of the longest
// chains on the plan's side stream (forked from st and joined back) and the
// 256-thread kernel of the others.
int enqueue_execute(BatchPlan* p, const float* pts, int32_t* out_order, float* out_radius, void* ws,
                    size_t ws_bytes, hipStream_t st) {
    BatchWs w;
    const int rc = batch_preprocess(p, pts, out_order, out_radius, ws, ws_bytes, st, w);
    if (rc != BS_OK) return rc;
    // both queues restart before either launch can pop
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, w.queue);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && p->nwide > 0) {
        // the largest objects: 1024-thread workgroups, enqueued first so that
        // they find whole CUs free
        e = hipEventRecord(p->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->fork, 0);
        if (e == hipSuccess) {
            if (p->wide_blocks > kBatchMaxBlocks)
                hipLaunchKernelGGL((batch_order_kernel<kWideBlock, kWideMaxBlocks>), dim3(p->wide_slots),
                                   dim3(kWideBlock), 0, p->side, w.desc, w.lpt, p->nwide, w.queue + 1);
            else
                hipLaunchKernelGGL((batch_order_kernel<kWideBlock, kBatchMaxBlocks>), dim3(p->wide_slots),
                                   dim3(kWideBlock), 0, p->side, w.desc, w.lpt, p->nwide, w.queue + 1);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(p->join, p->side);
    }
    if (e == hipSuccess && p->mwork > p->nwide) {
        hipLaunchKernelGGL((batch_order_kernel<kBatchBlock, kBatchMaxBlocks>), dim3(p->slots), dim3(kBatchBlock), 0, st, w.desc,
                           w.lpt + p->nwide, p->mwork - p->nwide, w.queue);
        e = hipGetLastError();
    }
    if (e == hipSuccess && p->nwide > 0) e = hipStreamWaitEvent(st, p->join, 0);
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "order launch: %s", hipGetErrorString(e));
    return BS_OK;
}

void drop_graph(BatchPlan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    for (const void*& k : p->graph_key) k = nullptr;
}

}  // namespace

int batch_plan_upload(BatchPlan* p) {
    if (!p || p->dev) return BS_OK;
    const size_t m1 = size_t(p->m) + 1;
    size_t off = 0;
    auto place = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(std::max<size_t>(bytes, 8));
        return at;
    };
    const size_t o_offs = place(m1 * 4), o_ks = place(m1 * 4), o_starts = place(m1 * 4), o_lpt = place(m1 * 4),
                 o_kept = place(m1 * 4), o_outo = place(m1 * 8), o_seeds = place(m1 * 8),
                 o_tiles = place(std::max<size_t>(p->h_tiles.size(), 1) * sizeof(SortTile));
    hipError_t e = hipMalloc(&p->dev, off);
    if (e != hipSuccess) {
        p->dev = nullptr;
        return set_error(BS_ERR_OUT_OF_MEMORY, "plan arrays: %s", hipGetErrorString(e));
    }
    char* b = static_cast<char*>(p->dev);
    p->d_offs = reinterpret_cast<int32_t*>(b + o_offs);
    p->d_ks = reinterpret_cast<int32_t*>(b + o_ks);
    p->d_starts = reinterpret_cast<int32_t*>(b + o_starts);
    p->d_lpt = reinterpret_cast<int32_t*>(b + o_lpt);
    p->d_kept = reinterpret_cast<int32_t*>(b + o_kept);
    p->d_outo = reinterpret_cast<int64_t*>(b + o_outo);
    p->d_seeds = reinterpret_cast<uint64_t*>(b + o_seeds);
    p->d_tiles = reinterpret_cast<SortTile*>(b + o_tiles);
    auto put = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    put(p->d_offs, p->h_offs.data(), p->h_offs.size() * 4);
    put(p->d_ks, p->h_k.data(), p->h_k.size() * 4);
    put(p->d_starts, p->h_start.data(), p->h_start.size() * 4);
    put(p->d_lpt, p->h_lpt.data(), p->h_lpt.size() * 4);
    put(p->d_kept, p->h_kept.data(), p->h_kept.size() * 4);
    put(p->d_outo, p->h_outo.data(), p->h_outo.size() * 8);
    put(p->d_seeds, p->h_seed.data(), p->h_seed.size() * 8);
    put(p->d_tiles, p->h_tiles.data(), p->h_tiles.size() * sizeof(SortTile));
    if (e != hipSuccess) {
        (void)hipFree(p->dev);
        p->dev = nullptr;
        return set_error(BS_ERR_HIP, "plan arrays: %s", hipGetErrorString(e));
    }
    return BS_OK;
}

int batch_plan_execute(BatchPlan* p, const float* pts, int32_t* out_order, float* out_radius, void* ws,
                       size_t ws_bytes, hipStream_t st) {
    if (!p) return set_error(BS_ERR_INVALID_ARG, "null plan");
    if (p->mwork == 0) return BS_OK;
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->use_graph || !p->dev) return enqueue_execute(p, pts, out_order, out_radius, ws, ws_bytes, st);
    // host checks first: nothing may fail inside the capture
    if (!pts || !out_order) return set_error(BS_ERR_INVALID_ARG, "null points or output");
    if (!ws || ws_bytes < p->ws_bytes)
        return set_error(BS_ERR_INVALID_ARG, "workspace %zu bytes < %zu needed", ws_bytes, p->ws_bytes);
    if (reinterpret_cast<uintptr_t>(ws) % kAlign)
        return set_error(BS_ERR_INVALID_ARG, "workspace not %zu-byte aligned", kAlign);
    const void* key[4] = {ws, pts, out_order, out_radius};
    if (!p->exec || !std::equal(key, key + 4, p->graph_key)) {
        // one graph for the whole execute: a capture stream forks the side
        // stream for the wide kernel and joins it back
        drop_graph(p);
        hipStream_t cap = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (e != hipSuccess) return set_error(BS_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        int rc = BS_OK;
        if (e == hipSuccess) {
            rc = enqueue_execute(p, pts, out_order, out_radius, ws, ws_bytes, cap);
            const hipError_t e2 = hipStreamEndCapture(cap, &p->graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess && rc == BS_OK) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cap);
        if (rc != BS_OK || e != hipSuccess) {
            drop_graph(p);
            return rc != BS_OK ? rc : set_error(BS_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
        }
        std::copy(key, key + 4, p->graph_key);
    }
    const hipError_t e = hipGraphLaunch(p->exec, st);
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "graph launch: %s", hipGetErrorString(e));
    return BS_OK;
}

int batch_plan_execute_sample(BatchPlan* p, int S, int K, float vicinity, const float* pts, int32_t* out_order,
                              float* out_radius, int32_t* out_count, void* ws, size_t ws_bytes, hipStream_t st) {
    if (!p) return set_error(BS_ERR_INVALID_ARG, "null plan");
    if (S < 0 || S > kSampleMaxSlots || K == 0 || !(vicinity >= 0.f) || (S == 0 && vicinity > 0.f))
        return set_error(BS_ERR_INVALID_ARG, "sampler: sample size %d (0..%d), growth %d (>= 1 or < 0), vicinity %g",
                         S, kSampleMaxSlots, K, double(vicinity));
    std::lock_guard<std::mutex> lk(p->mu);
    hipError_t e = hipSuccess;
    if (out_count && p->m_all > 0) {  // objects with no work made no picks
        hipLaunchKernelGGL(fill_i32_kernel, dim3(std::min((p->m_all + 255) / 256, 1024)), dim3(256), 0, st,
                           out_count, p->m_all, 0);
        if ((e = hipGetLastError()) != hipSuccess) return set_error(BS_ERR_HIP, "%s", hipGetErrorString(e));
    }
    if (p->mwork == 0) return BS_OK;
    BatchWs w;
    // the sampler's 256-thread workgroups hold at most kBatchMaxBlocks blocks
    const int rc = batch_preprocess(p, pts, out_order, out_radius, ws, ws_bytes, st, w, false, true);
    if (rc != BS_OK) return rc;
    const int m = p->m, N = p->N, tb = 256;
    if (!p->dev) {  // otherwise w.seeds and w.kept are the plan's device copies
        e = hipMemcpyAsync(w.seeds, p->h_seed.data(), size_t(m) * 8, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(w.kept, p->h_kept.data(), size_t(m) * 4, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return set_error(BS_ERR_HIP, "sampler upload: %s", hipGetErrorString(e));
    }
    hipLaunchKernelGGL(bpos_kernel, dim3((N + tb - 1) / tb), dim3(tb), 0, st, w.keys_s, w.ids, N, w.offs, w.pos_of);
    SampleParams prm{S, K, vicinity, 0};
    hipLaunchKernelGGL(bsdesc_kernel, dim3((m + tb - 1) / tb), dim3(tb), 0, st, m, w.hd, w.offs, w.seeds, w.kept,
                       w.pos_of, w.cellidx, prm, out_count, w.sdesc);
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, w.queue);
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per, reinterpret_cast<const void*>(sample_batch_kernel<kBatchBlock>), kBatchBlock, 0);
    if (cus <= 0) cus = 256;
    if (per <= 0) per = 1;
    if ((e = hipGetLastError()) != hipSuccess) return set_error(BS_ERR_HIP, "sampler setup: %s", hipGetErrorString(e));
    // the largest objects on 1024-thread workgroups, launched first on the
    // plan's side stream (as the exact ordering does), the others beside
    const int nw = p->nwide;
    if (nw > 0) {
        e = hipEventRecord(p->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->fork, 0);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(sample_batch_kernel<kWideBlock>, dim3(p->wide_slots), dim3(kWideBlock), 0, p->side,
                               w.desc, w.sdesc, w.lpt, nw, w.queue + 1);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(p->join, p->side);
    }
    if (e == hipSuccess && p->mwork > nw) {
        const int slots = std::max(1, std::min((cus - (nw > 0 ? p->wide_slots : 0)) * per, p->mwork - nw));
        hipLaunchKernelGGL(sample_batch_kernel<kBatchBlock>, dim3(slots), dim3(kBatchBlock), 0, st, w.desc, w.sdesc,
                           w.lpt + nw, p->mwork - nw, w.queue);
        e = hipGetLastError();
    }
    if (e == hipSuccess && nw > 0) e = hipStreamWaitEvent(st, p->join, 0);
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "sampler launch: %s", hipGetErrorString(e));
    return BS_OK;
}

int batch_work_count(const BatchPlan* p) { return p ? p->mwork : 0; }

int batch_morton_order(BatchPlan* p, const float* pts, int32_t* out_perm, void* ws, size_t ws_bytes,
                       hipStream_t st) {
    if (!p || !out_perm) return set_error(BS_ERR_INVALID_ARG, "null plan or output");
    if (p->N == 0) return BS_OK;
    std::lock_guard<std::mutex> lk(p->mu);
    BatchWs w;
    const int rc = batch_preprocess(p, pts, nullptr, nullptr, ws, ws_bytes, st, w, true);
    if (rc != BS_OK) return rc;
    hipLaunchKernelGGL(blocal_kernel, dim3((p->N + 255) / 256), dim3(256), 0, st, w.keys_s, w.vals_s, p->N, w.offs,
                       out_perm);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BS_OK : set_error(BS_ERR_HIP, "%s", hipGetErrorString(e));
}

int batch_plan_publish(BatchPlan* p, const float* pts, void* ws, size_t ws_bytes, const ServeRing& ring,
                       uint32_t base, hipStream_t st) {
    if (!p) return set_error(BS_ERR_INVALID_ARG, "null plan");
    if (p->mwork == 0) return BS_OK;
    if (p->h_io.empty()) return set_error(BS_ERR_INVALID_ARG, "serving needs per-job outputs");
    std::lock_guard<std::mutex> lk(p->mu);
    BatchWs w;
    const int rc = batch_preprocess(p, pts, nullptr, nullptr, ws, ws_bytes, st, w);
    if (rc != BS_OK) return rc;
    hipLaunchKernelGGL(publish_kernel, dim3(1), dim3(256), 0, st, w.desc, w.lpt, p->mwork,
                       static_cast<ObjDesc*>(ring.slots), ring.cap, base, ring.tail);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "publish: %s", hipGetErrorString(e));
    return BS_OK;
}

size_t serve_slot_bytes() { return sizeof(ObjDesc); }

hipError_t launch_serve(const ServeRing& ring, int workgroups, uint32_t idle_polls, hipStream_t st) {
    hipLaunchKernelGGL(serve_kernel, dim3(workgroups), dim3(kWideBlock), 0, st,
                       static_cast<const ObjDesc*>(ring.slots), ring.cap, ring.head, ring.tail, ring.stop,
                       idle_polls);
    return hipGetLastError();
}

}  // namespace bs
