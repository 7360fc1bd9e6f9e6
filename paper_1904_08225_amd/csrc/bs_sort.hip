// bs_sort.hip -- the sort and the scans of the grid builds (one object, or
// the objects of a batch), as plain kernels: nothing here records a memset,
// so a captured graph can hold a whole batch execute.
//
// A grid needs its object's candidates in Morton order (30-bit codes).  The
// objects of a batch are contiguous segments of one array and each is sorted
// where it lies.  Stable LSD radix sort, three passes of 10 bits; a tile of
// 4,096 keys lies inside one segment.  Per pass:
//   1. digit counts of every tile, stored digit-major within each segment
//      (segment j, digit d, tile t at base_j + d * T_j + t);
//   2. one exclusive scan over all counts: segment j's counts sum to its
//      length, so its region of the scan starts at its first element, and
//      (j, d, t) receives the output position of the tile's first key with
//      digit d;
//   3. a stable scatter: round r of a tile holds positions r * 256 + thread,
//      and a key's rank among the tile's keys with its digit is the count of
//      that digit in the earlier rounds, in the earlier wavefronts of its
//      round, and in the lower lanes of its wavefront (a match of the ten
//      digit bits by ballot).
// Keys may carry bits above the code (a batch keeps the object number
// there); only bits 0 .. 29 are sorted on.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bs_internal.h"

namespace bs {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = kSortTileKeys / kSortThreads;
constexpr int kSortDigitBits = 10;
constexpr int kSortBins = 1 << kSortDigitBits;
constexpr int kSortPasses = 3;
static_assert(kSortPasses * kSortDigitBits == 30, "three passes cover the 30-bit codes");
static_assert(kSortThreads % 64 == 0 && kSortTileKeys % kSortThreads == 0, "tile shape");

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kScanTopThreads = 1024;

__device__ __forceinline__ SortTile tile_of(const SortTile* tiles, int t, int n, int ntiles) {
    if (tiles) return tiles[t];
    SortTile s;
    s.start = t * kSortTileKeys;
    s.count = min(kSortTileKeys, n - s.start);
    s.hbase = t;
    s.ntiles = ntiles;
    return s;
}

template <class K>
__global__ void __launch_bounds__(kSortThreads)
    sort_count_kernel(const K* __restrict__ keys, const SortTile* __restrict__ tiles, int n, int ntiles, int shift,
                      uint32_t* __restrict__ hist) {
    __shared__ uint32_t cnt[kSortBins];
    const SortTile s = tile_of(tiles, int(blockIdx.x), n, ntiles);
    for (int d = threadIdx.x; d < kSortBins; d += kSortThreads) cnt[d] = 0u;
    __syncthreads();
    for (int p = threadIdx.x; p < s.count; p += kSortThreads)
        atomicAdd(&cnt[uint32_t(keys[s.start + p] >> shift) & (kSortBins - 1)], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < kSortBins; d += kSortThreads)
        hist[size_t(s.hbase) + size_t(d) * size_t(s.ntiles)] = cnt[d];
}

template <class K>
__global__ void __launch_bounds__(kSortThreads)
    sort_scatter_kernel(const K* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, K* __restrict__ keys_out,
                        uint32_t* __restrict__ vals_out, const SortTile* __restrict__ tiles, int n, int ntiles,
                        int shift, const uint32_t* __restrict__ pos) {
    constexpr int NW = kSortThreads / 64;
    __shared__ uint32_t next[kSortBins];       // output position of the digit's next key
    __shared__ uint16_t wcnt[NW][kSortBins];   // this round: keys of the digit in each wavefront
    const SortTile s = tile_of(tiles, int(blockIdx.x), n, ntiles);
    for (int d = threadIdx.x; d < kSortBins; d += kSortThreads) {
        next[d] = pos[size_t(s.hbase) + size_t(d) * size_t(s.ntiles)];
#pragma unroll
        for (int w = 0; w < NW; ++w) wcnt[w][d] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t below = (uint64_t(1) << lane) - 1u;
    for (int r = 0; r < kSortRounds; ++r) {
        const int p = r * kSortThreads + int(threadIdx.x);
        const bool live = p < s.count;
        K key = 0;
        uint32_t val = 0u, d = 0u;
        if (live) {
            key = keys_in[s.start + p];
            val = vals_in[s.start + p];
            d = uint32_t(key >> shift) & (kSortBins - 1);
        }
        uint64_t same = __ballot(live);
#pragma unroll
        for (int b = 0; b < kSortDigitBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            same &= bit ? m : ~m;
        }
        const int rank = __popcll(same & below);
        const bool leader = live && rank == 0;  // lowest lane of its digit in this wavefront
        if (leader) wcnt[wave][d] = uint16_t(__popcll(same));
        __syncthreads();
        if (live) {
            uint32_t at = next[d] + uint32_t(rank);
            for (int w = 0; w < wave; ++w) at += wcnt[w][d];
            keys_out[at] = key;
            vals_out[at] = val;
        }
        __syncthreads();
        if (leader) {
            atomicAdd(&next[d], uint32_t(wcnt[wave][d]));
            wcnt[wave][d] = 0;
        }
        __syncthreads();
    }
}

// Sum of each tile of kScanTile items.
__global__ void __launch_bounds__(kScanThreads)
    scan_tile_sums_kernel(const uint32_t* __restrict__ in, size_t n, uint32_t* __restrict__ sums) {
    __shared__ uint32_t part[kScanThreads / 64];
    const size_t base = size_t(blockIdx.x) * kScanTile;
    uint32_t v = 0u;
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads)
        if (base + size_t(i) < n) v += in[base + size_t(i)];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += uint32_t(__shfl_xor(int(v), o, 64));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0u;
        for (int w = 0; w < kScanThreads / 64; ++w) t += part[w];
        sums[blockIdx.x] = t;
    }
}

// Exclusive prefix of a wavefront's values (inclusive prefix minus own value).
__device__ __forceinline__ uint32_t wave_exclusive(uint32_t v, uint32_t* total) {
    const int lane = threadIdx.x & 63;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = uint32_t(__shfl_up(int(x), o, 64));
        if (lane >= o) x += y;
    }
    *total = uint32_t(__shfl(int(x), 63, 64));
    return x - v;
}

// One workgroup: the tile sums become their exclusive prefix, in place.
__global__ void __launch_bounds__(kScanTopThreads) scan_top_kernel(uint32_t* __restrict__ sums, int T) {
    constexpr int NW = kScanTopThreads / 64;
    __shared__ uint32_t wsum[NW];
    const int per = (T + kScanTopThreads - 1) / kScanTopThreads;
    const int a = min(T, int(threadIdx.x) * per), b = min(T, a + per);
    uint32_t local = 0u;
    for (int i = a; i < b; ++i) local += sums[i];
    uint32_t wt;
    const uint32_t ex = wave_exclusive(local, &wt);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) wsum[wave] = wt;
    __syncthreads();
    uint32_t off = ex;
    for (int w = 0; w < wave; ++w) off += wsum[w];
    for (int i = a; i < b; ++i) {
        const uint32_t v = sums[i];
        sums[i] = off;
        off += v;
    }
}

// Each tile's prefix from its offset: a thread holds kScanItems consecutive
// items.  In place is allowed (a thread reads its items before writing).
template <bool EXCLUSIVE>
__global__ void __launch_bounds__(kScanThreads)
    scan_tiles_kernel(const uint32_t* in, uint32_t* out, size_t n, const uint32_t* __restrict__ tile_off) {
    constexpr int NW = kScanThreads / 64;
    __shared__ uint32_t wsum[NW];
    const size_t base = size_t(blockIdx.x) * kScanTile + size_t(threadIdx.x) * kScanItems;
    uint32_t v[kScanItems];
    uint32_t local = 0u;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = base + size_t(j) < n ? in[base + size_t(j)] : 0u;
        local += v[j];
    }
    uint32_t wt;
    const uint32_t ex = wave_exclusive(local, &wt);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) wsum[wave] = wt;
    __syncthreads();
    uint32_t run = tile_off[blockIdx.x] + ex;
    for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint32_t x = v[j];
        if (!EXCLUSIVE) run += x;
        if (base + size_t(j) < n) out[base + size_t(j)] = run;
        if (EXCLUSIVE) run += x;
    }
}

size_t scan_sums_bytes(size_t n) { return align_up(std::max<size_t>((n + kScanTile - 1) / kScanTile, 1) * 4); }

template <bool EXCLUSIVE>
hipError_t scan_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* sums, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const size_t T = (n + kScanTile - 1) / kScanTile;
    if (T > size_t(1) << 26) return hipErrorInvalidValue;
    hipLaunchKernelGGL(scan_tile_sums_kernel, dim3(unsigned(T)), dim3(kScanThreads), 0, st, in, n, sums);
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanTopThreads), 0, st, sums, int(T));
    hipLaunchKernelGGL(scan_tiles_kernel<EXCLUSIVE>, dim3(unsigned(T)), dim3(kScanThreads), 0, st, in, out, n,
                       sums);
    return hipGetLastError();
}

size_t hist_entries(int64_t ntiles) { return size_t(kSortBins) * size_t(std::max<int64_t>(ntiles, 1)); }

template <class K>
hipError_t sort_codes(K* keys, K* keys_s, uint32_t* vals, uint32_t* vals_s, const SortTile* tiles, int n,
                      int ntiles, void* temp, hipStream_t st) {
    if (n <= 0 || ntiles <= 0) return hipSuccess;
    const size_t H = hist_entries(ntiles);
    uint32_t* hist = static_cast<uint32_t*>(temp);
    uint32_t* sums = reinterpret_cast<uint32_t*>(static_cast<char*>(temp) + align_up(H * 4));
    // passes alternate keys -> keys_s -> keys -> keys_s: the result lands in keys_s / vals_s
    K* kin[kSortPasses] = {keys, keys_s, keys};
    K* kout[kSortPasses] = {keys_s, keys, keys_s};
    uint32_t* vin[kSortPasses] = {vals, vals_s, vals};
    uint32_t* vout[kSortPasses] = {vals_s, vals, vals_s};
    for (int pass = 0; pass < kSortPasses; ++pass) {
        const int shift = pass * kSortDigitBits;
        hipLaunchKernelGGL(sort_count_kernel<K>, dim3(ntiles), dim3(kSortThreads), 0, st, kin[pass], tiles, n,
                           ntiles, shift, hist);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = scan_u32<true>(hist, hist, H, sums, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(sort_scatter_kernel<K>, dim3(ntiles), dim3(kSortThreads), 0, st, kin[pass], vin[pass],
                           kout[pass], vout[pass], tiles, n, ntiles, shift, hist);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

int64_t sort_tile_count(int64_t n) { return (n + kSortTileKeys - 1) / kSortTileKeys; }

std::vector<SortTile> sort_tiles(const int32_t* offs, int m) {
    std::vector<SortTile> t;
    int64_t base = 0;
    for (int j = 0; j < m; ++j) {
        const int n = offs[j + 1] - offs[j];
        const int T = int(sort_tile_count(n));
        for (int i = 0; i < T; ++i) {
            SortTile s;
            s.start = offs[j] + i * kSortTileKeys;
            s.count = std::min(kSortTileKeys, n - i * kSortTileKeys);
            s.hbase = int32_t(base + i);
            s.ntiles = T;
            t.push_back(s);
        }
        base += int64_t(kSortBins) * T;
    }
    return t;
}

size_t sort_temp_bytes(int64_t ntiles) {
    const size_t H = hist_entries(ntiles);
    return align_up(H * 4) + scan_sums_bytes(H);
}

size_t scan_temp_bytes(int64_t n) { return scan_sums_bytes(size_t(std::max<int64_t>(n, 1))); }

hipError_t sort_codes_u32(uint32_t* codes, uint32_t* codes_s, uint32_t* vals, uint32_t* vals_s, int n, void* temp,
                          hipStream_t st) {
    return sort_codes<uint32_t>(codes, codes_s, vals, vals_s, nullptr, n, int(sort_tile_count(n)), temp, st);
}

hipError_t sort_codes_segmented(uint64_t* keys, uint64_t* keys_s, uint32_t* vals, uint32_t* vals_s,
                                const SortTile* d_tiles, int ntiles, int n, void* temp, hipStream_t st) {
    return sort_codes<uint64_t>(keys, keys_s, vals, vals_s, d_tiles, n, ntiles, temp, st);
}

hipError_t inclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t st) {
    return scan_u32<false>(in, out, size_t(std::max<int64_t>(n, 0)), static_cast<uint32_t*>(temp), st);
}

}  // namespace bs
