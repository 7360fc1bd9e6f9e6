// bs_grid.h -- internal declarations of the grid-pruned ordering.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bs {

// Device-written description of one object's grid (chosen on the device).
struct GridHeader {
    uint32_t hist[31];   // adjacent sorted pairs first separated by each code prefix length
    int32_t level;       // cells: runs of sorted Morton codes sharing their top `level` bits
    int32_t C;           // occupied cells
    int32_t B;           // cells per block (power of two >= 64)
    int32_t NB;          // blocks (<= workgroup size)
    int32_t start_pos;   // sorted position of the start candidate
    int32_t start_cell;  // its cell
    uint32_t lead_id;    // after a leading full scan: its last pick (original index)
    uint32_t lead_m;     // and the bits of that pick's m
    int32_t pad[25];
};
static_assert(sizeof(GridHeader) == 256, "grid header size");

// What the ordering loop needs for one object.
struct GridObject {
    int k;
    uint32_t start_id;
    int C, B, NB;
    int start_pos, start_cell;
    float4* xyzm;              // [n] Morton-sorted x, y, z, m (m = -1 once chosen)
    const uint32_t* ids;       // [n] original index of each sorted candidate
    const float4* cstat;       // [2C] (lo.xyz, start) (hi.xyz, count)
    uint4* cdyn;               // [2C] (key lo, key hi, pos, -) (x, y, z, -)
    const float4* bstat;       // [2NB] block boxes
    const uint4* bdyn;         // [2NB] initial block bests (key lo, key hi, pos, cell) (x, y, z, -)
    const float4* sbstat;      // [2 ceil(NB/64)] superblock boxes
    int32_t* order;
    float* radius;
    uint64_t* ticks;           // optional: device wall clock after each step
    int max_picks;             // several-picks-per-round kernel: picks per round (<= 32)
    int t0;                    // index of the start pick in the order (0, or the picks a
                               // leading full scan made minus one)
    float start_m;             // m of the start pick (+inf, or its value after a leading scan)
};

// Byte offsets of the grid workspace pieces.
struct GridLayout {
    size_t dev_header, grid_header, codes, vals, codes_sorted, ids, flags, cellidx, cstart, xyzm,
        cstat, cdyn, bstat, bdyn, sbstat, lead_slots, temp;
    size_t temp_bytes;
    size_t total;
};

GridLayout grid_layout(int64_t n, int block);
int grid_block_size(int64_t n);
// Blocks of 64 cells one workgroup of `block` threads holds in LDS; `picks`
// > 1 selects the several-picks-per-round kernel (at most `picks` per round).
int grid_max_blocks(int block, int picks);
struct LaunchOpts;
// Candidates in Morton order (validation, codes, radix sort, gather) in the
// grid workspace, for the sorted cooperative scan.
struct DevHeader;
struct SortedPoints {
    DevHeader* hdr;
    const float4* xyzm;        // [n] x, y, z, +inf in Morton order
    const uint32_t* ids;       // [n] original index of each
    const uint32_t* codes;     // [n] their Morton codes, ascending
    const int32_t* start_pos;  // device: sorted position of the start
    void* slots;               // exchange records of the cooperative scan
};
hipError_t launch_sorted_points(const float* pts, int n, int start, void* ws, hipStream_t st, SortedPoints* out);
// The candidates' indices in Morton order (launch_sorted_points, then a copy).
hipError_t launch_morton_order(const float* pts, int n, int32_t* out_perm, void* ws, hipStream_t st);

// lead >= 2 (several-picks kernel only): picks 0 .. lead-1 come from the
// cooperative full scan of shape *lead_shape, which hands its state to the
// grid kernel; otherwise the grid kernel makes every pick.
struct ScanShape;
hipError_t launch_grid(const float* pts, int n, int k, int start, int32_t* order, float* radius,
                       void* ws, float target, int block, int picks, uint64_t* ticks,
                       hipStream_t st, const LaunchOpts* ev = nullptr, int lead = 0,
                       const ScanShape* lead_shape = nullptr);

}  // namespace bs
