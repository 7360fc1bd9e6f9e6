// bs_internal.h -- declarations shared by the HIP sources of libbluesurfels.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/bluesurfels.h"

namespace bs {

// Per-call device header at the start of every workspace (256 bytes).
struct DevHeader {
    uint32_t nonfinite;  // set by the validate kernel if any coordinate is not finite
    uint32_t error;      // set by a kernel whose bounded wait gave up
    uint32_t bbox[6];    // order-preserving uint encodings: min x,y,z then max x,y,z
    uint32_t pad[56];
};
static_assert(sizeof(DevHeader) == 256, "header size");

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Resident-scan launch shape.
struct ScanShape {
    int block = 0;       // threads per workgroup
    int per_thread = 0;  // candidates per thread
    int groups = 0;      // workgroups (1 = single-workgroup kernel)
};

// Largest cooperative grid this library launches for the resident scan.
constexpr int kMaxCoopGroups = 1024;

// Supported (block, per_thread) instantiations of the resident scan.
bool scan_shape_supported(int block, int per_thread);
// Choose a resident-scan shape for n candidates on a device with `cus`
// compute units; returns false if n does not fit in registers.
bool choose_scan_shape(int64_t n, int cus, int want_block, int want_pt, int want_groups,
                       ScanShape* out);
size_t scan_workspace_bytes(const ScanShape& s);
// Exchange records of a cooperative scan of `groups` workgroups.
size_t scan_slot_bytes(int groups);

// Kernel launchers (bs_scan.hip).  All return hipError_t of the launch.
hipError_t launch_init_header(DevHeader* hdr, hipStream_t st);
hipError_t launch_validate(const float* pts, int64_t n, DevHeader* hdr, hipStream_t st);
// Per-call launch options of the ordering kernels: optional events recorded
// on the launch stream right before and right after the ordering kernel
// itself (not the validation / grid build before it), and the poll limit of
// the cooperative kernels' bounded waits (0 = the default, about a second).
struct LaunchOpts {
    hipEvent_t begin = nullptr;
    hipEvent_t end = nullptr;
    uint32_t spin_limit = 0;
};
// Default poll limit of a bounded wait (each poll sleeps a few cycles).
constexpr uint32_t kDefaultSpinLimit = 1u << 21;
inline uint32_t spin_limit_of(const LaunchOpts* o) {
    return (o && o->spin_limit) ? o->spin_limit : kDefaultSpinLimit;
}
// After an ordering kernel whose bounded wait may give up: if the header's
// error word is set, every output becomes order = -2, radius = NaN (the
// outputs were left partly written).
hipError_t launch_finish(const DevHeader* hdr, int32_t* order, float* radius, int k, hipStream_t st);

// Picks 0 .. k_stop-1 (k_stop < 0: all k); with m_out / handoff the scan
// leaves its state for a following kernel (see scan_kernel).
hipError_t launch_scan(const ScanShape& s, const float* pts, int n, int k, int start,
                       int32_t* order, float* radius, DevHeader* hdr, void* scratch,
                       uint64_t* ticks, hipStream_t st, const LaunchOpts* ev = nullptr,
                       int k_stop = -1, float* m_out = nullptr, uint32_t* handoff = nullptr);

// Several exact picks per step (bs_scan_mp.hip): the candidates in Morton
// order in the grid workspace `ws` (grid_layout(n, 1024).total bytes), at
// most `picks` per step.  Shapes: 1024-thread workgroups, 2..256 of them.
bool scan_several_supported(const ScanShape& s);
hipError_t launch_scan_several(const ScanShape& s, const float* pts, int n, int k, int start, int32_t* order,
                               float* radius, void* ws, uint64_t* ticks, int picks, hipStream_t st,
                               const LaunchOpts* ev = nullptr);

// Batched plans (bs_batch.hip).
struct BatchPlan;
// wide: objects (largest k first) for 1024-thread workgroups in
// batch_plan_execute; 0 = automatic, -1 = none (see bs_tuning.batch_wide);
// wide_groups: those workgroups (0 = automatic, see bs_tuning.groups)
int batch_plan_create(const int64_t* h_offsets, const int64_t* h_k, const uint64_t* h_seed, int32_t m,
                      float target, int wide, int wide_groups, BatchPlan** out);
void batch_plan_free(BatchPlan* p);
// Device copies of the plan's arrays (synchronous; batch and hierarchy
// plans: their executes then upload nothing and run as one captured graph).
int batch_plan_upload(BatchPlan* p);
size_t batch_workspace_bytes(const BatchPlan* p);
int64_t batch_total_k(const BatchPlan* p);
// Each object's candidates in Morton order (indices within the object), at
// the object's rows of out_perm.
int batch_morton_order(BatchPlan* p, const float* pts, int32_t* out_perm, void* ws, size_t ws_bytes,
                       hipStream_t st);
// Objects ordered by the 1024-thread workgroups.
int batch_wide_count(const BatchPlan* p);
// Most exact picks per round of every object (1..32; 0 = by mean cell size).
void batch_set_picks(BatchPlan* p, int picks);
// Cut each object's Morton-prefix cells into runs of bounded length (for
// candidate sets made of compact groups, whose prefix cells are uneven).
void batch_set_split_cells(BatchPlan* p, bool split);
const int64_t* batch_out_offsets(const BatchPlan* p);
int batch_slots(const BatchPlan* p);
void batch_set_job_io(BatchPlan* p, const std::vector<int32_t*>& order, const std::vector<float*>& radius,
                      const std::vector<uint32_t*>& done);
// Serving ring: descriptors of published objects, consumed by a persistent
// kernel.  head = next descriptor to claim, tail = published count (both
// device memory); stop lives in pinned host memory.
struct ServeRing {
    void* slots = nullptr;      // cap descriptors of serve_slot_bytes() each
    uint32_t cap = 0;
    uint32_t* head = nullptr;
    uint32_t* tail = nullptr;
    const uint32_t* stop = nullptr;
};
int batch_work_count(const BatchPlan* p);  // objects with k > 0
// Preprocess the plan's objects on st, then append their descriptors
// (largest k first) at ring positions base, base + 1, ... and advance tail.
int batch_plan_publish(BatchPlan* p, const float* pts, void* ws, size_t ws_bytes, const ServeRing& ring,
                       uint32_t base, hipStream_t st);
size_t serve_slot_bytes();
// Persistent ordering workers: claim published descriptors until stop is set
// and nothing is left, or after idle_polls polls without work.
hipError_t launch_serve(const ServeRing& ring, int workgroups, uint32_t idle_polls, hipStream_t st);

int batch_plan_execute(BatchPlan* p, const float* pts, int32_t* out_order, float* out_radius, void* ws,
                       size_t ws_bytes, hipStream_t st);

// Ordered surfel records and the prefix-length estimate (bs_emit.hip).
constexpr int kMaxPrefixPm = 4096;  // largest p_m of the median estimate
hipError_t launch_emit(const float* pts, const float* nrm, const uint8_t* col, int64_t n, const int32_t* order,
                       int64_t k, void* out, hipStream_t st);
hipError_t launch_median_nn(const float* pts, int64_t n, const int32_t* order, int pm, float* out_rm,
                            hipStream_t st);

// Error reporting (bs_api.cpp).
int set_error(int code, const char* fmt, ...);

// One ordering on a caller-provided workspace (bs_api.cpp): argument checks,
// plan, launches.  start_index -1 derives the start from `seed`.
int order_impl(const float* d_points, int64_t n, int64_t k, uint64_t seed, int64_t start_index,
               int32_t* d_out_order, float* d_out_radius, uint64_t* d_ticks, const LaunchOpts* ev,
               void* d_workspace, size_t workspace_bytes, const bs_tuning* tuning, void* stream);

// Sort and scans of the grid builds (bs_sort.hip): a stable radix sort of
// 30-bit Morton codes (within segments for a batch) and an inclusive scan.
constexpr int kSortTileKeys = 4096;
struct SortTile {
    int32_t start, count;  // the tile's keys
    int32_t hbase;         // count index of (its segment, digit 0, this tile)
    int32_t ntiles;        // tiles of its segment
};
int64_t sort_tile_count(int64_t n);
// Tiles of the segments offs[j] .. offs[j+1]-1 (host).
std::vector<SortTile> sort_tiles(const int32_t* offs, int m);
size_t sort_temp_bytes(int64_t ntiles);
size_t scan_temp_bytes(int64_t n);
// One segment: (codes, vals) sorted by bits 0..29 into (codes_s, vals_s);
// codes and vals are overwritten.
hipError_t sort_codes_u32(uint32_t* codes, uint32_t* codes_s, uint32_t* vals, uint32_t* vals_s, int n, void* temp,
                          hipStream_t st);
// Segments given by device tiles (sort_tiles): each sorted where it lies.
hipError_t sort_codes_segmented(uint64_t* keys, uint64_t* keys_s, uint32_t* vals, uint32_t* vals_s,
                                const SortTile* d_tiles, int ntiles, int n, void* temp, hipStream_t st);
hipError_t inclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t st);

// The autotuned configuration for (n, k) on the current device, if any.
bool tuned_lookup(int64_t n, int64_t k, bs_tuning* out);
int forced_tuning(bs_tuning* out);

}  // namespace bs

// The C ABI's batch plan handle (opaque in the public header).
struct bs_batch_plan {
    bs::BatchPlan* p;
    int32_t m_all;
};
