// bs_sample.h -- internal declarations of the randomized progressive sampler
// (paper Sec. 3.2) and of the prefix quality measure (Sec. 3.3).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bs {

struct LaunchOpts;
struct BatchPlan;

// One object: the grid build of the exact grid ordering (1024-thread
// workgroup, cells of about `target` candidates), then the sampler kernel.
// The workspace is grid_layout(n, 1024).total bytes.
hipError_t launch_grid_sample(const float* pts, int n, int k, int start, uint64_t seed, int S, int K,
                              float vicinity, int32_t* order, float* radius, int32_t* count, void* ws,
                              float target, uint64_t* ticks, hipStream_t st, const LaunchOpts* ev);

// A batch plan's objects through the sampler (same preprocessing and
// workspace as batch_plan_execute); out_count: NULL or device int32[m].
int batch_plan_execute_sample(BatchPlan* p, int S, int K, float vicinity, const float* pts, int32_t* out_order,
                              float* out_radius, int32_t* out_count, void* ws, size_t ws_bytes, hipStream_t st);

// Each of the first p ordered surfels' distance to its nearest other one.
hipError_t launch_prefix_nn(const float* pts, int64_t n, const int32_t* order, int p, float* out, hipStream_t st);

}  // namespace bs
