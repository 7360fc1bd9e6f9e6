// bs_sample_api.cpp -- C ABI of the randomized progressive sampler (paper
// Sec. 3.2) and of the prefix nearest-neighbour measure (Sec. 3.3).  See
// include/bluesurfels.h.
#include <hip/hip_runtime.h>

#include "bs_grid.h"
#include "bs_internal.h"
#include "bs_sample.h"

namespace bs {
namespace {

constexpr int kSamplerMaxSlots = 256;     // one slot per thread of a 256-thread workgroup
constexpr float kSamplerCellPoints = 16.f;
constexpr int kPrefixNnMax = 1 << 20;

int check_params(const bs_sampler* s) {
    if (!s) return BS_OK;
    for (int r : s->reserved)
        if (r) return set_error(BS_ERR_INVALID_ARG, "sampler: reserved fields must be zero");
    if (s->sample_size < 0 || s->sample_size > kSamplerMaxSlots)
        return set_error(BS_ERR_INVALID_ARG, "sampler: sample_size %d outside 0..%d", s->sample_size,
                         kSamplerMaxSlots);
    if (s->growth_rounds == 0) return set_error(BS_ERR_INVALID_ARG, "sampler: growth_rounds must be >= 1 or < 0");
    if (!(s->vicinity >= 0.f) || s->vicinity > 1e18f)
        return set_error(BS_ERR_INVALID_ARG, "sampler: vicinity must be finite and >= 0");
    if (s->sample_size == 0 && s->vicinity > 0.f)
        return set_error(BS_ERR_INVALID_ARG, "sampler: vicinity removal needs a sample (sample_size > 0)");
    return BS_OK;
}

bs_sampler params_or_defaults(const bs_sampler* s) { return s ? *s : bs_sampler_defaults(); }

}  // namespace
}  // namespace bs

using namespace bs;

extern "C" {

bs_sampler bs_sampler_defaults(void) {
    bs_sampler s{};
    s.sample_size = 200;
    s.growth_rounds = 500;
    s.vicinity = 0.f;
    return s;
}

size_t bs_sample_workspace_size(int64_t n) {
    if (n < 1 || n >= (int64_t(1) << 31)) return 0;
    return grid_layout(n, 1024).total;
}

int bs_sample(const float* d_points, int64_t n, int64_t k, uint64_t seed, int64_t start_index,
              const bs_sampler* params, int32_t* d_out_order, float* d_out_radius, int32_t* d_out_count,
              void* d_workspace, size_t workspace_bytes, void* stream) {
    int rc = check_params(params);
    if (rc != BS_OK) return rc;
    if (k < 0) return set_error(BS_ERR_INVALID_ARG, "k=%lld < 0", (long long)k);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (k == 0) return BS_OK;  // nothing enqueued, the count is not written
    if (n < 1 || n >= (int64_t(1) << 31))
        return set_error(BS_ERR_INVALID_ARG, "n=%lld outside [1, 2^31)", (long long)n);
    if (k > n) return set_error(BS_ERR_INVALID_ARG, "k=%lld > n=%lld", (long long)k, (long long)n);
    if (!d_points || !d_out_order) return set_error(BS_ERR_INVALID_ARG, "null points or output");
    if (start_index < -1 || start_index >= n)
        return set_error(BS_ERR_INVALID_ARG, "start_index=%lld outside [-1, n)", (long long)start_index);
    const size_t need = bs_sample_workspace_size(n);
    if (!d_workspace || workspace_bytes < need)
        return set_error(BS_ERR_INVALID_ARG, "workspace %zu bytes < %zu needed", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign != 0)
        return set_error(BS_ERR_INVALID_ARG, "workspace not %zu-byte aligned", kAlign);
    const bs_sampler p = params_or_defaults(params);
    const int64_t start = start_index >= 0 ? start_index : bs_start_index(seed, n);
    const hipError_t e = launch_grid_sample(d_points, int(n), int(k), int(start), seed, p.sample_size,
                                            p.growth_rounds, p.vicinity, d_out_order, d_out_radius, d_out_count,
                                            d_workspace, kSamplerCellPoints, nullptr, st, nullptr);
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "sampler launch: %s", hipGetErrorString(e));
    return BS_OK;
}

int bs_prefix_nn(const float* d_points, int64_t n, const int32_t* d_order, int64_t p, float* d_out, void* stream) {
    if (!d_points || !d_order || !d_out) return set_error(BS_ERR_INVALID_ARG, "null pointer");
    if (p < 1 || p > kPrefixNnMax || n < p)
        return set_error(BS_ERR_INVALID_ARG, "p=%lld outside [1, min(n, %d)]", (long long)p, kPrefixNnMax);
    const hipError_t e = launch_prefix_nn(d_points, n, d_order, int(p), d_out, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "prefix nn launch: %s", hipGetErrorString(e));
    return BS_OK;
}

}  // extern "C"
