// bs_api.cpp -- C ABI of libbluesurfels: argument validation, workspace
// sizing, kernel choice and enqueueing.  See include/bluesurfels.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "bs_grid.h"
#include "bs_internal.h"
#include "bs_sample.h"

namespace bs {

namespace {
struct DeviceInfo {
    int cus = 0;
};
std::mutex g_dev_mu;
DeviceInfo g_dev[64];

int device_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (g_dev[dev].cus == 0) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return 0;
        g_dev[dev].cus = p.multiProcessorCount;
    }
    return g_dev[dev].cus;
}

constexpr int kMaxGridPicks = 32;     // picks per round of the grid kernel
constexpr int kMaxScanPicks = 256;    // picks per step of the cooperative full scan
constexpr int kDefaultGridPicks = 16;

bool tuning_clean(const bs_tuning* t) {
    if (!t) return true;
    for (int r : t->reserved)
        if (r != 0) return false;
    if (t->picks < 0 || t->picks > kMaxScanPicks) return false;
    if (t->lead_picks < -1 || t->batch_wide < -1 || t->spin_limit < 0) return false;
    return t->kernel >= BS_KERNEL_AUTO && t->kernel <= BS_KERNEL_GRID;
}

constexpr float kDefaultCellPoints = 32.f;       // one pick per round
constexpr float kDefaultCellPointsMulti = 8.f;   // several picks per round
constexpr int64_t kAutoResidentMax = 16384;  // one workgroup holds these in VGPRs
// Automatic leading full scan of the grid kernel: from this many candidates,
// for the first n / kAutoLeadDiv picks (while a pick's covering ball still
// holds many candidates, a step over all CUs beats one workgroup's pruned step).
constexpr int64_t kAutoLeadMinN = int64_t(1) << 18;
constexpr int64_t kAutoLeadDiv = 1024;
// Automatic several-picks cooperative scan: at most this many picks per step,
// and only above this many candidates (below, the one resident workgroup is
// as fast: 4,096 in 2.97 ms against 3.12 ms on four workgroups).
constexpr int kAutoScanPicks = 256;
constexpr int64_t kAutoSeveralMin = 4096;

struct Plan {
    int kernel = 0;
    ScanShape shape;     // resident kernels
    int grid_block = 0;  // grid kernel workgroup size
    int grid_picks = kDefaultGridPicks;
    float cell_points = kDefaultCellPoints;
    int lead = 0;          // picks made by a leading cooperative full scan (0: none)
    ScanShape lead_shape;  // its launch shape
    int scan_picks = 1;    // cooperative full scan: most exact picks per step
};

// Shape of the several-picks cooperative scan for n candidates: the most
// workgroups (fewest candidates per thread) that fit one per CU, two at
// least -- every workgroup offers three entries per step, so more workgroups
// accept more picks per step.  The automatic plan takes it from 4,097
// candidates: even a few workgroups beat the one resident workgroup, whose
// step is one pick (16,384 candidates: 5.4 ms on 16 workgroups of 1024 x 1
// against 38 ms).
bool choose_several_shape(int64_t n, int cus, int want_block, int want_pt, int want_groups, ScanShape* out) {
    static const int kBlocks[] = {1024, 512};
    static const int kPer[] = {1, 2, 4, 8, 12, 16, 24, 32};
    for (int b : kBlocks) {
        if (want_block > 0 && b != want_block) continue;
        for (int pt : kPer) {
            if (want_pt > 0 && pt != want_pt) continue;
            ScanShape s;
            if (!choose_scan_shape(n, cus, b, pt, want_groups, &s)) continue;
            if (s.groups >= 2 && s.groups <= cus && scan_several_supported(s)) {
                *out = s;
                return true;
            }
        }
    }
    return false;
}

// Resolve the kernel and its launch shape.
int plan_single(int64_t n, int64_t k, const bs_tuning* t, Plan* p) {
    bs_tuning tuned;
    if (!t) {
        const int f = forced_tuning(&tuned);  // environment override of the automatic choice
        if (f < 0)
            return set_error(BS_ERR_INVALID_ARG, "BS_FORCE_KERNEL=%s is not one of wg, scan, several, grid",
                             std::getenv("BS_FORCE_KERNEL"));
        if (f > 0 || tuned_lookup(n, k, &tuned)) t = &tuned;  // else the autotuner's choice for this size
    }
    const int cus = device_cus() > 0 ? device_cus() : 256;
    const int want = t ? t->kernel : BS_KERNEL_AUTO;
    const int wb = t ? t->block : 0, wp = t ? t->per_thread : 0, wg = t ? t->groups : 0;
    if (want == BS_KERNEL_AUTO && n > kAutoSeveralMin && choose_several_shape(n, cus, wb, wp, wg, &p->shape)) {
        p->kernel = BS_KERNEL_COOP;
        // 256 picks per step where the entries can exceed 128 (three a
        // workgroup); the 128-pick kernel's step is cheaper otherwise
        p->scan_picks = (t && t->picks > 1) ? t->picks : (p->shape.groups >= 64 ? kAutoScanPicks : 128);
        return BS_OK;
    }
    if (want == BS_KERNEL_GRID || (want == BS_KERNEL_AUTO && n > kAutoResidentMax)) {
        p->grid_picks = (t && t->picks > 0) ? t->picks : kDefaultGridPicks;
        if (p->grid_picks > kMaxGridPicks)
            return set_error(BS_ERR_UNSUPPORTED, "grid kernel: at most %d picks per round", kMaxGridPicks);
        const bool multi = p->grid_picks > 1;
        int b = wb > 0 ? wb : (multi ? 1024 : grid_block_size(n));
        if (b != 256 && b != 512 && b != 1024)
            return set_error(BS_ERR_UNSUPPORTED, "grid kernel block must be 256, 512 or 1024, got %d", b);
        p->kernel = BS_KERNEL_GRID;
        p->grid_block = b;
        // several picks per round favour more (smaller) cells: more superblocks
        p->cell_points = (t && t->cell_points > 0.f) ? t->cell_points
                                                      : (multi ? kDefaultCellPointsMulti : kDefaultCellPoints);
        if (p->cell_points < 1.f) p->cell_points = 1.f;
        // leading full scan (several-picks kernel only; needs a cooperative shape)
        const int lp = t ? t->lead_picks : 0;
        int64_t lead = 0;
        if (lp > 0) lead = lp;
        else if (lp == 0 && n >= kAutoLeadMinN) lead = n / kAutoLeadDiv;
        if (lead > k) lead = k;
        if (multi && lead >= 2 && choose_scan_shape(n, cus, 0, 0, 0, &p->lead_shape) &&
            p->lead_shape.groups > 1) {
            p->lead = int(lead);
        } else if (lp > 1 && multi) {
            return set_error(BS_ERR_UNSUPPORTED, "no cooperative scan holds n=%lld for lead_picks", (long long)n);
        }
        return BS_OK;
    }
    if (want == BS_KERNEL_AUTO) {
        if (choose_scan_shape(n, cus, wb, wp, wg, &p->shape)) {
            p->kernel = p->shape.groups > 1 ? BS_KERNEL_COOP : BS_KERNEL_WG;
            return BS_OK;
        }
        return set_error(BS_ERR_UNSUPPORTED, "no kernel holds n=%lld candidates", (long long)n);
    }
    if (want == BS_KERNEL_COOP && t && t->picks > 1) {
        if (!choose_several_shape(n, cus, wb, wp, wg, &p->shape))
            return set_error(BS_ERR_UNSUPPORTED, "no several-picks cooperative scan holds n=%lld with this tuning",
                             (long long)n);
        p->kernel = BS_KERNEL_COOP;
        p->scan_picks = t->picks;
        return BS_OK;
    }
    if (want == BS_KERNEL_WG || want == BS_KERNEL_COOP) {
        if (!choose_scan_shape(n, cus, wb, wp, want == BS_KERNEL_WG ? 1 : wg, &p->shape))
            return set_error(BS_ERR_UNSUPPORTED, "resident kernel cannot hold n=%lld with this tuning",
                             (long long)n);
        if (want == BS_KERNEL_WG && p->shape.groups != 1)
            return set_error(BS_ERR_UNSUPPORTED, "n=%lld does not fit one workgroup", (long long)n);
        if (want == BS_KERNEL_COOP && p->shape.groups > cus * 2)
            return set_error(BS_ERR_UNSUPPORTED, "cooperative grid of %d groups too large", p->shape.groups);
        p->kernel = want;
        return BS_OK;
    }
    return set_error(BS_ERR_UNSUPPORTED, "kernel %d not available", want);
}

size_t workspace_for(int64_t n, const Plan& p) {
    if (p.kernel == BS_KERNEL_GRID) return grid_layout(n, p.grid_block).total;
    if (p.scan_picks > 1) return grid_layout(n, 1024).total;
    return scan_workspace_bytes(p.shape);
}

}  // namespace



}  // namespace bs

using namespace bs;

extern "C" {



int64_t bs_start_index(uint64_t seed, int64_t n) {
    if (n < 1) return -1;
    // first output of SplitMix64 seeded with `seed`
    uint64_t z = seed + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return int64_t(z % uint64_t(n));
}

int bs_auto_kernel(int64_t n, int64_t k) {
    Plan p;
    if (n < 1 || n >= (int64_t(1) << 31)) return -1;
    if (plan_single(n, k, nullptr, &p) != BS_OK) return -1;
    return p.kernel;
}

int bs_plan_describe(int64_t n, int64_t k, const bs_tuning* tuning, bs_tuning* out) {
    if (!out) return set_error(BS_ERR_INVALID_ARG, "null output");
    if (n < 1 || n >= (int64_t(1) << 31) || k < 0 || k > n)
        return set_error(BS_ERR_INVALID_ARG, "n=%lld k=%lld outside 1 <= n < 2^31, 0 <= k <= n", (long long)n,
                         (long long)k);
    if (!tuning_clean(tuning)) return set_error(BS_ERR_INVALID_ARG, "bad tuning struct");
    Plan p;
    const int rc = plan_single(n, k, tuning, &p);
    if (rc != BS_OK) return rc;
    bs_tuning d;
    memset(&d, 0, sizeof(d));
    d.kernel = p.kernel;
    if (p.kernel == BS_KERNEL_GRID) {
        d.block = p.grid_block;
        d.cell_points = p.cell_points;
        d.picks = p.grid_picks;
        d.lead_picks = p.lead > 0 ? p.lead : -1;
        if (p.lead > 0) {
            d.per_thread = p.lead_shape.per_thread;
            d.groups = p.lead_shape.groups;
        }
    } else {
        d.block = p.shape.block;
        d.per_thread = p.shape.per_thread;
        d.groups = p.shape.groups;
        d.picks = p.scan_picks;
    }
    *out = d;
    return BS_OK;
}

int bs_emit_surfels(const float* d_points, const float* d_normals, const uint8_t* d_colors, int64_t n,
                    const int32_t* d_order, int64_t k, bs_surfel* d_out, void* stream) {
    static_assert(sizeof(bs_surfel) == 20, "surfel record size");
    if (k < 0 || n < 0) return set_error(BS_ERR_INVALID_ARG, "n=%lld k=%lld", (long long)n, (long long)k);
    if (k == 0) return BS_OK;
    if (!d_points || !d_order || !d_out) return set_error(BS_ERR_INVALID_ARG, "null points, order or output");
    const hipError_t e = launch_emit(d_points, d_normals, d_colors, n, d_order, k, d_out,
                                     reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "emit launch: %s", hipGetErrorString(e));
    return BS_OK;
}

int bs_prefix_median_nn(const float* d_points, int64_t n, const int32_t* d_order, int64_t p_m, float* d_out_rm,
                        void* stream) {
    if (!d_points || !d_order || !d_out_rm) return set_error(BS_ERR_INVALID_ARG, "null pointer");
    if (p_m < 2 || p_m > kMaxPrefixPm || n < p_m)
        return set_error(BS_ERR_INVALID_ARG, "p_m=%lld outside [2, min(n, %d)]", (long long)p_m, kMaxPrefixPm);
    const hipError_t e = launch_median_nn(d_points, n, d_order, int(p_m), d_out_rm,
                                          reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "median launch: %s", hipGetErrorString(e));
    return BS_OK;
}

int64_t bs_prefix_length(double r, double r_m, int64_t p_m, int64_t k) {
    if (k < 1) return 0;
    if (!(r > 0.0)) return k;
    const double q = r_m / r;
    const double p = std::ceil(double(p_m) * q * q);
    if (!(p >= 1.0)) return 1;
    return p > double(k) ? k : int64_t(p);
}

int64_t bs_prefix_for_radius(const float* h_radius, int64_t k, float r) {
    if (!h_radius || k < 1) return k < 1 ? 0 : k;
    // radii are non-increasing from index 1: binary search for the first <= r
    int64_t lo = 1, hi = k;  // answer in [lo, hi]; hi = k means none
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (h_radius[mid] <= r) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

size_t bs_morton_workspace_size(int64_t n) {
    if (n < 1 || n >= (int64_t(1) << 31)) return 0;
    return grid_layout(n, 1024).total;
}

int bs_morton_order(const float* d_points, int64_t n, int32_t* d_out_perm, void* d_workspace, size_t workspace_bytes,
                    void* stream) {
    if (n < 0 || n >= (int64_t(1) << 31)) return set_error(BS_ERR_INVALID_ARG, "n=%lld outside [0, 2^31)", (long long)n);
    if (n == 0) return BS_OK;
    if (!d_points || !d_out_perm || !d_workspace) return set_error(BS_ERR_INVALID_ARG, "null pointer");
    if (workspace_bytes < bs_morton_workspace_size(n))
        return set_error(BS_ERR_INVALID_ARG, "workspace %zu bytes < %zu needed", workspace_bytes,
                         bs_morton_workspace_size(n));
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
        return set_error(BS_ERR_INVALID_ARG, "workspace not %zu-byte aligned", kAlign);
    const hipError_t e = launch_morton_order(d_points, int(n), d_out_perm, d_workspace,
                                             reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "morton order: %s", hipGetErrorString(e));
    return BS_OK;
}

size_t bs_workspace_size(int64_t n, int64_t k, const bs_tuning* tuning) {
    if (n < 1 || n >= (int64_t(1) << 31) || k < 0 || k > n || !tuning_clean(tuning)) return 0;
    Plan p;
    if (plan_single(n, k, tuning, &p) != BS_OK) return 0;
    return workspace_for(n, p);
}

}  // extern "C"

int bs::order_impl(const float* d_points, int64_t n, int64_t k, uint64_t seed, int64_t start_index,
                   int32_t* d_out_order, float* d_out_radius, uint64_t* d_ticks, const LaunchOpts* ev,
                   void* d_workspace, size_t workspace_bytes, const bs_tuning* tuning, void* stream) {
    if (k < 0) return set_error(BS_ERR_INVALID_ARG, "k=%lld < 0", (long long)k);
    if (k == 0) return BS_OK;
    if (n < 1 || n >= (int64_t(1) << 31))
        return set_error(BS_ERR_INVALID_ARG, "n=%lld outside [1, 2^31)", (long long)n);
    if (k > n) return set_error(BS_ERR_INVALID_ARG, "k=%lld > n=%lld", (long long)k, (long long)n);
    if (!d_points || !d_out_order) return set_error(BS_ERR_INVALID_ARG, "null points or output");
    if (!tuning_clean(tuning)) return set_error(BS_ERR_INVALID_ARG, "bad tuning struct");
    if (start_index < -1 || start_index >= n)
        return set_error(BS_ERR_INVALID_ARG, "start_index=%lld outside [-1, n)", (long long)start_index);
    const int64_t start = start_index >= 0 ? start_index : bs_start_index(seed, n);

    Plan plan;
    int rc = plan_single(n, k, tuning, &plan);
    if (rc != BS_OK) return rc;
    const size_t need = workspace_for(n, plan);
    if (!d_workspace || workspace_bytes < need)
        return set_error(BS_ERR_INVALID_ARG, "workspace %zu bytes < %zu needed", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign != 0)
        return set_error(BS_ERR_INVALID_ARG, "workspace not %zu-byte aligned", kAlign);

    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    LaunchOpts opts = ev ? *ev : LaunchOpts{};
    opts.spin_limit = tuning ? uint32_t(tuning->spin_limit) : 0u;
    ev = &opts;
    hipError_t e = hipSuccess;
    if (plan.kernel == BS_KERNEL_GRID) {
        e = launch_grid(d_points, int(n), int(k), int(start), d_out_order, d_out_radius, d_workspace,
                        plan.cell_points, plan.grid_block, plan.grid_picks, d_ticks, st, ev, plan.lead,
                        plan.lead > 0 ? &plan.lead_shape : nullptr);
    } else if (plan.scan_picks > 1) {
        e = launch_scan_several(plan.shape, d_points, int(n), int(k), int(start), d_out_order, d_out_radius,
                                d_workspace, d_ticks, plan.scan_picks, st, ev);
    } else {
        DevHeader* hdr = reinterpret_cast<DevHeader*>(d_workspace);
        void* scratch = static_cast<char*>(d_workspace) + align_up(sizeof(DevHeader));
        e = launch_init_header(hdr, st);
        if (e == hipSuccess) e = launch_validate(d_points, n, hdr, st);
        if (e == hipSuccess)
            e = launch_scan(plan.shape, d_points, int(n), int(k), int(start), d_out_order, d_out_radius,
                            hdr, scratch, d_ticks, st, ev);
    }
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "launch failed: %s", hipGetErrorString(e));
    return BS_OK;
}

extern "C" {

int bs_order_ex(const float* d_points, const float* d_normals, const uint8_t* d_colors,
                int64_t n, int64_t k, uint64_t seed, int64_t start_index,
                int32_t* d_out_order, float* d_out_radius, void* d_workspace,
                size_t workspace_bytes, const bs_tuning* tuning, void* stream) {
    (void)d_normals;
    (void)d_colors;
    return order_impl(d_points, n, k, seed, start_index, d_out_order, d_out_radius, nullptr, nullptr,
                      d_workspace, workspace_bytes, tuning, stream);
}

int bs_order_profile(const float* d_points, int64_t n, int64_t k, int64_t start_index,
                     int32_t* d_out_order, float* d_out_radius, uint64_t* d_step_ticks,
                     void* event_begin, void* event_end,
                     void* d_workspace, size_t workspace_bytes, const bs_tuning* tuning,
                     void* stream) {
    LaunchOpts ev;
    ev.begin = reinterpret_cast<hipEvent_t>(event_begin);
    ev.end = reinterpret_cast<hipEvent_t>(event_end);
    return order_impl(d_points, n, k, 0, start_index, d_out_order, d_out_radius, d_step_ticks, &ev,
                      d_workspace, workspace_bytes, tuning, stream);
}

int bs_order_status(const void* d_workspace, void* stream) {
    if (!d_workspace) return set_error(BS_ERR_INVALID_ARG, "null workspace");
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "stream: %s", hipGetErrorString(e));
    uint32_t w[2] = {0, 0};  // DevHeader: nonfinite, error (every plan's workspace starts with it)
    e = hipMemcpy(w, d_workspace, sizeof(w), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "reading the workspace header: %s", hipGetErrorString(e));
    if (w[0]) return set_error(BS_ERR_INVALID_ARG, "a candidate coordinate is not finite (outputs -1 / NaN)");
    if (w[1])
        return set_error(BS_ERR_TIMEOUT, "a cooperative kernel's bounded wait gave up (outputs -2 / NaN)");
    return BS_OK;
}

double bs_wall_clock_hz(void) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0.0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0.0;
    return double(khz) * 1000.0;
}

int bs_order(const float* d_points, const float* d_normals, const uint8_t* d_colors, int64_t n,
             int64_t k, uint64_t seed, int32_t* d_out_order, float* d_out_radius, void* stream) {
    if (k < 0) return set_error(BS_ERR_INVALID_ARG, "k=%lld < 0", (long long)k);
    if (k == 0) return BS_OK;
    const size_t need = bs_workspace_size(n, k, nullptr);
    if (need == 0) {
        if (n < 1 || n >= (int64_t(1) << 31) || k > n)
            return set_error(BS_ERR_INVALID_ARG, "bad sizes n=%lld k=%lld", (long long)n, (long long)k);
        return set_error(BS_ERR_UNSUPPORTED, "no kernel for n=%lld", (long long)n);
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, need, st);
    if (e != hipSuccess || !ws) return set_error(BS_ERR_OUT_OF_MEMORY, "workspace of %zu bytes", need);
    int rc = bs_order_ex(d_points, d_normals, d_colors, n, k, seed, -1, d_out_order, d_out_radius,
                         ws, need, nullptr, stream);
    (void)hipFreeAsync(ws, st);
    return rc;
}

int bs_batch_plan_create(const int64_t* h_offsets, const int64_t* h_k, const uint64_t* h_seed,
                         int32_t m, const bs_tuning* tuning, bs_batch_plan** out_plan) {
    if (!out_plan) return set_error(BS_ERR_INVALID_ARG, "null plan pointer");
    *out_plan = nullptr;
    if (!tuning_clean(tuning) || (tuning && tuning->groups < 0)) return set_error(BS_ERR_INVALID_ARG, "bad tuning struct");
    if (tuning && tuning->picks > kMaxGridPicks)
        return set_error(BS_ERR_UNSUPPORTED, "batch plans: at most %d picks per round", kMaxGridPicks);
    const float target = (tuning && tuning->cell_points > 0.f) ? tuning->cell_points : kDefaultCellPointsMulti;
    bs::BatchPlan* p = nullptr;
    int rc = batch_plan_create(h_offsets, h_k, h_seed, m, target, tuning ? tuning->batch_wide : 0,
                               tuning ? tuning->groups : 0, &p);
    if (rc == BS_OK) batch_set_picks(p, tuning ? tuning->picks : 0);
    // bounded cells (same result): on the 1,000-part batch 0.804-0.808 s
    // against 0.811-0.817 s with plain Morton-prefix cells
    if (rc == BS_OK) batch_set_split_cells(p, true);
    if (rc == BS_OK) rc = batch_plan_upload(p);
    if (rc != BS_OK) {
        batch_plan_free(p);
        return rc;
    }
    *out_plan = new bs_batch_plan{p, m};
    return BS_OK;
}

size_t bs_batch_workspace_size(const bs_batch_plan* plan) {
    return plan ? batch_workspace_bytes(plan->p) : 0;
}

int64_t bs_batch_total_k(const bs_batch_plan* plan) { return plan ? batch_total_k(plan->p) : 0; }

int bs_batch_out_offsets(const bs_batch_plan* plan, int64_t* h_out_offsets) {
    if (!plan || !h_out_offsets) return set_error(BS_ERR_INVALID_ARG, "null argument");
    const int64_t* o = batch_out_offsets(plan->p);
    for (int32_t j = 0; j <= plan->m_all; ++j) h_out_offsets[j] = o[j];
    return BS_OK;
}

int bs_batch_plan_execute(bs_batch_plan* plan, const float* d_points, int32_t* d_out_order,
                          float* d_out_radius, void* d_workspace, size_t workspace_bytes,
                          void* stream) {
    if (!plan) return set_error(BS_ERR_INVALID_ARG, "null plan");
    return batch_plan_execute(plan->p, d_points, d_out_order, d_out_radius, d_workspace,
                              workspace_bytes, reinterpret_cast<hipStream_t>(stream));
}

int bs_batch_morton_order(bs_batch_plan* plan, const float* d_points, int32_t* d_out_perm, void* d_workspace,
                          size_t workspace_bytes, void* stream) {
    if (!plan) return set_error(BS_ERR_INVALID_ARG, "null plan");
    return batch_morton_order(plan->p, d_points, d_out_perm, d_workspace, workspace_bytes,
                              reinterpret_cast<hipStream_t>(stream));
}

int bs_batch_plan_execute_sample(bs_batch_plan* plan, const bs_sampler* params, const float* d_points,
                                 int32_t* d_out_order, float* d_out_radius, int32_t* d_out_count,
                                 void* d_workspace, size_t workspace_bytes, void* stream) {
    if (!plan) return set_error(BS_ERR_INVALID_ARG, "null plan");
    if (params)
        for (int r : params->reserved)
            if (r) return set_error(BS_ERR_INVALID_ARG, "sampler: reserved fields must be zero");
    const bs_sampler p = params ? *params : bs_sampler_defaults();
    return batch_plan_execute_sample(plan->p, p.sample_size, p.growth_rounds, p.vicinity, d_points, d_out_order,
                                     d_out_radius, d_out_count, d_workspace, workspace_bytes,
                                     reinterpret_cast<hipStream_t>(stream));
}

void bs_batch_plan_destroy(bs_batch_plan* plan) {
    if (!plan) return;
    batch_plan_free(plan->p);
    delete plan;
}

}  // extern "C"
