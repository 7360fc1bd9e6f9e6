// bs_noalloc.hip -- bs_order_noalloc: the ordering of bs_order_ex for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The workspace is a file-scope device array of kNoAllocScratchBytes, one
// copy per GPU, held from module load to process exit.  Host code never
// passes the array's name to a kernel (in host code it names a host-side
// stand-in): on a device's first call the array's device address is looked
// up with hipGetSymbolAddress, with that device current, and kept per
// device; that address is the workspace every later call on the device uses.
// Every call on a GPU shares the array, so calls that overlap on one GPU
// race (they must be ordered, e.g. on one stream).  The array keeps the last
// call's contents; the launchers initialise what must start cleared (the
// header, the exchange records) on every call.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bs_internal.h"

namespace bs {
namespace {

// 64 MiB: the several-picks scan's workspace (about 109 bytes per candidate)
// up to 524,288 candidates.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The array's device address on the current device (looked up once per device).
int scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return set_error(BS_ERR_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(BS_ERR_HIP, "scratch address on device %d: %s", dev, hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return BS_OK;
}

}  // namespace
}  // namespace bs

using namespace bs;

extern "C" {

size_t bs_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int bs_order_noalloc(const float* d_points, int64_t n, int64_t k, uint64_t seed, int64_t start_index,
                     int32_t* d_out_order, float* d_out_radius, const bs_tuning* tuning, void* stream) {
    if (k == 0 && n >= 0) return BS_OK;
    const size_t need = bs_workspace_size(n, k, tuning);
    if (need == 0)  // order_impl reports which argument is wrong
        return order_impl(d_points, n, k, seed, start_index, d_out_order, d_out_radius, nullptr, nullptr,
                          nullptr, 0, tuning, stream);
    if (need > kNoAllocScratchBytes)
        return set_error(BS_ERR_UNSUPPORTED,
                         "n=%lld k=%lld needs a %zu-byte workspace; the no-allocation entry holds %zu bytes "
                         "(the several-picks scan up to 524,288 candidates)",
                         (long long)n, (long long)k, need, kNoAllocScratchBytes);
    void* ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != BS_OK) return rc;
    return order_impl(d_points, n, k, seed, start_index, d_out_order, d_out_radius, nullptr, nullptr, ws,
                      kNoAllocScratchBytes, tuning, stream);
}

}  // extern "C"
