// bs_tune.cpp -- autotuner: picks the kernel and its launch shape (workgroup
// size, candidates per thread, grid cell occupancy, picks per round) for an
// ordering problem by timing candidate configurations on the caller's data,
// and keeps the winners in a per-device table that the automatic kernel
// choice consults.  Built on the public entry points only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "bs_internal.h"

namespace bs {

namespace {

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, bs_tuning> g_table;  // (device, log2 n, log2 k) -> tuning

int ilog2(int64_t v) {
    int r = 0;
    while ((int64_t(1) << (r + 1)) <= v) ++r;
    return r;
}

std::tuple<int, int, int> table_key(int dev, int64_t n, int64_t k) {
    return std::make_tuple(dev, ilog2(std::max<int64_t>(n, 1)), ilog2(std::max<int64_t>(k, 1)));
}

bs_tuning make_tuning(int kernel, int block, int per_thread, float cell_points, int picks) {
    bs_tuning t;
    std::memset(&t, 0, sizeof(t));
    t.kernel = kernel;
    t.block = block;
    t.per_thread = per_thread;
    t.cell_points = cell_points;
    t.picks = picks;
    return t;
}

// Configurations worth timing for (n, k).
std::vector<bs_tuning> single_candidates(int64_t n) {
    std::vector<bs_tuning> c;
    if (n <= 16384) {
        c.push_back(make_tuning(BS_KERNEL_WG, 0, 0, 0.f, 0));
        if (n > 4096)
            for (int pt : {1, 2, 4}) c.push_back(make_tuning(BS_KERNEL_COOP, 1024, pt, 0.f, 128));
        for (float cp : {4.f, 8.f}) c.push_back(make_tuning(BS_KERNEL_GRID, 1024, 0, cp, 16));
        c.push_back(make_tuning(BS_KERNEL_GRID, 256, 0, 8.f, 16));
        return c;
    }
    if (n <= 256 * 16384) {
        // several-picks cooperative scan: candidates per thread (more
        // workgroups offer more entries per step), the most picks per step
        // (a lower cap only binds late in the ordering, beyond the prefixes
        // timed here, and is never faster there)
        for (int pt : {1, 2, 4, 8, 12, 16}) c.push_back(make_tuning(BS_KERNEL_COOP, 1024, pt, 0.f, 256));
    }
    for (int block : {512, 1024})
        for (float cp : {8.f, 16.f}) c.push_back(make_tuning(BS_KERNEL_GRID, block, 0, cp, 16));
    return c;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Persistent tuning cache (environment BS_TUNE_CACHE = path of a text file).
// One line per size class and GPU architecture:
//   bluesurfels-tune-v1 <arch> <log2 n> <log2 k> <kernel> <block> <per_thread>
//                       <groups> <cell_points> <picks> <lead_picks> <batch_wide>
// bs_autotune rewrites the file with its winner (replacing the line of the
// same key, through a temporary file and a rename); the automatic choice
// reads it when its in-memory table has no entry.  Malformed lines are
// skipped.
constexpr const char* kCacheTag = "bluesurfels-tune-v1";
using CacheKey = std::tuple<std::string, int, int>;
std::map<CacheKey, bs_tuning> g_cache;  // entries of the loaded file
std::string g_cache_path;               // file g_cache was loaded from ("" = none)
bool g_cache_loaded = false;

std::string device_arch(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return std::string();
    std::string a(p.gcnArchName);
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

bool parse_cache_line(const char* line, CacheKey* key, bs_tuning* t) {
    char tag[32], arch[64];
    int l2n = 0, l2k = 0;
    bs_tuning v;
    std::memset(&v, 0, sizeof(v));
    const int got = std::sscanf(line, "%31s %63s %d %d %d %d %d %d %f %d %d %d", tag, arch, &l2n, &l2k, &v.kernel,
                                &v.block, &v.per_thread, &v.groups, &v.cell_points, &v.picks, &v.lead_picks,
                                &v.batch_wide);
    if (got != 12 || std::strcmp(tag, kCacheTag) != 0) return false;
    if (l2n < 0 || l2n > 31 || l2k < 0 || l2k > 31 || v.kernel < BS_KERNEL_AUTO || v.kernel > BS_KERNEL_GRID ||
        v.block < 0 || v.per_thread < 0 || v.groups < 0 || !(v.cell_points >= 0.f) || v.picks < 0 ||
        v.lead_picks < -1 || v.batch_wide < -1)
        return false;
    *key = CacheKey(arch, l2n, l2k);
    *t = v;
    return true;
}

std::map<CacheKey, bs_tuning> read_cache_file(const std::string& path) {
    std::map<CacheKey, bs_tuning> m;
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return m;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        CacheKey key;
        bs_tuning t;
        if (parse_cache_line(line, &key, &t)) m[key] = t;
    }
    std::fclose(f);
    return m;
}

// caller holds g_tune_mu
void load_cache_locked() {
    const char* env = std::getenv("BS_TUNE_CACHE");
    const std::string path = env ? env : "";
    if (g_cache_loaded && path == g_cache_path) return;
    g_cache = path.empty() ? std::map<CacheKey, bs_tuning>() : read_cache_file(path);
    g_cache_path = path;
    g_cache_loaded = true;
}

// caller holds g_tune_mu; returns false if the file could not be written
bool store_cache_locked(const std::string& arch, int64_t n, int64_t k, const bs_tuning& t) {
    const char* env = std::getenv("BS_TUNE_CACHE");
    if (!env || !*env || arch.empty()) return true;
    const std::string path = env;
    std::map<CacheKey, bs_tuning> m = read_cache_file(path);  // other processes' entries too
    m[CacheKey(arch, ilog2(std::max<int64_t>(n, 1)), ilog2(std::max<int64_t>(k, 1)))] = t;
    const std::string tmp = path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    bool ok = true;
    for (const auto& kv : m) {
        const bs_tuning& v = kv.second;
        ok = ok && std::fprintf(f, "%s %s %d %d %d %d %d %d %.9g %d %d %d\n", kCacheTag,
                                std::get<0>(kv.first).c_str(), std::get<1>(kv.first), std::get<2>(kv.first),
                                v.kernel, v.block, v.per_thread, v.groups, double(v.cell_points), v.picks,
                                v.lead_picks, v.batch_wide) > 0;
    }
    ok = (std::fclose(f) == 0) && ok;
    if (ok) ok = std::rename(tmp.c_str(), path.c_str()) == 0;
    if (!ok) std::remove(tmp.c_str());
    g_cache = m;
    g_cache_path = path;
    g_cache_loaded = true;
    return ok;
}

}  // namespace

bool tuned_lookup(int64_t n, int64_t k, bs_tuning* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_table.find(table_key(dev, n, k));
    if (it != g_table.end()) {
        *out = it->second;
        return true;
    }
    load_cache_locked();
    if (g_cache.empty()) return false;
    auto c = g_cache.find(CacheKey(device_arch(dev), ilog2(std::max<int64_t>(n, 1)), ilog2(std::max<int64_t>(k, 1))));
    if (c == g_cache.end()) return false;
    *out = c->second;
    return true;
}

// Environment BS_FORCE_KERNEL overrides the automatic choice (callers that
// pass no tuning): "wg" one resident workgroup, "scan" the cooperative full
// scan with one pick per step, "several" the cooperative scan with several
// exact picks per step, "grid" the grid-pruned kernel.  Returns 0 when unset,
// 1 with *out filled, -1 for an unknown value.
int forced_tuning(bs_tuning* out) {
    const char* env = std::getenv("BS_FORCE_KERNEL");
    if (!env || !*env) return 0;
    const std::string v = env;
    if (v == "wg") *out = make_tuning(BS_KERNEL_WG, 0, 0, 0.f, 0);
    else if (v == "scan") *out = make_tuning(BS_KERNEL_COOP, 0, 0, 0.f, 1);
    else if (v == "several") *out = make_tuning(BS_KERNEL_COOP, 1024, 0, 0.f, 256);
    else if (v == "grid") *out = make_tuning(BS_KERNEL_GRID, 0, 0, 0.f, 0);
    else return -1;
    return 1;
}

}  // namespace bs

using namespace bs;

extern "C" int bs_autotune(const float* d_points, int64_t n, int64_t k, uint64_t seed,
                           bs_tuning* out_tuning, void* stream) {
    if (!d_points || !out_tuning) return set_error(BS_ERR_INVALID_ARG, "null points or output tuning");
    if (n < 1 || n >= (int64_t(1) << 31) || k < 1 || k > n)
        return set_error(BS_ERR_INVALID_ARG, "autotune needs 1 <= k <= n < 2^31 (n=%lld k=%lld)",
                         (long long)n, (long long)k);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // two prefixes of the ordering; the cost of the whole ordering is
    // extrapolated from the second with the per-pick cost between them (the
    // early, wide steps cost more per pick than the later ones)
    const int64_t kp = std::min<int64_t>(k, std::max<int64_t>(1024, k / 8));
    const int64_t k1 = std::min<int64_t>(kp, std::max<int64_t>(512, k / 16));
    const std::vector<bs_tuning> cand = single_candidates(n);
    size_t ws_bytes = 0;
    for (const bs_tuning& t : cand) ws_bytes = std::max(ws_bytes, bs_workspace_size(n, kp, &t));
    if (ws_bytes == 0) return set_error(BS_ERR_UNSUPPORTED, "no candidate configuration for n=%lld", (long long)n);
    void* ws = nullptr;
    void* outo = nullptr;
    void* outr = nullptr;
    hipError_t e = hipMallocAsync(&ws, ws_bytes, st);
    if (e == hipSuccess) e = hipMallocAsync(&outo, size_t(kp) * 4, st);
    if (e == hipSuccess) e = hipMallocAsync(&outr, size_t(kp) * 4, st);
    if (e != hipSuccess) {
        if (ws) (void)hipFreeAsync(ws, st);
        if (outo) (void)hipFreeAsync(outo, st);
        return set_error(BS_ERR_OUT_OF_MEMORY, "autotune scratch: %s", hipGetErrorString(e));
    }
    Timer tm;
    float best_ms = INFINITY;
    bs_tuning best = cand[0];
    int rc = BS_OK;
    for (const bs_tuning& t : cand) {
        const size_t need = bs_workspace_size(n, kp, &t);
        if (need == 0) continue;  // does not hold n candidates
        // warm-up on a short prefix (module load, caches), then the timed prefixes
        int r = bs_order_ex(d_points, nullptr, nullptr, n, std::min<int64_t>(kp, 64), seed, -1,
                            static_cast<int32_t*>(outo), static_cast<float*>(outr), ws, need, &t, stream);
        if (r != BS_OK) continue;
        float ms[2] = {0.f, 0.f};
        const int64_t kk[2] = {k1, kp};
        for (int i = 0; i < 2 && r == BS_OK; ++i) {
            (void)hipEventRecord(tm.a, st);
            r = bs_order_ex(d_points, nullptr, nullptr, n, kk[i], seed, -1, static_cast<int32_t*>(outo),
                            static_cast<float*>(outr), ws, need, &t, stream);
            (void)hipEventRecord(tm.b, st);
            if (hipEventSynchronize(tm.b) != hipSuccess) {
                rc = set_error(BS_ERR_HIP, "autotune: device error while timing");
                break;
            }
            (void)hipEventElapsedTime(&ms[i], tm.a, tm.b);
        }
        if (rc != BS_OK) break;
        if (r != BS_OK) continue;
        float est = ms[1];
        if (k > kp && kp > k1) est += std::max(0.f, ms[1] - ms[0]) * float(k - kp) / float(kp - k1);
        if (est < best_ms) {
            best_ms = est;
            best = t;
        }
    }
    (void)hipFreeAsync(ws, st);
    (void)hipFreeAsync(outo, st);
    (void)hipFreeAsync(outr, st);
    if (rc != BS_OK) return rc;
    if (!std::isfinite(best_ms)) return set_error(BS_ERR_UNSUPPORTED, "autotune: no configuration ran");
    int dev = 0;
    (void)hipGetDevice(&dev);
    const std::string arch = device_arch(dev);
    bool stored = true;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_table[table_key(dev, n, k)] = best;
        stored = store_cache_locked(arch, n, k, best);
    }
    *out_tuning = best;
    if (!stored) return set_error(BS_ERR_INVALID_ARG, "autotune: could not write the tuning cache %s",
                                  std::getenv("BS_TUNE_CACHE"));
    return BS_OK;
}

extern "C" int bs_autotune_lookup(int64_t n, int64_t k, bs_tuning* out_tuning) {
    if (!out_tuning) return set_error(BS_ERR_INVALID_ARG, "null output tuning");
    if (!tuned_lookup(n, k, out_tuning)) return BS_ERR_NOT_READY;
    return BS_OK;
}

extern "C" void bs_autotune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_table.clear();
    g_cache.clear();
    g_cache_loaded = false;  // the next lookup reads the cache file again
}

// Batches up to this many picks in all are timed whole when choosing the
// share of the wide workgroups (about a second each at 7.4e7 picks).
constexpr int64_t kFullBatchTuneK = int64_t(1) << 27;

extern "C" int bs_batch_autotune(const int64_t* h_offsets, const int64_t* h_k, const uint64_t* h_seed,
                                 int32_t m, const float* d_points, bs_tuning* out_tuning, void* stream) {
    if (!out_tuning || !d_points || m < 1 || !h_offsets || !h_k)
        return set_error(BS_ERR_INVALID_ARG, "null batch autotune arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // sample: the largest objects by k (they set the makespan) and a spread
    // over the rest, each cut to a prefix of at most 4096 picks
    std::vector<int> idx(m);
    for (int i = 0; i < m; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return h_k[a] > h_k[b]; });
    std::vector<int> pick;
    for (int i = 0; i < m && i < 4; ++i) pick.push_back(idx[i]);
    for (int q = 1; q <= 12 && m > 4; ++q) pick.push_back(idx[std::min<int64_t>(m - 1, 4 + int64_t(q) * (m - 4) / 13)]);
    std::sort(pick.begin(), pick.end());
    pick.erase(std::unique(pick.begin(), pick.end()), pick.end());
    std::vector<int64_t> offs(1, 0), ks;
    std::vector<uint64_t> seeds;
    for (int j : pick) {
        const int64_t nj = h_offsets[j + 1] - h_offsets[j];
        if (nj < 0) return set_error(BS_ERR_INVALID_ARG, "offsets must be non-decreasing");
        offs.push_back(offs.back() + nj);
        ks.push_back(std::min<int64_t>(std::max<int64_t>(h_k[j], 0), std::min<int64_t>(nj, 4096)));
        seeds.push_back(h_seed ? h_seed[j] : 0);
    }
    const int64_t N = offs.back();
    if (N < 1 || N >= (int64_t(1) << 31)) return set_error(BS_ERR_INVALID_ARG, "bad sample size");
    float* sp = nullptr;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&sp), size_t(N) * 12, st);
    if (e != hipSuccess) return set_error(BS_ERR_OUT_OF_MEMORY, "autotune sample: %s", hipGetErrorString(e));
    for (size_t i = 0; e == hipSuccess && i < pick.size(); ++i) {
        const int j = pick[i];
        const size_t bytes = size_t(offs[i + 1] - offs[i]) * 12;
        if (bytes)
            e = hipMemcpyAsync(sp + 3 * offs[i], d_points + 3 * h_offsets[j], bytes, hipMemcpyDeviceToDevice, st);
    }
    int64_t total_k = 0;
    for (int64_t kk : ks) total_k += kk;
    void* outo = nullptr;
    void* outr = nullptr;
    if (e == hipSuccess) e = hipMallocAsync(&outo, size_t(std::max<int64_t>(total_k, 1)) * 4, st);
    if (e == hipSuccess) e = hipMallocAsync(&outr, size_t(std::max<int64_t>(total_k, 1)) * 4, st);
    Timer tm;
    float best_ms = INFINITY;
    float best_cp = 8.f;
    int rc = e == hipSuccess ? BS_OK : set_error(BS_ERR_HIP, "autotune sample copy: %s", hipGetErrorString(e));
    for (float cp : {4.f, 8.f, 16.f, 32.f}) {
        if (rc != BS_OK) break;
        bs_tuning t = make_tuning(BS_KERNEL_GRID, 0, 0, cp, 0);
        bs_batch_plan* plan = nullptr;
        if (bs_batch_plan_create(offs.data(), ks.data(), seeds.data(), int32_t(ks.size()), &t, &plan) != BS_OK)
            continue;
        const size_t wsb = bs_batch_workspace_size(plan);
        void* ws = nullptr;
        if (hipMallocAsync(&ws, std::max<size_t>(wsb, 256), st) != hipSuccess) {
            bs_batch_plan_destroy(plan);
            continue;
        }
        int r = bs_batch_plan_execute(plan, sp, static_cast<int32_t*>(outo), static_cast<float*>(outr), ws, wsb,
                                      stream);  // warm (captures the graph)
        // the sample runs for milliseconds: the fastest of three runs
        float ms = INFINITY;
        for (int rep = 0; rep < 3 && r == BS_OK && rc == BS_OK; ++rep) {
            (void)hipEventRecord(tm.a, st);
            r = bs_batch_plan_execute(plan, sp, static_cast<int32_t*>(outo), static_cast<float*>(outr), ws, wsb,
                                      stream);
            (void)hipEventRecord(tm.b, st);
            if (hipEventSynchronize(tm.b) != hipSuccess) rc = set_error(BS_ERR_HIP, "autotune: device error");
            float one = 0.f;
            if (r == BS_OK && rc == BS_OK && hipEventElapsedTime(&one, tm.a, tm.b) == hipSuccess) ms = std::min(ms, one);
        }
        (void)hipFreeAsync(ws, st);
        bs_batch_plan_destroy(plan);
        if (r != BS_OK || rc != BS_OK) continue;
        if (ms < best_ms) {
            best_ms = ms;
            best_cp = cp;
        }
    }
    (void)hipFreeAsync(sp, st);
    if (outo) (void)hipFreeAsync(outo, st);
    if (outr) (void)hipFreeAsync(outr, st);
    (void)hipStreamSynchronize(st);
    if (rc != BS_OK) return rc;
    if (!std::isfinite(best_ms)) return set_error(BS_ERR_UNSUPPORTED, "batch autotune: no configuration ran");
    bs_tuning best = make_tuning(BS_KERNEL_GRID, 0, 0, best_cp, 0);
    // The compute units given to the 1024-thread workgroups of the longest
    // chains against the 256-thread ones: that balance is a property of the
    // whole batch (a sample keeps the longest chain but not the total work),
    // so the whole batch is ordered once per candidate share, when it has
    // such chains and is small enough to time.
    int64_t full_k = 0;
    for (int j = 0; j < m; ++j) full_k += std::max<int64_t>(h_k[j], 0);
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    bs_batch_plan* probe = nullptr;
    if (cus >= 8 && full_k <= kFullBatchTuneK &&
        bs_batch_plan_create(h_offsets, h_k, h_seed, m, &best, &probe) == BS_OK) {
        const bool has_wide = batch_wide_count(probe->p) > 0;
        const size_t wsb = bs_batch_workspace_size(probe);
        bs_batch_plan_destroy(probe);
        void* ws = nullptr;
        outo = outr = nullptr;
        hipError_t ea = hipSuccess;
        if (has_wide) {
            ea = hipMallocAsync(&ws, std::max<size_t>(wsb, 256), st);
            if (ea == hipSuccess) ea = hipMallocAsync(&outo, size_t(std::max<int64_t>(full_k, 1)) * 4, st);
            if (ea == hipSuccess) ea = hipMallocAsync(&outr, size_t(std::max<int64_t>(full_k, 1)) * 4, st);
        }
        float best_full = INFINITY;
        for (int eighths = 4; has_wide && ea == hipSuccess && eighths <= 7; ++eighths) {
            bs_tuning t = best;
            t.groups = cus * eighths / 8;
            bs_batch_plan* plan = nullptr;
            if (bs_batch_plan_create(h_offsets, h_k, h_seed, m, &t, &plan) != BS_OK) continue;
            int r = bs_batch_plan_execute(plan, d_points, static_cast<int32_t*>(outo), static_cast<float*>(outr),
                                          ws, wsb, stream);  // warm (captures the graph)
            float ms = INFINITY;
            if (r == BS_OK) {
                (void)hipEventRecord(tm.a, st);
                r = bs_batch_plan_execute(plan, d_points, static_cast<int32_t*>(outo), static_cast<float*>(outr),
                                          ws, wsb, stream);
                (void)hipEventRecord(tm.b, st);
                if (hipEventSynchronize(tm.b) != hipSuccess) rc = set_error(BS_ERR_HIP, "autotune: device error");
                if (r == BS_OK && rc == BS_OK && hipEventElapsedTime(&ms, tm.a, tm.b) != hipSuccess) ms = INFINITY;
            }
            bs_batch_plan_destroy(plan);
            if (rc != BS_OK) break;
            if (ms < best_full) {
                best_full = ms;
                best.groups = t.groups;
            }
        }
        if (ws) (void)hipFreeAsync(ws, st);
        if (outo) (void)hipFreeAsync(outo, st);
        if (outr) (void)hipFreeAsync(outr, st);
        (void)hipStreamSynchronize(st);
        if (rc != BS_OK) return rc;
    }
    *out_tuning = best;
    return BS_OK;
}
