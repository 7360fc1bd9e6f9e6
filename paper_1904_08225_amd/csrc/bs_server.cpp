// bs_server.cpp -- serving loop with continuous batching under an HBM budget.
//
// Requests (ordering jobs of any size) are submitted from any host thread.
// A dispatcher thread admits pending jobs, in arrival order, into
// micro-batches whenever an in-flight slot (a stream) is free and the HBM
// budget allows; jobs that arrive while others run are admitted as slots
// and memory free up, and several micro-batches run on the device at the
// same time on different streams.  Each micro-batch copies its jobs'
// candidates into one staging buffer, runs the batched grid ordering (one
// workgroup per job, largest k first) straight into each job's own output
// buffers, and every job sets its own completion flag in pinned host
// memory, so a job's latency does not wait for the rest of its batch.
// Results are bit-identical to ordering each job alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bs_internal.h"

namespace bs {
namespace {

using Clock = std::chrono::steady_clock;

struct Job {
    uint64_t ticket;
    bs_job req;
    Clock::time_point submitted;
    Clock::time_point done_at;
    int flag_slot = -1;
    bool done = false;
    int status = BS_OK;
};

struct InFlight {
    int stream_index;
    bool long_jobs = false;
    BatchPlan* plan = nullptr;
    void* staging = nullptr;
    void* ws = nullptr;
    size_t bytes = 0;
    hipEvent_t finished = nullptr;
    std::vector<uint64_t> tickets;
};

}  // namespace

struct Server {
    bs_server_config cfg{};
    int device = 0;
    std::vector<hipStream_t> streams;
    std::vector<bool> stream_busy;
    uint32_t* flags = nullptr;       // pinned host, one per in-flight job slot
    uint32_t* d_flags = nullptr;     // device alias of flags
    int flag_cap = 0;
    std::vector<int> free_flags;

    std::mutex mu;
    std::condition_variable cv_work;   // dispatcher wake-up
    std::condition_variable cv_done;   // waiters
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Job> jobs;
    std::vector<InFlight> inflight;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread thread;

    // statistics
    int64_t submitted = 0, admitted = 0, completed = 0, rejected = 0, batches = 0;
    int64_t k_done = 0;
    size_t bytes_in_use = 0, bytes_peak = 0;
    std::vector<double> latencies_us;
    Clock::time_point t_first_submit{}, t_last_done{};
    bool any_submit = false;
    int last_error = BS_OK;
};

namespace {

// Lower bound of a job's device footprint (staging + grid preprocessing);
// admission itself uses the exact bytes of the micro-batch's plan.
size_t job_bytes_estimate(int64_t n, int64_t k) {
    (void)k;
    return size_t(n) * 64;
}

// Jobs of very different lengths are not mixed in one micro-batch: a batch
// holds its stream until its longest job ends.  Long jobs (k >= kLongK) may
// occupy at most half of the streams, so short jobs always find one.
constexpr int64_t kLongK = 32768;

bool is_long(const Job& j) { return j.req.k >= kLongK; }

// Launch one micro-batch on stream si (caller holds mu).  Takes, in arrival
// order, pending jobs of the oldest admissible job's length class.
bool launch_batch(Server& s, int si, int long_streams_busy) {
    std::vector<uint64_t> take;
    size_t bytes = 0;
    int64_t total_n = 0;
    const size_t budget = s.cfg.hbm_budget_bytes;
    const int max_long = std::max(1, int(s.streams.size()) / 2);
    int cls = -1;
    for (auto it = s.pending.begin(); it != s.pending.end();) {
        if (int(take.size()) >= s.cfg.max_jobs_per_batch || int(take.size()) >= int(s.free_flags.size())) break;
        const Job& j = s.jobs[*it];
        const int c = is_long(j) ? 1 : 0;
        if (cls < 0) {
            if (c == 1 && long_streams_busy >= max_long) {
                ++it;  // no stream for another long batch: look for short jobs
                continue;
            }
            cls = c;
        }
        if (c != cls) {
            ++it;
            continue;
        }
        const size_t b = job_bytes_estimate(j.req.n, j.req.k);
        if (s.bytes_in_use + bytes + b > budget) break;  // waits until memory frees up
        bytes += b;
        total_n += j.req.n;
        take.push_back(*it);
        it = s.pending.erase(it);
    }
    if (take.empty()) return false;

    std::vector<int64_t> offs(take.size() + 1, 0), ks(take.size());
    std::vector<uint64_t> seeds(take.size());
    std::vector<int32_t*> outo(take.size());
    std::vector<float*> outr(take.size());
    std::vector<uint32_t*> done(take.size());
    for (size_t i = 0; i < take.size(); ++i) {
        Job& j = s.jobs[take[i]];
        offs[i + 1] = offs[i] + j.req.n;
        ks[i] = j.req.k;
        seeds[i] = j.req.seed;
        outo[i] = j.req.d_out_order;
        outr[i] = j.req.d_out_radius;
        j.flag_slot = s.free_flags.back();
        s.free_flags.pop_back();
        s.flags[j.flag_slot] = 0u;
        done[i] = s.d_flags + j.flag_slot;
    }
    InFlight f;
    f.stream_index = si;
    hipStream_t st = s.streams[si];
    int rc = BS_OK;
    // admission on the exact bytes of the plan: give back jobs from the tail
    // of this batch until it fits the remaining budget
    while (true) {
        if (f.plan) {
            batch_plan_free(f.plan);
            f.plan = nullptr;
        }
        rc = batch_plan_create(offs.data(), ks.data(), seeds.data(), int32_t(take.size()),
                               s.cfg.cell_points > 0.f ? s.cfg.cell_points : 8.f, &f.plan);
        if (rc != BS_OK) break;
        total_n = offs[take.size()];
        f.bytes = batch_workspace_bytes(f.plan) + align_up(size_t(total_n) * 12);
        if (s.bytes_in_use + f.bytes <= budget) break;
        if (take.size() == 1) {
            batch_plan_free(f.plan);
            f.plan = nullptr;
            Job& j = s.jobs[take[0]];
            s.free_flags.push_back(j.flag_slot);
            j.flag_slot = -1;
            if (!s.inflight.empty()) {  // wait for memory to free up
                s.pending.insert(std::lower_bound(s.pending.begin(), s.pending.end(), take[0]), take[0]);
                return false;
            }
            j.done = true;  // can never fit
            j.status = BS_ERR_OVER_BUDGET;
            j.done_at = Clock::now();
            s.rejected += 1;
            s.cv_done.notify_all();
            return true;
        }
        Job& last = s.jobs[take.back()];
        s.free_flags.push_back(last.flag_slot);
        last.flag_slot = -1;
        s.pending.insert(std::lower_bound(s.pending.begin(), s.pending.end(), take.back()), take.back());
        take.pop_back();
        offs.resize(take.size() + 1);
        ks.resize(take.size());
        seeds.resize(take.size());
        outo.resize(take.size());
        outr.resize(take.size());
        done.resize(take.size());
    }
    f.tickets = take;
    hipError_t e = hipSuccess;
    if (rc == BS_OK) {
        batch_set_job_io(f.plan, outo, outr, done);
        e = hipMallocAsync(&f.staging, std::max<size_t>(size_t(total_n) * 12, 16), st);
        if (e == hipSuccess) e = hipMallocAsync(&f.ws, std::max<size_t>(batch_workspace_bytes(f.plan), 256), st);
        for (size_t i = 0; e == hipSuccess && i < take.size(); ++i) {
            const Job& j = s.jobs[take[i]];
            if (j.req.n > 0)
                e = hipMemcpyAsync(static_cast<char*>(f.staging) + size_t(offs[i]) * 12, j.req.d_points,
                                   size_t(j.req.n) * 12, hipMemcpyDeviceToDevice, st);
        }
        if (e == hipSuccess) {
            rc = batch_plan_execute(f.plan, static_cast<const float*>(f.staging), nullptr, nullptr, f.ws,
                                    batch_workspace_bytes(f.plan), st);
        } else {
            rc = BS_ERR_HIP;
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&f.finished, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(f.finished, st);
        if (f.staging) (void)hipFreeAsync(f.staging, st);
        if (f.ws) (void)hipFreeAsync(f.ws, st);
        if (e != hipSuccess && rc == BS_OK) rc = BS_ERR_HIP;
    }
    if (rc != BS_OK) {
        // fail the jobs of this batch; nothing of it is pending on the device
        if (f.finished) (void)hipEventSynchronize(f.finished);
        for (uint64_t t : take) {
            Job& j = s.jobs[t];
            j.done = true;
            j.status = rc;
            j.done_at = Clock::now();
            s.free_flags.push_back(j.flag_slot);
        }
        if (f.plan) batch_plan_free(f.plan);
        if (f.finished) (void)hipEventDestroy(f.finished);
        s.last_error = rc;
        s.cv_done.notify_all();
        return true;
    }
    f.long_jobs = is_long(s.jobs[take[0]]);
    s.bytes_in_use += f.bytes;
    s.bytes_peak = std::max(s.bytes_peak, s.bytes_in_use);
    s.admitted += int64_t(take.size());
    s.batches += 1;
    s.stream_busy[si] = true;
    s.inflight.push_back(std::move(f));
    return true;
}

// Record finished jobs and retire finished batches (caller holds mu).
bool reap(Server& s) {
    bool any = false;
    const auto now = Clock::now();
    for (size_t b = 0; b < s.inflight.size();) {
        InFlight& f = s.inflight[b];
        for (uint64_t t : f.tickets) {
            Job& j = s.jobs[t];
            if (!j.done && __atomic_load_n(&s.flags[j.flag_slot], __ATOMIC_ACQUIRE) != 0u) {
                j.done = true;
                j.done_at = now;
                s.completed += 1;
                s.k_done += j.req.k;
                s.latencies_us.push_back(
                    std::chrono::duration<double, std::micro>(j.done_at - j.submitted).count());
                s.t_last_done = now;
                any = true;
            }
        }
        if (hipEventQuery(f.finished) == hipSuccess) {
            for (uint64_t t : f.tickets) {
                Job& j = s.jobs[t];
                if (!j.done) {  // flag not seen (k = 0 jobs also set it): count it now
                    j.done = true;
                    j.done_at = now;
                    s.completed += 1;
                    s.k_done += j.req.k;
                    s.latencies_us.push_back(
                        std::chrono::duration<double, std::micro>(j.done_at - j.submitted).count());
                    s.t_last_done = now;
                }
                s.free_flags.push_back(j.flag_slot);
                j.flag_slot = -1;
            }
            s.bytes_in_use -= f.bytes;
            s.stream_busy[f.stream_index] = false;
            batch_plan_free(f.plan);
            (void)hipEventDestroy(f.finished);
            s.inflight.erase(s.inflight.begin() + long(b));
            any = true;
            continue;
        }
        ++b;
    }
    if (any) s.cv_done.notify_all();
    return any;
}

void dispatcher(Server* sp) {
    Server& s = *sp;
    (void)hipSetDevice(s.device);
    std::unique_lock<std::mutex> lk(s.mu);
    while (true) {
        reap(s);
        // admit while a stream is free and pending jobs fit
        bool launched = true;
        while (launched && !s.pending.empty()) {
            launched = false;
            int long_busy = 0;
            for (const InFlight& f : s.inflight) long_busy += f.long_jobs ? 1 : 0;
            for (size_t si = 0; si < s.streams.size(); ++si) {
                if (!s.stream_busy[si]) {
                    launched = launch_batch(s, int(si), long_busy);
                    break;
                }
            }
        }
        if (s.stop && s.pending.empty() && s.inflight.empty()) break;
        if (s.inflight.empty() && s.pending.empty())
            s.cv_work.wait_for(lk, std::chrono::milliseconds(5));
        else
            s.cv_work.wait_for(lk, std::chrono::microseconds(s.cfg.poll_us > 0 ? s.cfg.poll_us : 50));
    }
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * double(v.size() - 1);
    const size_t i = size_t(pos);
    const double f = pos - double(i);
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace
}  // namespace bs

using namespace bs;

extern "C" {

struct bs_server {
    bs::Server* s;
};

int bs_server_create(const bs_server_config* cfg, bs_server** out) {
    if (!out || !cfg) return set_error(BS_ERR_INVALID_ARG, "null server arguments");
    *out = nullptr;
    if (cfg->hbm_budget_bytes == 0) return set_error(BS_ERR_INVALID_ARG, "zero HBM budget");
    for (int r : cfg->reserved)
        if (r) return set_error(BS_ERR_INVALID_ARG, "reserved fields must be zero");
    Server* s = new Server();
    s->cfg = *cfg;
    if (s->cfg.max_inflight <= 0) s->cfg.max_inflight = 4;
    if (s->cfg.max_jobs_per_batch <= 0) s->cfg.max_jobs_per_batch = 512;
    s->device = cfg->device;
    hipError_t e = hipSetDevice(s->device);
    for (int i = 0; e == hipSuccess && i < s->cfg.max_inflight; ++i) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) {
            s->streams.push_back(st);
            s->stream_busy.push_back(false);
        }
    }
    s->flag_cap = s->cfg.max_inflight * s->cfg.max_jobs_per_batch;
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->flags), size_t(s->flag_cap) * 4,
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s->d_flags), s->flags, 0);
    if (e != hipSuccess) {
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        if (s->flags) (void)hipHostFree(s->flags);
        delete s;
        return set_error(BS_ERR_HIP, "server setup: %s", hipGetErrorString(e));
    }
    for (int i = s->flag_cap - 1; i >= 0; --i) {
        s->flags[i] = 0u;
        s->free_flags.push_back(i);
    }
    s->thread = std::thread(dispatcher, s);
    *out = new bs_server{s};
    return BS_OK;
}

int bs_server_submit(bs_server* srv, const bs_job* job, uint64_t* ticket) {
    if (!srv || !job || !ticket) return set_error(BS_ERR_INVALID_ARG, "null argument");
    Server& s = *srv->s;
    if (job->k < 0 || job->n < 0 || job->k > job->n || job->n >= (int64_t(1) << 31))
        return set_error(BS_ERR_INVALID_ARG, "bad job sizes n=%lld k=%lld", (long long)job->n,
                         (long long)job->k);
    if (job->k > 0 && (!job->d_points || !job->d_out_order))
        return set_error(BS_ERR_INVALID_ARG, "null job pointers");
    if (job_bytes_estimate(job->n, job->k) > s.cfg.hbm_budget_bytes) {
        std::lock_guard<std::mutex> lk(s.mu);
        s.rejected += 1;
        return set_error(BS_ERR_OVER_BUDGET, "job needs about %zu bytes, budget is %zu",
                         job_bytes_estimate(job->n, job->k), s.cfg.hbm_budget_bytes);
    }
    std::lock_guard<std::mutex> lk(s.mu);
    Job j;
    j.ticket = s.next_ticket++;
    j.req = *job;
    j.submitted = Clock::now();
    if (!s.any_submit) {
        s.t_first_submit = j.submitted;
        s.any_submit = true;
    }
    s.submitted += 1;
    *ticket = j.ticket;
    s.jobs.emplace(j.ticket, j);
    s.pending.push_back(j.ticket);
    s.cv_work.notify_one();
    return BS_OK;
}

int bs_server_poll(bs_server* srv, uint64_t ticket, int* done) {
    if (!srv || !done) return set_error(BS_ERR_INVALID_ARG, "null argument");
    Server& s = *srv->s;
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.jobs.find(ticket);
    if (it == s.jobs.end()) return set_error(BS_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    *done = it->second.done ? 1 : 0;
    return it->second.done ? it->second.status : BS_OK;
}

int bs_server_wait(bs_server* srv, uint64_t ticket, int64_t timeout_us) {
    if (!srv) return set_error(BS_ERR_INVALID_ARG, "null server");
    Server& s = *srv->s;
    std::unique_lock<std::mutex> lk(s.mu);
    auto it = s.jobs.find(ticket);
    if (it == s.jobs.end()) return set_error(BS_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    const auto deadline = Clock::now() + std::chrono::microseconds(timeout_us < 0 ? int64_t(1) << 40 : timeout_us);
    while (!s.jobs[ticket].done) {
        if (s.cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !s.jobs[ticket].done)
            return set_error(BS_ERR_TIMEOUT, "ticket %llu not done", (unsigned long long)ticket);
    }
    return s.jobs[ticket].status;
}

int bs_server_drain(bs_server* srv, int64_t timeout_us) {
    if (!srv) return set_error(BS_ERR_INVALID_ARG, "null server");
    Server& s = *srv->s;
    std::unique_lock<std::mutex> lk(s.mu);
    const auto deadline = Clock::now() + std::chrono::microseconds(timeout_us < 0 ? int64_t(1) << 40 : timeout_us);
    while (!(s.pending.empty() && s.inflight.empty())) {
        s.cv_work.notify_one();
        if (s.cv_done.wait_until(lk, deadline) == std::cv_status::timeout &&
            !(s.pending.empty() && s.inflight.empty()))
            return set_error(BS_ERR_TIMEOUT, "server not drained");
    }
    return s.last_error;
}

int bs_server_stats(bs_server* srv, bs_serving_stats* out) {
    if (!srv || !out) return set_error(BS_ERR_INVALID_ARG, "null argument");
    Server& s = *srv->s;
    std::lock_guard<std::mutex> lk(s.mu);
    bs_serving_stats st{};
    st.submitted = s.submitted;
    st.admitted = s.admitted;
    st.completed = s.completed;
    st.rejected = s.rejected;
    st.queued = int64_t(s.pending.size());
    st.inflight_batches = int64_t(s.inflight.size());
    st.batches = s.batches;
    st.ordered_surfels = s.k_done;
    st.p50_us = percentile(s.latencies_us, 0.50);
    st.p99_us = percentile(s.latencies_us, 0.99);
    st.max_us = s.latencies_us.empty() ? 0.0 : *std::max_element(s.latencies_us.begin(), s.latencies_us.end());
    double sum = 0.0;
    for (double v : s.latencies_us) sum += v;
    st.mean_us = s.latencies_us.empty() ? 0.0 : sum / double(s.latencies_us.size());
    st.elapsed_s = s.any_submit && s.completed
                       ? std::chrono::duration<double>(s.t_last_done - s.t_first_submit).count()
                       : 0.0;
    st.surfels_per_s = st.elapsed_s > 0 ? double(s.k_done) / st.elapsed_s : 0.0;
    st.hbm_in_use = s.bytes_in_use;
    st.hbm_peak = s.bytes_peak;
    *out = st;
    return BS_OK;
}

void bs_server_destroy(bs_server* srv) {
    if (!srv) return;
    Server* s = srv->s;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->thread.joinable()) s->thread.join();
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->flags) (void)hipHostFree(s->flags);
    delete s;
    delete srv;
}

}  // extern "C"
