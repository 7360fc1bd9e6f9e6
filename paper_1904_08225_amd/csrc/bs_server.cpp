// bs_server.cpp -- serving loop with continuous batching under an HBM budget.
//
// Requests (ordering jobs of any size) are submitted from any host thread.
// A persistent kernel of ordering workers (1024-thread workgroups, each
// holding a whole compute unit, on half the compute units by default, so that
// the preprocessing kernels of later micro-batches find free CUs) stays
// resident on the device and takes jobs from a device ring.
// A dispatcher thread admits pending jobs in arrival order while they fit the
// HBM budget, groups the admitted jobs into micro-batches, copies their
// candidates into one staging buffer, builds all their grids with the
// batched preprocessing on a preprocessing stream, and appends their
// descriptors to the ring.  Idle workers claim descriptors as soon as they
// are published, so a job only waits for a free worker, never for another
// job.  Each job sets its own completion flag in pinned host memory; once all
// jobs of a micro-batch are done, its memory returns to the budget.  Results
// are bit-identical to ordering each job alone.
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

// The dispatcher raises the stop flag as soon as the server has no job
// queued or on the device (the workers then leave within one poll, so a
// device-wide synchronisation by the caller does not wait for them), and
// relaunches the workers for the next job.  As a safety net the workers also
// leave by themselves after this many empty polls (each about 5 us).
constexpr uint32_t kIdlePolls = 4u << 20;

struct Job {
    uint64_t ticket;
    bs_job req;
    Clock::time_point submitted;
    Clock::time_point done_at;
    int flag_slot = -1;
    bool done = false;
    int status = BS_OK;
};

// An admitted micro-batch whose jobs are on the device.
struct InFlight {
    BatchPlan* plan = nullptr;
    void* staging = nullptr;
    void* ws = nullptr;
    size_t bytes = 0;
    std::vector<uint64_t> tickets;  // jobs with device work
};

}  // namespace

struct Server {
    bs_server_config cfg{};
    int device = 0;
    int workgroups = 0;
    hipStream_t prep = nullptr;    // preprocessing and publishing, in admission order
    hipStream_t serve = nullptr;   // the persistent workers
    hipEvent_t serve_end = nullptr;
    bool serve_launched = false;
    bool serve_stopping = false;   // stop raised for the running workers
    uint32_t* flags = nullptr;     // pinned host, one per job on the device
    uint32_t* d_flags = nullptr;   // device alias of flags
    int flag_cap = 0;
    std::vector<int> free_flags;
    ServeRing ring;
    uint32_t* stop_flag = nullptr;  // pinned host (ring.stop is its device alias)
    uint32_t published = 0;

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

void finish_job(Server& s, Job& j, int status, Clock::time_point now) {
    j.done = true;
    j.status = status;
    j.done_at = now;
    if (status == BS_OK) {
        s.completed += 1;
        s.k_done += j.req.k;
        s.latencies_us.push_back(std::chrono::duration<double, std::micro>(j.done_at - j.submitted).count());
        s.t_last_done = now;
    }
}

bool workers_running(Server& s) { return s.serve_launched && hipEventQuery(s.serve_end) != hipSuccess; }

// Make sure all workers run.  Workers told to stop are idle and leave within
// one poll: wait for them, then start a full set.
int ensure_workers(Server& s) {
    if (workers_running(s)) {
        if (!s.serve_stopping) return BS_OK;
        (void)hipEventSynchronize(s.serve_end);
    }
    __atomic_store_n(&s.stop_flag[0], 0u, __ATOMIC_RELEASE);
    s.serve_stopping = false;
    hipError_t e = launch_serve(s.ring, s.workgroups, kIdlePolls, s.serve);
    if (e == hipSuccess) e = hipEventRecord(s.serve_end, s.serve);
    if (e != hipSuccess) return set_error(BS_ERR_HIP, "serve launch: %s", hipGetErrorString(e));
    s.serve_launched = true;
    return BS_OK;
}

// Nothing queued or on the device: let the workers leave.
void stop_workers(Server& s) {
    if (s.serve_stopping || !workers_running(s)) return;
    __atomic_store_n(&s.stop_flag[0], 1u, __ATOMIC_RELEASE);
    s.serve_stopping = true;
}

// Admit one micro-batch from the front of the pending queue (caller holds
// mu).  Returns false when nothing could be admitted now.
bool admit_batch(Server& s) {
    std::vector<uint64_t> take;
    size_t bytes = 0;
    const size_t budget = s.cfg.hbm_budget_bytes;
    const auto now = Clock::now();
    bool any = false;
    while (!s.pending.empty()) {
        if (int(take.size()) >= s.cfg.max_jobs_per_batch || int(take.size()) >= int(s.free_flags.size())) break;
        Job& j = s.jobs[s.pending.front()];
        if (j.req.k == 0) {  // nothing to order
            s.pending.pop_front();
            s.admitted += 1;
            finish_job(s, j, BS_OK, now);
            any = true;
            continue;
        }
        const size_t b = job_bytes_estimate(j.req.n, j.req.k);
        if (s.bytes_in_use + bytes + b > budget) break;  // waits until memory frees up
        bytes += b;
        take.push_back(s.pending.front());
        s.pending.pop_front();
    }
    if (any) s.cv_done.notify_all();
    if (take.empty()) return any;

    // exact bytes of the plan: give jobs back from the tail until it fits
    InFlight f;
    std::vector<int64_t> offs, ks;
    std::vector<uint64_t> seeds;
    int rc = BS_OK;
    while (true) {
        offs.assign(take.size() + 1, 0);
        ks.resize(take.size());
        seeds.resize(take.size());
        for (size_t i = 0; i < take.size(); ++i) {
            const Job& j = s.jobs[take[i]];
            offs[i + 1] = offs[i] + j.req.n;
            ks[i] = j.req.k;
            seeds[i] = j.req.seed;
        }
        if (f.plan) batch_plan_free(f.plan);
        f.plan = nullptr;
        rc = batch_plan_create(offs.data(), ks.data(), seeds.data(), int32_t(take.size()),
                               s.cfg.cell_points > 0.f ? s.cfg.cell_points : 8.f, -1, &f.plan);
        if (rc != BS_OK) break;
        f.bytes = batch_workspace_bytes(f.plan) + align_up(size_t(offs.back()) * 12);
        if (s.bytes_in_use + f.bytes <= budget) break;
        if (take.size() == 1) {
            batch_plan_free(f.plan);
            f.plan = nullptr;
            if (!s.inflight.empty()) {  // wait for memory to free up
                s.pending.push_front(take[0]);
                return false;
            }
            Job& j = s.jobs[take[0]];  // can never fit
            finish_job(s, j, BS_ERR_OVER_BUDGET, now);
            s.rejected += 1;
            s.cv_done.notify_all();
            return true;
        }
        s.pending.push_front(take.back());
        take.pop_back();
    }
    std::vector<int32_t*> outo(take.size());
    std::vector<float*> outr(take.size());
    std::vector<uint32_t*> done(take.size());
    for (size_t i = 0; i < take.size(); ++i) {
        Job& j = s.jobs[take[i]];
        outo[i] = j.req.d_out_order;
        outr[i] = j.req.d_out_radius;
        j.flag_slot = s.free_flags.back();
        s.free_flags.pop_back();
        s.flags[j.flag_slot] = 0u;
        done[i] = s.d_flags + j.flag_slot;
    }
    hipError_t e = hipSuccess;
    if (rc == BS_OK) {
        batch_set_job_io(f.plan, outo, outr, done);
        e = hipMallocAsync(&f.staging, std::max<size_t>(size_t(offs.back()) * 12, 16), s.prep);
        if (e == hipSuccess) e = hipMallocAsync(&f.ws, std::max<size_t>(batch_workspace_bytes(f.plan), 256), s.prep);
        for (size_t i = 0; e == hipSuccess && i < take.size(); ++i) {
            const Job& j = s.jobs[take[i]];
            if (j.req.ready_event)  // the producer of the points
                e = hipStreamWaitEvent(s.prep, reinterpret_cast<hipEvent_t>(j.req.ready_event), 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(static_cast<char*>(f.staging) + size_t(offs[i]) * 12, j.req.d_points,
                               size_t(j.req.n) * 12, hipMemcpyDeviceToDevice, s.prep);
        }
        if (e == hipSuccess) {
            rc = batch_plan_publish(f.plan, static_cast<const float*>(f.staging), f.ws,
                                    batch_workspace_bytes(f.plan), s.ring, s.published, s.prep);
            if (rc == BS_OK) rc = ensure_workers(s);
        } else {
            rc = set_error(BS_ERR_HIP, "staging: %s", hipGetErrorString(e));
        }
    }
    if (rc != BS_OK) {
        // nothing of this batch is pending on the device: fail its jobs
        (void)hipStreamSynchronize(s.prep);
        for (uint64_t t : take) {
            Job& j = s.jobs[t];
            finish_job(s, j, rc, now);
            s.free_flags.push_back(j.flag_slot);
            j.flag_slot = -1;
        }
        if (f.staging) (void)hipFreeAsync(f.staging, s.prep);
        if (f.ws) (void)hipFreeAsync(f.ws, s.prep);
        if (f.plan) batch_plan_free(f.plan);
        s.last_error = rc;
        s.cv_done.notify_all();
        return true;
    }
    s.published += uint32_t(batch_work_count(f.plan));
    f.tickets = take;
    s.bytes_in_use += f.bytes;
    s.bytes_peak = std::max(s.bytes_peak, s.bytes_in_use);
    s.admitted += int64_t(take.size());
    s.batches += 1;
    s.inflight.push_back(std::move(f));
    return true;
}

// Record finished jobs and release finished micro-batches (caller holds mu).
bool reap(Server& s) {
    bool any = false;
    const auto now = Clock::now();
    for (size_t b = 0; b < s.inflight.size();) {
        InFlight& f = s.inflight[b];
        bool all = true;
        for (uint64_t t : f.tickets) {
            Job& j = s.jobs[t];
            if (!j.done && __atomic_load_n(&s.flags[j.flag_slot], __ATOMIC_ACQUIRE) != 0u) {
                finish_job(s, j, BS_OK, now);
                s.free_flags.push_back(j.flag_slot);
                j.flag_slot = -1;
                any = true;
            }
            all = all && j.done;
        }
        if (all) {  // no worker touches this batch any more
            (void)hipFreeAsync(f.staging, s.prep);
            (void)hipFreeAsync(f.ws, s.prep);
            batch_plan_free(f.plan);
            s.bytes_in_use -= f.bytes;
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
        while (!s.pending.empty() && int(s.inflight.size()) < s.cfg.max_inflight && admit_batch(s)) {
        }
        if (!s.inflight.empty()) {
            if (ensure_workers(s) != BS_OK) s.last_error = BS_ERR_HIP;
        } else if (s.pending.empty()) {
            stop_workers(s);
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

void release(Server* s) {
    if (s->serve) (void)hipStreamSynchronize(s->serve);
    if (s->prep) (void)hipStreamSynchronize(s->prep);
    if (s->serve_end) (void)hipEventDestroy(s->serve_end);
    if (s->ring.slots) (void)hipFree(s->ring.slots);
    if (s->ring.head) (void)hipFree(s->ring.head);
    if (s->serve) (void)hipStreamDestroy(s->serve);
    if (s->prep) (void)hipStreamDestroy(s->prep);
    if (s->flags) (void)hipHostFree(s->flags);
    if (s->stop_flag) (void)hipHostFree(s->stop_flag);
    delete s;
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
    if (cfg->workgroups < 0 || cfg->max_inflight < 0 || cfg->max_jobs_per_batch < 0)
        return set_error(BS_ERR_INVALID_ARG, "negative server sizes");
    Server* s = new Server();
    s->cfg = *cfg;
    if (s->cfg.max_inflight <= 0) s->cfg.max_inflight = 64;
    if (s->cfg.max_jobs_per_batch <= 0) s->cfg.max_jobs_per_batch = 512;
    s->device = cfg->device;
    hipError_t e = hipSetDevice(s->device);
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device);
    s->workgroups = cfg->workgroups > 0 ? cfg->workgroups : std::max(cus / 2, 1);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->prep, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->serve, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->serve_end, hipEventDisableTiming);
    s->flag_cap = s->cfg.max_inflight * s->cfg.max_jobs_per_batch;
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->flags), size_t(s->flag_cap) * 4,
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s->d_flags), s->flags, 0);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->stop_flag), 64, hipHostMallocMapped | hipHostMallocCoherent);
    uint32_t* d_stop = nullptr;
    if (e == hipSuccess) {
        s->stop_flag[0] = 0u;
        e = hipHostGetDevicePointer(reinterpret_cast<void**>(&d_stop), s->stop_flag, 0);
    }
    // ring: one slot per completion flag (a published job holds a flag until
    // it is done, so an unclaimed descriptor is never overwritten)
    s->ring.cap = uint32_t(s->flag_cap);
    s->ring.stop = d_stop;
    if (e == hipSuccess) e = hipMalloc(&s->ring.slots, size_t(s->flag_cap) * serve_slot_bytes());
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->ring.head), 256);
    if (e == hipSuccess) e = hipMemset(s->ring.head, 0, 256);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    s->ring.tail = s->ring.head ? s->ring.head + 32 : nullptr;  // its own 128-byte line
    if (e != hipSuccess) {
        const int rc = set_error(BS_ERR_HIP, "server setup: %s", hipGetErrorString(e));
        release(s);
        return rc;
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
    if (s->thread.joinable()) s->thread.join();  // every job is done
    __atomic_store_n(&s->stop_flag[0], 1u, __ATOMIC_RELEASE);  // workers leave once nothing is left
    release(s);
    delete srv;
}

}  // extern "C"
