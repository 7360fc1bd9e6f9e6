// bs_dispatch.cpp -- the serving dispatcher: continuous batching under a
// device-memory budget (host code only; see bs_dispatch.h).
//
// Jobs are queued in arrival order.  A dispatcher thread admits the queue's
// head into micro-batches while the batch's exact device bytes fit the
// budget, starts each on the device (copies, preprocessing, publication into
// the workers' ring), watches the jobs' completion flags and returns a
// batch's memory to the budget when all its jobs are done.  Each job is timed
// from submit to the moment its flag is seen.
//
// Worker life cycle: a set of persistent workers runs while published jobs
// are unfinished.  When nothing is queued, in flight or being published the
// workers are told to stop (they leave once nothing is left to claim).  A
// batch whose preprocessing is overdue -- it has not begun on the device
// stall_us after every earlier batch was published (the preprocessing
// stream is in order, so only those can hold it up) -- also stops them: the
// device is then running it behind the persistent workers (two streams on
// one in-order hardware queue), the workers' exit lets it run, and the next
// workers start once the publication is done.  So a job never waits for the
// workers' own idle time-out, and slow preprocessing alone (large batches,
// pool growth) does not count as a stall.
//
// While the workers are told to stop, no batch is started: a job published
// then would be claimed by whichever workers had not yet left, and a new
// full set can only start once the last of them is gone, so the set would
// shrink to the workers that happened to be busy.  Admission resumes, and a
// full set is launched, once every worker has left (at once when they were
// idle; after the claimed jobs when a publication was overdue).
#include "bs_dispatch.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace bs {

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
    uint64_t ticket = 0;
    bs_job req{};
    Clock::time_point submitted{}, done_at{};
    int flag_slot = -1;
    bool done = false;
    int status = BS_OK;
};

struct InFlight {
    void* batch = nullptr;
    size_t bytes = 0;
    std::vector<uint64_t> tickets;
    Clock::time_point started{};
    Clock::time_point head_since{};  // every earlier batch was published by then
    bool at_head = false;            // head_since is set
    bool began = false;              // its preprocessing has begun on the device
    bool published = false;
    bool all_done = false;
};

}  // namespace

struct Server {
    DispatchConfig cfg;
    ServeDevice* dev = nullptr;
    std::vector<int> free_flags;
    bool workers_stopping = false;

    std::mutex mu;
    std::condition_variable cv_work;
    std::condition_variable cv_done;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Job> jobs;
    std::vector<InFlight> inflight;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread thread;

    int64_t submitted = 0, admitted = 0, completed = 0, rejected = 0, batches = 0;
    int64_t k_done = 0, stall_stops = 0, launches = 0;
    size_t bytes_in_use = 0, bytes_peak = 0;
    std::vector<double> latencies_us;
    Clock::time_point t_first_submit{}, t_last_done{};
    bool any_submit = false;
    int last_error = BS_OK;
};

size_t job_bytes_estimate(int64_t n, int64_t k) {
    (void)k;
    return size_t(n) * 64;
}

namespace {

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

// Admit one micro-batch from the head of the queue (caller holds mu).
// Returns false when nothing could be admitted now.
bool admit_batch(Server& s) {
    std::vector<uint64_t> take;
    size_t est = 0;
    const size_t budget = s.cfg.budget;
    const auto now = Clock::now();
    bool any = false;
    while (!s.pending.empty()) {
        if (int(take.size()) >= s.cfg.max_jobs_per_batch || take.size() >= s.free_flags.size()) break;
        Job& j = s.jobs[s.pending.front()];
        if (j.req.k == 0) {  // nothing to order
            s.pending.pop_front();
            s.admitted += 1;
            finish_job(s, j, BS_OK, now);
            any = true;
            continue;
        }
        const size_t b = job_bytes_estimate(j.req.n, j.req.k);
        if (s.bytes_in_use + est + b > budget) break;  // waits until memory frees up
        est += b;
        take.push_back(s.pending.front());
        s.pending.pop_front();
    }
    if (any) s.cv_done.notify_all();
    if (take.empty()) return any;

    // the exact bytes of the batch: give jobs back from the tail until it fits
    InFlight f;
    std::vector<const bs_job*> reqs;
    int rc = BS_OK;
    while (true) {
        reqs.clear();
        for (uint64_t t : take) reqs.push_back(&s.jobs[t].req);
        if (f.batch) s.dev->discard(f.batch);
        f.batch = nullptr;
        rc = s.dev->prepare(reqs, &f.bytes, &f.batch);
        if (rc != BS_OK) break;
        if (s.bytes_in_use + f.bytes <= budget) break;
        if (take.size() == 1) {
            s.dev->discard(f.batch);
            f.batch = nullptr;
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
    std::vector<int> flags(take.size());
    for (size_t i = 0; i < take.size(); ++i) {
        Job& j = s.jobs[take[i]];
        j.flag_slot = s.free_flags.back();
        s.free_flags.pop_back();
        s.dev->clear_flag(j.flag_slot);
        flags[i] = j.flag_slot;
    }
    if (rc == BS_OK) rc = s.dev->start(f.batch, reqs, flags);
    if (rc != BS_OK) {  // nothing of this batch runs on the device: fail its jobs
        for (uint64_t t : take) {
            Job& j = s.jobs[t];
            finish_job(s, j, rc, now);
            if (j.flag_slot >= 0) s.free_flags.push_back(j.flag_slot);
            j.flag_slot = -1;
        }
        if (f.batch) s.dev->discard(f.batch);
        s.last_error = rc;
        s.cv_done.notify_all();
        return true;
    }
    f.tickets = take;
    f.started = now;
    s.bytes_in_use += f.bytes;
    s.bytes_peak = std::max(s.bytes_peak, s.bytes_in_use);
    s.admitted += int64_t(take.size());
    s.batches += 1;
    s.inflight.push_back(std::move(f));
    return true;
}

// Record finished jobs and release finished batches (caller holds mu).
void reap(Server& s) {
    bool any = false;
    const auto now = Clock::now();
    bool earlier_published = true;  // every batch before this one (admission order)
    for (size_t b = 0; b < s.inflight.size();) {
        InFlight& f = s.inflight[b];
        if (!f.published) f.published = s.dev->published(f.batch);
        if (!f.began) f.began = f.published || s.dev->began(f.batch);
        if (earlier_published && !f.at_head) {
            f.at_head = true;
            f.head_since = now;
        }
        earlier_published = earlier_published && f.published;
        bool all = true;
        for (uint64_t t : f.tickets) {
            Job& j = s.jobs[t];
            if (!j.done && s.dev->flag(j.flag_slot)) {
                finish_job(s, j, BS_OK, now);
                s.free_flags.push_back(j.flag_slot);
                j.flag_slot = -1;
                any = true;
            }
            all = all && j.done;
        }
        if (all && f.published) {  // no worker touches this batch any more
            s.dev->release(f.batch);
            s.bytes_in_use -= f.bytes;
            s.inflight.erase(s.inflight.begin() + long(b));
            any = true;
            continue;
        }
        ++b;
    }
    if (any) s.cv_done.notify_all();
}

// Start, keep or stop the workers (caller holds mu).
void manage_workers(Server& s) {
    const auto now = Clock::now();
    bool claimable = false, publishing = false, overdue = false;
    for (const InFlight& f : s.inflight) {
        if (f.published) claimable = true;  // published with unfinished jobs (finished ones are reaped)
        else {
            publishing = true;
            overdue = overdue || (!f.began && f.at_head &&
                                  now - f.head_since > std::chrono::microseconds(s.cfg.stall_us));
        }
    }
    const bool running = s.dev->workers_running();
    if (running) {
        if (!s.workers_stopping && (overdue || (!claimable && !publishing && s.pending.empty()))) {
            s.dev->stop_workers();
            s.workers_stopping = true;
            if (overdue) s.stall_stops += 1;
        }
        return;
    }
    s.workers_stopping = false;  // every worker has left
    // no workers on the device: start a set when there is work for them
    // (an overdue publication has the device to itself until it is done)
    if (claimable || (publishing && !overdue)) {
        if (s.dev->launch_workers() != BS_OK) {
            s.last_error = BS_ERR_HIP;
            return;
        }
        s.workers_stopping = false;
        s.launches += 1;
    }
}

void dispatcher(Server* sp) {
    Server& s = *sp;
    std::unique_lock<std::mutex> lk(s.mu);
    while (true) {
        reap(s);
        // nothing starts while the workers are leaving (file comment)
        const bool hold = s.workers_stopping && s.dev->workers_running();
        while (!hold && !s.pending.empty() && int(s.inflight.size()) < s.cfg.max_inflight && admit_batch(s)) {
        }
        manage_workers(s);
        if (s.stop && s.pending.empty() && s.inflight.empty()) break;
        if (s.inflight.empty() && s.pending.empty())
            s.cv_work.wait_for(lk, std::chrono::milliseconds(5));
        else
            s.cv_work.wait_for(lk, std::chrono::microseconds(s.cfg.poll_us > 0 ? s.cfg.poll_us : 50));
    }
    if (s.dev->workers_running()) {
        s.dev->stop_workers();
        s.workers_stopping = true;
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

int server_create(const DispatchConfig& cfg, ServeDevice* dev, Server** out) {
    if (!dev || !out) {
        delete dev;
        return set_error(BS_ERR_INVALID_ARG, "null server arguments");
    }
    Server* s = new Server();
    s->cfg = cfg;
    s->dev = dev;
    for (int i = dev->flag_capacity() - 1; i >= 0; --i) s->free_flags.push_back(i);
    s->thread = std::thread(dispatcher, s);
    *out = s;
    return BS_OK;
}

int server_submit(Server* sv, const bs_job* job, uint64_t* ticket) {
    if (!sv || !job || !ticket) return set_error(BS_ERR_INVALID_ARG, "null argument");
    Server& s = *sv;
    if (job->k < 0 || job->n < 0 || job->k > job->n || job->n >= (int64_t(1) << 31))
        return set_error(BS_ERR_INVALID_ARG, "bad job sizes n=%lld k=%lld", (long long)job->n, (long long)job->k);
    if (job->k > 0 && (!job->d_points || !job->d_out_order))
        return set_error(BS_ERR_INVALID_ARG, "null job pointers");
    if (job_bytes_estimate(job->n, job->k) > s.cfg.budget) {
        std::lock_guard<std::mutex> lk(s.mu);
        s.rejected += 1;
        return set_error(BS_ERR_OVER_BUDGET, "job needs about %zu bytes, budget is %zu",
                         job_bytes_estimate(job->n, job->k), s.cfg.budget);
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

int server_poll(Server* sv, uint64_t ticket, int* done) {
    if (!sv || !done) return set_error(BS_ERR_INVALID_ARG, "null argument");
    Server& s = *sv;
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.jobs.find(ticket);
    if (it == s.jobs.end()) return set_error(BS_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    *done = it->second.done ? 1 : 0;
    return it->second.done ? it->second.status : BS_OK;
}

int server_wait(Server* sv, uint64_t ticket, int64_t timeout_us) {
    if (!sv) return set_error(BS_ERR_INVALID_ARG, "null server");
    Server& s = *sv;
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

int server_drain(Server* sv, int64_t timeout_us) {
    if (!sv) return set_error(BS_ERR_INVALID_ARG, "null server");
    Server& s = *sv;
    std::unique_lock<std::mutex> lk(s.mu);
    const auto deadline = Clock::now() + std::chrono::microseconds(timeout_us < 0 ? int64_t(1) << 40 : timeout_us);
    while (!(s.pending.empty() && s.inflight.empty())) {
        s.cv_work.notify_one();
        if (s.cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !(s.pending.empty() && s.inflight.empty()))
            return set_error(BS_ERR_TIMEOUT, "server not drained");
    }
    return s.last_error;
}

int server_stats(Server* sv, bs_serving_stats* out) {
    if (!sv || !out) return set_error(BS_ERR_INVALID_ARG, "null argument");
    Server& s = *sv;
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
    st.elapsed_s = s.any_submit && s.completed ? std::chrono::duration<double>(s.t_last_done - s.t_first_submit).count()
                                              : 0.0;
    st.surfels_per_s = st.elapsed_s > 0 ? double(s.k_done) / st.elapsed_s : 0.0;
    st.hbm_in_use = s.bytes_in_use;
    st.hbm_peak = s.bytes_peak;
    st.worker_launches = s.launches;
    st.stall_stops = s.stall_stops;
    *out = st;
    return BS_OK;
}

int64_t server_stall_stops(Server* sv) {
    if (!sv) return 0;
    std::lock_guard<std::mutex> lk(sv->mu);
    return sv->stall_stops;
}

int64_t server_worker_launches(Server* sv) {
    if (!sv) return 0;
    std::lock_guard<std::mutex> lk(sv->mu);
    return sv->launches;
}

void server_destroy(Server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->thread.joinable()) sv->thread.join();  // every job is done, the workers told to stop
    sv->dev->quiesce();
    delete sv->dev;
    delete sv;
}

}  // namespace bs
