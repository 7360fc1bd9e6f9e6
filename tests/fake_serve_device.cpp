// fake_serve_device.cpp -- a CPU stand-in for the serving device, so that
// the dispatcher (admission, budget accounting, the worker life cycle) is
// tested without a GPU.  TEST INFRASTRUCTURE: built by tests/test_dispatch_cpu.py
// together with the product's dispatcher source and the CPU oracle.
//
// A job's pointers are host memory here; a worker orders it with the oracle.
// Workers are host threads that claim published jobs from a queue and leave
// when the stop flag is up and nothing is left (or after an idle time-out).
// A batch is published by one "preprocessing" thread in admission order,
// after a delay.  In shared-queue mode publications and worker launches go
// through one in-order queue, like two streams on one in-order hardware
// queue: a publication enqueued after a worker launch waits until those
// workers have left, and a launch enqueued after a publication starts once
// it is done.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "../paper_1904_08225_amd/csrc/bs_dispatch.h"

extern "C" {
int oracle_greedy32(const float* P, int64_t n, int64_t k, int64_t start, int32_t* order, float* radius,
                    int64_t* n_live, int64_t* n_ball, int64_t* n_dec);
int64_t oracle_start_index(uint64_t seed, int64_t n);
}

namespace {

using Clock = std::chrono::steady_clock;

struct FakeBatch {
    std::vector<bs_job> jobs;
    std::vector<int> flags;
    std::atomic<bool> began{false};
    std::atomic<bool> published{false};
};

struct QueueItem {
    FakeBatch* batch;  // a publication, or nullptr: a launch of the workers
};

struct Claim {
    bs_job job;
    int flag;
};

class FakeDevice final : public bs::ServeDevice {
public:
    FakeDevice(int workers, bool shared_queue, int publish_delay_us, int bytes_per_candidate, int idle_ms,
               int exit_us)
        : workers_(workers), shared_(shared_queue), delay_us_(publish_delay_us), bpc_(bytes_per_candidate),
          idle_ms_(idle_ms), exit_us_(exit_us), flags_(4096) {
        for (auto& f : flags_) f.store(0u);
        prep_ = std::thread([this] { prep_loop(); });
    }
    ~FakeDevice() override { quiesce(); }

    int prepare(const std::vector<const bs_job*>& jobs, size_t* bytes, void** batch) override {
        FakeBatch* b = new FakeBatch();
        size_t sz = 0;
        for (const bs_job* j : jobs) {
            b->jobs.push_back(*j);
            sz += size_t(j->n) * size_t(bpc_);
        }
        *bytes = sz;
        *batch = b;
        return BS_OK;
    }
    void discard(void* batch) override { delete static_cast<FakeBatch*>(batch); }
    int start(void* batch, const std::vector<const bs_job*>&, const std::vector<int>& flags) override {
        FakeBatch* b = static_cast<FakeBatch*>(batch);
        b->flags = flags;
        std::lock_guard<std::mutex> lk(mu_);
        queue_.push_back(QueueItem{b});
        cv_.notify_all();
        return BS_OK;
    }
    bool began(void* batch) override { return static_cast<FakeBatch*>(batch)->began.load(); }
    bool published(void* batch) override { return static_cast<FakeBatch*>(batch)->published.load(); }
    void release(void* batch) override { delete static_cast<FakeBatch*>(batch); }
    bool flag(int slot) override { return flags_[size_t(slot)].load(std::memory_order_acquire) != 0u; }
    void clear_flag(int slot) override { flags_[size_t(slot)].store(0u); }
    int flag_capacity() const override { return int(flags_.size()); }

    int launch_workers() override {
        std::lock_guard<std::mutex> lk(mu_);
        reap_threads();
        stop_.store(false);
        launched_.store(true);
        if (shared_) {
            queue_.push_back(QueueItem{nullptr});  // started by the queue thread in order
            cv_.notify_all();
        } else {
            start_workers();
        }
        launches_ += 1;
        return BS_OK;
    }
    bool workers_running() override { return launched_.load(); }
    void stop_workers() override {
        stop_.store(true);
        cv_.notify_all();
    }
    void quiesce() override {
        stop_workers();
        {
            std::lock_guard<std::mutex> lk(mu_);
            shutdown_ = true;
            cv_.notify_all();
        }
        std::vector<std::thread> ts;
        {
            std::lock_guard<std::mutex> lk(mu_);
            ts.swap(threads_);
        }
        for (auto& t : ts)
            if (t.joinable()) t.join();
        if (prep_.joinable()) prep_.join();
    }
    int64_t launches() const { return launches_; }
    // Most jobs ordered at once since the last call (and reset).
    int take_peak() { return peak_.exchange(0); }

private:
    void reap_threads() {  // caller holds mu_; joins workers that have left
        if (running_.load() != 0) return;
        for (auto& t : threads_)
            if (t.joinable()) t.join();
        threads_.clear();
    }

    void start_workers() {  // caller holds mu_
        for (int w = 0; w < workers_; ++w) {
            running_.fetch_add(1);
            threads_.emplace_back([this, w] { worker_loop(w); });
        }
    }

    // Publications in order; in shared mode also the worker launches, each
    // holding the queue until its workers have left.
    void prep_loop() {
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            cv_.wait(lk, [this] { return shutdown_ || !queue_.empty(); });
            if (queue_.empty()) {
                if (shutdown_) return;
                continue;
            }
            QueueItem it = queue_.front();
            if (!it.batch) {  // a launch: its workers run, the queue waits for them
                start_workers();
                cv_.wait(lk, [this] { return running_.load() == 0; });
                queue_.pop_front();
                launched_.store(false);
                cv_.notify_all();
                continue;
            }
            it.batch->began.store(true);
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(delay_us_));
            lk.lock();
            queue_.pop_front();
            FakeBatch* b = it.batch;
            for (size_t i = 0; i < b->jobs.size(); ++i) ring_.push_back(Claim{b->jobs[i], b->flags[i]});
            b->published.store(true);
            cv_.notify_all();
        }
    }

    // Worker w notices the stop flag w * exit_us / workers after it was
    // raised (a device worker sees it at its next poll, and the kernel's end
    // is seen later still): until then it keeps claiming what is published.
    void worker_loop(int w) {
        auto idle_since = Clock::now();
        bool stop_seen = false;
        Clock::time_point leave_at{};
        while (true) {
            Claim c{};
            bool got = false;
            {
                std::unique_lock<std::mutex> lk(mu_);
                if (!ring_.empty()) {
                    c = ring_.front();
                    ring_.pop_front();
                    got = true;
                } else if (stop_.load() && !stop_seen) {
                    stop_seen = true;
                    leave_at = Clock::now() + std::chrono::microseconds(int64_t(exit_us_) * w / workers_);
                    continue;
                } else if ((stop_seen && Clock::now() >= leave_at) ||
                           Clock::now() - idle_since > std::chrono::milliseconds(idle_ms_)) {
                    if (running_.fetch_sub(1) == 1 && !shared_) launched_.store(false);
                    cv_.notify_all();
                    return;
                } else {
                    cv_.wait_for(lk, std::chrono::microseconds(200));
                }
            }
            if (!got) continue;
            stop_seen = false;  // the flag is read again after the job
            const int now_active = active_.fetch_add(1) + 1;
            for (int p = peak_.load(); now_active > p && !peak_.compare_exchange_weak(p, now_active);) {
            }
            const bs_job& j = c.job;
            if (j.k > 0)
                oracle_greedy32(j.d_points, j.n, j.k, oracle_start_index(j.seed, j.n), j.d_out_order,
                                j.d_out_radius, nullptr, nullptr, nullptr);
            active_.fetch_sub(1);
            flags_[size_t(c.flag)].store(1u, std::memory_order_release);
            idle_since = Clock::now();
        }
    }

    int workers_;
    bool shared_;
    int delay_us_, bpc_, idle_ms_, exit_us_;
    std::atomic<int> active_{0}, peak_{0};
    std::vector<std::atomic<uint32_t>> flags_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<QueueItem> queue_;
    std::deque<Claim> ring_;
    std::vector<std::thread> threads_;
    std::thread prep_;
    std::atomic<int> running_{0};
    std::atomic<bool> launched_{false};  // a launch is queued or its workers run
    std::atomic<bool> stop_{false};
    bool shutdown_ = false;
    int64_t launches_ = 0;
};

}  // namespace

extern "C" {

struct FakeServer {
    bs::Server* s;
    FakeDevice* dev;  // owned by s
};

void* fake_server_create(size_t budget, int max_jobs_per_batch, int workers, int shared_queue, int publish_delay_us,
                         int stall_us, int bytes_per_candidate, int idle_ms, int exit_us) {
    bs::DispatchConfig cfg;
    cfg.budget = budget;
    cfg.max_inflight = 8;
    cfg.max_jobs_per_batch = max_jobs_per_batch;
    cfg.poll_us = 50;
    cfg.stall_us = stall_us;
    auto* dev = new FakeDevice(workers, shared_queue != 0, publish_delay_us, bytes_per_candidate, idle_ms, exit_us);
    bs::Server* s = nullptr;
    if (bs::server_create(cfg, dev, &s) != BS_OK) return nullptr;
    return new FakeServer{s, dev};
}

static bs::Server* srv_of(void* h) { return static_cast<FakeServer*>(h)->s; }

int fake_server_submit(void* s, const float* pts, int64_t n, int64_t k, uint64_t seed, int32_t* out_order,
                       float* out_radius, uint64_t* ticket) {
    bs_job j{};
    j.d_points = pts;
    j.n = n;
    j.k = k;
    j.seed = seed;
    j.d_out_order = out_order;
    j.d_out_radius = out_radius;
    return bs::server_submit(srv_of(s), &j, ticket);
}

int fake_server_wait(void* s, uint64_t t, int64_t timeout_us) {
    return bs::server_wait(srv_of(s), t, timeout_us);
}

int fake_server_poll(void* s, uint64_t t, int* done) { return bs::server_poll(srv_of(s), t, done); }

int fake_server_drain(void* s, int64_t timeout_us) { return bs::server_drain(srv_of(s), timeout_us); }

int fake_server_stats(void* s, bs_serving_stats* out) { return bs::server_stats(srv_of(s), out); }

int64_t fake_server_stall_stops(void* s) { return bs::server_stall_stops(srv_of(s)); }

int64_t fake_server_launches(void* s) { return bs::server_worker_launches(srv_of(s)); }

int fake_server_take_peak(void* s) { return static_cast<FakeServer*>(s)->dev->take_peak(); }

void fake_server_destroy(void* s) {
    bs::server_destroy(srv_of(s));
    delete static_cast<FakeServer*>(s);
}

}  // extern "C"
