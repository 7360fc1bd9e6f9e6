// bs_server.cpp -- the serving loop on the GPU: the device side of the
// dispatcher of bs_dispatch.cpp, and the bs_server_* C ABI.
//
// A persistent kernel of ordering workers (1024-thread workgroups, each
// holding a whole compute unit, on three quarters of the compute units by
// default, so that the preprocessing kernels of later micro-batches find free
// CUs) takes jobs
// from a device ring.  For each admitted micro-batch the device copies the
// jobs' candidates into one staging buffer (after each job's producer event),
// builds all their grids with the batched preprocessing on a preprocessing
// stream and appends their descriptors to the ring; an event after the
// publication tells the dispatcher when the jobs became claimable.  Idle
// workers claim descriptors as soon as they are published, so a job only
// waits for a free worker, never for another job.  Each job sets its own
// completion flag in pinned host memory.  Results are bit-identical to
// ordering each job alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "bs_dispatch.h"
#include "bs_internal.h"

namespace bs {
namespace {

// The workers also leave by themselves after this many empty polls (each
// about 5 us) -- a safety net; the dispatcher stops them when idle.
constexpr uint32_t kIdlePolls = 4u << 20;

struct HipBatch {
    BatchPlan* plan = nullptr;
    void* staging = nullptr;
    void* ws = nullptr;
    hipEvent_t began = nullptr;      // recorded before the batch's first operation
    hipEvent_t published = nullptr;
    int64_t candidates = 0;
};

class HipServeDevice final : public ServeDevice {
public:
    int init(const bs_server_config& cfg) {
        cfg_ = cfg;
        device_ = cfg.device;
        hipError_t e = hipSetDevice(device_);
        int cus = 0;
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device_);
        // Workers on every CU would leave none for the preprocessing of the
        // next micro-batches, which would then wait for the workers' idle
        // exit (the stall rule sees preprocessing that has begun, not CU
        // starvation): at most seven eighths.  Queued at once, the 2,000
        // requests of the serving stream ran at 42.8, 55.5 and 45.5 M
        // surfels/s with half, three quarters and seven eighths of the CUs.
        const int most = std::max(cus - cus / 8, 1);
        workgroups_ = std::min(cfg.workgroups > 0 ? cfg.workgroups : std::max(cus - cus / 4, 1), most);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&prep_, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&serve_, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&serve_end_, hipEventDisableTiming);
        flag_cap_ = cfg.max_inflight * cfg.max_jobs_per_batch;
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&flags_), size_t(flag_cap_) * 4,
                              hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&d_flags_), flags_, 0);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&stop_), 64, hipHostMallocMapped | hipHostMallocCoherent);
        uint32_t* d_stop = nullptr;
        if (e == hipSuccess) {
            stop_[0] = 0u;
            e = hipHostGetDevicePointer(reinterpret_cast<void**>(&d_stop), stop_, 0);
        }
        // one ring slot per completion flag: a published job holds its flag
        // until it is done, so an unclaimed descriptor is never overwritten
        ring_.cap = uint32_t(flag_cap_);
        ring_.stop = d_stop;
        if (e == hipSuccess) e = hipMalloc(&ring_.slots, size_t(flag_cap_) * serve_slot_bytes());
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ring_.head), 256);
        if (e == hipSuccess) e = hipMemset(ring_.head, 0, 256);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        ring_.tail = ring_.head ? ring_.head + 32 : nullptr;  // its own 128-byte line
        if (e != hipSuccess) return set_error(BS_ERR_HIP, "server setup: %s", hipGetErrorString(e));
        for (int i = 0; i < flag_cap_; ++i) flags_[i] = 0u;
        return BS_OK;
    }

    ~HipServeDevice() override {
        if (serve_) (void)hipStreamSynchronize(serve_);
        if (prep_) (void)hipStreamSynchronize(prep_);
        if (serve_end_) (void)hipEventDestroy(serve_end_);
        if (ring_.slots) (void)hipFree(ring_.slots);
        if (ring_.head) (void)hipFree(ring_.head);
        if (serve_) (void)hipStreamDestroy(serve_);
        if (prep_) (void)hipStreamDestroy(prep_);
        if (flags_) (void)hipHostFree(flags_);
        if (stop_) (void)hipHostFree(stop_);
    }

    int prepare(const std::vector<const bs_job*>& jobs, size_t* bytes, void** batch) override {
        (void)hipSetDevice(device_);
        std::vector<int64_t> offs(jobs.size() + 1, 0), ks(jobs.size());
        std::vector<uint64_t> seeds(jobs.size());
        for (size_t i = 0; i < jobs.size(); ++i) {
            offs[i + 1] = offs[i] + jobs[i]->n;
            ks[i] = jobs[i]->k;
            seeds[i] = jobs[i]->seed;
        }
        HipBatch* b = new HipBatch();
        const int rc = batch_plan_create(offs.data(), ks.data(), seeds.data(), int32_t(jobs.size()),
                                         cfg_.cell_points > 0.f ? cfg_.cell_points : 8.f, -1, 0, &b->plan);
        if (rc != BS_OK) {
            delete b;
            return rc;
        }
        // bounded cells: the largest jobs' Morton-prefix cells are uneven
        batch_set_split_cells(b->plan, true);
        b->candidates = offs.back();
        *bytes = batch_workspace_bytes(b->plan) + align_up(size_t(offs.back()) * 12);
        *batch = b;
        return BS_OK;
    }

    void discard(void* batch) override {
        HipBatch* b = static_cast<HipBatch*>(batch);
        if (!b) return;
        if (b->plan) batch_plan_free(b->plan);
        delete b;
    }

    int start(void* batch, const std::vector<const bs_job*>& jobs, const std::vector<int>& flags) override {
        HipBatch* b = static_cast<HipBatch*>(batch);
        std::vector<int32_t*> outo(jobs.size());
        std::vector<float*> outr(jobs.size());
        std::vector<uint32_t*> done(jobs.size());
        for (size_t i = 0; i < jobs.size(); ++i) {
            outo[i] = jobs[i]->d_out_order;
            outr[i] = jobs[i]->d_out_radius;
            done[i] = d_flags_ + flags[i];
        }
        batch_set_job_io(b->plan, outo, outr, done);
        hipError_t e = hipEventCreateWithFlags(&b->published, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->began, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(b->began, prep_);
        if (e == hipSuccess) e = hipMallocAsync(&b->staging, std::max<size_t>(size_t(b->candidates) * 12, 16), prep_);
        if (e == hipSuccess)
            e = hipMallocAsync(&b->ws, std::max<size_t>(batch_workspace_bytes(b->plan), 256), prep_);
        int64_t at = 0;
        for (size_t i = 0; e == hipSuccess && i < jobs.size(); ++i) {
            if (jobs[i]->ready_event)  // the producer of the points
                e = hipStreamWaitEvent(prep_, reinterpret_cast<hipEvent_t>(jobs[i]->ready_event), 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(static_cast<char*>(b->staging) + size_t(at) * 12, jobs[i]->d_points,
                                   size_t(jobs[i]->n) * 12, hipMemcpyDeviceToDevice, prep_);
            at += jobs[i]->n;
        }
        int rc = BS_OK;
        if (e == hipSuccess) {
            rc = batch_plan_publish(b->plan, static_cast<const float*>(b->staging), b->ws,
                                    batch_workspace_bytes(b->plan), ring_, published_, prep_);
            if (rc == BS_OK) e = hipEventRecord(b->published, prep_);
        }
        if (e != hipSuccess && rc == BS_OK) rc = set_error(BS_ERR_HIP, "staging: %s", hipGetErrorString(e));
        if (rc != BS_OK) {
            (void)hipStreamSynchronize(prep_);
            free_memory(b);
            return rc;
        }
        published_ += uint32_t(batch_work_count(b->plan));
        return BS_OK;
    }

    bool began(void* batch) override { return hipEventQuery(static_cast<HipBatch*>(batch)->began) == hipSuccess; }

    bool published(void* batch) override {
        return hipEventQuery(static_cast<HipBatch*>(batch)->published) == hipSuccess;
    }

    void release(void* batch) override {
        HipBatch* b = static_cast<HipBatch*>(batch);
        free_memory(b);
        discard(b);
    }

    bool flag(int slot) override { return __atomic_load_n(&flags_[slot], __ATOMIC_ACQUIRE) != 0u; }
    void clear_flag(int slot) override { flags_[slot] = 0u; }
    int flag_capacity() const override { return flag_cap_; }

    int launch_workers() override {
        __atomic_store_n(&stop_[0], 0u, __ATOMIC_RELEASE);
        hipError_t e = launch_serve(ring_, workgroups_, kIdlePolls, serve_);
        if (e == hipSuccess) e = hipEventRecord(serve_end_, serve_);
        if (e != hipSuccess) return set_error(BS_ERR_HIP, "serve launch: %s", hipGetErrorString(e));
        launched_ = true;
        return BS_OK;
    }

    bool workers_running() override { return launched_ && hipEventQuery(serve_end_) != hipSuccess; }

    void stop_workers() override { __atomic_store_n(&stop_[0], 1u, __ATOMIC_RELEASE); }

    void quiesce() override {
        stop_workers();
        if (serve_) (void)hipStreamSynchronize(serve_);
        if (prep_) (void)hipStreamSynchronize(prep_);
    }

private:
    void free_memory(HipBatch* b) {
        if (b->staging) (void)hipFreeAsync(b->staging, prep_);
        if (b->ws) (void)hipFreeAsync(b->ws, prep_);
        if (b->published) (void)hipEventDestroy(b->published);
        if (b->began) (void)hipEventDestroy(b->began);
        b->staging = b->ws = nullptr;
        b->published = b->began = nullptr;
    }

    bs_server_config cfg_{};
    int device_ = 0, workgroups_ = 0, flag_cap_ = 0;
    hipStream_t prep_ = nullptr, serve_ = nullptr;
    hipEvent_t serve_end_ = nullptr;
    bool launched_ = false;
    uint32_t* flags_ = nullptr;
    uint32_t* d_flags_ = nullptr;
    uint32_t* stop_ = nullptr;
    ServeRing ring_;
    uint32_t published_ = 0;
};

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
    if (cfg->workgroups < 0 || cfg->max_inflight < 0 || cfg->max_jobs_per_batch < 0 || cfg->stall_us < 0)
        return set_error(BS_ERR_INVALID_ARG, "negative server sizes");
    bs_server_config c = *cfg;
    if (c.max_inflight <= 0) c.max_inflight = 64;
    if (c.max_jobs_per_batch <= 0) c.max_jobs_per_batch = 512;
    HipServeDevice* dev = new HipServeDevice();
    int rc = dev->init(c);
    if (rc != BS_OK) {
        delete dev;
        return rc;
    }
    DispatchConfig dc;
    dc.budget = c.hbm_budget_bytes;
    dc.max_inflight = c.max_inflight;
    dc.max_jobs_per_batch = c.max_jobs_per_batch;
    dc.poll_us = c.poll_us > 0 ? c.poll_us : 50;
    dc.stall_us = c.stall_us > 0 ? c.stall_us : 5000;
    Server* s = nullptr;
    rc = server_create(dc, dev, &s);
    if (rc != BS_OK) return rc;
    *out = new bs_server{s};
    return BS_OK;
}

int bs_server_submit(bs_server* srv, const bs_job* job, uint64_t* ticket) {
    if (!srv) return set_error(BS_ERR_INVALID_ARG, "null server");
    return server_submit(srv->s, job, ticket);
}

int bs_server_poll(bs_server* srv, uint64_t ticket, int* done) {
    if (!srv) return set_error(BS_ERR_INVALID_ARG, "null server");
    return server_poll(srv->s, ticket, done);
}

int bs_server_wait(bs_server* srv, uint64_t ticket, int64_t timeout_us) {
    if (!srv) return set_error(BS_ERR_INVALID_ARG, "null server");
    return server_wait(srv->s, ticket, timeout_us);
}

int bs_server_drain(bs_server* srv, int64_t timeout_us) {
    if (!srv) return set_error(BS_ERR_INVALID_ARG, "null server");
    return server_drain(srv->s, timeout_us);
}

int bs_server_stats(bs_server* srv, bs_serving_stats* out) {
    if (!srv) return set_error(BS_ERR_INVALID_ARG, "null server");
    return server_stats(srv->s, out);
}

void bs_server_destroy(bs_server* srv) {
    if (!srv) return;
    server_destroy(srv->s);
    delete srv;
}

}  // extern "C"
