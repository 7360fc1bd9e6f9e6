// bs_dispatch.h -- the serving loop's dispatcher, written against a small
// device interface so that admission, budget accounting and the worker
// life cycle run the same over the GPU (bs_server.cpp) and over a CPU stand-in
// (the test suite's fake device).  Host code only: no HIP types here.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/bluesurfels.h"

namespace bs {

int set_error(int code, const char* fmt, ...);

// What the dispatcher needs from a device.  Every call comes from the
// dispatcher thread (or the server's creation and destruction).
class ServeDevice {
public:
    virtual ~ServeDevice() = default;
    // Plan a micro-batch of jobs on the host; *bytes = the device memory it
    // holds while in flight (exact).  *batch is the device's handle.
    virtual int prepare(const std::vector<const bs_job*>& jobs, size_t* bytes, void** batch) = 0;
    // Drop a prepared batch that will not start.
    virtual void discard(void* batch) = 0;
    // Enqueue the batch's copies, preprocessing and publication; job i sets
    // completion flag flags[i] when its outputs are complete.
    virtual int start(void* batch, const std::vector<const bs_job*>& jobs, const std::vector<int>& flags) = 0;
    // The batch's preprocessing has begun on the device (everything queued
    // before it on the device has run).
    virtual bool began(void* batch) = 0;
    // The batch's jobs are in the ring (the workers can claim them).
    virtual bool published(void* batch) = 0;
    // Every job of the batch is done: release its memory.
    virtual void release(void* batch) = 0;
    virtual bool flag(int slot) = 0;
    virtual void clear_flag(int slot) = 0;
    virtual int flag_capacity() const = 0;
    // Start a full set of workers with the stop flag cleared.
    virtual int launch_workers() = 0;
    virtual bool workers_running() = 0;
    // Raise the stop flag: workers leave once nothing is left to claim.
    virtual void stop_workers() = 0;
    // Wait for all device activity (the server is being destroyed).
    virtual void quiesce() = 0;
};

struct DispatchConfig {
    size_t budget = 0;             // device bytes the in-flight batches may hold
    int max_inflight = 64;         // micro-batches on the device at once
    int max_jobs_per_batch = 512;
    int poll_us = 50;              // dispatcher period while busy
    int64_t stall_us = 5000;       // preprocessing overdue when not begun this long after it could
};

struct Server;

// Takes ownership of dev (deleted by server_destroy, or on failure).
int server_create(const DispatchConfig& cfg, ServeDevice* dev, Server** out);
int server_submit(Server* s, const bs_job* job, uint64_t* ticket);
int server_poll(Server* s, uint64_t ticket, int* done);
int server_wait(Server* s, uint64_t ticket, int64_t timeout_us);
int server_drain(Server* s, int64_t timeout_us);
int server_stats(Server* s, bs_serving_stats* out);
// Times the dispatcher stopped the workers because a publication was overdue.
int64_t server_stall_stops(Server* s);
// Times it launched a set of workers.
int64_t server_worker_launches(Server* s);
void server_destroy(Server* s);

// Lower bound of a job's device footprint, used before planning.
size_t job_bytes_estimate(int64_t n, int64_t k);

}  // namespace bs
