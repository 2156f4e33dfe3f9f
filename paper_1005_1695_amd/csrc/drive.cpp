// Native job generator for the streamed and serving workloads.
//
// Open loop (window == 0): job k is submitted at its scheduled arrival time
// whatever the state of earlier jobs, and its latency counts from that
// scheduled time, so queueing delay caused by a busy device is measured
// rather than hidden (no coordinated omission).  Closed loop (window > 0): at
// most `window` jobs are in the system; a job is submitted as soon as one
// finishes and its latency counts from its submit time.
#include <atomic>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <string.h>
#include <time.h>
#include <vector>

#include "internal.h"

namespace crystal {

struct DriveCtx {
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<uint64_t> done{0};
};

static void drive_cb(crystal_task *, void *user)
{
    DriveCtx *c = static_cast<DriveCtx *>(user);
    {
        std::lock_guard<std::mutex> lk(c->mu);
        c->done.fetch_add(1);
    }
    c->cv.notify_one();
}

static void sleep_until_ns(int64_t target)
{
    for (;;) {
        const int64_t now = now_ns();
        const int64_t left = target - now;
        if (left <= 0)
            return;
        if (left > 200000) { // coarse sleep, then spin the last 0.2 ms
            struct timespec ts;
            const int64_t nap = left - 150000;
            ts.tv_sec = nap / 1000000000ll;
            ts.tv_nsec = nap % 1000000000ll;
            nanosleep(&ts, nullptr);
        }
    }
}

} // namespace crystal

using namespace crystal;

extern "C" int crystal_drive(crystal_drive_job *jobs, uint64_t n, const crystal_direct_params *direct,
                             const crystal_cdc_params *cdc, uint32_t window,
                             crystal_drive_result *res)
{
    if (!jobs || !res)
        return fail(CRYSTAL_EINVAL, "jobs and res are required");
    std::vector<crystal_task> tasks(n);
    std::vector<crystal_buf *> bin(n, nullptr), bout(n, nullptr);
    std::vector<int64_t> sched(n, 0);
    for (uint64_t k = 0; k < n; k++) {
        int rc = crystal_buffer_wrap(const_cast<void *>(jobs[k].h_in), jobs[k].bytes, &bin[k]);
        if (rc == CRYSTAL_OK)
            rc = crystal_buffer_wrap(jobs[k].h_out, jobs[k].out_cap, &bout[k]);
        if (rc != CRYSTAL_OK) {
            for (uint64_t i = 0; i <= k; i++) {
                if (bin[i])
                    crystal_buffer_release(bin[i]);
                if (bout[i])
                    crystal_buffer_release(bout[i]);
            }
            return rc;
        }
    }
    DriveCtx ctx;
    std::vector<char> submitted(n, 0);
    const int64_t t0 = now_ns();
    for (uint64_t k = 0; k < n; k++) {
        if (window == 0) {
            sched[k] = t0 + (int64_t)(jobs[k].arrival_s * 1e9);
            sleep_until_ns(sched[k]);
        } else {
            std::unique_lock<std::mutex> lk(ctx.mu);
            ctx.cv.wait(lk, [&] { return k - ctx.done.load() < window; });
        }
        crystal_task &t = tasks[k];
        memset(&t, 0, sizeof t);
        t.in_bytes = jobs[k].bytes;
        t.params = jobs[k].kernel_id == CRYSTAL_K_CDC ? (const void *)cdc : (const void *)direct;
        t.callback = drive_cb;
        t.user = &ctx;
        const int64_t ts = now_ns();
        if (window)
            sched[k] = ts;
        const int rc = crystal_submit(&t, jobs[k].kernel_id, bin[k], bout[k]);
        if (rc != CRYSTAL_OK) {
            jobs[k].status = rc;
            std::lock_guard<std::mutex> lk(ctx.mu);
            ctx.done.fetch_add(1); // counts as finished for the window
        } else {
            submitted[k] = 1;
        }
    }
    int64_t last = t0;
    res->bytes = res->ok = res->failed = 0;
    for (uint64_t k = 0; k < n; k++) {
        if (!submitted[k]) {
            res->failed++;
            continue;
        }
        const int st = crystal_wait(&tasks[k], -1);
        jobs[k].status = st;
        jobs[k].latency_s = (tasks[k].t_done_ns - sched[k]) * 1e-9;
        jobs[k].admit_wait_s = (tasks[k].t_admit_ns - sched[k]) * 1e-9;
        if (tasks[k].t_done_ns > last)
            last = tasks[k].t_done_ns;
        if (st == CRYSTAL_OK) {
            res->ok++;
            res->bytes += jobs[k].bytes;
        } else {
            res->failed++;
        }
    }
    res->wall_s = (last - t0) * 1e-9;
    for (uint64_t k = 0; k < n; k++) {
        crystal_buffer_release(bin[k]);
        crystal_buffer_release(bout[k]);
    }
    return CRYSTAL_OK;
}
