// Job layer (the CrystalGPU design of Sec. 4.2 on one MI355X).
//
// State machine per job, as in the paper's three queues (Sec. 4.2): the
// caller takes buffers from the idle pool (crystal_buffer_acquire), submits a
// job to the outstanding queue, and a master thread dispatches it.  Here:
//   - one dispatcher thread pops the outstanding queue in FIFO order and
//     admits the head job only when the device slab has room for its input,
//     output and scratch (first fit) and fewer than max_in_flight jobs are
//     running.  The stages of the three-stage pipeline (Fig. 4) go on
//     separate streams: every copy-in is enqueued on one copy-in stream, so
//     the host link is never idle behind a kernel; the job's kernels and its
//     copy-out go on the least-loaded compute stream, which first waits on
//     the job's copy-in event.  Consecutive jobs thus overlap copy-in,
//     compute and copy-out;
//   - one completion thread per compute stream waits for that stream's jobs
//     in order (a stream completes in order), returns their device memory,
//     runs the callback and wakes waiters -- the asynchronous notification
//     the paper adds on top of a runtime that only offers polling (Sec. 4.1).
// Buffers are carved from one pinned host slab so copies never go through a
// driver staging buffer (Sec. 2.1, Sec. 3).
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <stdlib.h>
#include <string.h>
#include <thread>
#include <vector>

#include "internal.h"

struct crystal_buf {
    void *host;
    size_t size;
    size_t pool_off, pool_len; // region of the host slab (pooled buffers)
    bool pooled;
    std::atomic<int> refs;
};

namespace crystal {

static inline size_t al(size_t x, size_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over offsets [0, size) with coalescing free list.
class RangeAlloc {
  public:
    void reset(size_t size)
    {
        free_.clear();
        if (size)
            free_[0] = size;
        size_ = free_bytes_ = min_free_ = size;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes)
                continue;
            *off = it->first;
            const size_t rest = it->second - bytes, o2 = it->first + bytes;
            free_.erase(it);
            if (rest)
                free_[o2] = rest;
            free_bytes_ -= bytes;
            min_free_ = std::min(min_free_, free_bytes_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        size_t o = off, len = bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                o = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + bytes == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[o] = len;
        free_bytes_ += bytes;
    }
    size_t size() const { return size_; }
    size_t free_bytes() const { return free_bytes_; }
    size_t min_free() const { return min_free_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, free_bytes_ = 0, min_free_ = 0;
};

struct Job {
    crystal_task *t;
    int kernel;
    crystal_buf *in, *out;
    size_t n;
    size_t need, dev_off;
    size_t in_region;
    int stream;
    uint32_t seg_bytes;
    CdcParams cp;
    CdcGeom g;
    uint64_t cap;
    size_t d2h;
    uint8_t *d_out_ptr = nullptr; // device bytes copied back
};

// Device bytes a job needs and the layout inside its region:
// [input | output | scratch], each 256-byte aligned.
struct JobPlan {
    size_t in_region, out_region, ws_region, d2h;
};

static bool plan_job(int kernel, size_t n, const void *params, Job *j, JobPlan *p,
                     const char **why)
{
    p->in_region = al(n ? n : 1, 256);
    p->out_region = p->ws_region = 0;
    switch (kernel) {
    case CRYSTAL_K_NOP:
        p->d2h = n;
        break;
    case CRYSTAL_K_MD5:
        p->out_region = 256;
        p->d2h = 16;
        break;
    case CRYSTAL_K_MD5_DIRECT:
    case CRYSTAL_K_SHA1_DIRECT: {
        const size_t dlen = kernel == CRYSTAL_K_MD5_DIRECT ? 16 : 20;
        uint32_t seg = 4096;
        if (params) {
            const auto *dp = static_cast<const crystal_direct_params *>(params);
            if (dp->segment_bytes)
                seg = dp->segment_bytes;
        }
        if (seg % 64 || seg > (1u << 30)) {
            *why = "segment_bytes must be a multiple of 64 and <= 2^30";
            return false;
        }
        if (j)
            j->seg_bytes = seg;
        const uint64_t nseg = (n + seg - 1) / seg;
        p->d2h = dlen * (nseg + 1);
        p->out_region = al(p->d2h, 256);
        break;
    }
    case CRYSTAL_K_CDC: {
        CdcParams cp;
        if (!cdc_resolve(static_cast<const crystal_cdc_params *>(params), &cp, why))
            return false;
        CdcGeom g = cdc_geometry(n, cp);
        const uint64_t cap = cdc_max_chunks(n, cp);
        p->d2h = 8 + 24 * cap;
        p->out_region = al(p->d2h, 256);
        p->ws_region = al(g.total, 256);
        if (j) {
            j->cp = cp;
            j->g = g;
            j->cap = cap;
        }
        break;
    }
    default:
        *why = "unknown kernel id";
        return false;
    }
    return true;
}

// Jobs dispatched together: their copy-ins go back to back on the copy-in
// stream, then one compute stream runs their kernels and their copy-outs, and
// one event marks the batch done.  With a job-table slot, direct-hashing jobs
// of the same segment size share one segment launch, and all serial chains
// of the batch -- the roots of those direct jobs and the chunk digests of
// every chunking job -- run in one chains launch, so the batch waits for its
// longest chain rather than for the sum of its jobs' chains.
struct Batch {
    std::vector<Job *> jobs;
    int stream = 0;
    int in_stream = 0; // copy-in stream
    uint64_t est_us = 0; // estimated serial time on its compute stream
    hipEvent_t ev_in = nullptr, ev = nullptr;
    int slot = -1; // job-table slot
};

// Job-table slots: pinned host staging + device copy, one per batch in flight.
// Arrays of kMaxBatch + 1 words: direct (MD5) group off, len, seg_base,
// out_off; chunking jobs in_off, out_off, ord_off, cap, lane0; SHA-1 direct
// group off, len, seg_base, out_off.
constexpr uint32_t kMaxBatch = 32;
constexpr size_t kLoneMaxBytes = (size_t)1 << 20;
constexpr size_t kTabN = kMaxBatch + 1;
constexpr size_t kSlotWords = 13 * kTabN;
constexpr size_t kSlotBytes = 8 * kSlotWords;

struct Lib {
    crystal_config cfg;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_dispatch, cv_done, cv_pool;
    std::vector<std::unique_ptr<std::condition_variable>> cv_stream;
    std::deque<Job *> outstanding;
    std::vector<std::deque<Batch *>> running;
    std::vector<uint64_t> load_us; // per compute stream: sum of its running batches' est_us
    RangeAlloc dev_alloc, host_alloc;
    uint8_t *dev_slab = nullptr, *host_slab = nullptr;
    bool own_dev = false;
    std::vector<hipStream_t> streams_in; // copy-in stage, batches rotate over them
    std::vector<hipStream_t> streams; // compute (+ copy-out) stages
    bool own_streams = false;
    std::vector<hipEvent_t> events;
    std::vector<hipEvent_t> free_events;
    uint64_t *table_host = nullptr, *table_dev = nullptr;
    std::vector<int> free_slots;
    std::set<crystal_buf *> bufs;
    std::thread dispatcher;
    std::vector<std::thread> completers;
    bool stop_dispatch = false, stop_complete = false;
    uint32_t inflight = 0;
    uint32_t rr = 0, rr_in = 0;
    uint64_t submitted = 0, completed = 0, failed = 0, bytes_in = 0, bytes_out = 0;
};

static std::mutex g_init_mu;
static Lib *g_lib = nullptr;

// The done flag lives in task->internal[1]; status is written before the
// callback runs, done after it returns, so a finished task may be freed.
static inline int *done_flag(const crystal_task *t)
{
    return reinterpret_cast<int *>(const_cast<void **>(&t->internal[1]));
}

static void finish_task(Lib *L, crystal_task *t, int status)
{
    t->t_done_ns = now_ns();
    t->status = status;
    if (t->callback)
        t->callback(t, t->user);
    {
        std::lock_guard<std::mutex> lk(L->mu);
        __atomic_store_n(done_flag(t), 1, __ATOMIC_RELEASE);
    }
    L->cv_done.notify_all();
}

// Serial time a batch holds its compute stream, in microseconds: its longest
// chain at about 0.6 us per compression (a direct job's segment plus its root
// over the segment digests; a chunking job's longest possible chunk; a
// whole-message MD5), plus a few microseconds of launches per job.  A 64 MiB
// direct job's root alone is 4097 compressions, about 2.5 ms.
static uint64_t batch_est_us(const Batch *b)
{
    uint64_t chain = 0;
    for (const Job *j : b->jobs) {
        uint64_t c = 0;
        switch (j->kernel) {
        case CRYSTAL_K_MD5_DIRECT:
        case CRYSTAL_K_SHA1_DIRECT: {
            const uint64_t nseg = (j->n + j->seg_bytes - 1) / j->seg_bytes;
            const bool md5 = j->kernel == CRYSTAL_K_MD5_DIRECT;
            c = j->seg_bytes / 64 + 1 + (md5 ? 16 : 20) * nseg / 64 + 1;
            if (!md5)
                c = c * 19 / 10; // a SHA-1 compression: 613 ops against MD5's 324
            break;
        }
        case CRYSTAL_K_CDC:
            c = (j->n < j->cp.max_len ? j->n : j->cp.max_len) / 64 + 1;
            break;
        case CRYSTAL_K_MD5:
            c = j->n / 64 + 1;
            break;
        default:
            break;
        }
        chain = std::max(chain, c);
    }
    return chain * 6 / 10 + 5 * b->jobs.size();
}

// The compute stream with the least estimated work queued (ties: fewer
// batches, then round robin).  Counting batches alone sent small jobs behind
// a large direct job's root chain, which holds its stream for milliseconds.
static int pick_stream(Lib *L)
{
    const int S = (int)L->streams.size();
    int best = -1;
    uint64_t best_w = 0;
    size_t best_n = 0;
    for (int k = 0; k < S; k++) {
        const int s = (int)((L->rr + k) % S);
        const uint64_t w = L->load_us[s];
        const size_t q = L->running[s].size();
        if (best < 0 || w < best_w || (w == best_w && q < best_n)) {
            best = s;
            best_w = w;
            best_n = q;
        }
    }
    L->rr = (L->rr + 1) % S;
    return best;
}

// Enqueue one batch: copy-ins (and the batch's job table) on its copy-in
// stream, an event there, and on the batch's compute stream: wait for that
// event, kernels, copy-outs, the completion event.  Batches rotate over the
// copy-in streams (crystal_init picks how many): one stream's copies run
// back to back, each paying a fixed cost, while copies on two or more
// streams overlap those costs and come closer to the link's rate (8 MiB
// copies alone: 52 GB/s on one stream, 53-57 on two to four; 64 MiB copies:
// 57 GB/s either way).  More streams than the process has hardware queues
// make streams share a queue, where a copy can wait behind another stream's
// kernels.
//
// A lone batch (one job of at most kLoneMaxBytes while nothing else runs)
// takes no job-table slot: its kernels use the one-job launches, which saves
// the table's copy (about 7 us on a 1 MiB job).  Its copy-in stays on the
// copy-in stream: moving it to the compute stream saved a little more alone
// but made the serving mix slower (its copies then share the link with later
// arrivals' instead of going first).
static hipError_t enqueue_batch(Lib *L, Batch *b)
{
    hipStream_t st = L->streams[b->stream];
    hipError_t e = hipSuccess;
    for (Job *j : b->jobs) {
        if (j->n && e == hipSuccess)
            e = hipMemcpyAsync(L->dev_slab + j->dev_off, j->in->host, j->n,
                               hipMemcpyHostToDevice, L->streams_in[b->in_stream]);
    }
    // grouped work needs a table slot: direct jobs with the first direct
    // job's segment size, and every chunking job
    std::vector<Job *> group, cdc, sgroup;
    if (b->slot >= 0) {
        for (Job *j : b->jobs) {
            if (j->kernel == CRYSTAL_K_MD5_DIRECT &&
                (group.empty() || j->seg_bytes == group[0]->seg_bytes))
                group.push_back(j);
            else if (j->kernel == CRYSTAL_K_SHA1_DIRECT &&
                     (sgroup.empty() || j->seg_bytes == sgroup[0]->seg_bytes))
                sgroup.push_back(j);
            else if (j->kernel == CRYSTAL_K_CDC)
                cdc.push_back(j);
        }
    }
    uint64_t total_seg = 0, chunk_lanes = 0, sha_seg = 0;
    uint64_t *dtab = nullptr;
    if ((!group.empty() || !cdc.empty() || !sgroup.empty()) && e == hipSuccess) {
        uint64_t *h = L->table_host + (size_t)b->slot * kSlotWords;
        dtab = L->table_dev + (size_t)b->slot * kSlotWords;
        uint64_t *h_off = h, *h_len = h + kTabN, *h_base = h + 2 * kTabN,
                 *h_out = h + 3 * kTabN;
        for (size_t k = 0; k < group.size(); k++) {
            Job *j = group[k];
            h_off[k] = j->dev_off;
            h_len[k] = j->n;
            h_base[k] = total_seg;
            h_out[k] = j->dev_off + j->in_region;
            total_seg += (j->n + j->seg_bytes - 1) / j->seg_bytes;
        }
        h_base[group.size()] = total_seg;
        uint64_t *c_in = h + 4 * kTabN, *c_out = h + 5 * kTabN, *c_ord = h + 6 * kTabN,
                 *c_cap = h + 7 * kTabN, *c_lane0 = h + 8 * kTabN;
        for (size_t k = 0; k < cdc.size(); k++) {
            Job *j = cdc[k];
            const size_t out_off = j->dev_off + j->in_region;
            c_in[k] = j->dev_off;
            c_out[k] = out_off;
            // where launch_chunk_order leaves the order (it makes none for
            // empty inputs)
            const uint64_t m = j->cap < j->g.ord_cap ? j->cap : j->g.ord_cap;
            c_ord[k] = (j->n && m) ? out_off + al(j->d2h, 256) + j->g.off_ord : kNoOrder;
            c_cap[k] = j->cap;
            c_lane0[k] = chunk_lanes;
            chunk_lanes += al(j->cap, 64);
        }
        c_lane0[cdc.size()] = chunk_lanes;
        uint64_t *s_off = h + 9 * kTabN, *s_len = h + 10 * kTabN, *s_base = h + 11 * kTabN,
                 *s_out = h + 12 * kTabN;
        for (size_t k = 0; k < sgroup.size(); k++) {
            Job *j = sgroup[k];
            s_off[k] = j->dev_off;
            s_len[k] = j->n;
            s_base[k] = sha_seg;
            s_out[k] = j->dev_off + j->in_region;
            sha_seg += (j->n + j->seg_bytes - 1) / j->seg_bytes;
        }
        s_base[sgroup.size()] = sha_seg;
        e = hipMemcpyAsync(dtab, h, kSlotBytes, hipMemcpyHostToDevice,
                           L->streams_in[b->in_stream]);
    }
    if (e == hipSuccess)
        e = hipEventRecord(b->ev_in, L->streams_in[b->in_stream]);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(st, b->ev_in, 0);
    if (e != hipSuccess)
        return e;
    JobTable gjt{nullptr, nullptr, nullptr, 0, 0};
    if (!group.empty()) {
        gjt = JobTable{dtab, dtab + kTabN, dtab + 2 * kTabN, (uint32_t)group.size(), 0,
                       dtab + 3 * kTabN};
        e = launch_md5_segments(L->dev_slab, gjt, group[0]->seg_bytes, total_seg, L->dev_slab,
                                st);
        if (e != hipSuccess)
            return e;
    }
    if (!sgroup.empty()) {
        // SHA-1 direct jobs: one segment launch and one root launch for the group
        const JobTable sjt{dtab + 9 * kTabN, dtab + 10 * kTabN, dtab + 11 * kTabN,
                           (uint32_t)sgroup.size(), 0, dtab + 12 * kTabN};
        e = launch_sha1_segments(L->dev_slab, sjt, sgroup[0]->seg_bytes, sha_seg, L->dev_slab,
                                 st);
        if (e == hipSuccess)
            e = launch_sha1_roots(L->dev_slab, sjt, sgroup[0]->seg_bytes, L->dev_slab, st);
        if (e != hipSuccess)
            return e;
    }
    for (Job *j : b->jobs) {
        uint8_t *d_in = L->dev_slab + j->dev_off;
        uint8_t *d_out = d_in + j->in_region;
        switch (j->kernel) {
        case CRYSTAL_K_NOP:
            e = launch_nop(st);
            d_out = d_in;
            break;
        case CRYSTAL_K_MD5:
            e = launch_md5_whole(d_in, j->n, d_out, st);
            break;
        case CRYSTAL_K_MD5_DIRECT: {
            if (std::find(group.begin(), group.end(), j) != group.end())
                break; // segments above, root in the chains launch
            JobTable jt{nullptr, nullptr, nullptr, 0, j->n};
            const uint64_t nseg = (j->n + j->seg_bytes - 1) / j->seg_bytes;
            e = launch_md5_segments(d_in, jt, j->seg_bytes, nseg, d_out, st);
            if (e == hipSuccess)
                e = launch_md5_roots(d_out, jt, j->seg_bytes, d_out + 16 * nseg, st);
            break;
        }
        case CRYSTAL_K_SHA1_DIRECT: {
            if (std::find(sgroup.begin(), sgroup.end(), j) != sgroup.end())
                break; // hashed by the group launches above
            JobTable jt{nullptr, nullptr, nullptr, 0, j->n};
            const uint64_t nseg = (j->n + j->seg_bytes - 1) / j->seg_bytes;
            e = launch_sha1_segments(d_in, jt, j->seg_bytes, nseg, d_out, st);
            if (e == hipSuccess)
                e = launch_sha1_roots(d_out, jt, j->seg_bytes, d_out + 20 * nseg, st);
            break;
        }
        case CRYSTAL_K_CDC: {
            uint8_t *d_ws = d_out + al(j->d2h, 256);
            uint64_t *cnt = reinterpret_cast<uint64_t *>(d_out);
            uint64_t *ends = cnt + 1;
            e = launch_cdc_candidates(d_in, j->g, j->cp, d_ws, st);
            const uint32_t *order = nullptr;
            if (e == hipSuccess)
                e = launch_cdc_select(j->g, j->cp, d_ws, cnt, ends, j->cap, st, &order);
            const bool chained = std::find(cdc.begin(), cdc.end(), j) != cdc.end();
            if (e == hipSuccess && !chained)
                e = launch_md5_chunks(d_in, ends, cnt, j->cap, order, nullptr, st);
            break;
        }
        }
        if (e != hipSuccess)
            return e;
        j->d_out_ptr = d_out;
    }
    if (!group.empty() || !cdc.empty()) {
        const ChainTable ct{dtab + 4 * kTabN, dtab + 5 * kTabN, dtab + 6 * kTabN,
                            dtab + 7 * kTabN, dtab + 8 * kTabN, (uint32_t)cdc.size()};
        e = launch_md5_chains(L->dev_slab, gjt, group.empty() ? 0 : group[0]->seg_bytes, ct,
                              chunk_lanes, st);
        if (e != hipSuccess)
            return e;
    }
    for (Job *j : b->jobs) {
        if (j->d2h) {
            e = hipMemcpyAsync(j->out->host, j->d_out_ptr, j->d2h, hipMemcpyDeviceToHost, st);
            if (e != hipSuccess)
                return e;
        }
    }
    return hipEventRecord(b->ev, st);
}

// Caller holds L->mu.
static void release_batch_resources(Lib *L, Batch *b)
{
    for (Job *j : b->jobs) {
        L->dev_alloc.release(j->dev_off, j->need);
        L->inflight--;
        j->in->refs--;
        j->out->refs--;
    }
    L->free_events.push_back(b->ev);
    L->free_events.push_back(b->ev_in);
    if (b->slot >= 0)
        L->free_slots.push_back(b->slot);
}

static void dispatcher_main(Lib *L)
{
    (void)hipSetDevice(L->device);
    std::unique_lock<std::mutex> lk(L->mu);
    for (;;) {
        if (L->stop_dispatch)
            break;
        // admit the FIFO head and as many following jobs as fit right now
        Batch *b = new Batch;
        while (!L->outstanding.empty() && b->jobs.size() < kMaxBatch) {
            Job *j = L->outstanding.front();
            size_t off = 0;
            if (L->inflight >= L->cfg.max_in_flight || !L->dev_alloc.alloc(j->need, &off))
                break;
            L->outstanding.pop_front();
            L->inflight++;
            j->dev_off = off;
            b->jobs.push_back(j);
        }
        if (b->jobs.empty()) {
            delete b;
            L->cv_dispatch.wait(lk); // new work or a completion frees room
            continue;
        }
        // batches <= jobs in flight, so the pools below always have entries
        b->ev = L->free_events.back();
        L->free_events.pop_back();
        b->ev_in = L->free_events.back();
        L->free_events.pop_back();
        bool idle = true;
        for (const auto &q : L->running)
            idle = idle && q.empty();
        // a lone batch (see enqueue_batch) takes no table slot
        const bool lone = idle && b->jobs.size() == 1 && b->jobs[0]->n <= kLoneMaxBytes;
        if (!lone && !L->free_slots.empty()) {
            b->slot = L->free_slots.back();
            L->free_slots.pop_back();
        }
        b->est_us = batch_est_us(b);
        b->stream = pick_stream(L);
        L->load_us[b->stream] += b->est_us;
        b->in_stream = (int)(L->rr_in++ % L->streams_in.size());
        for (Job *j : b->jobs) {
            j->stream = b->stream;
            j->t->stream_index = b->stream;
        }
        lk.unlock();
        const int64_t ta = now_ns();
        for (Job *j : b->jobs)
            j->t->t_admit_ns = ta;
        hipError_t e = enqueue_batch(L, b);
        if (e != hipSuccess) {
            // drain whatever was enqueued before releasing the regions
            (void)hipStreamSynchronize(L->streams_in[b->in_stream]);
            (void)hipStreamSynchronize(L->streams[b->stream]);
            set_error(CRYSTAL_EDEVICE, "job enqueue: %s", hipGetErrorString(e));
            lk.lock();
            L->load_us[b->stream] -= b->est_us;
            release_batch_resources(L, b);
            L->failed += b->jobs.size();
            lk.unlock();
            for (Job *j : b->jobs) {
                finish_task(L, j->t, CRYSTAL_EDEVICE);
                delete j;
            }
            delete b;
            lk.lock();
            continue;
        }
        lk.lock();
        L->running[b->stream].push_back(b);
        L->cv_stream[b->stream]->notify_one();
    }
}

static void completer_main(Lib *L, int s)
{
    (void)hipSetDevice(L->device);
    std::unique_lock<std::mutex> lk(L->mu);
    for (;;) {
        if (L->running[s].empty()) {
            if (L->stop_complete)
                break;
            L->cv_stream[s]->wait(lk);
            continue;
        }
        Batch *b = L->running[s].front();
        lk.unlock();
        hipError_t e = hipEventSynchronize(b->ev);
        std::vector<int> status(b->jobs.size(), CRYSTAL_OK);
        for (size_t k = 0; k < b->jobs.size(); k++) {
            Job *j = b->jobs[k];
            size_t out_bytes = j->d2h;
            if (e != hipSuccess) {
                status[k] = CRYSTAL_EDEVICE;
            } else if (j->kernel == CRYSTAL_K_CDC) {
                uint64_t nc;
                memcpy(&nc, j->out->host, 8);
                if (nc > j->cap)
                    status[k] = CRYSTAL_EDEVICE;
                else
                    out_bytes = 8 + 24 * nc;
            }
            j->t->out_bytes = status[k] == CRYSTAL_OK ? out_bytes : 0;
        }
        if (e != hipSuccess)
            set_error(CRYSTAL_EDEVICE, "job execution: %s", hipGetErrorString(e));
        lk.lock();
        L->running[s].pop_front();
        L->load_us[s] -= b->est_us;
        release_batch_resources(L, b);
        for (size_t k = 0; k < b->jobs.size(); k++) {
            if (status[k] == CRYSTAL_OK) {
                L->completed++;
                L->bytes_in += b->jobs[k]->n;
                L->bytes_out += b->jobs[k]->t->out_bytes;
            } else {
                L->failed++;
            }
        }
        lk.unlock();
        L->cv_dispatch.notify_one();
        for (size_t k = 0; k < b->jobs.size(); k++) {
            finish_task(L, b->jobs[k]->t, status[k]);
            delete b->jobs[k];
        }
        delete b;
        lk.lock();
    }
}

// HIP resources of a library instance that init created (or got as far as
// creating); null handles are skipped.  Threads must be stopped already.
static void release_resources(Lib *L)
{
    (void)hipSetDevice(L->device);
    for (hipEvent_t ev : L->events)
        (void)hipEventDestroy(ev);
    L->events.clear();
    if (L->own_streams) {
        for (hipStream_t s : L->streams_in)
            if (s)
                (void)hipStreamDestroy(s);
        for (hipStream_t s : L->streams)
            if (s)
                (void)hipStreamDestroy(s);
    }
    if (L->own_dev && L->dev_slab)
        (void)hipFree(L->dev_slab);
    if (L->host_slab)
        (void)hipHostFree(L->host_slab);
    if (L->table_host)
        (void)hipHostFree(L->table_host);
    if (L->table_dev)
        (void)hipFree(L->table_dev);
    L->dev_slab = L->host_slab = nullptr;
    L->table_host = L->table_dev = nullptr;
}

static Lib *lib_or_fail()
{
    Lib *L = g_lib;
    if (!L)
        fail(CRYSTAL_ESTATE, "library not initialised (crystal_init)");
    return L;
}

} // namespace crystal

using namespace crystal;

extern "C" {

size_t crystal_output_bytes(int kernel_id, size_t in_bytes, const void *params)
{
    JobPlan p;
    const char *why = "";
    if (!plan_job(kernel_id, in_bytes, params, nullptr, &p, &why))
        return 0;
    return p.d2h;
}

int crystal_init(const crystal_config *cfg_in)
{
    std::lock_guard<std::mutex> g(g_init_mu);
    if (g_lib)
        return fail(CRYSTAL_ESTATE, "already initialised");
    if (!cfg_in || cfg_in->max_input_bytes == 0)
        return fail(CRYSTAL_EINVAL, "max_input_bytes must be > 0");
    crystal_config cfg = *cfg_in;
    if (cfg.n_streams == 0)
        cfg.n_streams = 3;
    if (cfg.n_streams > 64)
        return fail(CRYSTAL_EINVAL, "n_streams must be <= 64");
    if (cfg.n_copy_streams == 0) {
        // A second copy-in stream only where the process has a hardware queue
        // for it (GPU_MAX_HW_QUEUES, HIP's default 4): past that, streams
        // share queues and a copy can wait behind another stream's kernels.
        // Measured: 256 x 8 MiB host-fed jobs on 2 compute streams ran at
        // 48.5-49.7 GB/s with 2 copy-in streams against 42-45 with one; the
        // serving mix on 3 compute streams fell from 47 to 35 GB/s with 2.
        uint32_t hwq = 4;
        if (const char *v = getenv("GPU_MAX_HW_QUEUES"))
            if (atoi(v) > 0)
                hwq = (uint32_t)atoi(v);
        cfg.n_copy_streams = (!cfg.streams && cfg.n_streams + 2 <= hwq) ? 2 : 1;
    }
    if (cfg.n_copy_streams > 8)
        return fail(CRYSTAL_EINVAL, "n_copy_streams must be <= 8");
    if (cfg.max_in_flight == 0)
        cfg.max_in_flight = 4 * cfg.n_streams;
    // largest output and device need over all kernels for the largest input
    size_t max_out = 0, max_need = 0;
    for (int k = 0; k <= CRYSTAL_K_SHA1_DIRECT; k++) {
        JobPlan p;
        const char *why;
        if (plan_job(k, cfg.max_input_bytes, nullptr, nullptr, &p, &why)) {
            max_out = std::max(max_out, p.d2h);
            max_need = std::max(max_need, p.in_region + p.out_region + p.ws_region);
        }
    }
    if (cfg.max_output_bytes == 0)
        cfg.max_output_bytes = max_out;
    if (cfg.host_pool_bytes == 0)
        cfg.host_pool_bytes = 4 * (cfg.max_input_bytes + cfg.max_output_bytes);
    if (cfg.device_pool_bytes == 0)
        cfg.device_pool_bytes = std::max<size_t>(8 * max_need, 256ull << 20);
    cfg.host_pool_bytes = al(cfg.host_pool_bytes, 4096);
    cfg.device_pool_bytes &= ~(size_t)255;

    std::unique_ptr<Lib> L(new Lib);
    L->cfg = cfg;
    L->device = cfg.device;
    // on any failure below, what was created so far is released
    auto bail = [&](int rc) {
        release_resources(L.get());
        return rc;
    };
    hipError_t e = hipSetDevice(cfg.device);
    if (e != hipSuccess)
        return hip_fail(e, "hipSetDevice");
    if (cfg.device_slab) {
        L->dev_slab = static_cast<uint8_t *>(cfg.device_slab);
    } else {
        e = hipMalloc((void **)&L->dev_slab, cfg.device_pool_bytes);
        if (e != hipSuccess) {
            L->dev_slab = nullptr;
            return bail(fail(CRYSTAL_ENOMEM, "device slab of %zu bytes: %s",
                             cfg.device_pool_bytes, hipGetErrorString(e)));
        }
        L->own_dev = true;
    }
    e = hipHostMalloc((void **)&L->host_slab, cfg.host_pool_bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        L->host_slab = nullptr;
        return bail(fail(CRYSTAL_ENOMEM, "pinned host slab of %zu bytes: %s",
                         cfg.host_pool_bytes, hipGetErrorString(e)));
    }
    L->dev_alloc.reset(cfg.device_pool_bytes);
    L->host_alloc.reset(cfg.host_pool_bytes);
    L->streams.assign(cfg.n_streams, nullptr);
    L->streams_in.assign(cfg.n_copy_streams, nullptr);
    const uint32_t K = cfg.n_copy_streams;
    if (cfg.streams) {
        for (uint32_t s = 0; s < K; s++)
            L->streams_in[s] = static_cast<hipStream_t>(cfg.streams[s]);
        for (uint32_t s = 0; s < cfg.n_streams; s++)
            L->streams[s] = static_cast<hipStream_t>(cfg.streams[K + s]);
    } else {
        L->own_streams = true;
        for (uint32_t s = 0; s < K && e == hipSuccess; s++)
            if ((e = hipStreamCreateWithFlags(&L->streams_in[s], hipStreamNonBlocking)) !=
                hipSuccess)
                L->streams_in[s] = nullptr;
        for (uint32_t s = 0; s < cfg.n_streams && e == hipSuccess; s++)
            if ((e = hipStreamCreateWithFlags(&L->streams[s], hipStreamNonBlocking)) !=
                hipSuccess)
                L->streams[s] = nullptr;
        if (e != hipSuccess)
            return bail(hip_fail(e, "hipStreamCreate"));
    }
    const uint32_t n_ev = 2 * (cfg.max_in_flight + 1);
    for (uint32_t i = 0; i < n_ev; i++) {
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess)
            return bail(hip_fail(e, "hipEventCreate"));
        L->events.push_back(ev);
        L->free_events.push_back(ev);
    }
    const uint32_t n_slots = cfg.max_in_flight + 1;
    e = hipHostMalloc((void **)&L->table_host, n_slots * kSlotBytes, hipHostMallocDefault);
    if (e != hipSuccess)
        L->table_host = nullptr;
    if (e == hipSuccess && (e = hipMalloc((void **)&L->table_dev, n_slots * kSlotBytes)) !=
                               hipSuccess)
        L->table_dev = nullptr;
    if (e != hipSuccess)
        return bail(fail(CRYSTAL_ENOMEM, "job-table ring: %s", hipGetErrorString(e)));
    for (uint32_t i = 0; i < n_slots; i++)
        L->free_slots.push_back((int)i);
    L->running.resize(cfg.n_streams);
    L->load_us.assign(cfg.n_streams, 0);
    for (uint32_t s = 0; s < cfg.n_streams; s++)
        L->cv_stream.emplace_back(new std::condition_variable);
    Lib *raw = L.release();
    raw->dispatcher = std::thread(dispatcher_main, raw);
    for (uint32_t s = 0; s < cfg.n_streams; s++)
        raw->completers.emplace_back(completer_main, raw, (int)s);
    g_lib = raw;
    return CRYSTAL_OK;
}

int crystal_finalize(void)
{
    std::lock_guard<std::mutex> g(g_init_mu);
    Lib *L = g_lib;
    if (!L)
        return fail(CRYSTAL_ESTATE, "not initialised");
    std::deque<Job *> cancelled;
    {
        std::lock_guard<std::mutex> lk(L->mu);
        L->stop_dispatch = true;
        cancelled.swap(L->outstanding);
    }
    L->cv_dispatch.notify_all();
    L->dispatcher.join();
    for (Job *j : cancelled) {
        {
            std::lock_guard<std::mutex> lk(L->mu);
            j->in->refs--;
            j->out->refs--;
            L->failed++;
        }
        finish_task(L, j->t, CRYSTAL_ECANCELED);
        delete j;
    }
    {
        std::lock_guard<std::mutex> lk(L->mu);
        L->stop_complete = true;
    }
    for (auto &cv : L->cv_stream)
        cv->notify_all();
    for (auto &th : L->completers)
        th.join();
    release_resources(L);
    for (crystal_buf *b : L->bufs)
        delete b;
    g_lib = nullptr;
    delete L;
    return CRYSTAL_OK;
}

int crystal_buffer_acquire(size_t bytes, int flags, crystal_buf **out)
{
    Lib *L = lib_or_fail();
    if (!L)
        return CRYSTAL_ESTATE;
    if (!out)
        return fail(CRYSTAL_EINVAL, "out is NULL");
    const size_t len = al(bytes ? bytes : 1, 4096);
    if (len > L->host_alloc.size())
        return fail(CRYSTAL_EINVAL, "%zu bytes exceed the host pool (%zu)", bytes,
                    L->host_alloc.size());
    std::unique_lock<std::mutex> lk(L->mu);
    size_t off;
    while (!L->host_alloc.alloc(len, &off)) {
        if (flags & CRYSTAL_NONBLOCK)
            return fail(CRYSTAL_EAGAIN, "host pool exhausted");
        if (L->stop_dispatch)
            return fail(CRYSTAL_ESTATE, "finalizing");
        L->cv_pool.wait(lk);
    }
    crystal_buf *b = new crystal_buf;
    b->host = L->host_slab + off;
    b->size = bytes;
    b->pool_off = off;
    b->pool_len = len;
    b->pooled = true;
    b->refs = 0;
    L->bufs.insert(b);
    *out = b;
    return CRYSTAL_OK;
}

int crystal_buffer_wrap(void *host_ptr, size_t bytes, crystal_buf **out)
{
    Lib *L = lib_or_fail();
    if (!L)
        return CRYSTAL_ESTATE;
    if (!out || (!host_ptr && bytes))
        return fail(CRYSTAL_EINVAL, "null pointer argument");
    crystal_buf *b = new crystal_buf;
    b->host = host_ptr;
    b->size = bytes;
    b->pool_off = b->pool_len = 0;
    b->pooled = false;
    b->refs = 0;
    std::lock_guard<std::mutex> lk(L->mu);
    L->bufs.insert(b);
    *out = b;
    return CRYSTAL_OK;
}

int crystal_buffer_release(crystal_buf *b)
{
    Lib *L = lib_or_fail();
    if (!L)
        return CRYSTAL_ESTATE;
    if (!b)
        return fail(CRYSTAL_EINVAL, "buffer is NULL");
    {
        std::lock_guard<std::mutex> lk(L->mu);
        if (!L->bufs.count(b))
            return fail(CRYSTAL_EINVAL, "unknown buffer");
        if (b->refs.load() > 0)
            return fail(CRYSTAL_EBUSY, "buffer in use by an unfinished task");
        if (b->pooled)
            L->host_alloc.release(b->pool_off, b->pool_len);
        L->bufs.erase(b);
    }
    const bool pooled = b->pooled;
    delete b;
    if (pooled)
        L->cv_pool.notify_all();
    return CRYSTAL_OK;
}

void *crystal_buffer_host(crystal_buf *b) { return b ? b->host : nullptr; }
size_t crystal_buffer_size(const crystal_buf *b) { return b ? b->size : 0; }

int crystal_submit(crystal_task *t, int kernel_id, crystal_buf *in, crystal_buf *out)
{
    Lib *L = lib_or_fail();
    if (!L)
        return CRYSTAL_ESTATE;
    if (!t || !in || !out)
        return fail(CRYSTAL_EINVAL, "task, in and out are required");
    const size_t n = t->in_bytes;
    if (n > in->size)
        return fail(CRYSTAL_EINVAL, "in_bytes %zu > input buffer %zu", n, in->size);
    if (n > L->cfg.max_input_bytes)
        return fail(CRYSTAL_EINVAL, "in_bytes %zu > max_input_bytes %zu", n,
                    L->cfg.max_input_bytes);
    Job *j = new Job();
    JobPlan p;
    const char *why = "";
    if (!plan_job(kernel_id, n, t->params, j, &p, &why)) {
        delete j;
        return fail(CRYSTAL_EINVAL, "%s", why);
    }
    if (out->size < p.d2h) {
        delete j;
        return fail(CRYSTAL_EINVAL, "output buffer %zu < required %zu", out->size, p.d2h);
    }
    j->t = t;
    j->kernel = kernel_id;
    j->in = in;
    j->out = out;
    j->n = n;
    j->in_region = p.in_region;
    j->need = p.in_region + p.out_region + p.ws_region;
    j->d2h = p.d2h;
    if (j->need > L->dev_alloc.size()) {
        delete j;
        return fail(CRYSTAL_EINVAL, "job needs %zu device bytes > pool %zu", j->need,
                    L->dev_alloc.size());
    }
    t->status = CRYSTAL_PENDING;
    t->out_bytes = 0;
    t->stream_index = -1;
    t->t_admit_ns = t->t_done_ns = 0;
    __atomic_store_n(done_flag(t), 0, __ATOMIC_RELEASE);
    t->internal[0] = j;
    t->t_submit_ns = now_ns();
    {
        std::lock_guard<std::mutex> lk(L->mu);
        if (L->stop_dispatch) {
            delete j;
            return fail(CRYSTAL_ESTATE, "finalizing");
        }
        in->refs++;
        out->refs++;
        L->outstanding.push_back(j);
        L->submitted++;
    }
    L->cv_dispatch.notify_one();
    return CRYSTAL_OK;
}

int crystal_poll(const crystal_task *t)
{
    if (!t)
        return fail(CRYSTAL_EINVAL, "task is NULL");
    if (!__atomic_load_n(done_flag(t), __ATOMIC_ACQUIRE))
        return 0;
    return t->status == CRYSTAL_OK ? 1 : t->status;
}

int crystal_wait(crystal_task *t, int64_t timeout_ns)
{
    Lib *L = lib_or_fail();
    if (!L)
        return CRYSTAL_ESTATE;
    if (!t)
        return fail(CRYSTAL_EINVAL, "task is NULL");
    std::unique_lock<std::mutex> lk(L->mu);
    auto done = [&] { return __atomic_load_n(done_flag(t), __ATOMIC_ACQUIRE) != 0; };
    if (timeout_ns < 0) {
        L->cv_done.wait(lk, done);
    } else if (!L->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done)) {
        return fail(CRYSTAL_ETIMEDOUT, "task not finished within %lld ns",
                    (long long)timeout_ns);
    }
    return t->status;
}

int crystal_get_stats(crystal_stats *s)
{
    Lib *L = lib_or_fail();
    if (!L)
        return CRYSTAL_ESTATE;
    if (!s)
        return fail(CRYSTAL_EINVAL, "stats is NULL");
    std::lock_guard<std::mutex> lk(L->mu);
    s->submitted = L->submitted;
    s->completed = L->completed;
    s->failed = L->failed;
    s->bytes_in = L->bytes_in;
    s->bytes_out = L->bytes_out;
    s->device_pool_bytes = L->dev_alloc.size();
    s->device_pool_free = L->dev_alloc.free_bytes();
    s->device_pool_min_free = L->dev_alloc.min_free();
    s->host_pool_bytes = L->host_alloc.size();
    s->host_pool_free = L->host_alloc.free_bytes();
    s->outstanding = (uint32_t)L->outstanding.size();
    uint32_t r = 0;
    for (auto &q : L->running)
        r += (uint32_t)q.size();
    s->running = r;
    return CRYSTAL_OK;
}

} // extern "C"
