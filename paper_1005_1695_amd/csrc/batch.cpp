// Batch plans: the batch-processing application class of Sec. 2.2 (many
// independent buffers available at once, throughput first).  A plan orders
// the buffers longest-first and replays a persistent MD5 launch (optionally
// split over several streams as parallel branches joined by events).  The
// tuner times every candidate configuration by replay.
//
// Replay uses direct stream launches.  Capturing the same sequence into a HIP
// graph (capture() below) is switched off: under the HIP runtime that PyTorch
// loads into the process, a plan built that way ended in a host segmentation
// fault whose cause has not been identified, so that path is not run.
#include <algorithm>
#include <numeric>
#include <string.h>
#include <vector>

#include "internal.h"

using namespace crystal;

struct crystal_batch {
    crystal_batch_desc d;
    int device;
    uint32_t n_simd;
    std::vector<uint32_t> len;     // host copy of the lengths
    uint32_t order_window = 0;     // sort window the device order holds
    uint32_t *d_order = nullptr;
    uint32_t *d_counters = nullptr;
    std::vector<uint64_t> work_prefix; // compressions, prefix over sorted order
    hipStream_t cap[8] = {};
    hipEvent_t ev[9] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    crystal_batch_tuning tun;
};

static const uint32_t kMaxBranches = 8;
static const bool kGraphReplay = false; // see the header comment

static void destroy_graph(crystal_batch *b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

static hipError_t set_order(crystal_batch *b, uint32_t W);

// Capture zero-counter + persistent kernel per branch.  Branch i covers a
// contiguous slice of the order holding about 1/S of the total work.
static hipError_t capture(crystal_batch *b, const crystal_batch_tuning &t)
{
    destroy_graph(b);
    const uint32_t S = t.n_streams;
    const uint64_t n = b->d.n_buf;
    const uint32_t waves = b->n_simd * t.waves_per_simd;
    uint32_t grid = (uint32_t)((uint64_t)waves * 64 / t.block);
    if (grid == 0)
        grid = 1;
    const uint32_t *order = t.sorted ? b->d_order : nullptr;
    hipError_t e = t.sorted ? set_order(b, t.sorted) : hipSuccess;
    if (e == hipSuccess)
        e = hipStreamBeginCapture(b->cap[0], hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return e;
    if (S > 1) {
        e = hipEventRecord(b->ev[0], b->cap[0]);
        for (uint32_t i = 1; i < S && e == hipSuccess; i++)
            e = hipStreamWaitEvent(b->cap[i], b->ev[0], 0);
    }
    const uint64_t total = b->work_prefix.back();
    uint64_t lo = 0;
    for (uint32_t i = 0; i < S && e == hipSuccess; i++) {
        uint64_t hi = n;
        if (i + 1 < S) {
            const uint64_t target = total * (i + 1) / S;
            hi = std::lower_bound(b->work_prefix.begin(), b->work_prefix.end(), target) -
                 b->work_prefix.begin();
            hi = std::min<uint64_t>(std::max<uint64_t>(hi, lo), n);
        }
        const uint32_t g = std::max<uint32_t>(1, grid / S);
        e = launch_zero_u32(b->d_counters + i, 1, b->cap[i]);
        if (e == hipSuccess && hi > lo) {
            const uint32_t *ord = order ? order + lo : nullptr;
            if (order) {
                e = launch_md5_batch_persistent((const uint8_t *)b->d.d_arena, b->d.d_off,
                                                b->d.d_len, ord, hi - lo,
                                                (uint8_t *)b->d.d_out, b->d_counters + i,
                                                t.grab, t.block, g, b->cap[i]);
            } else {
                // index order: slice offsets directly
                e = launch_md5_batch_persistent((const uint8_t *)b->d.d_arena,
                                                b->d.d_off + lo, b->d.d_len + lo, nullptr,
                                                hi - lo, (uint8_t *)b->d.d_out + 16 * lo,
                                                b->d_counters + i, t.grab, t.block, g,
                                                b->cap[i]);
            }
        }
        lo = hi;
    }
    if (S > 1) {
        for (uint32_t i = 1; i < S && e == hipSuccess; i++) {
            e = hipEventRecord(b->ev[i], b->cap[i]);
            if (e == hipSuccess)
                e = hipStreamWaitEvent(b->cap[0], b->ev[i], 0);
        }
    }
    hipGraph_t gr = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap[0], &gr);
    if (e == hipSuccess)
        e = e2;
    if (e != hipSuccess) {
        if (gr)
            (void)hipGraphDestroy(gr);
        return e;
    }
    b->graph = gr;
    e = hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0);
    return e;
}

// One replay by direct launches on the desc stream (branch i on plan stream
// i, forked from and joined back into the desc stream by events).
static hipError_t launch_direct(crystal_batch *b, const crystal_batch_tuning &t)
{
    hipStream_t s0 = (hipStream_t)b->d.stream;
    const uint32_t S = t.n_streams;
    const uint64_t n = b->d.n_buf;
    const uint32_t waves = b->n_simd * t.waves_per_simd;
    uint32_t grid = (uint32_t)((uint64_t)waves * 64 / t.block);
    if (grid == 0)
        grid = 1;
    const uint32_t *order = t.sorted ? b->d_order : nullptr;
    hipError_t e = hipSuccess;
    if (!t.sorted) { // work prefix of the index order
        uint64_t acc = 0;
        if (b->order_window != 0) {
            for (uint64_t i = 0; i < n; i++) {
                acc += (b->len[i] + 8) / 64 + 1;
                b->work_prefix[i] = acc;
            }
            b->order_window = 0;
        }
    } else {
        e = set_order(b, t.sorted);
    }
    if (S > 1 && e == hipSuccess) {
        e = hipEventRecord(b->ev[0], s0);
        for (uint32_t i = 1; i < S && e == hipSuccess; i++)
            e = hipStreamWaitEvent(b->cap[i], b->ev[0], 0);
    }
    const uint64_t total = b->work_prefix.back();
    uint64_t lo = 0;
    for (uint32_t i = 0; i < S && e == hipSuccess; i++) {
        hipStream_t si = i == 0 ? s0 : b->cap[i];
        uint64_t hi = n;
        if (i + 1 < S) {
            const uint64_t target = total * (i + 1) / S;
            hi = std::lower_bound(b->work_prefix.begin(), b->work_prefix.end(), target) -
                 b->work_prefix.begin();
            hi = std::min<uint64_t>(std::max<uint64_t>(hi, lo), n);
        }
        const uint32_t g = std::max<uint32_t>(1, grid / S);
        e = launch_zero_u32(b->d_counters + i, 1, si);
        if (e == hipSuccess && hi > lo) {
            if (order)
                e = launch_md5_batch_persistent((const uint8_t *)b->d.d_arena, b->d.d_off,
                                                b->d.d_len, order + lo, hi - lo,
                                                (uint8_t *)b->d.d_out, b->d_counters + i,
                                                t.grab, t.block, g, si);
            else
                e = launch_md5_batch_persistent((const uint8_t *)b->d.d_arena,
                                                b->d.d_off + lo, b->d.d_len + lo, nullptr,
                                                hi - lo, (uint8_t *)b->d.d_out + 16 * lo,
                                                b->d_counters + i, t.grab, t.block, g, si);
        }
        lo = hi;
    }
    if (S > 1) {
        for (uint32_t i = 1; i < S && e == hipSuccess; i++) {
            e = hipEventRecord(b->ev[i], b->cap[i]);
            if (e == hipSuccess)
                e = hipStreamWaitEvent(s0, b->ev[i], 0);
        }
    }
    return e;
}

// Lane order for a sort window W: W == 1 sorts the whole batch longest
// first; W > 1 sorts longest first inside each run of W consecutive buffers,
// so the 64 buffers a wave takes have nearly equal lengths (little lockstep
// waste) and still lie close together in the arena.  Also rebuilds the work
// prefix used to split the order across branches.
static hipError_t set_order(crystal_batch *b, uint32_t W)
{
    if (W == 0 || W == b->order_window)
        return hipSuccess;
    const uint64_t n = b->d.n_buf;
    std::vector<uint32_t> order(n);
    std::iota(order.begin(), order.end(), 0u);
    const uint64_t win = W == 1 ? n : W;
    for (uint64_t lo = 0; lo < n; lo += win) {
        const uint64_t hi = std::min<uint64_t>(n, lo + win);
        std::stable_sort(order.begin() + lo, order.begin() + hi,
                         [&](uint32_t x, uint32_t y) { return b->len[x] > b->len[y]; });
    }
    uint64_t acc = 0;
    for (uint64_t i = 0; i < n; i++) {
        acc += (b->len[order[i]] + 8) / 64 + 1;
        b->work_prefix[i] = acc;
    }
    hipError_t e = hipMemcpy(b->d_order, order.data(), 4 * n, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        b->order_window = W;
    return e;
}

static hipError_t replay(crystal_batch *b)
{
    if (kGraphReplay && b->exec)
        return hipGraphLaunch(b->exec, (hipStream_t)b->d.stream);
    return launch_direct(b, b->tun);
}

static hipError_t time_replays(crystal_batch *b, int reps, float *ms)
{
    hipStream_t s = (hipStream_t)b->d.stream;
    hipEvent_t a, z;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&z);
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; i++)
        e = replay(b);
    std::vector<float> v;
    for (int i = 0; i < reps && e == hipSuccess; i++) {
        e = hipEventRecord(a, s);
        if (e == hipSuccess)
            e = replay(b);
        if (e == hipSuccess)
            e = hipEventRecord(z, s);
        if (e == hipSuccess)
            e = hipEventSynchronize(z);
        float t = 0;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&t, a, z);
        v.push_back(t);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(z);
    if (e == hipSuccess) {
        std::sort(v.begin(), v.end());
        *ms = v[v.size() / 2];
    }
    return e;
}

static void free_plan(crystal_batch *b)
{
    destroy_graph(b);
    if (b->d_order)
        (void)hipFree(b->d_order);
    if (b->d_counters)
        (void)hipFree(b->d_counters);
    for (auto &s : b->cap)
        if (s)
            (void)hipStreamDestroy(s);
    for (auto &e : b->ev)
        if (e)
            (void)hipEventDestroy(e);
    delete b;
}

extern "C" {

int crystal_batch_plan(const crystal_batch_desc *d, int tune_flags,
                       const crystal_batch_tuning *fixed, crystal_batch **out)
{
    if (!d || !out || !d->d_arena || !d->d_off || !d->d_len || !d->d_out)
        return fail(CRYSTAL_EINVAL, "descriptor fields are required");
    if (d->n_buf == 0 || d->n_buf >= (1ull << 31))
        return fail(CRYSTAL_EINVAL, "n_buf must be in [1, 2^31)");
    crystal_batch *b = new crystal_batch;
    b->d = *d;
    (void)hipGetDevice(&b->device);
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, b->device);
    if (e != hipSuccess) {
        free_plan(b);
        return hip_fail(e, "hipGetDeviceProperties");
    }
    b->n_simd = (uint32_t)prop.multiProcessorCount * 4;
    // lengths on the host: lane orders and the work prefix are built from them
    b->len.resize(d->n_buf);
    e = hipMemcpy(b->len.data(), d->d_len, 4 * d->n_buf, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        free_plan(b);
        return hip_fail(e, "reading lengths");
    }
    b->work_prefix.resize(d->n_buf);
    uint64_t acc = 0;
    for (uint64_t i = 0; i < d->n_buf; i++) {
        acc += (b->len[i] + 8) / 64 + 1;
        b->work_prefix[i] = acc;
    }
    e = hipMalloc((void **)&b->d_order, 4 * d->n_buf);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->d_counters, 4 * kMaxBranches);
    for (uint32_t i = 0; i < kMaxBranches && e == hipSuccess; i++)
        e = hipStreamCreateWithFlags(&b->cap[i], hipStreamNonBlocking);
    for (uint32_t i = 0; i <= kMaxBranches && e == hipSuccess; i++)
        e = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
        free_plan(b);
        return hip_fail(e, "plan setup");
    }

    std::vector<crystal_batch_tuning> cands;
    crystal_batch_tuning def = {256, 4, 1, 1, 4096, 0.f};
    if (fixed) {
        def = *fixed;
        if (def.block == 0)
            def.block = 256;
        if (def.waves_per_simd == 0)
            def.waves_per_simd = 4;
        if (def.grab == 0)
            def.grab = 1;
        if (def.n_streams == 0)
            def.n_streams = 1;
    }
    if (def.block % 64 || def.block > 1024 || def.n_streams > kMaxBranches) {
        free_plan(b);
        return fail(CRYSTAL_EINVAL, "bad tuning: block %% 64, <= 1024; streams <= 8");
    }
    if (tune_flags == CRYSTAL_TUNE_FULL) {
        for (uint32_t sorted : {256u, 1024u, 4096u, 65536u, 1u, 0u})
            for (uint32_t S : {1u, 2u})
                for (uint32_t blk : {64u, 256u})
                    for (uint32_t wps : {2u, 4u, 8u})
                        for (uint32_t grab : {1u, 4u})
                            cands.push_back({blk, wps, grab, S, sorted, 0.f});
    } else {
        cands.push_back(def);
    }
    crystal_batch_tuning best = cands[0];
    best.replay_ms = -1.f;
    for (const auto &c : cands) {
        b->tun = c;
        e = kGraphReplay ? capture(b, c) : hipSuccess;
        float ms = 0;
        if (e == hipSuccess)
            e = time_replays(b, cands.size() > 1 ? 5 : 3, &ms);
        if (e != hipSuccess) {
            free_plan(b);
            return hip_fail(e, "batch capture/replay");
        }
        if (best.replay_ms < 0 || ms < best.replay_ms) {
            best = c;
            best.replay_ms = ms;
        }
    }
    b->tun = best;
    e = kGraphReplay ? capture(b, best) : hipSuccess;
    if (e != hipSuccess) {
        free_plan(b);
        return hip_fail(e, "batch capture");
    }
    *out = b;
    return CRYSTAL_OK;
}

int crystal_batch_run(crystal_batch *b, int iters)
{
    if (!b || iters < 0)
        return fail(CRYSTAL_EINVAL, "bad arguments");
    for (int i = 0; i < iters; i++) {
        hipError_t e = replay(b);
        if (e != hipSuccess)
            return hip_fail(e, "batch replay");
    }
    return CRYSTAL_OK;
}

int crystal_batch_get_tuning(const crystal_batch *b, crystal_batch_tuning *t)
{
    if (!b || !t)
        return fail(CRYSTAL_EINVAL, "bad arguments");
    *t = b->tun;
    return CRYSTAL_OK;
}

void crystal_batch_free(crystal_batch *b)
{
    if (b)
        free_plan(b);
}

} // extern "C"
