// Batch plans: the batch-processing application class of Sec. 2.2 (many
// independent buffers available at once, throughput first).  A plan orders
// the buffers longest-first and replays a persistent MD5 launch (optionally
// split over several streams as parallel branches joined by events).  The
// tuner times every candidate configuration by replay.
//
// Lane order.  Longest-first inside windows of W consecutive buffers gives
// each wave 64 near-equal lengths that lie close together in the arena (a
// global sort spreads every wave over the whole arena and runs at less than
// half the speed).  But a window holds fewer groups of 64 than there are
// waves in flight, so the last windows' longest groups would start at the
// very end and leave most SIMDs idle while they finish.  The plan therefore
// re-sorts the last `tail` entries longest first as one block: with a tail of
// a few rounds of resident lanes the launch ends on its shortest buffers.
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
    uint64_t order_tail = 0;       // tail re-sort the device order holds
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

static hipError_t set_order(crystal_batch *b, uint32_t W, uint64_t T);

static bool uses_order(const crystal_batch_tuning &t) { return t.sorted != 0 || t.tail != 0; }

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
    const uint32_t *order = uses_order(t) ? b->d_order : nullptr;
    hipError_t e = set_order(b, t.sorted, t.tail);
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
                                                t.grab, t.depth, t.block, g, b->cap[i]);
            } else {
                // index order: slice offsets directly
                e = launch_md5_batch_persistent((const uint8_t *)b->d.d_arena,
                                                b->d.d_off + lo, b->d.d_len + lo, nullptr,
                                                hi - lo, (uint8_t *)b->d.d_out + 16 * lo,
                                                b->d_counters + i, t.grab, t.depth, t.block,
                                                g, b->cap[i]);
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
    const uint32_t *order = uses_order(t) ? b->d_order : nullptr;
    hipError_t e = set_order(b, t.sorted, t.tail);
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
                                                t.grab, t.depth, t.block, g, si);
            else
                e = launch_md5_batch_persistent((const uint8_t *)b->d.d_arena,
                                                b->d.d_off + lo, b->d.d_len + lo, nullptr,
                                                hi - lo, (uint8_t *)b->d.d_out + 16 * lo,
                                                b->d_counters + i, t.grab, t.depth, t.block,
                                                g, si);
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

// Lane order for sort window W and tail T: W == 0 keeps index order, W == 1
// sorts the whole batch longest first, W > 1 sorts longest first inside each
// run of W consecutive buffers; then the last min(T, n) entries are re-sorted
// longest first as one block.  Also rebuilds the work prefix used to split
// the order across branches.  The device order is written only when the
// order differs from index order.
static hipError_t set_order(crystal_batch *b, uint32_t W, uint64_t T)
{
    const uint64_t n = b->d.n_buf;
    T = std::min<uint64_t>(T, n);
    if (b->order_window == W && b->order_tail == T)
        return hipSuccess;
    std::vector<uint32_t> order(n);
    std::iota(order.begin(), order.end(), 0u);
    auto longer = [&](uint32_t x, uint32_t y) { return b->len[x] > b->len[y]; };
    if (W != 0) {
        const uint64_t win = W == 1 ? n : W;
        for (uint64_t lo = 0; lo < n; lo += win)
            std::stable_sort(order.begin() + lo,
                             order.begin() + std::min<uint64_t>(n, lo + win), longer);
    }
    if (T > 1)
        std::stable_sort(order.end() - T, order.end(), longer);
    uint64_t acc = 0;
    for (uint64_t i = 0; i < n; i++) {
        acc += (b->len[order[i]] + 8) / 64 + 1;
        b->work_prefix[i] = acc;
    }
    hipError_t e = hipSuccess;
    if (W != 0 || T != 0)
        e = hipMemcpy(b->d_order, order.data(), 4 * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        b->order_window = W;
        b->order_tail = T;
    }
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
    b->order_window = 0; // the work prefix above is the index order's
    b->order_tail = 0;
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

    // a tail of four rounds of resident lanes
    auto tail_for = [&](uint32_t wps) { return 4u * b->n_simd * wps * 64u; };
    std::vector<crystal_batch_tuning> cands;
    crystal_batch_tuning def = {256, 1, 1, 1, 4096, 2, tail_for(1), 0.f};
    if (fixed) {
        def = *fixed;
        if (def.block == 0)
            def.block = 256;
        if (def.waves_per_simd == 0)
            def.waves_per_simd = 1;
        if (def.grab == 0)
            def.grab = 1;
        if (def.n_streams == 0)
            def.n_streams = 1;
        if (def.depth == 0)
            def.depth = 2;
    }
    if (def.block % 64 || def.block == 0 || def.block > 256 || def.depth > 3 ||
        def.n_streams > kMaxBranches) {
        free_plan(b);
        return fail(CRYSTAL_EINVAL,
                    "bad tuning: block a multiple of 64 up to 256; depth 1..3; streams <= 8");
    }
    if (tune_flags == CRYSTAL_TUNE_FULL) {
        // (loader depth, waves per SIMD) pairs that fit the depth's register
        // budget; grouped by order so each order is built once
        const uint32_t dw[][2] = {{1, 2}, {1, 4}, {2, 1}, {2, 2}, {2, 3}, {3, 1}, {3, 2}};
        for (uint32_t sorted : {4096u, 65536u})
            for (uint32_t wps : {1u, 2u, 3u, 4u})
                for (const auto &p : dw)
                    if (p[1] == wps)
                        for (uint32_t blk : {64u, 256u})
                            for (uint32_t S : {1u, 2u})
                                cands.push_back({blk, wps, 1, S, sorted, p[0], tail_for(wps),
                                                 0.f});
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
