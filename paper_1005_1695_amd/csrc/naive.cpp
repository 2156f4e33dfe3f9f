// Naive per-job path: the pattern the paper's framework replaces (Sec. 5.2,
// Fig. 6 -- allocate device buffers for every job, blocking copy in, kernel,
// blocking copy out, free; nothing reused, nothing overlapped).  It runs the
// same kernels as the job layer so the comparison isolates the framework.
#include <string.h>

#include "internal.h"

using namespace crystal;

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

extern "C" int crystal_naive_run(int kernel_id, const void *params, const void *h_in, size_t n,
                                 void *h_out, size_t out_cap, size_t *out_bytes,
                                 crystal_stage_times *st)
{
    const size_t need_out = crystal_output_bytes(kernel_id, n, params);
    if (need_out == 0 && kernel_id != CRYSTAL_K_NOP)
        return fail(CRYSTAL_EINVAL, "bad kernel id or parameters");
    if (out_cap < need_out || (n && !h_in) || (need_out && !h_out))
        return fail(CRYSTAL_EINVAL, "output capacity %zu < %zu or null buffer", out_cap,
                    need_out);
    crystal_stage_times t;
    memset(&t, 0, sizeof t);
    const int64_t t0 = now_ns();
    uint8_t *d_in = nullptr, *d_out = nullptr, *d_ws = nullptr;
    CdcParams cp;
    CdcGeom g;
    uint64_t cap = 0;
    uint32_t seg = 4096;
    if (kernel_id == CRYSTAL_K_CDC) {
        const char *why = "";
        if (!cdc_resolve(static_cast<const crystal_cdc_params *>(params), &cp, &why))
            return fail(CRYSTAL_EINVAL, "chunking params: %s", why);
        g = cdc_geometry(n, cp);
        cap = cdc_max_chunks(n, cp);
    } else if ((kernel_id == CRYSTAL_K_MD5_DIRECT || kernel_id == CRYSTAL_K_SHA1_DIRECT) &&
               params) {
        const auto *dp = static_cast<const crystal_direct_params *>(params);
        if (dp->segment_bytes)
            seg = dp->segment_bytes;
    }
    hipError_t e = hipMalloc((void **)&d_in, al256(n ? n : 1));
    if (e == hipSuccess && kernel_id != CRYSTAL_K_NOP)
        e = hipMalloc((void **)&d_out, al256(need_out));
    if (e == hipSuccess && kernel_id == CRYSTAL_K_CDC)
        e = hipMalloc((void **)&d_ws, al256(g.total));
    const int64_t t1 = now_ns();
    if (e == hipSuccess && n)
        e = hipMemcpy(d_in, h_in, n, hipMemcpyHostToDevice);
    const int64_t t2 = now_ns();
    size_t d2h = need_out;
    if (e == hipSuccess) {
        hipStream_t s = nullptr;
        switch (kernel_id) {
        case CRYSTAL_K_NOP:
            e = launch_nop(s);
            d_out = d_in;
            break;
        case CRYSTAL_K_MD5:
            e = launch_md5_whole(d_in, n, d_out, s);
            break;
        case CRYSTAL_K_MD5_DIRECT: {
            JobTable jt{nullptr, nullptr, nullptr, 0, n};
            const uint64_t nseg = (n + seg - 1) / seg;
            e = launch_md5_segments(d_in, jt, seg, nseg, d_out, s);
            if (e == hipSuccess)
                e = launch_md5_roots(d_out, jt, seg, d_out + 16 * nseg, s);
            break;
        }
        case CRYSTAL_K_SHA1_DIRECT: {
            JobTable jt{nullptr, nullptr, nullptr, 0, n};
            const uint64_t nseg = (n + seg - 1) / seg;
            e = launch_sha1_segments(d_in, jt, seg, nseg, d_out, s);
            if (e == hipSuccess)
                e = launch_sha1_roots(d_out, jt, seg, d_out + 20 * nseg, s);
            break;
        }
        case CRYSTAL_K_CDC: {
            uint64_t *cnt = reinterpret_cast<uint64_t *>(d_out);
            e = launch_cdc_candidates(d_in, g, cp, d_ws, s);
            const uint32_t *order = nullptr;
            if (e == hipSuccess)
                e = launch_cdc_select(g, cp, d_ws, cnt, cnt + 1, cap, s, &order);
            if (e == hipSuccess)
                e = launch_md5_chunks(d_in, cnt + 1, cnt, cap, order, nullptr, s);
            break;
        }
        }
        if (e == hipSuccess)
            e = hipDeviceSynchronize();
    }
    const int64_t t3 = now_ns();
    if (e == hipSuccess && d2h)
        e = hipMemcpy(h_out, d_out, d2h, hipMemcpyDeviceToHost);
    const int64_t t4 = now_ns();
    if (kernel_id == CRYSTAL_K_NOP)
        d_out = nullptr;
    (void)hipFree(d_in);
    if (d_out)
        (void)hipFree(d_out);
    if (d_ws)
        (void)hipFree(d_ws);
    const int64_t t5 = now_ns();
    if (e != hipSuccess)
        return hip_fail(e, "naive job");
    size_t ob = d2h;
    if (kernel_id == CRYSTAL_K_CDC) {
        uint64_t nc;
        memcpy(&nc, h_out, 8);
        ob = 8 + 24 * nc;
    }
    if (out_bytes)
        *out_bytes = ob;
    t.alloc_ms = (t1 - t0) * 1e-6;
    t.copy_in_ms = (t2 - t1) * 1e-6;
    t.kernel_ms = (t3 - t2) * 1e-6;
    t.copy_out_ms = (t4 - t3) * 1e-6;
    t.free_ms = (t5 - t4) * 1e-6;
    t.total_ms = (t5 - t0) * 1e-6;
    if (st)
        *st = t;
    return CRYSTAL_OK;
}
