// Device-level entry points, chunking geometry, error reporting.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <time.h>

#include "internal.h"

namespace crystal {

static thread_local char g_err[512] = "";

void set_error(int code, const char *fmt, ...)
{
    char msg[448];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    snprintf(g_err, sizeof g_err, "[%d] %s", code, msg);
}

int fail(int code, const char *fmt, ...)
{
    char msg[448];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    snprintf(g_err, sizeof g_err, "[%d] %s", code, msg);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(CRYSTAL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int64_t now_ns()
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

// ------------------------------------------------------------ chunk params

bool cdc_resolve(const crystal_cdc_params *p, CdcParams *o, const char **why)
{
    crystal_cdc_params d;
    memset(&d, 0, sizeof d);
    if (p)
        d = *p;
    if (d.window != 0 && d.window != kWindow) {
        *why = "window must be 48";
        return false;
    }
    if (d.mask_bits == 0)
        d.mask_bits = 13;
    if (d.min_len == 0)
        d.min_len = 2048;
    if (d.max_len == 0)
        d.max_len = 65536;
    if (d.mask_bits > 64) {
        *why = "mask_bits must be <= 64";
        return false;
    }
    if (d.max_len < d.min_len || d.max_len > (1ull << 31)) {
        *why = "need 1 <= min_len <= max_len <= 2^31";
        return false;
    }
    o->base = d.base;
    uint64_t b48 = 1;
    for (uint32_t i = 0; i < kWindow; i++)
        b48 *= d.base;
    o->b48 = b48;
    o->mask = d.mask_bits >= 64 ? ~0ull : ((1ull << d.mask_bits) - 1);
    o->mask_bits = d.mask_bits;
    o->min_len = d.min_len;
    o->max_len = d.max_len;
    return true;
}

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static const uint32_t kShortWarmTiles = 256; // inputs up to 256 tiles walk a short warm-up

CdcGeom cdc_geometry(uint64_t n, const CdcParams &p)
{
    CdcGeom g;
    memset(&g, 0, sizeof g);
    g.n = n;
    g.n_ranges = (n + kRangeBytes - 1) / kRangeBytes;
    uint64_t P = (p.max_len + kRangeBytes - 1) / kRangeBytes * kRangeBytes;
    if (P < 65536)
        P = 65536;
    g.tile_bytes = P;
    g.n_tiles = (uint32_t)((n + P - 1) / P);
    // Speculative warm-up D before each tile.  Two chains meet once both land
    // on the same candidate, typically within a chunk or two: with the 2 KiB
    // minimum and the 13-bit mask, a 16 KiB warm-up left about 1 tile in 1000
    // out of phase on random data.  A small input (its walk is on the job's
    // critical path, and a failing tile costs one short repair) walks about
    // two mean chunk lengths, 2 (min + 2^bits) rounded up to 4 KiB, at least
    // 16 KiB; a large one walks 2P, where the sequential repair of its many
    // tiles would cost more than the shorter walks save.
    uint64_t D = 2 * P;
    if (g.n_tiles <= kShortWarmTiles && p.mask_bits < 40) {
        uint64_t s = 2 * (p.min_len + (1ull << p.mask_bits));
        s = (s + kRangeBytes - 1) / kRangeBytes * kRangeBytes;
        if (s < 16384)
            s = 16384;
        if (s < D)
            D = s;
    }
    g.warm_bytes = D;
    g.tile_cap = (uint32_t)((P + p.min_len - 1) / p.min_len + 1);
    size_t o = 0;
    g.off_l1 = o;
    o = al256(o + g.n_ranges * 64 * 8);
    g.off_l2 = o;
    o = al256(o + g.n_ranges * 8);
    g.off_cnt = o;
    o = al256(o + g.n_ranges * 4);
    g.off_rscan = o;
    o = al256(o + g.n_ranges * 8);
    g.off_exit = o;
    o = al256(o + (size_t)g.n_tiles * 8);
    g.off_first = o;
    o = al256(o + (size_t)g.n_tiles * 8);
    g.off_tcnt = o;
    o = al256(o + (size_t)g.n_tiles * 4);
    g.off_starts = o;
    o = al256(o + (size_t)g.n_tiles * g.tile_cap * 8);
    g.off_toff = o;
    o = al256(o + (size_t)g.n_tiles * 8);
    g.off_flags = o;
    o = al256(o + (size_t)g.n_tiles * 4);
    g.off_bad = o;
    o = al256(o + 8);
    g.off_misc = o;
    o = al256(o + 64);
    g.off_hist = o;
    o = al256(o + 2 * 64 * 4);
    g.ord_cap = n / p.min_len + 1;
    g.off_ord = o;
    o = al256(o + g.ord_cap * 4);
    g.total = o;
    return g;
}

uint64_t cdc_max_chunks(uint64_t n, const CdcParams &p)
{
    return n == 0 ? 0 : n / p.min_len + 1;
}

} // namespace crystal

using namespace crystal;

extern "C" {

const char *crystal_last_error(void) { return g_err; }

} // extern "C"

// Direct hashing with MD5 (16-byte digests) or SHA-1 (20-byte digests):
// validation and launches shared by the device-level entry points.
enum class DirectHash { Md5, Sha1 };

static int direct_segments(DirectHash h, const void *d_in, const uint64_t *d_job_off,
                           const uint64_t *d_job_len, const uint64_t *d_seg_base,
                           uint32_t n_jobs, uint64_t n_segments, uint32_t segment_bytes,
                           void *d_seg_digests, void *stream)
{
    if (segment_bytes == 0)
        segment_bytes = 4096;
    if (segment_bytes % 64 || segment_bytes > (1u << 30))
        return fail(CRYSTAL_EINVAL, "segment_bytes must be a multiple of 64 and <= 2^30");
    if (n_jobs == 0 || n_segments == 0)
        return CRYSTAL_OK;
    if (!d_in || !d_job_off || !d_job_len || !d_seg_base || !d_seg_digests)
        return fail(CRYSTAL_EINVAL, "null pointer argument");
    JobTable jt{d_job_off, d_job_len, d_seg_base, n_jobs, 0};
    hipError_t e = h == DirectHash::Md5
                       ? launch_md5_segments((const uint8_t *)d_in, jt, segment_bytes,
                                             n_segments, (uint8_t *)d_seg_digests,
                                             (hipStream_t)stream)
                       : launch_sha1_segments((const uint8_t *)d_in, jt, segment_bytes,
                                              n_segments, (uint8_t *)d_seg_digests,
                                              (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "segments launch");
    return CRYSTAL_OK;
}

static int direct_roots(DirectHash h, const uint64_t *d_seg_base, uint32_t n_jobs,
                        uint32_t segment_bytes, const void *d_seg_digests, void *d_roots,
                        void *stream)
{
    if (segment_bytes == 0)
        segment_bytes = 4096;
    if (segment_bytes % 64 || segment_bytes > (1u << 30))
        return fail(CRYSTAL_EINVAL, "segment_bytes must be a multiple of 64 and <= 2^30");
    if (n_jobs == 0)
        return CRYSTAL_OK;
    if (!d_seg_base || !d_roots)
        return fail(CRYSTAL_EINVAL, "null pointer argument");
    JobTable jt{nullptr, nullptr, d_seg_base, n_jobs, 0};
    hipError_t e = h == DirectHash::Md5
                       ? launch_md5_roots((const uint8_t *)d_seg_digests, jt, segment_bytes,
                                          (uint8_t *)d_roots, (hipStream_t)stream)
                       : launch_sha1_roots((const uint8_t *)d_seg_digests, jt, segment_bytes,
                                           (uint8_t *)d_roots, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "roots launch");
    return CRYSTAL_OK;
}

static int direct_both(DirectHash h, const void *d_in, const uint64_t *d_job_off,
                       const uint64_t *d_job_len, const uint64_t *d_seg_base, uint32_t n_jobs,
                       uint64_t n_segments, uint32_t segment_bytes, void *d_seg_digests,
                       void *d_roots, void *stream)
{
    if (segment_bytes % 64 || segment_bytes > (1u << 30))
        return fail(CRYSTAL_EINVAL, "segment_bytes must be a multiple of 64 and <= 2^30");
    if (n_jobs == 0)
        return CRYSTAL_OK;
    if (!d_job_off || !d_job_len || !d_seg_base || !d_roots ||
        (n_segments && (!d_in || !d_seg_digests)))
        return fail(CRYSTAL_EINVAL, "null pointer argument");
    int rc = direct_segments(h, d_in, d_job_off, d_job_len, d_seg_base, n_jobs, n_segments,
                             segment_bytes, d_seg_digests, stream);
    if (rc)
        return rc;
    return direct_roots(h, d_seg_base, n_jobs, segment_bytes, d_seg_digests, d_roots, stream);
}

extern "C" {

int crystal_md5_direct_device(const void *d_in, const uint64_t *d_job_off,
                              const uint64_t *d_job_len, const uint64_t *d_seg_base,
                              uint32_t n_jobs, uint64_t n_segments, uint32_t segment_bytes,
                              void *d_seg_digests, void *d_roots, void *stream)
{
    return direct_both(DirectHash::Md5, d_in, d_job_off, d_job_len, d_seg_base, n_jobs,
                       n_segments, segment_bytes, d_seg_digests, d_roots, stream);
}

int crystal_md5_segments_device(const void *d_in, const uint64_t *d_job_off,
                                const uint64_t *d_job_len, const uint64_t *d_seg_base,
                                uint32_t n_jobs, uint64_t n_segments, uint32_t segment_bytes,
                                void *d_seg_digests, void *stream)
{
    return direct_segments(DirectHash::Md5, d_in, d_job_off, d_job_len, d_seg_base, n_jobs,
                           n_segments, segment_bytes, d_seg_digests, stream);
}

int crystal_md5_roots_device(const uint64_t *d_seg_base, uint32_t n_jobs,
                             uint32_t segment_bytes, const void *d_seg_digests, void *d_roots,
                             void *stream)
{
    return direct_roots(DirectHash::Md5, d_seg_base, n_jobs, segment_bytes, d_seg_digests,
                        d_roots, stream);
}

int crystal_sha1_direct_device(const void *d_in, const uint64_t *d_job_off,
                               const uint64_t *d_job_len, const uint64_t *d_seg_base,
                               uint32_t n_jobs, uint64_t n_segments, uint32_t segment_bytes,
                               void *d_seg_digests, void *d_roots, void *stream)
{
    return direct_both(DirectHash::Sha1, d_in, d_job_off, d_job_len, d_seg_base, n_jobs,
                       n_segments, segment_bytes, d_seg_digests, d_roots, stream);
}

int crystal_sha1_segments_device(const void *d_in, const uint64_t *d_job_off,
                                 const uint64_t *d_job_len, const uint64_t *d_seg_base,
                                 uint32_t n_jobs, uint64_t n_segments, uint32_t segment_bytes,
                                 void *d_seg_digests, void *stream)
{
    return direct_segments(DirectHash::Sha1, d_in, d_job_off, d_job_len, d_seg_base, n_jobs,
                           n_segments, segment_bytes, d_seg_digests, stream);
}

int crystal_sha1_roots_device(const uint64_t *d_seg_base, uint32_t n_jobs,
                              uint32_t segment_bytes, const void *d_seg_digests, void *d_roots,
                              void *stream)
{
    return direct_roots(DirectHash::Sha1, d_seg_base, n_jobs, segment_bytes, d_seg_digests,
                        d_roots, stream);
}

int crystal_md5_batch_device(const void *d_arena, const uint64_t *d_off, const uint32_t *d_len,
                             const uint32_t *d_order, uint64_t n_buf, void *d_out,
                             uint32_t block, uint32_t grid, void *stream)
{
    if (block == 0)
        block = 256;
    if (block % 64 || block > 1024)
        return fail(CRYSTAL_EINVAL, "block must be a multiple of 64 and <= 1024");
    if (n_buf == 0)
        return CRYSTAL_OK;
    if (!d_arena || !d_off || !d_len || !d_out)
        return fail(CRYSTAL_EINVAL, "null pointer argument");
    hipError_t e = launch_md5_batch((const uint8_t *)d_arena, d_off, d_len, d_order, n_buf,
                                    (uint8_t *)d_out, block, grid, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "md5_batch launch");
    return CRYSTAL_OK;
}

size_t crystal_cdc_workspace_bytes(uint64_t n, const crystal_cdc_params *p)
{
    CdcParams cp;
    const char *why;
    if (!cdc_resolve(p, &cp, &why))
        return 0;
    return cdc_geometry(n, cp).total;
}

uint64_t crystal_cdc_max_chunks(uint64_t n, const crystal_cdc_params *p)
{
    CdcParams cp;
    const char *why;
    if (!cdc_resolve(p, &cp, &why))
        return 0;
    return cdc_max_chunks(n, cp);
}

static int cdc_prepare(uint64_t n, const crystal_cdc_params *p, size_t ws_bytes,
                       CdcParams *cp, CdcGeom *g)
{
    const char *why = "";
    if (!cdc_resolve(p, cp, &why))
        return fail(CRYSTAL_EINVAL, "chunking params: %s", why);
    *g = cdc_geometry(n, *cp);
    if (ws_bytes < g->total)
        return fail(CRYSTAL_EINVAL, "workspace %zu < required %zu", ws_bytes, g->total);
    return CRYSTAL_OK;
}

int crystal_cdc_candidates_device(const void *d_in, uint64_t n, const crystal_cdc_params *p,
                                  void *d_ws, size_t ws_bytes, uint64_t *d_count,
                                  uint64_t *d_cand, uint64_t cap, void *stream)
{
    CdcParams cp;
    CdcGeom g;
    int rc = cdc_prepare(n, p, ws_bytes, &cp, &g);
    if (rc)
        return rc;
    if ((n && (!d_in || !d_ws)) || (d_cand && !d_count))
        return fail(CRYSTAL_EINVAL, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_cdc_candidates((const uint8_t *)d_in, g, cp, (uint8_t *)d_ws, s);
    if (e != hipSuccess)
        return hip_fail(e, "cdc_candidates launch");
    if (d_count) {
        e = launch_cdc_compact(g, (uint8_t *)d_ws, d_count, d_cand, cap, s);
        if (e != hipSuccess)
            return hip_fail(e, "cdc_compact launch");
    }
    return CRYSTAL_OK;
}

int crystal_cdc_select_device(uint64_t n, const crystal_cdc_params *p, void *d_ws,
                              size_t ws_bytes, uint64_t *d_n_chunks, uint64_t *d_ends,
                              uint64_t cap, void *stream)
{
    CdcParams cp;
    CdcGeom g;
    int rc = cdc_prepare(n, p, ws_bytes, &cp, &g);
    if (rc)
        return rc;
    if (!d_n_chunks || (n && (!d_ws || !d_ends)))
        return fail(CRYSTAL_EINVAL, "null pointer argument");
    if (cap < cdc_max_chunks(n, cp))
        return fail(CRYSTAL_EINVAL, "cap %llu < crystal_cdc_max_chunks %llu",
                    (unsigned long long)cap, (unsigned long long)cdc_max_chunks(n, cp));
    hipError_t e = launch_cdc_select(g, cp, (uint8_t *)d_ws, d_n_chunks, d_ends, cap,
                                     (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "cdc_select launch");
    return CRYSTAL_OK;
}

int crystal_md5_chunks_device(const void *d_in, const uint64_t *d_ends,
                              const uint64_t *d_n_chunks, uint64_t cap, void *d_digests,
                              void *stream)
{
    if (cap == 0)
        return CRYSTAL_OK;
    if (!d_in || !d_ends || !d_n_chunks || !d_digests)
        return fail(CRYSTAL_EINVAL, "null pointer argument");
    hipError_t e = launch_md5_chunks((const uint8_t *)d_in, d_ends, d_n_chunks, cap, nullptr,
                                     (uint8_t *)d_digests, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "md5_chunks launch");
    return CRYSTAL_OK;
}

int crystal_cdc_device(const void *d_in, uint64_t n, const crystal_cdc_params *p, void *d_ws,
                       size_t ws_bytes, uint64_t *d_n_chunks, uint64_t *d_ends,
                       void *d_digests, uint64_t cap, void *stream)
{
    CdcParams cp;
    CdcGeom g;
    int rc = cdc_prepare(n, p, ws_bytes, &cp, &g);
    if (rc)
        return rc;
    if (!d_n_chunks || (n && (!d_in || !d_ws || !d_ends)) || (cap && !d_digests))
        return fail(CRYSTAL_EINVAL, "null pointer argument");
    if (cap < cdc_max_chunks(n, cp))
        return fail(CRYSTAL_EINVAL, "cap %llu < crystal_cdc_max_chunks %llu",
                    (unsigned long long)cap, (unsigned long long)cdc_max_chunks(n, cp));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_cdc_candidates((const uint8_t *)d_in, g, cp, (uint8_t *)d_ws, s);
    if (e != hipSuccess)
        return hip_fail(e, "cdc_candidates launch");
    const uint32_t *order = nullptr;
    e = launch_cdc_select(g, cp, (uint8_t *)d_ws, d_n_chunks, d_ends, cap, s,
                          cap ? &order : nullptr);
    if (e != hipSuccess)
        return hip_fail(e, "cdc_select launch");
    if (cap == 0)
        return CRYSTAL_OK;
    e = launch_md5_chunks((const uint8_t *)d_in, d_ends, d_n_chunks, cap, order,
                          (uint8_t *)d_digests, s);
    if (e != hipSuccess)
        return hip_fail(e, "md5_chunks launch");
    return CRYSTAL_OK;
}

int crystal_window_hash_device(const void *d_in, uint64_t n, uint64_t base, uint64_t *d_w,
                               void *stream)
{
    if (n == 0)
        return CRYSTAL_OK;
    if (!d_in || !d_w)
        return fail(CRYSTAL_EINVAL, "null pointer argument");
    hipError_t e = launch_window_hash((const uint8_t *)d_in, n, base, d_w, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "window_hash launch");
    return CRYSTAL_OK;
}

} // extern "C"
