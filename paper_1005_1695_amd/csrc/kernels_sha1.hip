// SHA-1 direct hashing: per-segment digests and digest-of-digests roots, the
// hashing the paper's own application measures (Sec. 5.2).  One lane hashes
// one message; see sha1_device.h.  Digests are 20 bytes, stored at a 20-byte
// stride (4-byte aligned).
#include "internal.h"
#include "sha1_device.h"

namespace crystal {

// Segment s of a launch (same job-table conventions as the MD5 segment
// kernel): locate its job, hash it, store its digest at index s, or in its
// job's own output region when out_off is set.
__device__ __forceinline__ void sha1_one_segment(const uint8_t *__restrict__ in,
                                                 const JobTable &jt, uint32_t seg_bytes,
                                                 uint64_t s, uint8_t *__restrict__ dig)
{
    uint64_t off = 0, len = jt.single_len, local = s;
    uint8_t *dst = dig + 20 * s;
    if (jt.n_jobs) {
        uint32_t lo = 0, hi = jt.n_jobs;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (jt.seg_base[mid] <= s)
                lo = mid;
            else
                hi = mid;
        }
        off = jt.off[lo];
        len = jt.len[lo];
        local = s - jt.seg_base[lo];
        if (jt.out_off)
            dst = dig + jt.out_off[lo] + 20 * local;
    }
    const uint64_t start = local * seg_bytes;
    const uint64_t rem = len - start;
    const uint64_t n = rem < seg_bytes ? rem : seg_bytes;
    const uint8_t *p = in + off + start;
    uint32_t H[5];
    if (((uintptr_t)p & 15) == 0)
        sha1_message_a16(p, n, H);
    else
        sha1_message_any(p, n, H);
    sha1_store(dst, H);
}

// One segment per lane (the dispatcher balances waves, as for MD5).
__global__ __launch_bounds__(256) void k_sha1_segments(const uint8_t *__restrict__ in,
                                                       JobTable jt, uint32_t seg_bytes,
                                                       uint64_t n_segments,
                                                       uint8_t *__restrict__ dig)
{
    const uint64_t G = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_segments;
         s += G)
        sha1_one_segment(in, jt, seg_bytes, s, dig);
}

// Lane j: SHA-1 over job j's concatenated 20-byte segment digests.  The
// digest array starts 16-byte aligned in every layout the library writes
// (a separate digest array, or a 256-aligned job output region) except for
// job j > 0 of a shared array, whose start 20 * seg_base[j] may be only
// 4-byte aligned; the realigning loader covers those.
__global__ __launch_bounds__(64) void k_sha1_roots(const uint8_t *__restrict__ dig,
                                                   JobTable jt, uint32_t seg_bytes,
                                                   uint8_t *__restrict__ roots)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nj = jt.n_jobs ? jt.n_jobs : 1;
    if (j >= nj)
        return;
    uint64_t b0 = 0, nseg;
    if (jt.n_jobs) {
        b0 = jt.seg_base[j];
        nseg = jt.seg_base[j + 1] - b0;
    } else {
        nseg = (jt.single_len + seg_bytes - 1) / seg_bytes;
    }
    const uint8_t *src = dig + 20 * b0;
    uint8_t *dst = roots + 20 * j;
    if (jt.n_jobs && jt.out_off) {
        src = dig + jt.out_off[j];
        dst = const_cast<uint8_t *>(src) + 20 * nseg;
    }
    uint32_t H[5];
    if (((uintptr_t)src & 15) == 0)
        sha1_message_a16(src, 20 * nseg, H);
    else
        sha1_message_any(src, 20 * nseg, H);
    sha1_store(dst, H);
}

static inline uint32_t blocks_of(uint64_t n, uint32_t b) { return (uint32_t)((n + b - 1) / b); }

static const uint64_t kSha1MaxLanes = (uint64_t)1 << 30;

hipError_t launch_sha1_segments(const uint8_t *in, const JobTable &jt, uint32_t seg_bytes,
                                uint64_t n_segments, uint8_t *seg_digests, hipStream_t s)
{
    if (n_segments == 0)
        return hipSuccess;
    const uint64_t lanes = n_segments < kSha1MaxLanes ? n_segments : kSha1MaxLanes;
    hipLaunchKernelGGL(k_sha1_segments, dim3(blocks_of(lanes, 256)), dim3(256), 0, s, in, jt,
                       seg_bytes, n_segments, seg_digests);
    return hipGetLastError();
}

hipError_t launch_sha1_roots(const uint8_t *seg_digests, const JobTable &jt, uint32_t seg_bytes,
                             uint8_t *roots, hipStream_t s)
{
    const uint32_t nj = jt.n_jobs ? jt.n_jobs : 1;
    hipLaunchKernelGGL(k_sha1_roots, dim3(blocks_of(nj, 64)), dim3(64), 0, s, seg_digests, jt,
                       seg_bytes, roots);
    return hipGetLastError();
}

} // namespace crystal
