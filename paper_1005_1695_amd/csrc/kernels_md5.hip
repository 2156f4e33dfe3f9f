// MD5 kernels: per-segment direct hashing, digest-of-digests roots, whole
// buffers, batched small buffers (plain and persistent) and per-chunk
// digests.  One lane hashes one message; see md5_device.h.
#include "internal.h"
#include "md5_device.h"

namespace crystal {

// Job of segment s in a multi-job launch: the largest j with
// seg_base[j] <= s (which also skips empty jobs).
__device__ __forceinline__ uint32_t segment_job(const JobTable &jt, uint64_t s)
{
    uint32_t lo = 0, hi = jt.n_jobs;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (jt.seg_base[mid] <= s)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// The common segment: full 4 KiB and 16-byte aligned.  Its loader is compiled
// for that constant length, which keeps the kernel at 80 registers (six waves
// per SIMD); ragged last segments, other segment sizes and unaligned jobs take
// the lighter single-buffered loaders.
constexpr uint64_t kFullSegment = 4096;

// Segment s of a launch: locate its job, hash it, store its digest at index s
// (or in its job's own output region).  Only s stays live across the hashing
// (the destination is looked up again afterwards).
__device__ __forceinline__ void md5_one_segment(const uint8_t *__restrict__ in,
                                                const JobTable &jt, uint32_t seg_bytes,
                                                uint64_t s, uint8_t *__restrict__ dig)
{
    uint64_t off = 0, len = jt.single_len, local = s;
    if (jt.n_jobs) {
        const uint32_t j = segment_job(jt, s);
        off = jt.off[j];
        len = jt.len[j];
        local = s - jt.seg_base[j];
    }
    const uint64_t start = local * seg_bytes;
    const uint64_t rem = len - start;
    const uint64_t n = rem < seg_bytes ? rem : seg_bytes;
    const uint8_t *p = in + off + start;
    uint32_t st[4];
    const bool aligned = ((uintptr_t)p & 15) == 0;
    if (aligned && n == kFullSegment)
        md5_message_a16_db<1>(p, kFullSegment, st);
    else if (aligned)
        md5_message_a16(p, n, st);
    else
        md5_message_any(p, n, st);
    uint8_t *dst = dig + 16 * s;
    if (jt.n_jobs && jt.out_off) {
        const uint32_t j = segment_job(jt, s);
        dst = dig + jt.out_off[j] + 16 * (s - jt.seg_base[j]);
    }
    md5_store(dst, st);
}

// One segment per lane.  Each wave's work is one segment per lane, so the
// hardware dispatcher balances waves across SIMDs as they free up: a static
// split (a fixed number of segments per lane) was measured to lose far more
// to the slowest SIMD when other kernels (the root chains of the previous
// batch) share the chip.  The loop only covers launches beyond the grid cap.
// Six waves per SIMD need at most 80 registers (the compiler moves one value
// that lives across the whole loop to scratch to get there).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_md5_segments(const uint8_t *__restrict__ in,
                                                      JobTable jt, uint32_t seg_bytes,
                                                      uint64_t n_segments,
                                                      uint8_t *__restrict__ dig)
{
    const uint64_t G = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_segments;
         s += G)
        md5_one_segment(in, jt, seg_bytes, s, dig);
}

// Lane j computes the root of job j: MD5 over its segment digests, which are
// contiguous and 16-byte aligned in the digest array.  Each lane is one long
// serial chain with few waves around it, usually beside a segment kernel that
// keeps HBM busy; load latency is then several microseconds, so its loader
// reads three 128-byte groups (six compressions) ahead.  (Raising these waves' issue priority was measured to
// slow a concurrently running segment kernel by far more than it sped the
// chains up, so they run at the default priority.)
__device__ __forceinline__ void md5_root_of_job(const uint8_t *__restrict__ dig,
                                                const JobTable &jt, uint32_t seg_bytes,
                                                uint32_t j, uint8_t *__restrict__ roots)
{
    uint64_t b0 = 0, nseg;
    if (jt.n_jobs) {
        b0 = jt.seg_base[j];
        nseg = jt.seg_base[j + 1] - b0;
    } else {
        nseg = (jt.single_len + seg_bytes - 1) / seg_bytes;
    }
    const uint8_t *src = dig + 16 * b0;
    uint8_t *dst = roots + 16 * j;
    if (jt.n_jobs && jt.out_off) {
        src = dig + jt.out_off[j];
        dst = const_cast<uint8_t *>(src) + 16 * nseg;
    }
    uint32_t st[4];
    md5_message_a16_db<3>(src, 16 * nseg, st);
    md5_store(dst, st);
}

__global__ __launch_bounds__(64) void k_md5_roots(const uint8_t *__restrict__ dig,
                                                  JobTable jt, uint32_t seg_bytes,
                                                  uint8_t *__restrict__ roots)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nj = jt.n_jobs ? jt.n_jobs : 1;
    if (j >= nj)
        return;
    md5_root_of_job(dig, jt, seg_bytes, j, roots);
}

__global__ __launch_bounds__(64) void k_md5_whole(const uint8_t *__restrict__ in,
                                                  uint64_t n, uint8_t *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    uint32_t st[4];
    if (((uintptr_t)in & 15) == 0)
        md5_message_a16_db<2>(in, n, st);
    else
        md5_message_any_db<2>(in, n, st);
    md5_store(out, st);
}

__device__ __forceinline__ void md5_one_buffer(const uint8_t *__restrict__ arena,
                                               const uint64_t *__restrict__ off,
                                               const uint32_t *__restrict__ len,
                                               uint64_t m, uint8_t *__restrict__ out)
{
    const uint8_t *p = arena + off[m];
    const uint64_t l = len[m];
    uint32_t st[4];
    if (((uintptr_t)p & 15) == 0)
        md5_message_a16_db<1>(p, l, st);
    else
        md5_message_any(p, l, st);
    md5_store(out + 16 * m, st);
}

// Grid-stride batch: lane i takes buffers order[i], order[i + G], ...
__global__ void k_md5_batch(const uint8_t *__restrict__ arena,
                            const uint64_t *__restrict__ off,
                            const uint32_t *__restrict__ len,
                            const uint32_t *__restrict__ order, uint64_t n,
                            uint8_t *__restrict__ out)
{
    const uint64_t G = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += G) {
        const uint64_t m = order ? order[i] : i;
        md5_one_buffer(arena, off, len, m, out);
    }
}

// One buffer of a batch with a loader that keeps D 128-byte groups per lane
// in flight ahead of the compression.  Deeper look-ahead means fewer, larger
// reads per lane: on the batch's scattered per-lane streams this raises the
// bandwidth the memory system delivers, at the cost of registers.
template <int D>
__device__ __forceinline__ void md5_one_buffer_d(const uint8_t *__restrict__ arena,
                                                 const uint64_t *__restrict__ off,
                                                 const uint32_t *__restrict__ len, uint64_t m,
                                                 uint8_t *__restrict__ out)
{
    const uint8_t *p = arena + off[m];
    const uint64_t l = len[m];
    uint32_t st[4];
    if (((uintptr_t)p & 15) == 0)
        md5_message_a16_db<D>(p, l, st);
    else
        md5_message_any(p, l, st);
    md5_store(out + 16 * m, st);
}

// Register budget per depth: D = 1 fits 4 waves per SIMD, D = 2 three and
// D = 3 two.
template <int D> struct BatchWaves;
template <> struct BatchWaves<1> { static constexpr int value = 4; };
template <> struct BatchWaves<2> { static constexpr int value = 3; };
template <> struct BatchWaves<3> { static constexpr int value = 2; };

// Persistent batch: each wave repeatedly takes the next grab*64 entries of
// the (longest-first) order from a global counter, so waves that drew short
// buffers come back for more.  Every wave leaves once the counter passes n.
template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BatchWaves<D>::value)))
void k_md5_batch_persistent(const uint8_t *__restrict__ arena, const uint64_t *__restrict__ off,
                            const uint32_t *__restrict__ len,
                            const uint32_t *__restrict__ order, uint64_t n,
                            uint8_t *__restrict__ out, uint32_t *__restrict__ counter,
                            uint32_t grab)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t span = grab * 64u;
    for (;;) {
        uint32_t base = 0;
        if (lane == 0)
            base = atomicAdd(counter, span);
        base = __shfl(base, 0, 64);
        if ((uint64_t)base >= n)
            break;
        for (uint32_t k = 0; k < grab; k++) {
            const uint64_t i = (uint64_t)base + 64u * k + lane;
            if (i < n) {
                const uint64_t m = order ? order[i] : i;
                md5_one_buffer_d<D>(arena, off, len, m, out);
            }
        }
    }
}

__global__ void k_zero_u32(uint32_t *p, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0;
}

// Digest of chunk k, the bytes [ends[k-1], ends[k]); chunk starts are
// arbitrary byte offsets, so the realigning loader is used, reading three
// 128-byte groups ahead (the kernels that run these chains hold few waves, so
// the registers are free).  With dig == nullptr the digest goes right after
// the ends array (ends + nc), the packed job output layout; that address is
// only 8-byte aligned.
__device__ __forceinline__ void md5_one_chunk(const uint8_t *__restrict__ in,
                                              const uint64_t *__restrict__ ends, uint64_t nc,
                                              uint64_t k, uint8_t *__restrict__ dig)
{
    const uint64_t lo = k ? ends[k - 1] : 0;
    const uint64_t hi = ends[k];
    uint32_t st[4];
    md5_message_any_db<3>(in + lo, hi - lo, st);
    if (dig) {
        md5_store(dig + 16 * k, st);
    } else {
        uint64_t *q = const_cast<uint64_t *>(ends) + nc + 2 * k;
        q[0] = (uint64_t)st[0] | ((uint64_t)st[1] << 32);
        q[1] = (uint64_t)st[2] | ((uint64_t)st[3] << 32);
    }
}

// Lane i hashes chunk order[i] (chunk i without an order).  One wave per
// workgroup: these are long serial chains, and single-wave groups let the
// dispatcher spread them over SIMDs (four-wave groups put four chains' waves
// on one CU).
__global__ __launch_bounds__(64) void k_md5_chunks(const uint8_t *__restrict__ in,
                                                   const uint64_t *__restrict__ ends,
                                                   const uint64_t *__restrict__ n_chunks,
                                                   uint64_t cap,
                                                   const uint32_t *__restrict__ order,
                                                   uint8_t *__restrict__ dig)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t nc = *n_chunks;
    if (nc > cap)
        nc = cap;
    if (i >= nc)
        return;
    md5_one_chunk(in, ends, nc, order ? order[i] : i, dig);
}

// The serial chains of a batch of jobs in one launch: lanes [0, jt.n_jobs)
// compute the roots of a direct-hashing group (job table jt, outputs in each
// job's own region), then each chunking job j owns the 64-aligned lane range
// [lane0[j], lane0[j+1]) and its lane i hashes the job's chunk order[i] into
// the packed output at out_off[j].  One launch runs all these chains side by
// side, so a batch waits for its longest chain instead of the sum of its
// jobs' longest chains.
__global__ __launch_bounds__(64) void k_md5_chains(uint8_t *__restrict__ slab, JobTable jt,
                                                   uint32_t seg_bytes, ChainTable ct)
{
    const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lane < jt.n_jobs) {
        md5_root_of_job(slab, jt, seg_bytes, (uint32_t)lane, slab);
        return;
    }
    if (ct.n_jobs == 0)
        return;
    const uint64_t l = lane - jt.n_jobs;
    if (l >= ct.lane0[ct.n_jobs])
        return;
    uint32_t lo = 0, hi = ct.n_jobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ct.lane0[mid] <= l)
            lo = mid;
        else
            hi = mid;
    }
    const uint64_t i = l - ct.lane0[lo];
    const uint64_t *ends = reinterpret_cast<const uint64_t *>(slab + ct.out_off[lo]) + 1;
    uint64_t nc = ends[-1];
    if (nc > ct.cap[lo])
        nc = ct.cap[lo];
    if (i >= nc)
        return;
    const uint64_t ord = ct.ord_off[lo];
    const uint64_t k =
        ord != kNoOrder ? reinterpret_cast<const uint32_t *>(slab + ord)[i] : i;
    md5_one_chunk(slab + ct.in_off[lo], ends, nc, k, nullptr);
}

__global__ void k_nop() {}

// ------------------------------------------------------------------ launch

static inline uint32_t blocks_for(uint64_t n, uint32_t b)
{
    return (uint32_t)((n + b - 1) / b);
}

// Grid cap of the segment kernel (lanes); launches beyond it loop.
static const uint64_t kSegMaxLanes = (uint64_t)1 << 30;
static const uint64_t kOneWavePerSimd = 256 * 4 * 64;

hipError_t launch_md5_segments(const uint8_t *in, const JobTable &jt,
                               uint32_t seg_bytes, uint64_t n_segments,
                               uint8_t *seg_digests, hipStream_t s)
{
    if (n_segments == 0)
        return hipSuccess;
    const uint64_t lanes = n_segments < kSegMaxLanes ? n_segments : kSegMaxLanes;
    // launches of at most one wave per SIMD (256 CUs x 4 SIMDs x 64 lanes)
    // spread over more CUs in single-wave groups: 4-7 % faster measured
    // there; larger launches are not sensitive to the group size
    const uint32_t block = lanes <= kOneWavePerSimd ? 64 : 256;
    hipLaunchKernelGGL(k_md5_segments, dim3(blocks_for(lanes, block)), dim3(block), 0, s, in,
                       jt, seg_bytes, n_segments, seg_digests);
    return hipGetLastError();
}

hipError_t launch_md5_roots(const uint8_t *seg_digests, const JobTable &jt,
                            uint32_t seg_bytes, uint8_t *roots, hipStream_t s)
{
    const uint32_t nj = jt.n_jobs ? jt.n_jobs : 1;
    hipLaunchKernelGGL(k_md5_roots, dim3(blocks_for(nj, 64)), dim3(64), 0, s,
                       seg_digests, jt, seg_bytes, roots);
    return hipGetLastError();
}

hipError_t launch_md5_whole(const uint8_t *in, uint64_t n, uint8_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_md5_whole, dim3(1), dim3(64), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_md5_batch(const uint8_t *arena, const uint64_t *off,
                            const uint32_t *len, const uint32_t *order,
                            uint64_t n, uint8_t *out, uint32_t block,
                            uint32_t grid, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    if (grid == 0)
        grid = blocks_for(n, block);
    hipLaunchKernelGGL(k_md5_batch, dim3(grid), dim3(block), 0, s, arena, off, len,
                       order, n, out);
    return hipGetLastError();
}

hipError_t launch_md5_batch_persistent(const uint8_t *arena, const uint64_t *off,
                                       const uint32_t *len, const uint32_t *order,
                                       uint64_t n, uint8_t *out, uint32_t *counter,
                                       uint32_t grab, uint32_t depth, uint32_t block,
                                       uint32_t grid, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    if (block == 0 || block > 256 || block % 64 || depth < 1 || depth > 3)
        return hipErrorInvalidValue;
    if (depth == 1)
        hipLaunchKernelGGL(k_md5_batch_persistent<1>, dim3(grid), dim3(block), 0, s, arena,
                           off, len, order, n, out, counter, grab);
    else if (depth == 2)
        hipLaunchKernelGGL(k_md5_batch_persistent<2>, dim3(grid), dim3(block), 0, s, arena,
                           off, len, order, n, out, counter, grab);
    else
        hipLaunchKernelGGL(k_md5_batch_persistent<3>, dim3(grid), dim3(block), 0, s, arena,
                           off, len, order, n, out, counter, grab);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_md5_chunks(const uint8_t *in, const uint64_t *ends,
                             const uint64_t *n_chunks, uint64_t cap,
                             const uint32_t *order, uint8_t *digests, hipStream_t s)
{
    if (cap == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_md5_chunks, dim3(blocks_for(cap, 64)), dim3(64), 0, s,
                       in, ends, n_chunks, cap, order, digests);
    return hipGetLastError();
}

hipError_t launch_md5_chains(uint8_t *slab, const JobTable &jt, uint32_t seg_bytes,
                             const ChainTable &ct, uint64_t n_chunk_lanes, hipStream_t s)
{
    const uint64_t lanes = jt.n_jobs + n_chunk_lanes;
    if (lanes == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_md5_chains, dim3(blocks_for(lanes, 64)), dim3(64), 0, s, slab, jt,
                       seg_bytes, ct);
    return hipGetLastError();
}

hipError_t launch_nop(hipStream_t s)
{
    hipLaunchKernelGGL(k_nop, dim3(1), dim3(64), 0, s);
    return hipGetLastError();
}

} // namespace crystal
