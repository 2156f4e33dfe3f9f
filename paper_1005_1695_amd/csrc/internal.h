// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "crystal.h"

namespace crystal {

// ------------------------------------------------------------- direct hashing
// Job table of a multi-job direct-hashing launch.  n_jobs == 0 selects the
// single-job form: one job at offset 0 of length single_len.
// out_off == nullptr: segment digests form one array indexed by global
// segment number and roots go to a separate array.  Otherwise job j's
// output is its own region at byte offset out_off[j] from the digest base:
// its segment digests, then its root (the job layer's output layout).
struct JobTable {
    const uint64_t *off;
    const uint64_t *len;
    const uint64_t *seg_base;
    uint32_t n_jobs;
    uint64_t single_len;
    const uint64_t *out_off = nullptr;
};

hipError_t launch_md5_segments(const uint8_t *in, const JobTable &jt,
                               uint32_t seg_bytes, uint64_t n_segments,
                               uint8_t *seg_digests, hipStream_t s);
hipError_t launch_md5_roots(const uint8_t *seg_digests, const JobTable &jt,
                            uint32_t seg_bytes, uint8_t *roots, hipStream_t s);
hipError_t launch_md5_whole(const uint8_t *in, uint64_t n, uint8_t *out, hipStream_t s);
// SHA-1 direct hashing (20-byte digests; same job-table conventions).
hipError_t launch_sha1_segments(const uint8_t *in, const JobTable &jt, uint32_t seg_bytes,
                                uint64_t n_segments, uint8_t *seg_digests, hipStream_t s);
hipError_t launch_sha1_roots(const uint8_t *seg_digests, const JobTable &jt, uint32_t seg_bytes,
                             uint8_t *roots, hipStream_t s);
hipError_t launch_md5_batch(const uint8_t *arena, const uint64_t *off,
                            const uint32_t *len, const uint32_t *order,
                            uint64_t n, uint8_t *out, uint32_t block,
                            uint32_t grid, hipStream_t s);
// Persistent batch: waves take `grab`*64 buffers at a time from *counter,
// which must be 0 at launch (launch_zero_u32 before it keeps that graph-safe).
hipError_t launch_md5_batch_persistent(const uint8_t *arena, const uint64_t *off,
                                       const uint32_t *len, const uint32_t *order,
                                       uint64_t n, uint8_t *out, uint32_t *counter,
                                       uint32_t grab, uint32_t depth, uint32_t block,
                                       uint32_t grid, hipStream_t s);
hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t s);
// Digest of each chunk; lane i takes chunk order[i] (order == nullptr: chunk i).
hipError_t launch_md5_chunks(const uint8_t *in, const uint64_t *ends,
                             const uint64_t *n_chunks, uint64_t cap,
                             const uint32_t *order, uint8_t *digests, hipStream_t s);
hipError_t launch_nop(hipStream_t s);

// Chunking jobs of a batch whose chunk digests run in one chains launch.  All
// offsets are bytes from the slab base; job j's output region holds
// [u64 n][u64 ends[cap]...] and receives the packed digests after ends[n].
constexpr uint64_t kNoOrder = ~0ull;
struct ChainTable {
    const uint64_t *in_off;  // input of job j
    const uint64_t *out_off; // output region of job j
    const uint64_t *ord_off; // chunk order (uint32 per lane), or kNoOrder
    const uint64_t *cap;     // chunk capacity of job j
    const uint64_t *lane0;   // n_jobs + 1 entries: first lane of job j (64-aligned)
    uint32_t n_jobs;
};
// Roots of the direct group jt (outputs in the jobs' own regions, jt.out_off
// set; jt.n_jobs may be 0) and the chunk digests of ct, one launch.
hipError_t launch_md5_chains(uint8_t *slab, const JobTable &jt, uint32_t seg_bytes,
                             const ChainTable &ct, uint64_t n_chunk_lanes, hipStream_t s);

// ---------------------------------------------------------------- chunking
// Byte range owned by one candidate lane; one bit-summary word per range.
constexpr uint64_t kRangeBytes = 4096;
constexpr uint32_t kWindow = 48;

struct CdcGeom {
    uint64_t n;
    uint64_t n_ranges;   // ceil(n / kRangeBytes)
    uint64_t tile_bytes; // selection tile P (>= max_len)
    uint64_t warm_bytes; // speculative warm-up D before each tile
    uint32_t n_tiles;
    uint32_t tile_cap;   // max chunk starts one tile can hold
    uint64_t ord_cap;    // chunk order entries (the most chunks n bytes can hold)
    size_t off_l1, off_l2, off_cnt, off_rscan, off_exit, off_first, off_tcnt,
        off_starts, off_toff, off_flags, off_bad, off_misc, off_hist, off_ord, total;
};

// Resolved parameters (defaults applied, validated).
struct CdcParams {
    uint64_t base, b48, mask, min_len, max_len;
    uint32_t mask_bits;
};

bool cdc_resolve(const crystal_cdc_params *p, CdcParams *out, const char **why);
CdcGeom cdc_geometry(uint64_t n, const CdcParams &p);
uint64_t cdc_max_chunks(uint64_t n, const CdcParams &p);

hipError_t launch_cdc_candidates(const uint8_t *in, const CdcGeom &g,
                                 const CdcParams &p, uint8_t *ws, hipStream_t s);
hipError_t launch_cdc_compact(const CdcGeom &g, uint8_t *ws, uint64_t *d_count,
                              uint64_t *d_cand, uint64_t cap, hipStream_t s);
// Chunk ends from the candidate bitmap.  With `order` non-null it also makes
// the chunk order (as launch_chunk_order does) and returns it in *order.
hipError_t launch_cdc_select(const CdcGeom &g, const CdcParams &p, uint8_t *ws,
                             uint64_t *d_n_chunks, uint64_t *d_ends,
                             uint64_t cap, hipStream_t s, const uint32_t **order = nullptr);
// Chunk order for the digest launch: chunk indices grouped into 1 KiB length
// classes, longest class first (order inside a class unspecified).  Writes
// ws + g.off_ord and returns that pointer in *order.
hipError_t launch_chunk_order(const CdcGeom &g, uint8_t *ws, const uint64_t *d_n_chunks,
                              const uint64_t *d_ends, uint64_t cap, const uint32_t **order,
                              hipStream_t s);
hipError_t launch_window_hash(const uint8_t *in, uint64_t n, uint64_t base,
                              uint64_t *w, hipStream_t s);

// ------------------------------------------------------------- host helpers
void set_error(int code, const char *fmt, ...);
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int64_t now_ns();

} // namespace crystal
