/*
 * crystal.h -- C ABI of the MI355X hashing-offload library.
 *
 * The library follows the task abstraction of CrystalGPU (Gharaibeh,
 * Al-Kiswany, Ripeanu): an application hands the framework "jobs" -- copy
 * input to the GPU, run a kernel, copy results back (Sec. 2.1) -- and the
 * framework reuses pre-allocated pinned-host and device buffers and overlaps
 * the copy-in / kernel / copy-out stages of consecutive jobs (Sec. 4.2,
 * Fig. 4).  The job API mirrors the paper's public interface (Fig. 3):
 *
 *     paper                          this library
 *     init(max_in, max_out)          crystal_init
 *     finalize()                     crystal_finalize
 *     job_get() / job_put()          crystal_buffer_acquire / _release
 *     job_submit(job)                crystal_submit(task, kernel_id, in, out)
 *     job_synch(job)                 crystal_wait
 *     job_query(job)                 crystal_poll
 *     job_t.callback_func            crystal_task.callback
 *
 * The work a job performs is one of a fixed set of hashing kernels used by
 * content-addressable storage (Sec. 2.2, Sec. 5.2): direct block hashing
 * (MD5 of each fixed-size segment, then MD5 of the concatenated segment
 * digests) and content-defined chunking (48-byte polynomial rolling hash,
 * chunk boundaries with minimum and maximum lengths, MD5 of each chunk).
 * The device-level entry points run the same kernels on memory that is
 * already resident on the GPU.
 *
 * Conventions for every function:
 *   - return 0 (CRYSTAL_OK) on success, a negative CRYSTAL_E* code on error;
 *     crystal_last_error() then holds a thread-local message.
 *   - "d_" pointers are device memory of the current HIP device, "h_"
 *     pointers host memory.  Streams are hipStream_t passed as void*; NULL is
 *     the null stream.  Device-level calls are asynchronous on that stream.
 *   - Byte arrays of digests are the raw 16-byte MD5 form (RFC 1321
 *     Sec. 3.5: words A,B,C,D, each little-endian).
 *   - Readability: every input buffer of a device-level call must be readable
 *     up to the next 16-byte boundary after its last byte (kernels load whole
 *     aligned vectors; bytes past the end never enter a digest).
 *   - All functions are thread-safe unless stated otherwise.
 */
#ifndef CRYSTAL_H
#define CRYSTAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------- status codes */
#define CRYSTAL_OK 0
#define CRYSTAL_EINVAL (-1)    /* bad argument, size or kernel id */
#define CRYSTAL_EAGAIN (-2)    /* non-blocking request could not be met now */
#define CRYSTAL_ENOMEM (-3)    /* pool or device allocation failed */
#define CRYSTAL_EBUSY (-4)     /* buffer still referenced by a running task */
#define CRYSTAL_ETIMEDOUT (-5) /* wait deadline passed */
#define CRYSTAL_EDEVICE (-6)   /* HIP runtime reported an error */
#define CRYSTAL_ESTATE (-7)    /* library not initialised / already initialised */
#define CRYSTAL_ECANCELED (-8) /* task cancelled by crystal_finalize */
#define CRYSTAL_PENDING 1      /* crystal_task.status while not finished */

/* ------------------------------------------------------------- kernel ids */
#define CRYSTAL_K_NOP 0        /* copy in, empty kernel, copy the same bytes out
                                  (the framework-overhead job of Sec. 5.1) */
#define CRYSTAL_K_MD5_DIRECT 1 /* direct block hashing */
#define CRYSTAL_K_CDC 2        /* content-defined chunking + per-chunk MD5 */
#define CRYSTAL_K_MD5 3        /* one MD5 of the whole input */
#define CRYSTAL_K_SHA1_DIRECT 4 /* direct block hashing with SHA-1 (FIPS 180-4), the
                                   digest of the paper's measurements (Sec. 5.2) */

/* Direct hashing parameters.  segment_bytes: multiple of 64, 0 = 4096. */
typedef struct crystal_direct_params {
    uint32_t segment_bytes;
    uint32_t reserved;
} crystal_direct_params;

/* Chunking parameters.  Window hash at byte i >= 47:
 *   W_i = sum_{k=0}^{47} in[i-47+k] * base^(47-k)  (mod 2^64),
 * i is a candidate when (W_i & (2^mask_bits - 1)) == 0.  Walking the input,
 * a chunk that started at s ends after byte i when (i+1-s >= min_len and i is
 * a candidate) or i+1-s == max_len; the last chunk ends at the input end.
 * Zero fields take defaults: mask_bits 13, min_len 2048, max_len 65536.
 * window must be 0 or 48.  1 <= min_len <= max_len <= 2^31, mask_bits <= 64. */
typedef struct crystal_cdc_params {
    uint64_t base;
    uint64_t min_len;
    uint64_t max_len;
    uint32_t mask_bits;
    uint32_t window;
} crystal_cdc_params;

/* ======================================================================
 * Job API (Sec. 3, Fig. 2-3; design Sec. 4.2)
 * ==================================================================== */

#define CRYSTAL_F_DEFAULT 0u

typedef struct crystal_config {
    size_t max_input_bytes;   /* largest job input (Fig. 3 init); > 0 */
    size_t max_output_bytes;  /* largest job output; 0 = derived from input */
    size_t host_pool_bytes;   /* pinned host slab behind buffer_acquire;
                                 0 = 4 * (max_input + max_output) */
    size_t device_pool_bytes; /* device slab from which each admitted job
                                 takes input, output and scratch; 0 = 8 *
                                 per-job need of the largest job */
    uint32_t n_streams;       /* compute streams jobs are spread over (each
                                 also carries its jobs' copy-out); 0 = 3 */
    uint32_t max_in_flight;   /* dispatched but unfinished jobs; 0 = 4*n_streams */
    int32_t device;           /* HIP device ordinal */
    uint32_t flags;           /* CRYSTAL_F_* */
    void *device_slab;        /* optional caller-owned device memory of
                                 device_pool_bytes (e.g. from PyTorch); the
                                 library then allocates no device pool itself */
    void **streams;           /* optional caller-owned streams:
                                 n_copy_streams + n_streams entries, copy-in
                                 streams first, then the compute streams */
    uint32_t n_copy_streams;  /* copy-in streams that batches rotate over,
                                 1..8; 0 = 2 if the library creates its
                                 streams and n_streams + 2 fits the process's
                                 hardware queues (GPU_MAX_HW_QUEUES, default
                                 4), else 1 */
} crystal_config;

typedef struct crystal_buf crystal_buf; /* opaque pooled/wrapped host buffer */
typedef struct crystal_task crystal_task;
typedef void (*crystal_callback)(crystal_task *task, void *user);

/* A job descriptor.  Caller-owned; must stay alive and unmodified from
 * crystal_submit until it is finished (crystal_poll != 0). */
struct crystal_task {
    /* set by the caller */
    size_t in_bytes;           /* bytes of the input buffer to process */
    const void *params;        /* crystal_direct_params / crystal_cdc_params
                                  for that kernel, or NULL for defaults */
    crystal_callback callback; /* optional; runs on a library completion
                                  thread once the output is in host memory;
                                  must not block; may release buffers */
    void *user;
    /* written by the library */
    volatile int32_t status;   /* CRYSTAL_PENDING, then 0 or a CRYSTAL_E* */
    int32_t stream_index;      /* stream the job ran on */
    size_t out_bytes;          /* bytes of output written */
    int64_t t_submit_ns;       /* CLOCK_MONOTONIC timestamps */
    int64_t t_admit_ns;        /* device memory reserved, copies enqueued */
    int64_t t_done_ns;         /* output in host memory */
    void *internal[4];         /* library use */
};

/* Start the library on cfg->device: pinned host slab, device slab, streams,
 * events, the dispatcher and completion threads.  CRYSTAL_ESTATE if already
 * initialised, CRYSTAL_ENOMEM if a slab cannot be allocated. */
int crystal_init(const crystal_config *cfg);

/* Cancel jobs not yet dispatched (they finish with CRYSTAL_ECANCELED), wait
 * for dispatched ones, stop the threads and free everything the library
 * allocated.  Buffers not yet released become invalid. */
int crystal_finalize(void);

/* Take a pinned host buffer of at least `bytes` from the pool (the paper's
 * job_get).  flags & CRYSTAL_NONBLOCK: CRYSTAL_EAGAIN instead of waiting when
 * the pool cannot serve it now.  CRYSTAL_EINVAL if bytes exceeds the pool. */
#define CRYSTAL_NONBLOCK 1
int crystal_buffer_acquire(size_t bytes, int flags, crystal_buf **out);

/* Wrap caller-owned host memory as a buffer, without copying.  For full link
 * speed it should be pinned (hipHostMalloc, torch pin_memory).  The memory
 * must outlive every task that uses it; the caller keeps ownership. */
int crystal_buffer_wrap(void *host_ptr, size_t bytes, crystal_buf **out);

/* Return a buffer (the paper's job_put).  CRYSTAL_EBUSY while a submitted,
 * unfinished task references it.  Allowed inside a callback. */
int crystal_buffer_release(crystal_buf *b);

void *crystal_buffer_host(crystal_buf *b);
size_t crystal_buffer_size(const crystal_buf *b);

/* Queue a job (the paper's job_submit): in->[0, t->in_bytes) is copied to a
 * pooled device region, kernel_id runs on it, and its output is copied into
 * `out`.  Returns immediately.  CRYSTAL_EINVAL for an unknown kernel, an
 * input larger than max_input_bytes or than `in`, or an `out` smaller than
 * crystal_output_bytes(kernel_id, in_bytes, params).
 * Output layouts:
 *   MD5_DIRECT: n_seg digests (16 B each) then the root digest (16 B)
 *   SHA1_DIRECT: n_seg digests (20 B each) then the root digest (20 B);
 *               the root is SHA-1 of the concatenated segment digests
 *   CDC:        uint64 n_chunks, uint64 ends[n_chunks] (exclusive end
 *               offsets, last = in_bytes), then n_chunks 16-byte digests
 *   MD5:        one 16-byte digest
 *   NOP:        the input bytes */
int crystal_submit(crystal_task *t, int kernel_id, crystal_buf *in, crystal_buf *out);

/* Worst-case output bytes of a job (size `out` for this). */
size_t crystal_output_bytes(int kernel_id, size_t in_bytes, const void *params);

/* Block until the task finishes (the paper's job_synch) or timeout_ns passes
 * (< 0: no limit).  Returns the task status or CRYSTAL_ETIMEDOUT.  Do not wait
 * on a task from its own callback. */
int crystal_wait(crystal_task *t, int64_t timeout_ns);

/* 1 finished OK, 0 pending, < 0 finished with that error (job_query). */
int crystal_poll(const crystal_task *t);

/* Thread-local description of the last error on this thread. */
const char *crystal_last_error(void);

typedef struct crystal_stats {
    uint64_t submitted, completed, failed;
    uint64_t bytes_in, bytes_out;
    uint64_t device_pool_bytes, device_pool_free, device_pool_min_free;
    uint64_t host_pool_bytes, host_pool_free;
    uint32_t outstanding, running;
} crystal_stats;
int crystal_get_stats(crystal_stats *s);

/* ======================================================================
 * Device-level hot path: same kernels, device-resident data, caller-owned
 * memory, asynchronous on `stream`.
 * ==================================================================== */

/* Direct hashing of n_jobs inputs in one launch.  Job j is
 * d_in[d_job_off[j], d_job_off[j] + d_job_len[j]); d_seg_base (n_jobs+1
 * entries) is the prefix sum of ceil(len_j / segment_bytes), n_segments its
 * last entry.  Writes segment digests to d_seg_digests (n_segments x 16 B,
 * job j's at index d_seg_base[j]) and job roots to d_roots (n_jobs x 16 B).
 * segment_bytes: multiple of 64 (0 = 4096).  Job starts 16-byte aligned run
 * the vector-load path; other starts are hashed correctly, more slowly. */
int crystal_md5_direct_device(const void *d_in, const uint64_t *d_job_off,
                              const uint64_t *d_job_len,
                              const uint64_t *d_seg_base, uint32_t n_jobs,
                              uint64_t n_segments, uint32_t segment_bytes,
                              void *d_seg_digests, void *d_roots, void *stream);

/* The two steps of crystal_md5_direct_device, callable on their own (same
 * arguments): segment digests only, then roots from those digests. */
int crystal_md5_segments_device(const void *d_in, const uint64_t *d_job_off,
                                const uint64_t *d_job_len,
                                const uint64_t *d_seg_base, uint32_t n_jobs,
                                uint64_t n_segments, uint32_t segment_bytes,
                                void *d_seg_digests, void *stream);
int crystal_md5_roots_device(const uint64_t *d_seg_base, uint32_t n_jobs,
                             uint32_t segment_bytes, const void *d_seg_digests,
                             void *d_roots, void *stream);

/* Direct hashing with SHA-1 (FIPS 180-4; the digest of the paper's own
 * direct-hashing measurements, Sec. 5.2): same arguments and job layout as
 * crystal_md5_direct_device, with 20-byte digests -- d_seg_digests holds
 * n_segments x 20 B (job j's at byte 20 * d_seg_base[j]), d_roots n_jobs x
 * 20 B, and each root is SHA-1 over the job's concatenated segment digests.
 * The digest array must be readable up to the next 16-byte boundary after
 * its last byte (the root loader reads whole 16-byte vectors).  The two
 * steps are callable on their own, as for MD5. */
int crystal_sha1_direct_device(const void *d_in, const uint64_t *d_job_off,
                               const uint64_t *d_job_len,
                               const uint64_t *d_seg_base, uint32_t n_jobs,
                               uint64_t n_segments, uint32_t segment_bytes,
                               void *d_seg_digests, void *d_roots, void *stream);
int crystal_sha1_segments_device(const void *d_in, const uint64_t *d_job_off,
                                 const uint64_t *d_job_len,
                                 const uint64_t *d_seg_base, uint32_t n_jobs,
                                 uint64_t n_segments, uint32_t segment_bytes,
                                 void *d_seg_digests, void *stream);
int crystal_sha1_roots_device(const uint64_t *d_seg_base, uint32_t n_jobs,
                              uint32_t segment_bytes, const void *d_seg_digests,
                              void *d_roots, void *stream);

/* MD5 of n_buf buffers: buffer m is d_arena[d_off[m], d_off[m] + d_len[m]),
 * digest to d_out + 16 m.  d_order (optional, n_buf entries) is the order in
 * which lanes take buffers (e.g. longest first); NULL = index order.
 * block: workgroup size (multiple of 64, <= 1024, 0 = 256); grid: workgroups
 * (0 = enough for one buffer per lane).  Lanes loop over buffers. */
int crystal_md5_batch_device(const void *d_arena, const uint64_t *d_off,
                             const uint32_t *d_len, const uint32_t *d_order,
                             uint64_t n_buf, void *d_out, uint32_t block,
                             uint32_t grid, void *stream);

/* Scratch bytes the chunking calls need for an input of n bytes. */
size_t crystal_cdc_workspace_bytes(uint64_t n, const crystal_cdc_params *p);
/* Capacity (chunk count) that is always enough for an input of n bytes. */
uint64_t crystal_cdc_max_chunks(uint64_t n, const crystal_cdc_params *p);

/* Whole chunking pipeline on d_in[0, n): candidates, boundary selection,
 * per-chunk MD5.  Writes the chunk count to *d_n_chunks (device), the end
 * offsets to d_ends and the digests to d_digests (cap entries each;
 * cap >= crystal_cdc_max_chunks).  d_ws: crystal_cdc_workspace_bytes bytes. */
int crystal_cdc_device(const void *d_in, uint64_t n, const crystal_cdc_params *p,
                       void *d_ws, size_t ws_bytes, uint64_t *d_n_chunks,
                       uint64_t *d_ends, void *d_digests, uint64_t cap,
                       void *stream);

/* Step 1: candidate positions.  Leaves the candidate set in d_ws (read by
 * crystal_cdc_select_device) and, when d_cand is non-NULL, also writes the
 * ascending positions (at most cap) to d_cand and their count to *d_count. */
int crystal_cdc_candidates_device(const void *d_in, uint64_t n,
                                  const crystal_cdc_params *p, void *d_ws,
                                  size_t ws_bytes, uint64_t *d_count,
                                  uint64_t *d_cand, uint64_t cap, void *stream);

/* Step 2: chunk ends from the candidate set a preceding
 * crystal_cdc_candidates_device call left in d_ws for the same n and p. */
int crystal_cdc_select_device(uint64_t n, const crystal_cdc_params *p,
                              void *d_ws, size_t ws_bytes, uint64_t *d_n_chunks,
                              uint64_t *d_ends, uint64_t cap, void *stream);

/* Step 3: MD5 of each chunk [end_{k-1}, end_k) of d_in (end_{-1} = 0); the
 * count is read from *d_n_chunks on the device, cap bounds it. */
int crystal_md5_chunks_device(const void *d_in, const uint64_t *d_ends,
                              const uint64_t *d_n_chunks, uint64_t cap,
                              void *d_digests, void *stream);

/* Diagnostic: the full 64-bit window hash W_i at every byte (0 for i < 47). */
int crystal_window_hash_device(const void *d_in, uint64_t n, uint64_t base,
                               uint64_t *d_w, void *stream);

/* ======================================================================
 * Batching (the paper's batch-processing class, Sec. 2.2 B): many small
 * independent buffers hashed by one persistent launch per branch, planned
 * once (longest-first order, tuned launch shape) and replayed.  Replays are
 * direct stream launches; HIP-graph capture of the replay is switched off in
 * this version.
 * ==================================================================== */

typedef struct crystal_batch_desc {
    const void *d_arena;   /* device bytes */
    const uint64_t *d_off; /* n_buf offsets into d_arena */
    const uint32_t *d_len; /* n_buf lengths */
    uint64_t n_buf;
    void *d_out;           /* n_buf x 16 B digests */
    void *stream;          /* stream replays are launched on */
} crystal_batch_desc;

typedef struct crystal_batch_tuning {
    uint32_t block;          /* workgroup size: 64, 128, 192 or 256 */
    uint32_t waves_per_simd; /* persistent grid = 256 CUs x 4 SIMDs x this */
    uint32_t grab;           /* buffers a wave takes per work-counter grab,
                                in units of 64 */
    uint32_t n_streams;      /* parallel branches (streams joined by events) */
    uint32_t sorted;         /* lane order: 0 = index order, 1 = longest first
                                over the whole batch, W > 1 = longest first
                                within each run of W consecutive buffers */
    uint32_t depth;          /* loader depth: 128-byte groups per lane read
                                ahead of its compression, 1..3 (0 = 2) */
    uint32_t tail;           /* the last `tail` entries of the lane order
                                are re-sorted longest first as one block, so
                                the launch ends on its shortest buffers
                                (0 = no re-sort; clamped to n_buf) */
    float replay_ms;         /* measured time of one replay */
} crystal_batch_tuning;

typedef struct crystal_batch crystal_batch;

#define CRYSTAL_TUNE_NONE 0  /* use *fixed (or defaults) */
#define CRYSTAL_TUNE_FULL 1  /* grid search, replay-timed */

/* Build a plan: length-sort the buffers (longest first), choose launch
 * parameters (tune_flags) by timing replays.  CRYSTAL_TUNE_FULL searches the
 * loader depth, waves per SIMD, workgroup size and sort window, with a tail
 * of four rounds of resident lanes.
 * The library allocates the plan's own small device tables.  *fixed may be
 * NULL. */
int crystal_batch_plan(const crystal_batch_desc *d, int tune_flags,
                       const crystal_batch_tuning *fixed, crystal_batch **out);
/* Replay the plan `iters` times on the desc's stream (asynchronous). */
int crystal_batch_run(crystal_batch *b, int iters);
int crystal_batch_get_tuning(const crystal_batch *b, crystal_batch_tuning *t);
void crystal_batch_free(crystal_batch *b);

/* ======================================================================
 * Naive per-job path (the "original" application pattern the paper
 * improves on, Sec. 5.2 Fig. 6): allocate device buffers, blocking copy in,
 * the same kernels, blocking copy out, free -- serialised, no pooling.
 * ==================================================================== */
typedef struct crystal_stage_times {
    double alloc_ms, copy_in_ms, kernel_ms, copy_out_ms, free_ms, total_ms;
} crystal_stage_times;

int crystal_naive_run(int kernel_id, const void *params, const void *h_in,
                      size_t n, void *h_out, size_t out_cap, size_t *out_bytes,
                      crystal_stage_times *st);

/* ======================================================================
 * Stream / serving driver: feeds a list of jobs through the job API from a
 * native generator thread.  Open loop: job k is submitted at its scheduled
 * arrival time whether or not earlier jobs are done, and its latency is
 * measured from that scheduled time.  Closed loop (arrival_s all 0): jobs
 * are submitted as fast as the task layer accepts them.  Requires
 * crystal_init.
 * ==================================================================== */
typedef struct crystal_drive_job {
    const void *h_in;   /* host input (pinned for full speed) */
    uint64_t bytes;
    void *h_out;        /* host output, >= crystal_output_bytes */
    uint64_t out_cap;
    double arrival_s;   /* scheduled submit time from the start */
    int32_t kernel_id;
    int32_t status;     /* written: final task status */
    double latency_s;   /* written: done - scheduled arrival */
    double admit_wait_s;/* written: admitted - scheduled arrival */
} crystal_drive_job;

typedef struct crystal_drive_result {
    double wall_s;      /* first scheduled arrival to last completion */
    uint64_t bytes;     /* input bytes of successful jobs */
    uint64_t ok, failed;
} crystal_drive_result;

/* window == 0: open loop; window > 0: closed loop, at most `window` jobs in
 * the system.  direct / cdc: parameters of the two job kinds (NULL =
 * defaults).  Per-job status, latency and admission wait are written back
 * into jobs[]. */
int crystal_drive(crystal_drive_job *jobs, uint64_t n_jobs,
                  const crystal_direct_params *direct,
                  const crystal_cdc_params *cdc, uint32_t window,
                  crystal_drive_result *res);

#ifdef __cplusplus
}
#endif
#endif /* CRYSTAL_H */
