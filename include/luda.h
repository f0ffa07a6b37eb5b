/*
 * luda.h -- GPU compaction of LSM-tree tables on AMD Instinct MI355X (gfx950).
 *
 * One compaction job merges the selected table of level i with the tables of
 * level i+1 whose key ranges overlap it, drops stale versions, and writes new
 * tables for level i+1 (paper Sec. II-A, "LSM-tree Compaction"; Phases 1-3:
 * unpack, delete-and-sort, pack).  The whole path runs on the GPU: block
 * checksums and prefix-shared key restoration, the merge and drop, and the
 * re-encoding into data blocks, index block, Bloom filter block and footer
 * (Sec. III-A overview, Sec. III-C kernels).
 *
 * Table format: LevelDB's table layout (the paper's prototype is built on
 * LevelDB 1.22, Sec. IV-A), uncompressed blocks (Sec. IV-A), with:
 *   - block trailer: type byte 0 + masked CRC32C of (contents || type);
 *   - internal key = user key || fixed64 LE tag, tag = (seq << 8) | type,
 *     type 1 = value, 0 = deletion;
 *   - index entry key = the block's last internal key, verbatim;
 *   - filter block named "filter.luda.bloom.xxh64": one Bloom filter per
 *     2 KiB window of block start offsets (base_lg 11), bits = max(64, n*b),
 *     k = clamp(b*69/100, 1, 30), probes from XXH64(user key, seed 0).
 * Output tables are byte-for-byte those of the sequential writer rules:
 *   - a data block is finished right after the entry that makes
 *     (entry bytes + 4 * restart points + 4) >= block_size;
 *   - a table is finished right after the block that makes its data bytes
 *     (blocks + 5-byte trailers) >= target_file_size.
 * Drop rule (the stale versions of paper Sec. II-A; live snapshots are a
 * reading of it).  Versions of a user key are ordered newest first (largest
 * tag; equal tags: the earlier input, then the earlier position).  A reader
 * at snapshot s sees the newest version with sequence number <= s, a reader
 * of the current state the newest version.  A version survives iff some
 * such reader sees it: the newest version, and each version v with a
 * snapshot in [seq(v), seq(next newer version)).  When `bottommost` is set,
 * a surviving deletion is dropped too unless a surviving value of its key is
 * older than it.  With no snapshots: the newest version of each user key
 * survives, and a surviving deletion is dropped only when `bottommost` is
 * set.
 *
 * Threading: a context is used by one thread at a time.  Errors are returned
 * as status codes; no exception crosses this interface.
 */
#ifndef LUDA_H
#define LUDA_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LUDA_OK 0
#define LUDA_INVALID_ARG (-1)      /* null pointer, zero block size, ... */
#define LUDA_CORRUPT_FORMAT (-2)   /* bad magic, handle, varint, restart array, key */
#define LUDA_CORRUPT_CHECKSUM (-3) /* a block's masked CRC32C does not match */
#define LUDA_UNSORTED_INPUT (-4)   /* internal keys of one table not strictly increasing */
#define LUDA_UNSUPPORTED (-5)      /* compressed block, or a size beyond the GPU path's limits */
#define LUDA_NOMEM (-6)            /* device or host allocation failed */
#define LUDA_DEVICE (-7)           /* HIP runtime error or a device-side wait gave up */
#define LUDA_CANCELLED (-8)        /* a served job withdrawn before it started (luda_server_cancel) */

/* where a reported corruption lies */
#define LUDA_WHERE_FOOTER 0
#define LUDA_WHERE_INDEX 1
#define LUDA_WHERE_DATA 2

typedef struct luda_ctx luda_ctx;

/* A borrowed byte range: host memory for luda_compact, device memory for the
 * *_dev entry points.  Must stay valid and unchanged until the call returns. */
typedef struct {
  const uint8_t *data;
  uint64_t size;
} luda_buf;

typedef struct {
  uint32_t block_size;         /* data block target bytes (> 0), e.g. 4096 */
  uint32_t restart_interval;   /* entries per restart point (> 0), e.g. 16 */
  uint32_t bloom_bits_per_key; /* Bloom filter bits per key (> 0), e.g. 10 */
  uint32_t bottommost;         /* 1: the output level is the last level */
  uint64_t target_file_size;   /* output table cut threshold in bytes (> 0) */
  const uint64_t *snapshots;   /* live snapshot sequence numbers, strictly ascending, each < 2^56, in host
                                  memory (for every entry point); copied during the call (by
                                  luda_server_submit: before it returns); NULL when n_snapshots is 0 */
  uint32_t n_snapshots;        /* at most LUDA_MAX_SNAPSHOTS; 0: no snapshots */
  uint32_t compression;        /* output data blocks: 0 stored raw (the prototype, Sec. IV-A); 1 stored as
                                  Snappy streams (block type 1) when that saves >= 1/8 of their bytes.
                                  Inputs may hold type-1 data blocks whatever this is. */
} luda_options;
#define LUDA_MAX_SNAPSHOTS 65536

/* The first corruption in reading order: inputs in order; inside an input the
 * footer, the index block, then data blocks in index order; inside a block
 * the trailer (phase 0), the restart array (1), then entries in order (2). */
typedef struct {
  int32_t status;
  uint32_t input;  /* input index inside its job */
  uint32_t where;  /* LUDA_WHERE_* */
  uint32_t phase;  /* 0 trailer, 1 restart array, 2 entries (footer: 0) */
  uint64_t block;  /* data block number inside the input (where == DATA) */
  uint64_t offset; /* byte offset inside the block contents; for the footer,
                      inside the file; saturates at 2^23 - 1 */
} luda_error;

/* One output table.  Its key range is what the store installs it under in
 * level i+1 (the new tables replace the inputs there, Sec. II-A): the smallest
 * and largest internal keys (user key || fixed64 tag) it holds, as byte
 * ranges of luda_result.data (both are stored whole in the table: the first
 * entry of its first data block, and the key of its last index entry). */
typedef struct {
  uint64_t offset;       /* start of this table inside luda_result.data */
  uint64_t size;         /* bytes */
  uint64_t num_entries;  /* entries written to it */
  uint64_t smallest_off; /* smallest internal key: luda_result.data[smallest_off .. + smallest_len) */
  uint64_t smallest_len;
  uint64_t largest_off;  /* largest internal key: luda_result.data[largest_off .. + largest_len) */
  uint64_t largest_len;
} luda_file;

/* Result of one job.  `data` holds every output table back to back; it and
 * `files` are owned by the library until luda_result_free(). */
typedef struct {
  int32_t status;
  luda_error error;
  uint32_t num_files;
  luda_file *files;
  uint8_t *data;       /* host memory (luda_compact), device memory (*_dev) */
  uint64_t data_size;
  uint64_t entries_in, entries_out, dropped_shadowed, dropped_tombstones;
  uint64_t bytes_in, bytes_out;
  double ms_total;     /* wall time of the call */
  void *internal;      /* library bookkeeping */
} luda_result;

/* One job of a batch: inputs[0] is the upper (newest) table. */
typedef struct {
  const luda_buf *inputs;
  uint32_t n_inputs;
  luda_options options;
} luda_job;

/* Create a context on a HIP device: its stream, checksum tables and pinned
 * staging memory (the GPU side of the paper's host/GPU split, Sec. III-A).
 * Returns LUDA_OK, LUDA_NOMEM or LUDA_DEVICE; *out is NULL on failure. */
int luda_ctx_create(int device, luda_ctx **out);
/* Waits for the context's stream, then frees its buffers and the context. */
void luda_ctx_destroy(luda_ctx *ctx);

/* Use a caller-owned HIP stream (hipStream_t) for all work; NULL restores
 * the context's own stream.  The caller keeps ownership of the stream.
 * (The paper overlaps transfers with kernels on streams, Sec. III-D.) */
int luda_set_stream(luda_ctx *ctx, void *hip_stream);

/* Device memory from the caller (e.g. PyTorch's caching allocator), so that
 * one allocator owns the device instead of two.  alloc(user, bytes, stream)
 * returns device memory usable on `stream` (the context's stream, a
 * hipStream_t) or NULL; free(user, ptr, bytes, stream) gives it back, and is
 * called only after the context's stream has finished with it, or with a
 * NULL stream for an output buffer released by luda_result_free (the
 * caller's reads of it must be complete by then, as for any result).  With
 * an allocator set every device buffer of the context's calls comes from it:
 * working buffers and output tables; the library's own pool of output
 * buffers is not used.  NULL (or a struct with alloc == NULL) restores
 * hipMalloc.  The buffers the context already holds are given back to the
 * allocator they came from first.  alloc and free must both be set or both
 * NULL (else LUDA_INVALID_ARG); they may be called from the thread that
 * calls into the context only. */
typedef struct {
  void *(*alloc)(void *user, uint64_t bytes, void *stream);
  void (*free)(void *user, void *ptr, uint64_t bytes, void *stream);
  void *user;
} luda_allocator;
int luda_set_allocator(luda_ctx *ctx, const luda_allocator *allocator);

/* Most device bytes the context's working buffers and output-table buffer
 * may hold at once (0: no limit, the default).  Buffers a call does not use
 * are released first when a call needs more; a call that needs more than the
 * limit by itself fails with LUDA_NOMEM.  The served form gives each worker
 * the server's HBM budget.  luda_mem_held returns what the context holds. */
int luda_set_mem_limit(luda_ctx *ctx, uint64_t bytes);
uint64_t luda_mem_held(luda_ctx *ctx);

/* Compact one job whose inputs are in host memory: the compaction of paper
 * Sec. II-A (Phase 1 unpack: checksums and key restoration; Phase 2 sort
 * and drop of stale versions; Phase 3 pack into new tables), run on the GPU
 * as in Sec. III-A (copy in, kernels, copy out).  inputs[0] is the upper
 * (newest) table, then the overlapping lower tables; input bytes are
 * borrowed until return.  Output tables are returned in host memory owned by
 * the library until luda_result_free.  Zero inputs, or all entries dropped,
 * give LUDA_OK with zero files.  On error no file is returned, the status is
 * also the return value, and out->error locates the first corruption. */
int luda_compact(luda_ctx *ctx, const luda_buf *inputs, uint32_t n_inputs, const luda_options *opt,
                 luda_result *out);

/* As luda_compact (Sec. II-A, III-A), with inputs already in device memory
 * (the kernels' part of Sec. III-A alone; PCIe copies are the caller's); the
 * output tables stay in device memory (out->data is a device pointer owned
 * by the library until luda_result_free). */
int luda_compact_dev(luda_ctx *ctx, const luda_buf *dev_inputs, uint32_t n_inputs,
                     const luda_options *opt, luda_result *out);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc.  The same
 * compaction as luda_compact_dev, but it allocates no device memory and no
 * pinned host memory: every working buffer of the call is carved from a
 * static device array of LUDA_SCRATCH_BYTES (one copy per GPU, held until
 * the process ends), and the output tables are written into the caller's
 * device buffer out_buf of out_cap bytes (out_cap must cover the tables'
 * total size plus 64 bytes).  On success out->data points into out_buf, and
 * luda_result_free releases only the file list.  A call whose working buffers
 * exceed the scratch array (about 200 bytes per entry plus key bytes: some
 * 1.2 million entries), or whose tables exceed out_cap, fails with
 * LUDA_NOMEM and a message naming the limit.  Every context of the process
 * on one GPU shares that GPU's array, which keeps the last call's contents;
 * the library therefore runs these calls one at a time per GPU (a call that
 * overlaps another on the same GPU waits for it).  Arguments, inputs and
 * errors as for luda_compact_dev. */
#define LUDA_SCRATCH_BYTES (256ull << 20)
int luda_compact_dev_noalloc(luda_ctx *ctx, const luda_buf *dev_inputs, uint32_t n_inputs,
                             const luda_options *opt, uint8_t *out_buf, uint64_t out_cap, luda_result *out);

/* Compact many independent jobs (each one job of Sec. II-A) in one pass:
 * every stage runs once over all jobs together (the paper runs one job at a
 * time; batching is this library's own form).  `device_inputs` selects
 * device (1) or host (0) memory for the inputs and outputs.  results[]
 * receives one result per job; a job that fails never changes another job's
 * bytes.  Returns LUDA_OK unless the batch as a whole could not run (then
 * every result carries that status). */
int luda_compact_batch(luda_ctx *ctx, const luda_job *jobs, uint32_t n_jobs, int device_inputs,
                       luda_result *results);

/* Write ordered entries into tables with the same writer as the compaction
 * (Phase 3 of Sec. II-A without the merge: a memtable flush).  Entries are
 * struct-of-arrays in device memory: user keys back to back with n + 1
 * offsets, tags, values back to back with n + 1 offsets; internal keys must
 * be strictly increasing (else LUDA_UNSORTED_INPUT).  Output tables stay in
 * device memory.  Used to build input tables on the device. */
int luda_build_tables_dev(luda_ctx *ctx, uint64_t n, const uint8_t *keys, const uint64_t *koff,
                          const uint64_t *tags, const uint8_t *vals, const uint64_t *voff,
                          const luda_options *opt, luda_result *out);

/* Release a result's tables and file list.  Device outputs go back to the
 * library's pool of output buffers on their device (reused by later calls
 * on any context; the pool holds up to half of the device's memory, its
 * smallest buffers freed first past that; luda_pool_trim): device work
 * the caller queued that reads them must have completed before this call
 * (e.g. its stream synchronized).  Host outputs go back to the pinned pool
 * (luda_pin_reserve).  ctx may be NULL; thread-safe for distinct results,
 * also results of one batched pass. */
void luda_result_free(luda_ctx *ctx, luda_result *r);

/* Name of a status code ("OK", "CORRUPT_CHECKSUM", ...); a static string. */
const char *luda_status_str(int status);
/* Text of the context's last failure (owned by the context, valid until its
 * next call); "" if none. */
const char *luda_last_error(luda_ctx *ctx);

/* Device times (milliseconds) of the last call (the stage costs the paper
 * discusses in Sec. III-B and IV-C), measured with HIP events on
 * the context's stream: "kernel:<name>" for the hot kernels (always), and
 * stage spans when the environment variable LUDA_STAGE_TIMES is set.
 * names[] and ms[] receive up to `cap` entries; returns the count. */
int luda_stage_times(luda_ctx *ctx, const char **names, double *ms, int cap);

/* Counters of the last call (the compaction volume of Sec. IV-C, e.g.
 * "data_bytes_in": bytes of the input data blocks with trailers,
 * "data_bytes_out", "entries_in", "survivors").
 * Same calling convention as luda_stage_times. */
int luda_last_counters(luda_ctx *ctx, const char **names, double *values, int cap);

/* Diagnostics: copy `bytes` bytes at `offset` of the named internal device
 * buffer of the last call into host memory `dst` (e.g. "tu_kp0", "surv").
 * Returns LUDA_OK, or LUDA_INVALID_ARG for an unknown name or range. */
int luda_debug_read(luda_ctx *ctx, const char *name, void *dst, uint64_t offset, uint64_t bytes);

/* Launch parameters of a context (how the parallel work of Sec. III-C is
 * laid out on this GPU).  They change only how work is laid out on the
 * device, never the output bytes. */
typedef struct {
  uint32_t crc_waves;     /* waves per workgroup of the data-block checksum kernel: 4, 8 or 16 (default 8) */
  uint32_t encode_waves;  /* most waves per workgroup of the block encoder, 2..16 (default 4; LDS may
                             allow fewer) */
  uint32_t stride_blocks; /* workgroups per compute unit of the grid-stride kernels, 1..64 (default 16) */
} luda_params;

/* Read the context's parameters into *out (LUDA_INVALID_ARG for NULL). */
int luda_get_params(luda_ctx *ctx, luda_params *out);
/* Set them for the context's later calls; LUDA_INVALID_ARG for a value
 * outside the ranges above (the context keeps its old ones). */
int luda_set_params(luda_ctx *ctx, const luda_params *p);

/* Autotuner (this library's own; the paper fixes its launch shapes, Sec.
 * III-C): runs the given jobs (as luda_compact_batch) rounds + 1 times
 * for each candidate setting, coordinate by coordinate, keeps the setting
 * with the least wall time in the context and returns it (and its time in
 * *best_ms, may be NULL).  Outputs are discarded.  Returns LUDA_OK or the
 * first failure of a run. */
int luda_autotune(luda_ctx *ctx, const luda_job *jobs, uint32_t n_jobs, int device_inputs, uint32_t rounds,
                  luda_params *best, double *best_ms);

/* Cooperative sort (paper Sec. III-D: the decoded tuples go to the CPU,
 * are sorted there and come back): with on != 0, the merge step of this
 * context's calls copies every entry's key, tag and key length to host
 * memory, sorts them on up to 16 host threads and uploads the order; the
 * outputs are the same bytes as with the device merge (on == 0, the
 * default).  For measuring the paper's design choice against the device
 * merge. */
int luda_set_host_sort(luda_ctx *ctx, int on);

/* Host memory for results in host memory is pinned (page-locked), so that
 * the device-to-host copies (the return path of Sec. III-A and III-D) run at
 * link speed.  It comes from a process-wide
 * pool of 1 GiB pinned segments, at most 32 GiB, kept until the process
 * ends; a result larger than a segment gets one of its own, released once
 * the result is freed, and past the cap results go to ordinary memory.
 * Pinning costs about as much time as copying the same bytes, so a caller
 * that knows how much result data it will hold at once can pin it ahead of
 * time: this grows the pool by whole segments until it holds `bytes` (or
 * the cap).  Returns the pool's size in bytes afterwards (smaller than asked
 * if the system refused to pin more).  Thread-safe; needs a HIP device. */
uint64_t luda_pin_reserve(uint64_t bytes);

/* Free the device's pooled output buffers (those of freed results, kept for
 * reuse across calls, as the new tables of Sec. II-A are handed to the
 * store; see luda_result_free).  Returns the bytes freed.  Buffers held by
 * live results and contexts are not touched.  Thread-safe. */
uint64_t luda_pool_trim(int device);

/* Host-side self check of the CRC32C tables the block checksums use (Sec.
 * II-A: every block carries a checksum; no device needed).  Returns 0 when
 * every table agrees with the bitwise definition, else the failing check. */
int luda_selftest_crc(void);

/* ------------------------------------------------------------------------
 * Served form: a request loop in front of the batched compaction (the
 * paper's store issues compaction jobs to the GPU as they arise, Sec. III-A;
 * admission and continuous batching are this library's own).  Jobs are
 * submitted as they arrive (any thread).  A job's expected device footprint
 * is 3 x its input bytes + 1 MiB (outputs up to its input bytes, working set
 * up to twice them: entries of 110 bytes or more on average); a job whose
 * footprint exceeds the whole budget is refused (LUDA_NOMEM).  A job is
 * admitted when its footprint fits under the budget beside the jobs already
 * admitted.  Each worker (its own context and HIP stream, its device memory
 * limited to the budget by luda_set_mem_limit) repeatedly takes the admitted
 * jobs waiting at that moment, up to max_batch_jobs, and runs them as one
 * batched pass (luda_compact_batch); with several workers, batches that
 * arrive while others are on the GPU run on the device at the same time.  If
 * a pass of several jobs fails as a whole (e.g. LUDA_NOMEM), each of its
 * jobs is run again alone.  A job's outputs are identical to those of
 * luda_compact_dev on the same inputs, whatever it is batched with.
 */
typedef struct luda_server luda_server;

typedef struct {
  uint64_t hbm_budget;     /* bytes (> 0) */
  uint32_t max_batch_jobs; /* jobs per batched pass; 0 = no limit */
  uint32_t workers;        /* concurrent batched passes (1..8) */
  uint32_t host_outputs;   /* 1: results are copied to host memory before completion;
                              creation then pins host memory for hbm_budget / 2 bytes
                              of results (luda_pin_reserve) */
} luda_server_cfg;

/* Create a server on a HIP device (its workers' contexts and threads).
 * LUDA_INVALID_ARG for a bad config; a context's failure status otherwise. */
int luda_server_create(int device, const luda_server_cfg *cfg, luda_server **out);

/* Submit a job whose inputs are in device memory; the input bytes are
 * borrowed until the job completes (the descriptor is copied).  Returns
 * LUDA_OK and a ticket, LUDA_NOMEM (no ticket) for a job whose expected
 * footprint exceeds the budget, or LUDA_INVALID_ARG. */
int luda_server_submit(luda_server *s, const luda_job *job, uint64_t *ticket);

/* Withdraw a job that no worker has taken yet: it completes at once with
 * status LUDA_CANCELLED (collect it with luda_server_poll; its inputs are no
 * longer borrowed).  Returns LUDA_OK if it was withdrawn, 1 if it has
 * already started or completed (it then completes normally), or
 * LUDA_INVALID_ARG for an unknown ticket. */
int luda_server_cancel(luda_server *s, uint64_t ticket);

/* Device memory of the server: bytes its workers' contexts hold now
 * (luda_mem_held), and bytes in use on the device as a whole
 * (hipMemGetInfo: total - free).  Returns 2. */
int luda_server_memory(luda_server *s, uint64_t *held_by_workers, uint64_t *device_used);

/* Collect a job: with wait != 0 blocks until it completes.  Returns LUDA_OK
 * and moves its result into *out (free it with luda_result_free(NULL, out)),
 * 1 if it has not completed (wait == 0), or LUDA_INVALID_ARG for an unknown
 * ticket.  *latency_ms (may be NULL) receives completion minus submission
 * time. */
int luda_server_poll(luda_server *s, uint64_t ticket, int wait, luda_result *out, double *latency_ms);

/* Counters since creation (the throughput and latency figures of Sec. IV-B
 * and IV-D come from these jobs): jobs completed, batched passes run, the
 * largest batch, and the peak of admitted (expected) bytes.  Returns the
 * number of values. */
int luda_server_stats(luda_server *s, uint64_t *jobs, uint64_t *batches, uint64_t *max_batch,
                      uint64_t *peak_admitted);

/* Stop the workers (after the jobs already submitted have completed) and
 * free the server, its contexts and any results not collected. */
void luda_server_destroy(luda_server *s);

#ifdef __cplusplus
}
#endif
#endif
