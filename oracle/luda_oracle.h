/*
 * luda_oracle.h -- plain sequential CPU compactor (TEST INFRASTRUCTURE ONLY).
 *
 * This is the checker against which the GPU library is tested.  It shares no
 * code with the GPU path, and only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  The product path never calls it.
 *
 * It computes, sequentially and in the paper's order, one compaction job
 * (paper Sec. II-A, "LSM-tree Compaction"):
 *   Phase 1 Unpack  -- verify each data block's checksum, restore the full keys
 *                      from the shared-prefix encoding;
 *   Phase 2 Sort    -- merge all restored pairs in key order and drop stale
 *                      versions and (at the bottom level) deletions;
 *   Phase 3 Pack    -- group pairs into blocks by the block size, compute shared
 *                      keys and block checksums, then the index and the Bloom
 *                      filter block of each table.
 * The byte layout is LevelDB's table layout (the paper builds on LevelDB 1.22,
 * Sec. IV-A; blocks hold shared-prefix keys, values and a checksum, Sec. II-A)
 * with these writer choices: block trailers carry a masked CRC32C; index
 * entries use the verbatim last internal key of each block; the filter block
 * holds one Bloom filter per 2 KiB window of block start offsets, built with
 * XXH64 double hashing at the configured bits per key (10 in the paper).
 * With compression on, data blocks are stored as Snappy raw streams (block
 * type 1) when that saves at least an eighth of their bytes; the stream
 * follows the deterministic rules written out above ref_snappy_compress in
 * luda_oracle.c.  Inputs may hold type-1 data blocks whatever the option.
 * Parity unpinned: agreement with a stock Snappy library (none is available
 * here); the codec is pinned by hand-assembled streams, closed forms of the
 * writer's rules and an independent decoder in the tests.
 */
#ifndef LUDA_ORACLE_H
#define LUDA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  REF_OK = 0,
  REF_INVALID_ARG = -1,
  REF_CORRUPT_FORMAT = -2,
  REF_CORRUPT_CHECKSUM = -3,
  REF_UNSORTED_INPUT = -4,
  REF_UNSUPPORTED = -5,
  REF_NOMEM = -6,
};

enum { REF_WHERE_FOOTER = 0, REF_WHERE_INDEX = 1, REF_WHERE_DATA = 2 };
enum { REF_PHASE_TRAILER = 0, REF_PHASE_RESTARTS = 1, REF_PHASE_ENTRIES = 2 };

typedef struct {
  uint32_t block_size;         /* data block target bytes */
  uint32_t restart_interval;   /* entries between restart points (>= 1) */
  uint32_t bloom_bits_per_key; /* Bloom filter bits per key (>= 1) */
  uint32_t bottommost;         /* 1: drop deletions that no kept value lies under */
  uint64_t target_file_size;   /* output file cut threshold (>= 1) */
  const uint64_t *snapshots;   /* live snapshot sequence numbers, strictly ascending, < 2^56 */
  uint32_t n_snapshots;        /* 0: no snapshots */
  uint32_t compression;        /* data blocks: 0 stored raw, 1 Snappy when it saves >= 1/8 */
} ref_options;

typedef struct {
  int32_t status;  /* REF_* */
  uint32_t input;  /* input table index */
  uint32_t where;  /* REF_WHERE_* */
  uint32_t phase;  /* REF_PHASE_* inside a block */
  uint64_t block;  /* data block number (where == DATA) */
  uint64_t offset; /* byte offset inside the block contents (or the file, for the footer) */
} ref_error;

/* A borrowed, sorted list of entries (struct of arrays). */
typedef struct {
  uint64_t n;
  const uint8_t *keys;   /* concatenated user keys */
  const uint64_t *koff;  /* n + 1 */
  const uint64_t *tags;  /* (sequence << 8) | type */
  const uint8_t *vals;   /* concatenated values */
  const uint64_t *voff;  /* n + 1 */
} ref_entries;

/* Decoded entries (owned by the oracle; free with ref_free_decoded). */
typedef struct {
  uint64_t n;
  uint8_t *keys;
  uint64_t *koff;
  uint64_t *tags;
  uint8_t *vals;
  uint64_t *voff;
} ref_decoded;

typedef struct {
  uint32_t num_files;
  uint64_t *file_off;          /* num_files + 1 offsets into data */
  uint8_t *data;               /* all output tables back to back */
  uint64_t entries_in, entries_out, dropped_shadowed, dropped_tombstones;
  uint64_t bytes_in, bytes_out;
  /* stage trace, for stage-level comparisons */
  uint32_t n_inputs;
  uint64_t *input_first;       /* n_inputs + 1: decoded-entry index range per input */
  uint64_t *surv;              /* entries_out: decoded-entry index of each survivor */
  uint64_t n_blocks;
  uint64_t *block_first;       /* n_blocks + 1: first survivor of each output data block */
  uint64_t *file_first_block;  /* num_files + 1 */
} ref_result;

/* checksums and hashes */
uint32_t ref_crc32c_bitwise(const uint8_t *p, uint64_t n);
uint32_t ref_crc32c(const uint8_t *p, uint64_t n);
uint32_t ref_crc32c_extend(uint32_t crc, const uint8_t *p, uint64_t n);
uint32_t ref_mask_crc(uint32_t crc);
uint32_t ref_unmask_crc(uint32_t masked);
uint64_t ref_xxh64(const uint8_t *p, uint64_t n, uint64_t seed);

/* varints: put returns the byte count; get returns bytes consumed, 0 on error */
int ref_put_varint64(uint8_t *dst, uint64_t v);
int ref_get_varint32(const uint8_t *p, const uint8_t *limit, uint32_t *v);
int ref_get_varint64(const uint8_t *p, const uint8_t *limit, uint64_t *v);

/* Bloom filter over n user keys: writes ref_bloom_size() bytes */
uint64_t ref_bloom_size(uint64_t n, uint32_t bits_per_key);
void ref_bloom_build(const uint8_t *keys, const uint64_t *koff, uint64_t n, uint32_t bits_per_key,
                     uint8_t *out);
int ref_bloom_may_match(const uint8_t *filter, uint64_t len, const uint8_t *key, uint64_t klen);

/* Snappy raw streams (block type 1): decompress returns REF_OK with a
 * malloc'd buffer, or REF_CORRUPT_FORMAT with *err_off at the first element
 * that cannot be decoded; compress writes at most ref_snappy_max(n) bytes. */
int ref_snappy_decompress(const uint8_t *src, uint64_t n, uint8_t **out, uint64_t *out_len,
                          uint64_t *err_off);
uint64_t ref_snappy_max(uint64_t n);
uint64_t ref_snappy_compress(const uint8_t *src, uint64_t n, uint8_t *dst);

/* Phase 3 over an already ordered list (used to write input tables too). */
int ref_build_tables(const ref_entries *in, const ref_options *opt, ref_result **out);

/* Phase 1 for one table. */
int ref_decode_table(const uint8_t *sst, uint64_t size, uint32_t input_index, ref_decoded **out,
                     ref_error *err);

/* The whole job: inputs[0] is the upper (newest) table, then the lower ones. */
int ref_compact(const uint8_t *const *inputs, const uint64_t *sizes, uint32_t n_inputs,
                const ref_options *opt, ref_result **out, ref_error *err);

void ref_free_result(ref_result *r);
void ref_free_decoded(ref_decoded *d);

#ifdef __cplusplus
}
#endif
#endif
