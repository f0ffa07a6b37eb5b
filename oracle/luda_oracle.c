/*
 * luda_oracle.c -- plain sequential CPU compactor (TEST INFRASTRUCTURE ONLY).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this file's library; the GPU library shares none of its code.
 *
 * Each function states the passage of the paper it follows:
 *   Sec. II-A "LSM-tree Compaction": block = shared keys + values + checksum;
 *     a table = data blocks + index + Bloom filter block; Phases 1-3.
 *   Sec. IV-A "Configuration and Methodology": LevelDB 1.22 format, 10 bits/key
 *     Bloom filters, 4 KiB blocks, no compression.
 * The layout details the paper leaves open follow LevelDB's published table
 * format, with the writer choices listed in luda_oracle.h.
 */
#define _GNU_SOURCE /* qsort_r */
#include "luda_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* CRC32C (Castagnoli).  The checksum of Sec. II-A ("typically CRC32"); the
 * Castagnoli polynomial with LevelDB's masking.  Reflected polynomial
 * 0x82F63B78, initial value and final xor 0xFFFFFFFF. */

#define CRC32C_POLY_REFLECTED 0x82F63B78u

uint32_t ref_crc32c_bitwise(const uint8_t *p, uint64_t n) {
  uint32_t crc = 0xFFFFFFFFu;
  for (uint64_t i = 0; i < n; i++) {
    crc ^= p[i];
    for (int b = 0; b < 8; b++) crc = (crc >> 1) ^ (CRC32C_POLY_REFLECTED & (0u - (crc & 1u)));
  }
  return crc ^ 0xFFFFFFFFu;
}

static uint32_t crc_table[256];
static int crc_table_ready = 0;

static void crc_table_init(void) {
  /* table[b] = the register after shifting byte b through eight bitwise steps */
  for (uint32_t b = 0; b < 256; b++) {
    uint32_t r = b;
    for (int k = 0; k < 8; k++) r = (r >> 1) ^ (CRC32C_POLY_REFLECTED & (0u - (r & 1u)));
    crc_table[b] = r;
  }
  crc_table_ready = 1;
}

uint32_t ref_crc32c_extend(uint32_t crc, const uint8_t *p, uint64_t n) {
  if (!crc_table_ready) crc_table_init();
  uint32_t r = crc ^ 0xFFFFFFFFu;
  for (uint64_t i = 0; i < n; i++) r = crc_table[(r ^ p[i]) & 0xFFu] ^ (r >> 8);
  return r ^ 0xFFFFFFFFu;
}

uint32_t ref_crc32c(const uint8_t *p, uint64_t n) { return ref_crc32c_extend(0, p, n); }

/* LevelDB stores a rotated-and-offset CRC so that a CRC of data that itself
 * contains CRCs does not degenerate. */
#define CRC_MASK_DELTA 0xa282ead8u
uint32_t ref_mask_crc(uint32_t c) { return ((c >> 15) | (c << 17)) + CRC_MASK_DELTA; }
uint32_t ref_unmask_crc(uint32_t m) {
  uint32_t r = m - CRC_MASK_DELTA;
  return (r >> 17) | (r << 15);
}

/* ------------------------------------------------------------------------ */
/* XXH64, written from the published xxHash specification (Y. Collet,
 * "xxHash fast digest algorithm", XXH64 section).  Used as the Bloom hash. */

#define XP1 0x9E3779B185EBCA87ull
#define XP2 0xC2B2AE3D27D4EB4Full
#define XP3 0x165667B19E3779F9ull
#define XP4 0x85EBCA77C2B2AE63ull
#define XP5 0x27D4EB2F165667C5ull

static uint64_t rotl64(uint64_t x, int r) { return (x << r) | (x >> (64 - r)); }
static uint64_t rd64(const uint8_t *p) {
  uint64_t v = 0;
  for (int i = 7; i >= 0; i--) v = (v << 8) | p[i];
  return v;
}
static uint32_t rd32(const uint8_t *p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
static uint64_t xx_round(uint64_t acc, uint64_t lane) {
  acc += lane * XP2;
  acc = rotl64(acc, 31);
  return acc * XP1;
}
static uint64_t xx_merge(uint64_t acc, uint64_t v) {
  acc ^= xx_round(0, v);
  return acc * XP1 + XP4;
}

uint64_t ref_xxh64(const uint8_t *p, uint64_t n, uint64_t seed) {
  const uint8_t *end = p + n;
  uint64_t acc;
  if (n >= 32) {
    uint64_t v1 = seed + XP1 + XP2, v2 = seed + XP2, v3 = seed, v4 = seed - XP1;
    while ((uint64_t)(end - p) >= 32) {
      v1 = xx_round(v1, rd64(p));
      v2 = xx_round(v2, rd64(p + 8));
      v3 = xx_round(v3, rd64(p + 16));
      v4 = xx_round(v4, rd64(p + 24));
      p += 32;
    }
    acc = rotl64(v1, 1) + rotl64(v2, 7) + rotl64(v3, 12) + rotl64(v4, 18);
    acc = xx_merge(acc, v1);
    acc = xx_merge(acc, v2);
    acc = xx_merge(acc, v3);
    acc = xx_merge(acc, v4);
  } else {
    acc = seed + XP5;
  }
  acc += n;
  while ((uint64_t)(end - p) >= 8) {
    acc ^= xx_round(0, rd64(p));
    acc = rotl64(acc, 27) * XP1 + XP4;
    p += 8;
  }
  if ((uint64_t)(end - p) >= 4) {
    acc ^= (uint64_t)rd32(p) * XP1;
    acc = rotl64(acc, 23) * XP2 + XP3;
    p += 4;
  }
  while (p < end) {
    acc ^= (uint64_t)(*p) * XP5;
    acc = rotl64(acc, 11) * XP1;
    p++;
  }
  acc ^= acc >> 33;
  acc *= XP2;
  acc ^= acc >> 29;
  acc *= XP3;
  acc ^= acc >> 32;
  return acc;
}

/* ------------------------------------------------------------------------ */
/* varints (unsigned LEB128, low group first) and fixed-width little endian */

int ref_put_varint64(uint8_t *dst, uint64_t v) {
  int n = 0;
  while (v >= 128) {
    dst[n++] = (uint8_t)(v | 128);
    v >>= 7;
  }
  dst[n++] = (uint8_t)v;
  return n;
}

/* A varint32 is at most 5 bytes and its value must fit 32 bits. */
int ref_get_varint32(const uint8_t *p, const uint8_t *limit, uint32_t *v) {
  uint64_t r = 0;
  for (int i = 0; i < 5; i++) {
    if (p + i >= limit) return 0;
    uint8_t b = p[i];
    r |= (uint64_t)(b & 127) << (7 * i);
    if (!(b & 128)) {
      if (r > 0xFFFFFFFFull) return 0;
      *v = (uint32_t)r;
      return i + 1;
    }
  }
  return 0;
}

/* A varint64 is at most 10 bytes and its value must fit 64 bits. */
int ref_get_varint64(const uint8_t *p, const uint8_t *limit, uint64_t *v) {
  uint64_t r = 0;
  for (int i = 0; i < 10; i++) {
    if (p + i >= limit) return 0;
    uint8_t b = p[i];
    if (i == 9 && b > 1) return 0;
    r |= (uint64_t)(b & 127) << (7 * i);
    if (!(b & 128)) {
      *v = r;
      return i + 1;
    }
  }
  return 0;
}

static void put_fixed32(uint8_t *d, uint32_t v) {
  for (int i = 0; i < 4; i++) d[i] = (uint8_t)(v >> (8 * i));
}
static void put_fixed64(uint8_t *d, uint64_t v) {
  for (int i = 0; i < 8; i++) d[i] = (uint8_t)(v >> (8 * i));
}

/* ------------------------------------------------------------------------ */
/* growable byte buffer */

typedef struct {
  uint8_t *p;
  uint64_t n, cap;
  int oom;
} buf_t;

static int buf_reserve(buf_t *b, uint64_t extra) {
  if (b->oom) return 0;
  if (b->n + extra <= b->cap) return 1;
  uint64_t nc = b->cap ? b->cap : 4096;
  while (nc < b->n + extra) nc *= 2;
  uint8_t *q = (uint8_t *)realloc(b->p, nc);
  if (!q) {
    b->oom = 1;
    return 0;
  }
  b->p = q;
  b->cap = nc;
  return 1;
}
static void buf_put(buf_t *b, const void *src, uint64_t n) {
  if (!buf_reserve(b, n)) return;
  if (n) memcpy(b->p + b->n, src, n);
  b->n += n;
}
static void buf_byte(buf_t *b, uint8_t v) { buf_put(b, &v, 1); }
static void buf_varint(buf_t *b, uint64_t v) {
  uint8_t t[10];
  buf_put(b, t, (uint64_t)ref_put_varint64(t, v));
}
static void buf_fixed32(buf_t *b, uint32_t v) {
  uint8_t t[4];
  put_fixed32(t, v);
  buf_put(b, t, 4);
}
static void buf_fixed64(buf_t *b, uint64_t v) {
  uint8_t t[8];
  put_fixed64(t, v);
  buf_put(b, t, 8);
}

/* growable u64 array */
typedef struct {
  uint64_t *p;
  uint64_t n, cap;
  int oom;
} vec_t;
static void vec_push(vec_t *v, uint64_t x) {
  if (v->oom) return;
  if (v->n == v->cap) {
    uint64_t nc = v->cap ? v->cap * 2 : 64;
    uint64_t *q = (uint64_t *)realloc(v->p, nc * sizeof(uint64_t));
    if (!q) {
      v->oom = 1;
      return;
    }
    v->p = q;
    v->cap = nc;
  }
  v->p[v->n++] = x;
}

/* ------------------------------------------------------------------------ */
/* Bloom filter (Sec. II-A: each table carries a Bloom filter block; Sec. IV-A:
 * 10 bits per key).  bits = max(64, n * b) rounded up to whole bytes; k =
 * b * 69 / 100 clamped to [1, 30]; probe g, g + h2, g + 2 h2, ... (mod 2^32)
 * with (g, h2) the low and high halves of XXH64(key, seed 0); k is stored in
 * the filter's last byte. */

static uint32_t bloom_k(uint32_t bits_per_key) {
  uint32_t k = bits_per_key * 69u / 100u;
  if (k < 1) k = 1;
  if (k > 30) k = 30;
  return k;
}

uint64_t ref_bloom_size(uint64_t n, uint32_t bits_per_key) {
  uint64_t bits = n * bits_per_key;
  if (bits < 64) bits = 64;
  return (bits + 7) / 8 + 1;
}

void ref_bloom_build(const uint8_t *keys, const uint64_t *koff, uint64_t n, uint32_t bits_per_key,
                     uint8_t *out) {
  uint64_t bytes = ref_bloom_size(n, bits_per_key) - 1;
  uint64_t bits = bytes * 8;
  uint32_t k = bloom_k(bits_per_key);
  memset(out, 0, bytes);
  for (uint64_t i = 0; i < n; i++) {
    uint64_t h = ref_xxh64(keys + koff[i], koff[i + 1] - koff[i], 0);
    uint32_t g = (uint32_t)h, delta = (uint32_t)(h >> 32);
    for (uint32_t j = 0; j < k; j++) {
      uint64_t pos = (uint64_t)g % bits;
      out[pos >> 3] |= (uint8_t)(1u << (pos & 7));
      g += delta;
    }
  }
  out[bytes] = (uint8_t)k;
}

int ref_bloom_may_match(const uint8_t *filter, uint64_t len, const uint8_t *key, uint64_t klen) {
  if (len < 2) return 0;
  uint64_t bits = (len - 1) * 8;
  uint32_t k = filter[len - 1];
  if (k > 30) return 1; /* reserved encodings match everything */
  uint64_t h = ref_xxh64(key, klen, 0);
  uint32_t g = (uint32_t)h, delta = (uint32_t)(h >> 32);
  for (uint32_t j = 0; j < k; j++) {
    uint64_t pos = (uint64_t)g % bits;
    if (!(filter[pos >> 3] & (1u << (pos & 7)))) return 0;
    g += delta;
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Internal keys: user key || fixed64(tag), tag = (sequence << 8) | type.
 * Order: user key bytewise ascending (a proper prefix sorts first), then tag
 * descending (newer versions first). */

static int cmp_user(const uint8_t *a, uint64_t la, const uint8_t *b, uint64_t lb) {
  uint64_t m = la < lb ? la : lb;
  int c = m ? memcmp(a, b, m) : 0;
  if (c) return c;
  return la < lb ? -1 : (la > lb ? 1 : 0);
}

static int cmp_internal(const uint8_t *a, uint64_t la, uint64_t ta, const uint8_t *b, uint64_t lb,
                        uint64_t tb) {
  int c = cmp_user(a, la, b, lb);
  if (c) return c;
  return ta > tb ? -1 : (ta < tb ? 1 : 0);
}


/* ------------------------------------------------------------------------ */
/* A read-only view of entries by pointer, so values need not be copied. */

typedef struct {
  uint64_t n;
  const uint8_t **kp;
  const uint64_t *kl;
  const uint64_t *tag;
  const uint8_t **vp;
  const uint64_t *vl;
} view_t;

static void bloom_build_view(const view_t *v, uint64_t e0, uint64_t e1, uint32_t bits_per_key,
                             uint8_t *out) {
  uint64_t n = e1 - e0;
  uint64_t bytes = ref_bloom_size(n, bits_per_key) - 1;
  uint64_t bits = bytes * 8;
  uint32_t k = bloom_k(bits_per_key);
  memset(out, 0, bytes);
  for (uint64_t i = e0; i < e1; i++) {
    uint64_t h = ref_xxh64(v->kp[i], v->kl[i], 0);
    uint32_t g = (uint32_t)h, delta = (uint32_t)(h >> 32);
    for (uint32_t j = 0; j < k; j++) {
      uint64_t pos = (uint64_t)g % bits;
      out[pos >> 3] |= (uint8_t)(1u << (pos & 7));
      g += delta;
    }
  }
  out[bytes] = (uint8_t)k;
}

/* ------------------------------------------------------------------------ */
/* Compressed blocks (block type 1).  The paper's prototype stores blocks
 * uncompressed and names compression as future work (Sec. IV-A); its base,
 * LevelDB, compresses data blocks with Snappy.  The stored form of a type-1
 * block is a Snappy raw stream, written here from the public format
 * description: a varint32 of the uncompressed length, then elements whose
 * tag byte's low two bits select a literal (0), a copy with an 11-bit offset
 * and length 4..11 (1), a copy with a 16-bit offset (2) or with a 32-bit
 * offset (3); copies may overlap the bytes they produce. */

/* Decode a stream of n bytes.  Returns REF_OK and a malloc'd buffer of the
 * declared length, or REF_CORRUPT_FORMAT with *err_off = the offset of the
 * first element that cannot be decoded (0 for a bad length preamble, n when
 * the stream ends before the declared length is produced). */
int ref_snappy_decompress(const uint8_t *src, uint64_t n, uint8_t **out, uint64_t *out_len,
                          uint64_t *err_off) {
  *out = NULL;
  *out_len = 0;
  *err_off = 0;
  uint32_t len;
  int a = ref_get_varint32(src, src + n, &len);
  if (!a) return REF_CORRUPT_FORMAT;
  /* an element of b bytes yields at most 64/3 * b bytes, so a stream of n
   * bytes never yields 22 * n: a larger declared length fails before the
   * buffer is full */
  uint64_t cap = len < 22 * n ? len : 22 * n;
  uint8_t *o = (uint8_t *)malloc(cap + 1);
  if (!o) return REF_NOMEM;
  uint64_t ip = (uint64_t)a, op = 0;
  while (ip < n) {
    uint64_t t = ip;
    uint8_t tag = src[ip++];
    uint64_t L, off = 0;
    int kind = tag & 3;
    if (kind == 0) {
      L = (uint64_t)(tag >> 2) + 1;
      if (L > 60) {
        uint32_t nb = (uint32_t)(L - 60); /* 1..4 length bytes follow */
        if (nb > n - ip) goto bad;
        L = 0;
        for (uint32_t k = 0; k < nb; k++) L |= (uint64_t)src[ip + k] << (8 * k);
        L += 1;
        ip += nb;
      }
      if (L > n - ip || L > len - op) goto bad;
      memcpy(o + op, src + ip, L);
      ip += L;
      op += L;
      continue;
    }
    if (kind == 1) {
      if (1 > n - ip) goto bad;
      L = ((tag >> 2) & 7) + 4;
      off = ((uint64_t)(tag >> 5) << 8) | src[ip];
      ip += 1;
    } else if (kind == 2) {
      if (2 > n - ip) goto bad;
      L = (uint64_t)(tag >> 2) + 1;
      off = (uint64_t)src[ip] | ((uint64_t)src[ip + 1] << 8);
      ip += 2;
    } else {
      if (4 > n - ip) goto bad;
      L = (uint64_t)(tag >> 2) + 1;
      off = rd32(src + ip);
      ip += 4;
    }
    if (off == 0 || off > op || L > len - op) goto bad;
    for (uint64_t k = 0; k < L; k++) o[op + k] = o[op - off + k];
    op += L;
    continue;
  bad:
    free(o);
    *err_off = t;
    return REF_CORRUPT_FORMAT;
  }
  if (op != len) {
    free(o);
    *err_off = n;
    return REF_CORRUPT_FORMAT;
  }
  *out = o;
  *out_len = len;
  return REF_OK;
}

/* The writer's compressor.  Any valid stream decodes to the same bytes; the
 * bytes of the stream itself follow from these rules, which the GPU writer
 * follows as well:
 *   - the block is cut into 64 KiB fragments; copies stay inside a fragment;
 *   - inside a fragment, positions are taken in groups of 64; each position p
 *     with 4 bytes left looks up a 4096-entry table under the hash of those
 *     4 bytes (Knuth's multiplicative hash: the little-endian word times
 *     0x9E3779B1, top 12 bits), whose entry is the last earlier position with
 *     that hash among the groups before p's group; after the group's lookups,
 *     every position of the group is entered, later positions last;
 *   - parsing is greedy from the fragment start: at position p, if its
 *     candidate's 4 bytes equal p's, the copy runs as far as the bytes keep
 *     agreeing (up to the fragment end) and p moves past it; otherwise p
 *     moves on by one and the byte joins the pending literal;
 *   - a literal is one element however long; a copy of length L at offset d
 *     is split into pieces of 64 while L >= 68, one of 60 if L is then above
 *     64, and a last piece in the 2-byte form (tag 1) when it is at most 11
 *     long with d < 2048, else in the 3-byte form (tag 2). */

#define SNAPPY_FRAGMENT 65536u
#define SNAPPY_GROUP 64u
#define SNAPPY_HASH_BITS 12

/* A literal of k > 60 bytes has a header of 2 or more bytes and the copy
 * after it may save only one byte (4 raw bytes in 3), so a stream can exceed
 * its input by about one byte per 65; n / 6 + 32 covers that with room. */
uint64_t ref_snappy_max(uint64_t n) { return n + n / 6 + 32; }

static uint32_t snappy_hash(uint32_t v) { return (v * 0x9E3779B1u) >> (32 - SNAPPY_HASH_BITS); }

static uint64_t put_literal(uint8_t *d, const uint8_t *s, uint64_t k) {
  if (k == 0) return 0;
  uint64_t p = 0, m = k - 1;
  if (m < 60) {
    d[p++] = (uint8_t)(m << 2);
  } else {
    uint32_t nb = 1;
    while (nb < 4 && (m >> (8 * nb))) nb++;
    d[p++] = (uint8_t)((59 + nb) << 2);
    for (uint32_t i = 0; i < nb; i++) d[p++] = (uint8_t)(m >> (8 * i));
  }
  memcpy(d + p, s, k);
  return p + k;
}

static uint64_t put_copy_piece(uint8_t *d, uint64_t off, uint64_t L) {
  if (L <= 11 && off < 2048) {
    d[0] = (uint8_t)(1 | ((L - 4) << 2) | ((off >> 8) << 5));
    d[1] = (uint8_t)(off & 0xFF);
    return 2;
  }
  d[0] = (uint8_t)(2 | ((L - 1) << 2));
  d[1] = (uint8_t)(off & 0xFF);
  d[2] = (uint8_t)(off >> 8);
  return 3;
}

static uint64_t put_copy(uint8_t *d, uint64_t off, uint64_t L) {
  uint64_t p = 0;
  while (L >= 68) {
    d[p++] = (uint8_t)(2 | (63 << 2));
    d[p++] = (uint8_t)(off & 0xFF);
    d[p++] = (uint8_t)(off >> 8);
    L -= 64;
  }
  if (L > 64) {
    d[p++] = (uint8_t)(2 | (59 << 2));
    d[p++] = (uint8_t)(off & 0xFF);
    d[p++] = (uint8_t)(off >> 8);
    L -= 60;
  }
  return p + put_copy_piece(d + p, off, L);
}

/* Compress n bytes into dst (ref_snappy_max(n) bytes); returns the length. */
uint64_t ref_snappy_compress(const uint8_t *src, uint64_t n, uint8_t *dst) {
  uint64_t q = (uint64_t)ref_put_varint64(dst, n);
  int32_t table[1 << SNAPPY_HASH_BITS];
  int32_t cand[SNAPPY_GROUP];
  for (uint64_t f0 = 0; f0 < n; f0 += SNAPPY_FRAGMENT) {
    const uint8_t *r = src + f0;
    uint64_t m = n - f0 < SNAPPY_FRAGMENT ? n - f0 : SNAPPY_FRAGMENT;
    for (uint32_t h = 0; h < (1u << SNAPPY_HASH_BITS); h++) table[h] = -1;
    uint64_t pos = 0, lit = 0;
    for (uint64_t b = 0; b < m; b += SNAPPY_GROUP) {
      uint64_t e = b + SNAPPY_GROUP < m ? b + SNAPPY_GROUP : m;
      for (uint64_t p = b; p < e; p++) cand[p - b] = p + 4 <= m ? table[snappy_hash(rd32(r + p))] : -1;
      for (uint64_t p = b; p < e && p + 4 <= m; p++) table[snappy_hash(rd32(r + p))] = (int32_t)p;
      while (pos < e) {
        int32_t c = cand[pos - b];
        if (c >= 0 && memcmp(r + c, r + pos, 4) == 0) {
          uint64_t L = 4;
          while (pos + L < m && r[c + L] == r[pos + L]) L++;
          q += put_literal(dst + q, r + lit, pos - lit);
          q += put_copy(dst + q, pos - (uint64_t)c, L);
          pos += L;
          lit = pos;
        } else {
          pos++;
        }
      }
    }
    q += put_literal(dst + q, r + lit, m - lit);
  }
  return q;
}

/* ------------------------------------------------------------------------ */
/* Phase 3 "Pack" (Sec. II-A): group entries into data blocks by the block
 * size, prefix-compress each key against the previous key of its block (every
 * R-th entry of a block is a restart point and stores its key whole), then
 * checksum each block.  Each table then gets its filter block, metaindex
 * block, index block and footer.
 *   Block cut: right after the entry that makes
 *     (entry bytes so far) + 4 * (restart points) + 4 >= block_size.
 *   Table cut: right after the block that makes the table's data bytes
 *     (blocks plus their 5-byte trailers) >= target_file_size.
 * These are the greedy rules of LevelDB's table builder, which the paper's
 * prototype modifies (Sec. IV-A). */

#define FILTER_BASE_LG 11
static const char FILTER_NAME[] = "filter.luda.bloom.xxh64";
#define TABLE_MAGIC 0xdb4775248b80fb57ull

typedef struct {
  const ref_options *opt;
  const view_t *in;
  buf_t out;              /* all finished tables, back to back */
  vec_t file_off;         /* start of each table in out */
  vec_t block_first;      /* first entry of every data block, all tables */
  vec_t file_first_block; /* first global block index of each table */
  /* current table */
  int file_open;
  uint64_t file_base;
  vec_t blk_off, blk_size, blk_first, blk_end; /* this table's data blocks */
  /* current block */
  buf_t blk;
  vec_t restarts;
  uint32_t counter;
  buf_t last_key;
  uint64_t blk_n, blk_first_entry;
  buf_t ikey;
} packer_t;

static void append_typed_block(buf_t *out, const uint8_t *contents, uint64_t n, uint8_t type) {
  uint8_t tr[5];
  tr[0] = type;
  uint32_t crc = ref_crc32c_extend(ref_crc32c(contents, n), tr, 1);
  put_fixed32(tr + 1, ref_mask_crc(crc));
  buf_put(out, contents, n);
  buf_put(out, tr, 5);
}

/* filter, metaindex and index blocks, and data blocks without compression:
 * block type 0 (the prototype stores every block uncompressed, Sec. IV-A) */
static void append_block(buf_t *out, const uint8_t *contents, uint64_t n) {
  append_typed_block(out, contents, n, 0);
}

/* A data block with compression on: stored as a type-1 block when the
 * compressed form saves at least an eighth of the raw bytes, else as type 0
 * (LevelDB's rule).  Returns the stored size. */
static uint64_t append_data_block(buf_t *out, const uint8_t *contents, uint64_t n, uint32_t compression) {
  if (compression == 1) {
    uint8_t *z = (uint8_t *)malloc(ref_snappy_max(n));
    if (!z) {
      out->oom = 1;
      return 0;
    }
    uint64_t zn = ref_snappy_compress(contents, n, z);
    if (zn < n - n / 8) {
      append_typed_block(out, z, zn, 1);
      free(z);
      return zn;
    }
    free(z);
  }
  append_block(out, contents, n);
  return n;
}

static void block_reset(packer_t *pk) {
  pk->blk.n = 0;
  pk->restarts.n = 0;
  vec_push(&pk->restarts, 0);
  pk->counter = 0;
  pk->last_key.n = 0;
  pk->blk_n = 0;
}

static void block_add(packer_t *pk, const uint8_t *ikey, uint64_t iklen, const uint8_t *val,
                      uint64_t vlen) {
  uint64_t shared = 0;
  if (pk->counter < pk->opt->restart_interval) {
    uint64_t m = pk->last_key.n < iklen ? pk->last_key.n : iklen;
    while (shared < m && pk->last_key.p[shared] == ikey[shared]) shared++;
  } else {
    vec_push(&pk->restarts, pk->blk.n);
    pk->counter = 0;
  }
  buf_varint(&pk->blk, shared);
  buf_varint(&pk->blk, iklen - shared);
  buf_varint(&pk->blk, vlen);
  buf_put(&pk->blk, ikey + shared, iklen - shared);
  buf_put(&pk->blk, val, vlen);
  pk->last_key.n = 0;
  buf_put(&pk->last_key, ikey, iklen);
  pk->counter++;
}

static uint64_t block_estimate(const packer_t *pk) { return pk->blk.n + 4 * pk->restarts.n + 4; }

static void flush_block(packer_t *pk, uint64_t end_entry) {
  for (uint64_t i = 0; i < pk->restarts.n; i++) buf_fixed32(&pk->blk, (uint32_t)pk->restarts.p[i]);
  buf_fixed32(&pk->blk, (uint32_t)pk->restarts.n);
  vec_push(&pk->blk_off, pk->out.n - pk->file_base);
  vec_push(&pk->blk_first, pk->blk_first_entry);
  vec_push(&pk->blk_end, end_entry);
  vec_push(&pk->block_first, pk->blk_first_entry);
  vec_push(&pk->blk_size, append_data_block(&pk->out, pk->blk.p, pk->blk.n, pk->opt->compression));
  block_reset(pk);
}

static void internal_key(buf_t *b, const uint8_t *ukey, uint64_t klen, uint64_t tag) {
  b->n = 0;
  buf_put(b, ukey, klen);
  buf_fixed64(b, tag);
}

static void handle_bytes(buf_t *b, uint64_t off, uint64_t size) {
  b->n = 0;
  buf_varint(b, off);
  buf_varint(b, size);
}

static void finish_file(packer_t *pk) {
  const view_t *in = pk->in;
  const uint64_t nb = pk->blk_off.n;
  const uint32_t bpk = pk->opt->bloom_bits_per_key;
  buf_t tmp = {0}, hb = {0}, blk = {0};

  /* filter block: filter f holds the user keys of the blocks whose start
   * offset o satisfies (o >> 11) == f; filters run to the last block's window */
  uint64_t nfilt = (pk->blk_off.p[nb - 1] >> FILTER_BASE_LG) + 1;
  vec_t foff = {0};
  uint64_t b = 0;
  for (uint64_t f = 0; f < nfilt; f++) {
    vec_push(&foff, blk.n);
    uint64_t b0 = b;
    while (b < nb && (pk->blk_off.p[b] >> FILTER_BASE_LG) == f) b++;
    if (b == b0) continue; /* no block starts in this window: empty filter */
    uint64_t e0 = pk->blk_first.p[b0], e1 = pk->blk_end.p[b - 1];
    uint64_t sz = ref_bloom_size(e1 - e0, bpk);
    if (!buf_reserve(&blk, sz)) break;
    bloom_build_view(in, e0, e1, bpk, blk.p + blk.n);
    blk.n += sz;
  }
  uint32_t array_off = (uint32_t)blk.n;
  for (uint64_t f = 0; f < foff.n; f++) buf_fixed32(&blk, (uint32_t)foff.p[f]);
  buf_fixed32(&blk, array_off);
  buf_byte(&blk, FILTER_BASE_LG);
  uint64_t filter_off = pk->out.n - pk->file_base, filter_size = blk.n;
  append_block(&pk->out, blk.p, blk.n);

  /* metaindex block: a single entry naming the filter block (a restart) */
  handle_bytes(&hb, filter_off, filter_size);
  blk.n = 0;
  buf_varint(&blk, 0);
  buf_varint(&blk, sizeof(FILTER_NAME) - 1);
  buf_varint(&blk, hb.n);
  buf_put(&blk, FILTER_NAME, sizeof(FILTER_NAME) - 1);
  buf_put(&blk, hb.p, hb.n);
  buf_fixed32(&blk, 0);
  buf_fixed32(&blk, 1);
  uint64_t meta_off = pk->out.n - pk->file_base, meta_size = blk.n;
  append_block(&pk->out, blk.p, blk.n);

  /* index block: one entry per data block, key = the block's last internal
   * key, value = the block handle; every entry is a restart point */
  blk.n = 0;
  vec_t rs = {0};
  for (uint64_t i = 0; i < nb; i++) {
    uint64_t last = pk->blk_end.p[i] - 1;
    internal_key(&tmp, in->kp[last], in->kl[last], in->tag[last]);
    handle_bytes(&hb, pk->blk_off.p[i], pk->blk_size.p[i]);
    vec_push(&rs, blk.n);
    buf_varint(&blk, 0);
    buf_varint(&blk, tmp.n);
    buf_varint(&blk, hb.n);
    buf_put(&blk, tmp.p, tmp.n);
    buf_put(&blk, hb.p, hb.n);
  }
  for (uint64_t i = 0; i < rs.n; i++) buf_fixed32(&blk, (uint32_t)rs.p[i]);
  buf_fixed32(&blk, (uint32_t)rs.n);
  uint64_t index_off = pk->out.n - pk->file_base, index_size = blk.n;
  append_block(&pk->out, blk.p, blk.n);

  /* footer: metaindex handle, index handle, zero padding to 40 bytes, magic */
  uint8_t footer[48];
  memset(footer, 0, sizeof footer);
  int p = ref_put_varint64(footer, meta_off);
  p += ref_put_varint64(footer + p, meta_size);
  p += ref_put_varint64(footer + p, index_off);
  p += ref_put_varint64(footer + p, index_size);
  put_fixed64(footer + 40, TABLE_MAGIC);
  buf_put(&pk->out, footer, 48);

  if (tmp.oom || hb.oom || blk.oom || foff.oom || rs.oom) pk->out.oom = 1;
  free(tmp.p);
  free(hb.p);
  free(blk.p);
  free(foff.p);
  free(rs.p);
  pk->blk_off.n = pk->blk_size.n = pk->blk_first.n = pk->blk_end.n = 0;
  pk->file_open = 0;
}

static void pk_free(packer_t *pk) {
  free(pk->blk_off.p);
  free(pk->blk_size.p);
  free(pk->blk_first.p);
  free(pk->blk_end.p);
  free(pk->blk.p);
  free(pk->restarts.p);
  free(pk->last_key.p);
  free(pk->ikey.p);
}

/* Pack the whole (ordered) view; fills the tables and the block/file trace. */
static int pack_view(const view_t *in, const ref_options *opt, ref_result *res) {
  packer_t pk;
  memset(&pk, 0, sizeof pk);
  pk.opt = opt;
  pk.in = in;
  block_reset(&pk);
  for (uint64_t i = 0; i < in->n; i++) {
    if (!pk.file_open) {
      pk.file_open = 1;
      pk.file_base = pk.out.n;
      vec_push(&pk.file_off, pk.out.n);
      vec_push(&pk.file_first_block, pk.block_first.n);
    }
    if (pk.blk_n == 0) pk.blk_first_entry = i;
    internal_key(&pk.ikey, in->kp[i], in->kl[i], in->tag[i]);
    block_add(&pk, pk.ikey.p, pk.ikey.n, in->vp[i], in->vl[i]);
    pk.blk_n++;
    if (block_estimate(&pk) >= opt->block_size) {
      flush_block(&pk, i + 1);
      if (pk.out.n - pk.file_base >= opt->target_file_size) finish_file(&pk);
    }
  }
  if (pk.blk_n > 0) flush_block(&pk, in->n);
  if (pk.file_open) finish_file(&pk);
  vec_push(&pk.file_off, pk.out.n);
  vec_push(&pk.file_first_block, pk.block_first.n);
  vec_push(&pk.block_first, in->n);
  int oom = pk.out.oom || pk.file_off.oom || pk.block_first.oom || pk.file_first_block.oom ||
            pk.blk.oom || pk.ikey.oom;
  pk_free(&pk);
  res->num_files = (uint32_t)(pk.file_off.n - 1);
  res->file_off = pk.file_off.p;
  res->data = pk.out.p;
  res->bytes_out = pk.out.n;
  res->n_blocks = pk.block_first.n - 1;
  res->block_first = pk.block_first.p;
  res->file_first_block = pk.file_first_block.p;
  return oom ? REF_NOMEM : REF_OK;
}

static int check_options(const ref_options *opt) {
  if (!opt || opt->block_size < 1 || opt->restart_interval < 1 || opt->bloom_bits_per_key < 1 ||
      opt->target_file_size < 1 || opt->compression > 1 || (opt->n_snapshots && !opt->snapshots))
    return REF_INVALID_ARG;
  for (uint32_t i = 0; i < opt->n_snapshots; i++)
    if (opt->snapshots[i] >> 56 || (i && opt->snapshots[i] <= opt->snapshots[i - 1])) return REF_INVALID_ARG;
  return REF_OK;
}

int ref_build_tables(const ref_entries *in, const ref_options *opt, ref_result **out) {
  if (!in || !out || check_options(opt) != REF_OK) return REF_INVALID_ARG;
  *out = NULL;
  uint64_t n = in->n;
  view_t v;
  v.n = n;
  v.kp = (const uint8_t **)malloc((n + 1) * sizeof(void *));
  v.vp = (const uint8_t **)malloc((n + 1) * sizeof(void *));
  uint64_t *kl = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
  uint64_t *vl = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
  ref_result *r = (ref_result *)calloc(1, sizeof(ref_result));
  if (!v.kp || !v.vp || !kl || !vl || !r) {
    free(v.kp), free(v.vp), free(kl), free(vl), free(r);
    return REF_NOMEM;
  }
  for (uint64_t i = 0; i < n; i++) {
    v.kp[i] = in->keys + in->koff[i];
    kl[i] = in->koff[i + 1] - in->koff[i];
    v.vp[i] = in->vals + in->voff[i];
    vl[i] = in->voff[i + 1] - in->voff[i];
  }
  v.kl = kl;
  v.vl = vl;
  v.tag = in->tags;
  int rc = pack_view(&v, opt, r);
  r->entries_in = r->entries_out = n;
  free(v.kp), free(v.vp), free(kl), free(vl);
  if (rc != REF_OK) {
    ref_free_result(r);
    return rc;
  }
  *out = r;
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Phase 1 "Unpack" (Sec. II-A): recompute each data block's checksum, then
 * restore the full keys from the shared-prefix encoding.  The table is read
 * footer -> index block -> data blocks in index order; the filter and
 * metaindex blocks are not needed by a compaction and are not read.  The
 * first failure in that order is reported. */

typedef struct {
  int32_t status;
  uint32_t phase;
  uint64_t offset;
} blk_err;

typedef int (*visit_fn)(void *ctx, const uint8_t *key, uint64_t klen, const uint8_t *val,
                        uint64_t vlen);

/* Walk one block's entries with the format checks in order: restart array
 * (count, then each offset: first is 0, strictly increasing, inside the entry
 * area), then each entry in sequence (three varint32 headers inside the entry
 * area, shared <= previous key length, key delta and value inside the entry
 * area, shared == 0 at a restart point, no entry spanning a restart point),
 * then the caller's own checks on the restored key. */
static blk_err walk_block(const uint8_t *c, uint64_t size, visit_fn visit, void *ctx, buf_t *key) {
  blk_err e = {REF_OK, REF_PHASE_RESTARTS, 0};
  if (size < 4) {
    e.status = REF_CORRUPT_FORMAT;
    return e;
  }
  uint64_t nr = rd32(c + size - 4);
  if (nr == 0 || nr > (size - 4) / 4) {
    e.status = REF_CORRUPT_FORMAT;
    e.offset = size - 4;
    return e;
  }
  uint64_t data_end = size - 4 - 4 * nr;
  uint64_t prev = 0;
  for (uint64_t k = 0; k < nr; k++) {
    uint64_t r = rd32(c + data_end + 4 * k);
    if ((k == 0 ? r != 0 : r <= prev) || r >= data_end) {
      e.status = REF_CORRUPT_FORMAT;
      e.offset = data_end + 4 * k;
      return e;
    }
    prev = r;
  }
  e.phase = REF_PHASE_ENTRIES;
  key->n = 0;
  uint64_t o = 0, k = 0;
  const uint8_t *limit = c + data_end;
  while (o < data_end) {
    uint32_t shared, non_shared, vlen;
    const uint8_t *p = c + o;
    int a = ref_get_varint32(p, limit, &shared);
    int b = a ? ref_get_varint32(p + a, limit, &non_shared) : 0;
    int d = b ? ref_get_varint32(p + a + b, limit, &vlen) : 0;
    e.offset = o;
    if (!d) goto corrupt;
    p += a + b + d;
    if (shared > key->n) goto corrupt;
    if ((uint64_t)non_shared + vlen > (uint64_t)(limit - p)) goto corrupt;
    uint64_t end = (uint64_t)(p - c) + non_shared + vlen;
    if (k < nr && o == rd32(c + data_end + 4 * k)) {
      if (shared != 0) goto corrupt;
      k++;
    }
    if (k < nr && rd32(c + data_end + 4 * k) < end) goto corrupt;
    key->n = shared;
    buf_put(key, p, non_shared);
    if (key->oom) {
      e.status = REF_NOMEM;
      return e;
    }
    int rc = visit(ctx, key->p, key->n, p + non_shared, vlen);
    if (rc != REF_OK) {
      e.status = rc;
      return e;
    }
    o = end;
  }
  e.status = REF_OK;
  return e;
corrupt:
  e.status = REF_CORRUPT_FORMAT;
  return e;
}

/* Read the 5-byte trailer of the block at [off, off + size): the checksum
 * covers the contents and the type byte. */
static blk_err check_trailer(const uint8_t *sst, uint64_t off, uint64_t size, int allow_snappy) {
  blk_err e = {REF_OK, REF_PHASE_TRAILER, 0};
  const uint8_t *c = sst + off;
  uint32_t stored = ref_unmask_crc(rd32(c + size + 1));
  uint32_t actual = ref_crc32c(c, size + 1);
  if (stored != actual) {
    e.status = REF_CORRUPT_CHECKSUM;
    return e;
  }
  /* type 0: stored raw; type 1 (Snappy): data blocks only */
  if (c[size] > (allow_snappy ? 1 : 0)) e.status = REF_UNSUPPORTED;
  return e;
}

/* The raw contents of a data block whose trailer checked out: the stored
 * bytes themselves (type 0), or their decompression (type 1), kept in *keep
 * until the job ends (decoded values point into it).  A stream that cannot
 * be decoded is a trailer-phase error at the offending element's offset. */
static blk_err block_contents(const uint8_t *sst, uint64_t off, uint64_t size, const uint8_t **raw,
                              uint64_t *raw_size, vec_t *keep) {
  blk_err e = {REF_OK, REF_PHASE_TRAILER, 0};
  *raw = sst + off;
  *raw_size = size;
  if (sst[off + size] == 0) return e;
  uint8_t *z;
  uint64_t zn, at;
  e.status = ref_snappy_decompress(sst + off, size, &z, &zn, &at);
  if (e.status != REF_OK) {
    e.offset = at;
    return e;
  }
  vec_push(keep, (uint64_t)(uintptr_t)z);
  if (keep->oom) {
    free(z);
    e.status = REF_NOMEM;
    return e;
  }
  *raw = z;
  *raw_size = zn;
  return e;
}

typedef struct {
  uint64_t limit; /* blocks must end (with trailer) at or before this offset */
  vec_t off, size;
} index_ctx;

static int index_visit(void *vctx, const uint8_t *key, uint64_t klen, const uint8_t *val,
                       uint64_t vlen) {
  (void)key;
  (void)klen;
  index_ctx *x = (index_ctx *)vctx;
  uint64_t off, size;
  int a = ref_get_varint64(val, val + vlen, &off);
  int b = a ? ref_get_varint64(val + a, val + vlen, &size) : 0;
  if (!b || (uint64_t)(a + b) != vlen) return REF_CORRUPT_FORMAT;
  if (off > x->limit || size > x->limit - off || 5 > x->limit - off - size) return REF_CORRUPT_FORMAT;
  vec_push(&x->off, off);
  vec_push(&x->size, size);
  return (x->off.oom || x->size.oom) ? REF_NOMEM : REF_OK;
}

/* decoded entries of one job: keys are materialised, values stay in place */
typedef struct {
  buf_t keys;
  vec_t koff, tags, vptr, vlen, input_first;
  vec_t raw; /* decompressed data blocks (their values are pointed into) */
  int have_prev;
  uint64_t prev_koff, prev_klen, prev_tag;
} dec_t;

static int data_visit(void *vctx, const uint8_t *key, uint64_t klen, const uint8_t *val,
                      uint64_t vlen) {
  dec_t *d = (dec_t *)vctx;
  if (klen < 8) return REF_CORRUPT_FORMAT;
  uint64_t tag = rd64(key + klen - 8);
  if ((tag & 0xFF) > 1) return REF_CORRUPT_FORMAT; /* type is deletion (0) or value (1) */
  uint64_t ulen = klen - 8;
  if (d->have_prev &&
      cmp_internal(d->keys.p + d->prev_koff, d->prev_klen, d->prev_tag, key, ulen, tag) >= 0)
    return REF_UNSORTED_INPUT;
  d->prev_koff = d->keys.n;
  d->prev_klen = ulen;
  d->prev_tag = tag;
  d->have_prev = 1;
  vec_push(&d->koff, d->keys.n);
  buf_put(&d->keys, key, ulen);
  vec_push(&d->tags, tag);
  vec_push(&d->vptr, (uint64_t)(uintptr_t)val);
  vec_push(&d->vlen, vlen);
  if (d->keys.oom || d->koff.oom || d->tags.oom || d->vptr.oom || d->vlen.oom) return REF_NOMEM;
  return REF_OK;
}

static int decode_one(const uint8_t *sst, uint64_t size, uint32_t input, dec_t *d, ref_error *err) {
  err->status = REF_OK;
  err->input = input;
  err->where = REF_WHERE_FOOTER;
  err->phase = 0;
  err->block = 0;
  err->offset = 0;
  /* footer */
  if (size < 48) {
    err->status = REF_CORRUPT_FORMAT;
    return err->status;
  }
  const uint8_t *ft = sst + size - 48;
  if (rd64(ft + 40) != TABLE_MAGIC) {
    err->status = REF_CORRUPT_FORMAT;
    err->offset = size - 8;
    return err->status;
  }
  uint64_t moff, msize, ioff, isize;
  int a = ref_get_varint64(ft, ft + 40, &moff);
  int b = a ? ref_get_varint64(ft + a, ft + 40, &msize) : 0;
  if (!b) {
    err->status = REF_CORRUPT_FORMAT;
    err->offset = size - 48;
    return err->status;
  }
  int c = ref_get_varint64(ft + a + b, ft + 40, &ioff);
  int dd = c ? ref_get_varint64(ft + a + b + c, ft + 40, &isize) : 0;
  uint64_t limit = size - 48;
  if (!dd || ioff > limit || isize > limit - ioff || 5 > limit - ioff - isize) {
    err->status = REF_CORRUPT_FORMAT;
    err->offset = size - 48 + a + b;
    return err->status;
  }
  (void)moff;
  (void)msize;
  /* index block */
  err->where = REF_WHERE_INDEX;
  blk_err be = check_trailer(sst, ioff, isize, 0);
  index_ctx ix;
  memset(&ix, 0, sizeof ix);
  ix.limit = limit;
  buf_t key = {0};
  if (be.status == REF_OK) be = walk_block(sst + ioff, isize, index_visit, &ix, &key);
  if (be.status != REF_OK) {
    err->status = be.status;
    err->phase = be.phase;
    err->offset = be.offset;
    free(ix.off.p), free(ix.size.p), free(key.p);
    return err->status;
  }
  /* data blocks, in index order */
  err->where = REF_WHERE_DATA;
  d->have_prev = 0;
  for (uint64_t k = 0; k < ix.off.n; k++) {
    err->block = k;
    be = check_trailer(sst, ix.off.p[k], ix.size.p[k], 1);
    const uint8_t *raw = NULL;
    uint64_t raw_size = 0;
    if (be.status == REF_OK) be = block_contents(sst, ix.off.p[k], ix.size.p[k], &raw, &raw_size, &d->raw);
    if (be.status == REF_OK) be = walk_block(raw, raw_size, data_visit, d, &key);
    if (be.status != REF_OK) {
      err->status = be.status;
      err->phase = be.phase;
      err->offset = be.offset;
      break;
    }
  }
  free(ix.off.p), free(ix.size.p), free(key.p);
  if (err->where == REF_WHERE_DATA && err->status != REF_OK) return err->status;
  err->status = REF_OK;
  err->where = 0;
  err->block = 0;
  err->phase = 0;
  err->offset = 0;
  return REF_OK;
}

static void dec_free(dec_t *d) {
  for (uint64_t i = 0; i < d->raw.n; i++) free((void *)(uintptr_t)d->raw.p[i]);
  free(d->raw.p);
  free(d->keys.p);
  free(d->koff.p);
  free(d->tags.p);
  free(d->vptr.p);
  free(d->vlen.p);
  free(d->input_first.p);
}

int ref_decode_table(const uint8_t *sst, uint64_t size, uint32_t input_index, ref_decoded **out,
                     ref_error *err) {
  ref_error e0;
  if (!err) err = &e0;
  memset(err, 0, sizeof *err);
  if (!out || (!sst && size)) return REF_INVALID_ARG;
  *out = NULL;
  dec_t d;
  memset(&d, 0, sizeof d);
  err->status = REF_OK;
  int rc = decode_one(sst, size, input_index, &d, err);
  if (rc != REF_OK) {
    dec_free(&d);
    return rc;
  }
  uint64_t n = d.tags.n;
  ref_decoded *r = (ref_decoded *)calloc(1, sizeof *r);
  uint64_t vtot = 0;
  for (uint64_t i = 0; i < n; i++) vtot += d.vlen.p[i];
  if (r) {
    r->n = n;
    r->keys = d.keys.p;
    d.keys.p = NULL;
    r->koff = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
    r->tags = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
    r->vals = (uint8_t *)malloc(vtot + 1);
    r->voff = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
  }
  if (!r || !r->koff || !r->tags || !r->vals || !r->voff) {
    ref_free_decoded(r);
    dec_free(&d);
    return REF_NOMEM;
  }
  uint64_t vo = 0;
  for (uint64_t i = 0; i < n; i++) {
    r->koff[i] = d.koff.p[i];
    r->tags[i] = d.tags.p[i];
    r->voff[i] = vo;
    memcpy(r->vals + vo, (const uint8_t *)(uintptr_t)d.vptr.p[i], d.vlen.p[i]);
    vo += d.vlen.p[i];
  }
  r->koff[n] = d.keys.n;
  r->voff[n] = vo;
  dec_free(&d);
  *out = r;
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Phase 2 "(Delete and) Sort" (Sec. II-A): merge and sort all restored
 * entries in key order and drop stale ones.  Order: user key ascending, tag
 * descending, then (input index, position) ascending, which is the decoded
 * index since inputs are decoded in order.
 *
 * Which versions are stale (the paper names the rule, Sec. II-A, without
 * snapshots; live snapshots are the reading written out here).  A reader at
 * snapshot s sees, for each user key, its newest version with sequence <= s;
 * a reader of the current state sees the newest version.  A version is kept
 * iff some such reader sees it: the newest version of its key, and every
 * version v for which a snapshot s lies in [seq(v), seq(newer)), newer being
 * the next newer version of the key.  Every other version is shadowed.  At
 * the bottom level a kept deletion is dropped too when no kept value of its
 * key is older than it (no reader can then tell it from absence).  With no
 * snapshots this is: the newest version survives, and a surviving deletion
 * is dropped at the bottom level. */

/* snapshots below sequence q: two versions are seen by the same readers iff
 * this count is equal for both */
static uint32_t stripe_of(const ref_options *opt, uint64_t q) {
  uint32_t k = 0;
  while (k < opt->n_snapshots && opt->snapshots[k] < q) k++;
  return k;
}

typedef struct {
  const dec_t *d;
} sort_ctx;

static int cmp_decoded(const void *pa, const void *pb, void *vctx) {
  const dec_t *d = ((const sort_ctx *)vctx)->d;
  uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
  uint64_t ka = d->koff.p[a], kb = d->koff.p[b];
  uint64_t la = d->koff.p[a + 1] - ka, lb = d->koff.p[b + 1] - kb;
  int c = cmp_internal(d->keys.p + ka, la, d->tags.p[a], d->keys.p + kb, lb, d->tags.p[b]);
  if (c) return c;
  return a < b ? -1 : (a > b ? 1 : 0);
}

int ref_compact(const uint8_t *const *inputs, const uint64_t *sizes, uint32_t n_inputs,
                const ref_options *opt, ref_result **out, ref_error *err) {
  ref_error e0;
  if (!err) err = &e0;
  memset(err, 0, sizeof *err);
  if (!out || check_options(opt) != REF_OK || (n_inputs && (!inputs || !sizes))) {
    err->status = REF_INVALID_ARG;
    return REF_INVALID_ARG;
  }
  *out = NULL;
  dec_t d;
  memset(&d, 0, sizeof d);
  uint64_t bytes_in = 0;
  for (uint32_t i = 0; i < n_inputs; i++) {
    vec_push(&d.input_first, d.tags.n);
    bytes_in += sizes[i];
    if (!inputs[i] && sizes[i]) {
      err->status = REF_INVALID_ARG;
      dec_free(&d);
      return REF_INVALID_ARG;
    }
    int rc = decode_one(inputs[i], sizes[i], i, &d, err);
    if (rc != REF_OK) {
      dec_free(&d);
      return rc;
    }
  }
  vec_push(&d.input_first, d.tags.n);
  vec_push(&d.koff, d.keys.n); /* end sentinel for key lengths */
  const uint64_t n = d.tags.n;
  uint64_t *order = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
  uint64_t *surv = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
  ref_result *r = (ref_result *)calloc(1, sizeof *r);
  if (!order || !surv || !r || d.input_first.oom || d.koff.oom) {
    free(order), free(surv), free(r);
    dec_free(&d);
    err->status = REF_NOMEM;
    return REF_NOMEM;
  }
  for (uint64_t i = 0; i < n; i++) order[i] = i;
  sort_ctx sc = {&d};
  qsort_r(order, n, sizeof(uint64_t), cmp_decoded, &sc);

  /* one user key at a time: versions [g0, g1) of order, newest first */
  uint64_t m = 0, shadowed = 0, tomb = 0;
  uint8_t *keep = (uint8_t *)malloc(n + 1);
  if (!keep) {
    free(order), free(surv), free(r);
    dec_free(&d);
    err->status = REF_NOMEM;
    return REF_NOMEM;
  }
  for (uint64_t g0 = 0, g1; g0 < n; g0 = g1) {
    const uint64_t a0 = order[g0];
    for (g1 = g0 + 1; g1 < n; g1++) {
      const uint64_t b = order[g1];
      if (cmp_user(d.keys.p + d.koff.p[a0], d.koff.p[a0 + 1] - d.koff.p[a0], d.keys.p + d.koff.p[b],
                   d.koff.p[b + 1] - d.koff.p[b]) != 0)
        break;
    }
    for (uint64_t j = g0; j < g1; j++) {
      const uint64_t seq = d.tags.p[order[j]] >> 8;
      keep[j] = j == g0 || stripe_of(opt, seq) != stripe_of(opt, d.tags.p[order[j - 1]] >> 8);
      if (!keep[j]) shadowed++;
    }
    if (opt->bottommost) {
      int older_value = 0; /* a kept value older than the version at hand */
      for (uint64_t j = g1; j-- > g0;) {
        if (!keep[j]) continue;
        if ((d.tags.p[order[j]] & 0xFF) == 0) {
          if (!older_value) {
            keep[j] = 0;
            tomb++;
          }
        } else {
          older_value = 1;
        }
      }
    }
    for (uint64_t j = g0; j < g1; j++)
      if (keep[j]) surv[m++] = order[j];
  }
  free(keep);

  view_t v;
  v.n = m;
  v.kp = (const uint8_t **)malloc((m + 1) * sizeof(void *));
  v.vp = (const uint8_t **)malloc((m + 1) * sizeof(void *));
  uint64_t *kl = (uint64_t *)malloc((m + 1) * sizeof(uint64_t));
  uint64_t *vl = (uint64_t *)malloc((m + 1) * sizeof(uint64_t));
  uint64_t *tg = (uint64_t *)malloc((m + 1) * sizeof(uint64_t));
  int rc = REF_NOMEM;
  if (v.kp && v.vp && kl && vl && tg) {
    for (uint64_t j = 0; j < m; j++) {
      uint64_t a = surv[j];
      v.kp[j] = d.keys.p + d.koff.p[a];
      kl[j] = d.koff.p[a + 1] - d.koff.p[a];
      tg[j] = d.tags.p[a];
      v.vp[j] = (const uint8_t *)(uintptr_t)d.vptr.p[a];
      vl[j] = d.vlen.p[a];
    }
    v.kl = kl;
    v.vl = vl;
    v.tag = tg;
    rc = pack_view(&v, opt, r);
  }
  free(v.kp), free(v.vp), free(kl), free(vl), free(tg), free(order);
  r->entries_in = n;
  r->entries_out = m;
  r->dropped_shadowed = shadowed;
  r->dropped_tombstones = tomb;
  r->bytes_in = bytes_in;
  r->n_inputs = n_inputs;
  r->input_first = d.input_first.p;
  d.input_first.p = NULL;
  r->surv = surv;
  dec_free(&d);
  if (rc != REF_OK) {
    ref_free_result(r);
    err->status = rc;
    return rc;
  }
  *out = r;
  return REF_OK;
}

void ref_free_result(ref_result *r) {
  if (!r) return;
  free(r->file_off);
  free(r->data);
  free(r->input_first);
  free(r->surv);
  free(r->block_first);
  free(r->file_first_block);
  free(r);
}

void ref_free_decoded(ref_decoded *d) {
  if (!d) return;
  free(d->keys);
  free(d->koff);
  free(d->tags);
  free(d->vals);
  free(d->voff);
  free(d);
}
