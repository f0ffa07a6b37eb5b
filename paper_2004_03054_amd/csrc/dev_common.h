// Device-side building blocks shared by the compaction kernels (gfx950).
//
// Table format facts used throughout (LevelDB table layout, which the paper's
// prototype builds on, Sec. IV-A; block = shared keys + values + checksum,
// Sec. II-A):
//   internal key = user key || fixed64 LE tag, tag = (sequence << 8) | type,
//   type 1 = value, 0 = deletion; order: user key ascending, tag descending.
//   entry = varint32 shared | varint32 non_shared | varint32 value_len |
//           key delta | value;  block = entries | fixed32 restarts[] | fixed32 n
//   block trailer = type byte (0) | fixed32 masked CRC32C(contents || type).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "luda_internal.h"

namespace luda {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// error keys: a 64-bit key whose numeric order is the reading order
// (input, structure, block, phase, offset, status), so an atomicMin over all
// detected errors of a job yields the first one.
//   input 12 | where 2 | block 22 | phase 2 | offset 23 | status 3

__host__ __device__ inline uint64_t err_key(uint32_t input, uint32_t where, uint64_t block,
                                            uint32_t phase, uint64_t offset, uint32_t code) {
  if (input > 4095) input = 4095;
  if (block > 0x3FFFFF) block = 0x3FFFFF;
  if (offset > 0x7FFFFF) offset = 0x7FFFFF;
  return ((uint64_t)input << 52) | ((uint64_t)where << 50) | (block << 28) |
         ((uint64_t)phase << 26) | (offset << 3) | (uint64_t)code;
}

__device__ inline void report_err(unsigned long long* slot, uint64_t key) {
  atomicMin(slot, (unsigned long long)key);
}

// ---------------------------------------------------------------------------
// small helpers

__device__ inline uint32_t lane_id() { return __lane_id(); }

// orders the LDS accesses of one wave's lanes (a wave's LDS operations are
// performed in issue order, so only the compiler must not move them across)
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint32_t rd_u32_bytes(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

__device__ inline uint32_t ldg_u32_unaligned(const uint8_t* p) {
  uint32_t v;
  __builtin_memcpy(&v, p, 4);
  return v;
}

__device__ inline uint64_t ldg_u64_unaligned(const uint8_t* p) {
  uint64_t v;
  __builtin_memcpy(&v, p, 8);
  return v;
}

__device__ inline uint64_t bswap64(uint64_t x) { return __builtin_bswap64(x); }

// i mod R and i / R for a restart interval R >= 1 (a power of two, the
// usual case, takes a mask or a shift instead of a division)
__device__ __forceinline__ uint32_t mod_r(uint32_t i, uint32_t R) { return (R & (R - 1)) == 0 ? i & (R - 1) : i % R; }
__device__ __forceinline__ uint32_t div_r(uint32_t i, uint32_t R) {
  return (R & (R - 1)) == 0 ? i >> __builtin_ctz(R) : i / R;
}
// 16 bytes at a global address of any alignment (one global_load_dwordx4)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // buffer load/store operand
typedef uint4 __attribute__((aligned(1))) uint4_u1;
typedef const __attribute__((address_space(1))) uint4_u1 g_uint4_u1;
typedef const __attribute__((address_space(1))) uint4 g_uint4;
__device__ inline uint4 ldg16(uint64_t addr) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(g_uint4_u1*)addr;
#else
  uint4 v;
  __builtin_memcpy(&v, (const void*)addr, 16);
  return v;
#endif
}
// one byte at a global address
__device__ inline uint32_t ldg_u8(uint64_t addr) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const __attribute__((address_space(1))) uint8_t*)addr;
#else
  return *(const uint8_t*)addr;
#endif
}
// 16 bytes at a 16-byte aligned global address
__device__ inline uint4 ldg16a(uint64_t addr) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(g_uint4*)addr;
#else
  return *(const uint4*)addr;
#endif
}


template <typename T>
__device__ inline T wave_shfl(T v, int src) {
  return __shfl(v, src, WAVE);
}

__device__ inline uint64_t wave_ballot(bool p) { return __ballot(p); }

// inclusive prefix sum over the wave (u32)
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    uint32_t t = __shfl_up(v, d, WAVE);
    if (l >= (uint32_t)d) v += t;
  }
  return v;
}

__device__ inline uint64_t wave_incl_scan64(uint64_t v) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    uint64_t t = __shfl_up(v, d, WAVE);
    if (l >= (uint32_t)d) v += t;
  }
  return v;
}

__device__ inline uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    uint32_t t = __shfl_xor(v, d, WAVE);
    v = v > t ? v : t;
  }
  return v;
}

__device__ inline uint64_t wave_min64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    uint64_t t = __shfl_xor(v, d, WAVE);
    v = v < t ? v : t;
  }
  return v;
}

__device__ inline uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, WAVE);
  return v;
}

// varint32 from a byte pointer, bounded by `limit`.  Returns bytes used or 0.
__device__ inline uint32_t get_varint32(const uint8_t* p, const uint8_t* limit, uint32_t* v) {
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < 5; i++) {
    if (p + i >= limit) return 0;
    uint32_t b = p[i];
    r |= (uint64_t)(b & 127u) << (7 * i);
    if (!(b & 128u)) {
      if (r > 0xFFFFFFFFull) return 0;
      *v = (uint32_t)r;
      return (uint32_t)i + 1;
    }
  }
  return 0;
}

__device__ inline uint32_t get_varint64(const uint8_t* p, const uint8_t* limit, uint64_t* v) {
  uint64_t r = 0;
  for (int i = 0; i < 10; i++) {
    if (p + i >= limit) return 0;
    uint32_t b = p[i];
    if (i == 9 && b > 1) return 0;
    r |= (uint64_t)(b & 127u) << (7 * i);
    if (!(b & 128u)) {
      *v = r;
      return (uint32_t)i + 1;
    }
  }
  return 0;
}

__host__ __device__ inline uint32_t varint_len(uint64_t v) {
  uint32_t n = 1;
  while (v >= 128) {
    v >>= 7;
    n++;
  }
  return n;
}

__device__ inline uint32_t put_varint(uint8_t* d, uint64_t v) {
  uint32_t n = 0;
  while (v >= 128) {
    d[n++] = (uint8_t)(v | 128);
    v >>= 7;
  }
  d[n++] = (uint8_t)v;
  return n;
}

// ---------------------------------------------------------------------------
// CRC32C.  Raw register arithmetic (state 0, no final xor) is linear in the
// message bytes, so
//   crc32c(M) = raw(M with its first 4 bytes complemented) ^ 0xFFFFFFFF
// (the all-ones initial value acts like complementing the first 32 message
// bits), raw(A || B) = shift(raw(A), |B|) ^ raw(B), and leading zero bytes
// leave raw() unchanged.
//
// A wave folds a message as 16-byte chunks aligned to the message end: chunk
// c (c = 0 is the last) covers bytes [n - 16(c+1), n - 16c).  Lane l owns the
// chunks c = 63 - l + 64 i, so one wave step reads 1 KiB contiguously and a
// block's chunks are spread over the lanes within one chunk.  A chunk is
// folded by slicing-by-4 (four independent lookups per 4 bytes); each lane
// keeps a Horner sum over its chunks (a shift by 1024 zero bytes between
// them) and the lanes are joined by a 6-level tree of shifts by 16 * 2^k
// bytes.  Shifts are four table lookups; long messages are split into
// segments joined by multiplication with x^(8 len) mod P computed in GF(2).

constexpr uint32_t CRC_POLY = 0x82F63B78u;  // CRC32C, reflected

// LDS image: slicing-by-4 tables and shifts by 16 * 2^k zero bytes, k = 0..6
struct CrcLds {
  uint32_t t4[4][256];
  uint32_t sh[7][4][256];
};
// The same with tables of 11-bit indices: the raw CRC of a 4-byte word x is
// linear in x, so it is the xor of the CRCs of its bit fields [0, 11),
// [11, 22) and [22, 32), three lookups per word instead of four.  The global
// table image has this layout; kernels that need only CrcLds copy its head.
struct CrcLds11 {
  CrcLds b;
  uint32_t u0[2048];
  uint32_t u1[2048];
  uint32_t u2[1024];
};

__device__ __forceinline__ uint32_t crc_dword(const uint32_t (*t4)[256], uint32_t c, uint32_t d) {
  const uint32_t x = c ^ d;
  return t4[3][x & 0xFF] ^ t4[2][(x >> 8) & 0xFF] ^ t4[1][(x >> 16) & 0xFF] ^ t4[0][x >> 24];
}

__device__ __forceinline__ uint32_t crc_shift(const uint32_t (*sh)[256], uint32_t c) {
  return sh[0][c & 0xFF] ^ sh[1][(c >> 8) & 0xFF] ^ sh[2][(c >> 16) & 0xFF] ^ sh[3][c >> 24];
}

// mask bytes at message positions < 0 and complement positions 0..3
__device__ __forceinline__ uint32_t crc_edge(uint32_t d, int64_t p) {
  if (p >= 4) return d;
  uint32_t keep = 0, flip = 0;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    int64_t q = p + j;
    if (q >= 0) keep |= 0xFFu << (8 * j);
    if (q >= 0 && q < 4) flip |= 0xFFu << (8 * j);
  }
  return (d & keep) ^ flip;
}

// raw CRC, from register state r, of one 16-byte chunk held in registers
// that starts at message position p (bytes before position 0 are ignored)
__device__ __forceinline__ uint32_t crc_chunk_from(const CrcLds* T, uint32_t r, uint4 v, int64_t p) {
  if (p < 4) {
    v.x = crc_edge(v.x, p);
    v.y = crc_edge(v.y, p + 4);
    v.z = crc_edge(v.z, p + 8);
    v.w = crc_edge(v.w, p + 12);
  }
  r = crc_dword(T->t4, r, v.x);
  r = crc_dword(T->t4, r, v.y);
  r = crc_dword(T->t4, r, v.z);
  r = crc_dword(T->t4, r, v.w);
  return r;
}

__device__ __forceinline__ uint32_t crc_chunk(const CrcLds* T, uint4 v, int64_t p) {
  return crc_chunk_from(T, 0u, v, p);
}

// join the per-lane Horner sums: lane l's last chunk is followed by 63 - l
// chunks.  Returns the raw CRC to every lane.
__device__ __forceinline__ uint32_t crc_wave_join(const CrcLds* T, uint32_t acc) {
#pragma unroll
  for (int k = 0; k < 6; k++) {
    uint32_t other = __shfl_down(acc, 1u << k, WAVE);
    if (lane_id() + (1u << k) >= WAVE) other = 0;
    acc = crc_shift(T->sh[k], acc) ^ other;
  }
  return __shfl(acc, 0, WAVE);
}

__device__ __forceinline__ uint32_t ld_dword_from(const uint8_t* msg, int64_t p) {
  if (p >= 0) return ldg_u32_unaligned(msg + p);
  uint32_t v = 0;
#pragma unroll
  for (int k = 0; k < 4; k++)
    if (p + k >= 0) v |= (uint32_t)msg[p + k] << (8 * k);
  return v;
}

// load the 16 message bytes at positions [p, p + 16) of msg (p + 16 > 0);
// bytes before position 0 are not read
__device__ __forceinline__ uint4 ld_chunk(const uint8_t* msg, int64_t p) {
  if (p >= 0) return ldg16((uint64_t)(uintptr_t)(msg + p));
  if (p + 16 <= 0) return make_uint4(0, 0, 0, 0);
  return make_uint4(ld_dword_from(msg, p), ld_dword_from(msg, p + 4), ld_dword_from(msg, p + 8),
                    ld_dword_from(msg, p + 12));
}

__device__ __forceinline__ uint32_t crc_dword11(const CrcLds11* T, uint32_t c, uint32_t d) {
  const uint32_t x = c ^ d;
  return T->u0[x & 0x7FF] ^ T->u1[(x >> 11) & 0x7FF] ^ T->u2[x >> 22];
}

__device__ __forceinline__ uint32_t crc_chunk11(const CrcLds11* T, uint4 v) {
  uint32_t r = crc_dword11(T, 0u, v.x);
  r = crc_dword11(T, r, v.y);
  r = crc_dword11(T, r, v.z);
  return crc_dword11(T, r, v.w);
}

// raw CRC of one 16-byte chunk with no message position below 4 in it
__device__ __forceinline__ uint32_t crc_chunk_plain(const CrcLds* T, uint4 v) {
  uint32_t r = crc_dword(T->t4, 0u, v.x);
  r = crc_dword(T->t4, r, v.y);
  r = crc_dword(T->t4, r, v.z);
  return crc_dword(T->t4, r, v.w);
}

// Raw CRC (first 4 message bytes complemented) of message bytes
// [s0, s0 + len) of a message that starts at msg; len is a multiple of 16 or
// s0 <= 0 (a segment starting before the message counts only its bytes
// inside it).  Chunks are aligned to the segment end; those wholly before
// the message are leading zeros, which leave the raw CRC unchanged, and are
// skipped.  A lane takes its chunks first to last; the ones that reach below
// message position 4 come first and are folded by the edge rules, the rest
// plainly, CRC_Q chunks at a time with all their loads issued before the
// first fold.  Every lane must call.
constexpr int CRC_Q = 5;
__device__ __forceinline__ uint32_t wave_raw_crc(const CrcLds* T, const uint8_t* msg, int64_t s0, uint64_t len) {
  const uint32_t l = lane_id();
  const int64_t send = s0 + (int64_t)len;
  const int64_t J = min((int64_t)((len + 15) / 16), (send + 15) / 16);
  uint32_t acc = 0;
  const int64_t c_first = 63 - (int64_t)l;
  int64_t c = c_first < J ? c_first + 64 * ((J - 1 - c_first) / 64) : -1;
  for (; c >= 0 && send - 16 * (c + 1) < 4; c -= 64) {
    const int64_t p0 = send - 16 * (c + 1);
    acc = crc_shift(T->sh[6], acc) ^ crc_chunk(T, ld_chunk(msg, p0), p0);
  }
  const uint8_t* e = msg + send;  // chunk c is [e - 16 (c + 1), e - 16 c)
  for (; c >= 0; c -= 64 * CRC_Q) {
    uint4 v[CRC_Q];
#pragma unroll
    for (int q = 0; q < CRC_Q; q++)
      if (c - 64 * q >= 0) v[q] = ldg16((uint64_t)(uintptr_t)(e - 16 * (c - 64 * q + 1)));
#pragma unroll
    for (int q = 0; q < CRC_Q; q++)
      if (c - 64 * q >= 0) acc = crc_shift(T->sh[6], acc) ^ crc_chunk_plain(T, v[q]);
  }
  return crc_wave_join(T, acc);
}

// GF(2) arithmetic mod P in the reflected representation (bit 31 is x^0):
// the product of a and b reduced mod P.
__device__ __host__ inline uint32_t gf2_mulmod(uint32_t a, uint32_t b) {
  uint32_t p = 0;
  for (int i = 0; i < 32; i++) {
    if (a & (0x80000000u >> i)) p ^= b;
    b = (b & 1u) ? (b >> 1) ^ CRC_POLY : (b >> 1);
  }
  return p;
}

// x^(8 n) mod P: the multiplier that shifts a raw CRC over n zero bytes
__device__ __host__ inline uint32_t gf2_xpow8n(uint64_t n) {
  uint32_t result = 0x80000000u;  // x^0
  uint32_t sq = 0x00800000u;      // x^8
  while (n) {
    if (n & 1) result = gf2_mulmod(result, sq);
    sq = gf2_mulmod(sq, sq);
    n >>= 1;
  }
  return result;
}

// cooperative load of the global CRC tables (the head of the image) into LDS
template <typename L = CrcLds>
__device__ __forceinline__ void load_crc_tables(L* dst, const uint32_t* src, int tid, int nthreads) {
  uint4* d = (uint4*)dst;
  const uint4* s4 = (const uint4*)src;
  const int n = (int)(sizeof(L) / 16);
  for (int i = tid; i < n; i += nthreads) d[i] = s4[i];
}

__host__ __device__ inline uint32_t crc_mask(uint32_t c) {
  return ((c >> 15) | (c << 17)) + 0xa282ead8u;
}
__host__ __device__ inline uint32_t crc_unmask(uint32_t m) {
  uint32_t r = m - 0xa282ead8u;
  return (r >> 17) | (r << 15);
}


// ---------------------------------------------------------------------------
// XXH64 (published xxHash XXH64 algorithm), over a zero-padded 8-byte-aligned
// key slot.

constexpr uint64_t XP1 = 0x9E3779B185EBCA87ull;
constexpr uint64_t XP2 = 0xC2B2AE3D27D4EB4Full;
constexpr uint64_t XP3 = 0x165667B19E3779F9ull;
constexpr uint64_t XP4 = 0x85EBCA77C2B2AE63ull;
constexpr uint64_t XP5 = 0x27D4EB2F165667C5ull;

__device__ inline uint64_t rotl64(uint64_t x, int r) { return (x << r) | (x >> (64 - r)); }
__device__ inline uint64_t xxr(uint64_t acc, uint64_t lane) {
  acc += lane * XP2;
  acc = rotl64(acc, 31);
  return acc * XP1;
}
__device__ inline uint64_t xxm(uint64_t acc, uint64_t v) {
  acc ^= xxr(0, v);
  return acc * XP1 + XP4;
}

// key: 8-byte aligned words holding n bytes (little endian), zero padded
__device__ inline uint64_t xxh64_words(const uint64_t* w, uint32_t n) {
  uint64_t acc;
  uint32_t i = 0;  // word index
  if (n >= 32) {
    uint64_t v1 = XP1 + XP2, v2 = XP2, v3 = 0, v4 = 0 - XP1;
    uint32_t stripes = n / 32;
    for (uint32_t s = 0; s < stripes; s++) {
      v1 = xxr(v1, w[i]);
      v2 = xxr(v2, w[i + 1]);
      v3 = xxr(v3, w[i + 2]);
      v4 = xxr(v4, w[i + 3]);
      i += 4;
    }
    acc = rotl64(v1, 1) + rotl64(v2, 7) + rotl64(v3, 12) + rotl64(v4, 18);
    acc = xxm(acc, v1);
    acc = xxm(acc, v2);
    acc = xxm(acc, v3);
    acc = xxm(acc, v4);
  } else {
    acc = XP5;
  }
  acc += n;
  uint32_t rem = n - i * 8;
  while (rem >= 8) {
    acc ^= xxr(0, w[i]);
    acc = rotl64(acc, 27) * XP1 + XP4;
    i++;
    rem -= 8;
  }
  uint64_t last = rem ? w[i] : 0;
  uint32_t sh = 0;
  if (rem >= 4) {
    acc ^= (uint64_t)(uint32_t)last * XP1;
    acc = rotl64(acc, 23) * XP2 + XP3;
    sh = 32;
    rem -= 4;
  }
  while (rem) {
    acc ^= ((last >> sh) & 0xFF) * XP5;
    acc = rotl64(acc, 11) * XP1;
    sh += 8;
    rem--;
  }
  acc ^= acc >> 33;
  acc *= XP2;
  acc ^= acc >> 29;
  acc *= XP3;
  acc ^= acc >> 32;
  return acc;
}

// ---------------------------------------------------------------------------
// entry key access.  A decoded entry's user key lives in a zero-padded slot of
// KW bytes (KW a multiple of 8); kp0/kp1 hold its first 16 bytes big endian.

struct KeyRef {
  const uint64_t* heap;  // slot base (KW/8 words per entry)
  uint32_t kw8;          // words per slot
};

// byte i of the internal key (user key then 8 tag bytes, little endian)
__device__ inline uint32_t ikey_byte(const uint8_t* slot, uint32_t ulen, uint64_t tag, uint32_t i) {
  return i < ulen ? slot[i] : (uint32_t)((tag >> (8 * (i - ulen))) & 0xFF);
}

// internal key order of two entries: user key asc, then tag desc (-1, 0, 1)
__device__ inline int cmp_ikeys(const Tuples& t, uint32_t kw8, uint64_t a, uint64_t b) {
  uint64_t a0 = t.kp0[a], b0 = t.kp0[b];
  if (a0 != b0) return a0 < b0 ? -1 : 1;
  uint64_t a1 = t.kp1[a], b1 = t.kp1[b];
  if (a1 != b1) return a1 < b1 ? -1 : 1;
  uint32_t la = t.ulen[a], lb = t.ulen[b];
  uint32_t m = la < lb ? la : lb;
  if (m > 16) {
    const uint64_t* ha = t.heap + a * kw8;
    const uint64_t* hb = t.heap + b * kw8;
    for (uint32_t w = 2; w * 8 < m; w++) {
      uint64_t x = ha[w], y = hb[w];
      if (x != y) {
        // the first differing byte decides if it lies inside the common length
        uint64_t diff = x ^ y;
        uint32_t byte = (uint32_t)(__builtin_ctzll(diff) >> 3);
        if (w * 8 + byte < m) {
          uint32_t bx = (uint32_t)((x >> (8 * byte)) & 0xFF), by = (uint32_t)((y >> (8 * byte)) & 0xFF);
          return bx < by ? -1 : 1;
        }
        break;
      }
    }
  }
  if (la != lb) return la < lb ? -1 : 1;
  uint64_t ta = t.tag[a], tb = t.tag[b];
  if (ta != tb) return ta > tb ? -1 : 1;
  return 0;
}

// merge order: internal key order, then entry index (input, position) asc
__device__ inline int cmp_entries(const Tuples& t, uint32_t kw8, uint64_t a, uint64_t b) {
  int c = cmp_ikeys(t, kw8, a, b);
  if (c) return c;
  return a < b ? -1 : (a > b ? 1 : 0);
}

// same user key?
__device__ inline bool same_user_key(const Tuples& t, uint32_t kw8, uint64_t a, uint64_t b) {
  if (t.kp0[a] != t.kp0[b] || t.kp1[a] != t.kp1[b] || t.ulen[a] != t.ulen[b]) return false;
  uint32_t m = t.ulen[a];
  const uint64_t* ha = t.heap + a * kw8;
  const uint64_t* hb = t.heap + b * kw8;
  for (uint32_t w = 2; w * 8 < m; w++)
    if (ha[w] != hb[w]) return false;
  return true;
}

}  // namespace luda
