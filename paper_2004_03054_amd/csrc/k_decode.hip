// Phase 1 "Unpack" kernels (paper Sec. II-A Phase 1: recompute each data
// block's checksum, then restore the full keys from the shared-prefix
// encoding; Sec. III-C: data blocks of a table are processed in parallel).
// Each table is read footer -> index block -> data blocks.  The same block
// machinery serves index blocks (whose entries are data block handles) and
// data blocks (whose entries are key/value pairs):
//
//   k_footer     one thread per input: footer magic, index handle
//   k_blk_nr     one thread per block: restart count
//   k_crc_wave   16 lanes per block: masked CRC32C and block type
//   k_crc_multi  index blocks: one wave per 4 KiB segment; k_crc_join
//                joins the segments of each block
//   k_imap       one thread per restart interval: its block (binary search)
//   k_walk       one thread per restart interval: walks the interval's
//                entries (count pass, then emit pass after a prefix sum)
//   k_keys       one thread per entry: restores the internal key by tracing
//                each byte back through the shared-prefix chain
//   k_order      one thread per entry: internal keys strictly increase
//                inside a table; records how adjacent tables compare
#include "dev_common.h"
#include "kernels.h"
#include "crc_multi.h"

namespace luda {

__global__ void k_footer(Inputs in, WalkSet idx, unsigned long long* err) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= in.n) return;
  const uint8_t* p = (const uint8_t*)in.ptr[g];
  const uint64_t size = in.size[g];
  const uint32_t job = in.job[g], loc = in.local[g];
  idx.skip[g] = 1;
  idx.ptr[g] = (uint64_t)(uintptr_t)p;
  idx.size[g] = 0;
  idx.input[g] = g;
  idx.local[g] = 0;
  if (size < 48) {
    report_err(&err[job], err_key(loc, W_FOOTER, 0, FP_SHORT, 0, EC_FORMAT));
    return;
  }
  const uint8_t* ft = p + size - 48;
  if (ldg_u64_unaligned(ft + 40) != TABLE_MAGIC) {
    report_err(&err[job], err_key(loc, W_FOOTER, 0, FP_REL, 40, EC_FORMAT));
    return;
  }
  uint64_t moff, msize, ioff, isize;
  uint32_t a = get_varint64(ft, ft + 40, &moff);
  uint32_t b = a ? get_varint64(ft + a, ft + 40, &msize) : 0;
  if (!b) {
    report_err(&err[job], err_key(loc, W_FOOTER, 0, FP_REL, 0, EC_FORMAT));
    return;
  }
  uint32_t c = get_varint64(ft + a + b, ft + 40, &ioff);
  uint32_t d = c ? get_varint64(ft + a + b + c, ft + 40, &isize) : 0;
  const uint64_t limit = size - 48;
  if (!d || ioff > limit || isize > limit - ioff || 5 > limit - ioff - isize || isize > 0xFFFFFFF0ull) {
    report_err(&err[job], err_key(loc, W_FOOTER, 0, FP_REL, a + b, EC_FORMAT));
    return;
  }
  idx.ptr[g] = (uint64_t)(uintptr_t)(p + ioff);
  idx.size[g] = (uint32_t)isize;
  idx.skip[g] = 0;
}

__device__ inline void blk_err(const WalkSet& ws, const Inputs& in, uint32_t b, uint32_t phase, uint64_t off,
                               uint32_t code, unsigned long long* err) {
  const uint32_t g = ws.input[b];
  report_err(&err[in.job[g]], err_key(in.local[g], ws.where, ws.local[b], phase, off, code));
}

// restart count of every block (size >= 4, 1 <= n <= (size - 4) / 4).
// Data blocks, first pass (z.cap set): a block of type 1 (Snappy) gets no
// restart count yet; it is given staging room for its raw bytes instead (the
// declared length, but no more than 22x its stored bytes: an element of b
// bytes yields at most 64/3 b, so a longer declared length cannot be
// produced), counted in z.tot.  Second pass (z.only_z): the blocks that were
// decompressed, now pointing at their raw bytes.
__global__ void k_blk_nr(WalkSet ws, Inputs in, uint32_t* nr_out, unsigned long long* err, ZPass z) {
  const uint64_t nb = *ws.n_dev;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (uint64_t)gridDim.x * blockDim.x) {
    if (z.only_z && (!z.cap[b] || !z.ok[b])) {
      if (z.cap[b]) nr_out[b] = 0;
      continue;
    }
    uint32_t nr = 0;
    if (z.cap && !z.only_z) {
      uint64_t cap = 0;
      if (!ws.skip[b]) {
        const uint8_t* c = (const uint8_t*)ws.ptr[b];
        const uint32_t size = ws.size[b];
        if (c[size] == 1) {
          uint32_t len = 0;
          const uint64_t most = 22ull * size;
          const uint64_t raw = get_varint32(c, c + size, &len) ? (len < most ? len : most) : 0;
          cap = ((raw + 15) & ~15ull) + ZSTAGE_PAD;
          atomicAdd(&z.tot[0], 1ull);
          atomicAdd(&z.tot[1], (unsigned long long)cap);
        }
      }
      z.cap[b] = cap;
      if (cap) {
        nr_out[b] = 0;
        continue;
      }
    }
    if (!ws.skip[b]) {
      const uint8_t* c = (const uint8_t*)ws.ptr[b];
      const uint32_t size = ws.size[b];
      if (size < 4) {
        blk_err(ws, in, (uint32_t)b, P_RESTARTS, 0, EC_FORMAT, err);
      } else {
        const uint32_t v = ldg_u32_unaligned(c + size - 4);
        if (v == 0 || v > (size - 4) / 4) blk_err(ws, in, (uint32_t)b, P_RESTARTS, size - 4, EC_FORMAT, err);
        else nr = v;
      }
    }
    nr_out[b] = nr;
  }
}

// masked CRC32C of (contents || type byte) against the trailer, type 0
__device__ inline void finish_crc(const WalkSet& ws, const Inputs& in, uint32_t b, uint32_t raw, uint8_t* ok,
                                  unsigned long long* err) {
  const uint8_t* c = (const uint8_t*)ws.ptr[b];
  const uint32_t size = ws.size[b];
  const uint32_t crc = raw ^ 0xFFFFFFFFu;
  const uint32_t stored = crc_unmask(ldg_u32_unaligned(c + size + 1));
  uint8_t good = 1;
  if (crc != stored) {
    blk_err(ws, in, b, P_TRAILER, 0, EC_CHECKSUM, err);
    good = 0;
  } else if (c[size] != 0) {
    blk_err(ws, in, b, P_TRAILER, 0, EC_UNSUPPORTED, err);
    good = 0;
  }
  ok[b] = good;
}

// Data block checksums.  A block's message (contents and type byte) is cut
// into 16-byte chunks aligned to its end, and the chunks into rounds of
// CRC_GL * CRC_RUN chunks (512 B) counted from the end; the top round may
// reach before the message start.  A wave takes CRC_GPW blocks at a time,
// one group of CRC_GL lanes per block.  In each round lane j of a group
// takes CRC_RUN consecutive chunks (the lanes in address order) and runs the
// table CRC through them from state 0 with no shift in between; the lane
// adds that to its sum over the rounds by Horner's rule (one shift by a
// round per round), and the group joins its lanes' sums in log2(CRC_GL)
// steps, step l shifting by CRC_RUN * 2^l chunks.  Against one wave per
// block with one chunk per lane per step this halves the round shifts, joins
// in four steps instead of six, and leaves less of the top round idle on
// blocks of 4-5 KiB.  Leading zero bytes leave the raw CRC unchanged, so
// chunks wholly before the message are zeros and need no load.
struct CrcBlk {
  const uint8_t* p;
  uint64_t n;  // message bytes (contents + type byte); 0: none
  bool skip;
};

__device__ __forceinline__ CrcBlk crc_blk(const WalkSet& ws, uint64_t b, uint64_t nb) {
  const uint64_t bb = b < nb ? b : nb - 1;  // nb > 0
  CrcBlk r;
  r.skip = ws.skip[bb] != 0;
  r.p = (const uint8_t*)ws.ptr[bb];
  const uint32_t sz = ws.size[bb];
  r.n = (b < nb && !r.skip) ? (uint64_t)sz + 1 : 0;
  return r;
}

// masked CRC32C of (contents || type byte) against the trailer, type 0 or 1
// (called by one lane per block)
__device__ inline uint8_t check_crc(const WalkSet& ws, const Inputs& in, uint32_t b, uint32_t raw, uint32_t stored,
                                    uint32_t type, unsigned long long* err) {
  if ((raw ^ 0xFFFFFFFFu) != crc_unmask(stored)) {
    blk_err(ws, in, b, P_TRAILER, 0, EC_CHECKSUM, err);
    return 0;
  }
  if (type > 1) {  // 0: stored raw; 1: a Snappy stream, decompressed later
    blk_err(ws, in, b, P_TRAILER, 0, EC_UNSUPPORTED, err);
    return 0;
  }
  return 1;
}

constexpr uint32_t CRC_GL = 16;                     // lanes per block
constexpr uint32_t CRC_GPW = WAVE / CRC_GL;         // blocks per wave
constexpr uint32_t CRC_RUN = 2;                     // consecutive chunks per lane per round
constexpr uint32_t CRC_RB = CRC_GL * CRC_RUN * 16;  // bytes per round
constexpr uint32_t CRC_RQ = 2;                      // rounds whose loads are issued together
constexpr int CRC_SH_RUN = 1;                       // sh[k] shifts by 2^k chunks
constexpr int CRC_SH_ROUND = 5;
static_assert(CRC_RUN == (1u << CRC_SH_RUN) && CRC_GL * CRC_RUN == (1u << CRC_SH_ROUND), "shift tables");
static_assert(CRC_RQ >= 2, "the first load batch must hold both rounds that can reach below position 4");

__device__ __forceinline__ uint4 bytes_up(uint4 v, uint32_t s) {  // byte k <- byte k - s, zeros below s
  unsigned __int128 x = ((unsigned __int128)(((uint64_t)v.w << 32) | v.z) << 64) | (((uint64_t)v.y << 32) | v.x);
  x <<= 8 * s;
  return make_uint4((uint32_t)x, (uint32_t)(x >> 32), (uint32_t)(x >> 64), (uint32_t)(x >> 96));
}

// the chunk at message position p < 4 as the raw CRC sees it (bytes before
// the message zero, positions 0..3 complemented); it was loaded from
// position max(p, 0), or not at all when p <= -16
__device__ __forceinline__ uint4 crc_edge_chunk(uint4 v, int64_t p) {
  if (p <= -16) return make_uint4(0, 0, 0, 0);
  if (p < 0) v = bytes_up(v, (uint32_t)-p);
  v.x = crc_edge(v.x, p);
  v.y = crc_edge(v.y, p + 4);
  v.z = crc_edge(v.z, p + 8);
  v.w = crc_edge(v.w, p + 12);
  return v;
}

// loads of a lane's chunks in rounds i .. i + CRC_RQ - 1 (its run of round i
// starts at message position P0 + CRC_RB i); rounds past R and chunks wholly
// before the message read a fixed valid address instead.  EDGE: the rounds
// may reach below message position 4 (only the top two rounds can).
template <bool EDGE>
__device__ __forceinline__ void crc_loads(const CrcBlk& k, int64_t P0, uint32_t R, uint32_t i, uint64_t safe,
                                          uint4 (&v)[CRC_RQ][CRC_RUN]) {
#pragma unroll
  for (uint32_t q = 0; q < CRC_RQ; q++) {
    const int64_t pr = P0 + (int64_t)CRC_RB * (i + q);
#pragma unroll
    for (uint32_t s = 0; s < CRC_RUN; s++) {
      const int64_t p = pr + 16 * s;
      uint64_t a = (uint64_t)(uintptr_t)k.p + (uint64_t)(EDGE ? (p > 0 ? p : 0) : p);
      if (i + q >= R || (EDGE && p <= -16)) a = safe;
      v[q][s] = ldg16(a);
    }
  }
}

template <bool EDGE>
__device__ __forceinline__ void crc_rounds(const CrcLds11* T, int64_t P0, uint32_t R, uint32_t i,
                                           const uint4 (&v)[CRC_RQ][CRC_RUN], uint32_t& acc) {
#pragma unroll
  for (uint32_t q = 0; q < CRC_RQ; q++) {
    if (i + q < R) {
      const int64_t pr = P0 + (int64_t)CRC_RB * (i + q);
      uint32_t r = 0;
#pragma unroll
      for (uint32_t s = 0; s < CRC_RUN; s++) {
        uint4 x = v[q][s];
        if (EDGE && pr + 16 * (int64_t)s < 4) x = crc_edge_chunk(x, pr + 16 * (int64_t)s);
        r = crc_dword11(T, r, x.x);
        r = crc_dword11(T, r, x.y);
        r = crc_dword11(T, r, x.z);
        r = crc_dword11(T, r, x.w);
      }
      acc = (EDGE && q == 0) ? r : crc_shift(T->b.sh[CRC_SH_ROUND], acc) ^ r;
    }
  }
}

__global__ void __launch_bounds__(1024) k_crc_wave(WalkSet ws, Inputs in, const uint32_t* g_crc, uint8_t* ok,
                                                  unsigned long long* err, unsigned long long* bytes_total) {
  __shared__ CrcLds11 T;
  load_crc_tables(&T, g_crc, threadIdx.x, blockDim.x);
  __syncthreads();
  const uint64_t nb = *ws.n_dev;
  if (nb == 0) return;
  const uint32_t waves = blockDim.x / WAVE, wv = threadIdx.x / WAVE;
  const uint32_t j = lane_id() % CRC_GL, g = lane_id() / CRC_GL;
  const uint64_t stride = (uint64_t)gridDim.x * waves * CRC_GPW;
  const uint64_t safe = (uint64_t)(uintptr_t)g_crc;
  uint64_t bytes = 0;
  uint64_t b = ((uint64_t)blockIdx.x * waves + wv) * CRC_GPW + g;
  CrcBlk kn = crc_blk(ws, b, nb);
  for (; b - g < nb; b += stride) {
    const CrcBlk k = kn;
    kn = crc_blk(ws, b + stride, nb);
    const int64_t n = (int64_t)k.n;
    const uint32_t R = (uint32_t)((k.n + CRC_RB - 1) / CRC_RB);
    uint32_t Rw = R;  // the wave's most rounds
#pragma unroll
    for (uint32_t m = CRC_GL; m < WAVE; m <<= 1) Rw = max(Rw, (uint32_t)__shfl_xor((int)Rw, (int)m, WAVE));
    uint32_t type = 0, stored = 0;
    if (j == 0 && n) {  // type byte, then the stored CRC
      const uint64_t ta = (uint64_t)(uintptr_t)(k.p + n - 1);
      type = ldg_u8(ta);
      stored = ldg_u8(ta + 1) | (ldg_u8(ta + 2) << 8) | (ldg_u8(ta + 3) << 16) | (ldg_u8(ta + 4) << 24);
    }
    const int64_t P0 = n - (int64_t)CRC_RB * R + 16 * CRC_RUN * (int64_t)j;
    uint32_t acc = 0;
    uint4 v[CRC_RQ][CRC_RUN];
    if (Rw) {
      crc_loads<true>(k, P0, R, 0, safe, v);
      crc_rounds<true>(&T, P0, R, 0, v, acc);
    }
    for (uint32_t i = CRC_RQ; i < Rw; i += CRC_RQ) {
      crc_loads<false>(k, P0, R, i, safe, v);
      crc_rounds<false>(&T, P0, R, i, v, acc);
    }
#pragma unroll
    for (int l = 0; (1u << l) < CRC_GL; l++) {  // lane j + 2^l's sum follows lane j's by CRC_RUN 2^l chunks
      const uint32_t other = __shfl_down(acc, 1u << l, WAVE);
      acc = crc_shift(T.b.sh[CRC_SH_RUN + l], acc) ^ other;
    }
    if (j == 0 && b < nb) {
      uint8_t good = 0;
      if (!k.skip) {
        good = check_crc(ws, in, (uint32_t)b, acc, stored, type, err);
        bytes += k.n + 4;
      }
      ok[b] = good;
    }
  }
  if (j == 0 && bytes) atomicAdd(bytes_total, (unsigned long long)bytes);
}

// index blocks of the inputs, checked against their trailers
struct IndexMsgs {
  WalkSet ws;
  Inputs in;
  uint8_t* ok;
  unsigned long long* err;
  __device__ uint32_t count() const { return (uint32_t)*ws.n_dev; }
  __device__ void span(uint32_t m, const uint8_t** p, uint64_t* n) const {
    *p = (const uint8_t*)ws.ptr[m];
    *n = ws.skip[m] ? 0 : (uint64_t)ws.size[m] + 1;
  }
  __device__ void finish(uint32_t m, uint32_t raw) const { finish_crc(ws, in, m, raw, ok, err); }
  __device__ void empty(uint32_t m) const { ok[m] = 0; }
};

void launch_crc_index(WalkSet ws, Inputs in, const uint32_t* g_crc, uint8_t* ok, unsigned long long* err,
                      uint64_t cap, uint32_t* part, uint64_t* mseg, uint32_t grid, hipStream_t st) {
  launch_crc_msgs(IndexMsgs{ws, in, ok, err}, cap, g_crc, part, mseg, grid, st);
}

// interval -> block map: the block of interval i is the last b with
// ibase[b] <= i (blocks without intervals share their successor's base)
__global__ void k_imap(WalkSet ws, const uint64_t* ibase, const uint64_t* ni_dev, uint32_t* iblk) {
  const uint64_t nb = *ws.n_dev, ni = *ni_dev;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ni; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t lo = 0, hi = nb;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (ibase[mid] <= i) lo = mid;
      else hi = mid;
    }
    iblk[i] = (uint32_t)lo;
  }
}

// ---------------------------------------------------------------------------
// Interval walk.  Checks, in order, per entry (all CORRUPT_FORMAT at the
// entry offset): three varint32 headers inside the entry area, shared <=
// previous key length, key delta and value inside the area, shared == 0 for
// the interval's first entry (a restart point), the entry does not cross the
// next restart point; data blocks also need an internal key of >= 8 bytes;
// index entries need a block handle inside the table.  Before the walk the
// interval's own restart offset is checked (first 0, increasing, inside the
// entry area: RESTARTS phase).  KIND 0 = index block, 1 = data block;
// MODE 0 = count and check, 1 = emit.

// The data emit pass stages the entry records of a wave's 64 intervals in
// LDS (their outputs are one contiguous range) and stores them with
// contiguous, whole-line writes; a lane walking its interval would otherwise
// write each record field to 64 scattered places per instruction.  Records
// past EMIT_CAP in the range are stored directly.
constexpr uint32_t EMIT_CAP = 512;
constexpr uint32_t EMIT_WAVES = 4;  // waves per workgroup (the launch bound)

template <uint32_t CAP>
struct EmitStage {
  uint64_t kd[CAP], sn[CAP], vp[CAP];
  uint32_t vlen[CAP], blk[CAP], eoff[CAP];
};

template <int KIND, int MODE>
__global__ void __launch_bounds__(256) k_walk(WalkArgs A) {
  constexpr bool STAGED = KIND == 1 && MODE == 1;
  __shared__ EmitStage<STAGED ? EMIT_CAP : 1> stage_all[STAGED ? EMIT_WAVES : 1];
  EmitStage<STAGED ? EMIT_CAP : 1>& S = stage_all[STAGED ? threadIdx.x / WAVE : 0];
  const uint64_t ni = *A.ni_dev;
  uint32_t maxk_all = 0;  // longest key this thread saw (count pass over data blocks)
  const uint64_t lane0 = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(uint32_t)(WAVE - 1));
  // the loop runs the same number of times in every lane of a wave
  for (uint64_t i0 = lane0; i0 < ni; i0 += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = i0 + lane_id();
    uint64_t wbase = 0, wn = 0;  // this wave's output range (staged emit)
    if constexpr (STAGED) {
      wbase = A.ient[i0];
      wn = A.ient[min(i0 + WAVE, ni)] - wbase;
    }
    const uint32_t b = i < ni ? A.iblk[i] : 0u;
    const uint32_t k = i < ni ? (uint32_t)(i - A.ibase[b]) : 0u;
    uint32_t cnt = 0, maxk = 0;
    if (i < ni && A.ok[b]) {
      const uint8_t* c = (const uint8_t*)A.ws.ptr[b];
      const uint32_t size = A.ws.size[b];
      const uint32_t nr = A.nr[b];
      const uint64_t data_end = size - 4 - 4ull * nr;
      const uint32_t r = ldg_u32_unaligned(c + data_end + 4ull * k);
      const uint32_t pr = k ? ldg_u32_unaligned(c + data_end + 4ull * (k - 1)) : 0;
      if ((k == 0 ? r != 0 : r <= pr) || r >= data_end) {
        if (MODE == 0) blk_err(A.ws, A.in, b, P_RESTARTS, data_end + 4ull * k, EC_FORMAT, A.err);
      } else {
        uint64_t end = (k + 1 < nr) ? ldg_u32_unaligned(c + data_end + 4ull * (k + 1)) : data_end;
        if (end > data_end) end = data_end;
        uint64_t o = r, prev_len = 0;
        bool first = true;
        uint64_t out = (MODE == 1) ? A.ient[i] : 0;
        const uint32_t g = A.ws.input[b];
        const uint64_t limit = (KIND == 0) ? A.in.size[g] - 48 : 0;
        while (o < end) {
          // three varint32 headers from one 16-byte load (inside the table)
          uint8_t h[16];
          {
            const uint4 v = ldg16((uint64_t)(uintptr_t)(c + o));
            __builtin_memcpy(h, &v, 16);
          }
          const uint64_t avail = data_end - o;
          uint32_t f[3] = {0, 0, 0};
          uint32_t pos = 0;
          bool okh = true;
          for (int q = 0; q < 3 && okh; q++) {
            uint64_t vv = 0;
            bool done = false;
            for (int t = 0; t < 5; t++) {
              if (pos >= avail || pos >= 16) {
                okh = false;
                break;
              }
              const uint32_t byte = h[pos++];
              vv |= (uint64_t)(byte & 127u) << (7 * t);
              if (!(byte & 128u)) {
                done = true;
                break;
              }
            }
            if (!done || vv > 0xFFFFFFFFull) okh = false;
            f[q] = (uint32_t)vv;
          }
          bool bad = !okh;
          const uint32_t shared = f[0], ns = f[1], vlen = f[2];
          const uint64_t hdr = pos;
          if (!bad && !first && shared > prev_len) bad = true;
          if (!bad && (uint64_t)ns + vlen > data_end - (o + hdr)) bad = true;
          if (!bad && first && shared != 0) bad = true;
          const uint64_t e = o + hdr + (uint64_t)ns + vlen;
          if (!bad && e > end) bad = true;
          const uint64_t klen = (uint64_t)shared + ns;
          if (!bad && KIND == 1 && klen < 8) bad = true;
          if (!bad && KIND == 0) {
            // index entry value: the data block handle
            const uint8_t* v = c + o + hdr + ns;
            uint64_t boff, bsz;
            uint32_t x = get_varint64(v, v + vlen, &boff);
            uint32_t y = x ? get_varint64(v + x, v + vlen, &bsz) : 0;
            if (!y || x + y != vlen || boff > limit || bsz > limit - boff || 5 > limit - boff - bsz ||
                bsz > 0xFFFFFFF0ull) {
              bad = true;
            } else if (MODE == 1) {
              A.out_blk.ptr[out] = A.in.ptr[g] + boff;
              A.out_blk.size[out] = (uint32_t)bsz;
              A.out_blk.input[out] = g;
              A.out_blk.local[out] = (uint32_t)(out - A.in_blk0[g]);
              A.out_blk.skip[out] = 0;
            }
          }
          if (bad) {
            if (MODE == 0) blk_err(A.ws, A.in, b, P_ENTRIES, o, EC_FORMAT, A.err);
            break;
          }
          if constexpr (STAGED) {
            const uint64_t gaddr = (uint64_t)(uintptr_t)c;
            const uint64_t rel = out - wbase;
            if (rel < EMIT_CAP) {
              S.kd[rel] = gaddr + o + hdr;
              S.sn[rel] = (uint64_t)shared | ((uint64_t)ns << 32);
              S.vp[rel] = gaddr + o + hdr + ns;
              S.vlen[rel] = vlen;
              S.blk[rel] = b;
              S.eoff[rel] = (uint32_t)o;
            } else {
              A.tu.kd[out] = gaddr + o + hdr;
              A.tu.sn[out] = (uint64_t)shared | ((uint64_t)ns << 32);
              A.tu.vp[out] = gaddr + o + hdr + ns;
              A.tu.vlen[out] = vlen;
              A.tu.blk[out] = b;
              A.tu.eoff[out] = (uint32_t)o;
            }
          }
          out++;
          cnt++;
          if (klen > maxk) maxk = (uint32_t)(klen > 0xFFFFFFFFull ? 0xFFFFFFFFu : klen);
          prev_len = klen;
          first = false;
          o = e;
        }
      }
    }
    if (MODE == 0 && i < ni) A.icnt[i] = cnt;
    maxk_all = max(maxk_all, maxk);
    if constexpr (STAGED) {
      // every walk emits exactly the records its count pass counted (the same
      // checks stop both), so the staged part of the range is complete
      wave_sync();
      const uint32_t m = (uint32_t)min(wn, (uint64_t)EMIT_CAP);
      for (uint32_t q = lane_id(); q < m; q += WAVE) {
        A.tu.kd[wbase + q] = S.kd[q];
        A.tu.sn[wbase + q] = S.sn[q];
        A.tu.vp[wbase + q] = S.vp[q];
        A.tu.vlen[wbase + q] = S.vlen[q];
        A.tu.blk[wbase + q] = S.blk[q];
        A.tu.eoff[wbase + q] = S.eoff[q];
      }
      wave_sync();
    }
  }
  if (KIND == 1 && MODE == 0) {
    maxk_all = wave_max(maxk_all);
    if (lane_id() == 0 && maxk_all) atomicMax(A.maxklen, maxk_all);
  }
}

template __global__ void k_walk<0, 0>(WalkArgs);
template __global__ void k_walk<0, 1>(WalkArgs);
template __global__ void k_walk<1, 0>(WalkArgs);
template __global__ void k_walk<1, 1>(WalkArgs);

// ---------------------------------------------------------------------------
// k_keys: restore each internal key.  Byte q of entry e's key comes from the
// latest entry e' <= e (inside the same restart interval) whose shared count
// is <= q, at position q - shared(e') of e' 's key delta.  The key is built
// from up to MAXSEG such segments with 8-byte loads; longer chains fall back
// to bytes.

constexpr int MAXSEG = 6;

__device__ inline uint64_t load8_masked(const uint8_t* src, uint32_t nbytes) {
  // nbytes (1..8) bytes from src; the rest of the 8-byte load stays inside
  // the table (a key delta is followed by its value, later entries, the
  // restart array and the block trailer)
  uint64_t v;
  __builtin_memcpy(&v, src, 8);
  if (nbytes < 8) v &= (~0ull) >> (64 - 8 * nbytes);
  return v;
}

__global__ void k_keys(Tuples tu, WalkSet ws, Inputs in, uint32_t kw8, const uint64_t* n_dev,
                       unsigned long long* err) {
  const uint64_t n = *n_dev;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t sn = tu.sn[e];
    const uint32_t shared = (uint32_t)sn, ns = (uint32_t)(sn >> 32);
    const uint32_t klen = shared + ns;
    const uint32_t ulen = klen - 8;
    // segments [lo, hi) of the internal key and their sources
    uint32_t lo[MAXSEG], hi[MAXSEG];
    uint64_t src[MAXSEG];
    int nseg = 0;
    bool overflow = false;
    {
      uint32_t h = klen, s = shared;
      uint64_t cur = e, sa = tu.kd[e];
      for (;;) {
        if (s < h) {
          if (nseg == MAXSEG) {
            overflow = true;
            break;
          }
          lo[nseg] = s;
          hi[nseg] = h;
          src[nseg] = sa;
          nseg++;
          h = s;
        }
        if (h == 0) break;
        cur--;
        const uint64_t psn = tu.sn[cur];
        s = (uint32_t)psn;
        sa = tu.kd[cur];
      }
    }
    uint64_t* slot = tu.heap + e * kw8;
    uint64_t tag = 0;
    if (!overflow) {
      for (uint32_t w = 0; w < kw8; w++) {
        const uint32_t a0 = w * 8;
        uint64_t word = 0;
        if (a0 < ulen) {
          const uint32_t a1 = min(a0 + 8, ulen);
          for (int q = 0; q < nseg; q++) {
            const uint32_t x0 = max(a0, lo[q]), x1 = min(a1, hi[q]);
            if (x0 < x1) word |= load8_masked((const uint8_t*)src[q] + (x0 - lo[q]), x1 - x0) << (8 * (x0 - a0));
          }
        }
        slot[w] = word;
      }
      for (int q = 0; q < nseg; q++) {
        const uint32_t x0 = max(ulen, lo[q]), x1 = min(klen, hi[q]);
        if (x0 < x1) tag |= load8_masked((const uint8_t*)src[q] + (x0 - lo[q]), x1 - x0) << (8 * (x0 - ulen));
      }
    } else {
      for (uint32_t w = 0; w < kw8; w++) slot[w] = 0;
      uint8_t* sb = (uint8_t*)slot;
      uint32_t h = klen, s = shared;
      uint64_t cur = e, sa = tu.kd[e];
      for (;;) {
        if (s < h) {
          const uint8_t* d = (const uint8_t*)sa;
          for (uint32_t q = s; q < h; q++) {
            const uint32_t byte = d[q - s];
            if (q < ulen) sb[q] = (uint8_t)byte;
            else tag |= (uint64_t)byte << (8 * (q - ulen));
          }
          h = s;
        }
        if (h == 0) break;
        cur--;
        s = (uint32_t)tu.sn[cur];
        sa = tu.kd[cur];
      }
    }
    tu.kp0[e] = bswap64(slot[0]);
    tu.kp1[e] = kw8 > 1 ? bswap64(slot[1]) : 0;
    tu.tag[e] = tag;
    tu.ulen[e] = ulen;
    if ((tag & 0xFF) > 1) blk_err(ws, in, tu.blk[e], P_ENTRIES, tu.eoff[e], EC_FORMAT, err);
  }
}

// k_order: entries of one table strictly increase; and for the first entry
// of every table after a job's first, how it compares with the previous
// table's last entry (in_cmp: -1 less, 0 equal, 1 greater, 2 no entries).
__global__ void k_order(Tuples tu, WalkSet ws, Inputs in, const uint64_t* in_e0, uint32_t kw8, const uint64_t* n_dev,
                        int32_t* in_cmp, unsigned long long* err) {
  const uint64_t n = *n_dev;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t b = tu.blk[e];
    const uint32_t g = ws.input[b];
    if (e != in_e0[g]) {
      if (cmp_ikeys(tu, kw8, e - 1, e) >= 0) blk_err(ws, in, b, P_ENTRIES, tu.eoff[e], EC_UNSORTED, err);
    } else if (e > 0 && in.local[g] > 0) {
      const uint32_t pg = ws.input[tu.blk[e - 1]];
      if (in.job[pg] == in.job[g] && pg == g - 1) in_cmp[g] = cmp_ikeys(tu, kw8, e - 1, e);
    }
  }
}

}  // namespace luda
