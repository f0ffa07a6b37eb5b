// Phase 3 "Pack" writers (paper Sec. II-A Phase 3; Sec. III-C: encode fills
// data blocks and checksums them with no data exchange between blocks, filter
// builds each table's Bloom filter block).  Values move once: from the input
// table bytes straight into the output block (the paper's lazy value
// movement, Sec. III-D, without the intermediate pair buffer).
//
//   k_gaps         one thread per gap chunk of a block (a 16-byte chunk not
//                  wholly inside one value): assembles it into the gap buffer
//   k_encode       one wave per output data block: every 16-byte chunk of
//                  the block is one load (from a value, or from the gap
//                  buffer), stored and folded into the block's CRC
//   k_key_hash     one thread per surviving key: its XXH64
//   k_filter_small one thread per small filter window: bits in a private LDS
//                  slot
//   k_filter       one wave per larger filter window: bits in LDS, then stored
//   k_index_write  one thread per data block: its index entry and restart slot
//   k_meta         one thread per file: filter tail, metaindex, trailers' type
//                  bytes, footer
//   k_crc_multi    checksums of each file's filter, metaindex and index
//                  blocks, segments of them spread over the grid
#include "dev_common.h"
#include "kernels.h"
#include "crc_multi.h"

namespace luda {

__device__ inline uint32_t vlen32(uint32_t v) {
  return 1u + (v >= (1u << 7)) + (v >= (1u << 14)) + (v >= (1u << 21)) + (v >= (1u << 28));
}

typedef unsigned __int128 u128;

__device__ inline u128 shr_bytes(u128 v, uint32_t o) { return o >= 16 ? (u128)0 : v >> (8 * o); }
__device__ inline u128 shl_bytes(u128 v, uint32_t o) { return o >= 16 ? (u128)0 : v << (8 * o); }
__device__ inline u128 keep_bytes(u128 v, uint32_t n) {
  return n >= 16 ? v : v & ((((u128)1) << (8 * n)) - 1);
}

// the n (1..16) bytes at address a as a little-endian 128-bit value; only
// [a, a + n) need be readable: the loads are aligned 16-byte loads, and an
// aligned load holding a readable byte never leaves that byte's page
__device__ inline u128 load_span(const uint8_t* a, uint32_t n) {
  const uintptr_t x = (uintptr_t)a;
  const uint32_t s = (uint32_t)(x & 15);
  const uint64_t p = (uint64_t)(x - s);
  const uint4 w0 = ldg16a(p);
  u128 r = ((u128)(((uint64_t)w0.w << 32) | w0.z) << 64) | (((uint64_t)w0.y << 32) | w0.x);
  r >>= 8 * s;
  if (s + n > 16) {
    const uint4 w1 = ldg16a(p + 16);
    const u128 h = ((u128)(((uint64_t)w1.w << 32) | w1.z) << 64) | (((uint64_t)w1.y << 32) | w1.x);
    r |= h << (8 * (16 - s));
  }
  return keep_bytes(r, n);
}

__device__ inline uint64_t pack_varint(uint32_t v, uint32_t* len) {
  uint64_t r = 0;
  uint32_t n = 0;
  while (v >= 128) {
    r |= (uint64_t)((v & 127u) | 128u) << (8 * n);
    v >>= 7;
    n++;
  }
  r |= (uint64_t)v << (8 * n);
  *len = n + 1;
  return r;
}

// bytes [q0, q0 + n) of an internal key (user key from its zero-padded slot
// of kw8 words, then the 8-byte tag)
__device__ inline u128 ikey_span(const uint64_t* slot, uint32_t kw8, uint32_t ul, uint64_t tag, uint32_t q0,
                                 uint32_t n) {
  u128 r;
  if (q0 < ul) {
    const uint32_t w = q0 >> 3, b = q0 & 7;
    const uint64_t a0 = slot[w];
    const uint64_t a1 = (w + 1 < kw8) ? slot[w + 1] : 0;
    const uint64_t a2 = (w + 2 < kw8) ? slot[w + 2] : 0;
    r = (((u128)a1 << 64) | a0) >> (8 * b);
    if (b) r |= (u128)a2 << (128 - 8 * b);
    r = keep_bytes(r, ul - q0) | shl_bytes((u128)tag, ul - q0);
  } else {
    r = shr_bytes((u128)tag, q0 - ul);
  }
  return keep_bytes(r, n);
}

// overlap of block segment [a, b) with the chunk's bytes at positions >= 0:
// source offset o, chunk offset d, length n (0: none)
struct Ov {
  uint32_t o, d, n;
};
__device__ inline Ov overlap(int64_t p0, int64_t a, int64_t b) {
  const int64_t x0 = max(a, max(p0, (int64_t)0)), x1 = min(b, p0 + 16);
  Ov r;
  r.n = x0 < x1 ? (uint32_t)(x1 - x0) : 0u;
  r.o = (uint32_t)(x0 - a);
  r.d = (uint32_t)(x0 - p0);
  return r;
}

// Message bytes [p0, p0 + 16) of block B (positions outside [0, n) give
// zeros), assembled from the overlapping parts: each entry's header, key
// delta and value, then restart offsets, the restart count and the type
// byte (0).  No entry before i0 reaches p0.  Ents gives entry i's start
// (st(i)) and record (rec(i)).
template <class Ents>
__device__ uint4 enc_bytes(const EncodeArgs& A, const BlockRec& B, const Ents& X, int64_t p0, uint32_t i0) {
  const uint32_t R = B.R, cnt = B.cnt, size = B.size;
  const uint32_t nrest = div_r(cnt + R - 1, R);
  const uint32_t data_end = size - 4 * nrest - 4;
  const uint32_t* off = A.ent_off + B.s0;
  u128 acc = 0;
  const int64_t pend = p0 + 16, q0 = p0 < 0 ? 0 : p0;
  if (q0 < (int64_t)data_end) {
    for (uint32_t i = i0; i < cnt; i++) {
      const int64_t st = X.st(i);
      if (st >= pend) break;
      const EncRec r = X.rec(i);
      const uint32_t sh = mod_r(i, R) == 0 ? 0u : r.shared;
      const uint32_t ns = r.ulen + 8 - sh;
      uint32_t la, lb, lc;
      const uint64_t va = pack_varint(sh, &la), vb = pack_varint(ns, &lb), vc = pack_varint(r.vlen, &lc);
      const int64_t ks = st + la + lb + lc, vs = ks + ns, en = vs + r.vlen;
      const Ov h = overlap(p0, st, ks);
      if (h.n) {
        const u128 H = (u128)va | ((u128)vb << (8 * la)) | ((u128)vc << (8 * (la + lb)));
        acc |= shl_bytes(keep_bytes(shr_bytes(H, h.o), h.n), h.d);
      }
      const Ov k = overlap(p0, ks, vs);
      if (k.n) acc |= shl_bytes(ikey_span(A.tu.heap + (uint64_t)r.e * A.kw8, A.kw8, r.ulen, r.tag, sh + k.o, k.n), k.d);
      const Ov v = overlap(p0, vs, en);
      if (v.n) acc |= shl_bytes(load_span((const uint8_t*)r.vp + v.o, v.n), v.d);
    }
  }
  if (pend > (int64_t)data_end) {
    const int64_t from = q0 > (int64_t)data_end ? q0 : (int64_t)data_end;
    for (uint32_t r = (uint32_t)((from - data_end) >> 2); r < nrest; r++) {
      const int64_t a = (int64_t)data_end + 4ll * r;
      if (a >= pend) break;
      const Ov o = overlap(p0, a, a + 4);
      if (o.n) acc |= shl_bytes(keep_bytes((u128)(off[(uint64_t)r * R] >> (8 * o.o)), o.n), o.d);
    }
    const int64_t a = (int64_t)size - 4;
    const Ov o = overlap(p0, a, a + 4);
    if (o.n) acc |= shl_bytes(keep_bytes((u128)(nrest >> (8 * o.o)), o.n), o.d);
  }
  return make_uint4((uint32_t)acc, (uint32_t)(acc >> 32), (uint32_t)(acc >> 64), (uint32_t)(acc >> 96));
}

// ---------------------------------------------------------------------------
// Gap chunks.  A block message is cut into 16-byte chunks aligned to its end
// (chunk m covers positions [16 m - gshift, 16 m - gshift + 16), gshift =
// 16 J16 - n).  The chunks lying wholly inside one value (its interior) are
// copied from the input by the encoder; every other chunk (headers, key
// deltas, value edges, the restart array and the block tail) is a gap chunk,
// assembled here once into the gap buffer.  Slot 0 of a block holds its
// message bytes [0, 16) instead (what the encoder stores for a first chunk
// that starts before the message); slots 1.. hold the gap chunks in order.
// One thread per slot.

// Threads go to blocks in groups of GAP_GROUP lanes of one wave: lane j of a
// block's group takes its slots j, j + GAP_GROUP, ...  A block of at most
// GAP_GROUP entries has its entries staged in LDS by the group first (one
// round of loads), a larger one is read from global memory.

struct GapEnt {
  EncRec r;
  uint32_t st, ia, pieces, cum;
};

struct EntsGlobal {
  const EncodeArgs* A;
  uint64_t s0;
  __device__ uint32_t st(uint32_t i) const { return A->ent_off[s0 + i]; }
  __device__ EncRec rec(uint32_t i) const { return A->rec[s0 + i]; }
  __device__ uint32_t gb(uint32_t i) const { return A->entl[s0 + i].ia - A->entl[s0 + i].cum; }
  __device__ uint32_t after(uint32_t i) const { return A->entl[s0 + i].cum + A->entl[s0 + i].pieces; }
};

struct EntsLds {
  const GapEnt* L;
  __device__ uint32_t st(uint32_t i) const { return L[i].st; }
  __device__ EncRec rec(uint32_t i) const { return L[i].r; }
  __device__ uint32_t gb(uint32_t i) const { return L[i].ia - L[i].cum; }
  __device__ uint32_t after(uint32_t i) const { return L[i].cum + L[i].pieces; }
};

// gap slot g of block B into the gap buffer
template <class Ents>
__device__ __forceinline__ void gap_slot(const EncodeArgs& A, const BlockRec& B, const Ents& X, uint64_t g0,
                                         uint64_t g) {
  const uint32_t n = B.size + 1, J16 = (n + 15) / 16, gshift = 16 * J16 - n;
  int64_t p0 = 0;
  uint32_t lo = 0;
  if (g > 0) {
    // gap chunk g - 1: after the interior of the last entry with fewer gap
    // chunks before its interior (ia - cum) than g
    const uint64_t gq = g - 1;
    uint64_t m = gq;
    if ((uint64_t)X.gb(0) <= gq) {
      uint32_t hi = B.cnt;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)X.gb(mid) <= gq) lo = mid;
        else hi = mid;
      }
      m = gq + X.after(lo);
    }
    p0 = 16 * (int64_t)m - (int64_t)gshift;
  }
  A.gapbuf[g0 + g] = enc_bytes(A, B, X, p0, lo);
}

// Entry-major form of the gap chunks of a block of at most GAP_GROUP
// entries, GAP_SLOTS gap slots and keys of at most GAP_KW8 words: the slots
// are an LDS image of the block's gap bytes.  Message position p before
// entry i's value interior lies in gap slot 1 + (p + gshift) / 16 - cum_i,
// so its image byte is 16 (1 - cum_i) + gshift + p; after the interior it
// is 16 pieces_i lower.  Each lane writes its entry's header, key delta and
// value edges byte by byte (slot 0 also receives message bytes [0, 16),
// interior ones included),
// the lanes write the restart array and count, and the image is stored
// whole.  Bytes no entry writes (before the message, the type byte) stay 0.

__device__ __forceinline__ uint32_t byte_of(uint64_t lo, uint64_t hi, uint32_t k) {  // byte k (< 16) of hi:lo
  return (uint32_t)((k < 8 ? lo >> (8 * k) : hi >> (8 * (k - 8))) & 0xFF);
}

// this lane's entry x (index i in block B) into the image I
__device__ __forceinline__ void gap_entry_bytes(const EncodeArgs& A, const BlockRec& B, const GapEnt& x, uint32_t i,
                                                uint32_t gshift, uint8_t* I) {
  const EncRec& r = x.r;
  const uint32_t sh = mod_r(i, B.R) == 0 ? 0u : r.shared;
  const uint32_t klen = r.ulen + 8, nsk = klen - sh;
  uint32_t la, lb, lc;
  const uint64_t va = pack_varint(sh, &la), vb = pack_varint(nsk, &lb), vc = pack_varint(r.vlen, &lc);
  const u128 H = (u128)va | ((u128)vb << (8 * la)) | ((u128)vc << (8 * (la + lb)));
  const uint64_t h0 = (uint64_t)H, h1 = (uint64_t)(H >> 64);
  const uint32_t hlen = la + lb + lc;
  const int32_t bb = 16 * (1 - (int32_t)x.cum) + (int32_t)gshift, ba = bb - 16 * (int32_t)x.pieces;
  const uint32_t st = x.st, ks = st + hlen, vs = ks + nsk, en = vs + r.vlen;
  const uint32_t i0 = x.pieces ? 16 * x.ia - gshift : en, i1 = x.pieces ? 16 * (x.ia + x.pieces) - gshift : en;
  auto put = [&](uint32_t p, int32_t base, uint32_t v) {
    I[base + (int32_t)p] = (uint8_t)v;
    if (p < 16) I[p] = (uint8_t)v;
  };
  for (uint32_t k = 0; k < hlen; k++) put(st + k, bb, byte_of(h0, h1, k));
  // key delta: internal key bytes [sh, klen) (user key words, then the tag)
  const uint64_t* slot = A.tu.heap + (uint64_t)r.e * A.kw8;
  uint64_t kw[GAP_KW8];
#pragma unroll
  for (uint32_t w = 0; w < GAP_KW8; w++) kw[w] = w < A.kw8 ? slot[w] : 0ull;
  for (uint32_t k = 0; k < nsk; k++) {
    const uint32_t q = sh + k;
    uint32_t v;
    if (q < r.ulen) {
      const uint32_t w = q >> 3;
      const uint64_t word = w == 0 ? kw[0] : (w == 1 ? kw[1] : kw[2]);
      v = (uint32_t)((word >> (8 * (q & 7))) & 0xFF);
    } else {
      v = (uint32_t)((r.tag >> (8 * (q - r.ulen))) & 0xFF);
    }
    put(ks + k, bb, v);
  }
  // value edges: [vs, i0) and [i1, en), at most 30 bytes with no interior
  const uint8_t* vp = (const uint8_t*)r.vp;
  const uint32_t nh = min(i0, en) - vs;
  for (uint32_t k0 = 0; k0 < nh; k0 += 15) {
    const uint32_t n = min(15u, nh - k0);
    const u128 v = load_span(vp + k0, n);
    const uint64_t v0 = (uint64_t)v, v1 = (uint64_t)(v >> 64);
    for (uint32_t k = 0; k < n; k++) put(vs + k0 + k, bb, byte_of(v0, v1, k));
  }
  if (x.pieces && i0 < 16) {  // interior bytes below position 16: slot 0 only
    const uint32_t nz = min(i1, 16u) - i0;
    const u128 v = load_span(vp + (i0 - vs), nz);
    const uint64_t v0 = (uint64_t)v, v1 = (uint64_t)(v >> 64);
    for (uint32_t k = 0; k < nz; k++) I[i0 + k] = (uint8_t)byte_of(v0, v1, k);
  }
  if (x.pieces) {
    const uint32_t nt = en - i1;
    if (nt) {
      const u128 v = load_span(vp + (i1 - vs), nt);
      const uint64_t v0 = (uint64_t)v, v1 = (uint64_t)(v >> 64);
      for (uint32_t k = 0; k < nt; k++) put(i1 + k, ba, byte_of(v0, v1, k));
    }
  }
}

// blocks whose gap chunks are written entry-major
__device__ __forceinline__ bool gap_entry_major(const EncodeArgs& A, const BlockRec& B, uint64_t ns) {
  return A.kw8 <= GAP_KW8 && gap_em_block(B.cnt, B.size, ns);
}

// EM = false: the blocks written chunk by chunk; EM = true: the others
// (two kernels, so that each keeps its own register budget)
template <bool EM>
__global__ void __launch_bounds__(256) k_gaps(EncodeArgs A) {
  constexpr uint32_t G = EM ? GAP_EM_GROUP : GAP_GROUP;  // lanes per block
  __shared__ GapEnt lds[EM ? 1 : 256 / GAP_GROUP][GAP_GROUP];
  __shared__ uint4 img_all[EM ? 256 / GAP_EM_GROUP : 1][GAP_SLOTS];
  const uint64_t nb = *A.nblocks;
  const uint64_t groups = (uint64_t)gridDim.x * blockDim.x / G;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t j = threadIdx.x % G;
  for (uint64_t b = tid / G; b < nb; b += groups) {
    const BlockRec B = A.blk[b];
    const uint64_t g0 = A.gap_base[b], ns = A.gap_base[b + 1] - g0;
    if (gap_entry_major(A, B, ns) != EM) continue;
    if constexpr (EM) {
      uint4* img = img_all[threadIdx.x / G];
      const uint32_t n = B.size + 1, J16 = (n + 15) / 16, gshift = 16 * J16 - n;
      for (uint64_t g = j; g < ns; g += G) img[g] = make_uint4(0, 0, 0, 0);
      wave_sync();
      for (uint32_t i = j; i < B.cnt; i += G) {
        const EntL e = A.entl[B.s0 + i];
        GapEnt x;
        x.r = A.rec[B.s0 + i];
        x.st = A.ent_off[B.s0 + i];
        x.ia = e.ia;
        x.pieces = e.pieces;
        x.cum = e.cum;
        gap_entry_bytes(A, B, x, i, gshift, (uint8_t*)img);
      }
      // the restart array and the count follow every interior of the block
      const uint32_t R = B.R, nrest = div_r(B.cnt + R - 1, R);
      const uint32_t data_end = B.size - 4 * nrest - 4;
      const int32_t bt = 16 * (1 - (int32_t)(J16 + 1 - (uint32_t)ns)) + (int32_t)gshift;
      uint8_t* I = (uint8_t*)img;
      for (uint32_t q = j; q <= nrest; q += G) {
        const uint32_t v = q < nrest ? A.ent_off[B.s0 + (uint64_t)q * R] : nrest;
        const uint32_t p = data_end + 4 * q;
        for (uint32_t k = 0; k < 4; k++) {
          I[bt + (int32_t)(p + k)] = (uint8_t)(v >> (8 * k));
          if (p + k < 16) I[p + k] = (uint8_t)(v >> (8 * k));
        }
      }
      wave_sync();
      for (uint64_t g = j; g < ns; g += G) A.gapbuf[g0 + g] = img[g];
      wave_sync();
    } else if (B.cnt <= GAP_GROUP) {
      GapEnt* L = lds[threadIdx.x / GAP_GROUP];
      if (j < B.cnt) {
        const EntL e = A.entl[B.s0 + j];
        GapEnt x;
        x.r = A.rec[B.s0 + j];
        x.st = A.ent_off[B.s0 + j];
        x.ia = e.ia;
        x.pieces = e.pieces;
        x.cum = e.cum;
        L[j] = x;
      }
      wave_sync();
      const EntsLds X{L};
      for (uint64_t g = j; g < ns; g += GAP_GROUP) gap_slot(A, B, X, g0, g);
      wave_sync();
    } else {
      const EntsGlobal X{&A, B.s0};
      for (uint64_t g = j; g < ns; g += GAP_GROUP) gap_slot(A, B, X, g0, g);
    }
  }
}

template __global__ void k_gaps<false>(EncodeArgs);
template __global__ void k_gaps<true>(EncodeArgs);

// ---------------------------------------------------------------------------
// Encoder: one wave per output data block.  Lane l takes the chunks
// c = 63 - l + 64 i (counted from the end of the message, first to last):
// an interior chunk is read from its value, a gap chunk from the gap buffer;
// each is stored into the output and folded into the lane's CRC register
// (Horner, a shift by 1024 bytes between a lane's chunks), and the lanes are
// joined at the end.  The chunk sources come from the block's entry layout
// (lane i holds entry i when the block has at most 64 entries; a binary
// search over it by shuffles finds a chunk's entry).
//
// Blocks are software-pipelined: while block X is stored and checksummed,
// the chunk loads of block X+1 are in flight, its layout was loaded one block
// ahead and its handle two blocks ahead.  Every load and store of the common
// path is issued by every lane (a lane with nothing to load reads a fixed
// valid address; stores go through a buffer descriptor of the block, and a
// lane with nothing to store uses an offset past its end, which the hardware
// drops), so each wait is for exactly the loads it needs.

constexpr uint32_t ENC_QS = ENC_PIPE_CHUNKS;  // chunks per lane in registers: blocks up to 5 KiB pipelined
constexpr uint32_t ENC_OOB = 0x80000000u;  // a buffer offset past any block

struct EncH {  // one block, the same in every lane
  uint64_t dst, s0, gap;
  uint32_t cnt, n, J16, gshift;
  bool valid, piped;
};

__device__ __forceinline__ EncH enc_handle(const EncodeArgs& A, uint64_t b, uint64_t nb) {
  const uint64_t bb = b < nb ? b : nb - 1;  // nb > 0
  const BlockRec r = A.blk[bb];
  EncH h;
  h.dst = r.dst;
  h.s0 = r.s0;
  h.gap = A.gap_base[bb];
  h.cnt = r.cnt;
  h.n = r.size + 1;
  h.J16 = (h.n + 15) / 16;
  h.gshift = 16 * h.J16 - h.n;
  h.valid = b < nb;
  h.piped = enc_pipelined(r.size, r.cnt);
  return h;
}

// this lane's entry of the block (lanes past its end repeat the last one)
__device__ __forceinline__ EntL enc_entl(const EncodeArgs& A, const EncH& H) {
  return A.entl[H.s0 + min(lane_id(), H.cnt - 1)];  // cnt >= 1
}

// the source address of chunk m of block H, E being this lane's entry of it
// (the block has at most 64 entries)
__device__ __forceinline__ uint64_t enc_src(const EncodeArgs& A, const EncH& H, const EntL& E, uint32_t m) {
  // the last entry whose interior starts at or before m (entry 0 if none):
  // the same steps in every lane, so that every shuffle reads active lanes
  uint32_t lo = 0;
  for (uint32_t step = H.cnt > 1 ? 1u << (31 - __builtin_clz(H.cnt - 1)) : 0u; step; step >>= 1) {
    const uint32_t k = min(lo + step, H.cnt - 1);
    if ((uint32_t)__shfl((int)E.ia, (int)k, WAVE) <= m && lo + step < H.cnt) lo += step;
  }
  const uint32_t ia = __shfl((int)E.ia, (int)lo, WAVE), pieces = __shfl((int)E.pieces, (int)lo, WAVE);
  const uint32_t cum = __shfl((int)E.cum, (int)lo, WAVE);
  const uint64_t vsrc = ((uint64_t)(uint32_t)__shfl((int)(E.vsrc >> 32), (int)lo, WAVE) << 32) |
                        (uint32_t)__shfl((int)(uint32_t)E.vsrc, (int)lo, WAVE);
  if (ia <= m && m < ia + pieces) return vsrc + 16ull * m;
  const uint32_t g = ia <= m ? m - cum - pieces : m;  // gap chunks before m
  return (uint64_t)(uintptr_t)(A.gapbuf + H.gap + 1 + g);
}

// the same for any block: binary search over the global layout
__device__ __forceinline__ uint64_t enc_src_any(const EncodeArgs& A, const EncH& H, uint32_t m) {
  const EntL* E = A.entl + H.s0;
  uint32_t lo = 0, hi = H.cnt;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (E[mid].ia <= m) lo = mid;
    else hi = mid;
  }
  const EntL e = E[lo];
  if (e.ia <= m && m < e.ia + e.pieces) return e.vsrc + 16ull * m;
  const uint32_t g = e.ia <= m ? m - e.cum - e.pieces : m;
  return (uint64_t)(uintptr_t)(A.gapbuf + H.gap + 1 + g);
}

__device__ __forceinline__ int64_t enc_top(const EncH& H) {
  const int64_t c0 = 63 - (int64_t)lane_id();
  return c0 < (int64_t)H.J16 ? c0 + 64 * (((int64_t)H.J16 - 1 - c0) / 64) : -1;
}

// chunk loads of a pipelined block: ENC_QS chunks and the head slot
struct EncV {
  uint4 v[ENC_QS];
  uint4 head;
};

__device__ __forceinline__ void enc_load(const EncodeArgs& A, const EncH& H, const EntL& E, uint64_t safe, EncV& V) {
  const int64_t ct = enc_top(H);
#pragma unroll
  for (uint32_t q = 0; q < ENC_QS; q++) {
    const int64_t c = ct - 64 * (int64_t)q;
    const uint64_t src = enc_src(A, H, E, (uint32_t)((int64_t)H.J16 - 1 - (c >= 0 ? c : 0)));
    V.v[q] = ldg16(c >= 0 && H.valid ? src : safe);
  }
  V.head = ldg16(H.valid ? (uint64_t)(uintptr_t)(A.gapbuf + H.gap) : safe);
}

// stores and checksums a pipelined block from registers
__device__ __forceinline__ void enc_store(const CrcLds* T, const EncodeArgs& A, const EncH& H, const EncV& V) {
  const int64_t ct = enc_top(H);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(A.out + H.dst, (short)0, (int)(H.n + 4), 0x00020000);
  uint32_t acc = 0;
#pragma unroll
  for (uint32_t q = 0; q < ENC_QS; q++) {
    const int64_t c = ct - 64 * (int64_t)q;
    const int64_t p0 = (int64_t)H.n - 16 * (c + 1);
    const uint4 o = (q == 0 && p0 < 0) ? V.head : V.v[q];
    const u32x4 dv = {o.x, o.y, o.z, o.w};
    __builtin_amdgcn_raw_buffer_store_b128(dv, rs, c >= 0 ? (uint32_t)(p0 > 0 ? p0 : 0) : ENC_OOB, 0, 0);
    if (c >= 0) {
      if (q == 0) acc = p0 < 4 ? crc_chunk(T, V.v[0], p0) : crc_chunk_plain(T, V.v[0]);
      else acc = crc_shift(T->sh[6], acc) ^ crc_chunk_plain(T, V.v[q]);
    }
  }
  const uint32_t raw = crc_wave_join(T, acc);
  __builtin_amdgcn_raw_buffer_store_b32(crc_mask(raw ^ 0xFFFFFFFFu), rs, lane_id() == 0 ? H.n : ENC_OOB, 0, 0);
}

// Any block, 64 chunks per step.  Lane chunks cover 64 consecutive chunk
// indices m at each step, [64i, 64i + 64).  The entries whose interiors can
// hold them start at `base`, the entry found for the step's largest m one
// step earlier.  They are loaded 64 at a time (one per lane, coalesced) and
// searched by shuffles, as in the pipelined path.  A lane whose chunk lies
// past those 64 entries (more than 64 entries start in 1 KiB of the block)
// searches the global layout instead.  Every lane runs the same steps and
// issues the same loads, so each wait is exact.
__device__ void enc_block_any(const CrcLds* T, const EncodeArgs& A, const EncH& H, uint64_t safe) {
  uint8_t* dst = A.out + H.dst;
  const uint32_t n = H.n;
  const EntL* E = A.entl + H.s0;
  const int64_t ct = enc_top(H);
  const uint32_t steps = (H.J16 + 63) / 64;
  const int top_lane = 63 - (int)(H.J16 & 63);  // holds the largest m of every full step
  uint32_t base = 0, acc = 0;
  uint32_t wn = min(64u, H.cnt);  // entries in the window, >= 1
  EntL W = E[min(lane_id(), wn - 1)];
  for (uint32_t i = 0; i < steps; i++) {
    const int64_t c = ct - 64 * (int64_t)i;
    const bool act = c >= 0;
    const uint32_t m = act ? (uint32_t)((int64_t)H.J16 - 1 - c) : 64 * i;
    uint32_t lo = 0;
    for (uint32_t step = wn > 1 ? 1u << (31 - __builtin_clz(wn - 1)) : 0u; step; step >>= 1) {
      const uint32_t k = min(lo + step, wn - 1);
      if ((uint32_t)__shfl((int)W.ia, (int)k, WAVE) <= m && lo + step < wn) lo += step;
    }
    const uint32_t ia = __shfl((int)W.ia, (int)lo, WAVE), pieces = __shfl((int)W.pieces, (int)lo, WAVE);
    const uint32_t cum = __shfl((int)W.cum, (int)lo, WAVE);
    const uint64_t vsrc = ((uint64_t)(uint32_t)__shfl((int)(W.vsrc >> 32), (int)lo, WAVE) << 32) |
                          (uint32_t)__shfl((int)(uint32_t)W.vsrc, (int)lo, WAVE);
    uint64_t src;
    if (act && lo == 63 && base + 64 < H.cnt && E[base + 64].ia <= m) {
      src = enc_src_any(A, H, m);
    } else if (ia <= m && m < ia + pieces) {
      src = vsrc + 16ull * m;
    } else {
      const uint32_t g = ia <= m ? m - cum - pieces : m;  // gap chunks before m
      src = (uint64_t)(uintptr_t)(A.gapbuf + H.gap + 1 + g);
    }
    const uint4 v = ldg16(act ? src : safe);
    // the next step's window is loaded while this chunk is in flight (on the
    // last step too, in bounds and unused: no branch around the load)
    base += (uint32_t)__shfl((int)lo, top_lane, WAVE);
    wn = min(64u, H.cnt - base);
    W = E[base + min(lane_id(), wn - 1)];
    if (act) {
      const int64_t p0 = (int64_t)n - 16 * (c + 1);
      if (p0 >= 0) {
        __builtin_memcpy(dst + p0, &v, 16);
        acc = crc_shift(T->sh[6], acc) ^ (p0 < 4 ? crc_chunk(T, v, p0) : crc_chunk_plain(T, v));
      } else {
        const uint8_t* vb = (const uint8_t*)&v;
        for (int k = 0; k < 16; k++)
          if (p0 + k >= 0) dst[p0 + k] = vb[k];
        acc = crc_shift(T->sh[6], acc) ^ crc_chunk(T, v, p0);
      }
    }
  }
  const uint32_t raw = crc_wave_join(T, acc);
  if (lane_id() == 0) {
    const uint32_t m = crc_mask(raw ^ 0xFFFFFFFFu);
    __builtin_memcpy(dst + n, &m, 4);
  }
}

__global__ void __launch_bounds__(1024) k_encode(EncodeArgs A) {
  __shared__ CrcLds T;
  load_crc_tables(&T, A.g_crc, threadIdx.x, blockDim.x);
  __syncthreads();
  const uint64_t nb = *A.nblocks;
  if (nb == 0) return;
  // the wave index is the same in every lane: block handles are scalar loads
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const uint64_t stride = (uint64_t)gridDim.x * (blockDim.x / WAVE);
  const uint64_t safe = (uint64_t)(uintptr_t)A.g_crc;
  uint64_t b = (uint64_t)blockIdx.x * (blockDim.x / WAVE) + wv;
  if (b >= nb) return;
  EncH H0 = enc_handle(A, b, nb), H1 = enc_handle(A, b + stride, nb), H2 = enc_handle(A, b + 2 * stride, nb);
  EntL E1 = enc_entl(A, H1);
  EncV V0;
  if (H0.piped) {
    const EntL E0 = enc_entl(A, H0);
    enc_load(A, H0, E0, safe, V0);
  }
  for (; b < nb; b += stride) {
    const EncH H3 = enc_handle(A, b + 3 * stride, nb);
    EncV V1;
    if (H1.piped) enc_load(A, H1, E1, safe, V1);
    const EntL E2 = enc_entl(A, H2);
    if (H0.piped) enc_store(&T, A, H0, V0);  // other blocks: k_encode_big
    H0 = H1;
    H1 = H2;
    H2 = H3;
    E1 = E2;
    V0 = V1;
  }
}

// Blocks off the pipelined path (over 5 KiB or 64 entries): one wave per
// block.  The block's entry layout is staged in LDS first, so that every
// chunk's source is found by a binary search in LDS without waiting on
// memory; the chunk loads of ENCB_Q steps (64 chunks each) are then in
// flight together before they are stored and folded.  Blocks of more than
// ENCB_ENTS entries take the windowed walk of enc_block_any instead.
constexpr uint32_t ENCB_WAVES = 8;
constexpr uint32_t ENCB_ENTS = 64;
constexpr uint32_t ENCB_Q = 4;

struct EncbEnt {
  uint64_t vsrc;
  uint32_t ia, pieces, cum, pad;
};

__global__ void __launch_bounds__(ENCB_WAVES * 64) k_encode_big(EncodeArgs A, const uint64_t* list, uint64_t nlist) {
  __shared__ CrcLds T;
  __shared__ EncbEnt L[ENCB_WAVES][ENCB_ENTS];
  load_crc_tables(&T, A.g_crc, threadIdx.x, blockDim.x);
  __syncthreads();
  const uint64_t nb = *A.nblocks;
  const uint64_t ni = list ? nlist : nb;
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const uint64_t stride = (uint64_t)gridDim.x * ENCB_WAVES;
  const uint64_t safe = (uint64_t)(uintptr_t)A.g_crc;
  EncbEnt* E = L[wv];
  for (uint64_t i = (uint64_t)blockIdx.x * ENCB_WAVES + wv; i < ni; i += stride) {
    const uint64_t b = list ? list[i] : i;
    if (b >= nb) continue;
    const EncH H = enc_handle(A, b, nb);
    if (H.piped) continue;
    if (H.cnt > ENCB_ENTS) {
      enc_block_any(&T, A, H, safe);
      continue;
    }
    for (uint32_t i = lane_id(); i < H.cnt; i += WAVE) {
      const EntL e = A.entl[H.s0 + i];
      E[i] = EncbEnt{e.vsrc, e.ia, e.pieces, e.cum, 0};
    }
    wave_sync();
    uint8_t* dst = A.out + H.dst;
    const uint32_t n = H.n;
    const int64_t ct = enc_top(H);
    const uint32_t steps = (H.J16 + 63) / 64;
    uint32_t acc = 0;
    for (uint32_t i0 = 0; i0 < steps; i0 += ENCB_Q) {
      uint4 v[ENCB_Q];
#pragma unroll
      for (uint32_t q = 0; q < ENCB_Q; q++) {
        const int64_t c = ct - 64 * (int64_t)(i0 + q);
        uint64_t src = safe;
        if (c >= 0) {
          const uint32_t m = (uint32_t)((int64_t)H.J16 - 1 - c);
          uint32_t lo = 0, hi = H.cnt;  // the last entry whose interior starts at or before m (entry 0 if none)
          while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (E[mid].ia <= m) lo = mid;
            else hi = mid;
          }
          const EncbEnt e = E[lo];
          if (e.ia <= m && m < e.ia + e.pieces) {
            src = e.vsrc + 16ull * m;
          } else {
            const uint32_t g = e.ia <= m ? m - e.cum - e.pieces : m;  // gap chunks before m
            src = (uint64_t)(uintptr_t)(A.gapbuf + H.gap + 1 + g);
          }
        }
        v[q] = ldg16(src);
      }
#pragma unroll
      for (uint32_t q = 0; q < ENCB_Q; q++) {
        const int64_t c = ct - 64 * (int64_t)(i0 + q);
        if (c < 0) continue;
        const int64_t p0 = (int64_t)n - 16 * (c + 1);
        if (p0 >= 0) {
          __builtin_memcpy(dst + p0, &v[q], 16);
          acc = crc_shift(T.sh[6], acc) ^ (p0 < 4 ? crc_chunk(&T, v[q], p0) : crc_chunk_plain(&T, v[q]));
        } else {
          const uint8_t* vb = (const uint8_t*)&v[q];
          for (int k = 0; k < 16; k++)
            if (p0 + k >= 0) dst[p0 + k] = vb[k];
          acc = crc_shift(T.sh[6], acc) ^ crc_chunk(&T, v[q], p0);
        }
      }
    }
    const uint32_t raw = crc_wave_join(&T, acc);
    if (lane_id() == 0) {
      const uint32_t mk = crc_mask(raw ^ 0xFFFFFFFFu);
      __builtin_memcpy(dst + n, &mk, 4);
    }
    wave_sync();  // the layout slots are reused by the next block
  }
}

// ---------------------------------------------------------------------------

// XXH64 of every surviving user key (the Bloom probes derive from it)
__global__ void k_key_hash(const uint32_t* surv, Tuples tu, uint32_t kw8, uint64_t n, uint64_t* hash) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t e = surv[s];
  hash[s] = xxh64_words(tu.heap + (uint64_t)e * kw8, tu.ulen[e]);
}

__device__ inline uint32_t bloom_k(uint32_t bpk) {
  uint32_t k = bpk * 69u / 100u;
  return k < 1 ? 1 : (k > 30 ? 30 : k);
}

__device__ inline uint8_t* window_dst(const FilterArgs& A, uint64_t w, uint32_t f) {
  return A.out + A.of.out[f] + A.of.filter_off[f] + (A.win_off[w] - A.win_off[A.of.w0[f]]);
}

// Filters of at most FILTER_SMALL_BYTES bytes: one thread per window, bits in
// a private LDS slot (no atomics), then stored with the probe count.
constexpr uint32_t FILTER_SMALL_BYTES = 64;
constexpr uint32_t FILTER_SLOT_WORDS = FILTER_SMALL_BYTES / 4 + 1;  // padded against bank conflicts

__global__ void __launch_bounds__(256) k_filter_small(FilterArgs A) {
  __shared__ uint32_t slots[256 * FILTER_SLOT_WORDS];
  uint32_t* bits = slots + threadIdx.x * FILTER_SLOT_WORDS;
  const uint64_t nw = *A.nwin;
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t keys = A.win_keys[w];
    if (!keys) continue;
    const uint64_t bytes = A.win_bytes[w] - 1;
    if (bytes > FILTER_SMALL_BYTES) continue;
    const uint32_t f = A.win_file[w];
    const uint32_t k = bloom_k(A.jobs[A.of.job[f]].bloom_bits_per_key);
    const uint32_t nbits = (uint32_t)bytes * 8;
#pragma unroll
    for (uint32_t i = 0; i < FILTER_SMALL_BYTES / 4; i++) bits[i] = 0;
    const uint64_t s_first = A.ob.s0[A.win_fb[w]];
    for (uint32_t i = 0; i < keys; i++) {
      const uint64_t h = A.hash[s_first + i];
      uint32_t g = (uint32_t)h;
      const uint32_t d = (uint32_t)(h >> 32);
      for (uint32_t r = 0; r < k; r++) {
        const uint32_t pos = g % nbits;
        bits[pos >> 5] |= 1u << (pos & 31);
        g += d;
      }
    }
    uint8_t* dst = window_dst(A, w, f);
    const uint8_t* src = (const uint8_t*)bits;
    for (uint32_t q = 0; q < (uint32_t)bytes; q++) dst[q] = src[q];
    dst[bytes] = (uint8_t)k;
  }
}

// Larger filters: one wave per window, bits in LDS with atomics.
__global__ void __launch_bounds__(256) k_filter(FilterArgs A) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const uint32_t wv = threadIdx.x / WAVE, l = lane_id();
  const uint32_t waves = blockDim.x / WAVE;
  uint32_t* bits = (uint32_t*)(smem + (size_t)wv * A.lds_bytes);
  const uint64_t nw = *A.nwin;
  for (uint64_t w = (uint64_t)blockIdx.x * waves + wv; w < nw; w += (uint64_t)gridDim.x * waves) {
    const uint32_t keys = A.win_keys[w];
    if (!keys) continue;
    const uint64_t bytes = A.win_bytes[w] - 1;
    if (bytes <= FILTER_SMALL_BYTES) continue;
    const uint32_t f = A.win_file[w];
    const uint32_t k = bloom_k(A.jobs[A.of.job[f]].bloom_bits_per_key);
    const uint64_t nbits = bytes * 8;
    const uint32_t words = (uint32_t)((bytes + 1 + 3) / 4);
    for (uint32_t i = l; i < words; i += WAVE) bits[i] = 0;
    wave_sync();
    const uint64_t s_first = A.ob.s0[A.win_fb[w]];
    for (uint32_t i = l; i < keys; i += WAVE) {
      const uint64_t h = A.hash[s_first + i];
      uint32_t g = (uint32_t)h;
      const uint32_t d = (uint32_t)(h >> 32);
      for (uint32_t r = 0; r < k; r++) {
        const uint32_t pos = (uint32_t)((uint64_t)g % nbits);
        atomicOr(&bits[pos >> 5], 1u << (pos & 31));
        g += d;
      }
    }
    wave_sync();
    if (l == 0) ((uint8_t*)bits)[bytes] = (uint8_t)k;
    wave_sync();
    uint8_t* dst = window_dst(A, w, f);
    const uint8_t* src = (const uint8_t*)bits;
    const uint64_t tot = bytes + 1;
    for (uint64_t o = (uint64_t)l * 16; o < tot; o += WAVE * 16) {
      if (o + 16 <= tot) {
        uint4 v = *(const uint4*)(src + o);
        __builtin_memcpy(dst + o, &v, 16);
      } else {
        for (uint64_t q = o; q < tot; q++) dst[q] = src[q];
      }
    }
    wave_sync();
  }
}

// filter offsets array slot of each window
__global__ void k_filter_offsets(OutFiles of, const uint64_t* nwin, const uint32_t* win_file,
                                 const uint64_t* win_off, uint64_t cap, uint8_t* out) {
  const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= cap || w >= *nwin) return;
  const uint32_t f = win_file[w];
  const uint64_t w0 = of.w0[f];
  const uint64_t filters = win_off[w0 + of.nwin[f]] - win_off[w0];
  uint8_t* dst = out + of.out[f] + of.filter_off[f] + filters + 4 * (w - w0);
  const uint32_t v = (uint32_t)(win_off[w] - win_off[w0]);
  for (int k = 0; k < 4; k++) dst[k] = (uint8_t)(v >> (8 * k));
}

// One thread per data block: its index entry (shared 0, key length, handle
// length, the block's last internal key, the handle) and its restart slot.
// The entries of a wave's 64 blocks are one contiguous range when the blocks
// belong to one file: they are assembled in LDS, at the range's alignment,
// and stored as whole 16-byte lines (bytes at the two ends one at a time).
// Otherwise each thread writes its entry directly.
constexpr uint32_t IW_WAVES = 4;     // waves per workgroup (the launch bound)
constexpr uint32_t IW_CAP = 4096;    // staged bytes per wave

__device__ inline uint32_t put_index_entry(uint8_t* d, uint32_t klen, uint32_t hlen, const uint8_t* slot,
                                           uint32_t ulen, uint64_t tag, uint64_t boff, uint32_t bsz) {
  uint32_t p = 0;
  d[p++] = 0;
  p += put_varint(d + p, klen);
  p += put_varint(d + p, hlen);
  for (uint32_t i = 0; i < ulen; i++) d[p++] = slot[i];
  for (int i = 0; i < 8; i++) d[p++] = (uint8_t)(tag >> (8 * i));
  p += put_varint(d + p, boff);
  p += put_varint(d + p, bsz);
  return p;
}

__global__ void __launch_bounds__(IW_WAVES * 64) k_index_write(OutBlocks ob, OutFiles of, Tuples tu,
                                                               const uint32_t* surv, const uint64_t* ie_off,
                                                               const uint64_t* nblocks, uint32_t kw8, uint64_t cap,
                                                               uint8_t* out) {
  __shared__ __attribute__((aligned(16))) uint8_t stage_all[IW_WAVES][IW_CAP];
  uint8_t* S = stage_all[threadIdx.x / WAVE];
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = b < cap && b < *nblocks;  // the valid lanes of a wave are a prefix of it
  uint32_t f = 0, klen = 0, hlen = 0, ulen = 0, bsz = 0, len = 0;
  uint64_t b0 = 0, rel = 0, boff = 0, tag = 0;
  uint8_t* base = nullptr;
  const uint8_t* slot = nullptr;
  if (in) {
    f = ob.file[b];
    b0 = of.b0[f];
    rel = ie_off[b] - ie_off[b0];
    base = out + of.out[f] + of.index_off[f];
    const uint32_t e = surv[ob.s0[b] + ob.cnt[b] - 1];
    ulen = tu.ulen[e];
    klen = ulen + 8;
    boff = ob.off[b];
    bsz = ob.size[b];
    hlen = varint_len(boff) + varint_len(bsz);
    slot = (const uint8_t*)(tu.heap + (uint64_t)e * kw8);
    tag = tu.tag[e];
    len = 1 + varint_len(klen) + varint_len(hlen) + klen + hlen;
  }
  const uint64_t act = __ballot(in);
  if (!act) return;
  const int last = 63 - __builtin_clzll(act);
  const uint32_t f0 = (uint32_t)__shfl((int)f, 0, WAVE);
  const uint64_t lo = ((uint64_t)(uint32_t)__shfl((int)(rel >> 32), 0, WAVE) << 32) |
                      (uint32_t)__shfl((int)(uint32_t)rel, 0, WAVE);
  const uint64_t end = rel + len;
  const uint64_t hi = ((uint64_t)(uint32_t)__shfl((int)(end >> 32), last, WAVE) << 32) |
                      (uint32_t)__shfl((int)(uint32_t)end, last, WAVE);
  const uint64_t gb = (uint64_t)(uintptr_t)base;
  const uint64_t gbase = ((uint64_t)(uint32_t)__shfl((int)(gb >> 32), 0, WAVE) << 32) |
                         (uint32_t)__shfl((int)(uint32_t)gb, 0, WAVE);
  const uint64_t dst0 = gbase + lo;
  const uint32_t a = (uint32_t)(dst0 & 15);
  const bool one_file = __ballot(in && f != f0) == 0;
  if (one_file && a + (hi - lo) <= IW_CAP) {
    if (in) put_index_entry(S + a + (rel - lo), klen, hlen, slot, ulen, tag, boff, bsz);
    wave_sync();
    const uint64_t line0 = dst0 - a;  // 16-byte aligned
    const uint32_t nl = (uint32_t)((a + (hi - lo) + 15) / 16);
    for (uint32_t i = lane_id(); i < nl; i += WAVE) {
      uint8_t* g = (uint8_t*)(uintptr_t)(line0 + 16ull * i);
      const uint32_t k0 = 16 * i, k1 = k0 + 16;
      if (k0 >= a && k1 <= a + (uint32_t)(hi - lo)) {
        *(uint4*)g = *(const uint4*)(S + k0);
      } else {
        for (uint32_t k = k0; k < k1; k++)
          if (k >= a && k < a + (uint32_t)(hi - lo)) g[k - k0] = S[k];
      }
    }
    wave_sync();
  } else if (in) {
    put_index_entry(base + rel, klen, hlen, slot, ulen, tag, boff, bsz);
  }
  if (!in) return;
  // restart array slot
  const uint64_t entries = ie_off[b0 + of.nb[f]] - ie_off[b0];
  uint8_t* r = base + entries + 4 * (b - b0);
  for (int k = 0; k < 4; k++) r[k] = (uint8_t)(rel >> (8 * k));
}

__device__ inline void put_fixed32(uint8_t* d, uint32_t v) {
  for (int k = 0; k < 4; k++) d[k] = (uint8_t)(v >> (8 * k));
}

__global__ void k_meta(OutFiles of, const uint64_t* win_off, const uint64_t* nfiles, uint64_t cap, uint8_t* out) {
  const uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= cap || f >= *nfiles) return;
  uint8_t* F = out + of.out[f];
  // filter block tail: array offset, base lg; trailer type byte
  const uint64_t w0 = of.w0[f];
  const uint64_t filters = win_off[w0 + of.nwin[f]] - win_off[w0];
  uint8_t* fb = F + of.filter_off[f];
  put_fixed32(fb + filters + 4 * of.nwin[f], (uint32_t)filters);
  fb[filters + 4 * of.nwin[f] + 4] = FILTER_BASE_LG;
  fb[of.filter_size[f]] = 0;
  // metaindex: one restart entry naming the filter block
  uint8_t* mb = F + of.meta_off[f];
  const char name[] = "filter.luda.bloom.xxh64";
  uint32_t p = 0;
  uint8_t h[20];
  uint32_t hl = put_varint(h, of.filter_off[f]);
  hl += put_varint(h + hl, of.filter_size[f]);
  mb[p++] = 0;
  mb[p++] = 23;
  mb[p++] = (uint8_t)hl;
  for (int i = 0; i < 23; i++) mb[p++] = (uint8_t)name[i];
  for (uint32_t i = 0; i < hl; i++) mb[p++] = h[i];
  put_fixed32(mb + p, 0);
  put_fixed32(mb + p + 4, 1);
  mb[of.meta_size[f]] = 0;
  // index block: restart count and trailer type byte
  uint8_t* ib = F + of.index_off[f];
  put_fixed32(ib + of.index_size[f] - 4, of.nb[f]);
  ib[of.index_size[f]] = 0;
  // footer
  uint8_t* ft = ib + of.index_size[f] + 5;
  uint32_t q = put_varint(ft, of.meta_off[f]);
  q += put_varint(ft + q, of.meta_size[f]);
  q += put_varint(ft + q, of.index_off[f]);
  q += put_varint(ft + q, of.index_size[f]);
  for (; q < 40; q++) ft[q] = 0;
  for (int k = 0; k < 8; k++) ft[40 + k] = (uint8_t)(TABLE_MAGIC >> (8 * k));
}

// filter (kind 0), metaindex (1) and index (2) block of each file: the
// masked CRC goes into the block's trailer
struct FileMsgs {
  OutFiles of;
  const uint64_t* nfiles;
  uint64_t cap;
  uint8_t* out;
  __device__ uint32_t count() const { return 3 * (uint32_t)min(cap, *nfiles); }
  __device__ uint8_t* msg(uint32_t m, uint64_t* n) const {
    const uint32_t f = m / 3, kind = m % 3;
    const uint64_t off = kind == 0 ? of.filter_off[f] : kind == 1 ? of.meta_off[f] : of.index_off[f];
    const uint64_t size = kind == 0 ? of.filter_size[f] : kind == 1 ? of.meta_size[f] : of.index_size[f];
    *n = size + 1;
    return out + of.out[f] + off;
  }
  __device__ void span(uint32_t m, const uint8_t** p, uint64_t* n) const { *p = msg(m, n); }
  __device__ void finish(uint32_t m, uint32_t raw) const {
    uint64_t n;
    uint8_t* p = msg(m, &n);
    put_fixed32(p + n, crc_mask(raw ^ 0xFFFFFFFFu));
  }
  __device__ void empty(uint32_t) const {}
};

void launch_crc_files(OutFiles of, const uint64_t* nfiles, uint64_t cap, uint8_t* out, const uint32_t* g_crc,
                      uint32_t* part, uint64_t* mseg, uint32_t grid, hipStream_t st) {
  launch_crc_msgs(FileMsgs{of, nfiles, cap, out}, 3 * cap, g_crc, part, mseg, grid, st);
}

}  // namespace luda
