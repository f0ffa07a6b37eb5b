// Phase 3 "Pack" writers (paper Sec. II-A Phase 3; Sec. III-C: encode fills
// data blocks and checksums them with no data exchange between blocks, filter
// builds each table's Bloom filter block).  Values move once: from the input
// table bytes straight into the output block (the paper's lazy value
// movement, Sec. III-D, without the intermediate pair buffer).
//
//   k_encode       one wave per output data block: assembles the block in an
//                  LDS stage (value interiors as aligned 16-byte copies,
//                  headers, keys, value edges and the tail as bytes), then
//                  stores it in 16-byte chunks aligned to the block end and
//                  folds each chunk into the block's CRC in registers
//   k_encode_gen   the same bytes for blocks too large for the stage: every
//                  64-byte unit is generated in registers from the entry
//                  records
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

// One 16-byte chunk of block message bytes [p0, p0 + 16) (positions < 0 give
// zeros) assembled from segments: each overlapping entry's header, key delta
// and value, then restart offsets, the restart count and the type byte (0).
// i is the window entry holding position max(p0, 0) when that lies in the
// entry area.
__device__ uint4 enc_chunk_slow(const EncLds* L, uint32_t nw, uint32_t i, int64_t p0, uint32_t data_end,
                                uint32_t size, uint32_t nrest, uint32_t R, const uint32_t* blk_off,
                                const uint64_t* heap, uint32_t kw8) {
  u128 acc = 0;
  const int64_t pend = p0 + 16;
  for (; i < nw; i++) {
    const int64_t st = L->st[i];
    if (st >= pend || st >= (int64_t)data_end) break;
    const int64_t en = L->st[i + 1], vs = L->vs[i];
    const uint32_t sh = L->sh[i], ul = L->ul[i];
    const uint32_t ns = ul + 8 - sh;
    const int64_t ks = vs - ns;
    const Ov h = overlap(p0, st, ks);
    if (h.n) {
      uint32_t la, lb, lc;
      const uint64_t va = pack_varint(sh, &la), vb = pack_varint(ns, &lb), vc = pack_varint((uint32_t)(en - vs), &lc);
      const u128 H = (u128)va | ((u128)vb << (8 * la)) | ((u128)vc << (8 * (la + lb)));
      acc |= shl_bytes(keep_bytes(shr_bytes(H, h.o), h.n), h.d);
    }
    const Ov k = overlap(p0, ks, vs);
    if (k.n) acc |= shl_bytes(ikey_span(heap + (uint64_t)L->e[i] * kw8, kw8, ul, L->tag[i], sh + k.o, k.n), k.d);
    const Ov v = overlap(p0, vs, en);
    if (v.n) acc |= shl_bytes(load_span((const uint8_t*)L->vp[i] + v.o, v.n), v.d);
  }
  if (pend > (int64_t)data_end) {
    const int64_t rs = data_end;
    const int64_t from = max(p0, rs);
    const uint32_t r0 = (uint32_t)((from - rs) >> 2);
    for (uint32_t r = r0; r < nrest; r++) {
      const int64_t a = rs + 4ll * r;
      if (a >= pend) break;
      const Ov o = overlap(p0, a, a + 4);
      if (o.n) acc |= shl_bytes(keep_bytes((u128)(blk_off[(uint64_t)r * R] >> (8 * o.o)), o.n), o.d);
    }
    const int64_t a = (int64_t)size - 4;
    const Ov o = overlap(p0, a, a + 4);
    if (o.n) acc |= shl_bytes(keep_bytes((u128)(nrest >> (8 * o.o)), o.n), o.d);
  }
  uint4 v;
  v.x = (uint32_t)acc;
  v.y = (uint32_t)(acc >> 32);
  v.z = (uint32_t)(acc >> 64);
  v.w = (uint32_t)(acc >> 96);
  return v;
}

// One wave per output data block.  The block's message (contents || type
// byte) is produced as 16-byte chunks aligned to its end; lane l produces the
// chunks c = 63 - l + 64 i (c counted from the end) in increasing position,
// stores each and folds it into its CRC register (Horner with a shift by
// 1024 bytes), and the wave joins the 64 registers at the end.  Entry
// metadata is staged in LDS ENC_W entries at a time; a window after the first
// starts 8 entries before the previous one ended, so a chunk assigned to a
// window (by its first byte) never reaches past the window's entries (an
// entry is at least 4 bytes).
constexpr uint32_t ENC_B = 4;  // whole value chunks per lane in flight together
constexpr uint32_t ENC_T = 4;  // byte tasks per lane in flight together

constexpr uint32_t ENC_OVERLAP = 16;  // entries shared by consecutive windows (>= 64 bytes)
constexpr uint32_t GEN_UNIT = 64;     // bytes a lane folds per step in k_encode_gen

__global__ void __launch_bounds__(512) k_encode_gen(EncodeArgs A) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  CrcLds* T = (CrcLds*)smem;
  load_crc_tables(T, A.g_crc, threadIdx.x, blockDim.x);
  __syncthreads();
  const uint32_t wv = threadIdx.x / WAVE, l = lane_id();
  const uint32_t waves = blockDim.x / WAVE;
  EncLds* L = (EncLds*)(smem + sizeof(CrcLds)) + wv;
  // a lane folds 64-byte units (four chunks in sequence); units are joined
  // by multiplications with x^(8 m) mod P for m = 4096 (between a lane's
  // units) and 64 * 2^k (lanes)
  uint32_t kj[7];
#pragma unroll
  for (int k = 0; k < 7; k++) kj[k] = gf2_xpow8n((uint64_t)GEN_UNIT << k);
  const uint64_t nb = *A.nblocks;
  for (uint64_t b = (uint64_t)blockIdx.x * waves + wv; b < nb; b += (uint64_t)gridDim.x * waves) {
    const BlockRec B = A.blk[b];
    const uint32_t R = B.R, cnt = B.cnt, size = B.size;
    const uint64_t s0 = B.s0;
    const uint32_t nrest = (cnt + R - 1) / R;
    const uint32_t data_end = size - 4 * nrest - 4;
    const int64_t n = (int64_t)size + 1;
    uint8_t* dst = A.out + B.dst;
    const uint32_t* blk_off = A.ent_off + s0;
    const int64_t JU = (n + GEN_UNIT - 1) / GEN_UNIT;
    const int64_t u_first = 63 - (int64_t)l;
    int64_t uu = u_first < JU ? u_first + 64 * ((JU - 1 - u_first) / 64) : -1;
    uint32_t acc = 0;
    uint32_t k0 = 0;
    for (;;) {
      const uint32_t k1 = min(cnt, k0 + ENC_W);
      const uint32_t nw = k1 - k0;
      const bool last = (k1 == cnt);
      if (l < nw) {
        const uint32_t i = k0 + l;
        const EncRec r = A.rec[s0 + i];
        const uint32_t shared = (i % R == 0) ? 0u : r.shared;
        const uint32_t st = blk_off[i];
        const uint32_t ns = r.ulen + 8 - shared;
        L->st[l] = st;
        L->vs[l] = st + vlen32(shared) + vlen32(ns) + vlen32(r.vlen) + ns;
        L->e[l] = r.e;
        L->sh[l] = shared;
        L->ul[l] = r.ulen;
        L->vp[l] = r.vp;
        L->tag[l] = r.tag;
      }
      if (l == 0) L->st[nw] = last ? data_end : blk_off[k1];
      wave_sync();
      // units assigned to this window by their first byte; a unit never
      // reaches past the window's entries (the next window starts
      // ENC_OVERLAP entries, at least 64 bytes, earlier)
      const int64_t hi = last ? n : (int64_t)L->st[nw - ENC_OVERLAP];
      uint32_t cur = 0;
      while (uu >= 0) {
        const int64_t p = n - (int64_t)GEN_UNIT * (uu + 1);
        if ((p < 0 ? 0 : p) >= hi) break;
        uint4 v[4];
        uint32_t slow = 0;
#pragma unroll
        for (uint32_t q = 0; q < 4; q++) {
          const int64_t p0 = p + 16 * q;
          v[q] = make_uint4(0, 0, 0, 0);
          if (p0 + 16 <= 0) continue;
          const int64_t P = p0 < 0 ? 0 : p0;
          // entry holding P: the last with st <= P (from the lane's cursor)
          uint32_t lo_i = cur, hi_i = nw;
          while (hi_i - lo_i > 1) {
            const uint32_t mid = (lo_i + hi_i) >> 1;
            if ((int64_t)L->st[mid] <= P) lo_i = mid;
            else hi_i = mid;
          }
          cur = lo_i;
          const int64_t vs = L->vs[cur];
          if (p0 >= vs && p0 + 16 <= (int64_t)L->st[cur + 1]) v[q] = ldg16(L->vp[cur] + (uint64_t)(p0 - vs));
          else slow |= 1u << q;
        }
        // chunks that cross a segment boundary, one at a time
        while (slow) {
          const uint32_t q = __builtin_ctz(slow);
          slow &= slow - 1;
          const int64_t p0 = p + 16 * q;
          const int64_t P = p0 < 0 ? 0 : p0;
          uint32_t lo_i = 0, hi_i = nw;
          while (hi_i - lo_i > 1) {
            const uint32_t mid = (lo_i + hi_i) >> 1;
            if ((int64_t)L->st[mid] <= P) lo_i = mid;
            else hi_i = mid;
          }
          const uint4 r = enc_chunk_slow(L, nw, lo_i, p0, data_end, (uint32_t)size, nrest, R, blk_off, A.tu.heap, A.kw8);
#pragma unroll
          for (uint32_t u = 0; u < 4; u++)
            if (u == q) v[u] = r;
        }
#pragma unroll
        for (uint32_t q = 0; q < 4; q++) {
          const int64_t p0 = p + 16 * q;
          if (p0 >= 0) {
            __builtin_memcpy(dst + p0, &v[q], 16);
          } else if (p0 + 16 > 0) {
            const uint8_t* vb = (const uint8_t*)&v[q];
            for (int k = 0; k < 16; k++)
              if (p0 + k >= 0) dst[p0 + k] = vb[k];
          }
        }
        uint32_t ur = 0;
#pragma unroll
        for (uint32_t q = 0; q < 4; q++) ur = crc_chunk_from(T, ur, v[q], p + 16 * q);
        acc = gf2_mulmod(acc, kj[6]) ^ ur;
        uu -= 64;
      }
      wave_sync();
      if (last) break;
      k0 = k1 - ENC_OVERLAP;
    }
#pragma unroll
    for (int k = 0; k < 6; k++) {
      uint32_t other = __shfl_down(acc, 1u << k, WAVE);
      if (l + (1u << k) >= WAVE) other = 0;
      acc = gf2_mulmod(acc, kj[k]) ^ other;
    }
    if (l == 0) {
      const uint32_t m = crc_mask(acc ^ 0xFFFFFFFFu);
      __builtin_memcpy(dst + n, &m, 4);
    }
  }
}

// ---------------------------------------------------------------------------
// Staged encoder.  Per wave: [EncWin entry window | stage].  The block
// message (contents || type byte) sits at the end of the stage, which is
// 16-byte aligned, so the chunk grid of the CRC (16-byte chunks aligned to the
// message end) is the aligned grid of the stage.
//
// Blocks are software-pipelined: while block X is stored and checksummed
// from registers, the loads that fill block X+1 (its first window of value
// chunks and bytes) are in flight, its entry records were loaded one block
// ahead and its handle two blocks ahead.  Every global load and store of the
// common path is issued by every lane (a lane with nothing to load reads a
// fixed valid address; stores go through a buffer descriptor of the block,
// and a lane with nothing to store uses an offset past its end, which the
// hardware drops), so each wait is for exactly the loads it needs.

constexpr uint32_t ENC_QS = 5;           // chunks per lane held in registers: blocks up to 5 KiB pipelined
constexpr uint32_t ENC_OOB = 0x80000000u;  // a buffer offset past any block

struct EncH {  // one block, the same in every lane
  uint64_t dst, s0;
  uint32_t cnt, size, R;
  bool valid;
};

__device__ __forceinline__ EncH enc_handle(const EncodeArgs& A, uint64_t b, uint64_t nb) {
  const BlockRec r = A.blk[b < nb ? b : nb - 1];  // nb > 0
  EncH h;
  h.dst = r.dst;
  h.s0 = r.s0;
  h.cnt = r.cnt;
  h.size = r.size;
  h.R = r.R;
  h.valid = b < nb;
  return h;
}

struct EncE {  // this lane's entry of a window
  EncRec r;
  uint32_t st;
};

// entry k0 + l of block H (lanes past the block's end read its last entry)
__device__ __forceinline__ EncE enc_entry(const EncodeArgs& A, const EncH& H, uint32_t k0) {
  const uint32_t i = min(k0 + lane_id(), H.cnt - 1);  // cnt >= 1
  EncE e;
  e.r = A.rec[H.s0 + i];
  e.st = A.ent_off[H.s0 + i];
  return e;
}

struct EncL {
  uint32_t nw, ntasks, npieces;
  uint32_t rs;  // restart slot of this lane's entry: its index + 1, or 0
  uint32_t st;
};

// lays out entries k0 .. k0 + nw - 1 (lane l: entry k0 + l) into the window
__device__ __forceinline__ EncL enc_layout(EncWin* W, const EncH& H, uint32_t k0, const EncE& E, uint32_t gshift) {
  const uint32_t l = lane_id();
  EncL L;
  L.nw = min(H.cnt - k0, ENC_SW);
  L.rs = 0;
  L.st = E.st;
  uint32_t tasks = 0, pieces = 0;
  if (l < L.nw) {
    const uint32_t i = k0 + l;
    const EncRec& r = E.r;
    const uint32_t st = E.st;
    const uint32_t shared = (i % H.R == 0) ? 0u : r.shared;
    const uint32_t ns = r.ulen + 8 - shared;
    uint32_t la, lb, lc;
    const uint64_t va = pack_varint(shared, &la), vb = pack_varint(ns, &lb), vc = pack_varint(r.vlen, &lc);
    const u128 Hd = (u128)va | ((u128)vb << (8 * la)) | ((u128)vc << (8 * (la + lb)));
    const uint32_t hl = la + lb + lc;
    const uint32_t vs = st + hl + ns, en = vs + r.vlen;
    // a: first grid position >= vs; z: last grid position <= en (it can lie
    // before the message start, hence signed)
    const uint32_t a = vs + ((16u - ((vs + gshift) & 15u)) & 15u);
    const int64_t z = (int64_t)en - (int64_t)((en + gshift) & 15u);
    uint32_t h_end = en, t_beg = en;
    if ((int64_t)a + 16 <= z) {
      pieces = (uint32_t)((z - (int64_t)a) / 16);
      h_end = a;
      t_beg = (uint32_t)z;
    }
    W->vp[l] = r.vp;
    W->tag[l] = r.tag;
    W->h0[l] = (uint64_t)Hd;
    W->h1[l] = (uint64_t)(Hd >> 64);
    W->st[l] = st;
    W->hl[l] = hl;
    W->ns[l] = ns;
    W->sh[l] = shared;
    W->ul[l] = r.ulen;
    W->e[l] = r.e;
    W->vs[l] = vs;
    W->a[l] = a;
    W->hn[l] = h_end - vs;
    W->tb[l] = t_beg;
    tasks = hl + ns + (h_end - vs) + (en - t_beg);
    if (i % H.R == 0) L.rs = i / H.R + 1;
  }
  const uint32_t ti = wave_incl_scan(tasks), pi = wave_incl_scan(pieces);
  if (l < L.nw) {
    W->pb[l] = ti - tasks;
    W->pc[l] = pi - pieces;
  }
  L.ntasks = __shfl(ti, WAVE - 1, WAVE);
  L.npieces = __shfl(pi, WAVE - 1, WAVE);
  if (l == 0) {
    W->pb[L.nw] = L.ntasks;
    W->pc[L.nw] = L.npieces;
  }
  wave_sync();
  return L;
}

// one batch of a window's stage writes, loaded into registers: whole aligned
// value chunks kp0 + l + 64 t and byte tasks kt0 + l + 64 t
struct EncIss {
  uint4 v[ENC_B];
  uint32_t pos[ENC_B];  // stage position of the chunk, ~0: none
  uint32_t bl[ENC_T];   // loaded byte
  uint32_t bd[ENC_T];   // stage position of the byte | its value << 20 (0x100: the loaded one); ~0: none
};
constexpr uint32_t ENC_LOADED = 0x100u << 20;

__device__ __forceinline__ uint32_t win_find(const uint32_t* off, uint32_t nw, uint32_t k) {
  uint32_t lo = 0, hi = nw;  // off[lo] <= k < off[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= k) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void enc_issue(const EncWin* W, const EncodeArgs& A, const EncL& L, uint32_t kp0,
                                          uint32_t kt0, uint64_t safe, EncIss& I) {
  const uint32_t l = lane_id();
#pragma unroll
  for (uint32_t t = 0; t < ENC_B; t++) {
    const uint32_t k = kp0 + l + WAVE * t;
    uint64_t src = safe;
    I.pos[t] = ~0u;
    if (k < L.npieces) {
      const uint32_t lo = win_find(W->pc, L.nw, k);
      I.pos[t] = W->a[lo] + 16 * (k - W->pc[lo]);
      src = W->vp[lo] + (I.pos[t] - W->vs[lo]);
    }
    I.v[t] = ldg16(src);
  }
#pragma unroll
  for (uint32_t t = 0; t < ENC_T; t++) {
    const uint32_t k = kt0 + l + WAVE * t;
    uint64_t src = safe;
    I.bd[t] = ~0u;
    if (k < L.ntasks) {
      const uint32_t lo = win_find(W->pb, L.nw, k);
      uint32_t o = k - W->pb[lo];
      const uint32_t hl = W->hl[lo], ns = W->ns[lo];
      if (o < hl) {
        const uint32_t v = (uint32_t)((o < 8 ? W->h0[lo] >> (8 * o) : W->h1[lo] >> (8 * (o - 8))) & 0xFFu);
        I.bd[t] = (W->st[lo] + o) | (v << 20);
      } else if (o < hl + ns) {
        const uint32_t q = W->sh[lo] + (o - hl), ul = W->ul[lo];
        uint32_t v = ENC_LOADED;
        if (q < ul) src = (uint64_t)(uintptr_t)A.tu.heap + (uint64_t)W->e[lo] * A.kw8 * 8 + q;
        else v = ((uint32_t)(W->tag[lo] >> (8 * (q - ul))) & 0xFFu) << 20;
        I.bd[t] = (W->st[lo] + o) | v;
      } else {
        o -= hl + ns;
        const uint32_t hn = W->hn[lo], vs = W->vs[lo];
        const uint32_t off = (o < hn) ? o : (W->tb[lo] - vs) + (o - hn);
        src = W->vp[lo] + off;
        I.bd[t] = (vs + off) | ENC_LOADED;
      }
    }
    I.bl[t] = ldg_u8(src);
  }
}

__device__ __forceinline__ void enc_put(uint8_t* base, const EncIss& I) {
#pragma unroll
  for (uint32_t t = 0; t < ENC_T; t++)
    if (I.bd[t] != ~0u) base[I.bd[t] & 0xFFFFFu] = (uint8_t)(I.bd[t] >> 20 == 0x100u ? I.bl[t] : I.bd[t] >> 20);
#pragma unroll
  for (uint32_t t = 0; t < ENC_B; t++)
    if (I.pos[t] != ~0u) *(uint4*)(base + I.pos[t]) = I.v[t];
}

__device__ __forceinline__ void put_u32(uint8_t* d, uint32_t v) {
  d[0] = (uint8_t)v;
  d[1] = (uint8_t)(v >> 8);
  d[2] = (uint8_t)(v >> 16);
  d[3] = (uint8_t)(v >> 24);
}

struct EncG {  // the stage geometry of a block
  uint32_t n, J16, gshift, nrest, data_end;
  uint8_t* base;  // message byte p at base[p]
};

__device__ __forceinline__ EncG enc_geom(const EncH& H, uint8_t* stage_end) {
  EncG g;
  g.n = H.size + 1;
  g.J16 = (g.n + 15) / 16;
  g.gshift = 16 * g.J16 - g.n;
  g.nrest = (H.cnt + H.R - 1) / H.R;
  g.data_end = H.size - 4 * g.nrest - 4;
  g.base = stage_end - g.n;
  return g;
}

// writes the rest of block H into the stage once its first batch I (of the
// first window, laid out as L) has arrived: the first batch, the remaining
// batches and windows, the restart array, restart count and type byte
__device__ __forceinline__ void enc_commit(EncWin* W, const EncodeArgs& A, const EncH& H, const EncG& g,
                                           const EncL& L0, const EncIss& I0, uint64_t safe) {
  const uint32_t l = lane_id();
  enc_put(g.base, I0);
  if (L0.rs) put_u32(g.base + g.data_end + 4 * (L0.rs - 1), L0.st);
  EncL L = L0;
  uint32_t kp = WAVE * ENC_B, kt = WAVE * ENC_T;
  for (uint32_t k0 = 0;;) {
    while (kp < L.npieces || kt < L.ntasks) {
      EncIss I;
      enc_issue(W, A, L, kp, kt, safe, I);
      enc_put(g.base, I);
      kp += WAVE * ENC_B;
      kt += WAVE * ENC_T;
    }
    k0 += ENC_SW;
    if (k0 >= H.cnt) break;
    wave_sync();
    const EncE E = enc_entry(A, H, k0);
    L = enc_layout(W, H, k0, E, g.gshift);
    if (L.rs) put_u32(g.base + g.data_end + 4 * (L.rs - 1), L.st);
    kp = 0;
    kt = 0;
  }
  if (l == 0) {
    put_u32(g.base + H.size - 4, g.nrest);
    g.base[H.size] = 0;
  }
  wave_sync();
}

__device__ __forceinline__ u128 u4_to_u128(uint4 v) {
  return ((u128)(((uint64_t)v.w << 32) | v.z) << 64) | (((uint64_t)v.y << 32) | v.x);
}
__device__ __forceinline__ uint4 u128_to_u4(u128 x) {
  return make_uint4((uint32_t)x, (uint32_t)(x >> 32), (uint32_t)(x >> 64), (uint32_t)(x >> 96));
}

// block message in the stage -> output bytes and masked CRC, any size: lane l
// takes the chunks c = 63 - l + 64 i, first to last; only a lane's first
// chunk can reach below message position 4
__device__ __forceinline__ void enc_store_loop(const CrcLds* T, const EncH& H, const EncG& g, uint8_t* stage_end,
                                               uint8_t* dst) {
  const uint32_t n = g.n;
  uint32_t acc = 0;
  const int64_t c_first = 63 - (int64_t)lane_id();
  int64_t c = c_first < (int64_t)g.J16 ? c_first + 64 * (((int64_t)g.J16 - 1 - c_first) / 64) : -1;
  if (c >= 0 && (int64_t)n - 16 * (c + 1) < 4) {
    const int64_t p0 = (int64_t)n - 16 * (c + 1);
    const uint4 v = *(const uint4*)(stage_end - 16 * (c + 1));
    if (p0 >= 0) {
      __builtin_memcpy(dst + p0, &v, 16);
    } else {
      const uint8_t* vb = (const uint8_t*)&v;
      for (int k = 0; k < 16; k++)
        if (p0 + k >= 0) dst[p0 + k] = vb[k];
    }
    acc = crc_chunk(T, v, p0);
    c -= 64;
  }
  for (; c >= 0; c -= 64) {
    const uint32_t p0 = n - 16 * (uint32_t)(c + 1);
    const uint4 v = *(const uint4*)(stage_end - 16 * (c + 1));
    __builtin_memcpy(dst + p0, &v, 16);
    acc = crc_shift(T->sh[6], acc) ^ crc_chunk_plain(T, v);
  }
  const uint32_t raw = crc_wave_join(T, acc);
  if (lane_id() == 0) {
    const uint32_t m = crc_mask(raw ^ 0xFFFFFFFFu);
    __builtin_memcpy(dst + n, &m, 4);
  }
}

__global__ void __launch_bounds__(1024) k_encode(EncodeArgs A) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  CrcLds* T = (CrcLds*)smem;
  load_crc_tables(T, A.g_crc, threadIdx.x, blockDim.x);
  __syncthreads();
  const uint64_t nb = *A.nblocks;
  if (nb == 0) return;
  // the wave index is the same in every lane: block handles are scalar loads
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), l = lane_id();
  const uint32_t waves = blockDim.x / WAVE;
  uint8_t* wbase = smem + sizeof(CrcLds) + (size_t)wv * A.wave_lds;
  EncWin* W = (EncWin*)wbase;
  uint8_t* stage_end = wbase + A.wave_lds;
  const uint64_t stride = (uint64_t)gridDim.x * waves;
  const uint64_t safe = (uint64_t)(uintptr_t)A.g_crc;
  uint64_t b = (uint64_t)blockIdx.x * waves + wv;
  if (b >= nb) return;
  // prologue: block b staged, the next block's handle and first records
  EncH H = enc_handle(A, b, nb), Hn = enc_handle(A, b + stride, nb);
  {
    const EncG g = enc_geom(H, stage_end);
    const EncE E = enc_entry(A, H, 0);
    const EncL L = enc_layout(W, H, 0, E, g.gshift);
    EncIss I;
    enc_issue(W, A, L, 0, 0, safe, I);
    enc_commit(W, A, H, g, L, I, safe);
  }
  EncE En = enc_entry(A, Hn, 0);
  for (; b < nb; b += stride) {
    const EncH Hnn = enc_handle(A, b + 2 * stride, nb);
    const EncG g = enc_geom(H, stage_end);
    uint8_t* dst = A.out + H.dst;
    const bool piped = g.J16 <= 64 * ENC_QS && g.n >= 16;
    // the next block: first window laid out, its first batch in flight
    // (the window is free: this block is wholly in the stage)
    const EncG gn = enc_geom(Hn, stage_end);
    EncL Ln;
    EncIss In;
    if (Hn.valid) {
      Ln = enc_layout(W, Hn, 0, En, gn.gshift);
      enc_issue(W, A, Ln, 0, 0, safe, In);
    }
    if (piped) {
      // this block's chunks into registers, then stored and checksummed;
      // every lane issues ENC_QS chunk stores.  A first chunk that starts
      // before the message is stored as message bytes [0, 16) (the bytes past
      // it are the next chunk's)
      const int64_t c_first = 63 - (int64_t)l;
      const int64_t ct = c_first < (int64_t)g.J16 ? c_first + 64 * (((int64_t)g.J16 - 1 - c_first) / 64) : -1;
      const int64_t pt = (int64_t)g.n - 16 * (ct + 1);
      uint4 s[ENC_QS];
#pragma unroll
      for (uint32_t q = 0; q < ENC_QS; q++) {
        const int64_t c = ct - 64 * (int64_t)q;
        s[q] = c >= 0 ? *(const uint4*)(stage_end - 16 * (c + 1)) : make_uint4(0, 0, 0, 0);
      }
      if (ct >= 1 && pt < 0) {
        const uint4 nx = *(const uint4*)(stage_end - 16 * ct);  // chunk ct - 1
        const uint32_t sh = (uint32_t)(-pt);
        s[0] = u128_to_u4((u4_to_u128(s[0]) >> (8 * sh)) | (u4_to_u128(nx) << (8 * (16 - sh))));
      }
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, (int)(g.n + 4), 0x00020000);
      uint32_t acc = 0;
#pragma unroll
      for (uint32_t q = 0; q < ENC_QS; q++) {
        const int64_t c = ct - 64 * (int64_t)q;
        const int64_t p0 = (int64_t)g.n - 16 * (c + 1);
        const u32x4 dv = {s[q].x, s[q].y, s[q].z, s[q].w};
        __builtin_amdgcn_raw_buffer_store_b128(dv, rs, c >= 0 ? (uint32_t)(p0 > 0 ? p0 : 0) : ENC_OOB, 0, 0);
        if (c >= 0) {
          if (q == 0)
            acc = p0 < 4 ? crc_chunk(T, p0 < 0 ? u128_to_u4(u4_to_u128(s[0]) << (8 * (uint32_t)-p0)) : s[0], p0)
                         : crc_chunk_plain(T, s[0]);
          else
            acc = crc_shift(T->sh[6], acc) ^ crc_chunk_plain(T, s[q]);
        }
      }
      const uint32_t raw = crc_wave_join(T, acc);
      __builtin_amdgcn_raw_buffer_store_b32(crc_mask(raw ^ 0xFFFFFFFFu), rs, l == 0 ? g.n : ENC_OOB, 0, 0);
    } else {
      enc_store_loop(T, H, g, stage_end, dst);
    }
    wave_sync();
    // records of the block after next, then the next block completed in the
    // stage once its first batch has arrived
    const EncE Enn = enc_entry(A, Hnn, 0);
    if (Hn.valid) enc_commit(W, A, Hn, gn, Ln, In, safe);
    H = Hn;
    Hn = Hnn;
    En = Enn;
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

__global__ void k_index_write(OutBlocks ob, OutFiles of, Tuples tu, const uint32_t* surv, const uint64_t* ie_off,
                              const uint64_t* nblocks, uint32_t kw8, uint64_t cap, uint8_t* out) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= cap || b >= *nblocks) return;
  const uint32_t f = ob.file[b];
  const uint64_t b0 = of.b0[f];
  const uint64_t rel = ie_off[b] - ie_off[b0];
  uint8_t* base = out + of.out[f] + of.index_off[f];
  uint8_t* d = base + rel;
  const uint32_t e = surv[ob.s0[b] + ob.cnt[b] - 1];
  const uint32_t ulen = tu.ulen[e];
  const uint32_t klen = ulen + 8;
  const uint64_t boff = ob.off[b];
  const uint32_t bsz = ob.size[b];
  const uint32_t hlen = varint_len(boff) + varint_len(bsz);
  uint32_t p = 0;
  d[p++] = 0;
  p += put_varint(d + p, klen);
  p += put_varint(d + p, hlen);
  const uint8_t* slot = (const uint8_t*)(tu.heap + (uint64_t)e * kw8);
  for (uint32_t i = 0; i < ulen; i++) d[p++] = slot[i];
  const uint64_t tag = tu.tag[e];
  for (int i = 0; i < 8; i++) d[p++] = (uint8_t)(tag >> (8 * i));
  p += put_varint(d + p, boff);
  p += put_varint(d + p, bsz);
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

template __global__ void k_crc_multi<FileMsgs>(FileMsgs, const uint32_t*, uint32_t*, uint32_t*);

void launch_crc_files(OutFiles of, const uint64_t* nfiles, uint64_t cap, uint8_t* out, const uint32_t* g_crc,
                      uint32_t* part, uint32_t* ticket, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_crc_multi<FileMsgs>, dim3(grid), dim3(1024), 0, st, FileMsgs{of, nfiles, cap, out}, g_crc,
                     part, ticket);
}

}  // namespace luda
