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
//   k_crc_ranges   one workgroup of 16 waves per (file, filter | metaindex |
//                  index block)
#include "dev_common.h"
#include "kernels.h"

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
// Staged encoder.  Per wave: [EncWin entry window | stage].  The
// block message (contents || type byte) sits at the end of the stage, which
// is 16-byte aligned, so the chunk grid of the CRC (16-byte chunks aligned to
// the message end) is the aligned grid of the stage.

__global__ void __launch_bounds__(1024) k_encode(EncodeArgs A) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  CrcLds* T = (CrcLds*)smem;
  load_crc_tables(T, A.g_crc, threadIdx.x, blockDim.x);
  __syncthreads();
  const uint32_t wv = threadIdx.x / WAVE, l = lane_id();
  const uint32_t waves = blockDim.x / WAVE;
  uint8_t* wbase = smem + sizeof(CrcLds) + (size_t)wv * A.wave_lds;
  EncWin* W = (EncWin*)wbase;
  uint8_t* stage_end = wbase + A.wave_lds;
  const uint64_t nb = *A.nblocks;
  const uint64_t stride = (uint64_t)gridDim.x * waves;
  // the next block's record and its first window of entry records are
  // loaded while the current block is stored and checksummed
  uint64_t b = (uint64_t)blockIdx.x * waves + wv;
  BlockRec Bn;
  EncRec rn;
  uint32_t stn = 0;
  if (b < nb) {
    Bn = A.blk[b];
    if (l < min(Bn.cnt, ENC_SW)) {
      rn = A.rec[Bn.s0 + l];
      stn = A.ent_off[Bn.s0 + l];
    }
  }
  for (; b < nb; b += stride) {
    const BlockRec B = Bn;
    const EncRec r0 = rn;
    const uint32_t st0 = stn;
    const uint32_t R = B.R, cnt = B.cnt, size = B.size;
    const uint64_t s0 = B.s0;
    const uint32_t nrest = (cnt + R - 1) / R;
    const uint32_t data_end = size - 4 * nrest - 4;
    const uint32_t n = size + 1;
    uint8_t* dst = A.out + B.dst;
    const uint32_t* blk_off = A.ent_off + s0;
    const uint32_t J16 = (n + 15) / 16;
    uint8_t* base = stage_end - n;         // message byte p at base[p]
    const uint32_t gshift = 16 * J16 - n;  // chunk grid: positions 16 m - gshift
    // --- entries, a window at a time: one lane per entry lays out its
    // entry, then all lanes write the header, key delta and value-edge bytes
    // (byte tasks) and copy the whole aligned chunks of the values
    for (uint32_t k0 = 0; k0 < cnt; k0 += ENC_SW) {
      const uint32_t nw = min(cnt - k0, ENC_SW);
      uint32_t tasks = 0, pieces = 0;
      if (l < nw) {
        const uint32_t i = k0 + l;
        const EncRec r = k0 ? A.rec[s0 + i] : r0;
        const uint32_t st = k0 ? blk_off[i] : st0;
        const uint32_t shared = (i % R == 0) ? 0u : r.shared;
        const uint32_t ns = r.ulen + 8 - shared;
        uint32_t la, lb, lc;
        const uint64_t va = pack_varint(shared, &la), vb = pack_varint(ns, &lb), vc = pack_varint(r.vlen, &lc);
        const u128 H = (u128)va | ((u128)vb << (8 * la)) | ((u128)vc << (8 * (la + lb)));
        const uint32_t hl = la + lb + lc;
        const uint32_t vs = st + hl + ns, en = vs + r.vlen;
        // a: first grid position >= vs; z: last grid position <= en (it can
        // lie before the message start, hence signed)
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
        W->h0[l] = (uint64_t)H;
        W->h1[l] = (uint64_t)(H >> 64);
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
        if (i % R == 0) {  // restart slot of this entry
          uint8_t* d = base + data_end + 4 * (i / R);
          d[0] = (uint8_t)st;
          d[1] = (uint8_t)(st >> 8);
          d[2] = (uint8_t)(st >> 16);
          d[3] = (uint8_t)(st >> 24);
        }
      }
      const uint32_t ti = wave_incl_scan(tasks), pi = wave_incl_scan(pieces);
      if (l < nw) {
        W->pb[l] = ti - tasks;
        W->pc[l] = pi - pieces;
      }
      const uint32_t ntasks = __shfl(ti, WAVE - 1, WAVE), npieces = __shfl(pi, WAVE - 1, WAVE);
      if (l == 0) {
        W->pb[nw] = ntasks;
        W->pc[nw] = npieces;
      }
      wave_sync();
      // whole aligned chunks of the values, the first ENC_B per lane in flight
      // with the byte tasks below
      uint4 v[ENC_B];
#pragma unroll
      for (uint32_t t = 0; t < ENC_B; t++) {
        const uint32_t k = l + WAVE * t;
        if (k >= npieces) continue;
        uint32_t lo = 0, hi = nw;  // pc[lo] <= k < pc[hi]
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (W->pc[mid] <= k) lo = mid;
          else hi = mid;
        }
        const uint32_t pos = W->a[lo] + 16 * (k - W->pc[lo]);
        v[t] = ldg16(W->vp[lo] + (pos - W->vs[lo]));
      }
      // byte tasks, ENC_T per lane at a time: the sources of a batch are
      // worked out first so that its global loads are in flight together
      for (uint32_t kb = 0; kb < ntasks; kb += WAVE * ENC_T) {
        uint32_t byte[ENC_T], d[ENC_T];
        uint64_t src[ENC_T];
#pragma unroll
        for (uint32_t t = 0; t < ENC_T; t++) {
          const uint32_t k = kb + l + WAVE * t;
          src[t] = 0;
          byte[t] = 0;
          d[t] = ~0u;
          if (k >= ntasks) continue;
          uint32_t lo = 0, hi = nw;  // pb[lo] <= k < pb[hi]
          while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (W->pb[mid] <= k) lo = mid;
            else hi = mid;
          }
          uint32_t o = k - W->pb[lo];
          const uint32_t hl = W->hl[lo], ns = W->ns[lo];
          if (o < hl) {
            byte[t] = (uint32_t)((o < 8 ? W->h0[lo] >> (8 * o) : W->h1[lo] >> (8 * (o - 8))) & 0xFFu);
            d[t] = W->st[lo] + o;
          } else if (o < hl + ns) {
            const uint32_t q = W->sh[lo] + (o - hl), ul = W->ul[lo];
            if (q < ul) src[t] = (uint64_t)(uintptr_t)A.tu.heap + (uint64_t)W->e[lo] * A.kw8 * 8 + q;
            else byte[t] = (uint32_t)(W->tag[lo] >> (8 * (q - ul))) & 0xFFu;
            d[t] = W->st[lo] + o;
          } else {
            o -= hl + ns;
            const uint32_t hn = W->hn[lo], vs = W->vs[lo];
            const uint32_t off = (o < hn) ? o : (W->tb[lo] - vs) + (o - hn);
            src[t] = W->vp[lo] + off;
            d[t] = vs + off;
          }
        }
#pragma unroll
        for (uint32_t t = 0; t < ENC_T; t++)
          if (src[t]) byte[t] = ldg_u8(src[t]);
#pragma unroll
        for (uint32_t t = 0; t < ENC_T; t++)
          if (d[t] != ~0u) base[d[t]] = (uint8_t)byte[t];
      }
#pragma unroll
      for (uint32_t t = 0; t < ENC_B; t++) {
        const uint32_t k = l + WAVE * t;
        if (k >= npieces) continue;
        uint32_t lo = 0, hi = nw;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (W->pc[mid] <= k) lo = mid;
          else hi = mid;
        }
        *(uint4*)(base + W->a[lo] + 16 * (k - W->pc[lo])) = v[t];
      }
      // remaining whole chunks of long values, ENC_B per lane at a time
      for (uint32_t kb = WAVE * ENC_B; kb < npieces; kb += WAVE * ENC_B) {
        uint32_t pos[ENC_B];
#pragma unroll
        for (uint32_t t = 0; t < ENC_B; t++) {
          const uint32_t k = kb + l + WAVE * t;
          pos[t] = ~0u;
          if (k >= npieces) continue;
          uint32_t lo = 0, hi = nw;
          while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (W->pc[mid] <= k) lo = mid;
            else hi = mid;
          }
          pos[t] = W->a[lo] + 16 * (k - W->pc[lo]);
          v[t] = ldg16(W->vp[lo] + (pos[t] - W->vs[lo]));
        }
#pragma unroll
        for (uint32_t t = 0; t < ENC_B; t++)
          if (pos[t] != ~0u) *(uint4*)(base + pos[t]) = v[t];
      }
      wave_sync();
    }
    // --- restart count, type byte
    if (l == 0) {
      uint8_t* d = base + size - 4;
      d[0] = (uint8_t)nrest;
      d[1] = (uint8_t)(nrest >> 8);
      d[2] = (uint8_t)(nrest >> 16);
      d[3] = (uint8_t)(nrest >> 24);
      d[4] = 0;
    }
    wave_sync();
    // next block's records (in flight during the store and checksum)
    if (b + stride < nb) {
      Bn = A.blk[b + stride];
      if (l < min(Bn.cnt, ENC_SW)) {
        rn = A.rec[Bn.s0 + l];
        stn = A.ent_off[Bn.s0 + l];
      }
    }
    // --- store and checksum: lane l takes the chunks c = 63 - l + 64 i,
    // first to last; only a lane's first chunk can reach below message
    // position 4
    uint32_t acc = 0;
    const int64_t c_first = 63 - (int64_t)l;
    int64_t c = c_first < (int64_t)J16 ? c_first + 64 * (((int64_t)J16 - 1 - c_first) / 64) : -1;
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
    if (l == 0) {
      const uint32_t m = crc_mask(raw ^ 0xFFFFFFFFu);
      __builtin_memcpy(dst + n, &m, 4);
    }
    wave_sync();
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

// CRC of filter (kind 0), metaindex (1) and index (2) blocks of each file:
// one workgroup of 16 waves per block
__global__ void __launch_bounds__(1024) k_crc_ranges(OutFiles of, const uint64_t* nfiles, uint64_t cap, uint8_t* out,
                                                     const uint32_t* g_crc) {
  __shared__ CrcLds T;
  __shared__ uint32_t part[16];
  const uint64_t f = blockIdx.x / 3;
  const uint32_t kind = blockIdx.x % 3;
  if (f >= cap || f >= *nfiles) return;
  load_crc_tables(&T, g_crc, threadIdx.x, blockDim.x);
  __syncthreads();
  uint64_t off, size;
  if (kind == 0) {
    off = of.filter_off[f];
    size = of.filter_size[f];
  } else if (kind == 1) {
    off = of.meta_off[f];
    size = of.meta_size[f];
  } else {
    off = of.index_off[f];
    size = of.index_size[f];
  }
  uint8_t* msg = out + of.out[f] + off;
  const uint64_t n = size + 1;
  const uint32_t raw = wg16_raw_crc(&T, msg, n, part);
  if (threadIdx.x == 0) put_fixed32(msg + n, crc_mask(raw ^ 0xFFFFFFFFu));
}

}  // namespace luda
