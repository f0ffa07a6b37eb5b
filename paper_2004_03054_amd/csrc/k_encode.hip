// Phase 3 "Pack" writers (paper Sec. II-A Phase 3; Sec. III-C: encode fills
// data blocks and checksums them with no data exchange between blocks, filter
// builds each table's Bloom filter block).  Values move once: from the input
// table bytes straight into the output block (the paper's lazy value
// movement, Sec. III-D, without the intermediate pair buffer).
//
//   k_encode       one wave per output data block: assembles the block in
//                  16-byte chunks aligned to the block end (entries, restart
//                  array, count, type byte), stores each chunk and folds it
//                  into the block's CRC in registers
//   k_filter       one wave per filter window: Bloom bits in LDS, then stored
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

// byte o of the varint encoding (len bytes) of v
__device__ inline uint32_t varint_byte(uint32_t v, uint32_t o, uint32_t len) {
  return ((v >> (7 * o)) & 0x7Fu) | (o + 1 < len ? 0x80u : 0u);
}

// One 16-byte chunk of block message bytes [p0, p0 + 16) (positions < 0 give
// zeros), built byte by byte.  i is the window entry holding position
// max(p0, 0) when that position lies in the entry area.
__device__ uint4 enc_chunk_slow(const EncLds* L, uint32_t i, int64_t p0, uint32_t data_end, uint32_t size,
                                uint32_t nrest, uint32_t R, const uint32_t* blk_off, const uint64_t* heap,
                                uint32_t kw8) {
  uint32_t st = L->st[i], en = L->st[i + 1], vs = L->vs[i], sh = L->sh[i], ul = L->ul[i];
  uint32_t ns = ul + 8 - sh;
  uint32_t la = vlen32(sh), lb = vlen32(ns), lc = vlen32(en - vs);
  const uint64_t* slot = heap + (uint64_t)L->e[i] * kw8;
  uint64_t tag = L->tag[i];
  const uint8_t* vp = (const uint8_t*)L->vp[i];
  uint64_t lo = 0, hi = 0;
#pragma unroll
  for (int k = 0; k < 16; k++) {
    const int64_t p = p0 + k;
    uint32_t byte = 0;
    if (p >= 0) {
      if (p < (int64_t)data_end) {
        if (p >= (int64_t)en) {
          i++;
          st = L->st[i];
          en = L->st[i + 1];
          vs = L->vs[i];
          sh = L->sh[i];
          ul = L->ul[i];
          ns = ul + 8 - sh;
          la = vlen32(sh);
          lb = vlen32(ns);
          lc = vlen32(en - vs);
          slot = heap + (uint64_t)L->e[i] * kw8;
          tag = L->tag[i];
          vp = (const uint8_t*)L->vp[i];
        }
        const uint32_t pp = (uint32_t)p;
        const uint32_t ks = vs - ns;  // key delta start
        if (pp < ks) {
          uint32_t o = pp - st;
          if (o < la) {
            byte = varint_byte(sh, o, la);
          } else if (o < la + lb) {
            byte = varint_byte(ns, o - la, lb);
          } else {
            byte = varint_byte(en - vs, o - la - lb, lc);
          }
        } else if (pp < vs) {
          const uint32_t q = sh + (pp - ks);
          byte = q < ul ? (uint32_t)(slot[q >> 3] >> (8 * (q & 7))) & 0xFFu : (uint32_t)(tag >> (8 * (q - ul))) & 0xFFu;
        } else {
          byte = vp[pp - vs];
        }
      } else if (p < (int64_t)data_end + 4ll * nrest) {
        const uint32_t q = (uint32_t)p - data_end;
        byte = (blk_off[(uint64_t)(q >> 2) * R] >> (8 * (q & 3))) & 0xFFu;
      } else if (p < (int64_t)size) {
        byte = (nrest >> (8 * ((uint32_t)p - data_end - 4 * nrest))) & 0xFFu;
      }
    }
    if (k < 8) lo |= (uint64_t)byte << (8 * k);
    else hi |= (uint64_t)byte << (8 * (k - 8));
  }
  uint4 v;
  v.x = (uint32_t)lo;
  v.y = (uint32_t)(lo >> 32);
  v.z = (uint32_t)hi;
  v.w = (uint32_t)(hi >> 32);
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
__global__ void __launch_bounds__(512) k_encode(EncodeArgs A) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  CrcLds* T = (CrcLds*)smem;
  load_crc_tables(T, A.g_crc, threadIdx.x, blockDim.x);
  __syncthreads();
  const uint32_t wv = threadIdx.x / WAVE, l = lane_id();
  const uint32_t waves = blockDim.x / WAVE;
  EncLds* L = (EncLds*)(smem + sizeof(CrcLds)) + wv;
  const uint64_t nb = *A.nblocks;
  for (uint64_t b = (uint64_t)blockIdx.x * waves + wv; b < nb; b += (uint64_t)gridDim.x * waves) {
    const uint32_t j = A.ob.job[b];
    const uint32_t R = A.jobs[j].restart_interval;
    const uint64_t s0 = A.ob.s0[b];
    const uint32_t cnt = A.ob.cnt[b];
    const uint32_t size = A.ob.size[b];
    const uint32_t nrest = (cnt + R - 1) / R;
    const uint32_t data_end = size - 4 * nrest - 4;
    const int64_t n = (int64_t)size + 1;
    uint8_t* dst = A.out + A.of.out[A.ob.file[b]] + A.ob.off[b];
    const uint32_t* blk_off = A.ent_off + s0;
    const int64_t J16 = (n + 15) / 16;
    const int64_t c_first = 63 - (int64_t)l;
    int64_t cc = c_first < J16 ? c_first + 64 * ((J16 - 1 - c_first) / 64) : -1;
    uint32_t acc = 0;
    uint32_t k0 = 0;
    for (;;) {
      const uint32_t k1 = min(cnt, k0 + ENC_W);
      const uint32_t nw = k1 - k0;
      const bool last = (k1 == cnt);
      if (l < nw) {
        const uint32_t i = k0 + l;
        const uint64_t s = s0 + i;
        const uint32_t e = A.surv[s];
        const uint32_t shared = (i % R == 0) ? 0u : A.shr[s];
        const uint32_t ul = A.tu.ulen[e];
        const uint32_t vl = A.tu.vlen[e];
        const uint32_t st = blk_off[i];
        const uint32_t ns = ul + 8 - shared;
        L->st[l] = st;
        L->vs[l] = st + vlen32(shared) + vlen32(ns) + vlen32(vl) + ns;
        L->e[l] = e;
        L->sh[l] = shared;
        L->ul[l] = ul;
        L->vp[l] = A.tu.vp[e];
        L->tag[l] = A.tu.tag[e];
      }
      if (l == 0) L->st[nw] = last ? data_end : blk_off[k1];
      wave_sync();
      const int64_t hi = last ? n : (int64_t)L->st[nw - 8];
      uint32_t cur = 0;
      while (cc >= 0) {
        const int64_t p0 = n - 16 * (cc + 1);
        const int64_t P = p0 < 0 ? 0 : p0;
        if (P >= hi) break;
        // entry holding P: the last with st <= P (from the lane's cursor)
        uint32_t lo_i = cur, hi_i = nw;
        while (hi_i - lo_i > 1) {
          const uint32_t mid = (lo_i + hi_i) >> 1;
          if ((int64_t)L->st[mid] <= P) lo_i = mid;
          else hi_i = mid;
        }
        cur = lo_i;
        uint4 v;
        if (p0 >= (int64_t)L->vs[cur] && p0 + 16 <= (int64_t)L->st[cur + 1]) {
          __builtin_memcpy(&v, (const uint8_t*)L->vp[cur] + (p0 - L->vs[cur]), 16);
        } else {
          v = enc_chunk_slow(L, cur, p0, data_end, (uint32_t)size, nrest, R, blk_off, A.tu.heap, A.kw8);
        }
        if (p0 >= 0) {
          __builtin_memcpy(dst + p0, &v, 16);
        } else {
          const uint8_t* vb = (const uint8_t*)&v;
          for (int k = 0; k < 16; k++)
            if (p0 + k >= 0) dst[p0 + k] = vb[k];
        }
        acc = crc_shift(T->sh[6], acc) ^ crc_chunk(T, v, p0);
        cc -= 64;
      }
      wave_sync();
      if (last) break;
      k0 = k1 - 8;
    }
    const uint32_t raw = crc_wave_join(T, acc);
    if (l == 0) {
      const uint32_t m = crc_mask(raw ^ 0xFFFFFFFFu);
      __builtin_memcpy(dst + n, &m, 4);
    }
  }
}

// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_filter(FilterArgs A) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const uint32_t wv = threadIdx.x / WAVE, l = lane_id();
  const uint32_t waves = blockDim.x / WAVE;
  uint32_t* bits = (uint32_t*)(smem + (size_t)wv * A.lds_bytes);
  const uint64_t nw = *A.nwin;
  for (uint64_t w = (uint64_t)blockIdx.x * waves + wv; w < nw; w += (uint64_t)gridDim.x * waves) {
    const uint32_t keys = A.win_keys[w];
    if (!keys) continue;
    const uint32_t f = A.win_file[w];
    const uint32_t bpk = A.jobs[A.of.job[f]].bloom_bits_per_key;
    uint32_t k = bpk * 69u / 100u;
    k = k < 1 ? 1 : (k > 30 ? 30 : k);
    const uint64_t bytes = A.win_bytes[w] - 1;
    const uint64_t nbits = bytes * 8;
    const uint32_t words = (uint32_t)((bytes + 1 + 3) / 4);
    for (uint32_t i = l; i < words; i += WAVE) bits[i] = 0;
    wave_sync();
    const uint64_t s_first = A.ob.s0[A.win_fb[w]];
    for (uint32_t i = l; i < keys; i += WAVE) {
      const uint32_t e = A.surv[s_first + i];
      const uint64_t h = xxh64_words(A.tu.heap + (uint64_t)e * A.kw8, A.tu.ulen[e]);
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
    uint8_t* dst = A.out + A.of.out[f] + A.of.filter_off[f] + (A.win_off[w] - A.win_off[A.of.w0[f]]);
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
