// Phase 3 "Pack" writers (paper Sec. II-A Phase 3; Sec. III-C: encode fills
// data blocks and checksums them with no data exchange between blocks, filter
// builds each table's Bloom filter block).  Values move once: from the input
// table bytes straight into the output block (the paper's lazy value
// movement, Sec. III-D, without the intermediate pair buffer).
//
//   k_encode       one wave per output data block: assembles the block in
//                  16-byte chunks aligned to the block end (entries, restart
//                  array, count, type byte), stores it, CRCs it from LDS
//   k_filter       one wave per filter window: Bloom bits in LDS, then stored
//   k_index_write  one thread per data block: its index entry and restart slot
//   k_meta         one thread per file: filter tail, metaindex, trailers' type
//                  bytes, footer
//   k_crc_ranges   one workgroup per (file, filter | metaindex | index block)
#include "dev_common.h"
#include "kernels.h"

namespace luda {

// byte p of output block b's message (contents || type byte)
struct BlockGen {
  const EncodeArgs* A;
  uint64_t s0;
  uint32_t cnt, R;
  const uint32_t* est;  // entry starts in LDS (cnt + 1 values)
  uint64_t data_end;
  uint32_t nrest;
  uint32_t size;
  // cursor
  int32_t ci;  // current entry index (-1: none)
  uint64_t c_start, c_end;
  uint32_t c_shared, c_hl, c_ns, c_ulen, c_vlen;
  uint8_t c_hdr[15];
  const uint8_t* c_slot;
  uint64_t c_tag;
  const uint8_t* c_val;

  __device__ void load_entry(uint32_t i) {
    ci = (int32_t)i;
    c_start = est[i];
    c_end = est[i + 1];
    const uint64_t s = s0 + i;
    const bool restart = (i % R) == 0;
    c_shared = restart ? 0 : A->shr[s];
    const uint32_t e = A->surv[s];
    c_ulen = A->tu.ulen[e];
    const uint32_t klen = c_ulen + 8;
    c_ns = klen - c_shared;
    c_vlen = A->tu.vlen[e];
    c_slot = (const uint8_t*)(A->tu.heap + (uint64_t)e * A->kw8);
    c_tag = A->tu.tag[e];
    c_val = (const uint8_t*)A->tu.vp[e];
    uint32_t h = put_varint(c_hdr, c_shared);
    h += put_varint(c_hdr + h, c_ns);
    h += put_varint(c_hdr + h, c_vlen);
    c_hl = h;
  }

  __device__ uint32_t find_entry(uint64_t p) const {
    uint32_t lo = 0, hi = cnt;  // est[lo] <= p < est[hi]
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) / 2;
      if (est[mid] <= p) lo = mid;
      else hi = mid;
    }
    return lo;
  }

  __device__ uint32_t byte(uint64_t p) {
    if (p < data_end) {
      if (ci < 0 || p < c_start || p >= c_end) load_entry(find_entry(p));
      const uint64_t o = p - c_start;
      if (o < c_hl) return c_hdr[o];
      if (o < c_hl + c_ns) return ikey_byte(c_slot, c_ulen, c_tag, c_shared + (uint32_t)(o - c_hl));
      return c_val[o - c_hl - c_ns];
    }
    if (p < data_end + 4ull * nrest) {
      const uint64_t q = p - data_end;
      const uint32_t v = est[(q / 4) * R];
      return (v >> (8 * (q % 4))) & 0xFF;
    }
    if (p < (uint64_t)size) {
      const uint64_t q = p - data_end - 4ull * nrest;
      return (nrest >> (8 * q)) & 0xFF;
    }
    return 0;  // type byte: no compression
  }
};

__global__ void __launch_bounds__(256) k_encode(EncodeArgs A) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  CrcLds* T = (CrcLds*)smem;
  load_crc_tables(T, A.g_crc, threadIdx.x, blockDim.x);
  __syncthreads();
  const uint32_t wv = threadIdx.x / WAVE, l = lane_id();
  const uint32_t waves = blockDim.x / WAVE;
  uint8_t* wbase = smem + sizeof(CrcLds) + (size_t)wv * (A.stage_bytes + 4ull * A.ent_cap);
  uint8_t* stage_end = wbase + A.stage_bytes;
  uint32_t* est = (uint32_t*)stage_end;
  const uint64_t nb = *A.nblocks;
  for (uint64_t b = (uint64_t)blockIdx.x * waves + wv; b < nb; b += (uint64_t)gridDim.x * waves) {
    const uint32_t j = A.ob.job[b];
    const uint32_t R = A.jobs[j].restart_interval;
    const uint64_t s0 = A.ob.s0[b];
    const uint32_t cnt = A.ob.cnt[b];
    const uint32_t size = A.ob.size[b];
    const uint32_t n = size + 1;
    const uint32_t f = A.ob.file[b];
    uint8_t* dst = A.out + A.of.out[f] + A.ob.off[b];
    // entry starts
    uint32_t running = 0;
    for (uint32_t i0 = 0; i0 < cnt; i0 += WAVE) {
      const uint32_t i = i0 + l;
      uint32_t sz = 0;
      if (i < cnt) sz = (i % R == 0) ? A.sz_r[s0 + i] : A.sz_n[s0 + i];
      const uint32_t incl = wave_incl_scan(sz);
      if (i < cnt) est[i] = running + incl - sz;
      running += __shfl(incl, WAVE - 1, WAVE);
    }
    if (l == 0) est[cnt] = running;
    wave_sync();
    BlockGen G;
    G.A = &A;
    G.s0 = s0;
    G.cnt = cnt;
    G.R = R;
    G.est = est;
    G.data_end = running;
    G.nrest = (cnt + R - 1) / R;
    G.size = size;
    G.ci = -1;
    const uint32_t J16 = (n + 15) / 16;
    for (uint32_t q = l; q < J16; q += WAVE) {
      const int64_t p0 = (int64_t)n - 16ll * (J16 - q);
      uint8_t* sdst = stage_end - 16ull * (J16 - q);
      uint4 v;
      bool fast = false;
      if (p0 >= 0 && (uint64_t)p0 + 16 <= G.data_end) {
        const uint32_t i = G.find_entry((uint64_t)p0);
        if (G.ci != (int32_t)i) G.load_entry(i);
        const uint64_t vstart = G.c_start + G.c_hl + G.c_ns;
        if ((uint64_t)p0 >= vstart && (uint64_t)p0 + 16 <= G.c_end) {
          __builtin_memcpy(&v, G.c_val + ((uint64_t)p0 - vstart), 16);
          fast = true;
        }
      }
      if (!fast) {
        uint8_t tmp[16];
#pragma unroll
        for (int k = 0; k < 16; k++) {
          const int64_t p = p0 + k;
          tmp[k] = p >= 0 ? (uint8_t)G.byte((uint64_t)p) : 0;
        }
        __builtin_memcpy(&v, tmp, 16);
      }
      *(uint4*)sdst = v;
      if (p0 >= 0) {
        __builtin_memcpy(dst + p0, &v, 16);
      } else {
        const uint8_t* vb = (const uint8_t*)&v;
        for (int k = 0; k < 16; k++)
          if (p0 + k >= 0) dst[p0 + k] = vb[k];
      }
    }
    wave_sync();
    const uint32_t crc = wave_crc_lds(stage_end, n, T);
    if (l == 0) {
      const uint32_t m = crc_mask(crc);
      for (int k = 0; k < 4; k++) dst[n + k] = (uint8_t)(m >> (8 * k));
    }
    wave_sync();
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

// CRC of filter (kind 0), metaindex (1) and index (2) blocks of each file
struct CrcLdsWG2 {
  uint32_t t4[4][256];
  uint32_t sh[9][4][256];
};

__device__ inline uint32_t ld_dword_from(const uint8_t* msg, int64_t p) {
  if (p >= 0) return ldg_u32_unaligned(msg + p);
  uint32_t v = 0;
  for (int j = 0; j < 4; j++)
    if (p + j >= 0) v |= (uint32_t)msg[p + j] << (8 * j);
  return v;
}

__global__ void __launch_bounds__(256) k_crc_ranges(OutFiles of, const uint64_t* nfiles, uint64_t cap, uint8_t* out,
                                                    const uint32_t* g_t4, const uint32_t* g_sh) {
  __shared__ CrcLdsWG2 T;
  __shared__ uint32_t red[4];
  const uint64_t f = blockIdx.x / 3;
  const uint32_t kind = blockIdx.x % 3;
  if (f >= cap || f >= *nfiles) return;
  for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) (&T.t4[0][0])[i] = g_t4[i];
  for (int i = threadIdx.x; i < 9 * 4 * 256; i += blockDim.x) (&T.sh[0][0][0])[i] = g_sh[i];
  __syncthreads();
  uint64_t off, size;
  if (kind == 0) { off = of.filter_off[f]; size = of.filter_size[f]; }
  else if (kind == 1) { off = of.meta_off[f]; size = of.meta_size[f]; }
  else { off = of.index_off[f]; size = of.index_size[f]; }
  uint8_t* msg = out + of.out[f] + off;
  const uint64_t n = size + 1;
  const uint32_t tid = threadIdx.x;
  const uint64_t ROW = (uint64_t)CRC_SLICE * 256;
  const uint64_t rows = (n + ROW - 1) / ROW;
  uint32_t acc = 0;
  for (uint64_t r = 0; r < rows; r++) {
    const int64_t pos0 = (int64_t)n - (int64_t)(rows - r) * (int64_t)ROW + (int64_t)CRC_SLICE * tid;
    uint32_t rs = 0;
    for (uint32_t k = 0; k < CRC_DW; k++) {
      const int64_t p = pos0 + 4 * k;
      if (p + 4 <= 0) continue;
      rs = crc_dword(T.t4, rs, crc_edge(ld_dword_from(msg, p), p));
    }
    acc = (r ? crc_shift(T.sh[8], acc) : 0u) ^ rs;
  }
#pragma unroll
  for (int k = 0; k < 6; k++) {
    uint32_t other = __shfl_down(acc, 1u << k, WAVE);
    acc = crc_shift(T.sh[k], acc) ^ other;
  }
  const uint32_t w = tid / WAVE;
  if (lane_id() == 0) {
    uint32_t v = acc;
    for (uint32_t q = w; q < 3; q++) v = crc_shift(T.sh[6], v);
    red[w] = v;
  }
  __syncthreads();
  if (tid == 0) {
    const uint32_t crc = (red[0] ^ red[1] ^ red[2] ^ red[3]) ^ 0xFFFFFFFFu;
    put_fixed32(msg + n, crc_mask(crc));
  }
}

}  // namespace luda
