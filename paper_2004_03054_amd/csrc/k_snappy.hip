// Compressed data blocks (block type 1, Snappy raw streams).  The paper's
// prototype stores blocks uncompressed and names compression as future work
// (Sec. IV-A); LevelDB, its base, compresses data blocks with Snappy.
//
//   k_unsnappy   one wave per compressed input block: the stream's elements
//                are taken one at a time (their positions depend on every
//                earlier element), the bytes of each are produced by all 64
//                lanes at once into LDS, and the raw block is then stored to
//                staging memory.  Blocks whose raw bytes exceed the wave's LDS
//                share are produced directly in global memory instead.
//
// Stream format (public format description): a varint32 of the raw length,
// then elements whose tag's low two bits select a literal (0; length in the
// tag, or in 1-4 bytes after it) or a copy with an 11-bit (1), 16-bit (2) or
// 32-bit (3) offset back into the bytes produced; a copy may overlap the
// bytes it produces, so byte k of a copy at offset d is the byte at
// (start - d + k mod d) when d is smaller than the copy.
#include "dev_common.h"
#include "kernels.h"
#include "crc_multi.h"

namespace luda {

constexpr uint32_t UNZ_WAVES = 2;
constexpr uint32_t UNZ_LDS = 32768;  // raw bytes per wave produced in LDS

__device__ inline void unz_report(const WalkSet& ws, const Inputs& in, uint64_t b, uint64_t off,
                                  unsigned long long* err) {
  const uint32_t g = ws.input[b];
  report_err(&err[in.job[g]], err_key(in.local[g], ws.where, ws.local[b], P_TRAILER, off, EC_FORMAT));
}

// Produce the raw bytes of one stream.  Out is LDS (IN_LDS) or global memory;
// returns ~0 on success, else the offset of the first element that cannot be
// decoded (0: the length preamble; n: the stream ends short).
template <bool IN_LDS>
__device__ uint64_t unsnappy_wave(const uint8_t* src, uint32_t n, uint8_t* out, uint32_t* len_out) {
  const uint32_t lane = lane_id();
  uint32_t len = 0;
  const uint32_t a = get_varint32(src, src + n, &len);
  if (!a) return 0;
  *len_out = len;
  uint64_t ip = a, op = 0;
  while (ip < n) {
    const uint64_t t = ip;
    const uint32_t tag = ldg_u8((uint64_t)(uintptr_t)(src + ip));
    ip++;
    const uint32_t kind = tag & 3;
    uint64_t L, off = 0;
    if (kind == 0) {
      L = (uint64_t)(tag >> 2) + 1;
      if (L > 60) {
        const uint32_t nb = (uint32_t)(L - 60);
        if (nb > n - ip) return t;
        L = 0;
        for (uint32_t k = 0; k < nb; k++) L |= (uint64_t)ldg_u8((uint64_t)(uintptr_t)(src + ip + k)) << (8 * k);
        L += 1;
        ip += nb;
      }
      if (L > n - ip || L > len - op) return t;
      for (uint64_t k = lane; k < L; k += WAVE) out[op + k] = (uint8_t)ldg_u8((uint64_t)(uintptr_t)(src + ip + k));
      ip += L;
    } else {
      const uint32_t need = kind == 1 ? 1 : kind == 2 ? 2 : 4;
      if (need > n - ip) return t;
      if (kind == 1) {
        L = ((tag >> 2) & 7) + 4;
        off = ((uint64_t)(tag >> 5) << 8) | ldg_u8((uint64_t)(uintptr_t)(src + ip));
      } else {
        L = (uint64_t)(tag >> 2) + 1;
        off = 0;
        for (uint32_t k = 0; k < need; k++) off |= (uint64_t)ldg_u8((uint64_t)(uintptr_t)(src + ip + k)) << (8 * k);
      }
      ip += need;
      if (off == 0 || off > op || L > len - op) return t;
      // every byte read lies before op: produced by earlier elements
      for (uint64_t k = lane; k < L; k += WAVE) {
        const uint64_t kk = off < L ? k % off : k;
        out[op + k] = out[op - off + kk];
      }
    }
    op += L;
    if (IN_LDS) {
      wave_sync();
    } else {  // the next element may read what other lanes just stored
      __threadfence();
    }
  }
  if (op != len) return n;
  return ~0ull;
}

__global__ void __launch_bounds__(UNZ_WAVES * 64) k_unsnappy(WalkSet ws, Inputs in, uint8_t* ok, const uint64_t* zcap,
                                                             const uint64_t* zoff, uint8_t* stage,
                                                             unsigned long long* err) {
  __shared__ __align__(16) uint8_t lds[UNZ_WAVES][UNZ_LDS];
  const uint64_t nb = *ws.n_dev;
  const uint32_t wv = threadIdx.x / WAVE, lane = lane_id();
  for (uint64_t b = (uint64_t)blockIdx.x * UNZ_WAVES + wv; b < nb; b += (uint64_t)gridDim.x * UNZ_WAVES) {
    if (!zcap[b] || !ok[b]) continue;
    const uint8_t* src = (const uint8_t*)ws.ptr[b];
    const uint32_t n = ws.size[b];
    uint8_t* dst = stage + zoff[b];
    // the staging room holds min(declared, 22 n) bytes: a stream never
    // produces more, so a longer declared length fails before it is full
    uint32_t len = 0;
    uint32_t declared = 0;
    (void)get_varint32(src, src + n, &declared);
    uint64_t bad;
    const bool small = declared <= UNZ_LDS;
    if (small) bad = unsnappy_wave<true>(src, n, lds[wv], &len);
    else bad = unsnappy_wave<false>(src, n, dst, &len);
    if (bad != ~0ull) {
      if (lane == 0) {
        unz_report(ws, in, b, bad, err);
        ok[b] = 0;
      }
      continue;
    }
    if (small) {
      const uint8_t* L = lds[wv];
      for (uint32_t k = 16 * lane; k < len; k += 16 * WAVE) {
        if (k + 16 <= len) {
          *(uint4*)(dst + k) = *(const uint4*)(L + k);
        } else {
          for (uint32_t q = k; q < len; q++) dst[q] = L[q];
        }
      }
    }
    if (lane == 0) {
      ws.ptr[b] = (uint64_t)(uintptr_t)dst;
      ws.size[b] = len;
    }
  }
}

// ---------------------------------------------------------------------------
// Output side.  With compression on, a data block is first encoded raw into
// staging memory (the same encoder as the uncompressed path), then
// compressed by one wave; it is stored as a type-1 block when the stream
// saves at least an eighth of its raw bytes (LevelDB's rule), else raw.  The
// stored sizes then drive the file cuts and the layout, and k_zplace moves
// each block's stored bytes to its place in its table.
//
// The stream follows the oracle writer's rules exactly:
//   - 64 KiB fragments, no copy reaching into an earlier fragment;
//   - per fragment a 4096-entry table of positions; positions are taken in
//     groups of 64 (one per lane); each looks up the table under the hash of
//     its 4 bytes (the little-endian word times 0x9E3779B1, top 12 bits) as
//     the table stood before its group, then every position of the group is
//     entered (the table keeps the largest, i.e. last, position);
//   - a position whose candidate holds the same 4 bytes starts a copy that
//     runs while the bytes agree (up to the fragment end); greedy from the
//     fragment start, with everything between copies one literal;
//   - copies split into pieces of 64 while 68 or more remain, one of 60 if
//     more than 64 remain, and a last piece in the 2-byte form when it is at
//     most 11 long at an offset below 2048, else the 3-byte form.

constexpr uint32_t ZC_WAVES = 4;
constexpr uint32_t ZC_FRAG = 65536;
constexpr uint32_t ZC_HASH_BITS = 12;

__device__ inline uint32_t zc_hash(uint32_t v) { return (v * 0x9E3779B1u) >> (32 - ZC_HASH_BITS); }

__device__ inline uint32_t zc_lit_hdr(uint64_t k) {  // header bytes of a literal of k >= 1 bytes
  const uint64_t m = k - 1;
  return m < 60 ? 1 : m < 256 ? 2 : m < 65536 ? 3 : m < (1u << 24) ? 4 : 5;
}

__device__ inline uint32_t zc_copy_bytes(uint64_t off, uint64_t L) {
  uint32_t q = 0;
  while (L >= 68) {
    q += 3;
    L -= 64;
  }
  if (L > 64) {
    q += 3;
    L -= 60;
  }
  return q + ((L <= 11 && off < 2048) ? 2 : 3);
}

// literal of k bytes from src at out + q (all lanes); returns its length
__device__ inline uint64_t zc_put_literal(uint8_t* out, uint64_t q, const uint8_t* src, uint64_t k) {
  if (k == 0) return 0;
  const uint32_t h = zc_lit_hdr(k);
  if (lane_id() == 0) {
    const uint64_t m = k - 1;
    if (h == 1) {
      out[q] = (uint8_t)(m << 2);
    } else {
      out[q] = (uint8_t)((59 + (h - 1)) << 2);
      for (uint32_t i = 0; i + 1 < h; i++) out[q + 1 + i] = (uint8_t)(m >> (8 * i));
    }
  }
  for (uint64_t i = lane_id(); i < k; i += WAVE) out[q + h + i] = (uint8_t)ldg_u8((uint64_t)(uintptr_t)(src + i));
  return h + k;
}

__device__ inline void zc_piece(uint8_t* d, uint32_t* p, uint64_t off, uint64_t L, bool short_form) {
  if (short_form) {
    d[(*p)++] = (uint8_t)(1 | ((L - 4) << 2) | ((off >> 8) << 5));
    d[(*p)++] = (uint8_t)(off & 0xFF);
  } else {
    d[(*p)++] = (uint8_t)(2 | ((L - 1) << 2));
    d[(*p)++] = (uint8_t)(off & 0xFF);
    d[(*p)++] = (uint8_t)(off >> 8);
  }
}

__device__ inline uint64_t zc_put_copy(uint8_t* out, uint64_t q, uint64_t off, uint64_t L) {
  uint32_t p = 0;
  if (lane_id() == 0) {
    uint8_t* d = out + q;
    while (L >= 68) {
      zc_piece(d, &p, off, 64, false);
      L -= 64;
    }
    if (L > 64) {
      zc_piece(d, &p, off, 60, false);
      L -= 60;
    }
    zc_piece(d, &p, off, L, L <= 11 && off < 2048);
  }
  return (uint64_t)__shfl(p, 0, WAVE);
}

// The stream of n raw bytes at r.  Size pass (!WRITE): returns its length,
// or any value >= limit as soon as it reaches limit.  Write pass: writes it
// to out and returns its length.
template <bool WRITE>
__device__ uint64_t zc_wave(const uint8_t* r, uint32_t n, uint32_t* T, uint8_t* out, uint64_t limit) {
  const uint32_t lane = lane_id();
  uint64_t q = varint_len(n);
  if (WRITE && lane == 0) put_varint(out, n);
  for (uint64_t f0 = 0; f0 < n; f0 += ZC_FRAG) {
    const uint8_t* fr = r + f0;
    const uint32_t m = (uint32_t)min((uint64_t)ZC_FRAG, n - f0);
    for (uint32_t h = lane; h < (1u << ZC_HASH_BITS); h += WAVE) T[h] = 0;  // 0: empty, else position + 1
    wave_sync();
    uint32_t pos = 0, lit = 0;
    for (uint32_t b = 0; b < m; b += WAVE) {
      const uint32_t e = min(b + WAVE, m);
      const uint32_t p = b + lane;
      const bool has = p + 4 <= m;
      const uint32_t v = has ? ldg_u32_unaligned(fr + p) : 0u;
      const uint32_t h = zc_hash(v);
      const uint32_t c1 = has ? T[h] : 0u;  // the table as it stood before this group
      wave_sync();
      if (has) atomicMax(&T[h], p + 1);
      wave_sync();
      const bool match = c1 != 0 && ldg_u32_unaligned(fr + (c1 - 1)) == v;
      const uint64_t M = wave_ballot(match);
      while (pos < e) {
        const uint64_t Mr = M & (~0ull << (pos - b));
        if (!Mr) {
          pos = e;
          break;
        }
        const uint32_t at = (uint32_t)__builtin_ctzll(Mr);
        const uint32_t qp = b + at;
        const uint32_t c = (uint32_t)__shfl((int)c1, (int)at, WAVE) - 1;
        // the copy runs while the bytes agree, up to the fragment end
        uint32_t L = 4;
        const uint32_t most = m - qp;
        while (L < most) {
          const uint32_t k = L + lane;
          const bool eq = k < most && ldg_u8((uint64_t)(uintptr_t)(fr + c + k)) == ldg_u8((uint64_t)(uintptr_t)(fr + qp + k));
          const uint64_t ne = wave_ballot(!eq);
          if (ne) {
            L += (uint32_t)__builtin_ctzll(ne);
            break;
          }
          L += WAVE;
        }
        if (L > most) L = most;
        if (WRITE) {
          q += zc_put_literal(out, q, fr + lit, qp - lit);
          q += zc_put_copy(out, q, qp - c, L);
        } else {
          q += (qp > lit ? zc_lit_hdr(qp - lit) + (qp - lit) : 0) + zc_copy_bytes(qp - c, L);
          if (q >= limit) return q;
        }
        pos = qp + L;
        lit = pos;
      }
      if (!WRITE && q + (pos > lit ? pos - lit : 0) >= limit) return limit;  // the pending literal alone reaches it
    }
    if (WRITE) q += zc_put_literal(out, q, fr + lit, m - lit);
    else q += m > lit ? zc_lit_hdr(m - lit) + (m - lit) : 0;
  }
  return q;
}

// raw staging layout: every block's raw message (contents + 5-byte trailer)
// at a 16-byte aligned offset, with room after it
__global__ void k_zprep(OutBlocks ob, const uint64_t* nblocks, uint64_t cap, uint32_t* zraw, uint64_t* zstride) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= cap || b >= *nblocks) return;
  const uint32_t n = ob.size[b];
  zraw[b] = n;
  zstride[b] = (((uint64_t)n + 5 + 15) & ~15ull) + ZSTAGE_PAD;
}

// the encoder's block records for the raw staging layout
__global__ void k_block_dst_stage(OutBlocks ob, const uint64_t* zoff, const JobDesc* jobs, const uint64_t* nblocks,
                                  uint64_t cap, BlockRec* br) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= cap || b >= *nblocks) return;
  BlockRec r;
  r.dst = zoff[b];
  r.s0 = ob.s0[b];
  r.cnt = ob.cnt[b];
  r.size = ob.size[b];
  r.R = jobs[ob.job[b]].restart_interval;
  r.pad = 0;
  br[b] = r;
}

// one wave per block of a job with compression on: the stream's length
// first, then (when it saves an eighth) the stream itself into zbuf at the
// block's staging offset; the block's stored size and type follow
__global__ void __launch_bounds__(ZC_WAVES * 64) k_zsnappy(OutBlocks ob, const JobDesc* jobs, const uint64_t* nblocks,
                                                           const uint8_t* stage, const uint64_t* zoff,
                                                           const uint32_t* zraw, uint8_t* zbuf, uint8_t* ztype) {
  __shared__ uint32_t T[ZC_WAVES][1u << ZC_HASH_BITS];
  const uint64_t nb = *nblocks;
  const uint32_t wv = threadIdx.x / WAVE;
  for (uint64_t b = (uint64_t)blockIdx.x * ZC_WAVES + wv; b < nb; b += (uint64_t)gridDim.x * ZC_WAVES) {
    const uint32_t n = zraw[b];
    uint8_t type = 0;
    if (jobs[ob.job[b]].compression == 1) {
      const uint64_t limit = (uint64_t)n - n / 8;
      const uint8_t* r = stage + zoff[b];
      const uint64_t z = zc_wave<false>(r, n, T[wv], nullptr, limit);
      if (z < limit) {
        (void)zc_wave<true>(r, n, T[wv], zbuf + zoff[b], limit);
        type = 1;
        if (lane_id() == 0) {
          ob.size[b] = (uint32_t)z;
          ob.full[b] = z + 5;
        }
      }
    }
    if (lane_id() == 0) ztype[b] = type;
  }
}

// each block's stored bytes (raw from staging, or its stream) and type byte
// into its place in the output; the checksum follows (ZBlockMsgs)
__global__ void k_zplace(const BlockRec* br, const uint64_t* nblocks, const uint8_t* stage, const uint8_t* zbuf,
                         const uint64_t* zoff, const uint8_t* ztype, uint8_t* out) {
  const uint64_t nb = *nblocks;
  const uint32_t waves = blockDim.x / WAVE, wv = threadIdx.x / WAVE;
  for (uint64_t b = (uint64_t)blockIdx.x * waves + wv; b < nb; b += (uint64_t)gridDim.x * waves) {
    const BlockRec r = br[b];
    const uint8_t* src = (ztype[b] ? zbuf : stage) + zoff[b];
    uint8_t* dst = out + r.dst;
    for (uint64_t k = 16 * (uint64_t)lane_id(); k < r.size; k += 16 * WAVE) {
      if (k + 16 <= r.size) {
        *(uint4_u1*)(dst + k) = ldg16a((uint64_t)(uintptr_t)(src + k));  // dst of any alignment
      } else {
        for (uint64_t i = k; i < r.size; i++) dst[i] = src[i];
      }
    }
    if (lane_id() == 0) dst[r.size] = ztype[b];
  }
}

struct ZBlockMsgs {
  const BlockRec* br;
  const uint64_t* nblocks;
  uint64_t cap;
  uint8_t* out;
  __device__ uint32_t count() const { return (uint32_t)min(cap, *nblocks); }
  __device__ void span(uint32_t m, const uint8_t** p, uint64_t* n) const {
    *p = out + br[m].dst;
    *n = (uint64_t)br[m].size + 1;
  }
  __device__ void finish(uint32_t m, uint32_t raw) const {
    uint8_t* d = out + br[m].dst + br[m].size + 1;
    const uint32_t v = crc_mask(raw ^ 0xFFFFFFFFu);
    for (int k = 0; k < 4; k++) d[k] = (uint8_t)(v >> (8 * k));
  }
  __device__ void empty(uint32_t) const {}
};

void launch_crc_zblocks(const BlockRec* br, const uint64_t* nblocks, uint64_t cap, uint8_t* out, const uint32_t* g_crc,
                        uint32_t* part, uint64_t* mseg, uint32_t grid, hipStream_t st) {
  launch_crc_msgs(ZBlockMsgs{br, nblocks, cap, out}, cap, g_crc, part, mseg, grid, st);
}

// Per file whose first data block is stored compressed: its smallest
// internal key is not stored verbatim in the table, so it is written after
// the table (the file's stride in the output buffer grows by it).
__global__ void k_zslots(OutFiles of, OutBlocks ob, const uint32_t* surv, Tuples tu, const uint8_t* ztype,
                         const uint64_t* nfiles, uint64_t cap, uint64_t* stride) {
  const uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= cap || f >= *nfiles) return;
  const uint64_t b0 = of.b0[f];
  stride[f] = of.size[f] + (ztype[b0] ? (uint64_t)tu.ulen[surv[ob.s0[b0]]] + 8 : 0);
}

__global__ void k_zkeys(OutFiles of, OutBlocks ob, const uint32_t* surv, Tuples tu, const uint8_t* ztype,
                        uint32_t kw8, uint64_t nf, uint8_t* out) {
  const uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const uint64_t b0 = of.b0[f];
  if (!ztype[b0]) return;
  const uint32_t e = surv[ob.s0[b0]];
  const uint32_t ulen = tu.ulen[e];
  uint8_t* d = out + of.out[f] + of.size[f];
  const uint8_t* slot = (const uint8_t*)(tu.heap + (uint64_t)e * kw8);
  for (uint32_t i = 0; i < ulen; i++) d[i] = slot[i];
  const uint64_t tag = tu.tag[e];
  for (int i = 0; i < 8; i++) d[ulen + i] = (uint8_t)(tag >> (8 * i));
}

}  // namespace luda
