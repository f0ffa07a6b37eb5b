// Phase 1 "Unpack" kernels (paper Sec. II-A Phase 1; Sec. III-C: one unpack
// pass per table with its data blocks processed in parallel).  Each table is
// read footer -> index block -> data blocks; every block's masked CRC32C is
// verified before its entries are restored.
//
//   k_footer      one thread per input: footer magic + index handle
//   k_index_scan  one workgroup per input: index block CRC, restart array,
//                 entry walk, handle ranges; counts data blocks
//   k_index_emit  one workgroup per input: writes the flat block table
//   k_decode      persistent waves pull data blocks by ticket: stage the
//                 block in LDS, CRC it, walk restart intervals in parallel,
//                 and place the block's entries with a decoupled look-back
//   k_keys        one thread per entry: restores the internal key by tracing
//                 each byte back through the shared-prefix chain
//   k_order       one thread per entry: internal keys strictly increase
//                 inside a table; records how adjacent tables compare
#include "dev_common.h"
#include "kernels.h"

namespace luda {

__global__ void k_footer(Inputs in, unsigned long long* err) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= in.n) return;
  const uint8_t* p = (const uint8_t*)in.ptr[g];
  const uint64_t size = in.size[g];
  const uint32_t job = in.job[g], loc = in.local[g];
  in.nblk[g] = 0;
  in.maxblk[g] = 0;
  in.dbytes[g] = 0;
  in.idx_size[g] = ~0ull;  // marks a failed input
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
  if (!d || ioff > limit || isize > limit - ioff || 5 > limit - ioff - isize) {
    report_err(&err[job], err_key(loc, W_FOOTER, 0, FP_REL, a + b, EC_FORMAT));
    return;
  }
  in.idx_off[g] = ioff;
  in.idx_size[g] = isize;
}

// ---------------------------------------------------------------------------
// Workgroup CRC over a global byte range: 256 lanes, 68-byte slices, rows of
// 17408 bytes, joined with the shift-by-68*2^k tables (k = 0..8).

struct CrcLdsWG {
  uint32_t t4[4][256];
  uint32_t sh[9][4][256];
};

__device__ inline uint32_t ld_msg_dword(const uint8_t* msg, int64_t p) {
  // dword at message positions p..p+3 (p + 4 > 0); bytes before 0 read as 0
  if (p >= 0) return ldg_u32_unaligned(msg + p);
  uint32_t v = 0;
  for (int j = 0; j < 4; j++)
    if (p + j >= 0) v |= (uint32_t)msg[p + j] << (8 * j);
  return v;
}

__device__ uint32_t wg_crc_global(const uint8_t* msg, uint64_t n, const CrcLdsWG* T, uint32_t* red) {
  const uint32_t tid = threadIdx.x;  // blockDim.x == 256
  const uint64_t ROW = (uint64_t)CRC_SLICE * 256;
  const uint64_t rows = (n + ROW - 1) / ROW;
  uint32_t acc = 0;
  for (uint64_t r = 0; r < rows; r++) {
    const int64_t pos0 = (int64_t)n - (int64_t)(rows - r) * (int64_t)ROW + (int64_t)CRC_SLICE * tid;
    uint32_t rs = 0;
    for (uint32_t k = 0; k < CRC_DW; k++) {
      const int64_t p = pos0 + 4 * k;
      if (p + 4 <= 0) continue;
      uint32_t d = crc_edge(ld_msg_dword(msg, p), p);
      rs = crc_dword(T->t4, rs, d);
    }
    acc = (r ? crc_shift(T->sh[8], acc) : 0u) ^ rs;
  }
#pragma unroll
  for (int k = 0; k < 6; k++) {
    uint32_t other = __shfl_down(acc, 1u << k, WAVE);
    acc = crc_shift(T->sh[k], acc) ^ other;
  }
  const uint32_t w = tid / WAVE;
  if (lane_id() == 0) {
    // wave w covers 4352 bytes followed by (3 - w) more wave slices
    uint32_t v = acc;
    if (w <= 2) v = crc_shift(T->sh[6], v);   // +4352 (waves 0..2 get at least one)
    if (w <= 1) v = crc_shift(T->sh[6], v);   // +4352
    if (w == 0) v = crc_shift(T->sh[6], v);   // +4352
    red[w] = v;
  }
  __syncthreads();
  uint32_t raw = red[0] ^ red[1] ^ red[2] ^ red[3];
  __syncthreads();
  return raw ^ 0xFFFFFFFFu;
}

__device__ inline void load_tables_wg(CrcLdsWG* T, const uint32_t* g_t4, const uint32_t* g_sh) {
  uint32_t* d = &T->t4[0][0];
  for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) d[i] = g_t4[i];
  uint32_t* s = &T->sh[0][0][0];
  for (int i = threadIdx.x; i < 9 * 4 * 256; i += blockDim.x) s[i] = g_sh[i];
}

// Walk one restart interval [o, end) of a block's entry area [0, data_end).
// Checks, per entry in order (all CORRUPT_FORMAT at the entry offset): three
// varint32 headers inside the area, shared <= previous key length, key delta
// and value inside the area, shared == 0 for the interval's first entry (a
// restart point), the entry does not cross the interval end.  For data
// blocks also: internal key length >= 8.  Returns the first failing entry
// offset (or ~0ull) and counts the entries.
struct WalkOut {
  uint64_t err_off;
  uint32_t count;
  uint32_t maxklen;
};

template <bool DATA, typename Visit>
__device__ inline WalkOut walk_interval(const uint8_t* c, uint64_t data_end, uint64_t o, uint64_t end,
                                        Visit visit) {
  WalkOut w{~0ull, 0, 0};
  uint64_t prev_len = 0;
  bool first = true;
  const uint8_t* limit = c + data_end;
  while (o < end) {
    uint32_t shared, ns, vlen;
    const uint8_t* p = c + o;
    uint32_t a = get_varint32(p, limit, &shared);
    uint32_t b = a ? get_varint32(p + a, limit, &ns) : 0;
    uint32_t d = b ? get_varint32(p + a + b, limit, &vlen) : 0;
    if (!d) { w.err_off = o; return w; }
    const uint64_t hdr = a + b + d;
    if (!first && shared > prev_len) { w.err_off = o; return w; }
    if ((uint64_t)ns + vlen > data_end - (o + hdr)) { w.err_off = o; return w; }
    if (first && shared != 0) { w.err_off = o; return w; }
    const uint64_t e = o + hdr + ns + vlen;
    if (e > end) { w.err_off = o; return w; }
    const uint64_t klen = (uint64_t)shared + ns;
    if (DATA && klen < 8) { w.err_off = o; return w; }
    visit(o, hdr, shared, ns, vlen);
    w.count++;
    if (klen > w.maxklen) w.maxklen = (uint32_t)(klen > 0xFFFFFFFFull ? 0xFFFFFFFFu : klen);
    prev_len = klen;
    first = false;
    o = e;
  }
  return w;
}

// restart array checks: count (size >= 4, 1 <= n <= (size-4)/4), then each
// offset: first is 0, strictly increasing, inside the entry area
__device__ inline uint64_t check_restart_count(const uint8_t* c, uint64_t size, uint32_t* nr_out) {
  if (size < 4) return 0;  // offset 0
  uint32_t nr = rd_u32_bytes(c + size - 4);
  if (nr == 0 || nr > (size - 4) / 4) return size - 4;
  *nr_out = nr;
  return ~0ull;
}

__device__ inline bool bad_restart(const uint8_t* c, uint64_t data_end, uint32_t k) {
  uint32_t r = rd_u32_bytes(c + data_end + 4ull * k);
  if (k == 0) return r != 0 || r >= data_end;
  uint32_t pr = rd_u32_bytes(c + data_end + 4ull * (k - 1));
  return r <= pr || r >= data_end;
}

// ---------------------------------------------------------------------------

__device__ inline void index_block_common(const Inputs& in, uint32_t g, const uint8_t*& c,
                                          uint64_t& size, uint32_t& nr, uint64_t& data_end,
                                          bool& ok, unsigned long long* err, uint32_t job,
                                          uint32_t loc, uint32_t* sflag) {
  // restart array of the index block (index phase RESTARTS)
  const uint8_t* base = (const uint8_t*)in.ptr[g];
  c = base + in.idx_off[g];
  size = in.idx_size[g];
  ok = true;
  if (threadIdx.x == 0) *sflag = 0;
  __syncthreads();
  uint64_t eo = check_restart_count(c, size, &nr);
  if (eo != ~0ull) {
    if (threadIdx.x == 0) report_err(&err[job], err_key(loc, W_INDEX, 0, P_RESTARTS, eo, EC_FORMAT));
    ok = false;
    return;
  }
  data_end = size - 4 - 4ull * nr;
  for (uint32_t k = threadIdx.x; k < nr; k += blockDim.x) {
    if (bad_restart(c, data_end, k)) {
      report_err(&err[job], err_key(loc, W_INDEX, 0, P_RESTARTS, data_end + 4ull * k, EC_FORMAT));
      atomicOr(sflag, 1u);
    }
  }
  __syncthreads();
  if (*sflag) ok = false;
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_index_scan(Inputs in, const uint32_t* g_t4, const uint32_t* g_sh,
                                                    unsigned long long* err) {
  __shared__ CrcLdsWG T;
  __shared__ uint32_t red[4];
  __shared__ uint32_t sflag;
  __shared__ uint32_t scount;
  __shared__ uint32_t smax;
  __shared__ unsigned long long sbytes;
  const uint32_t g = blockIdx.x;
  if (in.idx_size[g] == ~0ull) return;  // footer failed
  const uint32_t job = in.job[g], loc = in.local[g];
  load_tables_wg(&T, g_t4, g_sh);
  if (threadIdx.x == 0) {
    scount = 0;
    smax = 0;
    sbytes = 0;
  }
  __syncthreads();
  const uint8_t* base = (const uint8_t*)in.ptr[g];
  const uint64_t ioff = in.idx_off[g], isize = in.idx_size[g];
  const uint32_t crc = wg_crc_global(base + ioff, isize + 1, &T, red);
  const uint32_t stored = crc_unmask(ldg_u32_unaligned(base + ioff + isize + 1));
  if (crc != stored || base[ioff + isize] != 0) {
    if (threadIdx.x == 0) {
      in.idx_size[g] = ~0ull;
      report_err(&err[job], err_key(loc, W_INDEX, 0, P_TRAILER, 0,
                                    crc != stored ? EC_CHECKSUM : EC_UNSUPPORTED));
    }
    return;
  }
  const uint8_t* c;
  uint64_t size, data_end;
  uint32_t nr = 0;
  bool ok;
  index_block_common(in, g, c, size, nr, data_end, ok, err, job, loc, &sflag);
  if (!ok) {
    if (threadIdx.x == 0) in.idx_size[g] = ~0ull;
    return;
  }
  const uint64_t limit = in.size[g] - 48;
  uint32_t cnt = 0, mx = 0;
  unsigned long long by = 0;
  bool bad = false;
  for (uint32_t k = threadIdx.x; k < nr; k += blockDim.x) {
    const uint64_t o = rd_u32_bytes(c + data_end + 4ull * k);
    const uint64_t end = (k + 1 < nr) ? rd_u32_bytes(c + data_end + 4ull * (k + 1)) : data_end;
    uint64_t herr = ~0ull;
    WalkOut w = walk_interval<false>(c, data_end, o, end,
                                     [&](uint64_t eo, uint64_t hdr, uint32_t, uint32_t ns, uint32_t vlen) {
      if (herr != ~0ull) return;
      const uint8_t* v = c + eo + hdr + ns;
      uint64_t boff, bsz;
      uint32_t x = get_varint64(v, v + vlen, &boff);
      uint32_t y = x ? get_varint64(v + x, v + vlen, &bsz) : 0;
      if (!y || x + y != vlen || boff > limit || bsz > limit - boff || 5 > limit - boff - bsz) {
        herr = eo;
        return;
      }
      if (bsz > mx) mx = (uint32_t)(bsz > 0xFFFFFFF0ull ? 0xFFFFFFF0ull : bsz);
      by += bsz + 5;
    });
    uint64_t first_bad = w.err_off < herr ? w.err_off : herr;
    if (first_bad != ~0ull) {
      report_err(&err[job], err_key(loc, W_INDEX, 0, P_ENTRIES, first_bad, EC_FORMAT));
      bad = true;
    }
    cnt += w.count;
  }
  if (bad) atomicOr(&sflag, 1u);
  atomicAdd(&scount, cnt);
  atomicMax(&smax, mx);
  atomicAdd(&sbytes, by);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (sflag) {
      in.idx_size[g] = ~0ull;
      in.nblk[g] = 0;
    } else {
      in.nblk[g] = scount;
      in.maxblk[g] = smax;
      in.dbytes[g] = sbytes;
    }
  }
}

// Write the flat data block table: block numbers follow the index order.
// Each thread owns a contiguous run of restart intervals so that a workgroup
// prefix over per-thread counts gives every entry's block number.
__global__ void __launch_bounds__(256) k_index_emit(Inputs in, const uint32_t* in_blk0, Blocks blk) {
  __shared__ uint32_t counts[256];
  const uint32_t g = blockIdx.x;
  if (in.idx_size[g] == ~0ull || in.nblk[g] == 0) return;
  const uint8_t* c = (const uint8_t*)in.ptr[g] + in.idx_off[g];
  const uint64_t size = in.idx_size[g];
  const uint32_t nr = rd_u32_bytes(c + size - 4);
  const uint64_t data_end = size - 4 - 4ull * nr;
  const uint32_t per = (nr + blockDim.x - 1) / blockDim.x;
  const uint32_t k0 = threadIdx.x * per;
  const uint32_t k1 = min(nr, k0 + per);
  uint32_t cnt = 0;
  for (uint32_t k = k0; k < k1; k++) {
    const uint64_t o = rd_u32_bytes(c + data_end + 4ull * k);
    const uint64_t end = (k + 1 < nr) ? rd_u32_bytes(c + data_end + 4ull * (k + 1)) : data_end;
    WalkOut w = walk_interval<false>(c, data_end, o, end, [&](uint64_t, uint64_t, uint32_t, uint32_t, uint32_t) {});
    cnt += w.count;
  }
  counts[threadIdx.x] = cnt;
  __syncthreads();
  // exclusive prefix (simple serial scan by thread 0; 256 values)
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int i = 0; i < (int)blockDim.x; i++) {
      uint32_t v = counts[i];
      counts[i] = s;
      s += v;
    }
  }
  __syncthreads();
  uint32_t bidx = in_blk0[g] + counts[threadIdx.x];
  uint32_t local = counts[threadIdx.x];
  for (uint32_t k = k0; k < k1; k++) {
    const uint64_t o = rd_u32_bytes(c + data_end + 4ull * k);
    const uint64_t end = (k + 1 < nr) ? rd_u32_bytes(c + data_end + 4ull * (k + 1)) : data_end;
    walk_interval<false>(c, data_end, o, end,
                         [&](uint64_t eo, uint64_t hdr, uint32_t, uint32_t ns, uint32_t vlen) {
      const uint8_t* v = c + eo + hdr + ns;
      uint64_t boff, bsz;
      uint32_t x = get_varint64(v, v + vlen, &boff);
      get_varint64(v + x, v + vlen, &bsz);
      blk.off[bidx] = boff;
      blk.size[bidx] = (uint32_t)bsz;
      blk.input[bidx] = g;
      blk.local[bidx] = local;
      bidx++;
      local++;
    });
  }
}

// ---------------------------------------------------------------------------
// k_decode

__device__ inline unsigned long long lb_load(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void lb_store(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of the per-block aggregates for ticket t (lane 0 only).
// A predecessor's word is published before it waits on anything, and tickets
// are taken only by running waves, so the wait always ends; a spin limit
// turns a lost word into a device error instead of a hang.
__device__ inline uint64_t lookback(unsigned long long* look, uint32_t t, uint64_t agg,
                                    uint32_t* dev_flags) {
  if (t == 0) {
    lb_store(&look[0], LB_INC | agg);
    return 0;
  }
  lb_store(&look[t], LB_AGG | agg);
  uint64_t excl = 0;
  int64_t j = (int64_t)t - 1;
  uint32_t spins = 0;
  while (j >= 0) {
    unsigned long long w = lb_load(&look[j]);
    unsigned long long f = w & ~LB_VAL;
    if (f == 0) {
      if (++spins > (1u << 24)) {
        atomicOr(dev_flags, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += w & LB_VAL;
    if (f == LB_INC) break;
    j--;
  }
  lb_store(&look[t], LB_INC | (excl + agg));
  return excl;
}



__global__ void __launch_bounds__(512) k_decode(DecodeArgs A) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  CrcLds* T = (CrcLds*)smem;
  load_crc_tables(T, A.g_crc, threadIdx.x, blockDim.x);
  __syncthreads();
  const uint32_t wv = threadIdx.x / WAVE;
  const uint32_t l = lane_id();
  uint8_t* stage = smem + sizeof(CrcLds) + (size_t)wv * A.stage_bytes;
  uint8_t* stage_end = stage + A.stage_bytes;
  uint32_t my_maxk = 0;

  for (;;) {
    uint32_t t = 0;
    if (l == 0) t = atomicAdd(A.ticket, 1u);
    t = __shfl(t, 0, WAVE);
    if (t >= A.blk.n) break;
    const uint32_t b = t;
    const uint32_t g = A.blk.input[b];
    const uint32_t job = A.in.job[g], loc = A.in.local[g];
    const uint32_t kblk = A.blk.local[b];
    const uint8_t* msg = (const uint8_t*)A.in.ptr[g] + A.blk.off[b];
    const uint32_t size = A.blk.size[b];
    const uint32_t n = size + 1;  // contents + type byte
    uint64_t ekey = ERR_NONE;
    uint32_t agg = 0;

    // stage: 16-byte chunks aligned to the message end
    const uint32_t J = (n + 15) / 16;
    for (uint32_t j = l; j < J; j += WAVE) {
      const int64_t p0 = (int64_t)n - 16ll * (J - j);
      uint8_t* dst = stage_end - 16ull * (J - j);
      if (p0 >= 0) {
        uint4 v;
        __builtin_memcpy(&v, msg + p0, 16);
        *(uint4*)dst = v;
      } else {
        for (int q = 0; q < 16; q++)
          if (p0 + q >= 0) dst[q] = msg[p0 + q];
      }
    }
    wave_sync();
    const uint32_t crc = wave_crc_lds(stage_end, n, T);
    const uint32_t stored = crc_unmask(ldg_u32_unaligned(msg + n));
    const uint8_t* c = stage_end - n;  // contents in LDS
    if (crc != stored) {
      ekey = err_key(loc, W_DATA, kblk, P_TRAILER, 0, EC_CHECKSUM);
    } else if (c[size] != 0) {
      ekey = err_key(loc, W_DATA, kblk, P_TRAILER, 0, EC_UNSUPPORTED);
    }
    uint32_t nr = 0;
    uint64_t data_end = 0;
    if (ekey == ERR_NONE) {
      uint64_t eo = check_restart_count(c, size, &nr);
      if (eo != ~0ull) ekey = err_key(loc, W_DATA, kblk, P_RESTARTS, eo, EC_FORMAT);
    }
    if (ekey == ERR_NONE) {
      data_end = size - 4 - 4ull * nr;
      uint64_t k_bad = ERR_NONE;
      for (uint32_t k = l; k < nr; k += WAVE)
        if (bad_restart(c, data_end, k)) { k_bad = k; break; }
      k_bad = wave_min64(k_bad);
      if (k_bad != ERR_NONE) ekey = err_key(loc, W_DATA, kblk, P_RESTARTS, data_end + 4 * k_bad, EC_FORMAT);
    }
    // walk 1: count and validate each restart interval.  Entries before the
    // block's first format error are still placed, so that a type or order
    // error among them (found later, on restored keys) is reported first.
    uint64_t first_bad = ~0ull;
    if (ekey == ERR_NONE) {
      for (uint32_t k0 = 0; k0 < nr; k0 += WAVE) {
        const uint32_t k = k0 + l;
        if (k < nr) {
          const uint64_t o = rd_u32_bytes(c + data_end + 4ull * k);
          const uint64_t end = (k + 1 < nr) ? rd_u32_bytes(c + data_end + 4ull * (k + 1)) : data_end;
          WalkOut w = walk_interval<true>(c, data_end, o, end, [](uint64_t, uint64_t, uint32_t, uint32_t, uint32_t) {});
          if (w.err_off < first_bad) first_bad = w.err_off;
          if (w.maxklen > my_maxk) my_maxk = w.maxklen;
        }
      }
      first_bad = wave_min64(first_bad);
      for (uint32_t k0 = 0; k0 < nr; k0 += WAVE) {
        const uint32_t k = k0 + l;
        if (k < nr) {
          const uint64_t o = rd_u32_bytes(c + data_end + 4ull * k);
          if (o < first_bad) {
            const uint64_t end = (k + 1 < nr) ? rd_u32_bytes(c + data_end + 4ull * (k + 1)) : data_end;
            agg += walk_interval<true>(c, data_end, o, end, [](uint64_t, uint64_t, uint32_t, uint32_t, uint32_t) {}).count;
          }
        }
      }
      agg = wave_sum(agg);
      if (first_bad != ~0ull) ekey = err_key(loc, W_DATA, kblk, P_ENTRIES, first_bad, EC_FORMAT);
    }
    if (ekey != ERR_NONE) {
      if (first_bad == ~0ull) agg = 0;  // trailer or restart array failure: nothing placed
      if (l == 0) report_err(&A.err[job], ekey);
    }
    // place the block's entries
    uint64_t excl = 0;
    if (l == 0) excl = lookback(A.blk.look, t, agg, A.dev_flags);
    excl = __shfl(excl, 0, WAVE);
    if (l == 0) {
      A.blk.e0[b] = excl;
      A.blk.ne[b] = agg;
    }
    if (agg) {
      // walk 2: write the entry records
      uint64_t running = excl;
      for (uint32_t k0 = 0; k0 < nr; k0 += WAVE) {
        const uint32_t k = k0 + l;
        uint32_t cnt = 0;
        uint64_t o = 0, end = 0;
        if (k < nr) {
          o = rd_u32_bytes(c + data_end + 4ull * k);
          end = (k + 1 < nr) ? rd_u32_bytes(c + data_end + 4ull * (k + 1)) : data_end;
          if (o < first_bad)
            cnt = walk_interval<true>(c, data_end, o, end, [](uint64_t, uint64_t, uint32_t, uint32_t, uint32_t) {}).count;
        }
        const uint32_t incl = wave_incl_scan(cnt);
        uint64_t e = running + incl - cnt;
        if (k < nr && cnt) {
          const uint64_t gaddr = (uint64_t)(uintptr_t)msg;
          walk_interval<true>(c, data_end, o, end,
                              [&](uint64_t eo, uint64_t hdr, uint32_t shared, uint32_t ns, uint32_t vlen) {
            if (e >= A.cap) { e++; return; }  // capacity retry: only the count matters
            A.tu.kd[e] = gaddr + eo + hdr;
            A.tu.sn[e] = (uint64_t)shared | ((uint64_t)ns << 32);
            A.tu.vp[e] = gaddr + eo + hdr + ns;
            A.tu.vlen[e] = vlen;
            A.tu.blk[e] = b;
            A.tu.eoff[e] = (uint32_t)eo;
            e++;
          });
        }
        running += __shfl(incl, WAVE - 1, WAVE);
      }
    }
    wave_sync();  // the stage is reused by the next block
  }
  my_maxk = wave_max(my_maxk);
  if (l == 0 && my_maxk) atomicMax(A.maxklen, my_maxk);
}

// ---------------------------------------------------------------------------
// k_keys: restore each internal key.  Byte q of entry e's key comes from the
// latest entry e' <= e (inside the same restart interval) whose shared count
// is <= q, at position q - shared(e') of e' 's key delta.

__global__ void k_keys(Tuples tu, Blocks blk, Inputs in, uint32_t kw8, uint64_t n,
                       unsigned long long* err) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint64_t sn = tu.sn[e];
  const uint32_t shared = (uint32_t)sn, ns = (uint32_t)(sn >> 32);
  const uint32_t klen = shared + ns;
  const uint32_t ulen = klen - 8;
  uint8_t* slot = (uint8_t*)(tu.heap + e * kw8);
  uint64_t tag = 0, kp0 = 0, kp1 = 0;
  uint32_t hi = klen;
  uint64_t cur = e;
  uint32_t s = shared;
  uint64_t src = tu.kd[e];
  for (;;) {
    if (s < hi) {
      const uint8_t* d = (const uint8_t*)src;
      for (uint32_t q = s; q < hi; q++) {
        const uint32_t byte = d[q - s];
        if (q < ulen) {
          slot[q] = (uint8_t)byte;
          if (q < 8) kp0 |= (uint64_t)byte << (8 * (7 - q));
          else if (q < 16) kp1 |= (uint64_t)byte << (8 * (15 - q));
        } else {
          tag |= (uint64_t)byte << (8 * (q - ulen));
        }
      }
      hi = s;
    }
    if (hi == 0) break;
    cur--;
    const uint64_t psn = tu.sn[cur];
    s = (uint32_t)psn;
    src = tu.kd[cur];
  }
  // zero padding of the slot
  for (uint32_t q = ulen; q < ((ulen + 7) & ~7u); q++) slot[q] = 0;
  for (uint32_t w = (ulen + 7) / 8; w < kw8; w++) tu.heap[e * kw8 + w] = 0;
  tu.kp0[e] = kp0;
  tu.kp1[e] = kp1;
  tu.tag[e] = tag;
  tu.ulen[e] = ulen;
  if ((tag & 0xFF) > 1) {
    const uint32_t b = tu.blk[e];
    const uint32_t g = blk.input[b];
    report_err(&err[in.job[g]], err_key(in.local[g], W_DATA, blk.local[b], P_ENTRIES, tu.eoff[e], EC_FORMAT));
  }
}

// k_order: entries of one table strictly increase; and for the first entry
// of every table after a job's first, how it compares with the previous
// table's last entry (in_cmp: -1 less, 0 equal, 1 greater, 2 no entries).
__global__ void k_order(Tuples tu, Blocks blk, Inputs in, const uint32_t* in_blk0, uint32_t kw8,
                        uint64_t n, int32_t* in_cmp, unsigned long long* err) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint32_t b = tu.blk[e];
  const uint32_t g = blk.input[b];
  const uint64_t first_e = blk.e0[in_blk0[g]];
  if (e != first_e) {
    if (cmp_ikeys(tu, kw8, e - 1, e) >= 0)
      report_err(&err[in.job[g]], err_key(in.local[g], W_DATA, blk.local[b], P_ENTRIES, tu.eoff[e], EC_UNSORTED));
  } else if (e > 0 && in.local[g] > 0) {
    const uint32_t pb = tu.blk[e - 1];
    const uint32_t pg = blk.input[pb];
    if (in.job[pg] == in.job[g] && pg == g - 1) in_cmp[g] = cmp_ikeys(tu, kw8, e - 1, e);
  }
}

}  // namespace luda
