// Phase 3 planning kernels (paper Sec. II-A Phase 3: group pairs into data
// blocks by the block size, then data blocks into tables; Sec. III-C: the
// shared_key step computes each block's prefix-compressed keys).
//
// The writer's cuts are greedy and therefore a chain: a block that starts at
// survivor s ends at next(s) - 1, where next(s) is the first position whose
// running size estimate (entry bytes + 4 per restart point + 4) reaches the
// block size; entry sizes depend on the position inside the block (every R-th
// entry is a restart point and stores its key whole).  Block starts are the
// orbit of the job's first survivor under next().  Tables are cut the same way
// over block sizes.  The orbit is found without a sequential walk:
//   k_seg_exit     per chunk of 2048 items: next() for every item, then
//                  pointer doubling in LDS gives each item's exit from the
//                  chunk and the number of starts it passes on the way
//   k_seg_compose  per job: every chunk's true entry point and start count.
//                  Short steps: the chunks' entry->exit maps (offsets below
//                  the largest step) composed by a Hillis-Steele scan.  Long
//                  steps: in order over the chunks, where a chunk whose
//                  candidate entry points all leave it at the same exit needs
//                  no entry (the usual case: greedy chains merge within a few
//                  segments)
//   k_seg_mark     per chunk: marks the orbit from the entry point by doubling
//                  and writes the starts in order
#include "dev_common.h"
#include "kernels.h"

namespace luda {

__device__ inline uint32_t job_of(const uint64_t* starts, uint32_t J, uint64_t p) {
  uint32_t lo = 0, hi = J;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (starts[mid] <= p) lo = mid;
    else hi = mid;
  }
  return lo;
}

// longest common prefix of two internal keys (user key || fixed64 LE tag)
__device__ inline uint32_t lcp_ikeys(const Tuples& tu, uint32_t kw8, uint64_t a, uint64_t b) {
  const uint32_t la = tu.ulen[a], lb = tu.ulen[b];
  const uint32_t m = la < lb ? la : lb;
  const uint64_t* ha = tu.heap + a * kw8;
  const uint64_t* hb = tu.heap + b * kw8;
  uint32_t i = 0;
  for (uint32_t w = 0; w * 8 < m; w++) {
    uint64_t x = ha[w], y = hb[w];
    if (x != y) {
      uint32_t byte = w * 8 + (uint32_t)(__builtin_ctzll(x ^ y) >> 3);
      if (byte < m) return byte;
      break;
    }
  }
  i = m;
  const uint32_t ka = la + 8, kb = lb + 8;
  const uint32_t mk = ka < kb ? ka : kb;
  const uint8_t* sa = (const uint8_t*)ha;
  const uint8_t* sb = (const uint8_t*)hb;
  const uint64_t ta = tu.tag[a], tb = tu.tag[b];
  while (i < mk && ikey_byte(sa, la, ta, i) == ikey_byte(sb, lb, tb, i)) i++;
  return i;
}

// per survivor: shared prefix with the previous survivor of its job, and the
// encoded entry size as a restart point and as a delta entry
__global__ void k_prep(const uint32_t* surv, Tuples tu, uint32_t kw8, const uint64_t* job_s0, uint32_t J,
                       uint64_t S, uint32_t* sz_r, uint32_t* sz_n, uint32_t* shr, EncRec* rec) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint32_t j = job_of(job_s0, J, s);
  const uint64_t e = surv[s];
  const uint32_t ulen = tu.ulen[e];
  const uint32_t klen = ulen + 8;
  const uint32_t vlen = tu.vlen[e];
  const uint32_t shared = (s == job_s0[j]) ? 0 : lcp_ikeys(tu, kw8, surv[s - 1], e);
  sz_r[s] = 1 + varint_len(klen) + varint_len(vlen) + klen + vlen;
  sz_n[s] = varint_len(shared) + varint_len(klen - shared) + varint_len(vlen) + (klen - shared) + vlen;
  shr[s] = shared;
  EncRec r;
  r.vp = tu.vp[e];
  r.tag = tu.tag[e];
  r.e = (uint32_t)e;
  r.shared = shared;
  r.ulen = ulen;
  r.vlen = vlen;
  rec[s] = r;
}

struct BlockNext {
  static constexpr bool kStaged = true;
  const JobDesc* jobs;
  const SegJob* sj;
  const uint32_t* sz_r;
  const uint32_t* sz_n;
  // (4 items per step, their loads issued first; indices clamped to the
  // job's last item, extras unused)
  __device__ uint32_t operator()(uint32_t j, uint32_t i) const {
    const uint64_t base = sj[j].base;
    const uint32_t m = sj[j].m;
    const uint32_t R = jobs[j].restart_interval;
    const uint64_t bs = jobs[j].block_size;
    uint64_t E = 0;
    uint64_t nrest = 0;
    for (uint32_t t4 = i; t4 < m; t4 += 4) {
      uint32_t a[4];
#pragma unroll
      for (uint32_t q = 0; q < 4; q++) {
        const uint32_t t = min(t4 + q, m - 1);
        a[q] = (mod_r(t - i, R) == 0 ? sz_r : sz_n)[base + t];
      }
#pragma unroll
      for (uint32_t q = 0; q < 4; q++) {
        const uint32_t t = t4 + q;
        if (t >= m) break;
        if (mod_r(t - i, R) == 0) nrest++;
        E += a[q];
        if (E + 4 * nrest + 4 >= bs) return t + 1;
      }
    }
    return m;
  }
  // sizes of items [lo, hi) are also in LDS (SR, SN at item - lo)
  __device__ uint32_t staged(uint32_t j, uint32_t i, uint32_t lo, uint32_t hi, const uint32_t* SR,
                             const uint32_t* SN) const {
    const uint64_t base = sj[j].base;
    const uint32_t m = sj[j].m;
    const uint32_t R = jobs[j].restart_interval;
    const uint64_t bs = jobs[j].block_size;
    uint64_t E = 0;
    uint32_t r = 0;  // (t - i) % R
    uint64_t nrest = 0;
    for (uint32_t t = i; t < m; t++) {
      const bool in = t < hi;
      if (r == 0) {
        E += in ? SR[t - lo] : sz_r[base + t];
        nrest++;
      } else {
        E += in ? SN[t - lo] : sz_n[base + t];
      }
      if (++r == R) r = 0;
      if (E + 4 * nrest + 4 >= bs) return t + 1;
    }
    return m;
  }
};

struct FileNext {
  static constexpr bool kStaged = false;
  const JobDesc* jobs;
  const SegJob* sj;
  const uint64_t* ob_excl;
  const uint64_t* ob_full;
  __device__ uint32_t operator()(uint32_t j, uint32_t b) const {
    const uint64_t base = sj[j].base;
    const uint32_t m = sj[j].m;
    const uint64_t target = jobs[j].target_file_size;
    const uint64_t start = ob_excl[base + b];
    uint32_t lo = b, hi = m;
    while (lo < hi) {
      uint32_t mid = lo + (hi - lo) / 2;
      uint64_t incl = ob_excl[base + mid] + ob_full[base + mid];
      if (incl - start >= target) hi = mid;
      else lo = mid + 1;
    }
    return lo < m ? lo + 1 : m;
  }
};

constexpr uint32_t SEG_STAGE_MIN = 12;     // stage when the chunk's first segment has this many items
constexpr uint32_t SEG_COMPOSE_SCAN = 32;  // longest step for which compose scans the chunk maps

template <typename Next>
__global__ void __launch_bounds__(256) k_seg_exit(const SegChunk* ch, const uint32_t* nch_dev, const SegJob* sj,
                                                  Next nf, uint32_t* nxt, uint32_t* ex, uint32_t* cnt,
                                                  uint32_t* job_bmax) {
  __shared__ uint32_t P[2][SEG_C];
  __shared__ uint32_t K[2][SEG_C];
  __shared__ uint32_t sbm;
  const uint32_t c = blockIdx.x;
  if (c >= *nch_dev) return;
  const SegChunk k = ch[c];
  const uint32_t j = k.job;
  const uint64_t base = sj[j].base;
  const uint32_t c0 = k.start, c1 = k.end, len = c1 - c0;
  if (threadIdx.x == 0) sbm = 0;
  uint32_t bm = 0;
  uint32_t hi = 0;
  bool staged = false;
  if constexpr (Next::kStaged) {
    // Long segments (many items each): the sizes of this chunk are read into
    // LDS once, instead of each item's walk reading them again (items past
    // the chunk are read directly).  Short segments read them directly.
    if (threadIdx.x == 0) sbm = nf(j, c0) - c0;  // the first item's segment length
    __syncthreads();
    staged = sbm >= SEG_STAGE_MIN;
    __syncthreads();
    if (threadIdx.x == 0) sbm = 0;
    if (staged) {  // in the second doubling buffers, free until the doubling starts
      hi = c1;
      for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
        P[1][i] = nf.sz_r[base + c0 + i];
        K[1][i] = nf.sz_n[base + c0 + i];
      }
    }
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
    uint32_t v;
    if constexpr (Next::kStaged) v = staged ? nf.staged(j, c0 + i, c0, hi, P[1], K[1]) : nf(j, c0 + i);
    else v = nf(j, c0 + i);
    P[0][i] = v;
    K[0][i] = 1;
    nxt[base + c0 + i] = v;
    const uint32_t step = v - (c0 + i);
    bm = step > bm ? step : bm;
  }
  __syncthreads();
  atomicMax(&sbm, bm);
  uint32_t cur = 0;
  for (uint32_t r = 0; (1u << r) < len; r++) {
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
      const uint32_t p = P[cur][i];
      if (p < c1) {
        P[cur ^ 1][i] = P[cur][p - c0];
        K[cur ^ 1][i] = K[cur][i] + K[cur][p - c0];
      } else {
        P[cur ^ 1][i] = p;
        K[cur ^ 1][i] = K[cur][i];
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
    ex[base + c0 + i] = P[cur][i];
    cnt[base + c0 + i] = K[cur][i];
  }
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(&job_bmax[j], sbm);
}

// one workgroup per job; dynamic LDS holds two buffers of `cap` 16-bit
// entries (the scan) or cap chunks' common exits
__global__ void __launch_bounds__(256) k_seg_compose(const SegJob* sj, uint32_t J, const uint32_t* ex,
                                                     const uint32_t* cnt, const uint32_t* job_bmax,
                                                     uint32_t* chunk_entry, uint32_t* chunk_seg0,
                                                     uint32_t* job_nseg, uint32_t cap) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  __shared__ uint32_t wsum[4];
  const uint32_t j = blockIdx.x;
  if (j >= J) return;
  const uint64_t base = sj[j].base;
  const uint32_t m = sj[j].m, nch = sj[j].nchunks, ch0 = sj[j].chunk0;
  if (m == 0) {
    if (threadIdx.x == 0) job_nseg[j] = 0;
    return;
  }
  const uint32_t bm = job_bmax[j] ? job_bmax[j] : 1;
  // A segment spans at most bm items, so with bm <= SEG_C a chunk's entry
  // point (its first start) lies in its first bm items.  Chains of greedy
  // cuts from different starting points merge within a few segments, so the
  // exits from all those candidates are usually one and the same: then the
  // chunk's exit is known without its entry, and only chunks whose
  // candidates disagree need the entry of the chunk before them.
  uint32_t* conv = (uint32_t*)smem;  // per chunk: the common exit, or DIFFER
  const uint32_t DIFFER = 0xFFFFFFFEu;
  const uint16_t END = 0xFFFF;
  if (bm <= SEG_COMPOSE_SCAN && (uint64_t)nch * bm <= cap) {
    // short steps: the chunks' entry->exit maps (offsets below bm) composed
    // with a Hillis-Steele scan in LDS
    uint16_t* A = (uint16_t*)smem;
    uint16_t* B = A + cap;
    const uint32_t tot = nch * bm;
    for (uint32_t idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      const uint32_t c = idx / bm, o = idx % bm;
      const uint64_t item = (uint64_t)c * SEG_C + o;
      uint16_t v = END;
      if (item < m) {
        const uint32_t x = ex[base + item];
        if (x < m) v = (uint16_t)(x - (c + 1) * SEG_C);
      }
      A[idx] = v;
    }
    __syncthreads();
    for (uint32_t s = 1; s < nch; s <<= 1) {
      for (uint32_t idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const uint32_t c = idx / bm, o = idx % bm;
        if (c >= s) {
          const uint16_t u = A[(c - s) * bm + o];
          B[idx] = (u == END) ? END : A[c * bm + u];
        } else {
          B[idx] = A[idx];
        }
      }
      __syncthreads();
      uint16_t* t = A;
      A = B;
      B = t;
    }
    for (uint32_t c = threadIdx.x; c < nch; c += blockDim.x) {
      const uint32_t e = (c == 0) ? 0 : A[(c - 1) * bm];
      chunk_entry[ch0 + c] = (e == END) ? 0xFFFFFFFFu : c * SEG_C + e;
    }
  } else if (bm <= SEG_C && nch <= cap / 2) {
    // each chunk's first candidate's exit, then one pass over all candidates
    for (uint32_t c = threadIdx.x; c < nch; c += blockDim.x) conv[c] = ex[base + (uint64_t)c * SEG_C];
    __syncthreads();
    const uint64_t tot = (uint64_t)nch * bm;
    for (uint64_t idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      const uint32_t c = (uint32_t)(idx / bm), o = (uint32_t)(idx % bm);
      const uint64_t item = (uint64_t)c * SEG_C + o;
      if (o > 0 && item < m && ex[base + item] != ex[base + (uint64_t)c * SEG_C]) conv[c] = DIFFER;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t e = 0;
      for (uint32_t c = 0; c < nch; c++) {
        if (e >= m) {
          chunk_entry[ch0 + c] = 0xFFFFFFFFu;
          continue;
        }
        chunk_entry[ch0 + c] = e;
        if (e < (c + 1) * SEG_C) e = conv[c] != DIFFER ? conv[c] : ex[base + e];
      }
    }
  } else if (threadIdx.x == 0) {
    // long steps or too many chunks: walk the chunk exits in order
    uint32_t e = 0;
    for (uint32_t c = 0; c < nch; c++) {
      if (e >= m) {
        chunk_entry[ch0 + c] = 0xFFFFFFFFu;
        continue;
      }
      chunk_entry[ch0 + c] = e;
      if (e < (c + 1) * SEG_C) e = ex[base + e];
    }
  }
  __syncthreads();
  // starts per chunk, exclusive prefix over the job's chunks
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < nch; c0 += blockDim.x) {
    const uint32_t c = c0 + threadIdx.x;
    uint32_t v = 0;
    if (c < nch) {
      const uint32_t e = chunk_entry[ch0 + c];
      const uint32_t cend = min(m, (c + 1) * SEG_C);
      if (e != 0xFFFFFFFFu && e < cend) v = cnt[base + e];
    }
    uint32_t x = wave_incl_scan(v);
    if (lane_id() == WAVE - 1) wsum[threadIdx.x / WAVE] = x;
    __syncthreads();
    uint32_t pre = 0;
    for (uint32_t w = 0; w < threadIdx.x / WAVE; w++) pre += wsum[w];
    const uint32_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (c < nch) chunk_seg0[ch0 + c] = carry + pre + x - v;
    __syncthreads();
    carry += total;
  }
  if (threadIdx.x == 0) job_nseg[j] = carry;
}

__global__ void __launch_bounds__(256) k_seg_mark(const SegChunk* ch, const uint32_t* nch_dev, const SegJob* sj,
                                                  const uint32_t* nxt, const uint32_t* chunk_entry,
                                                  const uint32_t* chunk_seg0, const uint64_t* job_seg_base,
                                                  uint32_t* seg_first) {
  __shared__ uint32_t Jp[2][SEG_C];
  __shared__ uint32_t mark[SEG_C];
  __shared__ uint32_t wsum[4];
  const uint32_t c = blockIdx.x;
  if (c >= *nch_dev) return;
  const SegChunk k = ch[c];
  const uint32_t j = k.job;
  const uint64_t base = sj[j].base;
  const uint32_t c0 = k.start, c1 = k.end, len = c1 - c0;
  const uint32_t e = chunk_entry[c];
  if (e == 0xFFFFFFFFu || e < c0 || e >= c1) return;
  for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
    Jp[0][i] = nxt[base + c0 + i];
    mark[i] = (c0 + i == e) ? 1u : 0u;
  }
  __syncthreads();
  uint32_t cur = 0;
  for (uint32_t r = 0; (1u << r) < len; r++) {
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
      const uint32_t p = Jp[cur][i];
      if (mark[i] && p < c1) mark[p - c0] = 1u;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
      const uint32_t p = Jp[cur][i];
      Jp[cur ^ 1][i] = p < c1 ? Jp[cur][p - c0] : p;
    }
    __syncthreads();
    cur ^= 1;
  }
  // ranks of the marked items (each thread owns a contiguous run of 8)
  const uint32_t per = SEG_C / 256;
  const uint32_t i0 = threadIdx.x * per;
  uint32_t v = 0;
  for (uint32_t q = 0; q < per; q++)
    if (i0 + q < len) v += mark[i0 + q];
  uint32_t x = wave_incl_scan(v);
  if (lane_id() == WAVE - 1) wsum[threadIdx.x / WAVE] = x;
  __syncthreads();
  uint32_t pre = 0;
  for (uint32_t w = 0; w < threadIdx.x / WAVE; w++) pre += wsum[w];
  uint64_t out = job_seg_base[j] + chunk_seg0[c] + pre + x - v;
  for (uint32_t q = 0; q < per; q++)
    if (i0 + q < len && mark[i0 + q]) seg_first[out++] = c0 + i0 + q;
}

void launch_seg_exit_blocks(const SegChunk* ch, const uint32_t* nch_dev, uint32_t grid, const SegJob* sj,
                            const JobDesc* jobs, const uint32_t* sz_r, const uint32_t* sz_n, uint32_t* nxt,
                            uint32_t* ex, uint32_t* cnt, uint32_t* job_bmax, hipStream_t st) {
  BlockNext nf{jobs, sj, sz_r, sz_n};
  hipLaunchKernelGGL(k_seg_exit<BlockNext>, dim3(grid ? grid : 1), dim3(256), 0, st, ch, nch_dev, sj, nf, nxt, ex,
                     cnt, job_bmax);
}

void launch_seg_exit_files(const SegChunk* ch, const uint32_t* nch_dev, uint32_t grid, const SegJob* sj,
                           const JobDesc* jobs, const uint64_t* ob_excl, const uint64_t* ob_full, uint32_t* nxt,
                           uint32_t* ex, uint32_t* cnt, uint32_t* job_bmax, hipStream_t st) {
  FileNext nf{jobs, sj, ob_excl, ob_full};
  hipLaunchKernelGGL(k_seg_exit<FileNext>, dim3(grid ? grid : 1), dim3(256), 0, st, ch, nch_dev, sj, nf, nxt, ex,
                     cnt, job_bmax);
}

void launch_seg_mark(const SegChunk* ch, const uint32_t* nch_dev, uint32_t grid, const SegJob* sj,
                     const uint32_t* nxt, const uint32_t* chunk_entry, const uint32_t* chunk_seg0,
                     const uint64_t* job_seg_base, uint32_t* seg_first, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_mark, dim3(grid ? grid : 1), dim3(256), 0, st, ch, nch_dev, sj, nxt, chunk_entry,
                     chunk_seg0, job_seg_base, seg_first);
}

// ---------------------------------------------------------------------------
// chunk tables and per-job segment descriptors built on the device

// SegJob for each job from per-job base offsets and counts; chunks of SEG_C
__global__ void k_make_segjobs(const uint64_t* base_excl, const uint32_t* counts, uint32_t J, SegJob* sj,
                               SegChunk* ch, uint32_t* nch_out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  uint32_t c = 0;
  for (uint32_t j = 0; j < J; j++) {
    const uint32_t m = counts[j];
    const uint32_t n = (m + SEG_C - 1) / SEG_C;
    sj[j].base = base_excl[j];
    sj[j].m = m;
    sj[j].chunk0 = c;
    sj[j].nchunks = n;
    for (uint32_t q = 0; q < n; q++) {
      ch[c + q].job = j;
      ch[c + q].start = q * SEG_C;
      ch[c + q].end = min(m, (q + 1) * SEG_C);
    }
    c += n;
  }
  *nch_out = c;
}

// exclusive scan of J u32 values into u64 (J + 1 outputs), one workgroup
__global__ void k_small_scan(const uint32_t* v, uint32_t J, uint64_t* out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  uint64_t s = 0;
  for (uint32_t j = 0; j < J; j++) {
    out[j] = s;
    s += v[j];
  }
  out[J] = s;
}

// ---------------------------------------------------------------------------
// output blocks

// One thread per output block: its record (first entry, count, contents
// size, job), each entry's offset in the block and the value interior of
// each entry in the chunk grid of the block message (contents and type
// byte): the whole chunks between the first grid position at or after the
// value start and the last one at or before its end.  The entries of a
// wave's 64 consecutive blocks are one contiguous range; their offsets and
// interiors are assembled in LDS and stored contiguously (a range past
// BM_CAP entries, or one that is not contiguous, is stored directly).
constexpr uint32_t BM_WAVES = 4;   // waves per workgroup (the launch bound)
constexpr uint32_t BM_CAP = 256;   // staged entries per wave
constexpr uint32_t BM_U = 4;       // entries per loop step

struct BmStage {
  EntL e[BM_CAP];
  uint32_t off[BM_CAP];
};

__global__ void __launch_bounds__(BM_WAVES * 64) k_block_meta(const uint64_t* job_ob0, uint32_t J, const SegJob* sj_s,
                                                              const JobDesc* jobs, const uint32_t* seg_first,
                                                              const uint32_t* sz_r, const uint32_t* sz_n,
                                                              const EncRec* rec, uint64_t cap, OutBlocks ob,
                                                              uint32_t* ent_off, EntL* entl, uint32_t* gapcnt) {
  __shared__ BmStage stage_all[BM_WAVES];
  BmStage& S = stage_all[threadIdx.x / WAVE];
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nb = job_ob0[J];
  if (b < cap && b >= nb) {
    ob.full[b] = 0;
    gapcnt[b] = 0;
  }
  const bool in = b < cap && b < nb;  // the valid lanes of a wave are a prefix of it
  uint32_t j = 0, first = 0, end = 0, R = 1;
  uint64_t sbase = 0;
  if (in) {
    j = job_of(job_ob0, J, b);
    sbase = sj_s[j].base;
    first = seg_first[b];
    end = (b + 1 < job_ob0[j + 1]) ? seg_first[b + 1] : sj_s[j].m;
    R = jobs[j].restart_interval;
  }
  const uint64_t s0 = sbase + first, s1 = sbase + end;  // this block's entries [s0, s1)
  if (!__ballot(in)) return;
  // staged when the wave's entries are contiguous and few enough
  const uint64_t prev_end = ((uint64_t)(uint32_t)__shfl_up((int)(s1 >> 32), 1, WAVE) << 32) |
                            (uint32_t)__shfl_up((int)(uint32_t)s1, 1, WAVE);
  const bool gap = in && lane_id() > 0 && prev_end != s0;
  const int last = 63 - __builtin_clzll(__ballot(in));
  const uint64_t lo = ((uint64_t)(uint32_t)__shfl((int)(s0 >> 32), 0, WAVE) << 32) |
                      (uint32_t)__shfl((int)(uint32_t)s0, 0, WAVE);
  const uint64_t hi = ((uint64_t)(uint32_t)__shfl((int)(s1 >> 32), last, WAVE) << 32) |
                      (uint32_t)__shfl((int)(uint32_t)s1, last, WAVE);
  const bool staged = !__ballot(gap) && hi - lo <= BM_CAP;
  if (in) {
    const uint32_t cnt = end - first;
    // the loops take BM_U entries per step with all their loads issued
    // first (indices clamped to the block's last entry, extras unused)
    uint64_t E = 0;
    for (uint64_t s = s0; s < s1; s += BM_U) {
      uint32_t a[BM_U];
#pragma unroll
      for (uint32_t q = 0; q < BM_U; q++) {
        const uint64_t t = min(s + q, s1 - 1);
        a[q] = (mod_r((uint32_t)(t - s0), R) == 0 ? sz_r : sz_n)[t];
      }
#pragma unroll
      for (uint32_t q = 0; q < BM_U; q++)
        if (s + q < s1) E += a[q];
    }
    const uint64_t content = E + 4ull * div_r(cnt + R - 1, R) + 4;
    ob.s0[b] = s0;
    ob.cnt[b] = cnt;
    ob.size[b] = content;
    ob.full[b] = content + 5;
    ob.job[b] = j;
    const uint32_t n = (uint32_t)content + 1, J16 = (n + 15) / 16, gshift = 16 * J16 - n;
    uint32_t cum = 0, off = 0;
    for (uint64_t s4 = s0; s4 < s1; s4 += BM_U) {
      EncRec rq[BM_U];
      uint32_t zq[BM_U];
#pragma unroll
      for (uint32_t q = 0; q < BM_U; q++) {
        const uint64_t t = min(s4 + q, s1 - 1);
        rq[q] = rec[t];
        zq[q] = (mod_r((uint32_t)(t - s0), R) == 0 ? sz_r : sz_n)[t];
      }
#pragma unroll
      for (uint32_t q = 0; q < BM_U; q++) {
        const uint64_t s = s4 + q;
        if (s >= s1) break;
        const EncRec rc = rq[q];
        const uint32_t i = (uint32_t)(s - s0);
        const bool restart = mod_r(i, R) == 0;
        const uint32_t sh = restart ? 0u : rc.shared;
        const uint32_t ns = rc.ulen + 8 - sh;
        const uint32_t vs = off + varint_len(sh) + varint_len(ns) + varint_len(rc.vlen) + ns;
        const uint32_t en = vs + rc.vlen;
        const uint32_t ia = (vs + gshift + 15) / 16;  // first grid position >= vs is 16 ia - gshift
        const uint32_t iz = (en + gshift) / 16;       // last grid position <= en is 16 iz - gshift
        const uint32_t pieces = iz > ia ? iz - ia : 0;
        EntL L;
        L.vsrc = rc.vp - (uint64_t)vs - (uint64_t)gshift;
        L.ia = ia;
        L.pieces = pieces;
        L.cum = cum;
        L.pad = 0;
        if (staged) {
          S.e[s - lo] = L;
          S.off[s - lo] = off;
        } else {
          entl[s] = L;
          ent_off[s] = off;
        }
        cum += pieces;
        off += zq[q];
      }
    }
    gapcnt[b] = J16 - cum + 1;  // and the head slot
  }
  if (staged) {
    wave_sync();
    const uint32_t m = (uint32_t)(hi - lo);
    for (uint32_t q = lane_id(); q < m; q += WAVE) {
      entl[lo + q] = S.e[q];
      ent_off[lo + q] = S.off[q];
    }
    wave_sync();
  }
}

// per output file: block range, data bytes, filter window count
__global__ void k_file_pre(const uint64_t* job_f0, uint32_t J, const uint64_t* job_ob0,
                           const uint32_t* file_first, const uint64_t* ob_excl, uint64_t cap, OutFiles of) {
  const uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= cap) return;
  if (f >= job_f0[J]) {
    of.nwin[f] = 0;
    of.size[f] = 0;
    return;
  }
  const uint32_t j = job_of(job_f0, J, f);
  const uint64_t fb0 = job_ob0[j] + file_first[f];
  const uint64_t fb1 = (f + 1 < job_f0[j + 1]) ? job_ob0[j] + file_first[f + 1] : job_ob0[j + 1];
  of.job[f] = j;
  of.b0[f] = fb0;
  of.nb[f] = (uint32_t)(fb1 - fb0);
  of.data[f] = ob_excl[fb1] - ob_excl[fb0];
  const uint64_t o_last = ob_excl[fb1 - 1] - ob_excl[fb0];
  of.nwin[f] = (o_last >> FILTER_BASE_LG) + 1;
}

__device__ inline uint32_t find_sorted(const uint64_t* a, uint64_t n, uint64_t v) {
  // largest i < n with a[i] <= v
  uint64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    uint64_t mid = (lo + hi) / 2;
    if (a[mid] <= v) lo = mid;
    else hi = mid;
  }
  return (uint32_t)lo;
}

// per output block: its file, offset inside the file, filter window, index
// entry size; accumulates window key counts
__global__ void k_block_post(const uint64_t* nfiles_total, OutFiles of, const uint64_t* ob_excl,
                             const uint64_t* job_ob0, uint32_t J, Tuples tu, const uint32_t* surv,
                             uint64_t cap, OutBlocks ob, uint32_t* win_keys, uint32_t* win_fb) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= cap) return;
  if (b >= job_ob0[J]) {
    ob.ie_size[b] = 0;
    return;
  }
  const uint32_t f = find_sorted(of.b0, *nfiles_total, b);
  const uint64_t boff = ob_excl[b] - ob_excl[of.b0[f]];
  const uint32_t w = (uint32_t)(boff >> FILTER_BASE_LG);
  ob.file[b] = f;
  ob.off[b] = boff;
  atomicAdd(&win_keys[of.w0[f] + w], ob.cnt[b]);
  bool first_in_win = (b == of.b0[f]);
  if (!first_in_win) {
    const uint64_t pboff = ob_excl[b - 1] - ob_excl[of.b0[f]];
    first_in_win = (pboff >> FILTER_BASE_LG) != w;
  }
  if (first_in_win) win_fb[of.w0[f] + w] = (uint32_t)b;
  const uint64_t last = surv[ob.s0[b] + ob.cnt[b] - 1];
  const uint32_t klen = tu.ulen[last] + 8;
  const uint32_t hlen = varint_len(boff) + varint_len(ob.size[b]);
  ob.ie_size[b] = 1 + varint_len(klen) + varint_len(hlen) + klen + hlen;
}

// per filter window: filter bytes (0 for a window where no block starts)
__global__ void k_win_size(const uint64_t* nwin_total, const uint64_t* file_w0_sorted, uint64_t nfiles,
                           OutFiles of, const JobDesc* jobs, const uint32_t* win_keys, uint64_t cap,
                           uint64_t* win_bytes, uint32_t* win_file, uint32_t* max_bytes) {
  __shared__ uint32_t m;
  if (threadIdx.x == 0) m = 0;
  __syncthreads();
  const uint64_t nw = *nwin_total;
  uint32_t mine = 0;
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < cap; w += (uint64_t)gridDim.x * blockDim.x) {
    if (w >= nw) {
      win_bytes[w] = 0;
      continue;
    }
    const uint32_t f = find_sorted(file_w0_sorted, nfiles, w);
    win_file[w] = f;
    const uint32_t keys = win_keys[w];
    uint64_t v = 0;
    if (keys) {
      const uint64_t bpk = jobs[of.job[f]].bloom_bits_per_key;
      uint64_t bits = (uint64_t)keys * bpk;
      if (bits < 64) bits = 64;
      v = (bits + 7) / 8 + 1;
    }
    win_bytes[w] = v;
    const uint32_t vv = (uint32_t)(v > 0xFFFFFFF0ull ? 0xFFFFFFF0ull : v);
    mine = vv > mine ? vv : mine;
  }
  mine = wave_max(mine);
  if (lane_id() == 0 && mine) atomicMax(&m, mine);
  __syncthreads();
  if (threadIdx.x == 0 && m) atomicMax(max_bytes, m);
}

// per file: the layout of filter, metaindex and index blocks and the footer
__global__ void k_file_layout(const uint64_t* nfiles_total, OutFiles of, const uint64_t* win_off,
                              const uint64_t* ie_off, uint64_t cap) {
  const uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= cap) return;
  if (f >= *nfiles_total) {
    of.size[f] = 0;
    return;
  }
  const uint64_t w0 = of.w0[f], nw = of.nwin[f];
  const uint64_t fb0 = of.b0[f], nb = of.nb[f];
  const uint64_t filters = win_off[w0 + nw] - win_off[w0];
  const uint64_t filter_off = of.data[f];
  const uint64_t filter_size = filters + 4 * nw + 4 + 1;
  const uint64_t meta_off = filter_off + filter_size + 5;
  const uint64_t hl = varint_len(filter_off) + varint_len(filter_size);
  const uint64_t meta_size = 3 + 23 + hl + 8;
  const uint64_t index_off = meta_off + meta_size + 5;
  const uint64_t index_size = (ie_off[fb0 + nb] - ie_off[fb0]) + 4 * nb + 4;
  of.filter_off[f] = filter_off;
  of.filter_size[f] = filter_size;
  of.meta_off[f] = meta_off;
  of.meta_size[f] = meta_size;
  of.index_off[f] = index_off;
  of.index_size[f] = index_size;
  of.size[f] = index_off + index_size + 5 + 48;
}

}  // namespace luda
