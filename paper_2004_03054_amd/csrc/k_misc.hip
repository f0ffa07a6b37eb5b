// Small bookkeeping kernels between the pipeline stages: totals, ranges,
// maxima and type conversions the host reads back or the next stage needs.
#include "dev_common.h"
#include "kernels.h"

namespace luda {

// gather device values into pinned host memory (one launch per readback)
__global__ void k_mail(MailSegs m, uint8_t* mail) {
  const uint32_t s = blockIdx.x;
  if (s >= m.n) return;
  const uint8_t* src = (const uint8_t*)m.src[s];
  uint8_t* dst = mail + m.dst[s];
  for (uint32_t i = threadIdx.x; i < m.bytes[s]; i += blockDim.x) dst[i] = src[i];
}

__global__ void k_mail_flag(uint64_t* flag, uint64_t seq) {
  if (threadIdx.x == 0 && blockIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// scatter host-staged bytes (pinned host memory) to device buffers
__global__ void k_upload(UpSegs u, const uint8_t* up) {
  const uint32_t s = blockIdx.x;
  if (s >= u.n) return;
  const uint8_t* src = up + u.src[s];
  uint8_t* dst = (uint8_t*)u.dst[s];
  const uint32_t nb = u.bytes[s];
  const uint32_t nw = nb / 8;
  for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) ((uint64_t*)dst)[i] = ((const uint64_t*)src)[i];
  for (uint32_t i = nw * 8 + threadIdx.x; i < nb; i += blockDim.x) dst[i] = src[i];
}

__global__ void k_gather_u64(const uint64_t* src, const uint64_t* idx, uint32_t n, uint64_t* out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = src[idx[i]];
}

// first output of each group: out[x] = ient[ibase[blk0_of ? blk0_of[x] : x]]
__global__ void k_ranges(const uint64_t* ient, const uint64_t* ibase, const uint64_t* blk0_of, uint32_t n,
                         uint64_t* out) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) out[x] = ient[ibase[blk0_of ? blk0_of[x] : x]];
}

__global__ void k_job_surv(const uint64_t* job_e0, const uint32_t* kpos, uint32_t J, uint64_t* job_s0) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j <= J) job_s0[j] = kpos[job_e0[j]];
}

__global__ void k_plan_stats(OutBlocks ob, const uint64_t* job_ob0, uint32_t J, uint64_t cap,
                             const uint32_t* gapcnt, uint32_t* stats) {
  __shared__ uint32_t m0, m1;
  if (threadIdx.x == 0) {
    m0 = 0;
    m1 = 0;
  }
  __syncthreads();
  const uint64_t nb = job_ob0[J];
  uint32_t sz = 0, cn = 0, tiny = 0, off = 0, em = 0;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb && b < cap;
       b += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t s = ob.size[b], c = ob.cnt[b];
    sz = max(sz, s);
    cn = max(cn, c);
    if (s < 15) tiny = 1;  // a message (contents + type byte) under 16 bytes
    off += enc_pipelined(s, c) ? 0 : 1;
    em += gap_em_block(c, s, gapcnt[b]) ? 1 : 0;
  }
  if (__ballot(tiny) && lane_id() == 0) atomicMax(&stats[2], 1u);
  off = wave_sum(off);
  if (off && lane_id() == 0) atomicAdd(&stats[3], off);
  em = wave_sum(em);
  if (em && lane_id() == 0) atomicAdd(&stats[4], em);
  sz = wave_max(sz);
  cn = wave_max(cn);
  if (lane_id() == 0) {
    atomicMax(&m0, sz);
    atomicMax(&m1, cn);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(&stats[0], m0);
    atomicMax(&stats[1], m1);
  }
}

// encoder records of the output blocks (after the file layout)
__global__ void k_block_dst(OutBlocks ob, OutFiles of, const JobDesc* jobs, const uint64_t* nblocks, uint64_t cap,
                            BlockRec* br, uint64_t* big_list, uint32_t* big_n, uint64_t big_cap) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = b < cap && b < *nblocks;
  BlockRec r{};
  if (in) {
    r.dst = of.out[ob.file[b]] + ob.off[b];
    r.s0 = ob.s0[b];
    r.cnt = ob.cnt[b];
    r.size = ob.size[b];
    r.R = jobs[ob.job[b]].restart_interval;
    r.pad = 0;
    br[b] = r;
  }
  if (!big_list) return;
  // one atomic per wave for its off-path blocks
  const bool big = in && !enc_pipelined(r.size, r.cnt);
  const uint64_t m = __ballot(big);
  if (!m) return;
  uint32_t base = 0;
  if (lane_id() == (uint32_t)__builtin_ctzll(m)) base = atomicAdd(big_n, (uint32_t)__popcll(m));
  base = (uint32_t)__shfl((int)base, __builtin_ctzll(m), WAVE);
  const uint64_t at = (uint64_t)base + __popcll(m & ((1ull << lane_id()) - 1));
  if (big && at < big_cap) big_list[at] = b;
}

// Per file: its entry count, and where its smallest and largest internal
// keys lie inside the file (the key range a store installs the new table
// under).  Both are stored whole: the first entry of the first data block is
// a restart point (shared 0), and every index entry is a restart point whose
// key is the last internal key of its block.
__global__ void k_file_entries(OutFiles of, OutBlocks ob, const uint32_t* surv, Tuples tu, const uint64_t* ie_off,
                               uint64_t nf, const uint8_t* ztype) {
  const uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const uint64_t b0 = of.b0[f], last = b0 + of.nb[f] - 1;
  of.entries[f] = ob.s0[last] + ob.cnt[last] - ob.s0[b0];
  const uint32_t e0 = surv[ob.s0[b0]];
  const uint32_t k0 = tu.ulen[e0] + 8;
  // first data block at file offset 0: varint shared (1 byte), non_shared, value length, key;
  // when that block is stored compressed, the key is kept right after the table
  of.keyr[4 * f + 0] = (ztype && ztype[b0]) ? of.size[f] : 1 + varint_len(k0) + varint_len(tu.vlen[e0]);
  of.keyr[4 * f + 1] = k0;
  const uint32_t e1 = surv[ob.s0[last] + ob.cnt[last] - 1];
  const uint32_t k1 = tu.ulen[e1] + 8;
  const uint32_t hlen = varint_len(ob.off[last]) + varint_len(ob.size[last]);
  // last index entry: varint shared (1 byte), non_shared, handle length, key
  of.keyr[4 * f + 2] = of.index_off[f] + (ie_off[last] - ie_off[b0]) + 1 + varint_len(k1) + varint_len(hlen);
  of.keyr[4 * f + 3] = k1;
}

}  // namespace luda

namespace luda {

// table writer input: ordered entries given as struct-of-arrays on the device
__global__ void k_ingest_max(const uint64_t* koff, uint64_t n, uint32_t* maxlen) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t v = 0;
  if (i < n) {
    const uint64_t l = koff[i + 1] - koff[i];
    v = l > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)l;
  }
  v = wave_max(v);
  if (lane_id() == 0) atomicMax(maxlen, v);
}

__global__ void k_ingest(const uint8_t* keys, const uint64_t* koff, const uint64_t* tags, const uint8_t* vals,
                         const uint64_t* voff, uint64_t n, Tuples tu, uint32_t kw8, uint32_t* surv) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k0 = koff[i];
  const uint32_t ulen = (uint32_t)(koff[i + 1] - k0);
  uint64_t* slot = tu.heap + i * kw8;
  uint64_t kp0 = 0, kp1 = 0;
  for (uint32_t w = 0; w < kw8; w++) {
    uint64_t word = 0;
    for (uint32_t b = 0; b < 8; b++) {
      const uint32_t q = w * 8 + b;
      if (q < ulen) {
        const uint64_t byte = keys[k0 + q];
        word |= byte << (8 * b);
        if (q < 8) kp0 |= byte << (8 * (7 - q));
        else if (q < 16) kp1 |= byte << (8 * (15 - q));
      }
    }
    slot[w] = word;
  }
  tu.kp0[i] = kp0;
  tu.kp1[i] = kp1;
  tu.tag[i] = tags[i];
  tu.ulen[i] = ulen;
  tu.vp[i] = (uint64_t)(uintptr_t)(vals + voff[i]);
  tu.vlen[i] = (uint32_t)(voff[i + 1] - voff[i]);
  surv[i] = (uint32_t)i;
}

__global__ void k_check_sorted(Tuples tu, uint32_t kw8, uint64_t n, uint32_t* bad) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 || i >= n) return;
  if (cmp_ikeys(tu, kw8, i - 1, i) >= 0) atomicOr(bad, 1u);
}

}  // namespace luda
