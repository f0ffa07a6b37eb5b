// Checksums of long messages (index, filter and metaindex blocks) spread
// over many workgroups: a message is cut into segments of CRCM_SEG bytes
// aligned to its end, each workgroup folds whole segments (a wave per KiB),
// and the last workgroup to finish a message joins its segment checksums.
// raw(A || B) = raw(A) * x^(8 |B|) ^ raw(B), so the join is a Horner sum
// with multiplications by powers of x^(8 CRCM_SEG) mod P.
#pragma once
#include "dev_common.h"

namespace luda {

constexpr uint32_t CRCM_WAVES = 16;
constexpr uint32_t CRCM_SEG = CRCM_WAVES * 1024;
static_assert(CRCM_SEG == CRC_SEG_BYTES, "segment size shared with the host");
constexpr uint32_t CRCM_POWS = 7;  // x^(8 CRCM_SEG 2^k) mod P, k = 0..6, after the tables in the image

// Joins the checksums r[0..ns) of consecutive segments of CRCM_SEG bytes
// (the first may be shorter: it stands for its bytes only).  Lane l owns the
// segments c = l + 64 i counted from the end, folded first to last with a
// shift of 64 segments between them; lane l's sum is then shifted over the l
// segments after its last one.  Every lane must call; the result is in every
// lane.
__device__ inline uint32_t crcm_join(uint32_t* r, uint64_t ns, const uint32_t* pows) {
  const uint32_t l = lane_id();
  uint32_t acc = 0;
  if (l < ns) {
    const uint64_t top = l + 64 * ((ns - 1 - l) / 64);  // this lane's first segment, from the end
    for (int64_t c = (int64_t)top; c >= 0; c -= 64) {
      const uint32_t v = __hip_atomic_load(r + (ns - 1 - (uint64_t)c), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      acc = gf2_mulmod(acc, pows[6]) ^ v;
    }
#pragma unroll
    for (int k = 0; k < 6; k++)
      if (l & (1u << k)) acc = gf2_mulmod(acc, pows[k]);
  }
#pragma unroll
  for (int k = 0; k < 6; k++) acc ^= __shfl_xor(acc, 1 << k, WAVE);
  return acc;
}

// Msgs provides count(), span(m, &p, &n) (message m: n bytes at p; n = 0:
// none), finish(m, raw) (once per message with n > 0, by one thread) and
// empty(m) (once per message with n = 0).  part holds one slot per segment
// (at least the sum over messages of ceil(n / CRCM_SEG)); ticket one counter
// per message, zero at launch and left at zero.  Messages are taken 1024 at
// a time: their spans are read in parallel and their segment counts summed
// in LDS, and segment w of the chunk goes to workgroup w mod gridDim.x.
template <class Msgs>
__global__ void __launch_bounds__(1024) k_crc_multi(Msgs M, const uint32_t* g_crc, uint32_t* part,
                                                    uint32_t* ticket) {
  __shared__ CrcLds T;
  __shared__ uint64_t pre[1025];  // segments before message m0 + i of the chunk
  __shared__ uint64_t mp[1024], mn[1024];
  __shared__ uint64_t wsum[CRCM_WAVES];
  __shared__ uint32_t wpart[CRCM_WAVES];
  __shared__ uint32_t last;
  load_crc_tables(&T, g_crc, threadIdx.x, blockDim.x);
  const uint32_t* pows = g_crc + sizeof(CrcLds11) / 4;
  const uint32_t nm = M.count();
  const uint32_t t = threadIdx.x, wv = t / WAVE;
  const uint64_t G = gridDim.x;
  uint64_t base = 0;  // segments of the chunks before this one
  for (uint32_t m0 = 0; m0 < nm; m0 += 1024) {
    const uint32_t mc = min(nm - m0, 1024u);
    uint64_t ns = 0;
    if (t < mc) {
      const uint8_t* p;
      uint64_t n;
      M.span(m0 + t, &p, &n);
      mp[t] = (uint64_t)(uintptr_t)p;
      mn[t] = n;
      ns = (n + CRCM_SEG - 1) / CRCM_SEG;
      if (ns == 0 && blockIdx.x == 0) M.empty(m0 + t);
    }
    const uint64_t inc = wave_incl_scan64(ns);
    if (lane_id() == WAVE - 1) wsum[wv] = inc;
    __syncthreads();
    uint64_t before = 0;
    for (uint32_t k = 0; k < wv; k++) before += wsum[k];
    pre[t + 1] = before + inc;
    if (t == 0) pre[0] = 0;
    __syncthreads();
    const uint64_t total = pre[mc];
    for (uint64_t w = base + (blockIdx.x + G - base % G) % G; w < base + total; w += G) {
      const uint64_t local = w - base;
      uint32_t lo = 0, hi = mc;  // pre[lo] <= local < pre[hi]
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= local) lo = mid;
        else hi = mid;
      }
      const uint64_t s = local - pre[lo], nsm = pre[lo + 1] - pre[lo], n = mn[lo];
      const uint8_t* p = (const uint8_t*)(uintptr_t)mp[lo];
      const int64_t s0 = (int64_t)n - (int64_t)(nsm - s) * CRCM_SEG + (int64_t)wv * 1024;
      const uint32_t r = (s0 + 1024 > 0) ? wave_raw_crc(&T, p, s0, 1024) : 0u;
      if (lane_id() == 0) wpart[wv] = r;
      __syncthreads();
      if (t == 0) {
        uint32_t acc = 0;
        for (uint32_t k = 0; k < CRCM_WAVES; k++) acc = crc_shift(T.sh[6], acc) ^ wpart[k];
        part[w] = acc;
        __threadfence();
        last = atomicAdd(&ticket[m0 + lo], 1u) + 1 == nsm;
      }
      __syncthreads();
      if (last && wv == 0) {
        __threadfence();
        const uint32_t raw = crcm_join(part + (w - s), nsm, pows);
        if (lane_id() == 0) {
          M.finish(m0 + lo, raw);
          ticket[m0 + lo] = 0;
        }
      }
      __syncthreads();
    }
    base += total;
    __syncthreads();
  }
}

}  // namespace luda
