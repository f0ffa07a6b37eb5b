// Checksums of long messages (index, filter and metaindex blocks) spread
// over many waves: a message is cut into segments of CRCM_SEG bytes aligned
// to its end and each wave folds whole segments on its own.  A message of
// one segment is finished by the wave that folds it; the segment checksums
// of longer ones are joined by k_crc_join, launched after k_crc_multi (the
// launch boundary orders the two, so no fence or counter is needed between
// waves).  raw(A || B) = raw(A) * x^(8 |B|) ^ raw(B), so the join is a
// Horner sum with multiplications by powers of x^(8 CRCM_SEG) mod P.
#pragma once
#include <algorithm>

#include "dev_common.h"

namespace luda {

constexpr uint32_t CRCM_WAVES = 16;  // waves per workgroup
constexpr uint32_t CRCM_SEG = 4096;  // bytes per segment (one wave step of four chunks per lane)
static_assert(CRCM_SEG == CRC_SEG_BYTES, "segment size shared with the host");
constexpr uint32_t CRCM_POWS = 7;  // x^(8 CRCM_SEG 2^k) mod P, k = 0..6, after the tables in the image

// Joins the checksums r[0..ns) of consecutive segments of CRCM_SEG bytes
// (the first may be shorter: it stands for its bytes only).  Lane l owns the
// segments c = l + 64 i counted from the end, folded first to last with a
// shift of 64 segments between them; lane l's sum is then shifted over the l
// segments after its last one.  Every lane must call; the result is in every
// lane.
__device__ inline uint32_t crcm_join(const uint32_t* r, uint64_t ns, const uint32_t* pows) {
  const uint32_t l = lane_id();
  uint32_t acc = 0;
  if (l < ns) {
    const uint64_t top = l + 64 * ((ns - 1 - l) / 64);  // this lane's first segment, from the end
    for (int64_t c = (int64_t)top; c >= 0; c -= 64) {
      const uint32_t v = r[ns - 1 - (uint64_t)c];
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
// (at least the sum over messages of ceil(n / CRCM_SEG)); mseg (count() + 1
// slots) receives each message's first segment and the total.  Messages are
// taken 1024 at a time: their spans are read in parallel and their segment
// counts summed in LDS, and segment w of the chunk goes to wave w mod (all
// waves of the grid).
template <class Msgs>
__global__ void __launch_bounds__(1024) k_crc_multi(Msgs M, const uint32_t* g_crc, uint32_t* part, uint64_t* mseg) {
  __shared__ CrcLds T;
  __shared__ uint64_t pre[1025];  // segments before message m0 + i of the chunk
  __shared__ uint64_t mp[1024], mn[1024];
  __shared__ uint64_t wsum[CRCM_WAVES];
  load_crc_tables(&T, g_crc, threadIdx.x, blockDim.x);
  const uint32_t nm = M.count();
  const uint32_t t = threadIdx.x, wv = t / WAVE;
  const uint64_t G = (uint64_t)gridDim.x * CRCM_WAVES, me = (uint64_t)blockIdx.x * CRCM_WAVES + wv;
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
    if (blockIdx.x == 0) {
      if (t < mc) mseg[m0 + t] = base + pre[t];
      if (t == 0 && m0 + mc == nm) mseg[nm] = base + total;
    }
    // the loop bounds and every branch below are the same in all lanes of a wave
    for (uint64_t w = base + (me + G - base % G) % G; w < base + total; w += G) {
      const uint64_t local = w - base;
      uint32_t lo = 0, hi = mc;  // pre[lo] <= local < pre[hi]
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= local) lo = mid;
        else hi = mid;
      }
      const uint64_t s = local - pre[lo], nsm = pre[lo + 1] - pre[lo], n = mn[lo];
      const uint8_t* p = (const uint8_t*)(uintptr_t)mp[lo];
      const int64_t s0 = (int64_t)n - (int64_t)(nsm - s) * CRCM_SEG;
      const uint32_t r = wave_raw_crc(&T, p, s0, CRCM_SEG);
      if (lane_id() == 0) {
        if (nsm == 1) M.finish(m0 + lo, r);
        else part[w] = r;
      }
    }
    base += total;
    __syncthreads();
  }
}

// Joins the segment checksums of the messages of more than one segment (one
// wave per message) and finishes them.
template <class Msgs>
__global__ void __launch_bounds__(256) k_crc_join(Msgs M, const uint32_t* g_crc, const uint32_t* part,
                                                  const uint64_t* mseg) {
  const uint32_t* pows = g_crc + sizeof(CrcLds11) / 4;
  const uint32_t nm = M.count();
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / WAVE);
  const uint64_t me = (uint64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  for (uint64_t m = me; m < nm; m += waves) {
    const uint64_t s0 = mseg[m], ns = mseg[m + 1] - s0;
    if (ns < 2) continue;
    const uint32_t raw = crcm_join(part + s0, ns, pows);
    if (lane_id() == 0) M.finish((uint32_t)m, raw);
  }
}

// both kernels over the messages of M (at most cap of them)
template <class Msgs>
void launch_crc_msgs(const Msgs& M, uint64_t cap, const uint32_t* g_crc, uint32_t* part, uint64_t* mseg,
                     uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_crc_multi<Msgs>, dim3(grid), dim3(1024), 0, st, M, g_crc, part, mseg);
  const uint32_t jg = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((cap + 3) / 4, 2048));
  hipLaunchKernelGGL(k_crc_join<Msgs>, dim3(jg), dim3(256), 0, st, M, g_crc, part, (const uint64_t*)mseg);
}

}  // namespace luda
