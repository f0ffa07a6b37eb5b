// Phase 2 "(Delete and) Sort" kernels (paper Sec. II-A Phase 2): merge all
// restored entries in key order and drop stale versions.  The paper sorts
// <K, V_offset> tuples instead of key-value pairs (Sec. III-D, lightweight
// sort); here the tuples are entry indices and every input table is already a
// sorted run, so the global order comes from merge-path merges of runs.
//
//   k_iota         identity order
//   k_merge        merge-path: each thread finds its diagonal split by binary
//                  search and merges ITEMS outputs
//   k_dedup_flags  keep the first (newest) entry of every user key, drop it
//                  too if it is a deletion at the bottom level
//   k_scatter      compact the kept entries
//   scans          tiled exclusive prefix sums (u32 / u64)
#include "dev_common.h"
#include "kernels.h"

namespace luda {

__global__ void k_iota(uint32_t* idx, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) idx[i] = (uint32_t)i;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

constexpr uint32_t MERGE_ITEMS = 8;

__global__ void k_merge(const MergeTask* tasks, uint32_t ntasks, const uint32_t* src, uint32_t* dst,
                        Tuples tu, uint32_t kw8, uint64_t total) {
  uint64_t p = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * MERGE_ITEMS;
  if (p >= total) return;
  const uint64_t p_end = p + MERGE_ITEMS < total ? p + MERGE_ITEMS : total;
  // the thread's outputs may straddle task boundaries (tasks tile [0, total))
  while (p < p_end) {
    uint32_t lo = 0, hi = ntasks;
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) / 2;
      if (tasks[mid].out0 <= p) lo = mid;
      else hi = mid;
    }
    const MergeTask T = tasks[lo];
    const uint64_t d = p - T.out0;
    const uint64_t len = (uint64_t)T.la + T.lb;
    const uint64_t dend = (T.out0 + len < p_end ? T.out0 + len : p_end) - T.out0;
    const uint32_t* A = src + T.a0;
    const uint32_t* B = src + T.b0;
    // merge-path split: number of A elements among the first d outputs
    uint64_t l2 = d > T.lb ? d - T.lb : 0, h2 = d < T.la ? d : T.la;
    while (l2 < h2) {
      uint64_t mid = (l2 + h2) / 2;
      if (cmp_entries(tu, kw8, A[mid], B[d - mid - 1]) < 0) l2 = mid + 1;
      else h2 = mid;
    }
    uint64_t i = l2, j = d - l2;
    for (uint64_t q = d; q < dend; q++) {
      uint32_t v;
      if (i < T.la && (j >= T.lb || cmp_entries(tu, kw8, A[i], B[j]) < 0)) v = A[i++];
      else v = B[j++];
      dst[T.out0 + q] = v;
    }
    p = T.out0 + dend;
  }
}

__device__ inline uint32_t find_job(const uint64_t* starts, uint32_t J, uint64_t p) {
  // starts: J + 1 ascending values; the job j with starts[j] <= p < starts[j+1]
  uint32_t lo = 0, hi = J;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (starts[mid] <= p) lo = mid;
    else hi = mid;
  }
  return lo;
}

// live snapshots below sequence number q (lower bound in an ascending list):
// two versions are seen by the same snapshot readers iff it is equal for both
__device__ inline uint32_t snap_stripe(const uint64_t* s, uint32_t n, uint64_t q) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (s[mid] < q) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Drop rule, per sorted position p (versions of a user key are adjacent,
// newest first).  A version is kept iff a reader sees it: it is the newest
// of its key, or a live snapshot lies between it and the next newer version
// (different stripes).  At the bottom level a kept deletion is dropped too
// unless a kept value of its key is older.  With no snapshots: the newest
// version is kept, and a kept deletion is dropped at the bottom level.
__global__ void __launch_bounds__(1024) k_dedup_flags(const uint32_t* ord, Tuples tu, uint32_t kw8, const JobDesc* jobs,
                                                     const uint64_t* snaps, const uint64_t* job_e0, uint32_t J,
                                                     uint64_t n, uint32_t* keep, unsigned long long* shadowed,
                                                     unsigned long long* tomb, const uint32_t* active) {
  if ((uint64_t)blockIdx.x * blockDim.x >= n) return;  // the whole workgroup
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = p < n;
  uint32_t j = 0;
  bool shadow = false, drop_del = false;
  if (live) {
    j = find_job(job_e0, J, p);
    if (!active[j]) {
      keep[p] = 0;
    } else {
      const uint32_t e = ord[p];
      const JobDesc jd = jobs[j];
      const bool first = (p == job_e0[j]) || !same_user_key(tu, kw8, ord[p - 1], e);
      const bool del = (tu.tag[e] & 0xFF) == 0;
      bool kept = first;
      if (jd.n_snap) {
        const uint64_t* S = snaps + jd.snap_first;
        const uint32_t se = snap_stripe(S, jd.n_snap, tu.tag[e] >> 8);
        kept = first || se != snap_stripe(S, jd.n_snap, tu.tag[ord[p - 1]] >> 8);
        if (kept && del && jd.bottommost) {
          // the older versions of the key, newest first: is one a kept value?
          bool older_value = false;
          uint32_t sprev = se;
          for (uint64_t q = p + 1; q < job_e0[j + 1]; q++) {
            const uint32_t f = ord[q];
            if (!same_user_key(tu, kw8, ord[q - 1], f)) break;
            const uint32_t sq = snap_stripe(S, jd.n_snap, tu.tag[f] >> 8);
            if (sq != sprev && (tu.tag[f] & 0xFF) != 0) {
              older_value = true;
              break;
            }
            sprev = sq;
          }
          drop_del = !older_value;
        }
      } else {
        drop_del = first && jd.bottommost && del;
      }
      shadow = !kept;
      keep[p] = (kept && !drop_del) ? 1u : 0u;
    }
  }
  // counts: one global atomic per workgroup when the whole workgroup is in
  // one job (atomics on one address serialise), per thread otherwise
  __shared__ unsigned long long s_sh, s_td;
  if (threadIdx.x == 0) {
    s_sh = 0;
    s_td = 0;
  }
  const uint64_t p0 = (uint64_t)blockIdx.x * blockDim.x;
  const uint64_t plast = min(p0 + blockDim.x, n) - 1;  // p0 < n: grid sized to n
  const uint32_t ja = find_job(job_e0, J, p0), jb = find_job(job_e0, J, plast);
  __syncthreads();
  if (ja == jb) {
    const uint32_t ns = (uint32_t)__popcll(wave_ballot(shadow));
    const uint32_t nd = (uint32_t)__popcll(wave_ballot(drop_del));
    if (lane_id() == 0) {
      if (ns) atomicAdd(&s_sh, (unsigned long long)ns);
      if (nd) atomicAdd(&s_td, (unsigned long long)nd);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (s_sh) atomicAdd(&shadowed[ja], s_sh);
      if (s_td) atomicAdd(&tomb[ja], s_td);
    }
  } else {
    if (shadow) atomicAdd(&shadowed[j], 1ull);
    if (drop_del) atomicAdd(&tomb[j], 1ull);
  }
}

__global__ void k_scatter(const uint32_t* ord, const uint32_t* keep, const uint32_t* pos, uint64_t n,
                          uint32_t* surv) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (keep[p]) surv[pos[p]] = ord[p];
}

// ---------------------------------------------------------------------------
// exclusive scans: tiles of SCAN_TILE elements, then one workgroup scans the
// tile sums (looping with a carry), then tiles add their prefix.

constexpr uint32_t SCAN_THREADS = 256;
constexpr uint32_t SCAN_PER = 8;
constexpr uint32_t SCAN_TILE = SCAN_THREADS * SCAN_PER;

template <typename T>
__device__ inline T block_excl_scan(T v, T* sh, T* total) {
  // 256 threads
  const uint32_t tid = threadIdx.x;
  const uint32_t l = lane_id(), w = tid / WAVE;
  T x = v;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    T t = __shfl_up(x, d, WAVE);
    if (l >= (uint32_t)d) x += t;
  }
  if (l == WAVE - 1) sh[w] = x;
  __syncthreads();
  T base = 0;
  for (uint32_t k = 0; k < w; k++) base += sh[k];
  T tot = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  *total = tot;
  return base + x - v;
}

template <typename TI, typename T>
__global__ void __launch_bounds__(256) k_scan_tiles(const TI* in, uint64_t cap, const uint64_t* n_dev, T* out,
                                                    T* tile_sums) {
  __shared__ T sh[4];
  const uint64_t n = n_dev ? *n_dev : cap;
  if ((uint64_t)blockIdx.x * SCAN_TILE >= n && blockIdx.x > 0) return;
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_PER;
  T vals[SCAN_PER];
  T s = 0;
#pragma unroll
  for (uint32_t k = 0; k < SCAN_PER; k++) {
    vals[k] = (base + k < n) ? (T)in[base + k] : (T)0;
    s += vals[k];
  }
  T total;
  T pre = block_excl_scan<T>(s, sh, &total);
#pragma unroll
  for (uint32_t k = 0; k < SCAN_PER; k++) {
    if (base + k < n) out[base + k] = pre;
    pre += vals[k];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

template <typename T>
__global__ void __launch_bounds__(256) k_scan_sums(T* tile_sums, uint64_t cap, const uint64_t* n_dev, T* total_out) {
  __shared__ T sh[4];
  const uint64_t n = n_dev ? *n_dev : cap;
  const uint64_t ntiles = n ? (n + SCAN_TILE - 1) / SCAN_TILE : 1;
  T carry = 0;
  for (uint64_t b = 0; b < ntiles; b += SCAN_THREADS) {
    const uint64_t i = b + threadIdx.x;
    T v = i < ntiles ? tile_sums[i] : (T)0;
    T tot;
    T pre = block_excl_scan<T>(v, sh, &tot);
    if (i < ntiles) tile_sums[i] = carry + pre;
    carry += tot;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

template <typename T>
__global__ void __launch_bounds__(256) k_scan_add(T* out, uint64_t cap, const uint64_t* n_dev, const T* tile_sums,
                                                  T* total_out) {
  const uint64_t n = n_dev ? *n_dev : cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = *total_out;
  if ((uint64_t)blockIdx.x * SCAN_TILE >= n) return;
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_PER;
  const T add = tile_sums[blockIdx.x];
#pragma unroll
  for (uint32_t k = 0; k < SCAN_PER; k++)
    if (base + k < n) out[base + k] += add;
}

// one workgroup for short arrays: passes of SCAN_TILE elements with a carry
template <typename TI, typename T>
__global__ void __launch_bounds__(256) k_scan_one(const TI* in, uint64_t cap, const uint64_t* n_dev, T* out) {
  __shared__ T sh[4];
  const uint64_t n = n_dev ? *n_dev : cap;
  T carry = 0;
  for (uint64_t t0 = 0; t0 < n; t0 += SCAN_TILE) {
    const uint64_t base = t0 + (uint64_t)threadIdx.x * SCAN_PER;
    T vals[SCAN_PER];
    T s = 0;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_PER; k++) {
      vals[k] = (base + k < n) ? (T)in[base + k] : (T)0;
      s += vals[k];
    }
    T total;
    T pre = carry + block_excl_scan<T>(s, sh, &total);
#pragma unroll
    for (uint32_t k = 0; k < SCAN_PER; k++) {
      if (base + k < n) out[base + k] = pre;
      pre += vals[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0) out[n] = carry;
}

template <typename TI, typename T>
void launch_scan(const TI* in, uint64_t cap, const uint64_t* n_dev, T* out, T* scratch, hipStream_t st) {
  if (cap <= SCAN_ONE_MAX) {
    hipLaunchKernelGGL((k_scan_one<TI, T>), dim3(1), dim3(SCAN_THREADS), 0, st, in, cap, n_dev, out);
    return;
  }
  const uint64_t ntiles = (cap + SCAN_TILE - 1) / SCAN_TILE;
  hipLaunchKernelGGL((k_scan_tiles<TI, T>), dim3((uint32_t)ntiles), dim3(SCAN_THREADS), 0, st, in, cap, n_dev, out,
                     scratch);
  hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(SCAN_THREADS), 0, st, scratch, cap, n_dev, scratch + ntiles);
  hipLaunchKernelGGL(k_scan_add<T>, dim3((uint32_t)ntiles), dim3(SCAN_THREADS), 0, st, out, cap, n_dev, scratch,
                     scratch + ntiles);
}

template void launch_scan<uint32_t, uint32_t>(const uint32_t*, uint64_t, const uint64_t*, uint32_t*, uint32_t*,
                                              hipStream_t);
template void launch_scan<uint32_t, uint64_t>(const uint32_t*, uint64_t, const uint64_t*, uint64_t*, uint64_t*,
                                              hipStream_t);
template void launch_scan<uint64_t, uint64_t>(const uint64_t*, uint64_t, const uint64_t*, uint64_t*, uint64_t*,
                                              hipStream_t);

}  // namespace luda
