// Host runtime of the GPU compaction path: the C-ABI of include/luda.h.
//
// One call runs the paper's per-job workflow (Sec. III-A overview: copy the
// selected tables to the GPU, unpack, sort and drop, pack, return the new
// tables), for one job or a batch of independent jobs at once.  Every stage
// is a device kernel.  Between stages the host only reads a few counters
// (gathered by one small kernel into pinned memory, then one stream sync),
// sizes buffers, and builds small work lists (staged in pinned memory and
// scattered to their device buffers by one kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "luda.h"
#include "luda_host_internal.h"
#include "kernels.h"

using namespace luda;

namespace {

// ---------------------------------------------------------------------------
// CRC32C tables built on the host and copied into LDS by the kernels:
// slicing-by-4 tables and "shift by 16 * 2^k zero bytes" (k = 0..6), each a
// set of four 256-entry tables indexed by the bytes of the 32-bit register.

constexpr uint32_t POLY = 0x82F63B78u;  // CRC32C, reflected
constexpr int NSH = 7;

uint32_t step_byte(uint32_t r, uint8_t b, const uint32_t* t0) { return t0[(r ^ b) & 0xFF] ^ (r >> 8); }

struct CrcTables {
  uint32_t t4[4][256];
  uint32_t sh[NSH][4][256];
  uint32_t u0[2048], u1[2048], u2[1024];  // 11-bit fields of a word
  uint32_t segk[8];                        // x^(8 CRC_SEG_BYTES 2^k) mod P, k = 0..6 (and a pad)
};
static_assert(offsetof(CrcTables, segk) == 53248, "the kernels find the segment constants after the 11-bit tables");
// LDS bytes of the slicing and shift tables (the head of the image), what
// the encoder stages next to its blocks
constexpr size_t CRC_LDS_BYTES = sizeof(uint32_t) * 4 * 256 * (1 + NSH);

void byte_table(uint32_t* t0) {
  for (uint32_t b = 0; b < 256; b++) {
    uint32_t r = b;
    for (int k = 0; k < 8; k++) r = (r >> 1) ^ (POLY & (0u - (r & 1u)));
    t0[b] = r;
  }
}

uint32_t shift_zeros(uint32_t r, uint64_t m, const uint32_t* t0) {
  for (uint64_t z = 0; z < m; z++) r = step_byte(r, 0, t0);
  return r;
}

uint32_t apply_shift(const uint32_t sh[4][256], uint32_t c) {
  return sh[0][c & 0xFF] ^ sh[1][(c >> 8) & 0xFF] ^ sh[2][(c >> 16) & 0xFF] ^ sh[3][c >> 24];
}

// GF(2) products mod P in the reflected representation, for the segment join constants and the self check
uint32_t h_mulmod(uint32_t a, uint32_t b) {
  uint32_t p = 0;
  for (int i = 0; i < 32; i++) {
    if (a & (0x80000000u >> i)) p ^= b;
    b = (b & 1u) ? (b >> 1) ^ POLY : (b >> 1);
  }
  return p;
}
uint32_t h_xpow8n(uint64_t n) {
  uint32_t result = 0x80000000u, sq = 0x00800000u;
  while (n) {
    if (n & 1) result = h_mulmod(result, sq);
    sq = h_mulmod(sq, sq);
    n >>= 1;
  }
  return result;
}

void build_crc_tables(CrcTables* T) {
  uint32_t t0[256];
  byte_table(t0);
  for (int b = 0; b < 256; b++) T->t4[0][b] = t0[b];
  for (int k = 1; k < 4; k++)
    for (int b = 0; b < 256; b++) T->t4[k][b] = (T->t4[k - 1][b] >> 8) ^ t0[T->t4[k - 1][b] & 0xFF];
  for (int k = 0; k < NSH; k++)
    for (int i = 0; i < 4; i++)
      for (uint32_t v = 0; v < 256; v++) T->sh[k][i][v] = shift_zeros(v << (8 * i), 16ull << k, t0);
  auto word = [&](uint32_t x) {
    return T->t4[3][x & 0xFF] ^ T->t4[2][(x >> 8) & 0xFF] ^ T->t4[1][(x >> 16) & 0xFF] ^ T->t4[0][x >> 24];
  };
  for (uint32_t i = 0; i < 2048; i++) {
    T->u0[i] = word(i);
    T->u1[i] = word(i << 11);
  }
  for (uint32_t i = 0; i < 1024; i++) T->u2[i] = word(i << 22);
  for (int k = 0; k < 8; k++) T->segk[k] = k < 7 ? h_xpow8n((uint64_t)CRC_SEG_BYTES << k) : 0;
}

struct DBuf {
  void* p = nullptr;
  size_t cap = 0;
  uint64_t gen = 0;  // the call that last used it
};

struct HostBlock;

// Host threads that copy one buffer together (the pageable-to-pinned step of
// uploads of host inputs).  copy() is called by one thread at a time.
class CopyPool {
 public:
  explicit CopyPool(unsigned n) : n_threads_(n) {
    for (unsigned i = 0; i < n; i++) th_.emplace_back([this, i] { loop(i); });
  }
  ~CopyPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  void copy(void* dst, const void* src, size_t n) {
    std::unique_lock<std::mutex> lk(mu_);
    dst_ = (uint8_t*)dst;
    src_ = (const uint8_t*)src;
    n_ = n;
    left_ = n_threads_;
    gen_++;
    cv_.notify_all();
    done_.wait(lk, [&] { return left_ == 0; });
  }

 private:
  void loop(unsigned i) {
    uint64_t seen = 0;
    for (;;) {
      uint8_t* d;
      const uint8_t* s;
      size_t n;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        d = dst_;
        s = src_;
        n = n_;
      }
      const size_t part = ((n + n_threads_ - 1) / n_threads_ + 4095) & ~size_t(4095);
      const size_t a = std::min(n, (size_t)i * part), b = std::min(n, a + part);
      if (b > a) memcpy(d + a, s + a, b - a);
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (--left_ == 0) done_.notify_one();
      }
    }
  }
  const unsigned n_threads_;
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  uint8_t* dst_ = nullptr;
  const uint8_t* src_ = nullptr;
  size_t n_ = 0;
  uint64_t gen_ = 0;
  unsigned left_ = 0;
  bool stop_ = false;
};

constexpr int UP_SLOTS = 3;

}  // namespace

struct luda_ctx {
  int device = 0;
  luda_params tp{8, 4, 16};  // launch parameters (luda_set_params / luda_autotune)
  hipStream_t own = nullptr;
  hipStream_t stream = nullptr;
  uint32_t* d_crc = nullptr;  // CrcTables image
  int n_cu = 256;
  size_t lds_limit = 64 * 1024;  // LDS per workgroup
  std::string last_error;
  std::map<std::string, DBuf> bufs;
  uint64_t call_gen = 0;   // calls so far (begin_call)
  uint64_t mem_limit = 0;  // most device bytes the named buffers may hold at once (0: no limit)
  // luda_compact_dev_noalloc: working buffers carved from the device's static
  // scratch array and output tables written to the caller's buffer
  struct Arena {
    uint8_t* base = nullptr;
    size_t cap = 0, used = 0, peak = 0;
    std::map<std::string, std::pair<void*, size_t>> named;
    uint8_t* out = nullptr;
    uint64_t out_cap = 0;
  };
  Arena* arena = nullptr;
  luda_allocator alloc{};  // caller's device allocator (luda_set_allocator); alloc.alloc == NULL: hipMalloc
  // pinned host memory: readbacks (written by k_mail) and staged uploads
  uint8_t* mail = nullptr;  // mail_cap bytes, then the readback flag (8 bytes)
  uint64_t mail_seq = 0;
  size_t mail_cap = 0;
  uint8_t* stage = nullptr;
  size_t stage_cap = 0, stage_used = 0;
  UpSegs up_pending{};
  // uploads of host inputs: pinned staging slots, their events, copy threads
  HostBlock* up_slot[UP_SLOTS] = {};
  hipEvent_t up_ev[UP_SLOTS] = {};
  bool up_busy[UP_SLOTS] = {};
  int up_next = 0;
  std::unique_ptr<CopyPool> copier;
  // stage timing (LUDA_STAGE_TIMES) and hot-kernel timing (always)
  bool timing = false;
  bool host_sort = false;  // cooperative sort: order the entries on the host (luda_set_host_sort)
  std::vector<std::pair<std::string, hipEvent_t>> marks;
  std::vector<hipEvent_t> event_pool;
  size_t event_used = 0;
  std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> kmarks;
  std::vector<hipEvent_t> kevents;
  size_t kevent_used = 0;
  std::vector<std::pair<std::string, double>> stage_ms;
  std::vector<std::pair<std::string, double>> counters;
};

namespace {

struct Fail {
  int status;
  std::string msg;
};

#define HIPCK(x)                                                                         \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      throw Fail{LUDA_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)};           \
  } while (0)

#define LAUNCH_CHECK() HIPCK(hipGetLastError())

// Runs fn and turns every exception into a status: Fail carries its own,
// a failed host allocation is LUDA_NOMEM, anything else (e.g. a thread that
// could not start) LUDA_DEVICE.  No exception crosses the C-ABI.
template <typename F>
int guarded(luda_ctx* c, F&& fn) {
  std::string msg;
  int st = LUDA_OK;
  try {
    fn();
    return LUDA_OK;
  } catch (const Fail& f) {
    st = f.status;
    msg = f.msg;
  } catch (const std::bad_alloc&) {
    st = LUDA_NOMEM;
    msg = "host allocation failed";
  } catch (const std::exception& e) {
    st = LUDA_DEVICE;
    msg = e.what();
  } catch (...) {
    st = LUDA_DEVICE;
    msg = "unexpected failure";
  }
  if (c) {
    try {
      c->last_error = msg;
    } catch (...) {
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipGetLastError();
  }
  return st;
}


// grow-only named device buffers
size_t dev_pool_trim(int device);
void dev_pool_put(int device, DBuf b);

// Device memory of the context: the caller's allocator when one is set,
// else hipMalloc.  A buffer is given back only once the context's stream has
// finished with it (hipFree waits for the device by itself).
hipError_t dmalloc(luda_ctx* c, void** p, size_t bytes) {
  if (!c->alloc.alloc) return hipMalloc(p, bytes);
  *p = c->alloc.alloc(c->alloc.user, bytes, (void*)c->stream);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
void dfree(luda_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  if (!c->alloc.alloc) {
    HIPCK(hipFree(p));
    return;
  }
  HIPCK(hipStreamSynchronize(c->stream));
  c->alloc.free(c->alloc.user, p, bytes, (void*)c->stream);
}
// the output-table buffer goes back to the device pool (hipMalloc'd) or to
// the caller's allocator
void release_out(luda_ctx* c, DBuf b) {
  if (!b.p) return;
  if (c->alloc.alloc)
    dfree(c, b.p, b.cap);
  else
    dev_pool_put(c->device, b);
}

// device bytes held by the context's named buffers
size_t held_bytes(const luda_ctx* c) {
  size_t n = 0;
  for (auto& kv : c->bufs) n += kv.second.cap;
  return n;
}

// Keep the named buffers within the context's memory limit when one of them
// grows to `want` bytes: buffers that the current call has not used are
// freed first; if the call itself needs more, it fails with LUDA_NOMEM.
void fit_limit(luda_ctx* c, const std::string& name, size_t want) {
  if (!c->mem_limit) return;
  const size_t own = c->bufs[name].cap;
  if (held_bytes(c) - own + want <= c->mem_limit) return;
  HIPCK(hipStreamSynchronize(c->stream));
  for (auto& kv : c->bufs)
    if (kv.first != name && kv.second.gen != c->call_gen && kv.second.p) {
      if (kv.first == "out_tables")
        release_out(c, kv.second);
      else
        dfree(c, kv.second.p, kv.second.cap);
      kv.second = DBuf{};
    }
  if (held_bytes(c) - own + want > c->mem_limit)
    throw Fail{LUDA_NOMEM, "the call needs more device memory than the context's limit of " +
                               std::to_string(c->mem_limit) + " bytes (" + name + ")"};
}

// a named buffer of the current call inside the scratch arena: reused when
// large enough, else carved anew after everything the call has carved so far
void* arena_buf(luda_ctx* c, const std::string& name, size_t bytes) {
  luda_ctx::Arena& a = *c->arena;
  auto it = a.named.find(name);
  if (it != a.named.end() && it->second.second >= bytes) return it->second.first;
  const size_t off = (a.used + 255) & ~size_t(255);
  if (off > a.cap || bytes > a.cap - off)
    throw Fail{LUDA_NOMEM, "the call's working buffers need more than the " + std::to_string(a.cap) +
                               " bytes of static scratch memory (at " + name + ")"};
  a.used = off + bytes;
  a.peak = std::max(a.peak, a.used);
  a.named[name] = {a.base + off, bytes};
  return a.base + off;
}

template <typename T>
T* dbuf(luda_ctx* c, const std::string& name, size_t count) {
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  bytes = (bytes + 255) & ~size_t(255);
  if (c->arena) return (T*)arena_buf(c, name, bytes);
  c->bufs[name].gen = c->call_gen;
  DBuf& b = c->bufs[name];
  if (b.cap < bytes) {
    size_t want = bytes + bytes / 8;
    if (c->mem_limit) {
      fit_limit(c, name, bytes);
      if (held_bytes(c) - b.cap + want > c->mem_limit) want = bytes;
    }
    if (b.p) {
      if (name == "out_tables")
        release_out(c, b);
      else
        dfree(c, b.p, b.cap);
    }
    b.p = nullptr;
    b.cap = 0;
    hipError_t e = dmalloc(c, &b.p, want);
    if (e != hipSuccess && dev_pool_trim(c->device) > 0) {  // the pooled output buffers give way first
      (void)hipGetLastError();
      e = dmalloc(c, &b.p, want);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Fail{LUDA_NOMEM, "device allocation of " + std::to_string(want) + " bytes for " + name + " failed"};
    }
    b.cap = want;
  }
  return (T*)b.p;
}

void fill_u32(luda_ctx* c, void* p, uint32_t v, uint64_t n);

// grid of the multi-workgroup checksum over messages of at most `bytes`
// bytes in total (segments of CRC_SEG_BYTES, one per message at least)
uint32_t crc_multi_grid(const luda_ctx* c, uint64_t bytes, uint64_t msgs) {
  // a wave per segment, 16 waves per workgroup
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((bytes / CRC_SEG_BYTES + msgs + 15) / 16, 2ull * c->n_cu));
}

inline uint32_t blocks_for(uint64_t n, uint32_t t = 256) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + t - 1) / t, 0x7FFFFFFFull));
}

// grid of a grid-stride kernel over at most cap items
uint32_t stride_grid(const luda_ctx* c, uint64_t cap, uint32_t t = 256) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((cap + t - 1) / t, (uint64_t)c->n_cu * c->tp.stride_blocks));
}

void fill_u32(luda_ctx* c, void* p, uint32_t v, uint64_t n) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n)), dim3(256), 0, c->stream, (uint32_t*)p, v, n);
  LAUNCH_CHECK();
}
void fill_u64(luda_ctx* c, void* p, uint64_t v, uint64_t n) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n)), dim3(256), 0, c->stream, (unsigned long long*)p,
                     (unsigned long long)v, n);
  LAUNCH_CHECK();
}
void sync(luda_ctx* c) { HIPCK(hipStreamSynchronize(c->stream)); }

// --- staged uploads: the bytes are copied into pinned memory now and moved
// to their device buffers by one kernel at the next flush (stream ordered).
// The staging area is only reused by the next call, after its final sync.
void up_flush(luda_ctx* c) {
  if (!c->up_pending.n) return;
  hipLaunchKernelGGL(k_upload, dim3(c->up_pending.n), dim3(256), 0, c->stream, c->up_pending,
                     (const uint8_t*)c->stage);
  LAUNCH_CHECK();
  c->up_pending.n = 0;
}

void up(luda_ctx* c, void* dev, const void* host, size_t bytes) {
  if (!bytes) return;
  const size_t off = (c->stage_used + 15) & ~size_t(15);
  if (off + bytes > c->stage_cap || bytes > 0xFFFFFFFFull) {
    up_flush(c);
    HIPCK(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return;
  }
  memcpy(c->stage + off, host, bytes);
  c->stage_used = off + bytes;
  if (c->up_pending.n == 16) up_flush(c);
  UpSegs& u = c->up_pending;
  u.dst[u.n] = (uint64_t)(uintptr_t)dev;
  u.bytes[u.n] = (uint32_t)bytes;
  u.src[u.n] = (uint32_t)off;
  u.n++;
}

// Waits for the work queued so far on the context's stream: a last kernel
// writes a sequence number into pinned memory and the host polls it for at
// most 2 ms; past that (a long stage, or a failed one, whose error the
// synchronisation reports) it synchronises the stream.
void wait_stream(luda_ctx* c) {
  const uint64_t seq = ++c->mail_seq;
  uint64_t* flag = (uint64_t*)(c->mail + c->mail_cap);
  hipLaunchKernelGGL(k_mail_flag, dim3(1), dim3(64), 0, c->stream, flag, seq);
  LAUNCH_CHECK();
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t k = 0;; k++) {
    if (__atomic_load_n((volatile uint64_t*)flag, __ATOMIC_ACQUIRE) == seq) return;
    if ((k & 255) == 255 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) break;
    __builtin_ia32_pause();
  }
  sync(c);
}

// --- readbacks: device ranges gathered into the pinned mailbox by one
// kernel per 12 ranges, then a wait for the stream
struct Mail {
  luda_ctx* c;
  std::vector<MailSegs> segs;
  size_t used = 0;
  // ranges that do not fit in the mailbox: copied into host memory of their own
  std::vector<std::pair<const void*, std::vector<uint8_t>>> big;
  explicit Mail(luda_ctx* c_) : c(c_) { segs.emplace_back(); }
  template <typename T>
  const T* add(const T* dev, size_t count) {
    const size_t bytes = count * sizeof(T);
    const size_t off = (used + 15) & ~size_t(15);
    if (off + bytes > c->mail_cap || bytes > 0xFFFFFFFFull) {
      big.emplace_back((const void*)dev, std::vector<uint8_t>(std::max<size_t>(bytes, 1)));
      return (const T*)big.back().second.data();
    }
    used = off + bytes;
    if (!bytes) return (const T*)(c->mail + off);
    if (segs.back().n == 12) segs.emplace_back();
    MailSegs& m = segs.back();
    m.src[m.n] = (uint64_t)(uintptr_t)dev;
    m.bytes[m.n] = (uint32_t)bytes;
    m.dst[m.n] = (uint32_t)off;
    m.n++;
    return (const T*)(c->mail + off);
  }
  void flush() {
    up_flush(c);
    for (auto& m : segs)
      if (m.n) {
        hipLaunchKernelGGL(k_mail, dim3(m.n), dim3(256), 0, c->stream, m, c->mail);
        LAUNCH_CHECK();
      }
    for (auto& b : big)
      if (b.first)
        HIPCK(hipMemcpyAsync(b.second.data(), b.first, b.second.size(), hipMemcpyDeviceToHost, c->stream));
    if (big.empty()) wait_stream(c);
    else sync(c);
  }
};

void mark(luda_ctx* c, const char* name) {
  if (!c->timing) return;
  if (c->event_used == c->event_pool.size()) {
    hipEvent_t e;
    HIPCK(hipEventCreate(&e));
    c->event_pool.push_back(e);
  }
  hipEvent_t e = c->event_pool[c->event_used++];
  HIPCK(hipEventRecord(e, c->stream));
  c->marks.emplace_back(name, e);
}

hipEvent_t kevent(luda_ctx* c) {
  if (c->kevent_used == c->kevents.size()) {
    hipEvent_t e;
    HIPCK(hipEventCreate(&e));
    c->kevents.push_back(e);
  }
  return c->kevents[c->kevent_used++];
}

// HIP events around one hot kernel launch on the context's stream
struct KTimer {
  luda_ctx* c;
  const char* name;
  hipEvent_t b;
  KTimer(luda_ctx* c_, const char* n) : c(c_), name(n) {
    b = kevent(c);
    HIPCK(hipEventRecord(b, c->stream));
  }
  void stop() {
    hipEvent_t e = kevent(c);
    HIPCK(hipEventRecord(e, c->stream));
    c->kmarks.push_back({name, {b, e}});
  }
};

// Called after the call's final sync, when results may already hold
// buffers: it never throws (a time that cannot be read is left out).
void collect_times(luda_ctx* c) noexcept {
  try {
    c->stage_ms.clear();
    if (c->timing && c->marks.size() > 1) {
      for (size_t i = 1; i < c->marks.size(); i++) {
        float t = 0;
        if (hipEventElapsedTime(&t, c->marks[i - 1].second, c->marks[i].second) == hipSuccess)
          c->stage_ms.emplace_back(c->marks[i].first, t);
        else
          (void)hipGetLastError();
      }
    }
    for (auto& km : c->kmarks) {
      float t = 0;
      if (hipEventElapsedTime(&t, km.second.first, km.second.second) == hipSuccess)
        c->stage_ms.emplace_back(std::string("kernel:") + km.first, t);
      else
        (void)hipGetLastError();
    }
  } catch (...) {
    c->stage_ms.clear();
  }
}

void begin_call(luda_ctx* c) {
  c->call_gen++;
  c->marks.clear();
  c->event_used = 0;
  c->kmarks.clear();
  c->kevent_used = 0;
  c->counters.clear();
  c->stage_used = 0;
  c->up_pending.n = 0;
}

int status_of(uint32_t code) {
  switch (code) {
    case EC_FORMAT: return LUDA_CORRUPT_FORMAT;
    case EC_CHECKSUM: return LUDA_CORRUPT_CHECKSUM;
    case EC_UNSUPPORTED: return LUDA_UNSUPPORTED;
    case EC_UNSORTED: return LUDA_UNSORTED_INPUT;
    case EC_LIMIT: return LUDA_UNSUPPORTED;
    default: return LUDA_DEVICE;
  }
}

luda_error decode_err(uint64_t key, const std::vector<uint64_t>& in_size, uint32_t in_first) {
  luda_error e;
  memset(&e, 0, sizeof e);
  e.status = status_of((uint32_t)(key & 7));
  e.input = (uint32_t)(key >> 52);
  e.where = (uint32_t)((key >> 50) & 3);
  e.block = (key >> 28) & 0x3FFFFF;
  e.phase = (uint32_t)((key >> 26) & 3);
  e.offset = (key >> 3) & 0x7FFFFF;
  if (e.where == W_FOOTER) {
    const uint64_t size = in_size[in_first + e.input];
    e.offset = (e.phase == FP_SHORT) ? 0 : size - 48 + e.offset;
    e.phase = 0;
    e.block = 0;
  }
  return e;
}

int check_opt(const luda_options* o) {
  if (!o || o->block_size == 0 || o->restart_interval == 0 || o->bloom_bits_per_key == 0 ||
      o->target_file_size == 0 || o->compression > 1 || o->n_snapshots > LUDA_MAX_SNAPSHOTS ||
      (o->n_snapshots && !o->snapshots))
    return LUDA_INVALID_ARG;
  for (uint32_t i = 0; i < o->n_snapshots; i++)
    if ((o->snapshots[i] >> 56) || (i && o->snapshots[i] <= o->snapshots[i - 1])) return LUDA_INVALID_ARG;
  return LUDA_OK;
}

// A device output buffer shared by the results of one call.  The last
// release hands it back to the context (as the spare output buffer) or frees
// it.
struct DevBlock {
  void* p = nullptr;
  size_t cap = 0;
  std::atomic<int> refs{0};  // results of one pass may be freed from several threads
  int device = 0;
  luda_allocator alloc{};  // the caller's allocator it came from (alloc.alloc == NULL: the device pool)
  DevBlock(void* p_, size_t cap_, int refs_, int device_, const luda_allocator& a)
      : p(p_), cap(cap_), refs(refs_), device(device_), alloc(a) {}
};

// Output buffers handed to results come back, when the results are freed, to
// a pool per device from which later calls take their output buffers.
// hipMalloc and hipFree of buffers of hundreds of MB or more cost
// milliseconds to seconds, and hipFree waits for the whole device, which
// would stall the passes of other contexts and server workers.  The pool
// holds up to half of the device's memory; past that its smallest buffers are
// freed first.  luda_pool_trim empties it.
std::mutex dev_pool_mu;
std::map<int, std::multimap<size_t, void*>> dev_pool;  // device -> (capacity -> buffer)
std::map<int, size_t> dev_pool_bytes;
std::map<int, size_t> dev_pool_cap;

void free_on(int device, void* p) {
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != device) (void)hipSetDevice(device);
  (void)hipFree(p);
  if (cur != device) (void)hipSetDevice(cur);
}

// the smallest pooled buffer of at least `bytes` and at most about 2x that
DBuf dev_pool_get(int device, size_t bytes) {
  std::lock_guard<std::mutex> lk(dev_pool_mu);
  auto& m = dev_pool[device];
  auto it = m.lower_bound(bytes);
  if (it == m.end() || it->first > 2 * bytes + (size_t(64) << 20)) return DBuf{};
  DBuf b{it->second, it->first};
  dev_pool_bytes[device] -= it->first;
  m.erase(it);
  return b;
}

void dev_pool_put(int device, DBuf b) {
  if (!b.p) return;
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> lk(dev_pool_mu);
    size_t& cap = dev_pool_cap[device];
    if (!cap) {
      size_t total = 0;
      cap = hipDeviceTotalMem(&total, device) == hipSuccess && total ? total / 2 : size_t(32) << 30;
    }
    if (b.cap > cap) {
      drop.push_back(b.p);
    } else {
      auto& m = dev_pool[device];
      m.emplace(b.cap, b.p);
      dev_pool_bytes[device] += b.cap;
      while (dev_pool_bytes[device] > cap) {  // the smallest go first
        drop.push_back(m.begin()->second);
        dev_pool_bytes[device] -= m.begin()->first;
        m.erase(m.begin());
      }
    }
  }
  for (void* p : drop) free_on(device, p);
}

size_t dev_pool_trim(int device) {
  std::multimap<size_t, void*> m;
  {
    std::lock_guard<std::mutex> lk(dev_pool_mu);
    m.swap(dev_pool[device]);
    dev_pool_bytes[device] = 0;
  }
  size_t n = 0;
  for (auto& kv : m) {
    free_on(device, kv.second);
    n += kv.first;
  }
  return n;
}

// Pinned host memory for results in host memory (device-to-host copies at
// full link speed, no page faults on first touch).  Pinning pages is slow
// (it costs about as much as the copy), so pinned memory is allocated in
// segments of PIN_SEG bytes that live until the process ends, up to PIN_CAP
// bytes in all; a result takes a range of one segment (first fit, freed
// ranges merge with their neighbours).  A result larger than a segment gets
// a segment of its own, unpinned again once it is free.  With PIN_CAP in use
// (results held by the caller), results go to ordinary memory.
constexpr size_t PIN_SEG = size_t(1) << 30;
constexpr size_t PIN_CAP = size_t(32) << 30;
constexpr size_t PIN_ALIGN = 4096;

struct PinSeg {
  uint8_t* p = nullptr;
  size_t cap = 0;
  std::map<size_t, size_t> free;  // offset -> length of the free ranges
};

struct HostBlock {
  void* p = nullptr;
  size_t cap = 0;
  int refs = 0;
  PinSeg* seg = nullptr;  // null: ordinary memory
};

std::mutex pin_mu;
std::vector<PinSeg*> pin_segs;
size_t pin_total = 0;

// first fit among the free ranges of the segments (pin_mu held)
HostBlock* pin_take(size_t n) {
  for (PinSeg* g : pin_segs)
    for (auto it = g->free.begin(); it != g->free.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      g->free.erase(it);
      if (len > n) g->free.emplace(off + n, len - n);
      return new HostBlock{g->p + off, n, 0, g};
    }
  return nullptr;
}

// a new segment of cap bytes, already counted in pin_total; pinning runs
// outside the lock, so that other threads keep taking ranges meanwhile
PinSeg* pin_grow(size_t cap) {
  void* p = nullptr;
  if (hipHostMalloc(&p, cap, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(pin_mu);
    pin_total -= cap;
    return nullptr;
  }
  return new PinSeg{(uint8_t*)p, cap, {}};
}

HostBlock* pin_get(size_t n) {
  n = std::max(PIN_ALIGN, (n + PIN_ALIGN - 1) & ~(PIN_ALIGN - 1));
  const size_t cap = std::max(PIN_SEG, (n + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1));
  bool grow = false;
  {
    std::lock_guard<std::mutex> lk(pin_mu);
    if (HostBlock* h = pin_take(n)) return h;
    if (pin_total + cap <= PIN_CAP) {
      pin_total += cap;
      grow = true;
    }
  }
  if (PinSeg* g = grow ? pin_grow(cap) : nullptr) {
    std::lock_guard<std::mutex> lk(pin_mu);
    if (cap > n) g->free.emplace(n, cap - n);
    pin_segs.push_back(g);
    return new HostBlock{g->p, n, 0, g};
  }
  void* p = malloc(n);
  return p ? new HostBlock{p, n, 0, nullptr} : nullptr;
}

// grow the pool by whole segments until it holds `bytes` (at most PIN_CAP)
size_t pin_reserve(size_t bytes) {
  bytes = std::min(bytes, PIN_CAP);
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(pin_mu);
      if (pin_total >= bytes || pin_total + PIN_SEG > PIN_CAP) return pin_total;
      pin_total += PIN_SEG;
    }
    PinSeg* g = pin_grow(PIN_SEG);
    std::lock_guard<std::mutex> lk(pin_mu);
    if (!g) return pin_total;
    g->free.emplace(0, PIN_SEG);
    pin_segs.push_back(g);
  }
}

void pin_put(HostBlock* h) {
  PinSeg* g = h->seg;
  if (!g) {
    free(h->p);
    delete h;
    return;
  }
  std::lock_guard<std::mutex> lk(pin_mu);
  size_t off = (size_t)((uint8_t*)h->p - g->p), len = h->cap;
  delete h;
  auto nx = g->free.lower_bound(off);
  if (nx != g->free.end() && nx->first == off + len) {  // merge with the next range
    len += nx->second;
    nx = g->free.erase(nx);
  }
  if (nx != g->free.begin()) {  // and with the previous one
    auto pv = std::prev(nx);
    if (pv->first + pv->second == off) {
      off = pv->first;
      len += pv->second;
      g->free.erase(pv);
    }
  }
  if (g->cap > PIN_SEG && len == g->cap) {  // an outsize segment, free again
    (void)hipHostFree(g->p);
    pin_total -= g->cap;
    pin_segs.erase(std::find(pin_segs.begin(), pin_segs.end(), g));
    delete g;
    return;
  }
  g->free.emplace(off, len);
}

struct ResultInternal {
  DevBlock* dev = nullptr;
  HostBlock* host = nullptr;  // host results: the pinned block they point into
};

void release_host(ResultInternal* ri) {
  if (!ri || !ri->host) return;
  HostBlock* h = ri->host;
  ri->host = nullptr;
  if (--h->refs == 0) pin_put(h);
}

void release_dev(luda_ctx* c, ResultInternal* ri) {
  if (!ri || !ri->dev) return;
  DevBlock* d = ri->dev;
  ri->dev = nullptr;  // this result no longer holds the buffer, whoever frees it
  if (--d->refs > 0) return;
  (void)c;
  if (d->alloc.alloc)
    d->alloc.free(d->alloc.user, d->p, d->cap, nullptr);
  else
    dev_pool_put(d->device, DBuf{d->p, d->cap});
  delete d;
}

// Host inputs live in pageable memory, which the runtime copies through its
// own staging at a fraction of the link speed.  Large inputs go instead in
// chunks through the context's pinned slots: host threads fill one slot
// while the DMA engine moves the previous one.  Small inputs are copied
// directly.
constexpr size_t UP_CHUNK = size_t(32) << 20;
constexpr size_t UP_DIRECT = size_t(4) << 20;

void upload_host(luda_ctx* c, uint8_t* dst, const uint8_t* src, size_t n) {
  if (n < UP_DIRECT) {
    HIPCK(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, c->stream));
    return;
  }
  if (!c->copier) {
    for (int s = 0; s < UP_SLOTS; s++) {
      if (!c->up_slot[s]) c->up_slot[s] = pin_get(UP_CHUNK);
      if (!c->up_ev[s]) HIPCK(hipEventCreateWithFlags(&c->up_ev[s], hipEventDisableTiming));
    }
    const unsigned hw = std::thread::hardware_concurrency();
    c->copier.reset(new CopyPool(std::max(1u, std::min(8u, hw ? hw / 2 : 1u))));
  }
  for (size_t off = 0; off < n; off += UP_CHUNK) {
    const size_t len = std::min(UP_CHUNK, n - off);
    const int s = c->up_next;
    c->up_next = (s + 1) % UP_SLOTS;
    HostBlock* h = c->up_slot[s];
    if (!h || !h->seg) {  // no pinned slot: the runtime's own staging
      HIPCK(hipMemcpyAsync(dst + off, src + off, len, hipMemcpyHostToDevice, c->stream));
      continue;
    }
    if (c->up_busy[s]) HIPCK(hipEventSynchronize(c->up_ev[s]));  // its last copy has left the slot
    c->copier->copy(h->p, src + off, len);
    HIPCK(hipMemcpyAsync(dst + off, h->p, len, hipMemcpyHostToDevice, c->stream));
    HIPCK(hipEventRecord(c->up_ev[s], c->stream));
    c->up_busy[s] = true;
  }
}

// the output buffer of this call, at least `bytes`: the context's own, else
// one from the pool (the too small one goes back there), else a new one
uint8_t* out_buffer(luda_ctx* c, size_t bytes) {
  if (c->arena) {
    if (bytes > c->arena->out_cap)
      throw Fail{LUDA_NOMEM, "the output tables need " + std::to_string(bytes) + " bytes; the output buffer has " +
                                 std::to_string(c->arena->out_cap)};
    return c->arena->out;
  }
  DBuf& b = c->bufs["out_tables"];
  if (b.cap < bytes && !c->alloc.alloc) {
    const size_t want = (bytes + 255) & ~size_t(255);
    DBuf got = dev_pool_get(c->device, want);
    dev_pool_put(c->device, DBuf{b.p, b.cap});
    b = DBuf{};
    if (got.p && c->mem_limit && held_bytes(c) + got.cap > c->mem_limit) {  // too large for the limit
      dev_pool_put(c->device, got);
      got = DBuf{};
    }
    b.p = got.p;
    b.cap = got.cap;
  }
  return dbuf<uint8_t>(c, "out_tables", bytes);
}

// ---------------------------------------------------------------------------
// The pipeline after survivors are known: block and file cuts, layout, and
// the writers.  Shared by compaction and the table writer.

struct PlanIn {
  uint32_t J;
  JobDesc* d_jobs;
  Tuples tu;
  uint32_t kw8;
  const uint32_t* d_surv;
  std::vector<uint64_t> job_s0;  // J + 1, host copy
  const uint64_t* d_job_s0;
  bool compress = false;  // some job stores data blocks compressed
};

struct PlanOut {
  uint64_t total_bytes = 0;
  uint8_t* d_out = nullptr;
  std::vector<uint64_t> file_out;  // nfiles + 1: where each table starts in the output buffer
  std::vector<uint64_t> file_size;  // each table's bytes (a key slot may follow a table)
  std::vector<uint64_t> file_entries;
  std::vector<uint64_t> file_keys;  // 4 per file (k_file_entries)
  std::vector<uint64_t> job_f0;  // J + 1
};

// a result's file record: its place in the result's data and its key range
void set_file(luda_file& x, const PlanOut& O, uint64_t f, uint64_t base) {
  x.offset = O.file_out[f] - base;
  x.size = O.file_size[f];
  x.num_entries = O.file_entries[f];
  x.smallest_off = x.offset + O.file_keys[4 * f + 0];
  x.smallest_len = O.file_keys[4 * f + 1];
  x.largest_off = x.offset + O.file_keys[4 * f + 2];
  x.largest_len = O.file_keys[4 * f + 3];
}

// the encoder over nblk output blocks (A.blk gives their destinations);
// `big`: some block is off the pipelined path (over 5 KiB of message, over
// 64 entries, or under 16 bytes), so k_encode_big runs after k_encode, over
// the nlist blocks of `list` when there is one, else over every block
void launch_encode(luda_ctx* c, const EncodeArgs& A, uint64_t nblk, bool big, const uint64_t* list = nullptr,
                   uint64_t nlist = 0) {
  const int waves = (int)c->tp.encode_waves;
  int occ = 0;
  HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_encode, waves * 64, 0));
  occ = std::max(occ, 1);
  const uint64_t want = (nblk + waves - 1) / waves;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)c->n_cu * occ));
  KTimer kt(c, "k_encode");
  hipLaunchKernelGGL(k_encode, dim3(grid), dim3(waves * 64), 0, c->stream, A);
  LAUNCH_CHECK();
  kt.stop();
  c->counters.emplace_back("encode_waves_per_group", (double)waves);
  c->counters.emplace_back("encode_groups", (double)grid);
  c->counters.emplace_back("encode_groups_per_cu", (double)occ);
  if (big) {
    const uint64_t items = list ? nlist : nblk;
    const uint32_t gb = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((items + 7) / 8, (uint64_t)c->n_cu * 3));
    KTimer kb(c, "k_encode_big");
    hipLaunchKernelGGL(k_encode_big, dim3(gb), dim3(512), 0, c->stream, A, list, nlist);
    LAUNCH_CHECK();
    kb.stop();
  }
}

void plan_and_write(luda_ctx* c, PlanIn& P, PlanOut& O) {
  const uint32_t J = P.J;
  const uint64_t S = P.job_s0[J];
  hipStream_t st = c->stream;
  O.job_f0.assign(J + 1, 0);
  O.file_out.assign(1, 0);
  if (S == 0) return;

  uint32_t* sz_r = dbuf<uint32_t>(c, "sz_r", S);
  uint32_t* sz_n = dbuf<uint32_t>(c, "sz_n", S);
  uint32_t* shr = dbuf<uint32_t>(c, "shr", S);
  EncRec* erec = dbuf<EncRec>(c, "enc_rec", S);
  hipLaunchKernelGGL(k_prep, dim3(blocks_for(S)), dim3(256), 0, st, P.d_surv, P.tu, P.kw8, P.d_job_s0, J, S, sz_r,
                     sz_n, shr, erec);
  LAUNCH_CHECK();
  mark(c, "prep");

  // --- block cuts over survivors: host-built chunk list
  std::vector<SegJob> sj(J);
  std::vector<SegChunk> ch;
  for (uint32_t j = 0; j < J; j++) {
    const uint64_t m = P.job_s0[j + 1] - P.job_s0[j];
    if (m > 0xFFFFFFF0ull) throw Fail{LUDA_UNSUPPORTED, "more than 2^32 surviving entries in one job"};
    sj[j].base = P.job_s0[j];
    sj[j].m = (uint32_t)m;
    sj[j].chunk0 = (uint32_t)ch.size();
    const uint32_t n = (uint32_t)((m + SEG_C - 1) / SEG_C);
    sj[j].nchunks = n;
    sj[j].pad = 0;
    for (uint32_t q = 0; q < n; q++)
      ch.push_back(SegChunk{j, q * SEG_C, (uint32_t)std::min<uint64_t>(m, (uint64_t)(q + 1) * SEG_C), 0});
  }
  const uint32_t nch = (uint32_t)ch.size();
  SegJob* d_sj = dbuf<SegJob>(c, "sj_b", J);
  SegChunk* d_ch = dbuf<SegChunk>(c, "ch_b", nch);
  uint32_t* d_nch = dbuf<uint32_t>(c, "nch_b", 1);
  up(c, d_sj, sj.data(), J * sizeof(SegJob));
  up(c, d_ch, ch.data(), nch * sizeof(SegChunk));
  up(c, d_nch, &nch, sizeof nch);
  up_flush(c);
  uint32_t* nxt = dbuf<uint32_t>(c, "seg_nxt", S);
  uint32_t* ex = dbuf<uint32_t>(c, "seg_ex", S);
  uint32_t* cnt = dbuf<uint32_t>(c, "seg_cnt", S);
  uint32_t* bmax = dbuf<uint32_t>(c, "seg_bmax", J);
  uint32_t* centry = dbuf<uint32_t>(c, "seg_centry", nch);
  uint32_t* cseg0 = dbuf<uint32_t>(c, "seg_cseg0", nch);
  uint32_t* nseg = dbuf<uint32_t>(c, "seg_nseg", J);
  uint64_t* job_ob0 = dbuf<uint64_t>(c, "job_ob0", J + 1);
  fill_u32(c, bmax, 0, J);
  launch_seg_exit_blocks(d_ch, d_nch, nch, d_sj, P.d_jobs, sz_r, sz_n, nxt, ex, cnt, bmax, st);
  LAUNCH_CHECK();
  const uint32_t cap = (uint32_t)std::min<size_t>(24576, (c->lds_limit - 2048) / 4);
  hipLaunchKernelGGL(k_seg_compose, dim3(J), dim3(256), 2 * cap * sizeof(uint16_t), st, d_sj, J, ex, cnt, bmax,
                     centry, cseg0, nseg, cap);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_small_scan, dim3(1), dim3(64), 0, st, nseg, J, job_ob0);
  LAUNCH_CHECK();
  uint32_t* seg_first = dbuf<uint32_t>(c, "seg_first_b", S);
  launch_seg_mark(d_ch, d_nch, nch, d_sj, nxt, centry, cseg0, job_ob0, seg_first, st);
  LAUNCH_CHECK();
  mark(c, "block_cuts");

  // --- output blocks
  uint64_t OB = 0;
  {
    Mail m(c);
    const uint64_t* nb = m.add(job_ob0 + J, 1);
    m.flush();
    OB = std::max<uint64_t>(*nb, 1);
  }
  OutBlocks ob;
  ob.s0 = dbuf<uint64_t>(c, "ob_s0", OB);
  ob.cnt = dbuf<uint32_t>(c, "ob_cnt", OB);
  ob.size = dbuf<uint32_t>(c, "ob_size", OB);
  ob.full = dbuf<uint64_t>(c, "ob_full", OB);
  ob.job = dbuf<uint32_t>(c, "ob_job", OB);
  ob.file = dbuf<uint32_t>(c, "ob_file", OB);
  ob.off = dbuf<uint64_t>(c, "ob_off", OB);
  ob.ie_size = dbuf<uint32_t>(c, "ob_ie", OB);
  uint32_t* ent_off = dbuf<uint32_t>(c, "ent_off", S);
  EntL* entl = dbuf<EntL>(c, "ent_layout", S);
  uint32_t* gapcnt = dbuf<uint32_t>(c, "gap_cnt", OB);
  hipLaunchKernelGGL(k_block_meta, dim3(blocks_for(OB)), dim3(256), 0, st, job_ob0, J, d_sj, P.d_jobs, seg_first,
                     sz_r, sz_n, erec, OB, ob, ent_off, entl, gapcnt);
  LAUNCH_CHECK();
  uint64_t* scan_tmp = dbuf<uint64_t>(c, "scan_tmp64", OB / 2048 + 8);
  uint64_t* gap_base = dbuf<uint64_t>(c, "gap_base", OB + 1);
  uint64_t* scan_gap = dbuf<uint64_t>(c, "scan_tmp_gap", OB / 2048 + 8);
  EncodeArgs A{};
  A.jobs = P.d_jobs;
  A.ob = ob;
  A.tu = P.tu;
  A.surv = P.d_surv;
  A.sz_r = sz_r;
  A.sz_n = sz_n;
  A.shr = shr;
  A.nblocks = job_ob0 + J;
  A.g_crc = c->d_crc;
  A.ent_off = ent_off;
  A.rec = erec;
  A.kw8 = P.kw8;
  A.entl = entl;
  A.gap_base = gap_base;
  // Compression: every block is encoded raw into staging first, then
  // compressed; the stored sizes (ob.size / ob.full) drive the cuts below.
  uint8_t* zstage = nullptr;
  uint8_t* zbuf = nullptr;
  uint64_t* zoff = nullptr;
  uint8_t* ztype = nullptr;
  if (P.compress) {
    uint32_t* zraw = dbuf<uint32_t>(c, "zw_raw", OB);
    uint64_t* zstride = dbuf<uint64_t>(c, "zw_stride", OB);
    zoff = dbuf<uint64_t>(c, "zw_off", OB + 1);
    ztype = dbuf<uint8_t>(c, "zw_type", OB);
    hipLaunchKernelGGL(k_zprep, dim3(blocks_for(OB)), dim3(256), 0, st, ob, job_ob0 + J, OB, zraw, zstride);
    LAUNCH_CHECK();
    launch_scan<uint64_t, uint64_t>(zstride, OB, nullptr, zoff, scan_tmp, st);
    LAUNCH_CHECK();
    launch_scan<uint32_t, uint64_t>(gapcnt, OB, nullptr, gap_base, scan_gap, st);
    LAUNCH_CHECK();
    uint64_t zbytes = 0;
    {
      Mail m(c);
      const uint64_t* zt = m.add(zoff + OB, 1);
      m.flush();
      zbytes = *zt;
    }
    zstage = dbuf<uint8_t>(c, "zw_stage", zbytes + 64);
    zbuf = dbuf<uint8_t>(c, "zw_buf", zbytes + 64);
    BlockRec* zrec = dbuf<BlockRec>(c, "zw_rec", OB);
    hipLaunchKernelGGL(k_block_dst_stage, dim3(blocks_for(OB)), dim3(256), 0, st, ob, zoff, P.d_jobs, job_ob0 + J,
                       OB, zrec);
    LAUNCH_CHECK();
    A.out = zstage;
    A.blk = zrec;
    A.gapbuf = dbuf<uint4>(c, "gap_buf", zbytes / 16 + 2 * OB + 1);
    hipLaunchKernelGGL(k_gaps<false>, dim3(stride_grid(c, OB * 16)), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_gaps<true>, dim3(stride_grid(c, OB * 16)), dim3(256), 0, st, A);
    LAUNCH_CHECK();
    launch_encode(c, A, OB, true);
    KTimer kz(c, "k_zsnappy");
    hipLaunchKernelGGL(k_zsnappy, dim3((uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((OB + 3) / 4,
                                                                                       (uint64_t)c->n_cu * 8))),
                       dim3(256), 0, st, ob, P.d_jobs, job_ob0 + J, zstage, zoff, zraw, zbuf, ztype);
    LAUNCH_CHECK();
    kz.stop();
  }
  uint64_t* ob_excl = dbuf<uint64_t>(c, "ob_excl", OB + 1);
  launch_scan<uint64_t, uint64_t>(ob.full, OB, nullptr, ob_excl, scan_tmp, st);
  LAUNCH_CHECK();

  // --- file cuts over output blocks: chunk list built on the device
  const uint32_t fch_cap = (uint32_t)(OB / SEG_C + J + 1);
  SegJob* d_sjf = dbuf<SegJob>(c, "sj_f", J);
  SegChunk* d_chf = dbuf<SegChunk>(c, "ch_f", fch_cap);
  uint32_t* d_nchf = dbuf<uint32_t>(c, "nch_f", 1);
  hipLaunchKernelGGL(k_make_segjobs, dim3(1), dim3(64), 0, st, job_ob0, nseg, J, d_sjf, d_chf, d_nchf);
  LAUNCH_CHECK();
  uint32_t* fnxt = dbuf<uint32_t>(c, "fseg_nxt", OB);
  uint32_t* fex = dbuf<uint32_t>(c, "fseg_ex", OB);
  uint32_t* fcnt = dbuf<uint32_t>(c, "fseg_cnt", OB);
  uint32_t* fbmax = dbuf<uint32_t>(c, "fseg_bmax", J);
  uint32_t* fcentry = dbuf<uint32_t>(c, "fseg_centry", fch_cap);
  uint32_t* fcseg0 = dbuf<uint32_t>(c, "fseg_cseg0", fch_cap);
  uint32_t* fnseg = dbuf<uint32_t>(c, "fseg_nseg", J);
  uint64_t* job_f0 = dbuf<uint64_t>(c, "job_f0", J + 1);
  fill_u32(c, fbmax, 0, J);
  launch_seg_exit_files(d_chf, d_nchf, fch_cap, d_sjf, P.d_jobs, ob_excl, ob.full, fnxt, fex, fcnt, fbmax, st);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_seg_compose, dim3(J), dim3(256), 2 * cap * sizeof(uint16_t), st, d_sjf, J, fex, fcnt, fbmax,
                     fcentry, fcseg0, fnseg, cap);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_small_scan, dim3(1), dim3(64), 0, st, fnseg, J, job_f0);
  LAUNCH_CHECK();
  uint32_t* file_first = dbuf<uint32_t>(c, "file_first", OB);
  launch_seg_mark(d_chf, d_nchf, fch_cap, d_sjf, fnxt, fcentry, fcseg0, job_f0, file_first, st);
  LAUNCH_CHECK();
  mark(c, "file_cuts");

  // --- per-file pre-layout (capacity: one file per block)
  const uint64_t FC = OB;
  OutFiles of;
  of.job = dbuf<uint32_t>(c, "of_job", FC);
  of.b0 = dbuf<uint64_t>(c, "of_b0", FC);
  of.nb = dbuf<uint32_t>(c, "of_nb", FC);
  of.data = dbuf<uint64_t>(c, "of_data", FC);
  of.nwin = dbuf<uint64_t>(c, "of_nwin", FC);
  of.w0 = dbuf<uint64_t>(c, "of_w0", FC + 1);
  of.filter_off = dbuf<uint64_t>(c, "of_foff", FC);
  of.filter_size = dbuf<uint64_t>(c, "of_fsize", FC);
  of.meta_off = dbuf<uint64_t>(c, "of_moff", FC);
  of.meta_size = dbuf<uint64_t>(c, "of_msize", FC);
  of.index_off = dbuf<uint64_t>(c, "of_ioff", FC);
  of.index_size = dbuf<uint64_t>(c, "of_isize", FC);
  of.size = dbuf<uint64_t>(c, "of_size", FC);
  of.out = dbuf<uint64_t>(c, "of_out", FC + 1);
  of.entries = dbuf<uint64_t>(c, "of_entries", FC);
  of.keyr = dbuf<uint64_t>(c, "of_keyr", 4 * FC);
  hipLaunchKernelGGL(k_file_pre, dim3(blocks_for(FC)), dim3(256), 0, st, job_f0, J, job_ob0, file_first, ob_excl,
                     FC, of);
  LAUNCH_CHECK();
  launch_scan<uint64_t, uint64_t>(of.nwin, FC, nullptr, of.w0, scan_tmp, st);
  LAUNCH_CHECK();
  // sizes needed to allocate window arrays and the encoder's LDS
  uint32_t* stats = dbuf<uint32_t>(c, "plan_stats", 5);
  fill_u32(c, stats, 0, 5);
  hipLaunchKernelGGL(k_plan_stats, dim3(std::min<uint32_t>(stride_grid(c, OB), c->n_cu)), dim3(256), 0, st, ob, job_ob0, J, OB,
                     gapcnt, stats);
  LAUNCH_CHECK();
  uint64_t NBLK, NF, NW;
  uint32_t max_bsize;
  bool big_blocks = true;
  uint64_t n_off = 0;  // blocks off the pipelined encoder's path
  uint64_t n_em = 0;   // blocks whose gap chunks are written entry-major
  {
    Mail m(c);
    const uint64_t* a = m.add(job_ob0 + J, 1);
    const uint64_t* b = m.add(job_f0 + J, 1);
    const uint64_t* w = m.add(of.w0 + FC, 1);
    const uint32_t* x = m.add(stats, 5);
    m.flush();
    NBLK = *a;
    NF = *b;
    NW = *w;
    max_bsize = x[0];
    big_blocks = x[3] != 0;
    n_off = x[3];
    n_em = P.kw8 <= GAP_KW8 ? x[4] : 0;
    c->counters.emplace_back("max_block_bytes", (double)max_bsize);
  }

  uint32_t* win_keys = dbuf<uint32_t>(c, "win_keys", NW);
  uint32_t* win_fb = dbuf<uint32_t>(c, "win_fb", NW);
  uint32_t* win_file = dbuf<uint32_t>(c, "win_file", NW);
  uint64_t* win_bytes = dbuf<uint64_t>(c, "win_bytes", NW);
  uint64_t* win_off = dbuf<uint64_t>(c, "win_off", NW + 1);
  fill_u32(c, win_keys, 0, NW);
  fill_u32(c, win_fb, 0xFFFFFFFFu, NW);
  hipLaunchKernelGGL(k_block_post, dim3(blocks_for(NBLK)), dim3(256), 0, st, job_f0 + J, of, ob_excl, job_ob0, J,
                     P.tu, P.d_surv, NBLK, ob, win_keys, win_fb);
  LAUNCH_CHECK();
  uint32_t* wstat = dbuf<uint32_t>(c, "win_stat", 1);
  fill_u32(c, wstat, 0, 1);
  hipLaunchKernelGGL(k_win_size, dim3(std::min<uint32_t>(stride_grid(c, NW), c->n_cu)), dim3(256), 0, st, of.w0 + FC,
                     of.w0, NF, of, P.d_jobs, win_keys, NW, win_bytes, win_file, wstat);
  LAUNCH_CHECK();
  uint64_t* scan_tmpw = dbuf<uint64_t>(c, "scan_tmpw", NW / 2048 + 8);
  launch_scan<uint64_t, uint64_t>(win_bytes, NW, nullptr, win_off, scan_tmpw, st);
  LAUNCH_CHECK();
  uint64_t* ie_off = dbuf<uint64_t>(c, "ie_off", NBLK + 1);
  launch_scan<uint32_t, uint64_t>(ob.ie_size, NBLK, nullptr, ie_off, scan_tmp, st);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_file_layout, dim3(blocks_for(NF)), dim3(256), 0, st, job_f0 + J, of, win_off, ie_off, NF);
  LAUNCH_CHECK();
  if (P.compress) {  // a table whose first block is compressed keeps its smallest key after it
    uint64_t* stride = dbuf<uint64_t>(c, "zw_fstride", NF);
    hipLaunchKernelGGL(k_zslots, dim3(blocks_for(NF)), dim3(256), 0, st, of, ob, P.d_surv, P.tu, ztype, job_f0 + J,
                       NF, stride);
    LAUNCH_CHECK();
    launch_scan<uint64_t, uint64_t>(stride, NF, nullptr, of.out, scan_tmp, st);
  } else {
    launch_scan<uint64_t, uint64_t>(of.size, NF, nullptr, of.out, scan_tmp, st);
  }
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_file_entries, dim3(blocks_for(NF)), dim3(256), 0, st, of, ob, P.d_surv, P.tu, ie_off, NF,
                     (const uint8_t*)ztype);
  LAUNCH_CHECK();
  BlockRec* brec = dbuf<BlockRec>(c, "blk_rec", NBLK);
  // a few blocks off the pipelined path are listed, so that k_encode_big
  // need not look at every block; when they are many it looks at every block
  uint64_t* off_list = nullptr;
  uint32_t* off_n = nullptr;
  if (!P.compress && n_off && n_off <= NBLK / 8) {
    off_list = dbuf<uint64_t>(c, "enc_off_list", n_off);
    off_n = dbuf<uint32_t>(c, "enc_off_n", 1);
    fill_u32(c, off_n, 0, 1);
  }
  hipLaunchKernelGGL(k_block_dst, dim3(blocks_for(NBLK)), dim3(256), 0, st, ob, of, P.d_jobs, job_ob0 + J, NBLK, brec,
                     off_list, off_n, n_off);
  LAUNCH_CHECK();
  O.file_out.assign(NF + 1, 0);
  O.file_size.assign(NF, 0);
  O.file_entries.assign(NF, 0);
  O.file_keys.assign(4 * NF, 0);
  uint32_t max_win = 0;
  uint64_t dout = 0;
  {
    Mail m(c);
    const uint64_t* fo = m.add(of.out, NF + 1);
    const uint64_t* fe = m.add(of.entries, NF);
    const uint64_t* fs = m.add(of.size, NF);
    const uint64_t* fk = m.add(of.keyr, 4 * NF);
    const uint64_t* jf = m.add(job_f0, J + 1);
    const uint32_t* mw = m.add(wstat, 1);
    const uint64_t* dx = m.add(ob_excl + NBLK, 1);
    m.flush();
    memcpy(O.file_out.data(), fo, (NF + 1) * 8);
    memcpy(O.file_entries.data(), fe, NF * 8);
    memcpy(O.file_size.data(), fs, NF * 8);
    memcpy(O.file_keys.data(), fk, NF * 32);
    memcpy(O.job_f0.data(), jf, (J + 1) * 8);
    max_win = *mw;
    dout = *dx;
  }
  mark(c, "layout");
  O.total_bytes = O.file_out[NF];
  c->counters.emplace_back("data_bytes_out", (double)dout);
  c->counters.emplace_back("data_blocks_out", (double)NBLK);
  c->counters.emplace_back("survivors", (double)S);
  c->counters.emplace_back("files_out", (double)NF);
  uint8_t* out = out_buffer(c, O.total_bytes + 64);
  O.d_out = out;

  // --- writers
  if (P.compress) {
    // stored bytes into place, then their trailers' checksums
    hipLaunchKernelGGL(k_zplace, dim3(std::max<uint32_t>(1, (uint32_t)std::min<uint64_t>((NBLK + 3) / 4,
                                                                                      (uint64_t)c->n_cu * 16))),
                       dim3(256), 0, st, brec, job_ob0 + J, zstage, zbuf, zoff, ztype, out);
    LAUNCH_CHECK();
    const uint64_t segs = dout / CRC_SEG_BYTES + NBLK + 1;
    uint32_t* part = dbuf<uint32_t>(c, "zw_crc_part", segs);
    uint64_t* mseg = dbuf<uint64_t>(c, "zw_crc_mseg", NBLK + 1);
    launch_crc_zblocks(brec, job_ob0 + J, NBLK, out, c->d_crc, part, mseg, crc_multi_grid(c, dout, NBLK), st);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_zkeys, dim3(blocks_for(NF)), dim3(256), 0, st, of, ob, P.d_surv, P.tu, ztype, P.kw8, NF,
                       out);
    LAUNCH_CHECK();
  } else {
    A.of = of;
    A.out = out;
    A.blk = brec;
    // gap chunks: every block's chunk slots (J16 + 1 at most), then the
    // chunks that are not value interiors assembled once
    launch_scan<uint32_t, uint64_t>(gapcnt, NBLK, nullptr, gap_base, scan_gap, st);
    LAUNCH_CHECK();
    const uint64_t slots = dout / 16 + 2 * NBLK + 1;
    A.gapbuf = dbuf<uint4>(c, "gap_buf", slots);
    KTimer kg(c, "k_gaps");
    // 16 threads per block; each kernel only when it has blocks
    if (n_em < NBLK) hipLaunchKernelGGL(k_gaps<false>, dim3(stride_grid(c, NBLK * 16)), dim3(256), 0, st, A);
    if (n_em) hipLaunchKernelGGL(k_gaps<true>, dim3(stride_grid(c, NBLK * GAP_EM_GROUP)), dim3(256), 0, st, A);
    LAUNCH_CHECK();
    kg.stop();
    launch_encode(c, A, NBLK, big_blocks, off_list, n_off);
  }
  mark(c, "encode");
  if (NW) {
    uint64_t* hash = dbuf<uint64_t>(c, "key_hash", S);
    FilterArgs F;
    F.jobs = P.d_jobs;
    F.ob = ob;
    F.of = of;
    F.tu = P.tu;
    F.surv = P.d_surv;
    F.nwin = of.w0 + FC;
    F.win_keys = win_keys;
    F.win_fb = win_fb;
    F.win_file = win_file;
    F.win_bytes = win_bytes;
    F.win_off = win_off;
    F.hash = hash;
    F.out = out;
    F.kw8 = P.kw8;
    F.lds_bytes = (uint32_t)(((uint64_t)max_win + 16 + 15) & ~15ull);
    KTimer kt(c, "k_filter");
    hipLaunchKernelGGL(k_key_hash, dim3(blocks_for(S)), dim3(256), 0, st, P.d_surv, P.tu, P.kw8, S, hash);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_filter_small, dim3(stride_grid(c, NW)), dim3(256), 0, st, F);
    LAUNCH_CHECK();
    if (max_win > 64 + 1) {
      const size_t budget = c->lds_limit - 2048;
      int waves = 4;
      while (waves > 1 && (size_t)F.lds_bytes * waves > budget) waves--;
      if ((size_t)F.lds_bytes * waves > budget)
        throw Fail{LUDA_UNSUPPORTED, "filter of " + std::to_string(max_win) + " bytes exceeds the filter kernel's LDS"};
      const uint32_t grid =
          (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((NW + waves - 1) / waves, (uint64_t)c->n_cu * 8));
      hipLaunchKernelGGL(k_filter, dim3(grid), dim3(waves * 64), (size_t)F.lds_bytes * waves, st, F);
      LAUNCH_CHECK();
    }
    kt.stop();
    hipLaunchKernelGGL(k_filter_offsets, dim3(blocks_for(NW)), dim3(256), 0, st, of, of.w0 + FC, win_file, win_off,
                       NW, out);
    LAUNCH_CHECK();
  }
  mark(c, "filter");
  hipLaunchKernelGGL(k_index_write, dim3(blocks_for(NBLK)), dim3(256), 0, st, ob, of, P.tu, P.d_surv, ie_off,
                     job_ob0 + J, P.kw8, NBLK, out);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_meta, dim3(blocks_for(NF)), dim3(256), 0, st, of, win_off, job_f0 + J, NF, out);
  LAUNCH_CHECK();
  {
    KTimer kt(c, "k_crc_tables");
    const uint64_t segs = O.total_bytes / CRC_SEG_BYTES + 3 * NF + 1;
    uint32_t* part = dbuf<uint32_t>(c, "of_crc_part", segs);
    uint64_t* mseg = dbuf<uint64_t>(c, "of_crc_mseg", 3 * NF + 1);
    launch_crc_files(of, job_f0 + J, NF, out, c->d_crc, part, mseg, crc_multi_grid(c, O.total_bytes, 3 * NF), st);
    LAUNCH_CHECK();
    kt.stop();
  }
  mark(c, "meta");
}

// ---------------------------------------------------------------------------
// The compaction pipeline over a batch.

struct HostJob {
  uint32_t in_first = 0, n_in = 0;
  uint64_t bytes_in = 0;
  bool failed = false;
  uint64_t err_key = ERR_NONE;
};

// one pass over a set of blocks: restart counts, checksums, interval map,
// count walk, and the prefix sums that place every interval's output
struct WalkPlan {
  uint32_t* nr;
  uint64_t* ibase;  // nb + 1
  uint8_t* ok;
  uint32_t* iblk;
  uint32_t* icnt;
  uint64_t* ient;   // ni + 1
  uint64_t NI = 0;  // intervals
};

// The paper's cooperative sort (Sec. III-D): the decoded entries' keys go to
// the host, are sorted there, and the order comes back.  Same order as the
// device merge: user key bytes ascending (a shorter key first), tag
// descending, then decode position (input, then position) ascending.  Jobs
// that already failed keep their decode order.
void host_sort_order(luda_ctx* c, const Tuples& tu, uint32_t kw8, uint64_t N, uint32_t J,
                     const std::vector<HostJob>& hj, const std::vector<uint64_t>& job_e0, uint32_t* d_ord) {
  hipStream_t st = c->stream;
  std::vector<uint64_t> heap(N * kw8), tag(N);
  std::vector<uint32_t> ulen(N), ord(N);
  HIPCK(hipMemcpyAsync(heap.data(), tu.heap, N * kw8 * 8, hipMemcpyDeviceToHost, st));
  HIPCK(hipMemcpyAsync(tag.data(), tu.tag, N * 8, hipMemcpyDeviceToHost, st));
  HIPCK(hipMemcpyAsync(ulen.data(), tu.ulen, N * 4, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  const uint8_t* kb = (const uint8_t*)heap.data();
  const uint64_t slot = (uint64_t)kw8 * 8;
  auto less = [&](uint32_t a, uint32_t b) {
    const uint32_t la = std::min<uint64_t>(ulen[a], slot), lb = std::min<uint64_t>(ulen[b], slot);
    const int cm = memcmp(kb + a * slot, kb + b * slot, std::min(la, lb));
    if (cm) return cm < 0;
    if (la != lb) return la < lb;
    if (tag[a] != tag[b]) return tag[a] > tag[b];
    return a < b;
  };
  for (uint64_t i = 0; i < N; i++) ord[i] = (uint32_t)i;
  const unsigned T = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  for (uint32_t j = 0; j < J; j++) {
    if (hj[j].failed) continue;
    uint32_t* a0 = ord.data() + job_e0[j];
    const uint64_t n = job_e0[j + 1] - job_e0[j];
    if (n < 2) continue;
    // T sorted pieces, then pairwise merges
    std::vector<uint64_t> cut(T + 1);
    for (unsigned t = 0; t <= T; t++) cut[t] = n * t / T;
    std::vector<std::thread> th;
    for (unsigned t = 0; t < T; t++) th.emplace_back([&, t] { std::sort(a0 + cut[t], a0 + cut[t + 1], less); });
    for (auto& x : th) x.join();
    for (unsigned w = 1; w < T; w *= 2) {
      th.clear();
      for (unsigned t = 0; t + w < T; t += 2 * w)
        th.emplace_back([&, t, w] {
          std::inplace_merge(a0 + cut[t], a0 + cut[t + w], a0 + cut[std::min(T, t + 2 * w)], less);
        });
      for (auto& x : th) x.join();
    }
  }
  HIPCK(hipMemcpyAsync(d_ord, ord.data(), N * 4, hipMemcpyHostToDevice, st));
  HIPCK(hipStreamSynchronize(st));  // ord is freed on return
}

void run_batch(luda_ctx* c, const luda_job* jobs, uint32_t J, bool dev_inputs, luda_result* results) {
  using clock = std::chrono::steady_clock;
  const auto t0 = clock::now();
  hipStream_t st = c->stream;
  begin_call(c);
  mark(c, "start");
  std::vector<HostJob> hj(J);
  std::vector<JobDesc> jd(J);
  std::vector<uint64_t> in_ptr, in_size, job_in_first(J + 1);
  std::vector<uint32_t> in_job, in_local;
  std::vector<uint64_t> snaps;  // every job's live snapshots, back to back
  uint64_t G = 0, total_in = 0;
  bool any_compression = false;
  for (uint32_t j = 0; j < J; j++) {
    if (snaps.size() + jobs[j].options.n_snapshots > 0xFFFFFFF0ull)
      throw Fail{LUDA_UNSUPPORTED, "too many snapshots in one call"};
    hj[j].in_first = (uint32_t)G;
    hj[j].n_in = jobs[j].n_inputs;
    job_in_first[j] = G;
    const luda_options& o = jobs[j].options;
    jd[j] = JobDesc{o.block_size, o.restart_interval, o.bloom_bits_per_key, o.bottommost ? 1u : 0u,
                    o.target_file_size, (uint32_t)G, jobs[j].n_inputs, (uint32_t)snaps.size(), o.n_snapshots,
                    o.compression, 0};
    if (o.compression) any_compression = true;
    snaps.insert(snaps.end(), o.snapshots, o.snapshots + o.n_snapshots);
    for (uint32_t i = 0; i < jobs[j].n_inputs; i++) {
      in_size.push_back(jobs[j].inputs[i].size);
      in_job.push_back(j);
      in_local.push_back(i);
      hj[j].bytes_in += jobs[j].inputs[i].size;
      total_in += (jobs[j].inputs[i].size + 255) & ~255ull;
    }
    G += jobs[j].n_inputs;
  }
  job_in_first[J] = G;
  if (G > 0xFFFFFFF0ull) throw Fail{LUDA_UNSUPPORTED, "too many inputs"};
  const uint32_t NG = (uint32_t)G;
  // inputs on the device
  if (dev_inputs) {
    for (uint32_t j = 0; j < J; j++)
      for (uint32_t i = 0; i < jobs[j].n_inputs; i++) in_ptr.push_back((uint64_t)(uintptr_t)jobs[j].inputs[i].data);
  } else {
    uint8_t* arena = dbuf<uint8_t>(c, "in_arena", total_in + 256);
    uint64_t off = 0;
    for (uint32_t j = 0; j < J; j++)
      for (uint32_t i = 0; i < jobs[j].n_inputs; i++) {
        const luda_buf& b = jobs[j].inputs[i];
        if (b.size) upload_host(c, arena + off, b.data, b.size);
        in_ptr.push_back((uint64_t)(uintptr_t)(arena + off));
        off += (b.size + 255) & ~255ull;
      }
  }
  mark(c, "h2d");
  JobDesc* d_jobs = dbuf<JobDesc>(c, "jobs", J);
  uint64_t* d_snaps = dbuf<uint64_t>(c, "snapshots", snaps.size());
  if (!snaps.empty()) up(c, d_snaps, snaps.data(), snaps.size() * 8);
  Inputs in;
  in.n = NG;
  uint64_t* d_in_ptr = dbuf<uint64_t>(c, "in_ptr", NG);
  uint64_t* d_in_size = dbuf<uint64_t>(c, "in_size", NG);
  uint32_t* d_in_job = dbuf<uint32_t>(c, "in_job", NG);
  uint32_t* d_in_local = dbuf<uint32_t>(c, "in_local", NG);
  uint64_t* d_job_in_first = dbuf<uint64_t>(c, "job_in_first", J + 1);
  uint64_t* d_ng = dbuf<uint64_t>(c, "n_inputs", 1);
  up(c, d_jobs, jd.data(), J * sizeof(JobDesc));
  up(c, d_in_ptr, in_ptr.data(), (size_t)NG * 8);
  up(c, d_in_size, in_size.data(), (size_t)NG * 8);
  up(c, d_in_job, in_job.data(), (size_t)NG * 4);
  up(c, d_in_local, in_local.data(), (size_t)NG * 4);
  up(c, d_job_in_first, job_in_first.data(), (size_t)(J + 1) * 8);
  up(c, d_ng, &G, 8);
  up_flush(c);
  in.ptr = d_in_ptr;
  in.size = d_in_size;
  in.job = d_in_job;
  in.local = d_in_local;
  unsigned long long* err = dbuf<unsigned long long>(c, "err", J);
  fill_u64(c, err, ERR_NONE, J);
  unsigned long long* d_bytes = dbuf<unsigned long long>(c, "data_bytes", 1);
  fill_u64(c, d_bytes, 0, 1);
  uint32_t* d_maxk = dbuf<uint32_t>(c, "maxklen", 1);
  fill_u32(c, d_maxk, 0, 1);

  WalkArgs WA;
  memset(&WA, 0, sizeof WA);
  WA.in = in;
  WA.err = err;

  // --- index blocks (one per input): footer, restart counts, checksums
  WalkSet ix;
  ix.ptr = dbuf<uint64_t>(c, "ix_ptr", NG);
  ix.size = dbuf<uint32_t>(c, "ix_size", NG);
  ix.input = dbuf<uint32_t>(c, "ix_input", NG);
  ix.local = dbuf<uint32_t>(c, "ix_local", NG);
  ix.skip = dbuf<uint8_t>(c, "ix_skip", NG);
  ix.n_dev = d_ng;
  ix.where = W_INDEX;
  WalkPlan IX;
  IX.nr = dbuf<uint32_t>(c, "ix_nr", NG);
  IX.ibase = dbuf<uint64_t>(c, "ix_ibase", (uint64_t)NG + 1);
  IX.ok = dbuf<uint8_t>(c, "ix_ok", NG);
  if (NG) {
    hipLaunchKernelGGL(k_footer, dim3(blocks_for(NG)), dim3(256), 0, st, in, ix, err);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_blk_nr, dim3(blocks_for(NG)), dim3(256), 0, st, ix, in, IX.nr, err, ZPass{});
    LAUNCH_CHECK();
    {
      const uint64_t segs = total_in / CRC_SEG_BYTES + NG + 1;
      uint32_t* part = dbuf<uint32_t>(c, "ix_crc_part", segs);
      uint64_t* mseg = dbuf<uint64_t>(c, "ix_crc_mseg", (uint64_t)NG + 1);
      launch_crc_index(ix, in, c->d_crc, IX.ok, err, NG, part, mseg, crc_multi_grid(c, total_in, NG), st);
      LAUNCH_CHECK();
    }

    uint64_t* scan_g = dbuf<uint64_t>(c, "scan_tmp_g", NG / 2048 + 8);
    launch_scan<uint32_t, uint64_t>(IX.nr, NG, nullptr, IX.ibase, scan_g, st);
    LAUNCH_CHECK();
    Mail m(c);
    const uint64_t* p = m.add(IX.ibase + NG, 1);
    m.flush();
    IX.NI = *p;
  } else {
    fill_u64(c, IX.ibase, 0, 1);
  }
  // index intervals: count data block handles, place them
  IX.iblk = dbuf<uint32_t>(c, "ix_iblk", IX.NI);
  IX.icnt = dbuf<uint32_t>(c, "ix_icnt", IX.NI);
  IX.ient = dbuf<uint64_t>(c, "ix_ient", IX.NI + 1);
  uint64_t NB = 0;
  WA.ws = ix;
  WA.ok = IX.ok;
  WA.nr = IX.nr;
  WA.ibase = IX.ibase;
  WA.iblk = IX.iblk;
  WA.ni_dev = IX.ibase + NG;
  WA.icnt = IX.icnt;
  WA.maxklen = d_maxk;
  if (IX.NI) {
    hipLaunchKernelGGL(k_imap, dim3(stride_grid(c, IX.NI)), dim3(256), 0, st, ix, IX.ibase, IX.ibase + NG, IX.iblk);
    LAUNCH_CHECK();
    hipLaunchKernelGGL((k_walk<0, 0>), dim3(stride_grid(c, IX.NI)), dim3(256), 0, st, WA);
    LAUNCH_CHECK();
    uint64_t* scan_i = dbuf<uint64_t>(c, "scan_tmp_i", IX.NI / 2048 + 8);
    launch_scan<uint32_t, uint64_t>(IX.icnt, IX.NI, nullptr, IX.ient, scan_i, st);
    LAUNCH_CHECK();
    Mail m(c);
    const uint64_t* p = m.add(IX.ient + IX.NI, 1);
    m.flush();
    NB = *p;
  } else {
    fill_u64(c, IX.ient, 0, 1);
  }
  if (NB > 0xFFFFFFF0ull) throw Fail{LUDA_UNSUPPORTED, "too many data blocks"};
  mark(c, "index");

  // --- data block table from the index entries
  WalkSet db;
  db.ptr = dbuf<uint64_t>(c, "db_ptr", NB);
  db.size = dbuf<uint32_t>(c, "db_size", NB);
  db.input = dbuf<uint32_t>(c, "db_input", NB);
  db.local = dbuf<uint32_t>(c, "db_local", NB);
  db.skip = dbuf<uint8_t>(c, "db_skip", NB);
  db.n_dev = IX.ient + IX.NI;
  db.where = W_DATA;
  // first data block of each input: the first output of its index block
  uint64_t* in_blk0 = dbuf<uint64_t>(c, "in_blk0", (uint64_t)NG + 1);
  hipLaunchKernelGGL(k_ranges, dim3(blocks_for((uint64_t)NG + 1)), dim3(256), 0, st, IX.ient, IX.ibase, nullptr,
                     NG + 1, in_blk0);
  LAUNCH_CHECK();
  if (IX.NI) {
    WA.ient = IX.ient;
    WA.out_blk = db;
    WA.in_blk0 = in_blk0;
    hipLaunchKernelGGL((k_walk<0, 1>), dim3(stride_grid(c, IX.NI)), dim3(256), 0, st, WA);
    LAUNCH_CHECK();
  }

  // --- data blocks: restart counts, checksums, count walk
  WalkPlan DB;
  DB.nr = dbuf<uint32_t>(c, "db_nr", NB);
  DB.ibase = dbuf<uint64_t>(c, "db_ibase", NB + 1);
  DB.ok = dbuf<uint8_t>(c, "db_ok", NB);
  uint64_t* zcap = dbuf<uint64_t>(c, "z_cap", NB);
  unsigned long long* ztot = dbuf<unsigned long long>(c, "z_tot", 2);
  fill_u64(c, ztot, 0, 2);
  if (NB) {
    hipLaunchKernelGGL(k_blk_nr, dim3(stride_grid(c, NB)), dim3(256), 0, st, db, in, DB.nr, err,
                       ZPass{zcap, ztot, nullptr, 0});
    LAUNCH_CHECK();
    uint64_t* scan_b = dbuf<uint64_t>(c, "scan_tmp_b", NB / 2048 + 8);
    launch_scan<uint32_t, uint64_t>(DB.nr, NB, nullptr, DB.ibase, scan_b, st);
    LAUNCH_CHECK();
    {
      const uint32_t cw = c->tp.crc_waves;
      int occ = 0;
      HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_crc_wave, cw * 64, 0));
      occ = std::max(occ, 1);
      const uint32_t grid =
          (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((NB + cw - 1) / cw, (uint64_t)c->n_cu * occ));
      KTimer kt(c, "k_crc_data");
      hipLaunchKernelGGL(k_crc_wave, dim3(grid), dim3(cw * 64), 0, st, db, in, c->d_crc, DB.ok, err, d_bytes);
      LAUNCH_CHECK();
      kt.stop();
      c->counters.emplace_back("crc_groups_per_cu", (double)occ);
      c->counters.emplace_back("crc_groups", (double)grid);
    }
    Mail m(c);
    const uint64_t* p = m.add(DB.ibase + NB, 1);
    const unsigned long long* by = m.add(d_bytes, 1);
    const unsigned long long* zt = m.add(ztot, 2);
    m.flush();
    DB.NI = *p;
    c->counters.emplace_back("data_bytes_in", (double)*by);
    const uint64_t zblocks = zt[0], zbytes = zt[1];
    if (zblocks) {
      // compressed blocks: raw bytes into staging, then their restart counts
      // and the interval bases again
      c->counters.emplace_back("compressed_blocks_in", (double)zblocks);
      uint8_t* stage = dbuf<uint8_t>(c, "z_stage", zbytes + 64);
      uint64_t* zoff = dbuf<uint64_t>(c, "z_off", NB + 1);
      uint64_t* scan_z = dbuf<uint64_t>(c, "scan_tmp_z", NB / 2048 + 8);
      launch_scan<uint64_t, uint64_t>(zcap, NB, nullptr, zoff, scan_z, st);
      LAUNCH_CHECK();
      KTimer kt(c, "k_unsnappy");
      hipLaunchKernelGGL(k_unsnappy, dim3(std::max<uint32_t>(1, (uint32_t)std::min<uint64_t>((zblocks + 1) / 2,
                                                                                         (uint64_t)c->n_cu * 8))),
                         dim3(128), 0, st, db, in, DB.ok, zcap, zoff, stage, err);
      LAUNCH_CHECK();
      kt.stop();
      hipLaunchKernelGGL(k_blk_nr, dim3(stride_grid(c, NB)), dim3(256), 0, st, db, in, DB.nr, err,
                         ZPass{zcap, ztot, DB.ok, 1});
      LAUNCH_CHECK();
      launch_scan<uint32_t, uint64_t>(DB.nr, NB, nullptr, DB.ibase, scan_b, st);
      LAUNCH_CHECK();
      Mail m2(c);
      const uint64_t* p2 = m2.add(DB.ibase + NB, 1);
      m2.flush();
      DB.NI = *p2;
    }
  } else {
    fill_u64(c, DB.ibase, 0, 1);
    c->counters.emplace_back("data_bytes_in", 0.0);
  }
  c->counters.emplace_back("data_blocks_in", (double)NB);
  mark(c, "data_crc");
  DB.iblk = dbuf<uint32_t>(c, "db_iblk", DB.NI);
  DB.icnt = dbuf<uint32_t>(c, "db_icnt", DB.NI);
  DB.ient = dbuf<uint64_t>(c, "db_ient", DB.NI + 1);
  WA.ws = db;
  WA.ok = DB.ok;
  WA.nr = DB.nr;
  WA.ibase = DB.ibase;
  WA.iblk = DB.iblk;
  WA.ni_dev = DB.ibase + NB;
  WA.icnt = DB.icnt;
  WA.ient = DB.ient;
  uint64_t N = 0;
  uint32_t maxklen = 0;
  if (DB.NI) {
    hipLaunchKernelGGL(k_imap, dim3(stride_grid(c, DB.NI)), dim3(256), 0, st, db, DB.ibase, DB.ibase + NB, DB.iblk);
    LAUNCH_CHECK();
    {
      KTimer kt(c, "k_walk_count");
      hipLaunchKernelGGL((k_walk<1, 0>), dim3(stride_grid(c, DB.NI)), dim3(256), 0, st, WA);
      LAUNCH_CHECK();
      kt.stop();
    }
    uint64_t* scan_e = dbuf<uint64_t>(c, "scan_tmp_e", DB.NI / 2048 + 8);
    launch_scan<uint32_t, uint64_t>(DB.icnt, DB.NI, nullptr, DB.ient, scan_e, st);
    LAUNCH_CHECK();
    Mail m(c);
    const uint64_t* p = m.add(DB.ient + DB.NI, 1);
    const uint32_t* mk = m.add(d_maxk, 1);
    m.flush();
    N = *p;
    maxklen = *mk;
  } else {
    fill_u64(c, DB.ient, 0, 1);
  }
  if (N > 0xFFFFFFF0ull) throw Fail{LUDA_UNSUPPORTED, "more than 2^32 entries in one call"};
  c->counters.emplace_back("entries_in", (double)N);
  const uint32_t ulen_max = maxklen > 8 ? maxklen - 8 : 0;
  const uint32_t kw8 = std::max<uint32_t>(2, (ulen_max + 7) / 8);
  c->counters.emplace_back("kw8", (double)kw8);
  if ((double)N * kw8 * 8 > 64e9) throw Fail{LUDA_UNSUPPORTED, "key slots would exceed 64 GB"};
  Tuples tu;
  tu.kd = dbuf<uint64_t>(c, "tu_kd", N);
  tu.sn = dbuf<uint64_t>(c, "tu_sn", N);
  tu.vp = dbuf<uint64_t>(c, "tu_vp", N);
  tu.vlen = dbuf<uint32_t>(c, "tu_vlen", N);
  tu.blk = dbuf<uint32_t>(c, "tu_blk", N);
  tu.eoff = dbuf<uint32_t>(c, "tu_eoff", N);
  tu.kp0 = dbuf<uint64_t>(c, "tu_kp0", N);
  tu.kp1 = dbuf<uint64_t>(c, "tu_kp1", N);
  tu.tag = dbuf<uint64_t>(c, "tu_tag", N);
  tu.ulen = dbuf<uint32_t>(c, "tu_ulen", N);
  tu.heap = dbuf<uint64_t>(c, "tu_heap", N * kw8);
  const uint64_t* d_n = DB.ient + DB.NI;
  // entry ranges of inputs and jobs
  uint64_t* in_e0 = dbuf<uint64_t>(c, "in_e0", (uint64_t)NG + 1);
  uint64_t* job_e0d = dbuf<uint64_t>(c, "job_e0", J + 1);
  hipLaunchKernelGGL(k_ranges, dim3(blocks_for((uint64_t)NG + 1)), dim3(256), 0, st, DB.ient, DB.ibase, in_blk0,
                     NG + 1, in_e0);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gather_u64, dim3(blocks_for(J + 1)), dim3(256), 0, st, in_e0, d_job_in_first, J + 1, job_e0d);
  LAUNCH_CHECK();
  int32_t* in_cmp = dbuf<int32_t>(c, "in_cmp", NG);
  fill_u32(c, in_cmp, 2u, NG);
  if (N) {
    WA.tu = tu;
    {
      KTimer kt(c, "k_walk_emit");
      hipLaunchKernelGGL((k_walk<1, 1>), dim3(stride_grid(c, DB.NI)), dim3(256), 0, st, WA);
      LAUNCH_CHECK();
      kt.stop();
    }
    {
      KTimer kt(c, "k_keys");
      hipLaunchKernelGGL(k_keys, dim3(stride_grid(c, N)), dim3(256), 0, st, tu, db, in, kw8, d_n, err);
      LAUNCH_CHECK();
      kt.stop();
    }
    hipLaunchKernelGGL(k_order, dim3(stride_grid(c, N)), dim3(256), 0, st, tu, db, in, in_e0, kw8, d_n, in_cmp, err);
    LAUNCH_CHECK();
  }
  std::vector<int32_t> h_cmp(NG);
  std::vector<uint64_t> job_e0(J + 1), in_e0h((size_t)NG + 1), errs(J);
  {
    Mail m(c);
    const int32_t* a = m.add(in_cmp, NG);
    const uint64_t* b = m.add(job_e0d, J + 1);
    const uint64_t* d = m.add(in_e0, (size_t)NG + 1);
    const uint64_t* e = m.add((const uint64_t*)err, J);
    m.flush();
    memcpy(h_cmp.data(), a, (size_t)NG * 4);
    memcpy(job_e0.data(), b, (size_t)(J + 1) * 8);
    memcpy(in_e0h.data(), d, ((size_t)NG + 1) * 8);
    memcpy(errs.data(), e, (size_t)J * 8);
  }
  mark(c, "keys");
  for (uint32_t j = 0; j < J; j++) {
    hj[j].err_key = errs[j];
    hj[j].failed = errs[j] != ERR_NONE;
  }

  // --- merge rounds: runs are maximal stretches of consecutive inputs where
  // each table's first key follows the previous table's last key
  struct Run {
    uint64_t a, n;
  };
  std::vector<std::vector<Run>> runs(J);
  bool need_merge = false;
  for (uint32_t j = 0; j < J; j++) {
    if (hj[j].failed) {
      if (job_e0[j + 1] > job_e0[j]) runs[j].push_back(Run{job_e0[j], job_e0[j + 1] - job_e0[j]});
      continue;
    }
    for (uint32_t i = 0; i < hj[j].n_in; i++) {
      const uint32_t g = hj[j].in_first + i;
      const uint64_t a = in_e0h[g], n = in_e0h[g + 1] - in_e0h[g];
      if (!n) continue;
      if (!runs[j].empty() && h_cmp[g] == -1 && runs[j].back().a + runs[j].back().n == a) runs[j].back().n += n;
      else runs[j].push_back(Run{a, n});
    }
    if (runs[j].size() > 1) need_merge = true;
  }
  uint32_t* ordA = dbuf<uint32_t>(c, "ordA", N);
  uint32_t* ordB = dbuf<uint32_t>(c, "ordB", N);
  if (c->host_sort && N) {
    host_sort_order(c, tu, kw8, N, J, hj, job_e0, ordA);
    need_merge = false;
  } else if (N) {
    hipLaunchKernelGGL(k_iota, dim3(blocks_for(N)), dim3(256), 0, st, ordA, N);
    LAUNCH_CHECK();
  }
  uint32_t* ord = ordA;
  int round = 0;
  while (need_merge) {
    std::vector<MergeTask> tasks;
    need_merge = false;
    for (uint32_t j = 0; j < J; j++) {
      std::vector<Run> next;
      const auto& rs = runs[j];
      for (size_t k = 0; k < rs.size(); k += 2) {
        if (k + 1 < rs.size()) {
          tasks.push_back(MergeTask{(uint32_t)rs[k].a, (uint32_t)rs[k].n, (uint32_t)rs[k + 1].a, (uint32_t)rs[k + 1].n,
                                    rs[k].a});
          next.push_back(Run{rs[k].a, rs[k].n + rs[k + 1].n});
        } else {
          tasks.push_back(MergeTask{(uint32_t)rs[k].a, (uint32_t)rs[k].n, 0, 0, rs[k].a});
          next.push_back(rs[k]);
        }
      }
      runs[j] = next;
      if (runs[j].size() > 1) need_merge = true;
    }
    // the tasks must tile [0, N) in order
    std::sort(tasks.begin(), tasks.end(), [](const MergeTask& x, const MergeTask& y) { return x.out0 < y.out0; });
    std::vector<MergeTask> tiled;
    uint64_t pos = 0;
    for (auto& t : tasks) {
      if (t.la + (uint64_t)t.lb == 0) continue;
      if (t.out0 > pos) tiled.push_back(MergeTask{(uint32_t)pos, (uint32_t)(t.out0 - pos), 0, 0, pos});
      tiled.push_back(t);
      pos = t.out0 + t.la + t.lb;
    }
    if (pos < N) tiled.push_back(MergeTask{(uint32_t)pos, (uint32_t)(N - pos), 0, 0, pos});
    MergeTask* d_tasks = dbuf<MergeTask>(c, "merge_tasks" + std::to_string(round), tiled.size());
    up(c, d_tasks, tiled.data(), tiled.size() * sizeof(MergeTask));
    up_flush(c);
    uint32_t* dst = (ord == ordA) ? ordB : ordA;
    const uint64_t threads = (N + MERGE_ITEMS_PER_THREAD - 1) / MERGE_ITEMS_PER_THREAD;
    KTimer kt(c, "k_merge");
    hipLaunchKernelGGL(k_merge, dim3(blocks_for(threads)), dim3(256), 0, st, d_tasks, (uint32_t)tiled.size(), ord, dst,
                       tu, kw8, N);
    LAUNCH_CHECK();
    kt.stop();
    ord = dst;
    round++;
  }
  mark(c, "merge");
  // --- drop shadowed versions and bottom-level deletions
  uint32_t* keep = dbuf<uint32_t>(c, "keep", N);
  uint32_t* kpos = dbuf<uint32_t>(c, "kpos", N + 1);
  uint32_t* scan32 = dbuf<uint32_t>(c, "scan_tmp32", N / 2048 + 8);
  unsigned long long* shadowed = dbuf<unsigned long long>(c, "shadowed", J);
  unsigned long long* tomb = dbuf<unsigned long long>(c, "tomb", J);
  fill_u64(c, shadowed, 0, J);
  fill_u64(c, tomb, 0, J);
  std::vector<uint32_t> active(J);
  for (uint32_t j = 0; j < J; j++) active[j] = hj[j].failed ? 0u : 1u;
  uint32_t* d_active = dbuf<uint32_t>(c, "job_active", J);
  up(c, d_active, active.data(), (size_t)J * 4);
  up_flush(c);
  uint32_t* surv = dbuf<uint32_t>(c, "surv", N);
  uint64_t* d_job_s0 = dbuf<uint64_t>(c, "job_s0", J + 1);
  if (N) {
    hipLaunchKernelGGL(k_dedup_flags, dim3(blocks_for(N, 1024)), dim3(1024), 0, st, ord, tu, kw8, d_jobs, d_snaps,
                       job_e0d, J, N, keep, shadowed, tomb, d_active);
    LAUNCH_CHECK();
  }
  launch_scan<uint32_t, uint32_t>(keep, N, nullptr, kpos, scan32, st);
  LAUNCH_CHECK();
  if (N) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(N)), dim3(256), 0, st, ord, keep, kpos, N, surv);
    LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_job_surv, dim3(blocks_for(J + 1)), dim3(256), 0, st, job_e0d, kpos, J, d_job_s0);
  LAUNCH_CHECK();
  PlanIn P;
  P.J = J;
  P.d_jobs = d_jobs;
  P.tu = tu;
  P.kw8 = kw8;
  P.d_surv = surv;
  P.job_s0.assign(J + 1, 0);
  P.d_job_s0 = d_job_s0;
  P.compress = any_compression;
  std::vector<uint64_t> h_shadow(J), h_tomb(J);
  {
    Mail m(c);
    const uint64_t* a = m.add(d_job_s0, J + 1);
    const uint64_t* b = m.add((const uint64_t*)shadowed, J);
    const uint64_t* d = m.add((const uint64_t*)tomb, J);
    m.flush();
    memcpy(P.job_s0.data(), a, (size_t)(J + 1) * 8);
    memcpy(h_shadow.data(), b, (size_t)J * 8);
    memcpy(h_tomb.data(), d, (size_t)J * 8);
  }
  mark(c, "dedup");

  PlanOut O;
  plan_and_write(c, P, O);

  // --- results
  const bool dev_out = dev_inputs;
  // host outputs: each job's tables into a pinned block of its own
  std::vector<HostBlock*> hblk(J, nullptr);
  if (!dev_out) {
    auto drop = [&] {
      (void)hipStreamSynchronize(st);  // copies already queued end first
      for (HostBlock*& h : hblk)
        if (h) pin_put(h), h = nullptr;
    };
    for (uint32_t j = 0; j < J; j++) {
      if (hj[j].failed) continue;
      const uint64_t b0 = O.file_out[O.job_f0[j]], b1 = O.file_out[O.job_f0[j + 1]];
      if (b1 == b0) continue;
      hblk[j] = pin_get(b1 - b0);
      if (!hblk[j]) {
        drop();
        throw Fail{LUDA_NOMEM, "host result allocation failed"};
      }
      const hipError_t e = hipMemcpyAsync(hblk[j]->p, O.d_out + b0, b1 - b0, hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) {
        drop();
        HIPCK(e);
      }
    }
  }
  mark(c, "d2h");
  wait_stream(c);
  const double ms = std::chrono::duration<double, std::milli>(clock::now() - t0).count();
  // device outputs: the output buffer is handed over to the results
  DevBlock* dblk = nullptr;
  if (dev_out && O.total_bytes && !c->arena) {
    DBuf& b = c->bufs["out_tables"];
    dblk = new DevBlock(b.p, b.cap, 0, c->device, c->alloc);
    b = DBuf{};
  }
  for (uint32_t j = 0; j < J; j++) {
    luda_result& r = results[j];
    memset(&r, 0, sizeof r);
    r.entries_in = job_e0[j + 1] - job_e0[j];
    r.bytes_in = hj[j].bytes_in;
    r.ms_total = ms;
    if (hj[j].failed) {
      r.error = decode_err(hj[j].err_key, in_size, hj[j].in_first);
      r.status = r.error.status;
      continue;
    }
    r.entries_out = P.job_s0[j + 1] - P.job_s0[j];
    r.dropped_shadowed = h_shadow[j];
    r.dropped_tombstones = h_tomb[j];
    const uint64_t f0 = O.job_f0[j], f1 = O.job_f0[j + 1];
    r.num_files = (uint32_t)(f1 - f0);
    ResultInternal* ri = new ResultInternal();
    r.internal = ri;
    if (r.num_files) {
      r.files = (luda_file*)calloc(r.num_files, sizeof(luda_file));
      const uint64_t base = O.file_out[f0];
      for (uint64_t f = f0; f < f1; f++) {
        set_file(r.files[f - f0], O, f, base);
      }
      r.data_size = O.file_out[f1] - base;
      for (uint64_t f = f0; f < f1; f++) r.bytes_out += O.file_size[f];
      if (dev_out && c->arena) {  // the caller's buffer: nothing to free
        r.data = O.d_out + base;
      } else if (dev_out) {
        r.data = (uint8_t*)dblk->p + base;
        ri->dev = dblk;
        dblk->refs++;
      } else {
        r.data = (uint8_t*)hblk[j]->p;
        ri->host = hblk[j];
        hblk[j]->refs = 1;
        hblk[j] = nullptr;
      }
    }
  }
  for (HostBlock* h : hblk)  // no result kept it
    if (h) pin_put(h);
  if (dblk && dblk->refs == 0) {  // no result kept it
    c->bufs["out_tables"] = DBuf{dblk->p, dblk->cap};
    delete dblk;
  }
  collect_times(c);
}

}  // namespace

int luda::result_to_host(luda_ctx* c, luda_result* r) { return results_to_host(c, r, 1); }

// One pinned block per result; the copies are queued together and waited
// for once.
int luda::results_to_host(luda_ctx* c, luda_result* res, uint32_t n) {
  std::vector<HostBlock*> hb(n, nullptr);
  int rc = LUDA_OK;
  bool any = false;
  for (uint32_t k = 0; k < n && rc == LUDA_OK; k++) {
    ResultInternal* ri = (ResultInternal*)res[k].internal;
    if (!ri || !ri->dev || !res[k].data_size) continue;
    hb[k] = pin_get(res[k].data_size);
    if (!hb[k])
      rc = LUDA_NOMEM;
    else if (hipMemcpyAsync(hb[k]->p, res[k].data, res[k].data_size, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      rc = LUDA_DEVICE;
    any = true;
  }
  if (any && hipStreamSynchronize(c->stream) != hipSuccess && rc == LUDA_OK) rc = LUDA_DEVICE;
  for (uint32_t k = 0; k < n; k++) {
    if (!hb[k]) continue;
    if (rc != LUDA_OK) {
      pin_put(hb[k]);
      continue;
    }
    ResultInternal* ri = (ResultInternal*)res[k].internal;
    release_dev(c, ri);
    hb[k]->refs = 1;
    ri->host = hb[k];
    res[k].data = (uint8_t*)hb[k]->p;
  }
  return rc;
}

// ---------------------------------------------------------------------------
// C-ABI

extern "C" {

int luda_selftest_crc(void) {
  static CrcTables T;
  static std::once_flag built;
  std::call_once(built, [] { build_crc_tables(&T); });
  uint32_t t0[256];
  byte_table(t0);
  // the byte table against the bitwise definition
  for (uint32_t b = 0; b < 256; b++) {
    uint32_t r = b;
    for (int k = 0; k < 8; k++) r = (r & 1u) ? (r >> 1) ^ POLY : (r >> 1);
    if (t0[b] != r || T.t4[0][b] != r) return 1;
  }
  // slicing-by-4 against bytewise on one dword
  const uint32_t c = 0xDEADBEEFu, d = 0x01020304u;
  uint32_t r = c;
  for (int i = 0; i < 4; i++) r = step_byte(r, (uint8_t)(d >> (8 * i)), t0);
  const uint32_t y = c ^ d;
  if (r != (T.t4[3][y & 0xFF] ^ T.t4[2][(y >> 8) & 0xFF] ^ T.t4[1][(y >> 16) & 0xFF] ^ T.t4[0][y >> 24])) return 2;
  // 11-bit field tables against bytewise on a few words
  for (uint32_t w : {0xDEADBEEFu, 0x01020304u, 0xFFFFFFFFu, 0x80000001u, 0x7FF003FFu}) {
    uint32_t q = 0;
    for (int i = 0; i < 4; i++) q = step_byte(q, (uint8_t)(w >> (8 * i)), t0);
    if (q != (T.u0[w & 0x7FF] ^ T.u1[(w >> 11) & 0x7FF] ^ T.u2[w >> 22])) return 6;
  }
  // shift tables and GF(2) multipliers against zero-byte processing
  uint32_t x = 0x12345678u;
  for (int k = 0; k < NSH; k++) {
    const uint64_t m = 16ull << k;
    const uint32_t z = shift_zeros(x, m, t0);
    if (apply_shift(T.sh[k], x) != z) return 3;
    if (h_mulmod(x, h_xpow8n(m)) != z) return 4;
    x = x * 2654435761u + 12345u;
  }
  for (uint64_t m = 1; m < 300; m += 37)
    if (h_mulmod(x, h_xpow8n(m)) != shift_zeros(x, m, t0)) return 5;
  return 0;
}

// Static scratch memory of luda_compact_dev_noalloc: one copy per GPU, held
// until the process ends.  Host code never uses the array's name as an
// address: the device address of each GPU's copy is looked up once, with that
// device current, and kept here.
static __device__ __align__(256) uint8_t scratch[LUDA_SCRATCH_BYTES];
static std::mutex scratch_mu;
static std::map<int, uint8_t*> scratch_ptr;  // device -> address of its copy of scratch

static void scratch_setup(int device) {
  std::lock_guard<std::mutex> g(scratch_mu);
  if (scratch_ptr.count(device)) return;
  void* p = nullptr;
  HIPCK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Fail{LUDA_DEVICE, "no device address for the static scratch array"};
  scratch_ptr[device] = (uint8_t*)p;
}

static uint8_t* scratch_of(int device) {
  std::lock_guard<std::mutex> g(scratch_mu);
  auto it = scratch_ptr.find(device);
  return it == scratch_ptr.end() ? nullptr : it->second;
}

int luda_ctx_create(int device, luda_ctx** out) {
  if (!out) return LUDA_INVALID_ARG;
  *out = nullptr;
  luda_ctx* c = new (std::nothrow) luda_ctx();
  if (!c) return LUDA_NOMEM;
  const int st = guarded(nullptr, [&] {
    c->device = device;
    HIPCK(hipSetDevice(device));
    HIPCK(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
    c->stream = c->own;
    hipDeviceProp_t prop;
    HIPCK(hipGetDeviceProperties(&prop, device));
    c->n_cu = prop.multiProcessorCount;
    c->lds_limit = prop.sharedMemPerBlock;
    // kernels whose dynamic LDS is sized at run time may use all of it
    const void* dyn[] = {(const void*)k_filter, (const void*)k_seg_compose};
    for (const void* f : dyn)
      HIPCK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_limit - 2048));
    static CrcTables T;  // built once, also when contexts are created on several threads
    static std::once_flag built;
    std::call_once(built, [] { build_crc_tables(&T); });
    HIPCK(hipMalloc((void**)&c->d_crc, sizeof(CrcTables)));
    HIPCK(hipMemcpy(c->d_crc, &T, sizeof(CrcTables), hipMemcpyHostToDevice));
    c->mail_cap = 8u << 20;
    HIPCK(hipHostMalloc((void**)&c->mail, c->mail_cap + 64, hipHostMallocCoherent));
    *(volatile uint64_t*)(c->mail + c->mail_cap) = 0;
    c->stage_cap = 16u << 20;
    HIPCK(hipHostMalloc((void**)&c->stage, c->stage_cap, hipHostMallocCoherent));
    c->timing = getenv("LUDA_STAGE_TIMES") != nullptr;
    scratch_setup(device);
  });
  if (st != LUDA_OK) {
    if (c->mail) (void)hipHostFree(c->mail);
    if (c->stage) (void)hipHostFree(c->stage);
    if (c->d_crc) (void)hipFree(c->d_crc);
    if (c->own) (void)hipStreamDestroy(c->own);
    delete c;
    return st;
  }
  *out = c;
  return LUDA_OK;
}

void luda_ctx_destroy(luda_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  c->copier.reset();
  for (int s = 0; s < UP_SLOTS; s++) {
    if (c->up_slot[s]) pin_put(c->up_slot[s]);
    if (c->up_ev[s]) (void)hipEventDestroy(c->up_ev[s]);
  }
  for (auto& kv : c->bufs) {
    try {
      if (kv.first == "out_tables")
        release_out(c, kv.second);
      else
        dfree(c, kv.second.p, kv.second.cap);
    } catch (...) {
    }
  }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  for (auto e : c->kevents) (void)hipEventDestroy(e);
  if (c->d_crc) (void)hipFree(c->d_crc);
  if (c->mail) (void)hipHostFree(c->mail);
  if (c->stage) (void)hipHostFree(c->stage);
  if (c->own) (void)hipStreamDestroy(c->own);
  delete c;
}

int luda_set_stream(luda_ctx* c, void* s) {
  if (!c) return LUDA_INVALID_ARG;
  c->stream = s ? (hipStream_t)s : c->own;
  return LUDA_OK;
}

int luda_set_allocator(luda_ctx* c, const luda_allocator* a) {
  if (!c || (a && (!a->alloc != !a->free))) return LUDA_INVALID_ARG;
  // the buffers already held came from the previous allocator: they go back to it
  const int st = guarded(c, [&] {
    HIPCK(hipSetDevice(c->device));
    HIPCK(hipStreamSynchronize(c->stream));
    for (auto& kv : c->bufs) {
      if (kv.first == "out_tables")
        release_out(c, kv.second);
      else
        dfree(c, kv.second.p, kv.second.cap);
      kv.second = DBuf{};
    }
    c->alloc = (a && a->alloc) ? *a : luda_allocator{};
  });
  return st;
}

int luda_set_mem_limit(luda_ctx* c, uint64_t bytes) {
  if (!c) return LUDA_INVALID_ARG;
  c->mem_limit = bytes;
  return LUDA_OK;
}

uint64_t luda_mem_held(luda_ctx* c) { return c ? (uint64_t)held_bytes(c) : 0; }

static int run_guarded(luda_ctx* c, const luda_job* jobs, uint32_t n, bool dev, luda_result* res) {
  const int st = guarded(c, [&] {
    HIPCK(hipSetDevice(c->device));
    run_batch(c, jobs, n, dev, res);
  });
  if (st == LUDA_NOMEM && !c->arena) {
    // buffers sized for a call that did not fit are given back: a later,
    // smaller call starts from nothing rather than from their sizes
    (void)guarded(c, [&] {
      HIPCK(hipStreamSynchronize(c->stream));
      for (auto& kv : c->bufs) {
        if (kv.first == "out_tables")
          release_out(c, kv.second);
        else
          dfree(c, kv.second.p, kv.second.cap);
        kv.second = DBuf{};
      }
    });
  }
  if (st != LUDA_OK)
    for (uint32_t j = 0; j < n; j++) {
      memset(&res[j], 0, sizeof(luda_result));
      res[j].status = st;
      res[j].error.status = st;
    }
  return st;
}

int luda_compact_batch(luda_ctx* c, const luda_job* jobs, uint32_t n_jobs, int device_inputs, luda_result* results) {
  if (!c || (n_jobs && (!jobs || !results))) return LUDA_INVALID_ARG;
  for (uint32_t j = 0; j < n_jobs; j++) {
    if (check_opt(&jobs[j].options) != LUDA_OK || (jobs[j].n_inputs && !jobs[j].inputs)) return LUDA_INVALID_ARG;
    for (uint32_t i = 0; i < jobs[j].n_inputs; i++)
      if (!jobs[j].inputs[i].data && jobs[j].inputs[i].size) return LUDA_INVALID_ARG;
  }
  if (!n_jobs) return LUDA_OK;
  return run_guarded(c, jobs, n_jobs, device_inputs != 0, results);
}

static int compact_one(luda_ctx* c, const luda_buf* inputs, uint32_t n, const luda_options* opt, luda_result* out,
                       bool dev) {
  if (!c || !out || (n && !inputs)) return LUDA_INVALID_ARG;
  memset(out, 0, sizeof *out);
  if (check_opt(opt) != LUDA_OK) {
    out->status = out->error.status = LUDA_INVALID_ARG;
    return LUDA_INVALID_ARG;
  }
  for (uint32_t i = 0; i < n; i++)
    if (!inputs[i].data && inputs[i].size) {
      out->status = out->error.status = LUDA_INVALID_ARG;
      return LUDA_INVALID_ARG;
    }
  luda_job job{inputs, n, *opt};
  int rc = run_guarded(c, &job, 1, dev, out);
  if (rc != LUDA_OK) return rc;
  return out->status;
}

int luda_compact(luda_ctx* c, const luda_buf* inputs, uint32_t n, const luda_options* opt, luda_result* out) {
  return compact_one(c, inputs, n, opt, out, false);
}

int luda_compact_dev_noalloc(luda_ctx* c, const luda_buf* inputs, uint32_t n, const luda_options* opt,
                             uint8_t* out_buf, uint64_t out_cap, luda_result* out) {
  if (!c || !out || (out_cap && !out_buf)) return LUDA_INVALID_ARG;
  uint8_t* base = scratch_of(c->device);
  if (!base) {
    memset(out, 0, sizeof *out);
    c->last_error = "no static scratch memory on this device";
    out->status = out->error.status = LUDA_DEVICE;
    return LUDA_DEVICE;
  }
  // every context on this GPU shares its copy of the array: one call at a time
  static std::mutex dev_mu[64];
  std::lock_guard<std::mutex> g(dev_mu[c->device & 63]);
  luda_ctx::Arena a;
  a.base = base;
  a.cap = LUDA_SCRATCH_BYTES;
  a.out = out_buf;
  a.out_cap = out_cap;
  c->arena = &a;
  const int rc = compact_one(c, inputs, n, opt, out, true);
  c->arena = nullptr;
  c->counters.emplace_back("scratch_bytes_used", (double)a.peak);
  return rc;
}

int luda_compact_dev(luda_ctx* c, const luda_buf* inputs, uint32_t n, const luda_options* opt, luda_result* out) {
  return compact_one(c, inputs, n, opt, out, true);
}

void luda_result_free(luda_ctx* c, luda_result* r) {
  if (!r) return;
  ResultInternal* ri = (ResultInternal*)r->internal;
  release_host(ri);
  release_dev(c, ri);
  delete ri;
  free(r->files);
  memset(r, 0, sizeof *r);
}

int luda_build_tables_dev(luda_ctx* c, uint64_t n, const uint8_t* keys, const uint64_t* koff, const uint64_t* tags,
                          const uint8_t* vals, const uint64_t* voff, const luda_options* opt, luda_result* out) {
  if (!c || !out || (n && (!keys || !koff || !tags || !vals || !voff))) return LUDA_INVALID_ARG;
  memset(out, 0, sizeof *out);
  if (check_opt(opt) != LUDA_OK) {
    out->status = out->error.status = LUDA_INVALID_ARG;
    return LUDA_INVALID_ARG;
  }
  const int st = guarded(c, [&] {
    HIPCK(hipSetDevice(c->device));
    if (n > 0xFFFFFFF0ull) throw Fail{LUDA_UNSUPPORTED, "more than 2^32 entries"};
    hipStream_t st = c->stream;
    begin_call(c);
    const auto t0 = std::chrono::steady_clock::now();
    uint32_t* d_max = dbuf<uint32_t>(c, "w_max", 2);
    fill_u32(c, d_max, 0, 2);
    if (n) {
      hipLaunchKernelGGL(k_ingest_max, dim3(blocks_for(n)), dim3(256), 0, st, koff, n, d_max);
      LAUNCH_CHECK();
    }
    uint32_t maxlen = 0;
    {
      Mail m(c);
      const uint32_t* p = m.add(d_max, 1);
      m.flush();
      maxlen = *p;
    }
    const uint32_t kw8 = std::max<uint32_t>(2, (maxlen + 7) / 8);
    Tuples tu;
    memset(&tu, 0, sizeof tu);
    tu.kp0 = dbuf<uint64_t>(c, "tu_kp0", n);
    tu.kp1 = dbuf<uint64_t>(c, "tu_kp1", n);
    tu.tag = dbuf<uint64_t>(c, "tu_tag", n);
    tu.ulen = dbuf<uint32_t>(c, "tu_ulen", n);
    tu.heap = dbuf<uint64_t>(c, "tu_heap", n * kw8);
    tu.vp = dbuf<uint64_t>(c, "tu_vp", n);
    tu.vlen = dbuf<uint32_t>(c, "tu_vlen", n);
    uint32_t* surv = dbuf<uint32_t>(c, "surv", n);
    if (n) {
      hipLaunchKernelGGL(k_ingest, dim3(blocks_for(n)), dim3(256), 0, st, keys, koff, tags, vals, voff, n, tu, kw8,
                         surv);
      LAUNCH_CHECK();
      hipLaunchKernelGGL(k_check_sorted, dim3(blocks_for(n)), dim3(256), 0, st, tu, kw8, n, d_max + 1);
      LAUNCH_CHECK();
    }
    uint32_t bad = 0;
    {
      Mail m(c);
      const uint32_t* p = m.add(d_max + 1, 1);
      m.flush();
      bad = *p;
    }
    if (bad) throw Fail{LUDA_UNSORTED_INPUT, "entries are not strictly increasing internal keys"};
    JobDesc jd{opt->block_size, opt->restart_interval, opt->bloom_bits_per_key, opt->bottommost ? 1u : 0u,
               opt->target_file_size, 0, 0, 0, 0, opt->compression, 0};
    JobDesc* d_jobs = dbuf<JobDesc>(c, "jobs", 1);
    uint64_t* d_job_s0 = dbuf<uint64_t>(c, "job_s0", 2);
    const uint64_t hs0[2] = {0, n};
    up(c, d_jobs, &jd, sizeof jd);
    up(c, d_job_s0, hs0, sizeof hs0);
    up_flush(c);
    PlanIn P;
    P.J = 1;
    P.d_jobs = d_jobs;
    P.tu = tu;
    P.kw8 = kw8;
    P.d_surv = surv;
    P.job_s0.assign(hs0, hs0 + 2);
    P.d_job_s0 = d_job_s0;
    P.compress = opt->compression != 0;
    PlanOut O;
    plan_and_write(c, P, O);
    sync(c);
    collect_times(c);
    out->status = LUDA_OK;
    out->entries_in = out->entries_out = n;
    out->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    const uint64_t nf = O.job_f0[1] - O.job_f0[0];
    out->num_files = (uint32_t)nf;
    ResultInternal* ri = new ResultInternal();
    out->internal = ri;
    if (nf) {
      DBuf& b = c->bufs["out_tables"];
      ri->dev = new DevBlock(b.p, b.cap, 1, c->device, c->alloc);
      b = DBuf{};
      out->files = (luda_file*)calloc(nf, sizeof(luda_file));
      for (uint64_t f = 0; f < nf; f++) {
        set_file(out->files[f], O, f, 0);
      }
      out->data = (uint8_t*)ri->dev->p;
      out->data_size = O.file_out[nf];
      for (uint64_t f = 0; f < nf; f++) out->bytes_out += O.file_size[f];
    }
  });
  if (st != LUDA_OK) {
    luda_result_free(c, out);
    out->status = out->error.status = st;
  }
  return st;
}

static bool params_ok(const luda_params* p) {
  return p && (p->crc_waves == 4 || p->crc_waves == 8 || p->crc_waves == 16) && p->encode_waves >= 2 &&
         p->encode_waves <= 16 && p->stride_blocks >= 1 && p->stride_blocks <= 64;
}

int luda_set_host_sort(luda_ctx* c, int on) {
  if (!c) return LUDA_INVALID_ARG;
  c->host_sort = on != 0;
  return LUDA_OK;
}

uint64_t luda_pin_reserve(uint64_t bytes) { return pin_reserve(bytes); }

uint64_t luda_pool_trim(int device) { return device < 0 ? 0 : dev_pool_trim(device); }

int luda_get_params(luda_ctx* c, luda_params* p) {
  if (!c || !p) return LUDA_INVALID_ARG;
  *p = c->tp;
  return LUDA_OK;
}

int luda_set_params(luda_ctx* c, const luda_params* p) {
  if (!c || !params_ok(p)) return LUDA_INVALID_ARG;
  c->tp = *p;
  return LUDA_OK;
}

int luda_autotune(luda_ctx* c, const luda_job* jobs, uint32_t n_jobs, int device_inputs, uint32_t rounds,
                  luda_params* best, double* best_ms) {
  if (!c || !jobs || !n_jobs || !best || rounds == 0) return LUDA_INVALID_ARG;
  std::vector<luda_result> res(n_jobs);
  auto run = [&](const luda_params& p, double* ms) -> int {
    c->tp = p;
    double t_min = 1e300;
    for (uint32_t r = 0; r < rounds + 1; r++) {  // the first run warms the buffers
      const auto t0 = std::chrono::steady_clock::now();
      const int rc = luda_compact_batch(c, jobs, n_jobs, device_inputs, res.data());
      const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      int bad = rc;
      for (auto& x : res) {
        if (x.status != LUDA_OK && bad == LUDA_OK) bad = x.status;
        luda_result_free(c, &x);
      }
      if (bad != LUDA_OK) return bad;
      if (r) t_min = std::min(t_min, t);
    }
    *ms = t_min;
    return LUDA_OK;
  };
  luda_params cur = c->tp;
  double cur_ms = 0;
  int rc = run(cur, &cur_ms);
  if (rc != LUDA_OK) return rc;
  // coordinate descent over the three parameters
  const uint32_t crc_c[] = {4, 8, 16}, enc_c[] = {4, 8, 12, 16}, str_c[] = {4, 8, 16, 32};
  for (int dim = 0; dim < 3; dim++) {
    const uint32_t* cand = dim == 0 ? crc_c : dim == 1 ? enc_c : str_c;
    const int nc = dim == 1 ? 4 : (dim == 0 ? 3 : 4);
    for (int k = 0; k < nc; k++) {
      luda_params p = cur;
      (dim == 0 ? p.crc_waves : dim == 1 ? p.encode_waves : p.stride_blocks) = cand[k];
      if (p.crc_waves == cur.crc_waves && p.encode_waves == cur.encode_waves && p.stride_blocks == cur.stride_blocks)
        continue;
      double ms = 0;
      rc = run(p, &ms);
      if (rc != LUDA_OK) {
        c->tp = cur;
        return rc;
      }
      if (ms < cur_ms) {
        cur = p;
        cur_ms = ms;
      }
    }
  }
  c->tp = cur;
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return LUDA_OK;
}

const char* luda_status_str(int s) {
  switch (s) {
    case LUDA_OK: return "OK";
    case LUDA_INVALID_ARG: return "INVALID_ARG";
    case LUDA_CORRUPT_FORMAT: return "CORRUPT_FORMAT";
    case LUDA_CORRUPT_CHECKSUM: return "CORRUPT_CHECKSUM";
    case LUDA_UNSORTED_INPUT: return "UNSORTED_INPUT";
    case LUDA_UNSUPPORTED: return "UNSUPPORTED";
    case LUDA_NOMEM: return "NOMEM";
    case LUDA_DEVICE: return "DEVICE";
    case LUDA_CANCELLED: return "CANCELLED";
    default: return "UNKNOWN";
  }
}

int luda_debug_read(luda_ctx* c, const char* name, void* dst, uint64_t offset, uint64_t bytes) {
  if (!c || !name || (!dst && bytes)) return LUDA_INVALID_ARG;
  auto it = c->bufs.find(name);
  if (it == c->bufs.end() || !it->second.p || offset + bytes > it->second.cap) return LUDA_INVALID_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LUDA_DEVICE;
  if (hipMemcpy(dst, (const uint8_t*)it->second.p + offset, bytes, hipMemcpyDeviceToHost) != hipSuccess)
    return LUDA_DEVICE;
  return LUDA_OK;
}

const char* luda_last_error(luda_ctx* c) { return c ? c->last_error.c_str() : ""; }

int luda_last_counters(luda_ctx* c, const char** names, double* values, int cap) {
  if (!c) return 0;
  int n = (int)c->counters.size();
  for (int i = 0; i < n && i < cap; i++) {
    if (names) names[i] = c->counters[i].first.c_str();
    if (values) values[i] = c->counters[i].second;
  }
  return n;
}

int luda_stage_times(luda_ctx* c, const char** names, double* ms, int cap) {
  if (!c) return 0;
  int n = (int)c->stage_ms.size();
  for (int i = 0; i < n && i < cap; i++) {
    if (names) names[i] = c->stage_ms[i].first.c_str();
    if (ms) ms[i] = c->stage_ms[i].second;
  }
  return n;
}

}  // extern "C"
