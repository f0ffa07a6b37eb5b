// Served form of the compaction library (include/luda.h, luda_server_*):
// jobs arrive one by one, are admitted under a device-memory budget, and
// workers run the admitted jobs that are waiting together as one batched
// pass.  Each worker owns a context, so its passes run on their own HIP
// stream; with several workers, passes overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "luda.h"
#include "luda_host_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct ServedJob {
  std::vector<luda_buf> inputs;
  std::vector<uint64_t> snapshots;  // the job's copy of its snapshot list
  luda_options opt{};
  uint64_t est = 0;  // admitted bytes
  Clock::time_point t_submit, t_done;
  luda_result res{};
  bool done = false;
};

// Expected device bytes of a job: its output tables (at most about its input
// bytes: the survivors' entries re-encoded, plus index and filter blocks of a
// similar share) and the pass's working set (entry records, merge order,
// plan and filter arrays: about 220 bytes per entry plus key slots, i.e. at
// most twice the input bytes for entries of 110 bytes or more on average).
uint64_t footprint(uint64_t input_bytes) { return 3 * input_bytes + (uint64_t(1) << 20); }

}  // namespace

struct luda_server {
  luda_server_cfg cfg{};
  int device = 0;
  std::vector<luda_ctx*> ctxs;
  std::vector<std::thread> threads;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_turn;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, std::unique_ptr<ServedJob>> jobs;
  uint64_t next_ticket = 1;
  uint64_t admitted = 0, peak = 0;
  uint64_t n_done = 0, n_batches = 0, max_batch = 0;
  uint64_t take_seq = 0, copy_turn = 0;  // host outputs: batches copy out in the order taken
  bool stop = false;
  std::unique_ptr<std::atomic<uint64_t>[]> held;  // device bytes each worker's context holds
};

namespace {

// the job at the head of the queue fits beside the admitted jobs (every job
// fits the budget alone: larger ones are refused at submission)
bool can_take(const luda_server* s) {
  if (s->pending.empty()) return false;
  const ServedJob* j = s->jobs.at(s->pending.front()).get();
  return s->admitted + j->est <= s->cfg.hbm_budget;
}

// run the jobs as one batched pass; if the pass fails as a whole (a limit of
// the batch, not of a job), each job runs again alone, so that a job's
// outcome never depends on what it was batched with
void run_jobs(luda_ctx* ctx, const std::vector<ServedJob*>& batch, std::vector<luda_result>& res) {
  std::vector<luda_job> cj(batch.size());
  for (size_t k = 0; k < batch.size(); k++) {
    cj[k].inputs = batch[k]->inputs.data();
    cj[k].n_inputs = (uint32_t)batch[k]->inputs.size();
    cj[k].options = batch[k]->opt;
  }
  const int rc = luda_compact_batch(ctx, cj.data(), (uint32_t)cj.size(), 1, res.data());
  if (rc == LUDA_OK || batch.size() == 1) return;
  for (size_t k = 0; k < batch.size(); k++) {
    luda_result_free(ctx, &res[k]);
    luda_compact_batch(ctx, &cj[k], 1, 1, &res[k]);
  }
}

void worker(luda_server* s, luda_ctx* ctx) {
  (void)hipSetDevice(s->device);
  for (;;) {
    std::vector<ServedJob*> batch;
    uint64_t est = 0, seq = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // a stopping server still runs the jobs already submitted, as the
      // budget frees up (it sleeps meanwhile)
      s->cv_work.wait(lk, [&] { return (s->stop && s->pending.empty()) || can_take(s); });
      if (s->stop && s->pending.empty()) return;
      while (!s->pending.empty() && (s->cfg.max_batch_jobs == 0 || batch.size() < s->cfg.max_batch_jobs)) {
        ServedJob* j = s->jobs.at(s->pending.front()).get();
        if (s->admitted + j->est > s->cfg.hbm_budget) break;
        s->admitted += j->est;
        est += j->est;
        batch.push_back(j);
        s->pending.pop_front();
      }
      s->peak = std::max(s->peak, s->admitted);
      if (!batch.empty()) {
        seq = s->take_seq++;
        s->n_batches++;
        s->max_batch = std::max<uint64_t>(s->max_batch, batch.size());
      }
    }
    if (batch.empty()) continue;
    std::vector<luda_result> res(batch.size());
    run_jobs(ctx, batch, res);
    s->held[std::find(s->ctxs.begin(), s->ctxs.end(), ctx) - s->ctxs.begin()] = luda_mem_held(ctx);
    // Each job completes when its own outputs are where the caller reads
    // them: with host outputs, the jobs of a batch complete one by one as
    // their copies end, not all at the end of the last copy.  The copies of
    // one batch at a time use the host link, batches in the order they were
    // taken (first come, first served), while other workers' passes compute.
    if (s->cfg.host_outputs) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_turn.wait(lk, [&] { return s->copy_turn == seq; });
    }
    for (size_t k = 0; k < batch.size(); k++) {
      if (s->cfg.host_outputs) {
        const int rc = luda::result_to_host(ctx, &res[k]);
        if (rc != LUDA_OK) {  // its outputs did not reach host memory: the job fails with that status
          const luda_result keep = res[k];
          luda_result_free(ctx, &res[k]);
          res[k].entries_in = keep.entries_in;
          res[k].bytes_in = keep.bytes_in;
          res[k].ms_total = keep.ms_total;
          res[k].status = res[k].error.status = rc;
        }
      }
      const Clock::time_point now = Clock::now();
      {
        std::lock_guard<std::mutex> lk(s->mu);
        batch[k]->res = res[k];
        batch[k]->done = true;
        batch[k]->t_done = now;
        s->n_done++;
      }
      if (s->cfg.host_outputs) s->cv_done.notify_all();
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->cfg.host_outputs) s->copy_turn++;
      s->admitted -= est;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
    s->cv_turn.notify_all();
  }
}

}  // namespace

extern "C" {

int luda_server_create(int device, const luda_server_cfg* cfg, luda_server** out) {
  if (!cfg || !out || cfg->hbm_budget == 0 || cfg->workers == 0 || cfg->workers > 8) return LUDA_INVALID_ARG;
  *out = nullptr;
  luda_server* s = new luda_server();
  s->cfg = *cfg;
  s->device = device;
  s->held.reset(new std::atomic<uint64_t>[cfg->workers]);
  for (uint32_t w = 0; w < cfg->workers; w++) {
    s->held[w] = 0;
    luda_ctx* c = nullptr;
    const int rc = luda_ctx_create(device, &c);
    if (rc != LUDA_OK) {
      for (luda_ctx* x : s->ctxs) luda_ctx_destroy(x);
      delete s;
      return rc;
    }
    luda_set_mem_limit(c, cfg->hbm_budget);  // no pass holds more than the budget
    s->ctxs.push_back(c);
  }
  if (cfg->host_outputs) {
    (void)hipSetDevice(device);
    luda_pin_reserve(cfg->hbm_budget / 2);  // admitted jobs' outputs fit in it
  }
  for (luda_ctx* c : s->ctxs) s->threads.emplace_back(worker, s, c);
  *out = s;
  return LUDA_OK;
}

int luda_server_submit(luda_server* s, const luda_job* job, uint64_t* ticket) {
  if (!s || !job || !ticket || (job->n_inputs && !job->inputs)) return LUDA_INVALID_ARG;
  auto j = std::make_unique<ServedJob>();
  uint64_t bytes = 0;
  for (uint32_t i = 0; i < job->n_inputs; i++) {
    j->inputs.push_back(job->inputs[i]);
    bytes += job->inputs[i].size;
  }
  j->opt = job->options;
  if (j->opt.n_snapshots) {
    if (!j->opt.snapshots || j->opt.n_snapshots > LUDA_MAX_SNAPSHOTS) return LUDA_INVALID_ARG;
    j->snapshots.assign(j->opt.snapshots, j->opt.snapshots + j->opt.n_snapshots);
    j->opt.snapshots = j->snapshots.data();
  }
  j->est = footprint(bytes);
  if (j->est > s->cfg.hbm_budget) return LUDA_NOMEM;  // it could never be admitted
  j->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return LUDA_INVALID_ARG;
    *ticket = s->next_ticket++;
    s->pending.push_back(*ticket);
    s->jobs.emplace(*ticket, std::move(j));
  }
  s->cv_work.notify_one();
  return LUDA_OK;
}

int luda_server_poll(luda_server* s, uint64_t ticket, int wait, luda_result* out, double* latency_ms) {
  if (!s || !out) return LUDA_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return LUDA_INVALID_ARG;
  ServedJob* j = it->second.get();
  if (wait) s->cv_done.wait(lk, [&] { return j->done; });
  if (!j->done) return 1;
  *out = j->res;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(j->t_done - j->t_submit).count();
  s->jobs.erase(it);
  return LUDA_OK;
}

int luda_server_cancel(luda_server* s, uint64_t ticket) {
  if (!s) return LUDA_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return LUDA_INVALID_ARG;
    auto q = std::find(s->pending.begin(), s->pending.end(), ticket);
    if (q == s->pending.end()) return 1;  // taken by a worker, or done
    s->pending.erase(q);
    ServedJob* j = it->second.get();
    memset(&j->res, 0, sizeof j->res);
    j->res.status = j->res.error.status = LUDA_CANCELLED;
    for (const luda_buf& b : j->inputs) j->res.bytes_in += b.size;
    j->done = true;
    j->t_done = Clock::now();
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();  // the next job in the queue may fit now
  return LUDA_OK;
}

int luda_server_memory(luda_server* s, uint64_t* held_by_workers, uint64_t* device_used) {
  if (!s) return 0;
  uint64_t h = 0;
  for (size_t w = 0; w < s->ctxs.size(); w++) h += s->held[w].load();
  if (held_by_workers) *held_by_workers = h;
  if (device_used) {
    size_t fr = 0, tot = 0;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->device);
    *device_used = hipMemGetInfo(&fr, &tot) == hipSuccess ? (uint64_t)(tot - fr) : 0;
    (void)hipSetDevice(cur);
  }
  return 2;
}

int luda_server_stats(luda_server* s, uint64_t* jobs, uint64_t* batches, uint64_t* max_batch,
                      uint64_t* peak_admitted) {
  if (!s) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  if (jobs) *jobs = s->n_done;
  if (batches) *batches = s->n_batches;
  if (max_batch) *max_batch = s->max_batch;
  if (peak_admitted) *peak_admitted = s->peak;
  return 4;
}

void luda_server_destroy(luda_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->threads) t.join();
  for (auto& kv : s->jobs)
    if (kv.second->done) luda_result_free(nullptr, &kv.second->res);
  for (luda_ctx* c : s->ctxs) luda_ctx_destroy(c);
  delete s;
}

}  // extern "C"
