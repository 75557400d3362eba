// Many counting jobs on one device: the batched form (a fixed list of
// independent jobs spread over a pool of worker streams) and the served form
// (jobs arriving while others run, admitted by their HBM footprint).
//
// Every job is still one whole pass of the counting path on one stream; what
// these forms add is concurrency between jobs.  One job's pass stops the host
// a few times to plan from device counters (bin sizes, tile plan, table
// size), and a small job does not fill 256 compute units, so running several
// jobs on separate streams, each driven by its own host thread, keeps the
// device busy through those gaps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kmc_internal.h"

namespace {

constexpr uint32_t kBatchWorkers = 4;  // streams of the batch pool
constexpr uint32_t kMaxActive = 16;    // server: jobs running at once, at most
constexpr uint32_t kMaxBypass = 8;     // server: later jobs that may overtake a waiting one

double now_us() {
  using namespace std::chrono;
  return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ------------------------------------------------------------------ batch

struct BatchPool {
  std::vector<kmc_ctx*> workers;
};

void pool_release(void* p) {
  auto* pool = static_cast<BatchPool*>(p);
  for (kmc_ctx* w : pool->workers) kmc_ctx_destroy(w);
  delete pool;
}

// ----------------------------------------------------------------- server

struct SrvJob {
  uint64_t ticket = 0;
  kmc_job job{};
  size_t footprint = 0;
  // larger than the whole budget: runs in a region of the arena (footprint
  // = the region, chosen when it is admitted), bounded by it
  bool oversize = false;
  uint32_t bypassed = 0;
  int state = 0;  // 0 queued, 1 running, 2 done
  kmc_status st = KMC_OK;
  kmc_table* table = nullptr;
  double t_submit = 0, t_start = 0;
  size_t ws_off = 0;
};

}  // namespace

struct kmc_server {
  int device = 0;
  uint64_t budget = 0;
  uint8_t* arena = nullptr;
  std::map<size_t, size_t> free_blocks;  // arena offset -> bytes, coalesced
  std::mutex mu;
  std::condition_variable cv_admit, cv_done;
  std::deque<SrvJob*> queue;
  std::unordered_map<uint64_t, SrvJob*> jobs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  kmc_server_stats stats{};
  std::vector<kmc_ctx*> workers;
  std::vector<std::thread> threads;
};

namespace {

// An oversize job runs in a region of the arena (bin groups and spilled
// records keep it inside): the whole arena less room for the largest other
// job queued or running, when that leaves at least kOversizeShare of it (so
// such jobs run beside it), else the whole arena (they wait).  A smaller
// region costs the job more bin groups, and records spilled to host memory
// once they exceed half of it.
constexpr double kOversizeShare = 0.75;

// First fit in the arena.
bool arena_take(kmc_server* s, size_t bytes, size_t* off) {
  bytes = align256(bytes);
  for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
    if (it->second < bytes) continue;
    const size_t o = it->first, rest = it->second - bytes;
    s->free_blocks.erase(it);
    if (rest) s->free_blocks.emplace(o + bytes, rest);
    *off = o;
    return true;
  }
  return false;
}

void arena_give(kmc_server* s, size_t off, size_t bytes) {
  bytes = align256(bytes);
  auto it = s->free_blocks.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != s->free_blocks.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    s->free_blocks.erase(nx);
  }
  if (it != s->free_blocks.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      s->free_blocks.erase(it);
    }
  }
}

// The next job to start, or nullptr.  Queue order, except that a job whose
// footprint does not fit now may be overtaken by later jobs that do, at most
// kMaxBypass times; after that it holds back the jobs behind it until it fits.
// Called with the lock held.
size_t oversize_region(kmc_server* s) {
  size_t beside = 0;
  for (const SrvJob* q : s->queue)
    if (!q->oversize) beside = std::max(beside, align256(q->footprint));
  for (const auto& kv : s->jobs)
    if (kv.second->state == 1 && !kv.second->oversize)
      beside = std::max(beside, align256(kv.second->footprint));
  const size_t least = (size_t)(kOversizeShare * (double)s->budget);
  if (beside && s->budget - std::min<size_t>(beside, s->budget) >= least)
    return (s->budget - beside) & ~(size_t)255;
  return s->budget;
}

SrvJob* pick(kmc_server* s) {
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
    SrvJob* j = *it;
    if (j->oversize) j->footprint = oversize_region(s);
    const bool ok = arena_take(s, j->footprint, &j->ws_off);
    if (ok) {
      for (auto jt = s->queue.begin(); jt != it; ++jt) (*jt)->bypassed++;
      s->queue.erase(it);
      return j;
    }
    if (j->bypassed >= kMaxBypass) return nullptr;
  }
  return nullptr;
}

void serve(kmc_server* s, kmc_ctx* w) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    SrvJob* j = nullptr;
    s->cv_admit.wait(lk, [&] { return s->stopping || (j = pick(s)) != nullptr; });
    if (!j) return;
    j->state = 1;
    j->t_start = now_us();
    s->stats.active++;
    s->stats.queued = (uint32_t)s->queue.size();
    s->stats.admitted_bytes += align256(j->footprint);
    s->stats.peak_admitted_bytes = std::max(s->stats.peak_admitted_bytes, s->stats.admitted_bytes);
    lk.unlock();
    kmc_table* t = nullptr;
    kmc_status st;
    if (j->oversize && s->arena) {
      // its region of the arena lent to the worker's context, which takes
      // every device buffer of the job from it; the region is the job's
      // budget (bin groups, records spilled to pinned host memory)
      (void)hipSetDevice(s->device);
      kmc::ctx_set_budget(w, j->footprint);
      kmc::ctx_lend_region(w, s->arena + j->ws_off, j->footprint);
      st = kmc_count_ex(w, &j->job.reads, &j->job.params, nullptr, &t);
      kmc::ctx_end_region(w);
      kmc::ctx_set_budget(w, 0);
      kmc::ctx_release_buffers(w);  // the spilled records' host memory
    } else if (!s->arena) {
      st = KMC_ERR_OUT_OF_MEMORY;
    } else {
      st = kmc::count_ws_impl(w, &j->job.reads, &j->job.params, nullptr, s->arena + j->ws_off,
                              j->footprint, true, &t);
    }
    const double t_done = now_us();
    if (t) {
      t->stats.us_queue = j->t_start - j->t_submit;
      t->stats.us_latency = t_done - j->t_submit;
    }
    lk.lock();
    arena_give(s, j->ws_off, j->footprint);
    s->stats.admitted_bytes -= align256(j->footprint);
    s->stats.active--;
    j->st = st;
    j->table = t;
    j->state = 2;
    if (st == KMC_OK) s->stats.completed++;
    else s->stats.failed++;
    s->cv_done.notify_all();
    s->cv_admit.notify_all();
  }
}

}  // namespace

extern "C" {

kmc_status kmc_batch_count(kmc_ctx* ctx, const kmc_job* jobs, uint32_t n_jobs, kmc_table** outs) {
  if (!ctx) return KMC_ERR_INVALID_ARG;
  if (n_jobs == 0) return KMC_OK;
  if (!jobs || !outs) return KMC_ERR_INVALID_ARG;
  std::fill(outs, outs + n_jobs, nullptr);
  kmc::ctx_set_error(ctx, "");
  // a malformed job fails the batch before any device work
  for (uint32_t i = 0; i < n_jobs; ++i) {
    size_t b = 0;
    kmc_status v = kmc_workspace_size(&jobs[i].reads, &jobs[i].params, &b);
    if (v != KMC_OK) {
      kmc::ctx_set_error(ctx, ("job " + std::to_string(i) + ": invalid arguments").c_str());
      return v;
    }
  }
  // largest jobs first, so that the streams run out of work together
  std::vector<uint32_t> order(n_jobs);
  for (uint32_t i = 0; i < n_jobs; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
    return jobs[a].reads.n_bases > jobs[b].reads.n_bases;
  });
  void** slot = kmc::ctx_ext(ctx, pool_release);
  auto* pool = static_cast<BatchPool*>(*slot);
  if (!pool) {
    pool = new (std::nothrow) BatchPool;
    if (!pool) return KMC_ERR_OUT_OF_MEMORY;
    *slot = pool;
  }
  const uint32_t want = kmc::ctx_batch_workers(ctx) ? kmc::ctx_batch_workers(ctx) : kBatchWorkers;
  const uint32_t n_workers = std::min(n_jobs, std::min(want, kMaxActive));
  while (pool->workers.size() < n_workers) {
    kmc_ctx* w = nullptr;
    kmc_status st = kmc_ctx_create(kmc::ctx_device(ctx), &w);
    if (st != KMC_OK) {
      kmc::ctx_set_error(ctx, "could not create a worker stream");
      return st;
    }
    pool->workers.push_back(w);
  }
  // the workers count with the caller's knobs (override or tuned)
  for (uint32_t t = 0; t < n_workers; ++t) kmc::ctx_copy_tuning(pool->workers[t], ctx);
  std::atomic<uint32_t> next{0};
  std::atomic<bool> failed{false};
  std::vector<kmc_status> status(n_jobs, KMC_OK);
  std::vector<std::string> why(n_jobs);
  auto work = [&](kmc_ctx* w) {
    for (;;) {
      if (failed.load()) return;
      const uint32_t i = next.fetch_add(1);
      if (i >= n_jobs) return;
      const uint32_t j = order[i];
      kmc_status st = kmc_count_ex(w, &jobs[j].reads, &jobs[j].params, nullptr, &outs[j]);
      if (st != KMC_OK) {
        status[j] = st;
        why[j] = kmc_last_error(w);
        failed = true;
      }
    }
  };
  std::vector<std::thread> threads;
  for (uint32_t t = 1; t < n_workers; ++t) {
    try {
      threads.emplace_back(work, pool->workers[t]);
    } catch (...) {
      break;  // fewer streams; the jobs still all run
    }
  }
  work(pool->workers[0]);
  for (auto& th : threads) th.join();
  if (!failed.load()) return KMC_OK;
  kmc_status first = KMC_OK;
  for (uint32_t j = 0; j < n_jobs; ++j) {
    if (status[j] != KMC_OK && first == KMC_OK) {
      first = status[j];
      kmc::ctx_set_error(ctx, ("job " + std::to_string(j) + ": " + why[j]).c_str());
    }
    kmc_table_free(outs[j]);
    outs[j] = nullptr;
  }
  return first;
}

// Candidate knobs of kmc_autotune: tile packing, first-digit bits, records
// per expansion task.
static const kmc_knobs kCandidates[] = {
    {3, 0, 0},  {2, 0, 0},  {3, -1, 0}, {3, 1, 0},  {3, 0, 512}, {3, 0, 1024},
    {2, 1, 0},  {2, 0, 512}, {3, 1, 512}, {2, -1, 0}, {3, -1, 512}, {2, 1, 512}};
static const uint32_t kWorkerCandidates[] = {2, 4, 8};

kmc_status kmc_autotune(kmc_ctx* ctx, const kmc_job* jobs, uint32_t n_jobs,
                        kmc_tune_report* report) {
  if (!ctx || (n_jobs && !jobs)) return KMC_ERR_INVALID_ARG;
  if (report) *report = kmc_tune_report{};
  // one sample per class: the largest job of each (key width, log2 bases)
  std::map<uint32_t, uint32_t> sample;
  for (uint32_t i = 0; i < n_jobs; ++i) {
    const uint32_t kw = jobs[i].params.k <= 32 ? 1 : 2;
    uint32_t l = 0;
    while (l < 63 && (2ull << l) <= jobs[i].reads.n_bases) ++l;
    const uint32_t cls = (kw - 1) * 64 + l;
    auto it = sample.find(cls);
    if (it == sample.end() || jobs[i].reads.n_bases > jobs[it->second].reads.n_bases)
      sample[cls] = i;
  }
  (void)kmc::ctx_override_knobs(ctx, nullptr);  // tuning replaces any override
  uint32_t n_cls = 0;
  for (const auto& kv : sample) {
    const kmc_job& J = jobs[kv.second];
    kmc_params P = J.params;
    P.flags |= KMC_FLAG_DEVICE_TABLE;
    double best_us = 1e300;
    kmc_knobs best = kCandidates[0];
    for (const kmc_knobs& cand : kCandidates) {
      kmc::ctx_override_knobs(ctx, &cand);
      double us = 0;
      for (int rep = 0; rep < 2; ++rep) {  // the first run sizes the cached buffers
        kmc_table* t = nullptr;
        const kmc_status st = kmc_count_ex(ctx, &J.reads, &P, nullptr, &t);
        if (st != KMC_OK) {
          kmc::ctx_override_knobs(ctx, nullptr);
          return st;
        }
        us = t->stats.us_total;
        kmc_table_free(t);
      }
      if (us < best_us) {
        best_us = us;
        best = cand;
      }
    }
    kmc::ctx_override_knobs(ctx, nullptr);
    kmc::ctx_set_tuned(ctx, J.params.k <= 32 ? 1 : 2, J.reads.n_bases, best);
    if (report && n_cls < KMC_TUNE_MAX_CLASSES) {
      kmc_tune_class& c = report->classes[n_cls];
      c.key_words = J.params.k <= 32 ? 1 : 2;
      c.sample_bases = J.reads.n_bases;
      c.knobs = best;
      c.us = best_us;
    }
    ++n_cls;
  }
  if (report) report->n_classes = std::min<uint32_t>(n_cls, KMC_TUNE_MAX_CLASSES);
  // batch streams: up to 64 of the jobs (every n_jobs/64-th, so the mix of
  // sizes is the batch's) as one batch with 2, 4 and 8 workers
  if (n_jobs > 1) {
    std::vector<kmc_job> sj;
    const uint32_t step = n_jobs > 64 ? n_jobs / 64 : 1;
    for (uint32_t i = 0; i < n_jobs && sj.size() < 64; i += step) {
      kmc_job j = jobs[i];
      j.params.flags |= KMC_FLAG_DEVICE_TABLE;
      sj.push_back(j);
    }
    std::vector<kmc_table*> outs(sj.size(), nullptr);
    double best_s = 1e300;
    uint32_t best_w = kBatchWorkers;
    for (uint32_t w : kWorkerCandidates) {
      kmc::ctx_set_batch_workers(ctx, w);
      double dt = 1e300;
      for (int rep = 0; rep < 3; ++rep) {  // the first run sizes the workers' buffers
        const double t0 = now_us();
        const kmc_status st = kmc_batch_count(ctx, sj.data(), (uint32_t)sj.size(), outs.data());
        if (rep > 0) dt = std::min(dt, now_us() - t0);
        for (auto*& t : outs) {
          kmc_table_free(t);
          t = nullptr;
        }
        if (st != KMC_OK) return st;
      }
      if (dt < best_s) {
        best_s = dt;
        best_w = w;
      }
    }
    kmc::ctx_set_batch_workers(ctx, best_w);
    if (report) report->batch_workers = best_w;
  }
  return KMC_OK;
}

kmc_status kmc_server_start(kmc_ctx* ctx, const kmc_server_cfg* cfg, kmc_server** out) {
  if (!out) return KMC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!ctx) return KMC_ERR_INVALID_ARG;
  const uint32_t max_active = (cfg && cfg->max_active) ? cfg->max_active : 4;
  if (max_active > kMaxActive) return KMC_ERR_INVALID_ARG;
  const int dev = kmc::ctx_device(ctx);
  if (hipSetDevice(dev) != hipSuccess) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  uint64_t budget = cfg ? cfg->hbm_budget : 0;
  if (!budget) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      (void)hipGetLastError();
      return KMC_ERR_DEVICE;
    }
    budget = (uint64_t)(0.9 * (double)free_b);
  }
  budget &= ~(uint64_t)255;
  if (budget < 256) return KMC_ERR_INVALID_ARG;
  auto* s = new (std::nothrow) kmc_server;
  if (!s) return KMC_ERR_OUT_OF_MEMORY;
  s->device = dev;
  s->budget = budget;
  s->stats.budget = budget;
  if (hipMalloc(&s->arena, budget) != hipSuccess) {
    (void)hipGetLastError();
    delete s;
    kmc::ctx_set_error(ctx, "could not reserve the server's HBM budget");
    return KMC_ERR_OUT_OF_MEMORY;
  }
  s->free_blocks.emplace(0, budget);
  for (uint32_t i = 0; i < max_active; ++i) {
    kmc_ctx* w = nullptr;
    if (kmc_ctx_create(dev, &w) != KMC_OK) break;
    s->workers.push_back(w);
  }
  try {
    for (kmc_ctx* w : s->workers) s->threads.emplace_back(serve, s, w);
  } catch (...) {
  }
  if (s->threads.empty()) {
    kmc_server_stop(s);
    return KMC_ERR_DEVICE;
  }
  *out = s;
  return KMC_OK;
}

kmc_status kmc_server_submit(kmc_server* s, const kmc_job* job, uint64_t* ticket) {
  if (!s || !job || !ticket) return KMC_ERR_INVALID_ARG;
  *ticket = 0;
  size_t fp = 0;
  kmc_status v = kmc_workspace_size(&job->reads, &job->params, &fp);
  if (v != KMC_OK) return v;
  auto* j = new (std::nothrow) SrvJob;
  if (!j) return KMC_ERR_OUT_OF_MEMORY;
  j->job = *job;
  j->footprint = fp;
  j->oversize = align256(fp) > s->budget;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) {
      delete j;
      return KMC_ERR_BUSY;
    }
    j->t_submit = now_us();
    j->ticket = s->next_ticket++;
    s->jobs.emplace(j->ticket, j);
    s->queue.push_back(j);
    s->stats.submitted++;
    s->stats.queued = (uint32_t)s->queue.size();
    *ticket = j->ticket;
  }
  s->cv_admit.notify_all();
  return KMC_OK;
}

kmc_status kmc_server_poll(kmc_server* s, uint64_t ticket, int32_t wait, kmc_table** out) {
  if (!out) return KMC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!s) return KMC_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return KMC_ERR_INVALID_ARG;
  SrvJob* j = it->second;
  if (j->state != 2) {
    if (!wait) return KMC_ERR_BUSY;
    s->cv_done.wait(lk, [&] { return j->state == 2; });
  }
  const kmc_status st = j->st;
  *out = j->table;
  s->jobs.erase(ticket);
  delete j;
  return st;
}

kmc_status kmc_server_stats_get(kmc_server* s, kmc_server_stats* stats) {
  if (!s || !stats) return KMC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *stats = s->stats;
  stats->queued = (uint32_t)s->queue.size();
  return KMC_OK;
}

void kmc_server_stop(kmc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    s->queue.clear();  // queued jobs never start
  }
  s->cv_admit.notify_all();
  for (auto& th : s->threads) th.join();
  for (auto& kv : s->jobs) {
    kmc_table_free(kv.second->table);
    delete kv.second;
  }
  for (kmc_ctx* w : s->workers) kmc_ctx_destroy(w);
  if (s->arena) {
    (void)hipSetDevice(s->device);
    (void)hipFree(s->arena);
  }
  delete s;
}

}  // extern "C"
