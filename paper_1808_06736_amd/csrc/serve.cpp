// Request loop for many independent NUFFTs on one GPU (continuous batching).
//
// Worker threads, each with its own HIP stream, take requests from one FIFO
// queue.  A request is admitted when a worker is free and its device memory
// fits the HBM budget (idle cached plans are evicted, least recently used
// first, to make room), so requests arriving while others run start as soon as
// a worker and memory free up, and their kernels overlap on the device.  While
// the head of the queue waits for memory, a later request that fits may start
// first (a bounded number of times).  A request's work waits for an event
// recorded at submit on the stream that wrote its inputs.  Plans
// are cached by problem shape (type, dim, modes, sign, tolerance, precision);
// a cached plan remembers the point set it last sorted, so a request that
// names the same points id skips setpts; a plan cached without a points id
// keeps only its parameters, tables and FFT plans (its grid, FFT work and
// point buffers are made again at its next request).  Latency is measured from submit to
// the end of the request's work on its stream.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "esn_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

// A request waiting for memory at the head of the queue lets requests among
// the next kBypassWindow start if they fit, at most kMaxBypass times.
constexpr size_t kBypassWindow = 8;
constexpr int kMaxBypass = 16;

struct Req {
  esn_request r;
  int bypassed = 0;            // times a later request started first
  hipEvent_t ready = nullptr;  // recorded at submit on the stream that wrote the inputs
  long long ticket = 0;
  Clock::time_point t_submit, t_done;
  int status = ESN_OK;
  bool done = false;
  int64_t est = 0;
  std::string key;
};

struct CachedPlan {
  esn_plan plan = nullptr;
  std::string key;
  long long points_id = 0;     // point set last sorted (0: unknown)
  int64_t bytes = 0;           // device bytes counted against the budget
  bool busy = false;
  uint64_t last_use = 0;
};

std::string plan_key(const esn_request& r) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%d/%d/%lld/%lld/%lld/%d/%.17g/%d", r.type, r.dim,
                (long long)r.nmodes[0], (long long)(r.dim > 1 ? r.nmodes[1] : 1),
                (long long)(r.dim > 2 ? r.nmodes[2] : 1), r.isign, r.eps, r.prec);
  return buf;
}

}  // namespace

struct esn_server_s {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Req>> queue;
  std::unordered_map<long long, std::shared_ptr<Req>> tickets;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::vector<std::unique_ptr<CachedPlan>> cache;
  esn_opts opts;
  int device = 0;
  int64_t budget = 0, in_use = 0, peak = 0;
  int running = 0;
  bool stop = false;
  long long next_ticket = 1;
  uint64_t use_clock = 0;
  // statistics
  std::vector<double> lat_ms;
  long long submitted = 0, completed = 0, failed = 0, rejected = 0;
  long long plan_hits = 0, plan_misses = 0, point_hits = 0;
  double pts_done = 0;
  Clock::time_point t_first, t_last;
  bool have_first = false;
};

namespace {

// Free idle cached plans (LRU first) until `need` more bytes fit.  Lock held.
void evict_for(esn_server_s* sv, int64_t need, const std::string& keep_key) {
  while (sv->in_use + need > sv->budget) {
    int victim = -1;
    for (int i = 0; i < (int)sv->cache.size(); i++) {
      CachedPlan* c = sv->cache[i].get();
      if (c->busy || c->key == keep_key) continue;
      if (victim < 0 || c->last_use < sv->cache[victim]->last_use) victim = i;
    }
    if (victim < 0) return;
    CachedPlan* c = sv->cache[victim].get();
    esn_destroy(c->plan);
    sv->in_use -= c->bytes;
    sv->cache.erase(sv->cache.begin() + victim);
  }
}

// Idle cached plan for this key, preferring one that holds these points.  Lock held.
CachedPlan* find_plan(esn_server_s* sv, const std::string& key, long long points_id) {
  CachedPlan* any = nullptr;
  for (auto& c : sv->cache) {
    if (c->busy || c->key != key) continue;
    if (points_id > 0 && c->points_id == points_id) return c.get();
    if (!any) any = c.get();
  }
  return any;
}

void finish(esn_server_s* sv, const std::shared_ptr<Req>& q, int status) {
  if (q->ready) {
    (void)hipEventDestroy(q->ready);
    q->ready = nullptr;
  }
  q->status = status;
  q->t_done = Clock::now();
  q->done = true;
  if (status >= 2) {
    sv->failed++;
    if (status == ESN_ERR_BUDGET) sv->rejected++;
  } else {
    sv->completed++;
    sv->lat_ms.push_back(std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count());
    sv->pts_done += (double)q->r.M;
    sv->t_last = q->t_done;
  }
}

void worker_loop(esn_server_s* sv, int slot) {
  (void)hipSetDevice(sv->device);
  hipStream_t stream = sv->streams[slot];
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // wait for an admissible request: the head of the queue, or, while the
    // head waits for memory, one of the next kBypassWindow requests (the head
    // may be passed kMaxBypass times before everything waits for it)
    std::shared_ptr<Req> q;
    CachedPlan* cp = nullptr;
    int64_t reserved = 0;
    for (;;) {
      if (sv->queue.empty()) {
        if (sv->stop) return;
        sv->cv_work.wait(lk);
        continue;
      }
      std::shared_ptr<Req> head = sv->queue.front();
      if (head->est > sv->budget) {                 // can never fit
        sv->queue.pop_front();
        finish(sv, head, ESN_ERR_BUDGET);
        sv->cv_done.notify_all();
        continue;
      }
      const size_t window =
          head->bypassed < kMaxBypass ? std::min(sv->queue.size(), kBypassWindow) : 1;
      for (size_t i = 0; i < window && !q; i++) {
        std::shared_ptr<Req> cand = sv->queue[i];
        if (cand->est > sv->budget) continue;       // failed when it reaches the head
        CachedPlan* c = find_plan(sv, cand->key, cand->r.points_id);
        // a cached plan's memory is already counted; it may grow with M
        const int64_t need = c ? std::max<int64_t>(0, cand->est - c->bytes) : cand->est;
        evict_for(sv, need, cand->key);
        if (sv->in_use + need <= sv->budget || (c && sv->running == 0)) {
          sv->queue.erase(sv->queue.begin() + (std::ptrdiff_t)i);
          if (i > 0) head->bypassed++;
          if (c) {
            c->busy = true;
            c->last_use = ++sv->use_clock;
            cp = c;
          }
          reserved = need;
          sv->in_use += need;
          q = cand;
        }
      }
      if (q) break;
      if (sv->running == 0) {                       // nothing will free memory
        sv->queue.pop_front();
        finish(sv, head, ESN_ERR_BUDGET);
        sv->cv_done.notify_all();
        continue;
      }
      sv->cv_work.wait(lk);                         // wait for memory to free up
    }
    sv->peak = std::max(sv->peak, sv->in_use);
    sv->running++;
    const bool hit = cp != nullptr;
    if (hit) sv->plan_hits++;
    else sv->plan_misses++;
    const bool same_points = hit && q->r.points_id > 0 && cp->points_id == q->r.points_id;
    if (same_points) sv->point_hits++;
    lk.unlock();

    // ---- run the request on this worker's stream ----
    int st = ESN_OK;
    esn_plan plan = hit ? cp->plan : nullptr;
    if (!plan) {
      st = esn_makeplan(q->r.type, q->r.dim, q->r.nmodes, q->r.isign, 1, q->r.eps, q->r.prec,
                        &plan, &sv->opts, (void*)stream);
    } else {
      st = esn::plan_set_stream(plan, stream);
    }
    int warn = st == ESN_WARN_EPS_TOO_SMALL ? st : ESN_OK;
    // inputs written on the caller's stream are complete before they are read
    if (st < 2 && q->ready && hipStreamWaitEvent(stream, q->ready, 0) != hipSuccess)
      st = ESN_ERR_HIP;
    if (st < 2 && !same_points)
      st = esn_setpts(plan, q->r.M, q->r.coord_prec, q->r.x, q->r.y, q->r.z);
    if (st < 2) st = esn_execute(plan, q->r.c, q->r.f);
    if (hipStreamSynchronize(stream) != hipSuccess && st < 2) st = ESN_ERR_HIP;
    if (st < 2 && warn) st = warn;
    // a plan kept for later requests gives back its working memory (grid, FFT
    // work, sorted points) unless its sorted points may be asked for again,
    // so that the cache holds many more plans within the budget; the buffers
    // come back (stream-ordered, no device-wide wait) at its next request
    if (plan && st < 2 && q->r.points_id == 0) (void)esn::plan_trim(plan);
    esn_info info{};
    if (plan) esn_get_info(plan, &info);

    lk.lock();
    sv->running--;
    sv->in_use -= reserved;
    if (plan) {
      if (!cp) {
        auto c = std::make_unique<CachedPlan>();
        c->plan = plan;
        c->key = q->key;
        cp = c.get();
        sv->cache.push_back(std::move(c));
      } else {
        sv->in_use -= cp->bytes;
      }
      cp->bytes = info.device_bytes;
      sv->in_use += cp->bytes;
      cp->points_id = (st < 2 && q->r.points_id > 0) ? q->r.points_id : 0;
      cp->busy = false;
      cp->last_use = ++sv->use_clock;
      if (st == ESN_ERR_HIP) {                      // do not keep a plan after a runtime error
        esn_destroy(cp->plan);
        sv->in_use -= cp->bytes;
        for (size_t i = 0; i < sv->cache.size(); i++)
          if (sv->cache[i].get() == cp) {
            sv->cache.erase(sv->cache.begin() + i);
            break;
          }
      }
    }
    sv->peak = std::max(sv->peak, sv->in_use);
    finish(sv, q, st);
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
  }
}

}  // namespace

extern "C" int esn_server_create(const esn_opts* opts, int nslots, long long hbm_budget_bytes,
                                 esn_server* out) {
  if (!out || nslots < 1 || nslots > 64 || hbm_budget_bytes <= 0) return ESN_ERR_BAD_ARG;
  *out = nullptr;
  auto* sv = new (std::nothrow) esn_server_s();
  if (!sv) return ESN_ERR_ALLOC;
  if (opts) sv->opts = *opts;
  else esn_default_opts(&sv->opts);
  sv->opts.debug = 0;
  sv->budget = hbm_budget_bytes;
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return ESN_ERR_HIP;
  }
  for (int i = 0; i < nslots; i++) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (auto t : sv->streams) (void)hipStreamDestroy(t);
      delete sv;
      return ESN_ERR_HIP;
    }
    sv->streams.push_back(s);
  }
  for (int i = 0; i < nslots; i++) sv->workers.emplace_back(worker_loop, sv, i);
  *out = sv;
  return ESN_OK;
}

extern "C" int esn_server_submit(esn_server sv, const esn_request* r, long long* ticket) {
  if (!sv || !r || !ticket) return ESN_ERR_BAD_ARG;
  if ((r->type != 1 && r->type != 2) || r->dim < 1 || r->dim > 3 || r->M < 0 ||
      (r->isign != 1 && r->isign != -1) || (r->prec != ESN_SINGLE && r->prec != ESN_DOUBLE) ||
      (r->coord_prec != ESN_SINGLE && r->coord_prec != ESN_DOUBLE) || !r->f ||
      (r->M > 0 && !r->c))
    return ESN_ERR_BAD_ARG;
  for (int m = 0; m < r->dim; m++)
    if (r->nmodes[m] < 1) return ESN_ERR_BAD_ARG;
  auto q = std::make_shared<Req>();
  q->r = *r;
  for (int m = r->dim; m < 3; m++) q->r.nmodes[m] = 1;
  q->key = plan_key(q->r);
  q->est = esn::plan_estimate_bytes(r->type, r->dim, q->r.nmodes, r->eps, r->prec, r->M);
  if (q->est < 0) return ESN_ERR_BAD_ARG;
  (void)hipSetDevice(sv->device);
  if (hipEventCreateWithFlags(&q->ready, hipEventDisableTiming) != hipSuccess) return ESN_ERR_HIP;
  if (hipEventRecord(q->ready, static_cast<hipStream_t>(r->stream)) != hipSuccess) {
    (void)hipEventDestroy(q->ready);
    return ESN_ERR_HIP;
  }
  q->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stop) {
    (void)hipEventDestroy(q->ready);
    return ESN_ERR_QUEUE;
  }
  q->ticket = sv->next_ticket++;
  if (!sv->have_first) {
    sv->t_first = q->t_submit;
    sv->have_first = true;
  }
  sv->submitted++;
  sv->tickets[q->ticket] = q;
  sv->queue.push_back(q);
  *ticket = q->ticket;
  sv->cv_work.notify_one();
  return ESN_OK;
}

extern "C" int esn_server_wait(esn_server sv, long long ticket, int* status, double* latency_ms) {
  if (!sv) return ESN_ERR_BAD_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return ESN_ERR_QUEUE;
  std::shared_ptr<Req> q = it->second;
  sv->cv_done.wait(lk, [&] { return q->done; });
  if (status) *status = q->status;
  if (latency_ms)
    *latency_ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count();
  sv->tickets.erase(ticket);
  return ESN_OK;
}

extern "C" int esn_server_stats(esn_server sv, esn_serve_stats* o) {
  if (!sv || !o) return ESN_ERR_BAD_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  std::memset(o, 0, sizeof(*o));
  o->submitted = sv->submitted;
  o->completed = sv->completed;
  o->failed = sv->failed;
  o->rejected = sv->rejected;
  o->queued = (long long)sv->queue.size();
  o->running = sv->running;
  o->plan_cache_hits = sv->plan_hits;
  o->plan_cache_misses = sv->plan_misses;
  o->point_cache_hits = sv->point_hits;
  o->hbm_in_use = sv->in_use;
  o->hbm_peak = sv->peak;
  o->cached_plans = (long long)sv->cache.size();
  if (!sv->lat_ms.empty()) {
    std::vector<double> v(sv->lat_ms);
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      const double pos = p * (double)(v.size() - 1);
      const size_t i = (size_t)pos;
      const double fr = pos - (double)i;
      return i + 1 < v.size() ? v[i] * (1 - fr) + v[i + 1] * fr : v[i];
    };
    o->p50_ms = pct(0.50);
    o->p99_ms = pct(0.99);
    double s = 0;
    for (double x : v) s += x;
    o->mean_ms = s / (double)v.size();
    o->max_ms = v.back();
    const double wall = std::chrono::duration<double>(sv->t_last - sv->t_first).count();
    o->pts_per_s = wall > 0 ? sv->pts_done / wall : 0;
  }
  return ESN_OK;
}

extern "C" int esn_server_reset_stats(esn_server sv) {
  if (!sv) return ESN_ERR_BAD_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->lat_ms.clear();
  sv->submitted = sv->completed = sv->failed = sv->rejected = 0;
  sv->plan_hits = sv->plan_misses = sv->point_hits = 0;
  sv->pts_done = 0;
  sv->have_first = false;
  sv->peak = sv->in_use;
  return ESN_OK;
}

extern "C" int esn_server_destroy(esn_server sv) {
  if (!sv) return ESN_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;                // workers finish the queue, then exit
  }
  sv->cv_work.notify_all();
  for (auto& t : sv->workers) t.join();
  (void)hipSetDevice(sv->device);
  for (auto& c : sv->cache) esn_destroy(c->plan);
  for (auto s : sv->streams) (void)hipStreamDestroy(s);
  delete sv;
  return ESN_OK;
}
