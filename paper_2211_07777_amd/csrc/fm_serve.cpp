// Serving loop of the library: a request queue with continuous admission.
//
// Requests (one Poisson solve each, any grid, boundary conditions and layout) wait in
// FIFO order until a device stream ("slot") and their workspace fit; the workspace comes
// from one device arena of a fixed HBM budget, sub-allocated first-fit.  Each admitted
// request runs on its own slot, so the work of several requests overlaps on the device;
// when a request finishes (its event has completed) its workspace and slot return to the
// pool and the next waiting requests are admitted.  Plans (the Green's spectrum and the
// twiddle tables) are cached by problem key and evicted least-recently-used when their
// device memory exceeds the plan budget and no request uses them.
//
// A request's solve is ordered after the work its submitter had enqueued on the
// producer stream (an event recorded at submission), and after the generation of its
// plan: a new plan is generated on the server's own stream without blocking the host,
// so submission and admission never wait for the device.
//
// Built on the library's public entry points and the deferred plan creation of
// fm_internal.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/fluxmi.h"
#include "fm_internal.h"

namespace {

size_t round256(size_t x) { return (x + 255) & ~size_t(255); }

// First-fit sub-allocator over [0, size) with coalescing free blocks.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round256(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round256(std::max<size_t>(bytes, 1));
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;  // offset -> size
  size_t used_ = 0;
};

struct PlanKey {
  int n[3];
  double h[3];
  int bc[6];
  int layout, green, prec, kind, ncomp;
  bool operator<(const PlanKey& o) const {
    return std::memcmp(this, &o, sizeof(PlanKey)) < 0;
  }
};

struct CachedPlan {
  fm_plan plan = nullptr;
  size_t bytes = 0;     // plan tables in HBM
  size_t ws_bytes = 0;  // workspace of one solve
  long long last_use = 0;
  int users = 0;        // waiting or running requests
  hipEvent_t ready = nullptr;  // generation still pending (deferred creation)
};

struct Request {
  long long ticket;
  CachedPlan* cp;
  const void* rhs;
  void* out;
  size_t ws_off = 0;
  hipEvent_t produced = nullptr;  // recorded on the submitter's stream
};

}  // namespace

struct fm_server_s {
  size_t budget = 0, plan_budget = 0;
  char* arena_base = nullptr;
  Arena arena;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<Request> slot_req;
  std::vector<bool> slot_busy;
  std::map<PlanKey, CachedPlan> cache;
  size_t plan_bytes = 0;
  std::deque<Request> waiting;
  std::vector<std::pair<long long, int>> finished;  // (ticket, status)
  std::vector<hipEvent_t> spare_events;             // producer events not in use
  hipStream_t gen_stream = nullptr;                 // plan generation
  long long next_ticket = 0, clock = 0;
  int tune = 0;
  fm_server_stats stats{};
  int running = 0;
  // test hook (FLUXMI_SERVER_FAIL_TICKET at server creation): the admission of this
  // ticket reports FM_E_HIP without enqueuing anything, so that the error path of a
  // request can be exercised from the host
  long long fail_ticket = -1;
};

namespace {

void hip_failed(hipError_t e) { fm::set_last_hip_error((int)e); }

// Plans whose generation has completed release their temporaries.
void settle_plans(fm_server_s* s) {
  for (auto& kv : s->cache) {
    CachedPlan& cp = kv.second;
    if (cp.ready && hipEventQuery(cp.ready) == hipSuccess) {
      fm::plan_generation_done(cp.plan);
      cp.ready = nullptr;
    }
  }
}

// A request leaves the server: its workspace (if admitted) and producer event return to
// the pools, and (ticket, status) joins the finished list.
void retire(fm_server_s* s, Request& r, bool admitted, int status) {
  if (admitted) s->arena.release(r.ws_off, r.cp->ws_bytes);
  r.cp->users -= 1;
  if (r.produced) s->spare_events.push_back(r.produced);
  r.produced = nullptr;
  s->finished.emplace_back(r.ticket, status);
  s->stats.finished += 1;
  if (status != FM_OK) s->stats.failed += 1;
}

void evict_plans(fm_server_s* s) {
  while (s->plan_bytes > s->plan_budget) {
    auto victim = s->cache.end();
    for (auto it = s->cache.begin(); it != s->cache.end(); ++it)
      if (it->second.users == 0 && (victim == s->cache.end() || it->second.last_use < victim->second.last_use))
        victim = it;
    if (victim == s->cache.end()) return;  // everything cached is in use
    fm_plan_destroy(victim->second.plan);
    s->plan_bytes -= victim->second.bytes;
    s->cache.erase(victim);
    ++s->stats.plan_evictions;
  }
}

// Finished slots return their workspace; then waiting requests are admitted in FIFO
// order (a request that does not fit yet keeps its place; later ones may pass it only
// within a short look-ahead, so that large requests are not starved).  A request whose
// solve cannot be enqueued finishes with that error status.
int progress(fm_server_s* s) {
  for (size_t k = 0; k < s->streams.size(); ++k) {
    if (!s->slot_busy[k]) continue;
    const hipError_t e = hipEventQuery(s->events[k]);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) {
      hip_failed(e);
      return FM_E_HIP;
    }
    retire(s, s->slot_req[k], true, FM_OK);
    s->slot_busy[k] = false;
    s->running -= 1;
  }
  settle_plans(s);
  const size_t lookahead = 8;
  for (size_t i = 0; i < s->waiting.size() && i < lookahead;) {
    size_t k = 0;
    while (k < s->slot_busy.size() && s->slot_busy[k]) ++k;
    if (k == s->slot_busy.size()) break;  // no free slot
    Request& r = s->waiting[i];
    size_t off = 0;
    if (!s->arena.alloc(r.cp->ws_bytes, &off)) {
      ++i;
      continue;
    }
    r.ws_off = off;
    hipStream_t st = s->streams[k];
    int rc = FM_OK;
    hipError_t e = hipStreamWaitEvent(st, r.produced, 0);
    if (e == hipSuccess && r.cp->ready) e = hipStreamWaitEvent(st, r.cp->ready, 0);
    if (e != hipSuccess) {
      hip_failed(e);
      rc = FM_E_HIP;
    }
    if (rc == FM_OK && r.ticket == s->fail_ticket) {
      fm::set_last_hip_error((int)hipErrorLaunchFailure);
      rc = FM_E_HIP;
    }
    if (rc == FM_OK) rc = fm_solve(r.cp->plan, r.rhs, r.out, s->arena_base + off, st);
    if (rc == FM_OK) {
      e = hipEventRecord(s->events[k], st);
      if (e != hipSuccess) {
        hip_failed(e);
        return FM_E_HIP;
      }
      s->slot_req[k] = r;
      s->slot_busy[k] = true;
      s->running += 1;
      s->stats.peak_inflight = std::max(s->stats.peak_inflight, s->running);
      s->stats.peak_workspace_bytes = std::max(s->stats.peak_workspace_bytes, s->arena.used());
    } else {
      retire(s, r, true, rc);
    }
    s->waiting.erase(s->waiting.begin() + (long)i);
  }
  return FM_OK;
}

}  // namespace

extern "C" {

int fm_server_create(fm_server* out, size_t workspace_budget_bytes, size_t plan_budget_bytes,
                     int slots, int tune_plans) {
  if (!out) return FM_E_NULL;
  *out = nullptr;
  if (slots < 1 || slots > 64 || workspace_budget_bytes == 0) return FM_E_ARG;
  fm_server_s* s = new (std::nothrow) fm_server_s();
  if (!s) return FM_E_NOMEM;
  s->budget = round256(workspace_budget_bytes);
  s->plan_budget = plan_budget_bytes;
  s->tune = tune_plans;
  if (const char* f = std::getenv("FLUXMI_SERVER_FAIL_TICKET")) s->fail_ticket = std::atoll(f);
  if (hipMalloc(&s->arena_base, s->budget) != hipSuccess) {
    delete s;
    return FM_E_NOMEM;
  }
  s->arena.reset(s->budget);
  s->streams.resize(slots, nullptr);
  s->events.resize(slots, nullptr);
  s->slot_req.resize(slots);
  s->slot_busy.assign(slots, false);
  {
    const hipError_t e = hipStreamCreateWithFlags(&s->gen_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      hip_failed(e);
      fm_server_destroy(s);
      return FM_E_HIP;
    }
  }
  for (int k = 0; k < slots; ++k) {
    hipError_t e = hipStreamCreateWithFlags(&s->streams[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->events[k], hipEventDisableTiming);
    if (e != hipSuccess) {
      hip_failed(e);
      fm_server_destroy(s);
      return FM_E_HIP;
    }
  }
  *out = s;
  return FM_OK;
}

int fm_server_submit(fm_server s, const int n[3], const double h[3], const int bc[3][2], int layout,
                     int green, int prec, int kind, int ncomp, const void* rhs_dev, void* out_dev,
                     void* hip_stream, long long* ticket) {
  if (!s || !n || !h || !bc || !rhs_dev || !out_dev || !ticket) return FM_E_NULL;
  PlanKey key;
  std::memset(&key, 0, sizeof key);
  for (int a = 0; a < 3; ++a) {
    key.n[a] = n[a];
    key.h[a] = h[a];
    key.bc[2 * a] = bc[a][0];
    key.bc[2 * a + 1] = bc[a][1];
  }
  key.layout = layout;
  key.green = green;
  key.prec = prec;
  key.kind = kind;
  key.ncomp = ncomp;
  // the producer event first: nothing of the request exists if it cannot be had
  hipEvent_t produced = nullptr;
  if (!s->spare_events.empty()) {
    produced = s->spare_events.back();
    s->spare_events.pop_back();
  } else {
    const hipError_t e = hipEventCreateWithFlags(&produced, hipEventDisableTiming);
    if (e != hipSuccess) {
      hip_failed(e);
      return FM_E_HIP;
    }
  }
  {
    const hipError_t e = hipEventRecord(produced, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) {
      s->spare_events.push_back(produced);
      hip_failed(e);
      return FM_E_HIP;
    }
  }
  auto it = s->cache.find(key);
  if (it == s->cache.end()) {
    CachedPlan cp;
    int rc = fm::plan_create_deferred(&cp.plan, n, h, bc, layout, green, prec, kind, ncomp, s->gen_stream,
                                      &cp.ready);
    if (rc == FM_OK) {
      fm_plan_workspace_bytes(cp.plan, &cp.ws_bytes);
      if (round256(cp.ws_bytes) > s->budget) rc = FM_E_NOMEM;  // can never be admitted
    }
    if (rc == FM_OK && s->tune) {
      // tuning times kernels on the host clock: the generation must be complete first.
      // Tune with a block of the arena when one is free, else with the plan's own.
      const hipError_t e = hipEventSynchronize(cp.ready);
      if (e != hipSuccess) {
        hip_failed(e);
        rc = FM_E_HIP;
      } else {
        fm::plan_generation_done(cp.plan);
        cp.ready = nullptr;
        size_t off = 0;
        const bool got = s->arena.alloc(cp.ws_bytes, &off);
        rc = fm_plan_tune(cp.plan, got ? s->arena_base + off : nullptr, nullptr);
        if (got) s->arena.release(off, cp.ws_bytes);
      }
    }
    if (rc) {
      if (cp.plan) fm_plan_destroy(cp.plan);
      s->spare_events.push_back(produced);
      return rc;
    }
    fm_plan_device_bytes(cp.plan, &cp.bytes);
    s->plan_bytes += cp.bytes;
    it = s->cache.emplace(key, cp).first;
    ++s->stats.plan_misses;
  } else {
    ++s->stats.plan_hits;
  }
  CachedPlan* cp = &it->second;
  cp->users += 1;
  cp->last_use = ++s->clock;
  Request r;
  r.ticket = s->next_ticket++;
  r.cp = cp;
  r.rhs = rhs_dev;
  r.out = out_dev;
  r.produced = produced;
  s->waiting.push_back(r);
  s->stats.submitted += 1;
  *ticket = r.ticket;
  evict_plans(s);
  return progress(s);
}

int fm_server_progress(fm_server s, long long* finished, int* status, int max_finished,
                       int* n_finished) {
  if (!s || !n_finished) return FM_E_NULL;
  const int rc = progress(s);
  int k = 0;
  if (finished) {
    const int take = std::min<int>(max_finished, (int)s->finished.size());
    for (; k < take; ++k) {
      finished[k] = s->finished[k].first;
      if (status) status[k] = s->finished[k].second;
    }
    s->finished.erase(s->finished.begin(), s->finished.begin() + take);
  }
  *n_finished = k;
  return rc;
}

int fm_server_wait_all(fm_server s) {
  if (!s) return FM_E_NULL;
  while (!s->waiting.empty() || s->running > 0) {
    for (size_t k = 0; k < s->streams.size(); ++k)
      if (s->slot_busy[k]) {
        const hipError_t e = hipEventSynchronize(s->events[k]);
        if (e != hipSuccess) {
          hip_failed(e);
          return FM_E_HIP;
        }
        break;
      }
    const int rc = progress(s);
    if (rc) return rc;
  }
  return FM_OK;
}

int fm_server_get_stats(fm_server s, fm_server_stats* st) {
  if (!s || !st) return FM_E_NULL;
  *st = s->stats;
  st->cached_plans = (int)s->cache.size();
  st->plan_bytes = s->plan_bytes;
  st->waiting = (int)s->waiting.size();
  st->running = s->running;
  return FM_OK;
}

int fm_server_destroy(fm_server s) {
  if (!s) return FM_OK;
  int rc = FM_OK;
  if (s->arena_base) rc = fm_server_wait_all(s);
  for (auto& kv : s->cache) fm_plan_destroy(kv.second.plan);
  for (hipEvent_t e : s->events)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : s->spare_events) (void)hipEventDestroy(e);
  for (Request& r : s->waiting)
    if (r.produced) (void)hipEventDestroy(r.produced);
  if (s->gen_stream) (void)hipStreamDestroy(s->gen_stream);
  for (hipStream_t st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  if (s->arena_base) (void)hipFree(s->arena_base);
  delete s;
  return rc;
}

}  // extern "C"
