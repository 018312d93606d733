// Continuous-batching server over streaming plans (fringe_serve.h): one
// streaming plan and one HIP stream per subarray, a worker thread that
// admits, launches and collects, and a queue of finished chunks with their
// candidates.  Host code only; the searches are the plans' kernels.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "fringe.h"
#include "fringe_serve.h"

namespace fringe {
void set_last_error(const char* msg);
}

namespace {

int serve_fail(int code, const char* msg) {
  fringe::set_last_error(msg);
  return code;
}

int64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return int64_t(ts.tv_sec) * 1000000000 + ts.tv_nsec;
}

struct Req {
  int sub = 0;
  int64_t tag = 0;
  const fringe_cf32* d = nullptr;
  int64_t t_submit = 0;
  int64_t t_launch = 0;
  int status = FRINGE_OK;
};

struct Done {
  fringe_serve_result r;
  std::vector<fringe_candidate> c;
};

}  // namespace

struct fringe_server_s {
  int device = 0;
  int n_subs = 0;
  int max_inflight = 0;
  int64_t max_candidates = 0;
  std::vector<fringe_plan_t> plans;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  // under mu: the queues, finished results, counters, flags
  std::mutex mu;
  std::condition_variable cv;
  std::vector<std::deque<Req>> queues;
  std::deque<Done> done;
  int64_t pending = 0;
  bool submitted = false;
  bool stop = false;
  // the worker's own
  std::vector<char> busy;
  std::vector<Req> running;
  int inflight = 0;
  std::vector<fringe_candidate> buf;
  std::thread worker;
};

namespace {

void finish(fringe_server_s* s, int sub, int status) {
  const Req& q = s->running[size_t(sub)];
  Done d{};
  d.r.sub = sub;
  d.r.tag = q.tag;
  d.r.t_submit_ns = q.t_submit;
  d.r.t_launch_ns = q.t_launch;
  d.r.status = status;
  if (status == FRINGE_OK) {
    int64_t total = 0;
    const int rc = candidates_get(s->plans[size_t(sub)], s->buf.data(),
                                  int64_t(s->buf.size()), &total);
    if (rc == FRINGE_OK || rc == FRINGE_E_CAPACITY) {
      const int64_t n = std::min<int64_t>(total, int64_t(s->buf.size()));
      d.c.assign(s->buf.begin(), s->buf.begin() + n);
      d.r.n_candidates = n;
      d.r.n_total = total;
    } else {
      d.r.status = rc;
    }
    fringe_plan_summary inf{};
    if (fringe_plan_info(s->plans[size_t(sub)], &inf) == FRINGE_OK) d.r.n_windows = inf.n_windows;
  }
  d.r.t_done_ns = now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  s->done.push_back(std::move(d));
  s->busy[size_t(sub)] = 0;
  --s->inflight;
}

// Admit (oldest waiting head first, one chunk per subarray, at most
// max_inflight in all), launch, and collect until stopped with nothing in
// flight.  When nothing is in flight it sleeps until a submission; while
// searches run it polls their events.
void work(fringe_server_s* s) {
  (void)hipSetDevice(s->device);
  std::vector<int> launch;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->inflight == 0) {
        s->cv.wait(lk, [&] {
          if (s->stop) return true;
          for (const auto& q : s->queues)
            if (!q.empty()) return true;
          return false;
        });
        if (s->stop) break;
      }
      if (!s->stop) {
        std::vector<int> ready;
        for (int i = 0; i < s->n_subs; ++i)
          if (!s->busy[size_t(i)] && !s->queues[size_t(i)].empty()) ready.push_back(i);
        std::sort(ready.begin(), ready.end(), [&](int a, int b) {
          const int64_t ta = s->queues[size_t(a)].front().t_submit;
          const int64_t tb = s->queues[size_t(b)].front().t_submit;
          return ta != tb ? ta < tb : a < b;
        });
        for (int i : ready) {
          if (s->inflight >= s->max_inflight) break;
          s->running[size_t(i)] = s->queues[size_t(i)].front();
          s->queues[size_t(i)].pop_front();
          s->busy[size_t(i)] = 1;
          ++s->inflight;
          launch.push_back(i);
        }
      }
    }
    for (int i : launch) {
      Req& q = s->running[size_t(i)];
      q.t_launch = now_ns();
      const fringe_cf32* p = q.d;
      int rc = fringe_search(s->plans[size_t(i)], &p, s->streams[size_t(i)]);
      if (rc == FRINGE_OK && hipEventRecord(s->events[size_t(i)], s->streams[size_t(i)]) != hipSuccess)
        rc = FRINGE_E_HIP;
      q.status = rc;
      if (rc != FRINGE_OK) finish(s, i, rc);
    }
    launch.clear();
    bool any = false;
    for (int i = 0; i < s->n_subs; ++i) {
      if (!s->busy[size_t(i)]) continue;
      const hipError_t e = hipEventQuery(s->events[size_t(i)]);
      if (e == hipErrorNotReady) continue;
      finish(s, i, e == hipSuccess ? FRINGE_OK : FRINGE_E_HIP);
      any = true;
    }
    if (!any) std::this_thread::yield();
  }
  // stopped: let the searches in flight end before the plans go
  for (int i = 0; i < s->n_subs; ++i)
    if (s->busy[size_t(i)]) (void)hipStreamSynchronize(s->streams[size_t(i)]);
}

void release(fringe_server_s* s) {
  for (auto p : s->plans)
    if (p) fringe_plan_destroy(p);
  for (auto st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  for (auto ev : s->events)
    if (ev) (void)hipEventDestroy(ev);
  delete s;
}

}  // namespace

extern "C" {

int64_t fringe_monotonic_ns(void) { return now_ns(); }

int fringe_server_create(const fringe_scan_desc* subs, int32_t n_subs,
                         const fringe_params* params, int32_t time_chunk,
                         int32_t max_inflight, fringe_server_t* out) {
  if (!out) return serve_fail(FRINGE_E_INVALID, "fringe_server_create: null output pointer");
  *out = nullptr;
  if (!subs || !params || n_subs < 1 || n_subs > 4096)
    return serve_fail(FRINGE_E_INVALID, "fringe_server_create: null argument or n_subs out of [1, 4096]");
  if (max_inflight < 0 || max_inflight > n_subs)
    return serve_fail(FRINGE_E_INVALID, "fringe_server_create: max_inflight out of [0, n_subs]");
  if (params->flags & (FRINGE_PLAIN | FRINGE_GRAPH))
    return serve_fail(FRINGE_E_UNSUPPORTED,
                      "fringe_server_create: FRINGE_PLAIN and FRINGE_GRAPH do not stream");
  auto* s = new fringe_server_s();
  s->n_subs = n_subs;
  s->max_inflight = max_inflight ? max_inflight : n_subs;
  s->max_candidates = params->max_candidates;
  if (hipGetDevice(&s->device) != hipSuccess) {
    release(s);
    return serve_fail(FRINGE_E_HIP, "fringe_server_create: hipGetDevice");
  }
  fringe_params p = *params;
  p.flags |= FRINGE_STREAMING;
  s->plans.assign(size_t(n_subs), nullptr);
  s->streams.assign(size_t(n_subs), nullptr);
  s->events.assign(size_t(n_subs), nullptr);
  for (int i = 0; i < n_subs; ++i) {
    int rc = fringe_plan(&subs[i], 1, &p, &s->plans[size_t(i)]);
    if (rc == FRINGE_OK && time_chunk) rc = fringe_plan_set_chunk(s->plans[size_t(i)], 0, time_chunk);
    if (rc != FRINGE_OK) {
      release(s);
      return rc;
    }
    if (hipStreamCreateWithFlags(&s->streams[size_t(i)], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->events[size_t(i)], hipEventDisableTiming) != hipSuccess) {
      release(s);
      return serve_fail(FRINGE_E_HIP, "fringe_server_create: stream or event creation");
    }
  }
  s->queues.resize(size_t(n_subs));
  s->busy.assign(size_t(n_subs), 0);
  s->running.resize(size_t(n_subs));
  s->buf.resize(size_t(std::max<int64_t>(1, params->max_candidates)));
  s->worker = std::thread(work, s);
  *out = s;
  return FRINGE_OK;
}

int fringe_server_set_shifts(fringe_server_t s, int32_t sub, const int32_t* d_shifts) {
  if (!s) return serve_fail(FRINGE_E_INVALID, "fringe_server_set_shifts: null server");
  if (sub < 0 || sub >= s->n_subs)
    return serve_fail(FRINGE_E_INVALID, "fringe_server_set_shifts: subarray out of range");
  // under the lock: a submission (which the worker needs before it touches
  // a plan) cannot slip in while the plan is made again
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->submitted)
    return serve_fail(FRINGE_E_STATE, "fringe_server_set_shifts: chunks were already submitted");
  return fringe_set_shifts(s->plans[size_t(sub)], 0, d_shifts);
}

int fringe_server_submit(fringe_server_t s, int32_t sub, int64_t tag, const fringe_cf32* d_chunk) {
  if (!s) return serve_fail(FRINGE_E_INVALID, "fringe_server_submit: null server");
  if (sub < 0 || sub >= s->n_subs)
    return serve_fail(FRINGE_E_INVALID, "fringe_server_submit: subarray out of range");
  if (!d_chunk) return serve_fail(FRINGE_E_INVALID, "fringe_server_submit: null chunk");
  Req q;
  q.sub = sub;
  q.tag = tag;
  q.d = d_chunk;
  q.t_submit = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return serve_fail(FRINGE_E_STATE, "fringe_server_submit: server stopping");
    s->queues[size_t(sub)].push_back(q);
    ++s->pending;
    s->submitted = true;
  }
  s->cv.notify_one();
  return FRINGE_OK;
}

int fringe_server_poll(fringe_server_t s, fringe_serve_result* out, int32_t capacity,
                       int32_t* n_out, fringe_candidate* cands, int64_t cand_capacity,
                       int64_t* n_cands) {
  if (!s || !n_out || !n_cands || capacity < 0 || cand_capacity < 0 ||
      (capacity > 0 && !out) || (cand_capacity > 0 && !cands))
    return serve_fail(FRINGE_E_INVALID, "fringe_server_poll: null or negative argument");
  *n_out = 0;
  *n_cands = 0;
  std::lock_guard<std::mutex> lk(s->mu);
  int64_t used = 0;
  while (*n_out < capacity && !s->done.empty()) {
    Done& d = s->done.front();
    const int64_t n = int64_t(d.c.size());
    if (used + n > cand_capacity) {
      if (*n_out == 0) {
        *n_cands = n;
        return serve_fail(FRINGE_E_CAPACITY, "fringe_server_poll: the oldest result's candidates "
                                             "exceed cand_capacity");
      }
      break;
    }
    out[*n_out] = d.r;
    if (n) std::copy(d.c.begin(), d.c.end(), cands + used);
    used += n;
    ++*n_out;
    --s->pending;
    s->done.pop_front();
  }
  *n_cands = used;
  return FRINGE_OK;
}

int fringe_server_pending(fringe_server_t s, int64_t* n) {
  if (!s || !n) return serve_fail(FRINGE_E_INVALID, "fringe_server_pending: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *n = s->pending;
  return FRINGE_OK;
}

int fringe_server_destroy(fringe_server_t s) {
  if (!s) return serve_fail(FRINGE_E_INVALID, "fringe_server_destroy: null server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_one();
  if (s->worker.joinable()) s->worker.join();
  release(s);
  return FRINGE_OK;
}

}  // extern "C"
