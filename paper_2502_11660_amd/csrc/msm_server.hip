// MSM server (msm_server_* in include/msm.h): a request loop that admits MSMs
// by the device-memory footprint of their workspace, runs admitted requests
// concurrently on a pool of streams, and retires them as their completion
// events fire.
//
// Memory: one arena of the whole budget is allocated at creation; requests
// take first-fit, 256-byte aligned ranges of it (sorted free list with
// coalescing), so a request never waits on an allocator call on the device.
// Admission is FIFO: a request that does not fit waits, and so does every
// later one, until retirements free enough of the arena.  Each admitted
// request runs the full pipeline (sort, accumulation, aggregation, group
// aggregation) on the stream with the fewest requests in flight, so requests
// that arrive while others run overlap with them on the device.
//
// Overlap trades latency for throughput: a later request's accumulation,
// which fills the device, delays an earlier request's latency-bound
// aggregation chains (no stream priorities are used).  So when fewer than
// OVERLAP_FROM requests are in flight, a new request's accumulation waits for
// the previous request to finish (only its digit sort overlaps), which keeps
// requests in arrival order at light load; with a backlog, requests overlap
// fully, which raises the throughput.
#include <algorithm>
#include <deque>
#include <map>
#include <vector>

#include "common.hpp"

using namespace msm;

namespace {

// in-flight requests from which a new request overlaps fully (see above)
constexpr int OVERLAP_FROM = 3;

struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  void reset(size_t bytes) {
    size = bytes;
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  bool alloc(size_t bytes, size_t& off) {
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      off = it->first;
      const size_t rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
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
  size_t free_bytes() const {
    size_t t = 0;
    for (const auto& kv : free_) t += kv.second;
    return t;
  }
};

struct Request {
  uint64_t ticket = 0;
  msm_job job{};
  Plan plan;
  size_t off = 0;
  int stream = -1;
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
  hipEvent_t done = nullptr;
};

}  // namespace

struct msm_server {
  int device = 0;
  int encoding = MSM_DIGITS_SIGNED;
  char* base = nullptr;
  Arena arena;
  std::vector<hipStream_t> streams;
  std::vector<int> load;  // requests in flight per stream
  std::deque<Request> queued;
  std::vector<Request> running;
  std::deque<uint64_t> finished;
  std::vector<hipEvent_t> events;  // idle completion events
  hipEvent_t gate = nullptr;  // recorded at the end of the last admitted request
  bool gate_used = false;
  uint64_t next_ticket = 1;
};

namespace {

int take_event(msm_server* s, hipEvent_t& e) {
  if (!s->events.empty()) {
    e = s->events.back();
    s->events.pop_back();
    return MSM_OK;
  }
  HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return MSM_OK;
}

// launch queued requests in order while their workspace fits
int admit(msm_server* s) {
  while (!s->queued.empty()) {
    Request& q = s->queued.front();
    size_t off = 0;
    if (!s->arena.alloc(q.plan.bytes, off)) break;
    int k = 0;
    for (int i = 1; i < (int)s->streams.size(); ++i)
      if (s->load[i] < s->load[k]) k = i;
    Request r = q;
    s->queued.pop_front();
    r.off = off;
    r.stream = k;
    // the request's kernels wait for what the caller enqueued before
    // submitting (no wait is enqueued when that work has already finished)
    int rc = MSM_OK;
    const hipError_t rq = hipEventQuery(r.ready);
    if (rq == hipErrorNotReady)
      rc = hipStreamWaitEvent(s->streams[k], r.ready, 0) == hipSuccess ? MSM_OK : MSM_EHIP;
    else if (rq != hipSuccess)
      rc = MSM_EHIP;
    if (rc == MSM_OK) rc = take_event(s, r.done);
    // (nothing to wait for when nothing is in flight or the previous
    // request has already finished)
    const bool in_order = s->gate_used && !s->running.empty() &&
                          (int)s->running.size() < OVERLAP_FROM &&
                          hipEventQuery(s->gate) == hipErrorNotReady;
    if (rc == MSM_OK)
      rc = enqueue_msm(r.plan, s->base + off, s->streams[k], in_order ? s->gate : nullptr);
    if (rc == MSM_OK && hipEventRecord(s->gate, s->streams[k]) != hipSuccess) rc = MSM_EHIP;
    if (rc == MSM_OK) s->gate_used = true;
    if (rc == MSM_OK && hipEventRecord(r.done, s->streams[k]) != hipSuccess) rc = MSM_EHIP;
    if (rc != MSM_OK) {
      s->arena.release(off, r.plan.bytes);
      if (r.done) s->events.push_back(r.done);
      s->events.push_back(r.ready);
      return rc;
    }
    s->events.push_back(r.ready);  // the wait is enqueued; the event can be reused
    ++s->load[k];
    s->running.push_back(r);
  }
  return MSM_OK;
}

// retire requests whose completion event has fired
int retire(msm_server* s) {
  int rc = MSM_OK;
  for (size_t i = 0; i < s->running.size();) {
    Request& r = s->running[i];
    const hipError_t e = hipEventQuery(r.done);
    if (e == hipErrorNotReady) {
      ++i;
      continue;
    }
    if (e != hipSuccess) {
      set_last_hip_error((int)e);
      rc = MSM_EHIP;
    }
    s->arena.release(r.off, r.plan.bytes);
    --s->load[r.stream];
    s->events.push_back(r.done);
    s->finished.push_back(r.ticket);
    s->running[i] = s->running.back();
    s->running.pop_back();
  }
  return rc;
}

void destroy(msm_server* s) {
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (Request& r : s->running) s->events.push_back(r.done);
  for (Request& r : s->queued) s->events.push_back(r.ready);
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  if (s->gate) (void)hipEventDestroy(s->gate);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  if (s->base) (void)hipFree(s->base);
  delete s;
}

int create(size_t budget, int nstreams, int encoding, msm_server* s) {
  HIPCHK(hipGetDevice(&s->device));
  s->encoding = encoding;
  HIPCHK(hipEventCreateWithFlags(&s->gate, hipEventDisableTiming));
  HIPCHK(hipMalloc((void**)&s->base, budget));
  s->arena.reset(budget);
  for (int i = 0; i < nstreams; ++i) {
    hipStream_t st = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    s->streams.push_back(st);
    s->load.push_back(0);
  }
  return MSM_OK;
}

}  // namespace

extern "C" {

int msm_server_create(size_t hbm_budget_bytes, int streams, int encoding, msm_server** out) {
  if (!out) return MSM_EINVAL;
  *out = nullptr;
  if (hbm_budget_bytes < 4096 || streams < 1 || streams > 16) return MSM_EINVAL;
  if (encoding != MSM_DIGITS_SIGNED && encoding != MSM_DIGITS_UNSIGNED &&
      encoding != MSM_DIGITS_GLV)
    return MSM_EINVAL;
  msm_server* s = new msm_server();
  const int rc = create(hbm_budget_bytes, streams, encoding, s);
  if (rc != MSM_OK) {
    destroy(s);
    return rc;
  }
  *out = s;
  return MSM_OK;
}

int msm_server_submit(msm_server* s, const msm_job* job, void* stream, uint64_t* ticket) {
  if (!s || !job || !ticket || !job->xyu || !job->scalars || !job->result) return MSM_EINVAL;
  Request r;
  r.job = *job;
  const int c = job->c == 0 ? default_window_for(job->n, s->encoding) : job->c;
  size_t n = job->n;
  Schedule sched;
  sched.chunk = job->chunk;
  sched.tree_quad = job->tree_quad;
  sched.tree_wide = job->tree_wide;
  if (!make_plan(&n, 1, c, s->encoding, r.plan, sched)) return MSM_EINVAL;
  if (r.plan.bytes > s->arena.size) return MSM_ENOSPC;
  r.plan.one.xyu = job->xyu;
  r.plan.one.scalars = job->scalars;
  r.plan.one.result = job->result;
  if (take_event(s, r.ready) != MSM_OK) return MSM_EHIP;
  if (hipEventRecord(r.ready, (hipStream_t)stream) != hipSuccess) {
    s->events.push_back(r.ready);
    return MSM_EHIP;
  }
  r.ticket = s->next_ticket++;
  *ticket = r.ticket;
  s->queued.push_back(r);
  int rc = retire(s);
  const int rc2 = admit(s);
  return rc != MSM_OK ? rc : rc2;
}

int msm_server_progress(msm_server* s, uint64_t* done, size_t cap, size_t* ndone) {
  if (!s || !ndone || (cap && !done)) return MSM_EINVAL;
  int rc = retire(s);
  const int rc2 = admit(s);
  size_t k = 0;
  while (k < cap && !s->finished.empty()) {
    done[k++] = s->finished.front();
    s->finished.pop_front();
  }
  *ndone = k;
  return rc != MSM_OK ? rc : rc2;
}

int msm_server_drain(msm_server* s) {
  if (!s) return MSM_EINVAL;
  for (;;) {
    int rc = retire(s);
    if (rc != MSM_OK) return rc;
    if ((rc = admit(s)) != MSM_OK) return rc;
    if (s->running.empty()) return s->queued.empty() ? MSM_OK : MSM_ENOSPC;
    HIPCHK(hipEventSynchronize(s->running.front().done));
  }
}

int msm_server_stats(msm_server* s, size_t* in_flight, size_t* queued, size_t* bytes_in_use) {
  if (!s) return MSM_EINVAL;
  if (in_flight) *in_flight = s->running.size();
  if (queued) *queued = s->queued.size();
  if (bytes_in_use) *bytes_in_use = s->arena.size - s->arena.free_bytes();
  return MSM_OK;
}

int msm_server_destroy(msm_server* s) {
  if (s) destroy(s);
  return MSM_OK;
}

}  // extern "C"
