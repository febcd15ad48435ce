// Batched MSMs (msm_batch_* in include/msm.h).
//
// Jobs are grouped into classes by window width and schedule (accumulation
// chunk size, aggregation-tree unit thresholds).  Each class is one pipeline
// (sort, accumulation, aggregation, group aggregation) whose kernels cover
// every window of every job in the class, so a batch of many small MSMs fills
// the chip like one large MSM and its many latency-bound group-aggregation
// chains run side by side in one launch.  Classes run concurrently: the first
// on the caller's stream, the others on the batch's own streams forked from
// and joined back into it.  With use_graph the whole launch sequence is
// captured once into a HIP graph and every run is a single graph launch.
#include <algorithm>
#include <map>
#include <vector>

#include "common.hpp"

using namespace msm;

struct msm_batch {
  int device = 0;
  char* ws = nullptr;
  std::vector<Plan> plans;
  std::vector<size_t> ws_off;
  std::vector<hipStream_t> side;  // stream of class k + 1
  std::vector<hipEvent_t> done;   // end of class k + 1
  hipEvent_t fork = nullptr, last = nullptr;
  hipStream_t cap = nullptr;  // capture stream
  bool use_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// a class: jobs with the same window width and schedule
typedef std::pair<int, Schedule> ClassKey;
typedef std::map<ClassKey, std::vector<size_t>> Classes;

Schedule schedule_of(const msm_job& jb) {
  Schedule s;
  s.chunk = jb.chunk;
  s.tree_quad = jb.tree_quad;
  s.tree_wide = jb.tree_wide;
  return s;
}

// classes of a job list: (window width, schedule) -> job indices (in job order)
bool classify(const msm_job* jobs, size_t njobs, int encoding, Classes& cls) {
  if (!jobs || njobs == 0 || njobs >= ((size_t)1 << 20)) return false;
  for (size_t i = 0; i < njobs; ++i) {
    const msm_job& jb = jobs[i];
    if (!jb.xyu || !jb.scalars || !jb.result || jb.n == 0) return false;
    if (jb.chunk < 0 || jb.tree_quad < 0 || jb.tree_wide < 0) return false;
    const int c = jb.c == 0 ? default_window_for(jb.n, encoding) : jb.c;
    if (num_windows(c, encoding) == 0) return false;
    cls[ClassKey(c, schedule_of(jb))].push_back(i);
  }
  return true;
}

bool plan_classes(const msm_job* jobs, const Classes& cls, int encoding, std::vector<Plan>& plans,
                  std::vector<size_t>& off, size_t& total) {
  total = 0;
  for (const auto& kv : cls) {
    std::vector<size_t> ns;
    for (size_t i : kv.second) ns.push_back(jobs[i].n);
    Plan pl;
    if (!make_plan(ns.data(), (uint32_t)ns.size(), kv.first.first, encoding, pl, kv.first.second))
      return false;
    plans.push_back(pl);
    off.push_back(total);
    total += align256(pl.bytes);
  }
  return true;
}

int enqueue_batch(msm_batch* b, hipStream_t st) {
  int rc;
  const size_t K = b->plans.size();
  if (K > 1) HIPCHK(hipEventRecord(b->fork, st));
  for (size_t k = 1; k < K; ++k) {
    HIPCHK(hipStreamWaitEvent(b->side[k - 1], b->fork, 0));
    if ((rc = enqueue_msm(b->plans[k], b->ws + b->ws_off[k], b->side[k - 1])) != MSM_OK) return rc;
    HIPCHK(hipEventRecord(b->done[k - 1], b->side[k - 1]));
  }
  if ((rc = enqueue_msm(b->plans[0], b->ws + b->ws_off[0], st)) != MSM_OK) return rc;
  for (size_t k = 1; k < K; ++k) HIPCHK(hipStreamWaitEvent(st, b->done[k - 1], 0));
  return MSM_OK;
}

void release(msm_batch* b) {
  if (b->last) (void)hipEventSynchronize(b->last);
  for (hipStream_t s : b->side) (void)hipStreamSynchronize(s);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipStream_t s : b->side) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->last) (void)hipEventDestroy(b->last);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

int create(const msm_job* jobs, size_t njobs, int encoding, void* ws, size_t ws_bytes,
           int use_graph, msm_batch* b) {
  Classes cls;
  if (!ws || !classify(jobs, njobs, encoding, cls)) return MSM_EINVAL;
  size_t total = 0;
  if (!plan_classes(jobs, cls, encoding, b->plans, b->ws_off, total)) return MSM_EINVAL;
  if (ws_bytes < total) return MSM_ENOSPC;
  HIPCHK(hipGetDevice(&b->device));
  b->ws = static_cast<char*>(ws);
  b->use_graph = use_graph != 0;
  // job tables: JobDesc per job; per segment the word offset of its job's
  // points from the first job's
  size_t k = 0;
  for (const auto& kv : cls) {
    Plan& pl = b->plans[k];
    std::vector<JobDesc> tab(kv.second.size());
    std::vector<int64_t> segoff(pl.S);
    const uint32_t* base_pts = jobs[kv.second[0]].xyu;
    uint32_t pt_off = 0, tile_off = 0;
    for (size_t j = 0; j < kv.second.size(); ++j) {
      const msm_job& jb = jobs[kv.second[j]];
      JobDesc& d = tab[j];
      d.xyu = jb.xyu;
      d.scalars = jb.scalars;
      d.result = jb.result;
      d.n = (uint32_t)(encoding == MSM_DIGITS_GLV ? 2 * jb.n : jb.n);
      d.pt_off = pt_off;
      d.tile_off = tile_off;
      d.tps = (uint32_t)((d.n + pl.tile_digits - 1) / pl.tile_digits);
      pt_off += d.n;
      tile_off += d.tps;
      const int64_t off = (int64_t)(jb.xyu - base_pts);
      for (int w = 0; w < pl.W; ++w) segoff[j * pl.W + w] = off;
    }
    pl.one = tab[0];
    char* base = b->ws + b->ws_off[k];
    HIPCHK(hipMemcpy(base + pl.o_jobs, tab.data(), tab.size() * sizeof(JobDesc),
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(base + pl.o_segoff, segoff.data(), segoff.size() * 8,
                     hipMemcpyHostToDevice));
    ++k;
  }
  for (size_t i = 1; i < b->plans.size(); ++i) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    b->side.push_back(s);
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->done.push_back(e);
  }
  HIPCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&b->last, hipEventDisableTiming));
  if (b->use_graph) HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  return MSM_OK;
}

}  // namespace

extern "C" {

size_t msm_batch_workspace_bytes(const msm_job* jobs, size_t njobs, int encoding) {
  Classes cls;
  if (!classify(jobs, njobs, encoding, cls)) return 0;
  std::vector<Plan> plans;
  std::vector<size_t> off;
  size_t total = 0;
  if (!plan_classes(jobs, cls, encoding, plans, off, total)) return 0;
  return total;
}

int msm_batch_create(const msm_job* jobs, size_t njobs, int encoding, void* ws, size_t ws_bytes,
                     int use_graph, msm_batch** out) {
  if (!out) return MSM_EINVAL;
  *out = nullptr;
  msm_batch* b = new msm_batch();
  const int rc = create(jobs, njobs, encoding, ws, ws_bytes, use_graph, b);
  if (rc != MSM_OK) {
    release(b);
    return rc;
  }
  *out = b;
  return MSM_OK;
}

int msm_batch_run(msm_batch* b, void* stream) {
  if (!b) return MSM_EINVAL;
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != b->device) return MSM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (!b->use_graph) {
    const int rc = enqueue_batch(b, st);
    if (rc != MSM_OK) return rc;
  } else {
    if (!b->exec) {
      HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
      const int rc = enqueue_batch(b, b->cap);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(b->cap, &g);
      if (rc != MSM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      HIPCHK(ec);
      b->graph = g;
      HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(b->exec, st));
  }
  HIPCHK(hipEventRecord(b->last, st));
  return MSM_OK;
}

int msm_batch_destroy(msm_batch* b) {
  if (b) release(b);
  return MSM_OK;
}

}  // extern "C"
