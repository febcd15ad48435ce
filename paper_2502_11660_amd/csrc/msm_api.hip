// C ABI of libmsm_gfx950.so (include/msm.h): argument checks, workspace plans,
// per-phase timing and the entry points, which enqueue the kernels of the
// other translation units on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace msm {

namespace {
thread_local int g_last_hip = 0;

const char* const kProfNames[PT_COUNT] = {"sort", "accum", "merge", "agg", "horner"};

struct ProfState {
  std::mutex mu;
  bool on = false;
  struct Rec {
    int tag;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
};
ProfState g_prof;

hipEvent_t prof_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Internal streams for the window-group pipeline.  msm_run forks from the
// caller's stream: accumulation stays on the caller's stream, bucket
// aggregation of finished groups runs on stream `agg`, the group-aggregation
// (Horner) steps on stream `hor`; the caller's stream finally waits for
// `hor`.  All streams have the default priority.  A set is held (locked) only
// while one call enqueues its work; a few sets per device let concurrent
// callers on different streams overlap.
// ---------------------------------------------------------------------------
struct StreamSet {
  std::mutex mu;
  bool init = false;
  hipStream_t agg = nullptr, hor = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::vector<hipEvent_t> accdone, aggdone;  // per window group
};

constexpr int kSetsPerDevice = 4;
constexpr int kMaxDevices = 16;
StreamSet g_sets[kMaxDevices][kSetsPerDevice];
std::atomic<unsigned> g_set_rr{0};

int ensure_events(std::vector<hipEvent_t>& v, size_t n) {
  while (v.size() < n) {
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    v.push_back(e);
  }
  return MSM_OK;
}

int init_set(StreamSet& ss) {
  if (ss.init) return MSM_OK;
  HIPCHK(hipStreamCreateWithFlags(&ss.agg, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&ss.hor, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&ss.join, hipEventDisableTiming));
  ss.init = true;
  return MSM_OK;
}
}  // namespace

void set_last_hip_error(int e) { g_last_hip = e; }

ProfScope::ProfScope(int t, hipStream_t s) : tag(t), st(s) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  if (!g_prof.on) return;
  a = prof_event();
  if (a && hipEventRecord(a, st) == hipSuccess) active = true;
}

ProfScope::~ProfScope() {
  if (!active) return;
  std::lock_guard<std::mutex> g(g_prof.mu);
  hipEvent_t b = prof_event();
  if (b && hipEventRecord(b, st) == hipSuccess) g_prof.recs.push_back({tag, a, b});
}

int num_windows(int c) { return (SCALAR_BITS + c - 1) / c; }

int default_window(size_t n) {
  // additions ~ n W (accumulation) + ~2.6 * 2^c W (aggregation incl. merges)
  int best = 8;
  double best_cost = 1e300;
  for (int c = 4; c <= 18; ++c) {
    double W = num_windows(c);
    double cost = (double)n * W + 2.6 * std::ldexp(1.0, c) * W;
    if (cost < best_cost) {
      best_cost = cost;
      best = c;
    }
  }
  return best;
}

bool make_plan(size_t n, int c, Plan& pl) {
  if (n == 0 || n >= (1u << 26) || c < 1 || c > 20) return false;
  pl = Plan();
  pl.c = c;
  pl.W = num_windows(c);
  pl.n = n;
  pl.M = (size_t)pl.W << c;
  pl.NW = n * (size_t)pl.W;
  // window groups (tunable through MSM_WINDOW_GROUPS; default one group)
  int want_groups = 1;
  if (const char* e = std::getenv("MSM_WINDOW_GROUPS")) want_groups = std::max(1, std::atoi(e));
  want_groups = std::min(want_groups, pl.W);
  pl.gw = (pl.W + want_groups - 1) / want_groups;
  pl.G = (pl.W + pl.gw - 1) / pl.gw;
  // accumulation chunk: a group's launch keeps about 2 waves per SIMD busy
  // (256 CUs x 4 SIMDs x 2 waves x 64 lanes = 131072 lanes), K in [16, 64]
  const size_t group_entries = n * (size_t)pl.gw;
  pl.K = 16;
  while (pl.K < 64 && group_entries / (2 * pl.K) >= 131072) pl.K *= 2;
  pl.group_chunks = (group_entries + pl.K - 1) / pl.K;
  pl.chunks = pl.group_chunks * pl.G;
  pl.ncounts = sort_counts_size(c, pl.W, n);
  if (pl.ncounts == (size_t)-1) return false;
  pl.nb = (pl.ncounts + 4095) / 4096;
  if (pl.nb > 4096) return false;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  pl.o_flags = take(4);
  pl.o_total = take(4);
  pl.o_maxspan = take(4);
  pl.o_hist = take((pl.M + 1) * 4);
  pl.o_counts = take(pl.ncounts * 4);
  pl.o_blocksums = take(4096 * 4);
  pl.o_digits = take(pl.NW * 4);
  pl.o_tmp = take(pl.NW * 8);
  pl.o_key = take(pl.NW * 4);
  pl.o_idx = take(pl.NW * 4);
  pl.o_head = take(pl.chunks * XYTZ_WORDS * 4);
  pl.o_tail = take(pl.chunks * XYTZ_WORDS * 4);
  pl.o_buckets = take(pl.M * XYTZ_WORDS * 4);
  pl.lvl_records = pl.M;  // the largest tree level holds W * 2^c records
  pl.o_lvl0 = take(pl.lvl_records * XYTZ_WORDS * 4);
  pl.o_lvl1 = take(pl.lvl_records * XYTZ_WORDS * 4);
  pl.o_wsum = take(2 * (size_t)pl.W * XYTZ_WORDS * 4);
  pl.o_qstate = take(XYTZ_WORDS * 4);
  pl.o_longlist = take((size_t)pl.G * (pl.group_chunks + 1) * 4);
  pl.bytes = o;
  return true;
}

}  // namespace msm

using namespace msm;

extern "C" {

int msm_last_hip_error(void) { return g_last_hip; }

const char* msm_status_string(int status) {
  switch (status) {
    case MSM_OK: return "MSM_OK";
    case MSM_EINVAL: return "MSM_EINVAL: invalid argument";
    case MSM_ENOSPC: return "MSM_ENOSPC: workspace too small";
    case MSM_EHIP: return "MSM_EHIP: HIP runtime error";
    default: return "unknown status";
  }
}

int msm_num_windows(int c) { return (c >= 1 && c <= 20) ? num_windows(c) : 0; }

int msm_default_window(size_t n) { return default_window(n); }

size_t msm_workspace_bytes(size_t n, int c) {
  if (c == 0) c = default_window(n);
  Plan pl;
  if (!make_plan(n, c, pl)) return 0;
  return pl.bytes;
}

int msm_fe_mul_batch(const uint32_t* a, const uint32_t* b, uint32_t* out, size_t count,
                     int canonical, void* stream) {
  if (!a || !b || !out || count == 0 || count >= (1u << 31)) return MSM_EINVAL;
  return launch_fe_mul(a, b, out, (uint32_t)count, canonical, (hipStream_t)stream);
}

int msm_padd_batch(const uint32_t* a_xytz, const uint32_t* b, uint32_t* out_xytz, size_t count,
                   int b_form, void* stream) {
  if (!a_xytz || !b || !out_xytz || count == 0 || count >= (1u << 31)) return MSM_EINVAL;
  if (b_form != MSM_FORM_XYTZ && b_form != MSM_FORM_XYU) return MSM_EINVAL;
  return launch_padd(a_xytz, b, out_xytz, (uint32_t)count, b_form, (hipStream_t)stream);
}

int msm_points_prepare(const uint32_t* xy_std, const uint32_t* inf, uint32_t* xyu, size_t n,
                       uint32_t* status, void* stream) {
  if (!xy_std || !xyu || !status || n == 0 || n >= (1u << 31)) return MSM_EINVAL;
  return launch_prepare(xy_std, inf, xyu, (uint32_t)n, status, (hipStream_t)stream);
}

int msm_gen_points(const uint32_t* k, size_t n, uint32_t* xy_std, uint32_t* inf, void* stream) {
  if (!k || !xy_std || !inf || n == 0 || n >= (1u << 31)) return MSM_EINVAL;
  return launch_gen_points(k, xy_std, inf, (uint32_t)n, (hipStream_t)stream);
}

int msm_bucket_accumulate(const uint32_t* xyu, const uint32_t* scalars, size_t n, int c,
                          uint32_t* buckets, void* ws, size_t ws_bytes, void* stream) {
  if (!xyu || !scalars || !buckets || !ws) return MSM_EINVAL;
  Plan pl;
  if (!make_plan(n, c, pl)) return MSM_EINVAL;
  if (ws_bytes < pl.bytes) return MSM_ENOSPC;
  hipStream_t st = (hipStream_t)stream;
  int rc;
  {
    ProfScope prof(PT_SORT, st);
    rc = launch_sort(pl, scalars, buckets, ws, st);
  }
  if (rc != MSM_OK) return rc;
  for (int g = 0; g < pl.G; ++g)
    if ((rc = launch_accumulate_group(pl, g, xyu, buckets, ws, st)) != MSM_OK) return rc;
  return MSM_OK;
}

int msm_run(const uint32_t* xyu, const uint32_t* scalars, size_t n, int c, uint32_t* result,
            void* ws, size_t ws_bytes, void* stream) {
  if (!xyu || !scalars || !result || !ws) return MSM_EINVAL;
  if (c == 0) c = default_window(n);
  Plan pl;
  if (!make_plan(n, c, pl)) return MSM_EINVAL;
  if (ws_bytes < pl.bytes) return MSM_ENOSPC;
  hipStream_t st = (hipStream_t)stream;
  uint32_t* buckets = ws_at<uint32_t>(ws, pl.o_buckets);
  int rc;
  {
    ProfScope prof(PT_SORT, st);
    rc = launch_sort(pl, scalars, buckets, ws, st);
  }
  if (rc != MSM_OK) return rc;
  if (pl.G == 1) {
    // one group: nothing to overlap, stay on the caller's stream
    if ((rc = launch_accumulate_group(pl, 0, xyu, buckets, ws, st)) != MSM_OK) return rc;
    if ((rc = launch_aggregate_group(pl, 0, buckets, ws, st)) != MSM_OK) return rc;
    if ((rc = launch_horner_group(pl, 0, ws, st)) != MSM_OK) return rc;
    return launch_finalize(pl, result, ws, st);
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return MSM_EINVAL;
  StreamSet& ss = g_sets[dev][g_set_rr.fetch_add(1) % kSetsPerDevice];
  std::lock_guard<std::mutex> lock(ss.mu);
  if ((rc = init_set(ss)) != MSM_OK) return rc;
  if ((rc = ensure_events(ss.accdone, pl.G)) != MSM_OK) return rc;
  if ((rc = ensure_events(ss.aggdone, pl.G)) != MSM_OK) return rc;
  HIPCHK(hipEventRecord(ss.fork, st));
  HIPCHK(hipStreamWaitEvent(ss.agg, ss.fork, 0));
  HIPCHK(hipStreamWaitEvent(ss.hor, ss.fork, 0));
  for (int g = 0; g < pl.G; ++g) {
    if ((rc = launch_accumulate_group(pl, g, xyu, buckets, ws, st)) != MSM_OK) return rc;
    HIPCHK(hipEventRecord(ss.accdone[g], st));
    HIPCHK(hipStreamWaitEvent(ss.agg, ss.accdone[g], 0));
    if ((rc = launch_aggregate_group(pl, g, buckets, ws, ss.agg)) != MSM_OK) return rc;
    HIPCHK(hipEventRecord(ss.aggdone[g], ss.agg));
    HIPCHK(hipStreamWaitEvent(ss.hor, ss.aggdone[g], 0));
    if ((rc = launch_horner_group(pl, g, ws, ss.hor)) != MSM_OK) return rc;
  }
  if ((rc = launch_finalize(pl, result, ws, ss.hor)) != MSM_OK) return rc;
  HIPCHK(hipEventRecord(ss.join, ss.hor));
  HIPCHK(hipStreamWaitEvent(st, ss.join, 0));
  return MSM_OK;
}

int msm_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  g_prof.on = on != 0;
  return MSM_OK;
}

int msm_profile_read(const char* phase, double* total_ms, int* launches) {
  if (!phase || !total_ms || !launches) return MSM_EINVAL;
  int tag = -1;
  for (int t = 0; t < PT_COUNT; ++t)
    if (std::strcmp(phase, kProfNames[t]) == 0) tag = t;
  if (tag < 0) return MSM_EINVAL;
  std::lock_guard<std::mutex> g(g_prof.mu);
  double tot = 0.0;
  int cnt = 0;
  std::vector<ProfState::Rec> keep;
  int rc = MSM_OK;
  for (auto& r : g_prof.recs) {
    if (r.tag != tag) {
      keep.push_back(r);
      continue;
    }
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) {
      set_last_hip_error((int)e);
      rc = MSM_EHIP;
    }
    tot += ms;
    ++cnt;
    g_prof.pool.push_back(r.a);
    g_prof.pool.push_back(r.b);
  }
  g_prof.recs.swap(keep);
  *total_ms = tot;
  *launches = cnt;
  return rc;
}

int msm_constants(uint32_t* out, size_t words) {
  if (!out || words < 96) return MSM_EINVAL;
  const uint32_t* tabs[8] = {kP, kOne, kR2, kK, kAlpha, kBeta, kGx, kGy};
  for (int t = 0; t < 8; ++t)
    for (int l = 0; l < NL; ++l) out[t * NL + l] = tabs[t][l];
  return MSM_OK;
}

}  // extern "C"
