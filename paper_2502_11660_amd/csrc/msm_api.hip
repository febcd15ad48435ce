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
  int mode = MSM_PROFILE_OFF;
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
  // timing only: no system-scope fence (cache writeback and invalidation)
  // when the event is recorded
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

void set_last_hip_error(int e) { g_last_hip = e; }

// set while msm_run_noalloc enqueues: no timing events are taken then (an
// event pool refill would create events)
static thread_local bool t_no_events = false;

ProfScope::ProfScope(int t, hipStream_t s) : tag(t), st(s) {
  if (t_no_events) return;
  std::lock_guard<std::mutex> g(g_prof.mu);
  if (g_prof.mode != MSM_PROFILE_PHASES) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  a = prof_event();
  if (a && hipEventRecord(a, st) == hipSuccess) active = true;
}

ProfScope::~ProfScope() {
  if (!active) return;
  std::lock_guard<std::mutex> g(g_prof.mu);
  hipEvent_t b = prof_event();
  if (b && hipEventRecord(b, st) == hipSuccess) g_prof.recs.push_back({tag, a, b});
}

bool prof_kernel_events(int tag, hipStream_t st, hipEvent_t* a, hipEvent_t* b) {
  if (t_no_events) return false;
  std::lock_guard<std::mutex> g(g_prof.mu);
  if (g_prof.mode != MSM_PROFILE_ACCUM_KERNEL || tag != PT_ACCUM) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
  *a = prof_event();
  *b = prof_event();
  if (*a && *b) return true;
  if (*a) g_prof.pool.push_back(*a);
  if (*b) g_prof.pool.push_back(*b);
  return false;
}

void prof_kernel_record(int tag, hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  g_prof.recs.push_back({tag, a, b});
}

int num_windows(int c, int encoding) {
  if (encoding == MSM_DIGITS_SIGNED) return (c >= 2 && c <= 20) ? (SCALAR_BITS + c) / c : 0;
  if (encoding == MSM_DIGITS_GLV) return (c >= 2 && c <= 20) ? (GLV_BITS + c) / c : 0;
  if (encoding == MSM_DIGITS_UNSIGNED) return (c >= 1 && c <= 20) ? (SCALAR_BITS + c - 1) / c : 0;
  return 0;
}

// Window width actually used for a requested width c: the smallest width
// that covers the digit bits with the same number of windows, so that no
// window (in particular the top one) is left with a few bits whose digits
// would crowd a handful of buckets.
int window_bits(int c, int encoding) {
  const int W = num_windows(c, encoding);
  if (W == 0) return 0;
  const int bits = encoding == MSM_DIGITS_UNSIGNED ? SCALAR_BITS
                   : encoding == MSM_DIGITS_GLV    ? GLV_BITS + 1
                                                   : SCALAR_BITS + 1;
  return (bits + W - 1) / W;
}

int default_window(size_t n) {
  // additions ~ n W (accumulation) + ~1.3 * 2^c W (signed-digit aggregation
  // of 2^(c-1) buckets per window, merges included); widths above 18 win
  // from n ~ 2^23 on (n = 2^24: c = 20 measured 5% faster than 17)
  int best = 8;
  double best_cost = 1e300;
  for (int c = 4; c <= 20; ++c) {
    double W = num_windows(c, MSM_DIGITS_SIGNED);
    double cost = (double)n * W + 1.3 * std::ldexp(1.0, c) * W;
    if (cost < best_cost) {
      best_cost = cost;
      best = c;
    }
  }
  return best;
}

int default_window_for(size_t n, int encoding) {
  if (encoding != MSM_DIGITS_GLV) return default_window(n);
  // split digits: 2n W entries of W = ceil(127 / c') windows, and 2^(c'-1)
  // buckets per window, each costing about as much as 3.9 entries (tree,
  // merges and the sort's identity fill: fitted to the n = 2^20 width sweep).
  // Measured picks: c' = 16 up to n ~ 2^21 (2^18: 18% faster than the
  // signed model's 15), c' = 19 above (2^22: 3%, 2^24: 10% faster than 16).
  int best = 16;
  double best_cost = 1e300;
  for (int c = 4; c <= 20; ++c) {
    const double W = num_windows(c, MSM_DIGITS_GLV);
    if (W == 0) continue;
    const int cw = window_bits(c, MSM_DIGITS_GLV);
    const double cost = 2.0 * (double)n * W + 3.9 * std::ldexp(1.0, cw - 1) * W;
    if (cost < best_cost) {
      best_cost = cost;
      best = c;
    }
  }
  return best;
}

// compute units of the current device (256 on MI355X; also the answer when
// no device is visible, e.g. for workspace queries on a host without GPU)
static int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0) {
    (void)hipGetLastError();
    return 256;
  }
  return cus;
}

bool make_plan(const size_t* ns, uint32_t J, int c_req, int encoding, Plan& pl,
               const Schedule& sched) {
  pl = Plan();
  const int W = num_windows(c_req, encoding);
  if (W == 0 || J == 0 || !ns) return false;
  if (sched.chunk < 0 || sched.tree_quad < 0 || sched.tree_wide < 0) return false;
  if (sched.tree_quad) pl.tree_quad = (uint64_t)sched.tree_quad;
  if (sched.tree_wide) pl.tree_wide = (uint64_t)sched.tree_wide;
  const int c = window_bits(c_req, encoding);
  pl.c = c;
  pl.W = W;
  pl.encoding = encoding;
  pl.bb = encoding == MSM_DIGITS_UNSIGNED ? c : c - 1;
  pl.J = J;
  // with the endomorphism split every input point contributes two points
  const size_t mult = encoding == MSM_DIGITS_GLV ? 2 : 1;
  for (uint32_t j = 0; j < J; ++j) {
    if (ns[j] == 0 || ns[j] >= ((size_t)1 << 26)) return false;
    const size_t nv = mult * ns[j];
    pl.N += nv;
    pl.max_n = std::max(pl.max_n, nv);
  }
  pl.S = (size_t)J * W;
  pl.M = pl.S << pl.bb;
  pl.NW = pl.N * (size_t)W;
  // entry positions, keys (s 2^bb + m) and point indices are 32-bit words
  if (pl.N >= ((size_t)1 << 31) || pl.NW >= ((size_t)1 << 31) || pl.M >= ((size_t)1 << 31))
    return false;
  sort_geometry(pl, ns, J, mult);
  if (pl.lo_bits > 8 || pl.nb > 4096 || pl.tiles >= ((size_t)1 << 31)) return false;
  if (J == 1) {
    pl.one.n = (uint32_t)(mult * ns[0]);
    pl.one.tps = (uint32_t)((mult * ns[0] + pl.tile_digits - 1) / pl.tile_digits);
  }
  // accumulation chunks: one per lane k_accum keeps resident in one round
  // (CUs x 4 SIMDs x 3 waves x 64 lanes; its register use allows 3 waves per
  // SIMD), so that every lane runs exactly once and no second, mostly idle
  // round follows; at least 16 entries per chunk.  Chunk lengths are
  // multiples of 4 (every chunk starts on a 16-byte boundary): Kx chunks of
  // K + 4 entries, then chunks of K, with K the multiple of 4 below the
  // average, so that the lanes' work differs by at most 4 entries instead of
  // all lanes taking the average rounded up to a multiple of 4 and some lanes
  // none.  A schedule's chunk gives every chunk the same length.
  const size_t lanes = (size_t)device_cus() * 4 * 3 * 64;
  if (sched.chunk) {
    pl.K = ((uint32_t)std::max(4, sched.chunk) + 3u) & ~3u;
    pl.Kx = 0;
  } else {
    const size_t k0 = std::max<size_t>(16, (pl.NW / lanes) & ~(size_t)3);
    pl.K = (uint32_t)k0;
    pl.Kx = pl.NW > k0 * lanes ? (uint32_t)((pl.NW - k0 * lanes + 3) / 4) : 0u;
  }
  {
    const size_t longer = (size_t)pl.Kx * (pl.K + 4);
    pl.chunks = pl.Kx + (pl.NW > longer ? (pl.NW - longer + pl.K - 1) / pl.K : 0);
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  const size_t rec = XYTZ_WORDS * 4;
  pl.o_flags = take((size_t)J * 4);
  pl.o_total = take(4);
  pl.o_offsets = take((pl.M + 1) * 4);
  pl.o_counts = take(pl.ncounts * 4);
  pl.o_blocksums = take(4096 * 4);
  pl.o_digits = take(pl.NW * 4);
  pl.o_tmp = take(pl.NW * 8);
  pl.o_key = take(pl.NW * 4 + 32);  // + 16-byte groups read past the end
  pl.o_idx = take(pl.NW * 4 + 32);
  pl.o_head = take(pl.chunks * rec);
  pl.o_tail = take(pl.chunks * rec);
  pl.o_longlist = take((pl.chunks + 1) * 4);
  // large sort partitions: each holds more than SORT_PART_CAP entries, so
  // there are at most NW / SORT_PART_CAP of them, and NW / SORT_BIG_ITEM +
  // that many items
  const size_t nbig_max = pl.NW / SORT_PART_CAP + 1;
  pl.o_big = take((nbig_max + 1) * 4);
  pl.o_bigdesc = take((nbig_max + 1) * 16);
  pl.o_bigcnt = take((pl.NW / SORT_BIG_ITEM + nbig_max + 1) * 256 * 4);
  pl.o_bigitem = take((pl.NW / SORT_BIG_ITEM + nbig_max + 1) * 4);
  // buckets, then the tree levels ping-pong between lvl0 (level 0's M
  // records) and the bucket array, which level 0 has consumed
  pl.o_buckets = take(pl.M * rec);
  pl.o_lvl0 = take(pl.M * rec);
  pl.o_lvl1 = pl.o_buckets;
  pl.o_wsum = take(2 * pl.S * rec);
  pl.o_qstate = take((size_t)J * rec);
  pl.o_jobs = take((size_t)J * sizeof(JobDesc));
  pl.o_segoff = take(pl.S * 8);
  pl.bytes = o;
  return true;
}

int enqueue_msm(const Plan& pl, void* ws, hipStream_t st, hipEvent_t accum_after) {
  uint32_t* buckets = ws_at<uint32_t>(ws, pl.o_buckets);
  int rc;
  {
    ProfScope prof(PT_SORT, st);
    rc = launch_sort(pl, buckets, ws, st);
  }
  if (rc != MSM_OK) return rc;
  if (accum_after) HIPCHK(hipStreamWaitEvent(st, accum_after, 0));
  if ((rc = launch_accumulate(pl, buckets, ws, st)) != MSM_OK) return rc;
  if ((rc = launch_aggregate(pl, buckets, ws, st)) != MSM_OK) return rc;
  return launch_horner(pl, ws, st);
}

// Scratch of msm_run_noalloc: a file-scope device array, one copy per GPU,
// held until the process ends.  Host code must not use the array's name as a
// device address; the address comes from hipGetSymbolAddress, taken once per
// device (with that device current) on the entry point's first call there.
constexpr size_t kScratchBytes = (size_t)MSM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static int scratch_of_current_device(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return MSM_EINVAL;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return MSM_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MSM_OK;
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

int msm_num_windows(int c, int encoding) { return num_windows(c, encoding); }

int msm_default_window(size_t n) { return default_window(n); }

int msm_window_bits(int c, int encoding) { return window_bits(c, encoding); }

size_t msm_workspace_bytes(size_t n, int c, int encoding) {
  if (c == 0) c = default_window_for(n, encoding);
  Plan pl;
  if (!make_plan(&n, 1, c, encoding, pl)) return 0;
  return pl.bytes;
}

int msm_fe_mul_batch(const uint32_t* a, const uint32_t* b, uint32_t* out, size_t count,
                     int canonical, void* stream) {
  if (!a || !b || !out || count == 0 || count >= (1u << 31)) return MSM_EINVAL;
  return launch_fe_mul(a, b, out, (uint32_t)count, canonical, (hipStream_t)stream);
}

int msm_padd_batch(const uint32_t* a_xytz, const uint32_t* b, uint32_t* out_xytz, size_t count,
                   int b_form, void* stream) {
  if (!a_xytz || !b || !out_xytz || count == 0 || count >= (1u << 29)) return MSM_EINVAL;
  if (b_form != MSM_FORM_XYTZ && b_form != MSM_FORM_XYU) return MSM_EINVAL;
  return launch_padd(a_xytz, b, out_xytz, (uint32_t)count, b_form, (hipStream_t)stream);
}

int msm_points_prepare(const uint32_t* xy_std, const uint32_t* inf, uint32_t* xyu, size_t n,
                       uint32_t* status, void* stream) {
  if (!xy_std || !xyu || !status || n == 0 || n >= (1u << 31)) return MSM_EINVAL;
  return launch_prepare(xy_std, inf, xyu, (uint32_t)n, status, false, (hipStream_t)stream);
}

int msm_points_prepare_endo(const uint32_t* xy_std, const uint32_t* inf, uint32_t* xyu, size_t n,
                            uint32_t* status, void* stream) {
  if (!xy_std || !xyu || !status || n == 0 || n >= (1u << 30)) return MSM_EINVAL;
  return launch_prepare(xy_std, inf, xyu, (uint32_t)n, status, true, (hipStream_t)stream);
}

int msm_gen_points(const uint32_t* k, size_t n, uint32_t* xy_std, uint32_t* inf, void* stream) {
  if (!k || !xy_std || !inf || n == 0 || n >= (1u << 31)) return MSM_EINVAL;
  return launch_gen_points(k, xy_std, inf, (uint32_t)n, (hipStream_t)stream);
}

int msm_bucket_accumulate(const uint32_t* xyu, const uint32_t* scalars, size_t n, int c,
                          int encoding, uint32_t* buckets, void* ws, size_t ws_bytes,
                          void* stream) {
  if (!xyu || !scalars || !buckets || !ws) return MSM_EINVAL;
  Plan pl;
  if (!make_plan(&n, 1, c, encoding, pl)) return MSM_EINVAL;
  if (ws_bytes < pl.bytes) return MSM_ENOSPC;
  pl.one.xyu = xyu;
  pl.one.scalars = scalars;
  hipStream_t st = (hipStream_t)stream;
  int rc;
  {
    ProfScope prof(PT_SORT, st);
    rc = launch_sort(pl, buckets, ws, st);
  }
  if (rc != MSM_OK) return rc;
  return launch_accumulate(pl, buckets, ws, st);
}

int msm_run(const uint32_t* xyu, const uint32_t* scalars, size_t n, int c, int encoding,
            uint32_t* result, void* ws, size_t ws_bytes, void* stream) {
  if (!xyu || !scalars || !result || !ws) return MSM_EINVAL;
  if (c == 0) c = default_window_for(n, encoding);
  Plan pl;
  if (!make_plan(&n, 1, c, encoding, pl)) return MSM_EINVAL;
  if (ws_bytes < pl.bytes) return MSM_ENOSPC;
  pl.one.xyu = xyu;
  pl.one.scalars = scalars;
  pl.one.result = result;
  return enqueue_msm(pl, ws, (hipStream_t)stream);
}

int msm_run_noalloc(const uint32_t* xyu, const uint32_t* scalars, size_t n, int c, int encoding,
                    uint32_t* result, void* stream) {
  if (!xyu || !scalars || !result) return MSM_EINVAL;
  if (c == 0) c = default_window_for(n, encoding);
  Plan pl;
  if (!make_plan(&n, 1, c, encoding, pl)) return MSM_EINVAL;
  if (pl.bytes > kScratchBytes) return MSM_ENOSPC;  // the MSM needs more than the scratch
  void* ws = nullptr;
  const int rc = scratch_of_current_device(&ws);
  if (rc != MSM_OK) return rc;
  pl.one.xyu = xyu;
  pl.one.scalars = scalars;
  pl.one.result = result;
  t_no_events = true;
  const int rc2 = enqueue_msm(pl, ws, (hipStream_t)stream);
  t_no_events = false;
  return rc2;
}

int msm_profile_enable(int mode) {
  if (mode < MSM_PROFILE_OFF || mode > MSM_PROFILE_ACCUM_KERNEL) return MSM_EINVAL;
  std::lock_guard<std::mutex> g(g_prof.mu);
  g_prof.mode = mode;
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
