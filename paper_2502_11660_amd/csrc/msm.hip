// gfx950 BLS12-377 G1 MSM: kernels and the C ABI declared in include/msm.h.
//
// Pipeline of msm_run (Pippenger, Sec. II-C), all on the caller's stream:
//   1. k_hist      per-window digit histogram (global atomics)
//   2. scan        exclusive prefix sum -> CSR offsets over (window, digit)
//   3. k_scatter   point indices scattered into digit order (key, idx)
//   4. k_accum     bucket accumulation: each lane sums a fixed-length chunk of
//                  the digit-sorted list with the mixed addition, writing whole
//                  buckets directly and the cut ends of split buckets to
//                  per-chunk partial slots (balanced work per lane)
//   5. k_merge_*   split buckets: tree over the head partials, then tail+head
//   6. k_agg_level bucket aggregation by chunked running sums (Sec. II-C: the
//                  accumulated buckets are combined iteratively)
//   7. k_horner    group aggregation Q = sum_w 2^(wc) S_w and the map back to
//                  Weierstrass affine coordinates
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/msm.h"
#include "curve.hpp"
#include "field.hpp"

using namespace msm;

namespace {

// ---------------------------------------------------------------------------
// constants of the Weierstrass <-> twisted-Edwards map (Montgomery form)
// x_w = alpha u - 1, y_w = beta v, u = (1 + y_e)/(1 - y_e), v = u / x_e
// ---------------------------------------------------------------------------
constexpr uint32_t kAlpha[NL] = {0x8894e1e4u, 0x3fabdfd0u, 0xcc1f55aau, 0xcbf921ddu,
                                 0x460edc0cu, 0xd17deff1u, 0x7897028du, 0xd394e81eu,
                                 0x0912681au, 0xc29c995du, 0xaff9d568u, 0x01515e6cu};
constexpr uint32_t kBeta[NL] = {0xa38cfd11u, 0xface0c97u, 0x0adb8383u, 0x8cc7c229u,
                                0xd44ae9cbu, 0x4765cd5fu, 0x22354029u, 0x9ae986d8u,
                                0x252ab9bdu, 0xc3dc7860u, 0xc8942395u, 0x00486011u};
constexpr uint32_t kBetaOverAlpha[NL] = {0xead605e4u, 0xfb7c0ab8u, 0xe2752c7au, 0x363b93d1u,
                                         0x144be536u, 0xd2246835u, 0x429f2077u, 0xeb8bf6ddu,
                                         0x0234d423u, 0x3a9efda2u, 0xba0c72a4u, 0x013c7943u};
// conventional generator G of BLS12-377 G1, Weierstrass affine
constexpr uint32_t kGx[NL] = {0x772451f4u, 0x260f33b9u, 0x169d5658u, 0xc54dd773u,
                              0x69a510ddu, 0x5c1551c4u, 0x425e1698u, 0x761662e4u,
                              0x6f065272u, 0xc97d78ccu, 0xb361fd4du, 0x00a41206u};
constexpr uint32_t kGy[NL] = {0xb8cb81f3u, 0x8193961fu, 0x5f44adb8u, 0x00638d4cu,
                              0xd4daf54au, 0xfafaf3dau, 0xd655cd18u, 0xc27849e2u,
                              0x01d52814u, 0x2ec3ddb4u, 0x26303c71u, 0x007da933u};
// G in prepared twisted-Edwards form (x_e, y_e, k x_e y_e)
constexpr uint32_t kGteX[NL] = {0x654b417fu, 0x5bab21b3u, 0x1d3e1fe0u, 0x042fff8au,
                                0xdf39dc37u, 0xb702072eu, 0x39426b02u, 0xa5625e78u,
                                0xb51c7d03u, 0xbf2dc368u, 0x28ac3263u, 0x00b3ad90u};
constexpr uint32_t kGteY[NL] = {0xef15101du, 0x3904973cu, 0xb1f14456u, 0xb45ed211u,
                                0x5dfac94eu, 0x90a86b86u, 0xfe3945cdu, 0xcdb19c57u,
                                0xef4f7097u, 0x972a8d46u, 0xa3d9cf77u, 0x00281a91u};
constexpr uint32_t kGteU[NL] = {0x4f3f8d58u, 0x719243efu, 0x4a7b9d48u, 0xf744d1fcu,
                                0xa77008dcu, 0x0ab712e3u, 0x1e09b26fu, 0x53f80798u,
                                0xef3f9f1bu, 0x24125ab8u, 0xfb63f6d1u, 0x01959f77u};

constexpr int SCALAR_BITS = 253;
constexpr int SCALAR_WORDS = 8;
constexpr uint32_t NO_KEY = 0xffffffffu;

thread_local int g_last_hip = 0;

// ---------------------------------------------------------------------------
// optional per-kernel timing: HIP events recorded on the launch stream around
// each pipeline kernel while profiling is enabled
// ---------------------------------------------------------------------------
enum ProfTag { PT_SORT = 0, PT_ACCUM, PT_MERGE, PT_AGG, PT_HORNER, PT_COUNT };
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

struct ProfScope {
  bool active = false;
  int tag;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(int t, hipStream_t s) : tag(t), st(s) {
    std::lock_guard<std::mutex> g(g_prof.mu);
    if (!g_prof.on) return;
    a = prof_event();
    if (a && hipEventRecord(a, st) == hipSuccess) active = true;
  }
  ~ProfScope() {
    if (!active) return;
    std::lock_guard<std::mutex> g(g_prof.mu);
    hipEvent_t b = prof_event();
    if (b && hipEventRecord(b, st) == hipSuccess) g_prof.recs.push_back({tag, a, b});
  }
};

#define HIPCHK(x)                       \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) {             \
      g_last_hip = (int)e_;             \
      return MSM_EHIP;                  \
    }                                   \
  } while (0)

inline unsigned grid_for(size_t n, unsigned block) { return (unsigned)((n + block - 1) / block); }

// ---------------------------------------------------------------------------
// Weierstrass <-> twisted-Edwards conversions (device)
// ---------------------------------------------------------------------------

// Twisted-Edwards extended (Montgomery form) -> Weierstrass affine, ordinary
// form, canonical.  Returns false for the identity (x = y = 0 written).
__device__ bool te_to_weierstrass(const xytz& q, fe& xw, fe& yw) {
  fe X = fe_canon(q.X);
  if (fe_is_zero_canon(X)) {
    xw = fe_zero();
    yw = fe_zero();
    return false;
  }
  const fe p2 = fe_const(kP2);
  fe zpy = fe_add(q.Z, q.Y);                  // Z + Y  < 4p
  fe zmy = fe_sub_plus(q.Z, q.Y, p2);         // Z - Y  < 4p
  fe den = fe_mul(zmy, q.X);                  // (Z - Y) X
  fe inv = fe_inv(den);
  fe u = fe_mul(fe_mul(zpy, q.X), inv);       // (Z+Y)/(Z-Y)
  fe v = fe_mul(fe_mul(zpy, q.Z), inv);       // u / x_e
  fe au = fe_mul(u, fe_const(kAlpha));
  xw = fe_from_mont(fe_sub_plus(au, fe_const(kOne), p2));
  yw = fe_from_mont(fe_mul(v, fe_const(kBeta)));
  return true;
}

// ---------------------------------------------------------------------------
// elementwise kernels
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_fe_mul(const uint32_t* __restrict__ a,
                                                const uint32_t* __restrict__ b,
                                                uint32_t* __restrict__ out, uint32_t count,
                                                int canonical) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  fe x = ld_soa(a, count, 0, i);
  fe y = ld_soa(b, count, 0, i);
  fe r = fe_mul(x, y);
  if (canonical) r = fe_canon(r);
  st_soa(out, count, 0, i, r);
}

template <int FORM>
__global__ void __launch_bounds__(256) k_padd(const uint32_t* __restrict__ a,
                                              const uint32_t* __restrict__ b,
                                              uint32_t* __restrict__ out, uint32_t count) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const fe p2 = fe_const(kP2);
  xytz pa;
  pa.X = ld_soa(a, count, 0, i);
  pa.Y = ld_soa(a, count, 1, i);
  pa.T = ld_soa(a, count, 2, i);
  pa.Z = ld_soa(a, count, 3, i);
  xytz r;
  if (FORM == MSM_FORM_XYU) {
    xyu pb;
    pb.X = ld_soa(b, count, 0, i);
    pb.Y = ld_soa(b, count, 1, i);
    pb.U = ld_soa(b, count, 2, i);
    r = padd_mixed(pa, pb, p2);
  } else {
    xytz pb;
    pb.X = ld_soa(b, count, 0, i);
    pb.Y = ld_soa(b, count, 1, i);
    pb.T = ld_soa(b, count, 2, i);
    pb.Z = ld_soa(b, count, 3, i);
    r = padd_full(pa, pb, p2);
  }
  st_soa(out, count, 0, i, fe_canon(r.X));
  st_soa(out, count, 1, i, fe_canon(r.Y));
  st_soa(out, count, 2, i, fe_canon(r.T));
  st_soa(out, count, 3, i, fe_canon(r.Z));
}

// Weierstrass affine (ordinary form) -> prepared (X, Y, U = k x y), Z = 1:
//   w = x + 1,  x_e = (beta/alpha) w / y,  y_e = (w - alpha) / (w + alpha)
// one inversion of y (w + alpha) per point.
__global__ void __launch_bounds__(256) k_prepare(const uint32_t* __restrict__ xy,
                                                 const uint32_t* __restrict__ inf,
                                                 uint32_t* __restrict__ out, uint32_t n,
                                                 uint32_t* __restrict__ status) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t* rec = out + (size_t)i * XYU_WORDS;
  if (inf && inf[i]) {
    st_aos(rec, 0, fe_zero());
    st_aos(rec, 1, fe_const(kOne));
    st_aos(rec, 2, fe_zero());
    return;
  }
  const fe p2 = fe_const(kP2);
  fe x = fe_to_mont(ld_soa(xy, n, 0, i));
  fe y = fe_to_mont(ld_soa(xy, n, 1, i));
  // on-curve check y^2 == x^3 + 1
  fe lhs = fe_canon(fe_sqr(y));
  fe rhs = fe_canon(fe_add(fe_mul(fe_sqr(x), x), fe_const(kOne)));
  uint32_t flags = 0;
  if (!fe_eq_canon(lhs, rhs)) flags |= MSM_FLAG_OFFCURVE;
  fe w = fe_add(x, fe_const(kOne));                  // < 4p
  fe wpa = fe_add(w, fe_const(kAlpha));              // < 6p
  fe wma = fe_sub_plus(w, fe_const(kAlpha), p2);     // < 6p
  fe den = fe_mul(y, wpa);
  if (fe_is_zero_canon(fe_canon(den))) flags |= MSM_FLAG_EXCEPT;
  fe inv = fe_inv(den);
  fe xe = fe_mul(fe_mul(fe_mul(w, wpa), inv), fe_const(kBetaOverAlpha));
  fe ye = fe_mul(fe_mul(wma, y), inv);
  fe u = fe_mul(fe_mul(xe, ye), fe_const(kK));
  st_aos(rec, 0, fe_canon(xe));
  st_aos(rec, 1, fe_canon(ye));
  st_aos(rec, 2, fe_canon(u));
  if (flags) atomicOr(status, flags);
}

// P_i = k_i G by most-significant-bit-first double-and-add in twisted-Edwards
// coordinates, then mapped to Weierstrass affine.
__global__ void __launch_bounds__(256) k_gen_points(const uint32_t* __restrict__ kk,
                                                    uint32_t* __restrict__ xy,
                                                    uint32_t* __restrict__ inf, uint32_t n) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const fe p2 = fe_const(kP2);
  xyu g;
  g.X = fe_const(kGteX);
  g.Y = fe_const(kGteY);
  g.U = fe_const(kGteU);
  uint32_t kw[SCALAR_WORDS];
#pragma unroll
  for (int j = 0; j < SCALAR_WORDS; ++j) kw[j] = kk[(size_t)i * SCALAR_WORDS + j];
  xytz acc = pt_identity();
  for (int j = SCALAR_WORDS - 1; j >= 0; --j) {
    uint32_t word = kw[j];
    for (int bit = 31; bit >= 0; --bit) {
      acc = pdbl(acc, p2);
      if ((word >> bit) & 1u) acc = padd_mixed(acc, g, p2);
    }
  }
  fe xw, yw;
  bool fin = te_to_weierstrass(acc, xw, yw);
  st_soa(xy, n, 0, i, xw);
  st_soa(xy, n, 1, i, yw);
  inf[i] = fin ? 0u : 1u;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// scalar slicing and digit sort
// ---------------------------------------------------------------------------

struct scalar256 {
  uint32_t w[SCALAR_WORDS];
};

__device__ __forceinline__ scalar256 ld_scalar(const uint32_t* __restrict__ s, uint32_t i,
                                               uint32_t* __restrict__ flags) {
  const uint4* q = reinterpret_cast<const uint4*>(s + (size_t)i * SCALAR_WORDS);
  uint4 a = q[0], b = q[1];
  scalar256 r;
  r.w[0] = a.x; r.w[1] = a.y; r.w[2] = a.z; r.w[3] = a.w;
  r.w[4] = b.x; r.w[5] = b.y; r.w[6] = b.z; r.w[7] = b.w;
  if (r.w[7] >> (SCALAR_BITS - 224)) {
    if (flags) atomicOr(flags, MSM_FLAG_RANGE);
    r.w[7] &= (1u << (SCALAR_BITS - 224)) - 1u;
  }
  return r;
}

// c-bit digit starting at bit position `pos` (c <= 20, pos < 253).
__device__ __forceinline__ uint32_t digit_at(const scalar256& s, int pos, int c) {
  int wi = pos >> 5, sh = pos & 31;
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int j = 0; j < SCALAR_WORDS; ++j) {
    lo = (j == wi) ? s.w[j] : lo;
    hi = (j == wi + 1) ? s.w[j] : hi;
  }
  uint64_t two = ((uint64_t)hi << 32) | lo;
  return (uint32_t)(two >> sh) & ((1u << c) - 1u);
}

__global__ void __launch_bounds__(256) k_hist(const uint32_t* __restrict__ scalars, uint32_t n,
                                              int c, int W, uint32_t* __restrict__ hist,
                                              uint32_t* __restrict__ flags) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  scalar256 s = ld_scalar(scalars, i, flags);
  for (int w = 0; w < W; ++w) {
    uint32_t d = digit_at(s, w * c, c);
    if (d) atomicAdd(&hist[((size_t)w << c) + d], 1u);
  }
}

__global__ void __launch_bounds__(256) k_scatter(const uint32_t* __restrict__ scalars, uint32_t n,
                                                 int c, int W, uint32_t* __restrict__ cursor,
                                                 uint32_t* __restrict__ key,
                                                 uint32_t* __restrict__ idx) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  scalar256 s = ld_scalar(scalars, i, nullptr);
  for (int w = 0; w < W; ++w) {
    uint32_t d = digit_at(s, w * c, c);
    if (d) {
      uint32_t b = ((uint32_t)w << c) + d;
      uint32_t pos = atomicAdd(&cursor[b], 1u);
      key[pos] = b;
      idx[pos] = i;
    }
  }
}

// Exclusive scan, three passes.  SCAN_ITEMS elements per block.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_ITEMS = SCAN_THREADS * SCAN_PER_THREAD;

// block-wide exclusive scan of one value per thread; returns the total
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t& excl) {
  __shared__ uint32_t wsum[SCAN_THREADS / 64];
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  uint32_t base = 0, total = 0;
#pragma unroll
  for (int j = 0; j < SCAN_THREADS / 64; ++j) {
    uint32_t t = wsum[j];
    base += (j < wid) ? t : 0u;
    total += t;
  }
  excl = base + x - v;
  __syncthreads();
  return total;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_block(const uint32_t* __restrict__ in,
                                                             uint32_t* __restrict__ out, size_t n,
                                                             uint32_t* __restrict__ blocksums) {
  size_t base = (size_t)blockIdx.x * SCAN_ITEMS + (size_t)threadIdx.x * SCAN_PER_THREAD;
  uint32_t v[SCAN_PER_THREAD];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0u;
    sum += v[j];
  }
  uint32_t excl;
  uint32_t total = block_exclusive_scan(sum, excl);
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) {
    if (base + j < n) out[base + j] = excl;
    excl += v[j];
  }
  if (threadIdx.x == 0) blocksums[blockIdx.x] = total;
}

// single block: exclusive scan of up to SCAN_ITEMS block sums; the grand
// total goes to *total_out
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_top(uint32_t* __restrict__ blocksums,
                                                           uint32_t nb,
                                                           uint32_t* __restrict__ total_out,
                                                           uint32_t* __restrict__ total_out2) {
  size_t base = (size_t)threadIdx.x * SCAN_PER_THREAD;
  uint32_t v[SCAN_PER_THREAD];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) {
    v[j] = (base + j < nb) ? blocksums[base + j] : 0u;
    sum += v[j];
  }
  uint32_t excl;
  uint32_t total = block_exclusive_scan(sum, excl);
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) {
    if (base + j < nb) blocksums[base + j] = excl;
    excl += v[j];
  }
  if (threadIdx.x == 0) {
    *total_out = total;
    *total_out2 = total;
  }
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_add(uint32_t* __restrict__ out, size_t n,
                                                           const uint32_t* __restrict__ blocksums,
                                                           uint32_t* __restrict__ copy) {
  size_t base = (size_t)blockIdx.x * SCAN_ITEMS;
  uint32_t add = blocksums[blockIdx.x];
  for (int j = threadIdx.x; j < SCAN_ITEMS; j += SCAN_THREADS) {
    size_t i = base + j;
    if (i < n) {
      uint32_t v = out[i] + add;
      out[i] = v;
      copy[i] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// bucket accumulation
// ---------------------------------------------------------------------------

__global__ void k_fill_empty_buckets(const uint32_t* __restrict__ offsets, uint32_t M,
                                     uint32_t* __restrict__ buckets) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= M) return;
  if (offsets[b] == offsets[b + 1]) st_xytz(buckets + (size_t)b * XYTZ_WORDS, pt_identity());
}

// Lane `ch` sums entries [ch*K, min(ch*K+K, N)) of the digit-sorted list.
// Segments of equal key inside the chunk are bucket pieces:
//   * a piece that is the whole bucket goes straight to buckets[key];
//   * the first piece, if its bucket began in an earlier chunk, goes to
//     head[ch] (it may also run on into later chunks);
//   * otherwise the last piece, if its bucket runs on into later chunks, goes
//     to tail[ch] (this chunk is where that bucket starts).
__global__ void __launch_bounds__(256) k_accum(const uint32_t* __restrict__ pts,
                                               const uint32_t* __restrict__ key,
                                               const uint32_t* __restrict__ idx,
                                               const uint32_t* __restrict__ total, uint32_t K,
                                               uint32_t* __restrict__ buckets,
                                               uint32_t* __restrict__ head,
                                               uint32_t* __restrict__ tail) {
  const uint32_t N = *total;
  const uint32_t ch = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t s64 = (uint64_t)ch * K;
  if (s64 >= N) return;
  const uint32_t s = (uint32_t)s64;
  const uint32_t e = (uint32_t)std::min<uint64_t>(s64 + K, N);
  const fe p2 = fe_const(kP2);

  uint32_t cur = key[s];
  const bool open_left = (s > 0) && (key[s - 1] == cur);
  bool first_seg = true;
  xytz acc = pt_identity();
  xyu P = ld_xyu(pts + (size_t)idx[s] * XYU_WORDS);
  for (uint32_t p = s; p < e; ++p) {
    const uint32_t k = key[p];
    if (k != cur) {
      uint32_t* dst = (first_seg && open_left) ? head + (size_t)ch * XYTZ_WORDS
                                               : buckets + (size_t)cur * XYTZ_WORDS;
      st_xytz(dst, acc);
      acc = pt_identity();
      cur = k;
      first_seg = false;
    }
    const uint32_t pn = (p + 1 < e) ? p + 1 : p;
    xyu Pn = ld_xyu(pts + (size_t)idx[pn] * XYU_WORDS);
    acc = padd_mixed(acc, P, p2);
    P = Pn;
  }
  const bool open_right = (e < N) && (key[e] == cur);
  uint32_t* dst;
  if (first_seg && open_left)
    dst = head + (size_t)ch * XYTZ_WORDS;
  else if (open_right)
    dst = tail + (size_t)ch * XYTZ_WORDS;
  else
    dst = buckets + (size_t)cur * XYTZ_WORDS;
  st_xytz(dst, acc);
}

// For chunk ch whose first piece continues a bucket b that started in chunk
// c0 and ends in chunk c1, the head partials of chunks c0+1..c1 are summed by
// a binary tree: at step t, chunk c with (c - c0 - 1) % 2^(t+1) == 0 adds the
// head of chunk c + 2^t if that chunk still belongs to b.
__global__ void __launch_bounds__(256) k_merge_step(const uint32_t* __restrict__ key,
                                                    const uint32_t* __restrict__ offsets,
                                                    const uint32_t* __restrict__ total,
                                                    uint32_t K, uint32_t t,
                                                    uint32_t* __restrict__ head) {
  const uint32_t N = *total;
  const uint32_t ch = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t s64 = (uint64_t)ch * K;
  if (ch == 0 || s64 >= N) return;
  const uint32_t s = (uint32_t)s64;
  const uint32_t b = key[s];
  if (key[s - 1] != b) return;  // first piece is not a continuation
  const uint32_t c0 = offsets[b] / K;
  const uint32_t c1 = (offsets[b + 1] - 1) / K;
  const uint32_t rel = ch - c0 - 1;
  const uint32_t stride = 1u << t;
  if ((rel & ((stride << 1) - 1)) != 0) return;
  if (ch + stride > c1) return;
  const fe p2 = fe_const(kP2);
  uint32_t* mine = head + (size_t)ch * XYTZ_WORDS;
  xytz a = ld_xytz(mine);
  xytz o = ld_xytz(head + (size_t)(ch + stride) * XYTZ_WORDS);
  st_xytz(mine, padd_full(a, o, p2));
}

// Chunk ch holding a tail partial (its last piece starts a bucket that runs
// into later chunks): bucket = tail[ch] + head[ch + 1] (the tree sum).
__global__ void __launch_bounds__(256) k_merge_final(const uint32_t* __restrict__ key,
                                                     const uint32_t* __restrict__ total,
                                                     uint32_t K, const uint32_t* __restrict__ head,
                                                     const uint32_t* __restrict__ tail,
                                                     uint32_t* __restrict__ buckets) {
  const uint32_t N = *total;
  const uint32_t ch = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t s64 = (uint64_t)ch * K;
  if (s64 >= N) return;
  const uint32_t s = (uint32_t)s64;
  const uint32_t e = (uint32_t)std::min<uint64_t>(s64 + K, N);
  const uint32_t last = key[e - 1];
  const bool open_right = (e < N) && (key[e] == last);
  if (!open_right) return;
  const bool open_left = (s > 0) && (key[s - 1] == key[s]);
  if (open_left && key[s] == last) return;  // whole chunk is a middle piece
  const fe p2 = fe_const(kP2);
  xytz a = ld_xytz(tail + (size_t)ch * XYTZ_WORDS);
  xytz o = ld_xytz(head + (size_t)(ch + 1) * XYTZ_WORDS);
  st_xytz(buckets + (size_t)last * XYTZ_WORDS, padd_full(a, o, p2));
}

// ---------------------------------------------------------------------------
// bucket aggregation
// ---------------------------------------------------------------------------
// Per window the value sum_b b*R[b] is carried as  sum_l P[l] + mu * sum_l l*R[l].
// One level folds chunks of L consecutive entries:
//   run = sum_j R[lL+j],  acc = sum_j j*R[lL+j]   (running sum from the top)
//   P'[l] = sum_j P[lL+j] + mu*acc,  R'[l] = run,  mu' = mu*L
// Level 0 has P = 0, R = buckets, mu = 1; when one entry is left, S_w = P[0].
__global__ void __launch_bounds__(256) k_agg_level(const uint32_t* __restrict__ Pin,
                                                   const uint32_t* __restrict__ Rin,
                                                   uint32_t Min, uint32_t L, uint32_t logmu,
                                                   uint32_t W, uint32_t* __restrict__ Pout,
                                                   uint32_t* __restrict__ Rout) {
  const uint32_t Mout = Min / L;
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= W * Mout) return;
  const uint32_t w = g / Mout, l = g % Mout;
  const fe p2 = fe_const(kP2);
  const size_t base = (size_t)w * Min + (size_t)l * L;
  xytz run = pt_identity();
  xytz acc = pt_identity();
  for (uint32_t j = L - 1; j >= 1; --j) {
    run = padd_full(run, ld_xytz(Rin + (base + j) * XYTZ_WORDS), p2);
    acc = padd_full(acc, run, p2);
  }
  run = padd_full(run, ld_xytz(Rin + base * XYTZ_WORDS), p2);
  for (uint32_t t = 0; t < logmu; ++t) acc = pdbl(acc, p2);
  if (Pin) {
    for (uint32_t j = 0; j < L; ++j) acc = padd_full(acc, ld_xytz(Pin + (base + j) * XYTZ_WORDS), p2);
  }
  st_xytz(Pout + (size_t)g * XYTZ_WORDS, acc);
  st_xytz(Rout + (size_t)g * XYTZ_WORDS, run);
}

// Group aggregation Q = sum_w 2^(w c) S_w by Horner (c doublings per window),
// then the result in Weierstrass affine form.
__global__ void k_horner(const uint32_t* __restrict__ S, uint32_t W, uint32_t c,
                         const uint32_t* __restrict__ flags, uint32_t* __restrict__ result) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const fe p2 = fe_const(kP2);
  xytz q = ld_xytz(S + (size_t)(W - 1) * XYTZ_WORDS);
  for (int w = (int)W - 2; w >= 0; --w) {
    for (uint32_t t = 0; t < c; ++t) q = pdbl(q, p2);
    q = padd_full(q, ld_xytz(S + (size_t)w * XYTZ_WORDS), p2);
  }
  fe xw, yw;
  bool fin = te_to_weierstrass(q, xw, yw);
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    result[l] = xw.v[l];
    result[NL + l] = yw.v[l];
  }
  result[2 * NL] = fin ? 0u : 1u;
  result[2 * NL + 1] = flags ? *flags : 0u;
  for (int l = 2 * NL + 2; l < MSM_RESULT_WORDS; ++l) result[l] = 0u;
}

// ---------------------------------------------------------------------------
// host-side planning
// ---------------------------------------------------------------------------

constexpr uint32_t ACC_CHUNK = 32;  // entries per accumulation lane
constexpr uint32_t AGG_CHUNK = 16;  // buckets per aggregation lane

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Plan {
  int c = 0, W = 0;
  size_t n = 0, M = 0, NW = 0, chunks = 0, nb = 0;
  // byte offsets into the workspace
  size_t o_flags = 0, o_total = 0, o_hist = 0, o_cursor = 0, o_blocksums = 0, o_key = 0,
         o_idx = 0, o_head = 0, o_tail = 0, o_buckets = 0, o_agg0 = 0, o_agg1 = 0, agg_entries = 0,
         bytes = 0;
  std::vector<uint32_t> agg_L;  // chunk length of each aggregation level
};

int num_windows(int c) { return (SCALAR_BITS + c - 1) / c; }

int default_window(size_t n) {
  // Work ~ n W + 2^(c+1) W mixed/complete additions; pick the minimiser.
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
  pl.c = c;
  pl.W = num_windows(c);
  pl.n = n;
  pl.M = (size_t)pl.W << c;
  pl.NW = n * (size_t)pl.W;
  pl.chunks = (pl.NW + ACC_CHUNK - 1) / ACC_CHUNK;
  pl.nb = (pl.M + SCAN_ITEMS - 1) / SCAN_ITEMS;
  if (pl.nb > (size_t)SCAN_ITEMS) return false;
  pl.agg_L.clear();
  size_t m = (size_t)1 << c;
  while (m > 1) {
    size_t L = std::min<size_t>(AGG_CHUNK, m);
    pl.agg_L.push_back((uint32_t)L);
    m /= L;
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  pl.o_flags = take(4);
  pl.o_total = take(4);
  pl.o_hist = take((pl.M + 1) * 4);
  pl.o_cursor = take(pl.M * 4);
  pl.o_blocksums = take(SCAN_ITEMS * 4);
  pl.o_key = take(pl.NW * 4);
  pl.o_idx = take(pl.NW * 4);
  pl.o_head = take(pl.chunks * XYTZ_WORDS * 4);
  pl.o_tail = take(pl.chunks * XYTZ_WORDS * 4);
  pl.o_buckets = take(pl.M * XYTZ_WORDS * 4);
  // aggregation ping-pong: level 1 output holds W * 2^c / L0 (P, R) pairs
  size_t first = pl.agg_L.empty() ? 1 : ((size_t)1 << c) / pl.agg_L[0];
  pl.agg_entries = (size_t)pl.W * std::max<size_t>(first, 1);
  pl.o_agg0 = take(2 * pl.agg_entries * XYTZ_WORDS * 4);
  pl.o_agg1 = take(2 * pl.agg_entries * XYTZ_WORDS * 4);
  pl.bytes = o;
  return true;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// Steps 1-5: sort by digit and accumulate into `buckets` (M records).
int enqueue_accumulate(const Plan& pl, const uint32_t* xyu_pts, const uint32_t* scalars,
                       uint32_t* buckets, void* ws, hipStream_t st) {
  uint32_t* flags = at<uint32_t>(ws, pl.o_flags);
  uint32_t* total = at<uint32_t>(ws, pl.o_total);
  uint32_t* hist = at<uint32_t>(ws, pl.o_hist);
  uint32_t* cursor = at<uint32_t>(ws, pl.o_cursor);
  uint32_t* blocksums = at<uint32_t>(ws, pl.o_blocksums);
  uint32_t* key = at<uint32_t>(ws, pl.o_key);
  uint32_t* idx = at<uint32_t>(ws, pl.o_idx);
  uint32_t* head = at<uint32_t>(ws, pl.o_head);
  uint32_t* tail = at<uint32_t>(ws, pl.o_tail);
  const uint32_t n = (uint32_t)pl.n;

  {
  ProfScope prof(PT_SORT, st);
  k_fill_u32<<<1, 64, 0, st>>>(flags, 1, 0u);
  k_fill_u32<<<std::min<unsigned>(grid_for(pl.M + 1, 256), 4096u), 256, 0, st>>>(hist, pl.M + 1, 0u);
  k_hist<<<grid_for(n, 256), 256, 0, st>>>(scalars, n, pl.c, pl.W, hist, flags);
  k_scan_block<<<(unsigned)pl.nb, SCAN_THREADS, 0, st>>>(hist, hist, pl.M, blocksums);
  // offsets[M] = total number of (point, window) entries with a non-zero digit
  k_scan_top<<<1, SCAN_THREADS, 0, st>>>(blocksums, (uint32_t)pl.nb, total, hist + pl.M);
  k_scan_add<<<(unsigned)pl.nb, SCAN_THREADS, 0, st>>>(hist, pl.M, blocksums, cursor);
  k_scatter<<<grid_for(n, 256), 256, 0, st>>>(scalars, n, pl.c, pl.W, cursor, key, idx);
  k_fill_empty_buckets<<<grid_for(pl.M, 256), 256, 0, st>>>(hist, (uint32_t)pl.M, buckets);
  }
  {
    ProfScope prof(PT_ACCUM, st);
    k_accum<<<grid_for(pl.chunks, 256), 256, 0, st>>>(xyu_pts, key, idx, total, ACC_CHUNK, buckets,
                                                      head, tail);
  }
  ProfScope prof_merge(PT_MERGE, st);
  // tree steps: spans of up to `chunks` chunks need ceil(log2(chunks)) steps
  uint32_t steps = 0;
  while (((size_t)1 << steps) < pl.chunks) ++steps;
  for (uint32_t t = 0; t < steps; ++t)
    k_merge_step<<<grid_for(pl.chunks, 256), 256, 0, st>>>(key, hist, total, ACC_CHUNK, t, head);
  k_merge_final<<<grid_for(pl.chunks, 256), 256, 0, st>>>(key, total, ACC_CHUNK, head, tail,
                                                          buckets);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

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
  hipStream_t st = (hipStream_t)stream;
  k_fe_mul<<<grid_for(count, 256), 256, 0, st>>>(a, b, out, (uint32_t)count, canonical);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int msm_padd_batch(const uint32_t* a_xytz, const uint32_t* b, uint32_t* out_xytz, size_t count,
                   int b_form, void* stream) {
  if (!a_xytz || !b || !out_xytz || count == 0 || count >= (1u << 31)) return MSM_EINVAL;
  if (b_form != MSM_FORM_XYTZ && b_form != MSM_FORM_XYU) return MSM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (b_form == MSM_FORM_XYU)
    k_padd<MSM_FORM_XYU><<<grid_for(count, 256), 256, 0, st>>>(a_xytz, b, out_xytz, (uint32_t)count);
  else
    k_padd<MSM_FORM_XYTZ><<<grid_for(count, 256), 256, 0, st>>>(a_xytz, b, out_xytz, (uint32_t)count);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int msm_points_prepare(const uint32_t* xy_std, const uint32_t* inf, uint32_t* xyu, size_t n,
                       uint32_t* status, void* stream) {
  if (!xy_std || !xyu || !status || n == 0 || n >= (1u << 31)) return MSM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  k_prepare<<<grid_for(n, 256), 256, 0, st>>>(xy_std, inf, xyu, (uint32_t)n, status);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int msm_gen_points(const uint32_t* k, size_t n, uint32_t* xy_std, uint32_t* inf, void* stream) {
  if (!k || !xy_std || !inf || n == 0 || n >= (1u << 31)) return MSM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  k_gen_points<<<grid_for(n, 256), 256, 0, st>>>(k, xy_std, inf, (uint32_t)n);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int msm_bucket_accumulate(const uint32_t* xyu, const uint32_t* scalars, size_t n, int c,
                          uint32_t* buckets, void* ws, size_t ws_bytes, void* stream) {
  if (!xyu || !scalars || !buckets || !ws) return MSM_EINVAL;
  Plan pl;
  if (!make_plan(n, c, pl)) return MSM_EINVAL;
  if (ws_bytes < pl.bytes) return MSM_ENOSPC;
  return enqueue_accumulate(pl, xyu, scalars, buckets, ws, (hipStream_t)stream);
}

int msm_run(const uint32_t* xyu, const uint32_t* scalars, size_t n, int c, uint32_t* result,
            void* ws, size_t ws_bytes, void* stream) {
  if (!xyu || !scalars || !result || !ws) return MSM_EINVAL;
  if (c == 0) c = default_window(n);
  Plan pl;
  if (!make_plan(n, c, pl)) return MSM_EINVAL;
  if (ws_bytes < pl.bytes) return MSM_ENOSPC;
  hipStream_t st = (hipStream_t)stream;
  uint32_t* buckets = at<uint32_t>(ws, pl.o_buckets);
  int rc = enqueue_accumulate(pl, xyu, scalars, buckets, ws, st);
  if (rc != MSM_OK) return rc;
  // aggregation levels
  const uint32_t* Pin = nullptr;
  const uint32_t* Rin = buckets;
  uint32_t Min = 1u << c;
  uint32_t logmu = 0;
  uint32_t* bufs[2] = {at<uint32_t>(ws, pl.o_agg0), at<uint32_t>(ws, pl.o_agg1)};
  const uint32_t* S = nullptr;
  int which = 0;
  {
  ProfScope prof(PT_AGG, st);
  for (uint32_t L : pl.agg_L) {
    uint32_t Mout = Min / L;
    uint32_t* Pout = bufs[which];
    uint32_t* Rout = bufs[which] + pl.agg_entries * XYTZ_WORDS;
    k_agg_level<<<grid_for((size_t)pl.W * Mout, 64), 64, 0, st>>>(Pin, Rin, Min, L, logmu,
                                                                  (uint32_t)pl.W, Pout, Rout);
    Pin = Pout;
    Rin = Rout;
    Min = Mout;
    uint32_t lg = 0;
    while ((1u << lg) < L) ++lg;
    logmu += lg;
    which ^= 1;
    S = Pout;
  }
  }
  if (!S) {
    // c = 0 bits cannot happen (c >= 1 gives 2 buckets); keep the compiler quiet
    return MSM_EINVAL;
  }
  {
    ProfScope prof(PT_HORNER, st);
    k_horner<<<1, 64, 0, st>>>(S, (uint32_t)pl.W, (uint32_t)c, at<uint32_t>(ws, pl.o_flags),
                               result);
  }
  HIPCHK(hipGetLastError());
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
  for (auto& r : g_prof.recs) {
    if (r.tag != tag) {
      keep.push_back(r);
      continue;
    }
    HIPCHK(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    tot += ms;
    ++cnt;
    g_prof.pool.push_back(r.a);
    g_prof.pool.push_back(r.b);
  }
  g_prof.recs.swap(keep);
  *total_ms = tot;
  *launches = cnt;
  return MSM_OK;
}

int msm_constants(uint32_t* out, size_t words) {
  if (!out || words < 96) return MSM_EINVAL;
  const uint32_t* tabs[8] = {kP, kOne, kR2, kK, kAlpha, kBeta, kGx, kGy};
  for (int t = 0; t < 8; ++t)
    for (int l = 0; l < NL; ++l) out[t * NL + l] = tabs[t][l];
  return MSM_OK;
}

}  // extern "C"
