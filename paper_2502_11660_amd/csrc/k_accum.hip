// Bucket accumulation (Sec. II-C): B[w][b] = sum of the points whose w-th
// digit is b, with the mixed addition (bucket XYTZ + prepared XYU, Sec. II-D).
//
// The digit-sorted entry list is cut into chunks of K entries and each lane
// sums one chunk, so every lane does the same number of additions whatever
// the bucket sizes.  Inside a chunk, runs of equal key are bucket pieces:
//   * a piece that is a whole bucket is written to buckets[key];
//   * the first piece, if its bucket began in an earlier chunk, goes to
//     head[chunk] (it may also continue into later chunks);
//   * otherwise the last piece, if its bucket continues into later chunks,
//     goes to tail[chunk] (the bucket starts in this chunk).
// A split bucket starting in chunk c0 and ending in chunk c1 is then
// tail[c0] + head[c0+1] + ... + head[c1]: one lane sums it when the span
// c1 - c0 is small; longer spans are first folded by a binary tree over the
// head partials.
#include <algorithm>

#include "common.hpp"

namespace msm {
namespace {

constexpr uint32_t SMALL_SPAN = 8;

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
  const uint32_t e = (uint32_t)(s64 + K < N ? s64 + K : N);
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
    xyu Pn = ld_xyu(pts + (size_t)idx[pn] * XYU_WORDS);  // prefetch the next point
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

// chunk ch holds a tail partial: returns true and the bucket / end chunk
__device__ __forceinline__ bool tail_of(const uint32_t* __restrict__ key,
                                        const uint32_t* __restrict__ offsets, uint32_t N,
                                        uint32_t K, uint32_t ch, uint32_t& b, uint32_t& c1) {
  const uint64_t s64 = (uint64_t)ch * K;
  if (s64 >= N) return false;
  const uint32_t s = (uint32_t)s64;
  const uint32_t e = (uint32_t)(s64 + K < N ? s64 + K : N);
  const uint32_t last = key[e - 1];
  if (!(e < N && key[e] == last)) return false;        // last piece ends here
  if (s > 0 && key[s - 1] == key[s] && key[s] == last)  // whole chunk is a middle piece
    return false;
  b = last;
  c1 = (offsets[b + 1] - 1) / K;
  return true;
}

// Split buckets with span <= SMALL_SPAN: one lane sums tail + heads.
__global__ void __launch_bounds__(256) k_merge_small(const uint32_t* __restrict__ key,
                                                     const uint32_t* __restrict__ offsets,
                                                     const uint32_t* __restrict__ total,
                                                     uint32_t K, const uint32_t* __restrict__ head,
                                                     const uint32_t* __restrict__ tail,
                                                     uint32_t* __restrict__ buckets) {
  const uint32_t N = *total;
  const uint32_t ch = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t b, c1;
  if (!tail_of(key, offsets, N, K, ch, b, c1)) return;
  const uint32_t span = c1 - ch;
  if (span > SMALL_SPAN) return;
  const fe p2 = fe_const(kP2);
  xytz acc = ld_xytz(tail + (size_t)ch * XYTZ_WORDS);
  for (uint32_t j = 1; j <= span; ++j)
    acc = padd_full(acc, ld_xytz(head + (size_t)(ch + j) * XYTZ_WORDS), p2);
  st_xytz(buckets + (size_t)b * XYTZ_WORDS, acc);
}

// Tree step t for buckets spanning more than SMALL_SPAN chunks: chunk c of
// such a bucket (c0 < c <= c1, its first piece continues the bucket) with
// (c - c0 - 1) % 2^(t+1) == 0 adds head[c + 2^t] if that chunk still belongs
// to the bucket.  Grid-stride over the chunks; exits at once when no bucket
// is long.
__global__ void __launch_bounds__(256) k_merge_step(const uint32_t* __restrict__ key,
                                                    const uint32_t* __restrict__ offsets,
                                                    const uint32_t* __restrict__ total,
                                                    const uint32_t* __restrict__ maxspan,
                                                    uint32_t K, uint32_t t,
                                                    uint32_t* __restrict__ head) {
  const uint32_t ms = *maxspan;
  if (ms <= SMALL_SPAN || (1u << t) >= ms) return;
  const uint32_t N = *total;
  const uint32_t nchunks = (N + K - 1) / K;
  const fe p2 = fe_const(kP2);
  for (uint32_t ch = blockIdx.x * blockDim.x + threadIdx.x; ch < nchunks;
       ch += gridDim.x * blockDim.x) {
    if (ch == 0) continue;
    const uint32_t s = ch * K;
    const uint32_t b = key[s];
    if (key[s - 1] != b) continue;
    const uint32_t c0 = offsets[b] / K;
    const uint32_t c1 = (offsets[b + 1] - 1) / K;
    if (c1 - c0 <= SMALL_SPAN) continue;
    const uint32_t rel = ch - c0 - 1;
    const uint32_t stride = 1u << t;
    if ((rel & ((stride << 1) - 1)) != 0 || ch + stride > c1) continue;
    uint32_t* mine = head + (size_t)ch * XYTZ_WORDS;
    st_xytz(mine, padd_full(ld_xytz(mine), ld_xytz(head + (size_t)(ch + stride) * XYTZ_WORDS), p2));
  }
}

// Long split buckets after the tree: bucket = tail[c0] + head[c0 + 1].
__global__ void __launch_bounds__(256) k_merge_long(const uint32_t* __restrict__ key,
                                                    const uint32_t* __restrict__ offsets,
                                                    const uint32_t* __restrict__ total,
                                                    const uint32_t* __restrict__ maxspan,
                                                    uint32_t K, const uint32_t* __restrict__ head,
                                                    const uint32_t* __restrict__ tail,
                                                    uint32_t* __restrict__ buckets) {
  if (*maxspan <= SMALL_SPAN) return;
  const uint32_t N = *total;
  const uint32_t nchunks = (N + K - 1) / K;
  const fe p2 = fe_const(kP2);
  for (uint32_t ch = blockIdx.x * blockDim.x + threadIdx.x; ch < nchunks;
       ch += gridDim.x * blockDim.x) {
    uint32_t b, c1;
    if (!tail_of(key, offsets, N, K, ch, b, c1) || c1 - ch <= SMALL_SPAN) continue;
    xytz a = ld_xytz(tail + (size_t)ch * XYTZ_WORDS);
    xytz o = ld_xytz(head + (size_t)(ch + 1) * XYTZ_WORDS);
    st_xytz(buckets + (size_t)b * XYTZ_WORDS, padd_full(a, o, p2));
  }
}

}  // namespace

int launch_accumulate(const Plan& pl, const uint32_t* xyu, uint32_t* buckets, void* ws,
                      hipStream_t st) {
  const uint32_t* total = ws_at<uint32_t>(ws, pl.o_total);
  const uint32_t* maxspan = ws_at<uint32_t>(ws, pl.o_maxspan);
  const uint32_t* offsets = ws_at<uint32_t>(ws, pl.o_hist);
  const uint32_t* key = ws_at<uint32_t>(ws, pl.o_key);
  const uint32_t* idx = ws_at<uint32_t>(ws, pl.o_idx);
  uint32_t* head = ws_at<uint32_t>(ws, pl.o_head);
  uint32_t* tail = ws_at<uint32_t>(ws, pl.o_tail);
  const uint32_t K = pl.K;
  {
    ProfScope prof(PT_ACCUM, st);
    k_accum<<<grid_for(pl.chunks, 256), 256, 0, st>>>(xyu, key, idx, total, K, buckets, head, tail);
  }
  ProfScope prof(PT_MERGE, st);
  k_merge_small<<<grid_for(pl.chunks, 256), 256, 0, st>>>(key, offsets, total, K, head, tail,
                                                          buckets);
  // a bucket holds at most n entries, so its span is at most ceil(n/K) chunks
  const size_t max_span = (pl.n + K - 1) / K + 1;
  if (max_span > SMALL_SPAN) {
    // these launches return at once unless some bucket spans > SMALL_SPAN chunks
    const unsigned g = std::min<unsigned>(grid_for(pl.chunks, 256), 64u);
    uint32_t steps = 0;
    while (((size_t)1 << steps) < max_span) ++steps;
    for (uint32_t t = 0; t < steps; ++t)
      k_merge_step<<<g, 256, 0, st>>>(key, offsets, total, maxspan, K, t, head);
    k_merge_long<<<g, 256, 0, st>>>(key, offsets, total, maxspan, K, head, tail, buckets);
  }
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // namespace msm
