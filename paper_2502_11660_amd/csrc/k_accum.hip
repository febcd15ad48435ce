// Bucket accumulation (Sec. II-C): every bucket receives the sum of its
// entries' points (negated for negative signed digits), with the mixed
// addition (bucket XYTZ + prepared XYU, Sec. II-D).
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
#include <hip/hip_ext.h>

#include <algorithm>

#include "common.hpp"
#include "curve28.hpp"

namespace msm {
namespace {

constexpr uint32_t SMALL_SPAN = 8;

// Chunk ch covers entries [ch K, min((ch+1) K, E)), E = offsets[M].  The
// entry's index word is the point index in its job with the digit's sign in
// bit 31; segoff[s] is the word offset of segment s's point array from pts
// (NULL: one job, points at pts).  Addressing from the kernel argument keeps
// the point loads global (not flat) memory instructions.

__device__ __forceinline__ const uint32_t* entry_point(const uint32_t* __restrict__ pts,
                                                       const int64_t* __restrict__ segoff,
                                                       uint32_t bb, uint32_t k, uint32_t e) {
  const int64_t off = segoff ? segoff[k >> bb] : 0;
  return pts + off + (int64_t)(e & 0x7fffffffu) * XYU_WORDS;
}

// Chunk ch of the sorted entries: the first X chunks hold K + 4 entries, the
// rest K (both multiples of 4).
__device__ __forceinline__ uint64_t chunk_start(uint32_t ch, uint32_t K, uint32_t X) {
  return (uint64_t)ch * K + 4ull * (ch < X ? ch : X);
}

// the chunk holding entry e
__device__ __forceinline__ uint32_t chunk_of(uint32_t e, uint32_t K, uint32_t X) {
  const uint64_t longer = (uint64_t)X * (K + 4);
  return e < longer ? (uint32_t)(e / (K + 4)) : X + (uint32_t)((e - longer) / K);
}

// One lane per chunk, on the carry-free 28-bit field form (curve28.hpp):
// points are converted from their 12-word records as they are loaded, the
// running sum stays in the 28-bit form and is converted back when it is
// stored.  (Measured against the 12-word form: 2.16 vs 2.30 ms at n = 2^20.
// Four waves per SIMD, reachable without spills when the addition forms C
// and D first, measured no faster than three.  Reading keys and indices in
// groups of four cut the kernel's HBM reads by 31% at the same time.)
__global__ void __launch_bounds__(256) k_accum(const uint32_t* __restrict__ pts,
                                                 const int64_t* __restrict__ segoff, uint32_t bb,
                                                 const uint32_t* __restrict__ key,
                                                 const uint32_t* __restrict__ idx,
                                                 const uint32_t* __restrict__ offsets, uint32_t M,
                                                 uint32_t K, uint32_t X,
                                                 uint32_t* __restrict__ buckets,
                                                 uint32_t* __restrict__ head,
                                                 uint32_t* __restrict__ tail) {
  const uint32_t E1 = offsets[M];
  const uint32_t ch = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t s64 = chunk_start(ch, K, X);
  if (s64 >= E1) return;
  const uint32_t s = (uint32_t)s64;
  const uint64_t e64 = s64 + K + (ch < X ? 4u : 0u);
  const uint32_t e = (uint32_t)(e64 < E1 ? e64 : E1);

  uint32_t cur = key[s];
  const bool open_left = (s > 0) && (key[s - 1] == cur);
  bool first_seg = true;
  xytz28 acc = pt28_identity();
  // Keys and indices are read four at a time with 16-byte loads (chunk
  // lengths are multiples of 4, so a chunk starts on a 16-byte boundary; the arrays carry
  // 32 bytes of padding for a last group that ends past E1).  A lane's
  // 128-byte line of keys would otherwise be fetched again for every entry:
  // the point gathers of all resident waves evict it between iterations.
  // The next group is loaded two entries ahead, while the current one's
  // last entry waits in (k3, i3).
  uint4 kq = *reinterpret_cast<const uint4*>(key + s);
  uint4 iq = *reinterpret_cast<const uint4*>(idx + s);
  uint32_t k3 = 0, i3 = 0;
  for (uint32_t i = 0; s + i < e; ++i) {
    const uint32_t r = i & 3u;
    uint32_t k, ie;
    if (r == 0) {
      k = kq.x;
      ie = iq.x;
    } else if (r == 1) {
      k = kq.y;
      ie = iq.y;
    } else if (r == 2) {
      k = kq.z;
      ie = iq.z;
      k3 = kq.w;
      i3 = iq.w;
      const uint32_t q = s + i + 2;  // the next group (in the padded arrays)
      kq = *reinterpret_cast<const uint4*>(key + q);
      iq = *reinterpret_cast<const uint4*>(idx + q);
    } else {
      k = k3;
      ie = i3;
    }
    if (k != cur) {
      uint32_t* dst = (first_seg && open_left) ? head + (size_t)ch * XYTZ_WORDS
                                               : buckets + (size_t)cur * XYTZ_WORDS;
      st_xytz(dst, pt28_to_words(acc));
      acc = pt28_identity();
      cur = k;
      first_seg = false;
    }
    const xyu28 P = pt28_from(ld_xyu(entry_point(pts, segoff, bb, k, ie)));
    acc = padd28_mixed_signed(acc, P, (ie >> 31) != 0u);
  }
  const bool open_right = (e < E1) && (key[e] == cur);
  uint32_t* dst;
  if (first_seg && open_left)
    dst = head + (size_t)ch * XYTZ_WORDS;
  else if (open_right)
    dst = tail + (size_t)ch * XYTZ_WORDS;
  else
    dst = buckets + (size_t)cur * XYTZ_WORDS;
  st_xytz(dst, pt28_to_words(acc));
}

// chunk ch holds a tail partial: returns true, the bucket and its last chunk
__device__ __forceinline__ bool tail_of(const uint32_t* __restrict__ key,
                                        const uint32_t* __restrict__ offsets, uint32_t E1,
                                        uint32_t K, uint32_t X, uint32_t ch, uint32_t& b,
                                        uint32_t& c1) {
  const uint64_t s64 = chunk_start(ch, K, X);
  if (s64 >= E1) return false;
  const uint32_t s = (uint32_t)s64;
  const uint64_t e64 = s64 + K + (ch < X ? 4u : 0u);
  const uint32_t e = (uint32_t)(e64 < E1 ? e64 : E1);
  const uint32_t last = key[e - 1];
  if (!(e < E1 && key[e] == last)) return false;          // last piece ends here
  if (s > 0 && key[s - 1] == key[s] && key[s] == last)     // whole chunk is a middle piece
    return false;
  b = last;
  c1 = chunk_of(offsets[b + 1] - 1, K, X);
  return true;
}

// Split buckets: one lane sums tail + heads when the span is at most
// SMALL_SPAN chunks; longer spans (skewed inputs) are appended to a work list
// for k_merge_long.  The block's tasks are packed in LDS first (span 1 at
// the front, longer spans at the back), so that a wave runs one kind and
// wholly idle waves leave at once.
__global__ void __launch_bounds__(256) k_merge_small(const uint32_t* __restrict__ key,
                                                     const uint32_t* __restrict__ offsets,
                                                     uint32_t M, uint32_t K, uint32_t X,
                                                     const uint32_t* __restrict__ head,
                                                     const uint32_t* __restrict__ tail,
                                                     uint32_t* __restrict__ buckets,
                                                     uint32_t* __restrict__ longlist) {
  __shared__ uint32_t task[256];
  __shared__ uint32_t cnt[2];
  const uint32_t tid = threadIdx.x;
  if (tid < 2) cnt[tid] = 0;
  __syncthreads();
  const uint32_t E1 = offsets[M];
  const uint32_t ch = blockIdx.x * blockDim.x + tid;
  uint32_t b = 0, c1 = 0;
  const bool has = tail_of(key, offsets, E1, K, X, ch, b, c1);
  const uint32_t span = has ? c1 - ch : 0u;
  if (has && span > SMALL_SPAN) {
    const uint32_t slot = atomicAdd(&longlist[0], 1u);
    longlist[1 + slot] = ch;
  } else if (has && span == 1) {
    task[atomicAdd(&cnt[0], 1u)] = ch;
  } else if (has) {
    task[255 - atomicAdd(&cnt[1], 1u)] = ch;
  }
  __syncthreads();
  const uint32_t n1 = cnt[0], n2 = cnt[1];
  if (!(tid < n1 || tid >= 256 - n2)) return;
  const uint32_t c = task[tid];
  // the tail's bucket ends after chunk c
  const uint32_t bk = key[(uint32_t)chunk_start(c + 1, K, X) - 1];
  const uint32_t sp = chunk_of(offsets[bk + 1] - 1, K, X) - c;
  xytz28 acc = pt28_from(ld_xytz(tail + (size_t)c * XYTZ_WORDS));
  for (uint32_t j = 1; j <= sp; ++j)
    acc = padd28_full(acc, pt28_from(ld_xytz(head + (size_t)(c + j) * XYTZ_WORDS)));
  st_xytz(buckets + (size_t)bk * XYTZ_WORDS, pt28_to_words(acc));
}

// Long split buckets, one block each: the block's threads sum strided heads
// of the span, then fold their partial sums pairwise through LDS (as many
// levels as the span needs), and thread 0 adds the tail.  The grid holds a
// block for every possible list entry (a long span covers more than
// SMALL_SPAN chunks of its own, so there are at most chunks / SMALL_SPAN, and
// up to 2048 blocks), so the entries run side by side; blocks past the list's
// count leave at once.
constexpr int LONG_THREADS = 128;
__global__ void __launch_bounds__(LONG_THREADS) k_merge_long(const uint32_t* __restrict__ key,
                                                             const uint32_t* __restrict__ offsets,
                                                             uint32_t K, uint32_t X,
                                                             const uint32_t* __restrict__ head,
                                                             const uint32_t* __restrict__ tail,
                                                             uint32_t* __restrict__ buckets,
                                                             const uint32_t* __restrict__ longlist) {
  __shared__ uint32_t part[LONG_THREADS][XYTZ_WORDS];
  const uint32_t count = longlist[0];
  for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
    const uint32_t ch = longlist[1 + item];
    // the tail's bucket ends after this chunk
    const uint32_t e_last = (uint32_t)chunk_start(ch + 1, K, X) - 1;
    const uint32_t b = key[e_last];
    const uint32_t c1 = chunk_of(offsets[b + 1] - 1, K, X);
    const uint32_t span = c1 - ch;
    const uint32_t nact = span < (uint32_t)LONG_THREADS ? span : (uint32_t)LONG_THREADS;
    if (threadIdx.x < nact) {
      xytz28 acc = pt28_identity();
      for (uint32_t j = ch + 1 + threadIdx.x; j <= c1; j += LONG_THREADS)
        acc = padd28_full(acc, pt28_from(ld_xytz(head + (size_t)j * XYTZ_WORDS)));
      st_xytz(part[threadIdx.x], pt28_to_words(acc));
    }
    __syncthreads();
    // fold partials [0, n) into [0, ceil(n / 2)) until one is left
    for (uint32_t n = nact; n > 1;) {
      const uint32_t half = (n + 1) >> 1;
      if (threadIdx.x + half < n) {
        const xytz28 a = pt28_from(ld_xytz(part[threadIdx.x]));
        const xytz28 o = pt28_from(ld_xytz(part[threadIdx.x + half]));
        st_xytz(part[threadIdx.x], pt28_to_words(padd28_full(a, o)));
      }
      __syncthreads();
      n = half;
    }
    if (threadIdx.x == 0) {
      const xytz28 t = pt28_from(ld_xytz(tail + (size_t)ch * XYTZ_WORDS));
      st_xytz(buckets + (size_t)b * XYTZ_WORDS,
              pt28_to_words(padd28_full(t, pt28_from(ld_xytz(part[0])))));
    }
    __syncthreads();
  }
}

}  // namespace

int launch_accumulate(const Plan& pl, uint32_t* buckets, void* ws, hipStream_t st) {
  const uint32_t* offsets = ws_at<uint32_t>(ws, pl.o_offsets);
  const uint32_t* key = ws_at<uint32_t>(ws, pl.o_key);
  const uint32_t* idx = ws_at<uint32_t>(ws, pl.o_idx);
  uint32_t* head = ws_at<uint32_t>(ws, pl.o_head);
  uint32_t* tail = ws_at<uint32_t>(ws, pl.o_tail);
  uint32_t* longlist = ws_at<uint32_t>(ws, pl.o_longlist);
  const int64_t* segoff = pl.J == 1 ? nullptr : ws_at<const int64_t>(ws, pl.o_segoff);
  const uint32_t K = pl.K, X = pl.Kx, M = (uint32_t)pl.M;
  const unsigned grid = grid_for(pl.chunks, 256);
  // longlist[0] was cleared by the digit sort's scatter pass
  hipEvent_t ea = nullptr, eb = nullptr;
  if (prof_kernel_events(PT_ACCUM, st, &ea, &eb)) {
    // timed by events attached to the dispatch itself
    hipExtLaunchKernelGGL(k_accum, dim3(grid), dim3(256), 0, st, ea, eb, 0, pl.one.xyu, segoff,
                          (uint32_t)pl.bb, key, idx, offsets, M, K, X, buckets, head, tail);
    prof_kernel_record(PT_ACCUM, ea, eb);
  } else {
    ProfScope prof(PT_ACCUM, st);
    k_accum<<<grid, 256, 0, st>>>(pl.one.xyu, segoff, (uint32_t)pl.bb, key, idx, offsets, M, K,
                                  X, buckets, head, tail);
  }
  ProfScope prof(PT_MERGE, st);
  k_merge_small<<<grid, 256, 0, st>>>(key, offsets, M, K, X, head, tail, buckets, longlist);
  // a block per possible entry (at most chunks / SMALL_SPAN), capped: the
  // common empty list then costs one short wave per block
  const unsigned long_grid =
      (unsigned)std::min<size_t>(2048, std::max<size_t>(1, pl.chunks / SMALL_SPAN));
  k_merge_long<<<long_grid, LONG_THREADS, 0, st>>>(key, offsets, K, X, head, tail, buckets,
                                                    longlist);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // namespace msm
