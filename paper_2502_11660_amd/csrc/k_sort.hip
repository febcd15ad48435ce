// Scalar slicing and digit sort (Sec. II-C: points are assigned to buckets by
// their sliced scalar values).  Produces, over the keys w*2^c + d of all
// windows w and non-zero digits d:
//   offsets[0..M]  CSR offsets of each bucket's entries (offsets[M] = total),
//   key[], idx[]   the (bucket, point) entries in bucket order.
#include "common.hpp"
#include "convert.hpp"

namespace msm {
namespace {

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

// Exclusive scan in three passes, SCAN_ITEMS elements per block.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_ITEMS = SCAN_THREADS * SCAN_PER_THREAD;

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

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_block(uint32_t* __restrict__ data, size_t n,
                                                             uint32_t* __restrict__ blocksums) {
  size_t base = (size_t)blockIdx.x * SCAN_ITEMS + (size_t)threadIdx.x * SCAN_PER_THREAD;
  uint32_t v[SCAN_PER_THREAD];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) {
    v[j] = (base + j < n) ? data[base + j] : 0u;
    sum += v[j];
  }
  uint32_t excl;
  uint32_t total = block_exclusive_scan(sum, excl);
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) {
    if (base + j < n) data[base + j] = excl;
    excl += v[j];
  }
  if (threadIdx.x == 0) blocksums[blockIdx.x] = total;
}

// one block: exclusive scan of nb <= SCAN_ITEMS block sums; the grand total
// goes to both total outputs
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_top(uint32_t* __restrict__ blocksums,
                                                           uint32_t nb,
                                                           uint32_t* __restrict__ total_a,
                                                           uint32_t* __restrict__ total_b) {
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
    *total_a = total;
    *total_b = total;
  }
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_add(uint32_t* __restrict__ data, size_t n,
                                                           const uint32_t* __restrict__ blocksums,
                                                           uint32_t* __restrict__ copy) {
  size_t base = (size_t)blockIdx.x * SCAN_ITEMS;
  uint32_t add = blocksums[blockIdx.x];
  for (int j = threadIdx.x; j < SCAN_ITEMS; j += SCAN_THREADS) {
    size_t i = base + j;
    if (i < n) {
      uint32_t v = data[i] + add;
      data[i] = v;
      copy[i] = v;
    }
  }
}

// Empty buckets get the identity; non-empty ones report how many chunk
// boundaries they cross (their span) to the per-MSM maximum.
__global__ void __launch_bounds__(256) k_fill_empty(const uint32_t* __restrict__ offsets,
                                                    uint32_t M, uint32_t K,
                                                    uint32_t* __restrict__ buckets,
                                                    uint32_t* __restrict__ maxspan) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t span = 0;
  if (b < M) {
    uint32_t o0 = offsets[b], o1 = offsets[b + 1];
    if (o0 == o1)
      st_xytz(buckets + (size_t)b * XYTZ_WORDS, pt_identity());
    else
      span = (o1 - 1) / K - o0 / K;
  }
  // wave maximum, then one atomic per wave
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    uint32_t o = __shfl_xor(span, d, 64);
    span = span > o ? span : o;
  }
  if ((threadIdx.x & 63) == 0 && span) atomicMax(maxspan, span);
}

}  // namespace

int launch_sort(const Plan& pl, const uint32_t* scalars, uint32_t* buckets, void* ws,
                hipStream_t st) {
  uint32_t* flags = ws_at<uint32_t>(ws, pl.o_flags);
  uint32_t* total = ws_at<uint32_t>(ws, pl.o_total);
  uint32_t* maxspan = ws_at<uint32_t>(ws, pl.o_maxspan);
  uint32_t* hist = ws_at<uint32_t>(ws, pl.o_hist);
  uint32_t* cursor = ws_at<uint32_t>(ws, pl.o_cursor);
  uint32_t* blocksums = ws_at<uint32_t>(ws, pl.o_blocksums);
  uint32_t* key = ws_at<uint32_t>(ws, pl.o_key);
  uint32_t* idx = ws_at<uint32_t>(ws, pl.o_idx);
  const uint32_t n = (uint32_t)pl.n;
  if (pl.nb > (size_t)SCAN_ITEMS) return MSM_EINVAL;

  int rc;
  if ((rc = launch_fill_u32(flags, 1, 0u, st)) != MSM_OK) return rc;
  if ((rc = launch_fill_u32(maxspan, 1, 0u, st)) != MSM_OK) return rc;
  if ((rc = launch_fill_u32(hist, pl.M + 1, 0u, st)) != MSM_OK) return rc;
  k_hist<<<grid_for(n, 256), 256, 0, st>>>(scalars, n, pl.c, pl.W, hist, flags);
  k_scan_block<<<(unsigned)pl.nb, SCAN_THREADS, 0, st>>>(hist, pl.M, blocksums);
  // offsets[M] = number of (point, window) entries with a non-zero digit
  k_scan_top<<<1, SCAN_THREADS, 0, st>>>(blocksums, (uint32_t)pl.nb, total, hist + pl.M);
  k_scan_add<<<(unsigned)pl.nb, SCAN_THREADS, 0, st>>>(hist, pl.M, blocksums, cursor);
  k_scatter<<<grid_for(n, 256), 256, 0, st>>>(scalars, n, pl.c, pl.W, cursor, key, idx);
  k_fill_empty<<<grid_for(pl.M, 256), 256, 0, st>>>(hist, (uint32_t)pl.M, pl.K, buckets, maxspan);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // namespace msm
