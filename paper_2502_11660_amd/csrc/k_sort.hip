// Scalar slicing and digit sort (Sec. II-C: points are assigned to buckets by
// their sliced scalar values).
//
// The entries are the (segment, point) pairs with a non-zero digit, where a
// segment is one window of one MSM.  Their key is seg * 2^c + digit; the sort
// produces, over all M = segments * 2^c buckets:
//   offsets[0..M]  CSR offsets of each bucket's entries (offsets[M] = total),
//   key[], idx[]   the entries in bucket order (idx = point index in its MSM),
// writes the identity into every empty bucket and the largest bucket span
// (in accumulation chunks) into *maxspan.
//
// It is a two-pass most-significant-digit counting sort with no global
// atomics:
//   slice   digits of every window, stored window-major (coalesced);
//   pass 1  per tile of one segment, an LDS histogram of the digit's high
//           bits; the (partition, tile) count matrix is scanned, and each tile
//           scatters its entries to (partition, tile) ranges through LDS
//           cursors;
//   pass 2  one block per partition (segment, high bits) counts the low
//           <= 8 bits in LDS, writes the bucket offsets, and places the
//           entries in bucket order.  Partitions up to PART_CAP entries are
//           staged in LDS; larger ones (skewed inputs) are streamed twice.
#include <algorithm>

#include "common.hpp"
#include "convert.hpp"

namespace msm {
namespace {

constexpr int SORT_THREADS = 256;
constexpr uint32_t TILE = 4096;      // entries per pass-1 tile
constexpr uint32_t PART_CAP = 8192;  // entries staged in LDS by pass 2

struct SortGeom {
  uint32_t S;         // segments
  uint32_t n;         // entries per segment (points of the MSM)
  uint32_t Tps;       // tiles per segment
  uint32_t c, lo_bits, hi_bits;
};

__device__ __forceinline__ uint32_t count_index(const SortGeom& g, uint32_t s, uint32_t hi,
                                                uint32_t tile) {
  return (s * (1u << g.hi_bits) + hi) * g.Tps + tile;
}

// digits[w * n + i] = w-th c-bit digit of scalar i (bits >= 253 flagged, ignored)
__global__ void __launch_bounds__(256) k_slice(const uint32_t* __restrict__ scalars, uint32_t n,
                                               int c, int W, uint32_t* __restrict__ digits,
                                               uint32_t* __restrict__ flags) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  scalar256 s = ld_scalar(scalars, i, flags);
  for (int w = 0; w < W; ++w) digits[(size_t)w * n + i] = digit_at(s, w * c, c);
}

// pass 1a: per-tile histogram of the high bits
__global__ void __launch_bounds__(SORT_THREADS) k_part_count(SortGeom g,
                                                             const uint32_t* __restrict__ digits,
                                                             uint32_t* __restrict__ counts) {
  __shared__ uint32_t hist[1u << 12];
  const uint32_t s = blockIdx.x / g.Tps, tile = blockIdx.x % g.Tps;
  const uint32_t H = 1u << g.hi_bits;
  for (uint32_t b = threadIdx.x; b < H; b += SORT_THREADS) hist[b] = 0;
  __syncthreads();
  const uint32_t e0 = tile * TILE, e1 = min(e0 + TILE, g.n);
  const uint32_t* dg = digits + (size_t)s * g.n;
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += SORT_THREADS) {
    uint32_t d = dg[e];
    if (d) atomicAdd(&hist[d >> g.lo_bits], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < H; b += SORT_THREADS)
    counts[count_index(g, s, b, tile)] = hist[b];
}

// pass 1b: scatter into (partition, tile) ranges; tmp entry = {idx, key}
__global__ void __launch_bounds__(SORT_THREADS) k_part_scatter(SortGeom g,
                                                               const uint32_t* __restrict__ digits,
                                                               const uint32_t* __restrict__ scanned,
                                                               uint2* __restrict__ tmp) {
  __shared__ uint32_t cur[1u << 12];
  const uint32_t s = blockIdx.x / g.Tps, tile = blockIdx.x % g.Tps;
  const uint32_t H = 1u << g.hi_bits;
  for (uint32_t b = threadIdx.x; b < H; b += SORT_THREADS) cur[b] = scanned[count_index(g, s, b, tile)];
  __syncthreads();
  const uint32_t e0 = tile * TILE, e1 = min(e0 + TILE, g.n);
  const uint32_t* dg = digits + (size_t)s * g.n;
  const uint32_t keybase = s << g.c;
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += SORT_THREADS) {
    uint32_t d = dg[e];
    if (d) {
      uint32_t pos = atomicAdd(&cur[d >> g.lo_bits], 1u);
      tmp[pos] = make_uint2(e, keybase + d);
    }
  }
}

// block-wide exclusive scan of the first L (<= 256) entries of v, in place;
// all SORT_THREADS threads must call it
__device__ void lds_exclusive_scan256(uint32_t* v, uint32_t L) {
  __shared__ uint32_t t[SORT_THREADS];
  const uint32_t i = threadIdx.x;
  uint32_t x = (i < L) ? v[i] : 0u;
  t[i] = x;
  __syncthreads();
  for (uint32_t d = 1; d < SORT_THREADS; d <<= 1) {
    uint32_t y = (i >= d) ? t[i - d] : 0u;
    __syncthreads();
    t[i] += y;
    __syncthreads();
  }
  if (i < L) v[i] = t[i] - x;
  __syncthreads();
}

// pass 2: one block per partition (segment s, high bits hi)
__global__ void __launch_bounds__(SORT_THREADS) k_part_sort(
    SortGeom g, const uint32_t* __restrict__ scanned, const uint32_t* __restrict__ total_p,
    const uint2* __restrict__ tmp, uint32_t K, uint32_t* __restrict__ key, uint32_t* __restrict__ idx,
    uint32_t* __restrict__ offsets, uint32_t* __restrict__ buckets, uint32_t* __restrict__ maxspan) {
  __shared__ uint2 ent[PART_CAP];
  __shared__ uint32_t hist[256], cur[256];
  __shared__ uint32_t bmax;
  const uint32_t H = 1u << g.hi_bits, L = 1u << g.lo_bits;
  const uint32_t p = blockIdx.x, s = p / H, hi = p % H;
  const uint32_t total = *total_p;
  const uint32_t start = scanned[count_index(g, s, hi, 0)];
  const uint32_t end = (p + 1 < g.S * H) ? scanned[count_index(g, (p + 1) / H, (p + 1) % H, 0)] : total;
  const uint32_t size = end - start;
  const bool staged = size <= PART_CAP;
  if (threadIdx.x < 256) hist[threadIdx.x] = 0;
  if (threadIdx.x == 0) bmax = 0;
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < size; j += SORT_THREADS) {
    uint2 e = tmp[start + j];
    if (staged) ent[j] = e;
    atomicAdd(&hist[e.y & (L - 1)], 1u);
  }
  __syncthreads();
  for (uint32_t lo = threadIdx.x; lo < L; lo += SORT_THREADS) cur[lo] = hist[lo];
  __syncthreads();
  lds_exclusive_scan256(cur, L);  // cur[lo] = local start of bucket lo
  const uint32_t bucket0 = (s << g.c) + hi * L;
  if (threadIdx.x < L) {
    const uint32_t lo = threadIdx.x, cnt = hist[lo], o = start + cur[lo];
    offsets[bucket0 + lo] = o;
    if (cnt == 0) {
      if (buckets) st_xytz(buckets + (size_t)(bucket0 + lo) * XYTZ_WORDS, pt_identity());
    } else {
      atomicMax(&bmax, (o + cnt - 1) / K - o / K);
    }
  }
  if (p == 0 && threadIdx.x == 0) offsets[g.S << g.c] = total;
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < size; j += SORT_THREADS) {
    uint2 e = staged ? ent[j] : tmp[start + j];
    uint32_t pos = start + atomicAdd(&cur[e.y & (L - 1)], 1u);
    key[pos] = e.y;
    idx[pos] = e.x;
  }
  if (threadIdx.x == 0 && bmax) atomicMax(maxspan, bmax);
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

// one block: exclusive scan of nb <= SCAN_ITEMS block sums; grand total out
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_top(uint32_t* __restrict__ blocksums,
                                                           uint32_t nb,
                                                           uint32_t* __restrict__ total_out) {
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
  if (threadIdx.x == 0) *total_out = total;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_add(uint32_t* __restrict__ data, size_t n,
                                                           const uint32_t* __restrict__ blocksums) {
  size_t base = (size_t)blockIdx.x * SCAN_ITEMS;
  uint32_t add = blocksums[blockIdx.x];
  for (int j = threadIdx.x; j < SCAN_ITEMS; j += SCAN_THREADS) {
    size_t i = base + j;
    if (i < n) data[i] += add;
  }
}

// Split of the c digit bits: enough high bits that a partition of uniformly
// distributed digits holds about n / 2^hi <= PART_CAP / 2 entries, at most 8
// low bits (pass-2 histogram) and at most 12 high bits (pass-1 histogram).
void split_bits(uint32_t c, size_t n, uint32_t& lo, uint32_t& hi) {
  uint32_t want = 0;
  while (want < 12 && (n >> want) > PART_CAP / 2) ++want;
  hi = std::max<uint32_t>(want, c > 8 ? c - 8 : 0);
  hi = std::min<uint32_t>(hi, std::min<uint32_t>(c, 12));
  lo = c - hi;
}

}  // namespace

size_t sort_counts_size(int c, int W, size_t n) {
  uint32_t lo, hi;
  split_bits((uint32_t)c, n, lo, hi);
  if (lo > 8) return (size_t)-1;
  const size_t Tps = (n + TILE - 1) / TILE;
  return (size_t)W * ((size_t)1 << hi) * Tps;
}

int launch_sort(const Plan& pl, const uint32_t* scalars, uint32_t* buckets, void* ws,
                hipStream_t st) {
  uint32_t* flags = ws_at<uint32_t>(ws, pl.o_flags);
  uint32_t* total = ws_at<uint32_t>(ws, pl.o_total);
  uint32_t* maxspan = ws_at<uint32_t>(ws, pl.o_maxspan);
  uint32_t* offsets = ws_at<uint32_t>(ws, pl.o_hist);
  uint32_t* counts = ws_at<uint32_t>(ws, pl.o_counts);
  uint32_t* blocksums = ws_at<uint32_t>(ws, pl.o_blocksums);
  uint32_t* digits = ws_at<uint32_t>(ws, pl.o_digits);
  uint2* tmp = ws_at<uint2>(ws, pl.o_tmp);
  uint32_t* key = ws_at<uint32_t>(ws, pl.o_key);
  uint32_t* idx = ws_at<uint32_t>(ws, pl.o_idx);
  const uint32_t n = (uint32_t)pl.n;

  SortGeom g;
  g.S = (uint32_t)pl.W;
  g.n = n;
  g.Tps = (n + TILE - 1) / TILE;
  g.c = (uint32_t)pl.c;
  split_bits(g.c, n, g.lo_bits, g.hi_bits);
  const size_t ncounts = (size_t)g.S * ((size_t)1 << g.hi_bits) * g.Tps;
  const size_t nb = (ncounts + SCAN_ITEMS - 1) / SCAN_ITEMS;
  if (nb > (size_t)SCAN_ITEMS || ncounts != pl.ncounts) return MSM_EINVAL;

  int rc;
  if ((rc = launch_fill_u32(flags, 1, 0u, st)) != MSM_OK) return rc;
  if ((rc = launch_fill_u32(maxspan, 1, 0u, st)) != MSM_OK) return rc;
  k_slice<<<grid_for(n, 256), 256, 0, st>>>(scalars, n, pl.c, pl.W, digits, flags);
  k_part_count<<<g.S * g.Tps, SORT_THREADS, 0, st>>>(g, digits, counts);
  k_scan_block<<<(unsigned)nb, SCAN_THREADS, 0, st>>>(counts, ncounts, blocksums);
  k_scan_top<<<1, SCAN_THREADS, 0, st>>>(blocksums, (uint32_t)nb, total);
  k_scan_add<<<(unsigned)nb, SCAN_THREADS, 0, st>>>(counts, ncounts, blocksums);
  k_part_scatter<<<g.S * g.Tps, SORT_THREADS, 0, st>>>(g, digits, counts, tmp);
  k_part_sort<<<g.S << g.hi_bits, SORT_THREADS, 0, st>>>(g, counts, total, tmp, pl.K, key, idx,
                                                          offsets, buckets, maxspan);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // namespace msm
