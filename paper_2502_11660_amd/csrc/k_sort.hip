// Scalar slicing and digit sort (Sec. II-C: points are assigned to buckets by
// their sliced scalar values).
//
// The entries are the (segment, point) pairs with a non-zero digit, where a
// segment is one window of one job.  An entry's key is s * 2^bb + m (segment
// s, bucket m of bb bits) and its index word is the point's index in its job
// with the digit's sign in bit 31.  Over all M = segments * 2^bb buckets the
// sort produces
//   offsets[0..M]  CSR offsets of each bucket's entries (offsets[M] = total),
//   key[], idx[]   the entries in bucket order,
// and writes the identity into every empty bucket.
//
// It is a two-pass most-significant-digit counting sort with no global
// atomics:
//   slice   digits of every window, stored segment-major (coalesced);
//   pass 1  per tile of one segment, an LDS histogram of the bucket index's
//           high bits; the (partition, tile) count matrix is scanned, and each
//           tile scatters its entries to (partition, tile) ranges through LDS
//           cursors;
//   pass 2  one block per partition (segment, high bits) counts the low
//           <= 8 bits in LDS, writes the bucket offsets, and places the
//           entries in bucket order.  Partitions up to PART_CAP entries are
//           staged in LDS; larger ones (skewed inputs) are sorted by many
//           blocks (k_big_*).
// Segments of one job hold n entries each; jobs may differ in n, so a block
// finds its job by binary search over the job table.
#include <algorithm>

#include "common.hpp"
#include "convert.hpp"

namespace msm {
namespace {

constexpr int SORT_THREADS = 256;
constexpr uint32_t TILE = SORT_TILE;  // entries per pass-1 tile
constexpr uint32_t PER_THREAD = TILE / SORT_THREADS;
constexpr uint32_t PART_CAP = SORT_PART_CAP;  // entries staged in LDS by pass 2
constexpr unsigned BIG_GRID = 512;    // blocks of the large-partition kernels

struct SortGeom {
  JobView jv;
  uint32_t W, S, bb, lo_bits, hi_bits;
  uint32_t tpb;  // pass-1 tiles per block: a block's group of tpb tiles shares one histogram
};

// Staged entries between the passes (tmp): the index word (point index |
// sign << 31) and the bucket key, 8 bytes; or, for jobs of at most 2^23
// points (PK), one word: index bits 0..22, the key's low (<= 8) bucket bits
// at 23..30, the sign at 31.  Pass 2 and the many-block sort need only the
// index word and the low bits (a partition's keys are its first bucket plus
// the low bits), so the packed form loses nothing and halves the staging
// traffic.
template <bool PK>
struct TmpEnt;
template <>
struct TmpEnt<false> {
  using T = uint2;
  __device__ static T make(uint32_t idxw, uint32_t key, uint32_t) { return make_uint2(idxw, key); }
  __device__ static uint32_t lo(const T& e, uint32_t L) { return e.y & (L - 1); }
  __device__ static uint32_t idx(const T& e) { return e.x; }
};
template <>
struct TmpEnt<true> {
  using T = uint32_t;
  __device__ static T make(uint32_t idxw, uint32_t, uint32_t lo) {
    return (idxw & 0x807fffffu) | (lo << 23);
  }
  __device__ static uint32_t lo(const T& e, uint32_t) { return (e >> 23) & 0xffu; }
  __device__ static uint32_t idx(const T& e) { return e & 0x807fffffu; }
};

// largest j with key(j) <= x, for a key non-decreasing in j (J >= 1)
template <typename F>
__device__ __forceinline__ uint32_t find_job(uint32_t J, uint32_t x, F key) {
  uint32_t lo = 0, hi = J - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (key(mid) <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// the segment, tile group and job of pass-1 block b (tile = the group's
// index in its segment; a group is tpb consecutive tiles of TILE digits)
struct TileRef {
  JobDesc d;
  uint32_t j, w, tile;
};

__device__ __forceinline__ TileRef tile_ref(const SortGeom& g, uint32_t b) {
  TileRef r;
  r.j = g.jv.tab ? find_job(g.jv.J, b, [&](uint32_t j) { return g.W * g.jv.tab[j].tile_off; }) : 0u;
  r.d = g.jv.get(r.j);
  const uint32_t local = b - g.W * r.d.tile_off;
  r.w = local / r.d.tps;
  r.tile = local % r.d.tps;
  return r;
}

// count-matrix index of (segment of job d window w, high bits hi, tile group)
__device__ __forceinline__ size_t count_index(const SortGeom& g, const JobDesc& d, uint32_t w,
                                              uint32_t hi, uint32_t tile) {
  const size_t seg_tile0 = (size_t)g.W * d.tile_off + (size_t)w * d.tps;
  return (seg_tile0 << g.hi_bits) + (size_t)hi * d.tps + tile;
}

// One signed digit: v (the window's c bits) plus the carry of the window
// below, as q | sign << 31; negative (v - 2^c) from 2^(c-1) on, except in
// the top window, which takes the carry.
__device__ __forceinline__ uint32_t signed_digit(uint32_t v0, uint32_t& carry, int c, bool top) {
  const uint32_t v = v0 + carry;
  if (v >= (1u << (c - 1)) && !top) {  // d = v - 2^c < 0
    carry = 1;
    return ((1u << c) - v) | (v == (1u << c) ? 0u : 0x80000000u);
  }
  carry = 0;
  return v;
}

// Digits of every window of every job.  Word (segment s = j W + w, point i)
// at W pt_off + w n + i holds q | sign << 31, where q = 0 drops the entry and
// otherwise bucket m = q - 1 (signed digits, q = |d|) or m = q (unsigned
// digits, q = d, so unsigned bucket 0 never receives points).  With the
// endomorphism split a job's n points are its n / 2 input points and their
// images, interleaved: point 2i takes the digits of s0 of scalar i, point
// 2i + 1 those of s1; one thread splits scalar i and writes both digit words
// of each window (n and pt_off are even there).  N counts threads: points,
// or point pairs with the split.
__global__ void __launch_bounds__(256) k_slice(JobView jv, uint32_t N, int c, int W, int encoding,
                                               uint32_t* __restrict__ digits,
                                               uint32_t* __restrict__ flags) {
  const uint32_t gt = blockIdx.x * blockDim.x + threadIdx.x;
  if (gt >= N) return;
  const uint32_t gi = encoding == MSM_DIGITS_GLV ? 2u * gt : gt;  // first point
  const uint32_t j = jv.tab ? find_job(jv.J, gi, [&](uint32_t k) { return jv.tab[k].pt_off; }) : 0u;
  const JobDesc d = jv.get(j);
  const uint32_t i = gi - d.pt_off;
  uint32_t* out = digits + (size_t)W * d.pt_off + i;
  if (encoding == MSM_DIGITS_GLV) {
    scalar256 s0, s1;
    glv_split(ld_scalar(d.scalars, i >> 1, flags + j), s0, s1);
    uint2* out2 = reinterpret_cast<uint2*>(out);
    uint32_t carry0 = 0, carry1 = 0;
    for (int w = 0; w < W; ++w) {
      const bool top = w + 1 == W;
      uint2 q;
      q.x = signed_digit(digit_at(s0, w * c, c), carry0, c, top);
      q.y = signed_digit(digit_at(s1, w * c, c), carry1, c, top);
      out2[(size_t)w * (d.n >> 1)] = q;
    }
    return;
  }
  const scalar256 s = ld_scalar(d.scalars, i, flags + j);
  if (encoding == MSM_DIGITS_UNSIGNED) {
    for (int w = 0; w < W; ++w) out[(size_t)w * d.n] = digit_at(s, w * c, c);
    return;
  }
  uint32_t carry = 0;
  for (int w = 0; w < W; ++w) out[(size_t)w * d.n] = signed_digit(digit_at(s, w * c, c), carry, c, w + 1 == W);
}

// bucket index and the entry's index word of a digit word q != 0
__device__ __forceinline__ uint32_t bucket_of(uint32_t q, uint32_t off) {
  return (q & 0x7fffffffu) - off;
}

// pass 1a: per-group histogram of the high bits (the group's tiles one
// after another into one LDS histogram)
__global__ void __launch_bounds__(SORT_THREADS) k_part_count(SortGeom g, uint32_t off,
                                                             const uint32_t* __restrict__ digits,
                                                             uint32_t* __restrict__ counts) {
  __shared__ uint32_t hist[1u << 12];
  const TileRef t = tile_ref(g, blockIdx.x);
  const uint32_t H = 1u << g.hi_bits;
  for (uint32_t b = threadIdx.x; b < H; b += SORT_THREADS) hist[b] = 0;
  __syncthreads();
  const uint32_t g0 = t.tile * TILE * g.tpb, g1 = min(g0 + TILE * g.tpb, t.d.n);
  const uint32_t* dg = digits + (size_t)g.W * t.d.pt_off + (size_t)t.w * t.d.n;
  for (uint32_t e0 = g0; e0 < g1; e0 += TILE) {
    const uint32_t e1 = min(e0 + TILE, g1);
    uint32_t dq[PER_THREAD];
#pragma unroll
    for (uint32_t r = 0; r < PER_THREAD; ++r) {  // loads first, clamped (e1 > e0)
      const uint32_t e = e0 + r * SORT_THREADS + threadIdx.x;
      dq[r] = dg[e < e1 ? e : e1 - 1];
    }
#pragma unroll
    for (uint32_t r = 0; r < PER_THREAD; ++r) {
      const uint32_t q = e0 + r * SORT_THREADS + threadIdx.x < e1 ? dq[r] : 0u;
      if (q) atomicAdd(&hist[bucket_of(q, off) >> g.lo_bits], 1u);
    }
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < H; b += SORT_THREADS)
    counts[count_index(g, t.d, t.w, b, t.tile)] = hist[b];
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

// block-wide exclusive scan of v[0..n) (n <= 16 SORT_THREADS) in place;
// returns the total; all SORT_THREADS threads must call it
__device__ uint32_t lds_exclusive_scan(uint32_t* v, uint32_t n) {
  __shared__ uint32_t sums[SORT_THREADS];
  __shared__ uint32_t total;
  const uint32_t per = (n + SORT_THREADS - 1) / SORT_THREADS;
  const uint32_t b0 = min(threadIdx.x * per, n), b1 = min(b0 + per, n);
  uint32_t sum = 0;
  for (uint32_t i = b0; i < b1; ++i) sum += v[i];
  sums[threadIdx.x] = sum;
  __syncthreads();
  lds_exclusive_scan256(sums, SORT_THREADS);
  uint32_t run = sums[threadIdx.x];
  if (threadIdx.x == SORT_THREADS - 1) total = run + sum;
  for (uint32_t i = b0; i < b1; ++i) {
    const uint32_t x = v[i];
    v[i] = run;
    run += x;
  }
  __syncthreads();
  return total;
}

// pass 1b: scatter into (partition, tile group) ranges; tmp entry =
// {idx | sign, key}.  Each tile of the group is first ordered by partition in
// LDS, so that consecutive threads write consecutive entries of each
// partition's range; a partition's cursor (gstart) then moves past the
// tile's entries for the next tile of the group.
template <bool PK>
__global__ void __launch_bounds__(SORT_THREADS) k_part_scatter(SortGeom g, uint32_t off,
                                                               const uint32_t* __restrict__ digits,
                                                               const uint32_t* __restrict__ scanned,
                                                               typename TmpEnt<PK>::T* __restrict__ tmp,
                                                               uint32_t* __restrict__ clear0,
                                                               uint32_t* __restrict__ clear1) {
  // two list counters of later passes start at zero (the large-partition
  // list of pass 2 and the long-merge list of the accumulation)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *clear0 = 0u;
    *clear1 = 0u;
  }
  // dynamic LDS, sized by the launch for H = 2^hi_bits partitions: the tile
  // stage, then per partition its global start and its local count / start
  extern __shared__ uint2 scatter_lds[];
  const uint32_t H = 1u << g.hi_bits;
  uint2* stage = scatter_lds;
  uint32_t* gstart = reinterpret_cast<uint32_t*>(scatter_lds + TILE);
  uint32_t* lstart = gstart + H;
  const TileRef t = tile_ref(g, blockIdx.x);
  for (uint32_t b = threadIdx.x; b < H; b += SORT_THREADS) {
    gstart[b] = scanned[count_index(g, t.d, t.w, b, t.tile)];
    lstart[b] = 0;
  }
  __syncthreads();
  const uint32_t g0 = t.tile * TILE * g.tpb, g1 = min(g0 + TILE * g.tpb, t.d.n);
  const uint32_t* dg = digits + (size_t)g.W * t.d.pt_off + (size_t)t.w * t.d.n;
  const uint32_t keybase = (t.j * g.W + t.w) << g.bb;
  for (uint32_t e0 = g0; e0 < g1; e0 += TILE) {
    const uint32_t e1 = min(e0 + TILE, g1);
    uint32_t part[PER_THREAD], rank[PER_THREAD], dq[PER_THREAD];
    uint2 ent[PER_THREAD];
    // all loads first (clamped, unconditional), so that they overlap
#pragma unroll
    for (uint32_t r = 0; r < PER_THREAD; ++r) {
      const uint32_t e = e0 + r * SORT_THREADS + threadIdx.x;
      dq[r] = dg[e < e1 ? e : e1 - 1];
    }
#pragma unroll
    for (uint32_t r = 0; r < PER_THREAD; ++r) {
      const uint32_t e = e0 + r * SORT_THREADS + threadIdx.x;
      const uint32_t q = e < e1 ? dq[r] : 0u;
      part[r] = H;  // no entry
      rank[r] = 0;
      ent[r] = make_uint2(0u, 0u);
      if (q) {
        const uint32_t m = bucket_of(q, off);
        part[r] = m >> g.lo_bits;
        rank[r] = atomicAdd(&lstart[part[r]], 1u);
        ent[r] = make_uint2(e | (q & 0x80000000u), keybase + m);
      }
    }
    __syncthreads();
    const uint32_t count = lds_exclusive_scan(lstart, H);
#pragma unroll
    for (uint32_t r = 0; r < PER_THREAD; ++r)
      if (part[r] < H) stage[lstart[part[r]] + rank[r]] = ent[r];
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < count; k += SORT_THREADS) {
      const uint2 en = stage[k];
      const uint32_t pr = (en.y - keybase) >> g.lo_bits;
      tmp[gstart[pr] + (k - lstart[pr])] =
          TmpEnt<PK>::make(en.x, en.y, (en.y - keybase) & ((1u << g.lo_bits) - 1));
    }
    if (g.tpb == 1) break;  // (a single tile needs no cursor update)
    __syncthreads();  // the stage and the local starts are read
    for (uint32_t b = threadIdx.x; b < H; b += SORT_THREADS)
      gstart[b] += (b + 1 < H ? lstart[b + 1] : count) - lstart[b];
    __syncthreads();  // every local start is read before the reset
    for (uint32_t b = threadIdx.x; b < H; b += SORT_THREADS) lstart[b] = 0;
    __syncthreads();
  }
}

// partition p's range [start, start + size) in tmp; partitions are contiguous
// in the count matrix, the next one starting tps entries later
__device__ __forceinline__ void part_range(const SortGeom& g, const uint32_t* __restrict__ scanned,
                                           uint32_t total, size_t ncounts, uint32_t p,
                                           uint32_t& start, uint32_t& size) {
  const uint32_t s = p >> g.hi_bits, hi = p & ((1u << g.hi_bits) - 1);
  const JobDesc d = g.jv.get(s / g.W);
  const size_t ci = count_index(g, d, s % g.W, hi, 0);
  start = scanned[ci];
  const uint32_t end = (ci + d.tps < ncounts) ? scanned[ci + d.tps] : total;
  size = end - start;
}

// first bucket of partition p
__device__ __forceinline__ uint32_t part_bucket0(const SortGeom& g, uint32_t p) {
  const uint32_t s = p >> g.hi_bits, hi = p & ((1u << g.hi_bits) - 1);
  return (s << g.bb) + (hi << g.lo_bits);
}

// pass 2: one block per partition (segment s, high bits hi).  Each thread
// keeps its share of the partition's entries in registers (ROWS rows of the
// block); after the bucket histogram and its scan, every entry takes its place
// in bucket order in LDS (index word and low bucket bits, 5 bytes an entry)
// and the block writes the partition out linearly.
template <uint32_t ROWS, bool PK>
__device__ __forceinline__ void part_sort_rows(const SortGeom& g, uint32_t p, uint32_t start,
                                               uint32_t size,
                                               const typename TmpEnt<PK>::T* __restrict__ tmp,
                                               uint32_t* __restrict__ key,
                                               uint32_t* __restrict__ idx,
                                               uint32_t* __restrict__ offsets,
                                               uint32_t* __restrict__ buckets, uint32_t* out_idx,
                                               uint8_t* out_lo, uint32_t* hist, uint32_t* cur) {
  const uint32_t L = 1u << g.lo_bits;
  if (threadIdx.x < 256) hist[threadIdx.x] = 0;
  __syncthreads();
  typename TmpEnt<PK>::T ev[ROWS];
  if (size > 0) {
    // all loads first (clamped, unconditional), so that they overlap
#pragma unroll
    for (uint32_t r = 0; r < ROWS; ++r) {
      const uint32_t k = r * SORT_THREADS + threadIdx.x;
      ev[r] = tmp[start + (k < size ? k : size - 1)];
    }
#pragma unroll
    for (uint32_t r = 0; r < ROWS; ++r)
      if (r * SORT_THREADS + threadIdx.x < size) atomicAdd(&hist[TmpEnt<PK>::lo(ev[r], L)], 1u);
  }
  __syncthreads();
  for (uint32_t lo = threadIdx.x; lo < L; lo += SORT_THREADS) cur[lo] = hist[lo];
  __syncthreads();
  lds_exclusive_scan256(cur, L);  // cur[lo] = local start of bucket lo
  const uint32_t bucket0 = part_bucket0(g, p);
  if (threadIdx.x < L) {
    const uint32_t lo = threadIdx.x;
    offsets[bucket0 + lo] = start + cur[lo];
    if (hist[lo] == 0 && buckets)
      st_xytz(buckets + (size_t)(bucket0 + lo) * XYTZ_WORDS, pt_identity());
  }
  __syncthreads();
  if (size > 0) {
#pragma unroll
    for (uint32_t r = 0; r < ROWS; ++r) {
      if (r * SORT_THREADS + threadIdx.x < size) {
        const uint32_t lo = TmpEnt<PK>::lo(ev[r], L);
        const uint32_t q = atomicAdd(&cur[lo], 1u);
        out_idx[q] = TmpEnt<PK>::idx(ev[r]);
        out_lo[q] = (uint8_t)lo;
      }
    }
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < size; q += SORT_THREADS) {
    key[start + q] = bucket0 + out_lo[q];
    idx[start + q] = out_idx[q];
  }
}

// Partitions of up to SHORT_ROWS rows (evenly spread digits) take the short
// form, larger ones up to PART_CAP entries the long one.  A partition of more
// than PART_CAP entries (skewed digits) is only listed in big[] here; the
// k_big_* kernels sort it with many blocks.
constexpr uint32_t SHORT_ROWS = 20;

template <bool PK>
__global__ void __launch_bounds__(SORT_THREADS) k_part_sort(
    SortGeom g, const uint32_t* __restrict__ scanned, const uint32_t* __restrict__ total_p,
    size_t ncounts, const typename TmpEnt<PK>::T* __restrict__ tmp, uint32_t* __restrict__ key,
    uint32_t* __restrict__ idx, uint32_t* __restrict__ offsets, uint32_t* __restrict__ buckets,
    uint32_t* __restrict__ big) {
  __shared__ uint32_t out_idx[PART_CAP];  // index words in bucket order
  __shared__ uint8_t out_lo[PART_CAP];    // their low bucket bits
  __shared__ uint32_t hist[256], cur[256];
  constexpr uint32_t ROWS = (PART_CAP + SORT_THREADS - 1) / SORT_THREADS;
  const uint32_t p = blockIdx.x;
  const uint32_t total = *total_p;
  uint32_t start, size;
  part_range(g, scanned, total, ncounts, p, start, size);
  if (p == 0 && threadIdx.x == 0) offsets[g.S << g.bb] = total;
  if (size > PART_CAP) {
    if (threadIdx.x == 0) big[1 + atomicAdd(&big[0], 1u)] = p;
    return;
  }
  if (size <= SHORT_ROWS * SORT_THREADS)
    part_sort_rows<SHORT_ROWS, PK>(g, p, start, size, tmp, key, idx, offsets, buckets, out_idx,
                                   out_lo, hist, cur);
  else
    part_sort_rows<ROWS, PK>(g, p, start, size, tmp, key, idx, offsets, buckets, out_idx, out_lo,
                             hist, cur);
}

// Large partitions, sorted by many blocks.  big[0] = their count n, big[1..n]
// their ids.  desc[4b .. 4b + 3] = id, start, size and first item of large
// partition b, desc[4n] = the item count; an item is BIG_CH consecutive
// entries of one large partition, item_of[item] its partition.  cnt[item * 256 + lo] holds the item's count
// of bucket lo, then its cursor (the bucket's start plus the entries of
// earlier items).
constexpr uint32_t BIG_CH = SORT_BIG_ITEM;


// numbering of the items (one block); item_of[item] = its large partition
__global__ void __launch_bounds__(SORT_THREADS) k_big_plan(
    SortGeom g, const uint32_t* __restrict__ scanned, const uint32_t* __restrict__ total_p,
    size_t ncounts, const uint32_t* __restrict__ big, uint32_t* __restrict__ desc,
    uint32_t* __restrict__ item_of) {
  __shared__ uint32_t chunks[16 * SORT_THREADS];
  const uint32_t nbig = big[0], total = *total_p;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nbig; base += 16 * SORT_THREADS) {
    const uint32_t n = min(16u * SORT_THREADS, nbig - base);
    for (uint32_t i = threadIdx.x; i < n; i += SORT_THREADS) {
      const uint32_t p = big[1 + base + i];
      uint32_t start, size;
      part_range(g, scanned, total, ncounts, p, start, size);
      desc[4 * (base + i) + 0] = p;
      desc[4 * (base + i) + 1] = start;
      desc[4 * (base + i) + 2] = size;
      chunks[i] = (size + BIG_CH - 1) / BIG_CH;
    }
    __syncthreads();
    const uint32_t tot = lds_exclusive_scan(chunks, n);
    for (uint32_t i = threadIdx.x; i < n; i += SORT_THREADS) {
      const uint32_t first = carry + chunks[i];
      desc[4 * (base + i) + 3] = first;
      const uint32_t items = (desc[4 * (base + i) + 2] + BIG_CH - 1) / BIG_CH;
      for (uint32_t k = 0; k < items; ++k) item_of[first + k] = base + i;
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) desc[4 * nbig] = carry;
}

// per item: histogram of the low bucket bits
template <bool PK>
__global__ void __launch_bounds__(SORT_THREADS) k_big_count(SortGeom g,
                                                            const uint32_t* __restrict__ big,
                                                            const uint32_t* __restrict__ desc,
                                                            const uint32_t* __restrict__ item_of,
                                                            const typename TmpEnt<PK>::T* __restrict__ tmp,
                                                            uint32_t* __restrict__ cnt) {
  __shared__ uint32_t hist[256];
  const uint32_t nbig = big[0];
  if (nbig == 0) return;
  const uint32_t items = desc[4 * nbig], L = 1u << g.lo_bits;
  for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
    const uint32_t b = item_of[item];
    const uint32_t start = desc[4 * b + 1], size = desc[4 * b + 2];
    const uint32_t e0 = (item - desc[4 * b + 3]) * BIG_CH, e1 = min(e0 + BIG_CH, size);
    if (threadIdx.x < 256) hist[threadIdx.x] = 0;
    __syncthreads();
    constexpr uint32_t PER = BIG_CH / SORT_THREADS;
    uint32_t kv[PER];
#pragma unroll
    for (uint32_t r = 0; r < PER; ++r) {  // loads first, clamped (e1 > e0)
      const uint32_t k = e0 + r * SORT_THREADS + threadIdx.x;
      kv[r] = TmpEnt<PK>::lo(tmp[start + (k < e1 ? k : e1 - 1)], L);
    }
#pragma unroll
    for (uint32_t r = 0; r < PER; ++r)
      if (e0 + r * SORT_THREADS + threadIdx.x < e1) atomicAdd(&hist[kv[r]], 1u);
    __syncthreads();
    for (uint32_t lo = threadIdx.x; lo < L; lo += SORT_THREADS)
      cnt[(size_t)item * 256 + lo] = hist[lo];
    __syncthreads();
  }
}

// per large partition: counts -> cursors, bucket offsets, identities
__global__ void __launch_bounds__(SORT_THREADS) k_big_scan(SortGeom g,
                                                           const uint32_t* __restrict__ big,
                                                           const uint32_t* __restrict__ desc,
                                                           uint32_t* __restrict__ cnt,
                                                           uint32_t* __restrict__ offsets,
                                                           uint32_t* __restrict__ buckets) {
  __shared__ uint32_t bstart[256];
  const uint32_t nbig = big[0], L = 1u << g.lo_bits, lo = threadIdx.x;
  for (uint32_t b = blockIdx.x; b < nbig; b += gridDim.x) {
    const uint32_t p = desc[4 * b], start = desc[4 * b + 1], size = desc[4 * b + 2];
    const uint32_t it0 = desc[4 * b + 3], nit = (size + BIG_CH - 1) / BIG_CH;
    uint32_t run = 0;
    if (lo < L) {
      for (uint32_t it = 0; it < nit; ++it) {
        uint32_t* c = cnt + (size_t)(it0 + it) * 256 + lo;
        const uint32_t v = *c;
        *c = run;
        run += v;
      }
    }
    if (lo < 256) bstart[lo] = run;
    __syncthreads();
    lds_exclusive_scan256(bstart, L);
    const uint32_t bucket0 = part_bucket0(g, p);
    if (lo < L) {
      offsets[bucket0 + lo] = start + bstart[lo];
      if (run == 0 && buckets)
        st_xytz(buckets + (size_t)(bucket0 + lo) * XYTZ_WORDS, pt_identity());
      for (uint32_t it = 0; it < nit; ++it) cnt[(size_t)(it0 + it) * 256 + lo] += bstart[lo];
    }
    __syncthreads();
  }
}

// per item: place its entries at the cursors
template <bool PK>
__global__ void __launch_bounds__(SORT_THREADS) k_big_scatter(SortGeom g,
                                                              const uint32_t* __restrict__ big,
                                                              const uint32_t* __restrict__ desc,
                                                              const uint32_t* __restrict__ item_of,
                                                              const uint32_t* __restrict__ cnt,
                                                              const typename TmpEnt<PK>::T* __restrict__ tmp,
                                                              uint32_t* __restrict__ key,
                                                              uint32_t* __restrict__ idx) {
  __shared__ uint32_t cur[256];
  const uint32_t nbig = big[0];
  if (nbig == 0) return;
  const uint32_t items = desc[4 * nbig], L = 1u << g.lo_bits;
  for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
    const uint32_t b = item_of[item];
    const uint32_t p = desc[4 * b], start = desc[4 * b + 1], size = desc[4 * b + 2];
    const uint32_t e0 = (item - desc[4 * b + 3]) * BIG_CH, e1 = min(e0 + BIG_CH, size);
    const uint32_t bucket0 = part_bucket0(g, p);
    for (uint32_t lo = threadIdx.x; lo < L; lo += SORT_THREADS) cur[lo] = cnt[(size_t)item * 256 + lo];
    constexpr uint32_t PER = BIG_CH / SORT_THREADS;
    typename TmpEnt<PK>::T ev[PER];
#pragma unroll
    for (uint32_t r = 0; r < PER; ++r) {  // loads first, clamped (e1 > e0)
      const uint32_t k = e0 + r * SORT_THREADS + threadIdx.x;
      ev[r] = tmp[start + (k < e1 ? k : e1 - 1)];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < PER; ++r) {
      if (e0 + r * SORT_THREADS + threadIdx.x < e1) {
        const uint32_t lo = TmpEnt<PK>::lo(ev[r], L);
        const uint32_t pos = start + atomicAdd(&cur[lo], 1u);
        key[pos] = bucket0 + lo;
        idx[pos] = TmpEnt<PK>::idx(ev[r]);
      }
    }
    __syncthreads();
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
  // a thread's 16 words are 64-byte aligned: 16-byte loads when all in range
  const bool whole = base + SCAN_PER_THREAD <= n;
  if (whole) {
    const uint4* q = reinterpret_cast<const uint4*>(data + base);
#pragma unroll
    for (int j = 0; j < SCAN_PER_THREAD / 4; ++j) {
      const uint4 w = q[j];
      v[4 * j] = w.x;
      v[4 * j + 1] = w.y;
      v[4 * j + 2] = w.z;
      v[4 * j + 3] = w.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < SCAN_PER_THREAD; ++j) v[j] = (base + j < n) ? data[base + j] : 0u;
  }
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) sum += v[j];
  uint32_t excl;
  uint32_t total = block_exclusive_scan(sum, excl);
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) {
    const uint32_t x = v[j];
    v[j] = excl;
    excl += x;
  }
  if (whole) {
    uint4* q = reinterpret_cast<uint4*>(data + base);
#pragma unroll
    for (int j = 0; j < SCAN_PER_THREAD / 4; ++j)
      q[j] = make_uint4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
  } else {
#pragma unroll
    for (int j = 0; j < SCAN_PER_THREAD; ++j)
      if (base + j < n) data[base + j] = v[j];
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

}  // namespace

// Split of the bb bucket bits: enough high bits that a partition of uniformly
// distributed digits of the largest job holds about max_n / 2^hi <=
// SORT_PART_TARGET entries, at most 8 low bits (pass-2 histogram) and at most 12
// high bits (pass-1 histogram).  Also the tile grouping and the count-matrix
// size.  A pass-1 block takes a group of tpb tiles with one histogram: tpb =
// 2^hi / (32 x staged entry bytes) keeps about 256 bytes of staged entries
// per (group, partition) for uniform digits (64 one-word or 32 two-word
// entries), so that the scatter writes long runs and the count matrix (groups
// x 2^hi, which with single tiles grows with the square of the input) stays
// small.  If the matrix still exceeds the two-level scan (SCAN_ITEMS^2
// counts), groups grow to 64 tiles, then the split takes fewer high bits
// (down to bb - 8), whose partitions, larger than the LDS stage, go to the
// many-block path.  Every single job the interface takes then fits (at
// n < 2^26 the matrix stays within 2^24 counts); plans that still do not
// (batches of thousands of jobs at widths of 18 and up, whose buckets alone
// would need hundreds of GB) are refused.
void sort_geometry(Plan& pl, const size_t* ns, uint32_t J, size_t mult) {
  const uint32_t bb = (uint32_t)pl.bb;
  uint32_t want = 0;
  while (want < 12 && (pl.max_n >> want) > SORT_PART_TARGET) ++want;
  const uint32_t hi_min = bb > 8 ? bb - 8 : 0;
  uint32_t hi = std::max<uint32_t>(want, hi_min);
  hi = std::min<uint32_t>(hi, std::min<uint32_t>(bb, 12));
  auto groups = [&](uint32_t tpb) {
    size_t gs = 0;
    for (uint32_t j = 0; j < J; ++j) gs += (mult * ns[j] + (size_t)SORT_TILE * tpb - 1) / ((size_t)SORT_TILE * tpb);
    return gs * (size_t)pl.W;
  };
  const size_t two_level = (size_t)SCAN_ITEMS * SCAN_ITEMS;
  // staged entry bytes: one word for jobs of at most 2^23 point records
  const uint32_t sb = pl.max_n <= ((size_t)1 << 23) ? 4u : 8u;
  uint32_t tpb = std::max<uint32_t>(1u, (1u << hi) / (32u * sb));
  while (tpb < 64 && (groups(tpb) << hi) > two_level) tpb <<= 1;
  while (hi > hi_min && (groups(tpb) << hi) > two_level) --hi;
  pl.hi_bits = hi;
  pl.lo_bits = bb - hi;
  pl.tpb = tpb;
  pl.tile_digits = SORT_TILE * tpb;
  pl.tiles = groups(tpb);
  pl.ncounts = pl.tiles << hi;
  pl.nb = (pl.ncounts + SCAN_ITEMS - 1) / SCAN_ITEMS;
  // one-word staged entries: 23 index bits and 8 low bucket bits
  pl.tmp_packed = pl.max_n <= ((size_t)1 << 23) && pl.lo_bits <= 8;
}

namespace {
struct SortBufs {
  uint32_t *digits, *counts, *total, *offsets, *key, *idx, *buckets;
  uint32_t *big, *bigdesc, *bigcnt, *bigitem, *longlist;
};

// pass-1 scatter, pass 2 and the many-block sort, on staged entries of
// either form
template <bool PK>
void sort_passes(const Plan& pl, const SortGeom& g, uint32_t off, const SortBufs& b,
                 typename TmpEnt<PK>::T* tmp, size_t scatter_lds, hipStream_t st) {
  k_part_scatter<PK><<<(unsigned)pl.tiles, SORT_THREADS, scatter_lds, st>>>(
      g, off, b.digits, b.counts, tmp, b.big, b.longlist);
  k_part_sort<PK><<<(unsigned)(pl.S << pl.hi_bits), SORT_THREADS, 0, st>>>(
      g, b.counts, b.total, pl.ncounts, tmp, b.key, b.idx, b.offsets, b.buckets, b.big);
  // large partitions (none for evenly spread digits: these return at once)
  k_big_plan<<<1, SORT_THREADS, 0, st>>>(g, b.counts, b.total, pl.ncounts, b.big, b.bigdesc,
                                         b.bigitem);
  k_big_count<PK><<<BIG_GRID, SORT_THREADS, 0, st>>>(g, b.big, b.bigdesc, b.bigitem, tmp,
                                                     b.bigcnt);
  k_big_scan<<<BIG_GRID, SORT_THREADS, 0, st>>>(g, b.big, b.bigdesc, b.bigcnt, b.offsets,
                                                b.buckets);
  k_big_scatter<PK><<<BIG_GRID, SORT_THREADS, 0, st>>>(g, b.big, b.bigdesc, b.bigitem, b.bigcnt,
                                                       tmp, b.key, b.idx);
}
}  // namespace

int launch_sort(const Plan& pl, uint32_t* buckets, void* ws, hipStream_t st) {
  uint32_t* flags = ws_at<uint32_t>(ws, pl.o_flags);
  uint32_t* total = ws_at<uint32_t>(ws, pl.o_total);
  uint32_t* offsets = ws_at<uint32_t>(ws, pl.o_offsets);
  uint32_t* counts = ws_at<uint32_t>(ws, pl.o_counts);
  uint32_t* blocksums = ws_at<uint32_t>(ws, pl.o_blocksums);
  uint32_t* digits = ws_at<uint32_t>(ws, pl.o_digits);
  uint32_t* key = ws_at<uint32_t>(ws, pl.o_key);
  uint32_t* idx = ws_at<uint32_t>(ws, pl.o_idx);
  if (pl.lo_bits > 8 || pl.hi_bits > 12 || pl.nb > (size_t)SCAN_ITEMS) return MSM_EINVAL;

  SortGeom g;
  g.jv = job_view(pl, ws);
  g.W = (uint32_t)pl.W;
  g.S = (uint32_t)pl.S;
  g.bb = (uint32_t)pl.bb;
  g.lo_bits = pl.lo_bits;
  g.hi_bits = pl.hi_bits;
  g.tpb = pl.tpb;
  const uint32_t off = pl.encoding == MSM_DIGITS_UNSIGNED ? 0u : 1u;

  int rc;
  if ((rc = launch_fill_u32(flags, pl.J, 0u, st)) != MSM_OK) return rc;
  const size_t slice_threads = pl.encoding == MSM_DIGITS_GLV ? pl.N / 2 : pl.N;
  k_slice<<<grid_for(slice_threads, 256), 256, 0, st>>>(g.jv, (uint32_t)slice_threads, pl.c, pl.W,
                                                        pl.encoding, digits, flags);
  k_part_count<<<(unsigned)pl.tiles, SORT_THREADS, 0, st>>>(g, off, digits, counts);
  k_scan_block<<<(unsigned)pl.nb, SCAN_THREADS, 0, st>>>(counts, pl.ncounts, blocksums);
  k_scan_top<<<1, SCAN_THREADS, 0, st>>>(blocksums, (uint32_t)pl.nb, total);
  k_scan_add<<<(unsigned)pl.nb, SCAN_THREADS, 0, st>>>(counts, pl.ncounts, blocksums);
  const size_t scatter_lds = TILE * sizeof(uint2) + 2 * ((size_t)4 << pl.hi_bits);
  SortBufs sb{digits, counts, total, offsets, key, idx, buckets,
              ws_at<uint32_t>(ws, pl.o_big), ws_at<uint32_t>(ws, pl.o_bigdesc),
              ws_at<uint32_t>(ws, pl.o_bigcnt), ws_at<uint32_t>(ws, pl.o_bigitem),
              ws_at<uint32_t>(ws, pl.o_longlist)};
  if (pl.tmp_packed)
    sort_passes<true>(pl, g, off, sb, ws_at<uint32_t>(ws, pl.o_tmp), scatter_lds, st);
  else
    sort_passes<false>(pl, g, off, sb, ws_at<uint2>(ws, pl.o_tmp), scatter_lds, st);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // namespace msm
