// Bucket aggregation and group aggregation (Sec. II-C).
//
// Bucket aggregation computes S_w = sum_b b B[w][b].  Writing b in binary,
// S_w = sum_t 2^t X_t with X_t = sum of the buckets whose index has bit t set.
// The X_t are built by a binary tree over the bucket index: a node covering
// 2^h consecutive buckets keeps V[t] (t < h, the sum over its buckets with bit
// t set) and S (the sum of all its buckets).  Merging left child L and right
// child R gives V[t] = L.V[t] + R.V[t] (t < h), V[h] = R.S, S = L.S + R.S.
// Every output of a level is one independent addition, the whole tree costs
// about 2 * 2^c additions per window (as many as the running-sum method) and
// its dependent depth is only c additions.  Large levels run one addition per
// lane; small ones use the four-lane quad unit (quad.hpp) to cut latency.
//
// Each window then forms S_w = sum_t 2^t X_t by Horner's rule on one quad, and
// group aggregation Q = sum_w 2^(w c) S_w is Horner's rule over the windows
// (c doublings per window), the dependent chain the paper assigns to its
// low-latency unit.  The result is mapped back to Weierstrass affine form.
#include "common.hpp"
#include "convert.hpp"
#include "quad.hpp"

namespace msm {
namespace {

// record of node n, slot s at a tree level with `slots` slots per node
__device__ __forceinline__ size_t rec_index(uint32_t w, uint32_t nodes, uint32_t n, uint32_t slots,
                                            uint32_t s) {
  return ((size_t)w * nodes + n) * slots + s;
}

// One level h -> h+1, one output record per lane.
__global__ void __launch_bounds__(256) k_tree_level(const uint32_t* __restrict__ in, uint32_t h,
                                                    uint32_t nodes_in, uint32_t w_lo,
                                                    uint32_t w_cnt, uint32_t* __restrict__ out,
                                                    int to_u) {
  const uint32_t nodes_out = nodes_in >> 1, slots_in = h + 1, slots_out = h + 2;
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (uint64_t)w_cnt * nodes_out * slots_out) return;
  const uint32_t s = (uint32_t)(g % slots_out);
  const uint32_t t = (uint32_t)(g / slots_out);
  const uint32_t n = t % nodes_out, w = w_lo + t / nodes_out;
  const uint32_t* L = in + rec_index(w, nodes_in, 2 * n, slots_in, 0) * XYTZ_WORDS;
  const uint32_t* R = L + (size_t)slots_in * XYTZ_WORDS;
  const fe p2 = fe_const(kP2);
  xytz r;
  if (s == h) {
    r = ld_xytz(R + (size_t)h * XYTZ_WORDS);
  } else {
    const uint32_t src = (s < h) ? s : h;
    r = padd_full(ld_xytz(L + (size_t)src * XYTZ_WORDS), ld_xytz(R + (size_t)src * XYTZ_WORDS), p2);
  }
  if (to_u && s <= h) r.T = fe_mul(r.T, fe_const(kK));
  st_xytz(out + rec_index(w, nodes_out, n, slots_out, s) * XYTZ_WORDS, r);
}

// Same level, four lanes per output record.
__global__ void __launch_bounds__(256) k_tree_level_quad(const uint32_t* __restrict__ in, uint32_t h,
                                                         uint32_t nodes_in, uint32_t w_lo,
                                                         uint32_t w_cnt,
                                                         uint32_t* __restrict__ out, int to_u) {
  const uint32_t nodes_out = nodes_in >> 1, slots_in = h + 1, slots_out = h + 2;
  const uint64_t g = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
  // whole quads only: the task count test is uniform across a quad
  if (g >= (uint64_t)w_cnt * nodes_out * slots_out) return;
  const uint32_t s = (uint32_t)(g % slots_out);
  const uint32_t t = (uint32_t)(g / slots_out);
  const uint32_t n = t % nodes_out, w = w_lo + t / nodes_out;
  const uint32_t* L = in + rec_index(w, nodes_in, 2 * n, slots_in, 0) * XYTZ_WORDS;
  const uint32_t* R = L + (size_t)slots_in * XYTZ_WORDS;
  const fe p2 = fe_const(kP2);
  fe r;
  if (s == h) {
    r = quad_ld(R + (size_t)h * XYTZ_WORDS);
  } else {
    const uint32_t src = (s < h) ? s : h;
    r = quad_add(quad_ld(L + (size_t)src * XYTZ_WORDS), quad_ld(R + (size_t)src * XYTZ_WORDS), p2);
  }
  if (to_u && s <= h) r = quad_to_u(r);
  quad_st(out + rec_index(w, nodes_out, n, slots_out, s) * XYTZ_WORDS, r);
}

// Per window: S_w = sum_t 2^t X_t (X_t in XYUZ form, slot t of the tree's
// root), by Horner's rule on one quad.  Writes S_w as XYTZ (record 2w) and
// XYUZ (record 2w + 1).
__global__ void __launch_bounds__(64) k_window_combine(const uint32_t* __restrict__ root,
                                                       uint32_t c, uint32_t w_lo, uint32_t w_cnt,
                                                       uint32_t* __restrict__ wsum) {
  const uint32_t wq = (blockIdx.x * blockDim.x + threadIdx.x) >> 2;
  if (wq >= w_cnt) return;
  const uint32_t w = w_lo + wq;
  const fe p2 = fe_const(kP2);
  const uint32_t* V = root + (size_t)w * (c + 1) * XYTZ_WORDS;
  fe acc = quad_add_u(quad_identity(), quad_ld(V + (size_t)(c - 1) * XYTZ_WORDS), p2);
  for (int t = (int)c - 2; t >= 0; --t) {
    acc = quad_dbl(acc, p2);
    acc = quad_add_u(acc, quad_ld(V + (size_t)t * XYTZ_WORDS), p2);
  }
  quad_st(wsum + (size_t)(2 * w) * XYTZ_WORDS, acc);
  quad_st(wsum + (size_t)(2 * w + 1) * XYTZ_WORDS, quad_to_u(acc));
}

// Group aggregation Q = sum_w 2^(w c) S_w by Horner's rule on one quad, over
// the windows w_hi down to w_lo of one group; the running value Q is kept in
// a record between groups (the top window starts it).
__global__ void __launch_bounds__(64) k_horner_steps(const uint32_t* __restrict__ wsum,
                                                     uint32_t W, uint32_t c, uint32_t w_lo,
                                                     uint32_t w_hi, uint32_t* __restrict__ state) {
  if (blockIdx.x != 0 || threadIdx.x >= 4) return;
  const fe p2 = fe_const(kP2);
  int w = (int)w_hi;
  fe q;
  if (w_hi == W - 1) {
    q = quad_ld(wsum + (size_t)(2 * w) * XYTZ_WORDS);
    --w;
  } else {
    q = quad_ld(state);
  }
  for (; w >= (int)w_lo; --w) {
    for (uint32_t t = 0; t < c; ++t) q = quad_dbl(q, p2);
    q = quad_add_u(q, quad_ld(wsum + (size_t)(2 * w + 1) * XYTZ_WORDS), p2);
  }
  quad_st(state, q);
}

// The affine Weierstrass result of the group-aggregation record.
__global__ void __launch_bounds__(64) k_finalize(const uint32_t* __restrict__ state,
                                                 const uint32_t* __restrict__ flags,
                                                 uint32_t* __restrict__ result) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  xytz Q = ld_xytz(state);
  fe xw, yw;
  bool fin = te_to_weierstrass(Q, xw, yw);
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    result[l] = xw.v[l];
    result[NL + l] = yw.v[l];
  }
  result[2 * NL] = fin ? 0u : 1u;
  result[2 * NL + 1] = flags ? *flags : 0u;
  for (int l = 2 * NL + 2; l < MSM_RESULT_WORDS; ++l) result[l] = 0u;
}

// below this many outputs a tree level runs on quads
constexpr uint64_t QUAD_BELOW = 16384;

}  // namespace

int launch_aggregate_group(const Plan& pl, int g, const uint32_t* buckets, void* ws,
                           hipStream_t st) {
  const uint32_t c = (uint32_t)pl.c;
  const uint32_t w_lo = (uint32_t)pl.group_lo(g), w_cnt = (uint32_t)(pl.group_hi(g) - pl.group_lo(g) + 1);
  uint32_t* lv[2] = {ws_at<uint32_t>(ws, pl.o_lvl0), ws_at<uint32_t>(ws, pl.o_lvl1)};
  uint32_t* wsum = ws_at<uint32_t>(ws, pl.o_wsum);
  ProfScope prof(PT_AGG, st);
  const uint32_t* in = buckets;
  uint32_t nodes = 1u << c;
  for (uint32_t h = 0; h < c; ++h) {
    uint32_t* out = lv[h & 1];
    const uint64_t outs = (uint64_t)w_cnt * (nodes >> 1) * (h + 2);
    const int to_u = (h + 1 == c) ? 1 : 0;
    if (outs >= QUAD_BELOW)
      k_tree_level<<<(unsigned)((outs + 255) / 256), 256, 0, st>>>(in, h, nodes, w_lo, w_cnt, out,
                                                                   to_u);
    else
      k_tree_level_quad<<<(unsigned)((4 * outs + 255) / 256), 256, 0, st>>>(in, h, nodes, w_lo,
                                                                           w_cnt, out, to_u);
    in = out;
    nodes >>= 1;
  }
  k_window_combine<<<grid_for(4 * (size_t)w_cnt, 64), 64, 0, st>>>(in, c, w_lo, w_cnt, wsum);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int launch_horner_group(const Plan& pl, int g, void* ws, hipStream_t st) {
  ProfScope prof(PT_HORNER, st);
  k_horner_steps<<<1, 64, 0, st>>>(ws_at<uint32_t>(ws, pl.o_wsum), (uint32_t)pl.W, (uint32_t)pl.c,
                                   (uint32_t)pl.group_lo(g), (uint32_t)pl.group_hi(g),
                                   ws_at<uint32_t>(ws, pl.o_qstate));
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int launch_finalize(const Plan& pl, uint32_t* result, void* ws, hipStream_t st) {
  ProfScope prof(PT_HORNER, st);
  k_finalize<<<1, 64, 0, st>>>(ws_at<uint32_t>(ws, pl.o_qstate), ws_at<uint32_t>(ws, pl.o_flags),
                               result);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // namespace msm
