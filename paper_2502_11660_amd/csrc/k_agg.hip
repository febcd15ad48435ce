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
                                                    uint32_t nodes_in, uint32_t W,
                                                    uint32_t* __restrict__ out, int to_u) {
  const uint32_t nodes_out = nodes_in >> 1, slots_in = h + 1, slots_out = h + 2;
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (uint64_t)W * nodes_out * slots_out) return;
  const uint32_t s = (uint32_t)(g % slots_out);
  const uint32_t t = (uint32_t)(g / slots_out);
  const uint32_t n = t % nodes_out, w = t / nodes_out;
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
                                                         uint32_t nodes_in, uint32_t W,
                                                         uint32_t* __restrict__ out, int to_u) {
  const uint32_t nodes_out = nodes_in >> 1, slots_in = h + 1, slots_out = h + 2;
  const uint64_t g = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
  // whole quads only: the task count test is uniform across a quad
  if (g >= (uint64_t)W * nodes_out * slots_out) return;
  const uint32_t s = (uint32_t)(g % slots_out);
  const uint32_t t = (uint32_t)(g / slots_out);
  const uint32_t n = t % nodes_out, w = t / nodes_out;
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
                                                       uint32_t c, uint32_t W,
                                                       uint32_t* __restrict__ wsum) {
  const uint32_t w = (blockIdx.x * blockDim.x + threadIdx.x) >> 2;
  if (w >= W) return;
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

// Group aggregation Q = sum_w 2^(w c) S_w by Horner's rule on one quad, then
// the affine Weierstrass result (one lane).
__global__ void __launch_bounds__(64) k_horner(const uint32_t* __restrict__ wsum, uint32_t W,
                                               uint32_t c, const uint32_t* __restrict__ flags,
                                               uint32_t* __restrict__ result) {
  if (blockIdx.x != 0 || threadIdx.x >= 4) return;
  const fe p2 = fe_const(kP2);
  fe q = quad_ld(wsum + (size_t)(2 * (W - 1)) * XYTZ_WORDS);
  for (int w = (int)W - 2; w >= 0; --w) {
    for (uint32_t t = 0; t < c; ++t) q = quad_dbl(q, p2);
    q = quad_add_u(q, quad_ld(wsum + (size_t)(2 * w + 1) * XYTZ_WORDS), p2);
  }
  xytz Q;
  Q.X = qbcast<0>(q);
  Q.Y = qbcast<1>(q);
  Q.T = qbcast<2>(q);
  Q.Z = qbcast<3>(q);
  if (threadIdx.x != 0) return;
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

int launch_aggregate(const Plan& pl, const uint32_t* buckets, uint32_t* result, void* ws,
                     hipStream_t st) {
  const uint32_t W = (uint32_t)pl.W, c = (uint32_t)pl.c;
  uint32_t* lv[2] = {ws_at<uint32_t>(ws, pl.o_lvl0), ws_at<uint32_t>(ws, pl.o_lvl1)};
  uint32_t* wsum = ws_at<uint32_t>(ws, pl.o_wsum);
  {
    ProfScope prof(PT_AGG, st);
    const uint32_t* in = buckets;
    uint32_t nodes = 1u << c;
    for (uint32_t h = 0; h < c; ++h) {
      uint32_t* out = lv[h & 1];
      const uint64_t outs = (uint64_t)W * (nodes >> 1) * (h + 2);
      const int to_u = (h + 1 == c) ? 1 : 0;
      if (outs >= QUAD_BELOW)
        k_tree_level<<<(unsigned)((outs + 255) / 256), 256, 0, st>>>(in, h, nodes, W, out, to_u);
      else
        k_tree_level_quad<<<(unsigned)((4 * outs + 255) / 256), 256, 0, st>>>(in, h, nodes, W, out,
                                                                             to_u);
      in = out;
      nodes >>= 1;
    }
    k_window_combine<<<grid_for(4 * (size_t)W, 64), 64, 0, st>>>(in, c, W, wsum);
  }
  {
    ProfScope prof(PT_HORNER, st);
    k_horner<<<1, 64, 0, st>>>(wsum, W, c, ws_at<uint32_t>(ws, pl.o_flags), result);
  }
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // namespace msm
