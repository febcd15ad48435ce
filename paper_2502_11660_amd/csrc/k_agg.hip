// Bucket aggregation and group aggregation (Sec. II-C).
//
// Bucket aggregation computes the window sum S_w = sum_b b B[w][b] (unsigned
// digits) or sum_m (m + 1) B[w][m] (signed digits: bucket m holds digit
// magnitude m + 1).  Writing the bucket index b in binary,
// sum_b b B[w][b] = sum_t 2^t X_t with X_t = sum of the buckets whose index
// has bit t set; signed digits add the sum of all buckets.
// The X_t are built by a binary tree over the bucket index: a node covering
// 2^h consecutive buckets keeps V[t] (t < h, the sum over its buckets with bit
// t set) and S (the sum of all its buckets).  Merging left child L and right
// child R gives V[t] = L.V[t] + R.V[t] (t < h), V[h] = R.S, S = L.S + R.S.
// Every output of a level is one independent addition, the whole tree costs
// about 2 * 2^c additions per window (as many as the running-sum method) and
// its dependent depth is only c additions.  Large levels run one addition per
// lane; small ones use the four-lane quad unit (quad.hpp) to cut latency.
//
// Each window then forms S_w by Horner's rule on one wide unit, and group
// aggregation Q = sum_w 2^(w c) S_w is Horner's rule over the windows of a job
// (c doublings per window), the dependent chain the paper assigns to its
// low-latency unit: one wide two-wave unit per job (wide_unit.hpp).  The
// result is mapped back to Weierstrass affine form.  A "window" below is a segment: one window of one
// job of the batch.
#include "common.hpp"
#include "convert.hpp"
#include "curve28.hpp"
#include "quad.hpp"
#include "wide_unit.hpp"

namespace msm {
namespace {

// record of node n, slot s at a tree level with `slots` slots per node
__device__ __forceinline__ size_t rec_index(uint32_t w, uint32_t nodes, uint32_t n, uint32_t slots,
                                            uint32_t s) {
  return ((size_t)w * nodes + n) * slots + s;
}

// One level h -> h+1, one addition per lane: addition a < h forms slot a,
// addition h the total (slot h + 1); the lane of addition 0 also copies
// slot h (= R.S), so that no lane of a wave idles through another's addition.
__global__ void __launch_bounds__(256) k_tree_level(const uint32_t* __restrict__ in, uint32_t h,
                                                    uint32_t nodes_in, uint32_t w_lo,
                                                    uint32_t w_cnt, uint32_t* __restrict__ out,
                                                    int to_u) {
  const uint32_t nodes_out = nodes_in >> 1, slots_in = h + 1, slots_out = h + 2;
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (uint64_t)w_cnt * nodes_out * slots_in) return;
  const uint32_t a = (uint32_t)(g % slots_in);
  const uint32_t t = (uint32_t)(g / slots_in);
  const uint32_t n = t % nodes_out, w = w_lo + t / nodes_out;
  const uint32_t* L = in + rec_index(w, nodes_in, 2 * n, slots_in, 0) * XYTZ_WORDS;
  const uint32_t* R = L + (size_t)slots_in * XYTZ_WORDS;
  uint32_t* O = out + rec_index(w, nodes_out, n, slots_out, 0) * XYTZ_WORDS;
  const fe p2 = fe_const(kP2);
  if (a == 0) {
    xytz c = ld_xytz(R + (size_t)h * XYTZ_WORDS);
    if (to_u) c.T = fe_mul(c.T, fe_const(kK));
    st_xytz(O + (size_t)h * XYTZ_WORDS, c);
  }
  const uint32_t s = a < h ? a : h + 1;  // output slot
  // the addition on the carry-free 28-bit form (curve28.hpp); U = k T there
  // uses k in that form, so U stays consistent with the point's scale
  xytz28 r = padd28_full(pt28_from(ld_xytz(L + (size_t)a * XYTZ_WORDS)),
                         pt28_from(ld_xytz(R + (size_t)a * XYTZ_WORDS)));
  if (to_u) r.T = f28_mul(r.T, f28_const(kK28));
  st_xytz(O + (size_t)s * XYTZ_WORDS, pt28_to_words(r));
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
  if (to_u) r = quad_to_u(r);
  quad_st(out + rec_index(w, nodes_out, n, slots_out, s) * XYTZ_WORDS, r);
}

// Same level, one wide unit (two waves) per output record, for levels with
// few outputs, where the latency of one addition sets the level's time.  The
// operands carry T (not U = k T), so the complete addition takes three
// product phases, four products per phase across the unit's four half-waves:
//   1: A = (Y1 - X1)(Y2 - X2), B = (Y1 + X1)(Y2 + X2), D = 2 Z1 Z2, V = T1 T2
//   2: C = k V, T3 = E H                      (E = B - A, H = B + A)
//   3: X3 = E F, Y3 = G H, Z3 = F G, T3 or U3 = k T3   (F = D - C, G = D + C)
// (subtractions add the pre-borrowed 3p).  The copy of R.S (output slot h)
// runs phase 3 alone on (X2, Y2, Z2, T2) times (1, 1, 1, 1 or k).  Every
// input below 2p gives products below 1.2p and product operands below 6p.
__global__ void __launch_bounds__(128) k_tree_level_wide(const uint32_t* __restrict__ in,
                                                         uint32_t h, uint32_t nodes_in,
                                                         uint32_t w_lo, uint32_t w_cnt,
                                                         uint32_t* __restrict__ out, int to_u) {
  __shared__ wunit_lds<2> s;
  const uint32_t nodes_out = nodes_in >> 1, slots_in = h + 1, slots_out = h + 2;
  const uint64_t g = blockIdx.x;  // one output record per block
  if (g >= (uint64_t)w_cnt * nodes_out * slots_out) return;
  const uint32_t slot = (uint32_t)(g % slots_out);
  const uint32_t t = (uint32_t)(g / slots_out);
  const uint32_t n = t % nodes_out, w = w_lo + t / nodes_out;
  const uint32_t src = slot < h ? slot : h;
  const uint32_t* L = in + rec_index(w, nodes_in, 2 * n, slots_in, src) * XYTZ_WORDS;
  const uint32_t* R = in + rec_index(w, nodes_in, 2 * n + 1, slots_in, src) * XYTZ_WORDS;
  wunit_init(s);
  // operand limbs: thread e loads limb e & 15 of coordinate (e >> 4) & 3 of
  // L (e < 64, into acc) or R (into opd[0])
  {
    const uint32_t e = threadIdx.x, coord = (e >> 4) & 3u, j = e & 15u;
    const limb_src v = wu_fetch(e < 64 ? L : R, coord, j);
    (e < 64 ? s.acc : s.opd[0])[16 * coord + j] = limb_extract(v, j);
  }
  unit_sync();
  const wslot q = wslot_here();
  const uint32_t wave = threadIdx.x >> 6;
  uint32_t* P1 = s.prod[0];  // A, B, D, V
  uint32_t* P2 = s.prod[1];  // C, T3
  uint32_t* O = s.opd[1];    // output X, Y, T or U, Z
  const uint32_t c3 = s.c3p[q.j];
  uint32_t l3, r3;           // this half's phase-3 operands
  if (slot == h) {
    const uint32_t* R2 = s.opd[0];
    l3 = q.k == 3 ? (to_u ? limb_of_const(kK, q.j) : limb_of_const(kOne, q.j))
                  : limb_of_const(kOne, q.j);
    r3 = R2[16 * (q.k == 2 ? 3u : (q.k == 3 ? 2u : q.k)) + q.j];  // X2, Y2, Z2, T2
  } else {
    {
      const uint32_t* X = s.acc;
      const uint32_t* Y = s.opd[0];
      const uint32_t x1 = X[q.j], y1 = X[16 + q.j], x2 = Y[q.j], y2 = Y[16 + q.j];
      uint32_t l = q.k == 0 ? (y1 + c3) - x1 : (q.k == 1 ? y1 + x1 : X[16 * (5u - q.k) + q.j]);
      uint32_t r = q.k == 0 ? (y2 + c3) - x2 : (q.k == 1 ? y2 + x2 : Y[16 * (5u - q.k) + q.j]);
      uint32_t v = wmul2_hi(q.act ? l : 0u, q.act ? r : 0u, s.mul[wave]);  // A, B, Z1 Z2, T1 T2
      if (q.k == 2) v <<= 1;                                               // D = 2 Z1 Z2
      if (!q.act) P1[16 * q.k + q.j] = v;
    }
    unit_sync();
    const uint32_t A = P1[q.j], B = P1[16 + q.j];
    if (wave == 0) {
      const uint32_t l = q.k == 0 ? limb_of_const(kK, q.j) : (B + c3) - A;
      const uint32_t r = q.k == 0 ? P1[48 + q.j] : B + A;
      const uint32_t v = wmul2_hi(q.act ? l : 0u, q.act ? r : 0u, s.mul[0]);  // C, T3
      if (!q.act) P2[16 * q.k + q.j] = v;
    }
    unit_sync();
    const uint32_t D = P1[32 + q.j], C = P2[q.j];
    const uint32_t E = (B + c3) - A, H = B + A, F = (D + c3) - C, G = D + C;
    l3 = q.k == 0 ? E : (q.k == 1 ? G : (q.k == 2 ? F : (to_u ? limb_of_const(kK, q.j)
                                                             : limb_of_const(kOne, q.j))));
    r3 = q.k == 0 ? F : (q.k == 1 ? H : (q.k == 2 ? G : P2[16 + q.j]));
  }
  const uint32_t v = wmul2_hi(q.act ? l3 : 0u, q.act ? r3 : 0u, s.mul[wave]);
  // X3, Y3, Z3, T3 / U3 to coordinates 0, 1, 3, 2
  if (!q.act) O[16 * (q.k == 2 ? 3u : (q.k == 3 ? 2u : q.k)) + q.j] = v;
  __syncthreads();  // the record's coordinates come from both waves
  const uint32_t lane = wlane();
  if (wave == 0 && lane < 4)
    st_aos(out + rec_index(w, nodes_out, n, slots_out, slot) * XYTZ_WORDS, (int)lane,
           words_of_limbs(O + 16 * lane));
}

// Per window (block w, one wide unit): S_w = sum_t 2^t X_t (+ S for signed
// digits) by Horner's rule over the bits t, with X_t (slot t < bb of the
// tree's root) and S (slot bb) in XYUZ form.  Writes S_w as XYTZ (record 2w)
// and XYUZ (record 2w + 1).  Each lane fetches its limb of the next slot
// while the current step runs.
__global__ void __launch_bounds__(128) k_window_combine(const uint32_t* __restrict__ root,
                                                        uint32_t bb, int add_total,
                                                        uint32_t* __restrict__ wsum) {
  __shared__ wunit_lds<2> s;
  const uint32_t w = blockIdx.x;
  wunit_init(s);  // accumulator = identity
  unit_sync();    // (written by wave 0 for both waves)
  const wslot q = wslot_here();
  const uint32_t* V = root + (size_t)w * (bb + 1) * XYTZ_WORDS;
  limb_src nxt = wu_fetch(V + (size_t)(bb - 1) * XYTZ_WORDS, q.k, q.j);
  const int steps = (int)bb + (add_total ? 1 : 0);
  uint32_t par = 0;
  for (int i = 0; i < steps; ++i) {
    // step i adds slot bb - 1 - i (i < bb) or the total (slot bb)
    const uint32_t* opd = s.opd[i & 1];
    // each lane writes the coordinate limb its own wave reads
    if (q.act) s.opd[i & 1][16 * q.k + q.j] = limb_extract(nxt, q.j);
    const int following = i + 1 < (int)bb ? (int)bb - 2 - i : (int)bb;  // clamped
    nxt = wu_fetch(V + (size_t)following * XYTZ_WORDS, q.k, q.j);
    wave_lds_sync();
    if (i >= 1 && i < (int)bb) wu_dbl(s, q, par);
    wu_add_u(s, opd, q, par);
  }
  __syncthreads();  // the accumulator's coordinates come from both waves
  if (threadIdx.x < 64) {
    // record 2w: XYTZ; record 2w + 1: XYUZ with U = k T (one more product,
    // in the first half of wave 0)
    wu_store_acc(s, wsum + (size_t)(2 * w) * XYTZ_WORDS);
    const bool h0 = q.k == 0 && q.act;
    const uint32_t u = wmul2(h0 ? s.acc[32 + q.j] : 0u, h0 ? limb_of_const(kK, q.j) : 0u, s.mul[0]);
    if (h0) s.prod[0][32 + q.j] = u;
    wave_lds_sync();
    const uint32_t lane = wlane();
    if (lane < 4) {
      const uint32_t* src = lane == 2 ? s.prod[0] + 32 : s.acc + 16 * lane;
      st_aos(wsum + (size_t)(2 * w + 1) * XYTZ_WORDS, (int)lane, words_of_limbs(src));
    }
  }
}

// Group aggregation of job j (block j, one wide unit): Q = sum_w 2^(w c) S_w
// by Horner's rule over the job's W windows.  Each lane loads its limb of the
// next window sum while the doublings of the current window run.
__global__ void __launch_bounds__(128) k_horner_wide(const uint32_t* __restrict__ wsum,
                                                     uint32_t W, uint32_t c,
                                                     uint32_t* __restrict__ qstate) {
  __shared__ wunit_lds<2> s;
  const uint32_t job = blockIdx.x;
  wunit_init(s);
  const wslot q = wslot_here();
  const uint32_t* ws = wsum + (size_t)2 * job * W * XYTZ_WORDS;
  const limb_src top = wu_fetch(ws + (size_t)(2 * (W - 1)) * XYTZ_WORDS, q.k, q.j);
  limb_src nxt = {0u, 0u};
  if (W >= 2) nxt = wu_fetch(ws + (size_t)(2 * W - 3) * XYTZ_WORDS, q.k, q.j);
  unit_sync();
  if (q.act) s.acc[16 * q.k + q.j] = limb_extract(top, q.j);  // S_{W-1}, XYTZ
  unit_sync();
  uint32_t par = 0;
  for (int w = (int)W - 2; w >= 0; --w) {
    // S_w, XYUZ (read after the doublings); then fetch S_{w-1}
    if (q.act) s.opd[0][16 * q.k + q.j] = limb_extract(nxt, q.j);
    if (w >= 1) nxt = wu_fetch(ws + (size_t)(2 * w - 1) * XYTZ_WORDS, q.k, q.j);
    for (uint32_t t = 0; t < c; ++t) wu_dbl(s, q, par);
    wu_add_u(s, s.opd[0], q, par);
  }
  __syncthreads();  // the accumulator's coordinates come from both waves
  if (threadIdx.x < 64) wu_store_acc(s, qstate + (size_t)job * XYTZ_WORDS);
}

// Twisted-Edwards extended (Montgomery form) -> Weierstrass affine, ordinary
// form, canonical, on one wave whose lanes all hold Q: the field inversion is
// lane-parallel (fe_inv_lanes) and the ten products around it run as wide
// products, two per step (one per half-wave), in five dependent steps:
//   d = (Z - Y) X, un = (Z + Y) X;   [d^-1]   im = d^-1 R^3 (Montgomery
//   inverse), vn = (Z + Y) Z;   u = un im, v = vn im;   u alpha, v beta;
//   x = (u alpha - 1) / R, y = v beta / R (out of Montgomery form).
// Returns false for the identity (x = y = 0 written).
__device__ bool wide_to_weierstrass(const xytz& Q, fe& xw, fe& yw, uint32_t* mul,
                                    uint32_t* stage) {
  if (fe_is_zero_canon(fe_canon(Q.X))) {
    xw = fe_zero();
    yw = fe_zero();
    return false;
  }
  const uint32_t lane = wlane(), h = lane >> 5, j = lane & 15u;
  const bool act = (lane & 31u) < 16u;
  const uint32_t c2p = 2u * kP24[j] + (j < 15 ? (1u << 26) : 0u) - (j >= 1 ? 4u : 0u);
  const uint32_t X = limb_of_const(Q.X.v, j), Y = limb_of_const(Q.Y.v, j),
                 Z = limb_of_const(Q.Z.v, j);
  // one step: half h multiplies its (l, r); the result limbs go to
  // stage[16 slot_h + j]
  auto step = [&](uint32_t l, uint32_t r, uint32_t slot0, uint32_t slot1) {
    const uint32_t v = wmul2_hi(act ? l : 0u, act ? r : 0u, mul);
    if (!act) stage[16 * (h ? slot1 : slot0) + j] = v;
    wave_lds_sync();
  };
  wmul2_init(mul);
  // stage slots: 0 d / im / u / u alpha / x, 1 un, 2 vn / v / v beta / y
  step(h ? Z + Y : (Z + c2p) - Y, X, 0, 1);  // d (< 1.2p), un
  const fe inv = fe_inv_lanes(fe_canon(words_of_limbs(stage)));
  const uint32_t iv = limb_of_const(inv.v, j);
  step(h ? Z + Y : iv, h ? Z : limb_of_const(kR3, j), 0, 2);  // im, vn
  step(h ? stage[32 + j] : stage[16 + j], stage[j], 0, 2);    // u, v
  step(stage[(h ? 32 : 0) + j], h ? limb_of_const(kBeta, j) : limb_of_const(kAlpha, j), 0, 2);
  const uint32_t am = (stage[j] + c2p) - limb_of_const(kOne, j);  // u alpha - 1 (Montgomery)
  step(h ? stage[32 + j] : am, j == 0 ? 1u : 0u, 0, 2);           // times 1 / R
  xw = fe_canon(words_of_limbs(stage));
  yw = fe_canon(words_of_limbs(stage + 32));
  return true;
}

// The affine Weierstrass result of each job, one wave per job (lane 0
// writes).
__global__ void __launch_bounds__(64) k_finalize(const uint32_t* __restrict__ qstate, JobView jv,
                                                 const uint32_t* __restrict__ flags) {
  __shared__ uint32_t mul[WMUL2_WORDS];
  __shared__ uint32_t stage[48];
  const uint32_t j = blockIdx.x;
  uint32_t* result = jv.get(j).result;
  xytz Q = ld_xytz(qstate + (size_t)j * XYTZ_WORDS);
  fe xw, yw;
  bool fin = wide_to_weierstrass(Q, xw, yw, mul, stage);
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    result[l] = xw.v[l];
    result[NL + l] = yw.v[l];
  }
  result[2 * NL] = fin ? 0u : 1u;
  result[2 * NL + 1] = flags[j];
  for (int l = 2 * NL + 2; l < MSM_RESULT_WORDS; ++l) result[l] = 0u;
}


}  // namespace

int launch_aggregate(const Plan& pl, const uint32_t* buckets, void* ws, hipStream_t st) {
  const uint32_t bb = (uint32_t)pl.bb, S = (uint32_t)pl.S;
  uint32_t* lv[2] = {ws_at<uint32_t>(ws, pl.o_lvl0), ws_at<uint32_t>(ws, pl.o_lvl1)};
  uint32_t* wsum = ws_at<uint32_t>(ws, pl.o_wsum);
  ProfScope prof(PT_AGG, st);
  const uint32_t* in = buckets;
  uint32_t nodes = 1u << bb;
  for (uint32_t h = 0; h < bb; ++h) {
    uint32_t* out = lv[h & 1];
    const uint64_t outs = (uint64_t)S * (nodes >> 1) * (h + 2);
    const int to_u = (h + 1 == bb) ? 1 : 0;
    const uint64_t adds = (uint64_t)S * (nodes >> 1) * (h + 1);
    // the schedule's unit thresholds (defaults: below 65536 outputs a level
    // runs on quads, up to 1024 outputs on wide units, one per output)
    if (outs >= pl.tree_quad)
      k_tree_level<<<(unsigned)((adds + 255) / 256), 256, 0, st>>>(in, h, nodes, 0, S, out, to_u);
    else if (outs > pl.tree_wide)
      k_tree_level_quad<<<(unsigned)((4 * outs + 255) / 256), 256, 0, st>>>(in, h, nodes, 0, S,
                                                                           out, to_u);
    else
      k_tree_level_wide<<<(unsigned)outs, 128, 0, st>>>(in, h, nodes, 0, S, out, to_u);
    in = out;
    nodes >>= 1;
  }
  k_window_combine<<<S, 128, 0, st>>>(in, bb, pl.encoding == MSM_DIGITS_UNSIGNED ? 0 : 1, wsum);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int launch_horner(const Plan& pl, void* ws, hipStream_t st) {
  ProfScope prof(PT_HORNER, st);
  const JobView jv = job_view(pl, ws);
  uint32_t* qstate = ws_at<uint32_t>(ws, pl.o_qstate);
  k_horner_wide<<<(unsigned)pl.J, 128, 0, st>>>(ws_at<uint32_t>(ws, pl.o_wsum), (uint32_t)pl.W,
                                                 (uint32_t)pl.c, qstate);
  k_finalize<<<(unsigned)pl.J, 64, 0, st>>>(qstate, jv, ws_at<uint32_t>(ws, pl.o_flags));
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // namespace msm
