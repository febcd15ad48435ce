// The paper's two PADD workloads outside an MSM (Sec. IV):
//
//  * latency: one accumulator adds the input points one after another, each
//    addition waiting for the previous one (the chain bucket and group
//    aggregation are made of); here on the wide two-wave unit, the four-lane
//    unit or one lane, with the complete addition;
//  * throughput: many independent accumulators, each fed prepared points and
//    returning its sum once at the end (the shape of bucket accumulation),
//    with the mixed addition.
#include "common.hpp"
#include "curve28.hpp"
#include "quad.hpp"
#include "wide_unit.hpp"

namespace msm {
namespace {

// One quad: acc = sum of the count XYTZ records, in order.
__global__ void __launch_bounds__(64) k_chain_quad(const uint32_t* __restrict__ pts,
                                                   uint32_t count, uint32_t* __restrict__ out) {
  if (threadIdx.x >= 4) return;
  const fe p2 = fe_const(kP2);
  fe acc = quad_identity();
  fe nxt = quad_ld(pts);
  for (uint32_t i = 0; i < count; ++i) {
    const fe cur = nxt;
    const uint32_t j = (i + 1 < count) ? i + 1 : i;
    nxt = quad_ld(pts + (size_t)j * XYTZ_WORDS);
    acc = quad_add(acc, cur, p2);
  }
  quad_st(out, acc);
}

// One lane: the same chain with the whole addition in one lane (the
// throughput unit's carry-free 28-bit form).
__global__ void __launch_bounds__(64) k_chain_lane(const uint32_t* __restrict__ pts,
                                                   uint32_t count, uint32_t* __restrict__ out) {
  if (threadIdx.x != 0) return;
  xytz28 acc = pt28_identity();
  xytz nxt = ld_xytz(pts);
  for (uint32_t i = 0; i < count; ++i) {
    const xytz28 cur = pt28_from(nxt);
    const uint32_t j = (i + 1 < count) ? i + 1 : i;
    nxt = ld_xytz(pts + (size_t)j * XYTZ_WORDS);
    acc = padd28_full(acc, cur);
  }
  st_xytz(out, pt28_to_words(acc));
}

// The wide unit: waves 0 and 1 run the additions (two phases of four
// products); wave 2 prepares the next operand (U = k T, one product) while
// they add the current one, and fetches the point after that.  Its slot
// write comes before the step's single unit_sync, which orders it before the
// next step's first phase (and after the previous reads of that slot).
__global__ void __launch_bounds__(192) k_chain_wide(const uint32_t* __restrict__ pts,
                                                    uint32_t count, uint32_t* __restrict__ out) {
  __shared__ wunit_lds<3> s;
  wunit_init(s);
  const wslot q = wslot_here();
  const bool prep = (threadIdx.x >> 6) == 2;
  const bool ld = prep && q.k == 4 && q.act;  // the prep wave's first half fetches
  const uint32_t kk = limb_of_const(kK, q.j);
  limb_src f[4];  // raw words of the point after the one being prepared
  uint32_t c[4];  // limbs of the point being prepared
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c[k] = limb_extract(wu_fetch(pts, k, q.j), q.j);
    f[k] = wu_fetch(pts + (count > 1 ? XYTZ_WORDS : 0), k, q.j);
  }
  unit_sync();  // scratch padding and constants
  if (prep) {
    const uint32_t u = wmul2(ld ? c[2] : 0u, ld ? kk : 0u, s.mul[2]);
    if (ld) {
      s.opd[0][q.j] = c[0];
      s.opd[0][16 + q.j] = c[1];
      s.opd[0][32 + q.j] = u;
      s.opd[0][48 + q.j] = c[3];
    }
  }
  unit_sync();
  uint32_t par = 0;
  for (uint32_t i = 0; i < count; ++i) {
    if (!prep) {
      wu_add_u(s, s.opd[i & 1], q, par);  // one unit_sync per step
    } else {
      // Unconditional and clamped (past the end it prepares a slot nobody
      // reads): a conditional fetch would make the compiler copy the fresh
      // registers at the merge and wait for the loads there.
#pragma unroll
      for (int k = 0; k < 4; ++k) c[k] = limb_extract(f[k], q.j);  // point i + 1
      const uint32_t nx = i + 2 < count ? i + 2 : count - 1;
#pragma unroll
      for (int k = 0; k < 4; ++k) f[k] = wu_fetch(pts + (size_t)nx * XYTZ_WORDS, k, q.j);
      const uint32_t u = wmul2(ld ? c[2] : 0u, ld ? kk : 0u, s.mul[2]);
      uint32_t* o = s.opd[(i + 1) & 1];
      if (ld) {
        o[q.j] = c[0];
        o[16 + q.j] = c[1];
        o[32 + q.j] = u;
        o[48 + q.j] = c[3];
      }
      unit_sync();  // the one sync of wu_add_u (the slot is written before it)
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) wu_store_acc(s, out);
}

// Accumulator a (one lane) sums the prepared points a, a + A, a + 2A, ...
// (consecutive lanes read consecutive records), on the carry-free 28-bit
// form like bucket accumulation.
__global__ void __launch_bounds__(256) k_acc_stream(const uint32_t* __restrict__ xyu_pts,
                                                    uint32_t n, uint32_t A,
                                                    uint32_t* __restrict__ out) {
  const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A) return;
  xytz28 acc = pt28_identity();
  // no prefetch of the next record: it would cost a wave per SIMD, and three
  // resident waves cover the load latency
  for (uint32_t i = a; i < n; i += A)
    acc = padd28_mixed(acc, pt28_from(ld_xyu(xyu_pts + (size_t)i * XYU_WORDS)));
  st_xytz(out + (size_t)a * XYTZ_WORDS, pt28_to_words(acc));
}

// Few accumulators: one wide unit per accumulator (block a) instead of one
// lane, so each step costs the wide unit's latency instead of a lane's.  The
// prepared point is the addition's second operand with Z2 = 1; each lane
// fetches its limb of the next point while the current addition runs.
__global__ void __launch_bounds__(128) k_acc_stream_wide(const uint32_t* __restrict__ xyu_pts,
                                                         uint32_t n, uint32_t A,
                                                         uint32_t* __restrict__ out) {
  __shared__ wunit_lds<2> s;
  const uint32_t a = blockIdx.x;
  wunit_init(s);
  const wslot q = wslot_here();
  const uint32_t one = limb_of_const(kOne, q.j);
  const uint32_t coord = q.k < 3 ? q.k : 0u;  // X, Y, U words of the record; Z2 = 1
  limb_src nxt = limb_fetch(xyu_pts + (size_t)(a < n ? a : 0u) * XYU_WORDS + coord * NL, q.j);
  unit_sync();
  uint32_t par = 0, step = 0;
  for (uint32_t i = a; i < n; i += A, ++step) {
    uint32_t* o = s.opd[step & 1];
    if (q.act) o[16 * q.k + q.j] = q.k == 3 ? one : limb_extract(nxt, q.j);
    const uint32_t nx = i + A < n ? i + A : i;  // clamped: loaded, not used
    nxt = limb_fetch(xyu_pts + (size_t)nx * XYU_WORDS + coord * NL, q.j);
    wave_lds_sync();  // each wave reads the coordinates its own lanes wrote
    wu_add_u(s, o, q, par);
  }
  __syncthreads();  // the accumulator's coordinates come from both waves
  if (threadIdx.x < 64) wu_store_acc(s, out + (size_t)a * XYTZ_WORDS);
}

// up to this many accumulators the stream runs on wide units
constexpr size_t STREAM_WIDE_UPTO = 1024;

}  // namespace
}  // namespace msm

using namespace msm;

extern "C" {

int msm_padd_chain(const uint32_t* pts_xytz, size_t count, int unit, uint32_t* out_xytz,
                   void* stream) {
  if (!pts_xytz || !out_xytz || count == 0 || count >= (1u << 31)) return MSM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (unit == MSM_UNIT_QUAD)
    k_chain_quad<<<1, 64, 0, st>>>(pts_xytz, (uint32_t)count, out_xytz);
  else if (unit == MSM_UNIT_LANE)
    k_chain_lane<<<1, 64, 0, st>>>(pts_xytz, (uint32_t)count, out_xytz);
  else if (unit == MSM_UNIT_WIDE)
    k_chain_wide<<<1, 192, 0, st>>>(pts_xytz, (uint32_t)count, out_xytz);
  else
    return MSM_EINVAL;
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int msm_accumulate_stream(const uint32_t* xyu, size_t n, size_t accumulators, uint32_t* out_xytz,
                          void* stream) {
  if (!xyu || !out_xytz || n == 0 || n >= (1u << 31) || accumulators == 0 ||
      accumulators >= (1u << 31))
    return MSM_EINVAL;
  if (accumulators <= STREAM_WIDE_UPTO)
    k_acc_stream_wide<<<(unsigned)accumulators, 128, 0, (hipStream_t)stream>>>(
        xyu, (uint32_t)n, (uint32_t)accumulators, out_xytz);
  else
    k_acc_stream<<<grid_for(accumulators, 256), 256, 0, (hipStream_t)stream>>>(
        xyu, (uint32_t)n, (uint32_t)accumulators, out_xytz);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // extern "C"
