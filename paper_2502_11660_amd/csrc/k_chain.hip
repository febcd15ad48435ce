// The paper's two PADD workloads outside an MSM (Sec. IV):
//
//  * latency: one accumulator adds the input points one after another, each
//    addition waiting for the previous one (the chain bucket and group
//    aggregation are made of); here on the four-lane latency unit or on one
//    lane, with the complete addition;
//  * throughput: many independent accumulators, each fed prepared points and
//    returning its sum once at the end (the shape of bucket accumulation),
//    with the mixed addition.
#include "common.hpp"
#include "quad.hpp"

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

// One lane: the same chain with the whole addition in one lane.
__global__ void __launch_bounds__(64) k_chain_lane(const uint32_t* __restrict__ pts,
                                                   uint32_t count, uint32_t* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const fe p2 = fe_const(kP2);
  xytz acc = pt_identity();
  xytz nxt = ld_xytz(pts);
  for (uint32_t i = 0; i < count; ++i) {
    const xytz cur = nxt;
    const uint32_t j = (i + 1 < count) ? i + 1 : i;
    nxt = ld_xytz(pts + (size_t)j * XYTZ_WORDS);
    acc = padd_full(acc, cur, p2);
  }
  st_xytz(out, acc);
}

// Accumulator a (one lane) sums the prepared points a, a + A, a + 2A, ...
// (consecutive lanes read consecutive records).
__global__ void __launch_bounds__(256) k_acc_stream(const uint32_t* __restrict__ xyu_pts,
                                                    uint32_t n, uint32_t A,
                                                    uint32_t* __restrict__ out) {
  const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A) return;
  const fe p2 = fe_const(kP2);
  xytz acc = pt_identity();
  if (a < n) {
    xyu nxt = ld_xyu(xyu_pts + (size_t)a * XYU_WORDS);
    for (uint32_t i = a; i < n; i += A) {
      const xyu cur = nxt;
      const uint32_t j = (i + A < n) ? i + A : i;
      nxt = ld_xyu(xyu_pts + (size_t)j * XYU_WORDS);
      acc = padd_mixed(acc, cur, p2);
    }
  }
  st_xytz(out + (size_t)a * XYTZ_WORDS, acc);
}

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
  k_acc_stream<<<grid_for(accumulators, 256), 256, 0, (hipStream_t)stream>>>(
      xyu, (uint32_t)n, (uint32_t)accumulators, out_xytz);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // extern "C"
