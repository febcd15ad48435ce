// Latency-oriented point arithmetic: four lanes per point (device code).
//
// Bucket and group aggregation are chains of dependent additions (Sec. II-C);
// the paper serves them with a separate low-latency PADD mapping, apart from
// the throughput mapping used for bucket accumulation (Sec. V-A).  On the GPU
// the latency of one addition done by one lane is the length of its
// instruction stream, so here four consecutive lanes ("a quad") share one
// point: lane q of the quad holds coordinate q (0: X, 1: Y, 2: T or U = kT,
// 3: Z).  The addition has four independent multiplications per phase, so
// each lane does one Montgomery multiply per phase; the four products are
// exchanged with DPP quad broadcasts (one instruction per word).  The quad
// serves the small levels of the aggregation tree (many independent
// additions per launch); the long chains run on the wider unit of
// wide_unit.hpp.
//
//   addition, both XYTZ            3 phases  (extra k * (T1 T2) on lane 2)
//
// All lanes of a quad must be active.  Values follow the lazy-reduction
// bounds of curve.hpp: every coordinate stays below 2p.
#pragma once
#include "curve.hpp"

namespace msm {

__device__ __forceinline__ int quad_lane() { return (int)(threadIdx.x & 3u); }

// broadcast lane K of the quad to all four lanes
template <int K>
__device__ __forceinline__ fe qbcast(const fe& v) {
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i)
    r.v[i] = (uint32_t)__builtin_amdgcn_mov_dpp((int)v.v[i], K * 0x55, 0xF, 0xF, false);
  return r;
}

// lane-dependent choice among four values
__device__ __forceinline__ fe qpick(int q, const fe& a0, const fe& a1, const fe& a2, const fe& a3) {
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    uint32_t lo = (q & 1) ? a1.v[i] : a0.v[i];
    uint32_t hi = (q & 1) ? a3.v[i] : a2.v[i];
    r.v[i] = (q & 2) ? hi : lo;
  }
  return r;
}

// Phase-2 step shared by all additions and the doubling: from the lane's
// phase-1 product (lane 0: A, lane 1: B, lane 2: C, lane 3: D) form
// E = B - A, F = D - C, G = D + C, H = B + A and return this lane's
// coordinate of (E F, G H, E H, F G).
__device__ __forceinline__ fe quad_finish(int q, const fe& prod, const fe& p2) {
  fe A = qbcast<0>(prod);
  fe B = qbcast<1>(prod);
  fe C = qbcast<2>(prod);
  fe D = qbcast<3>(prod);
  fe E = fe_sub_plus(B, A, p2);  // < 4p
  fe F = fe_sub_plus(D, C, p2);  // < 6p
  fe G = fe_add(D, C);           // < 6p
  fe H = fe_add(B, A);           // < 4p
  fe l = qpick(q, E, G, E, F);
  fe r = qpick(q, F, H, H, G);
  return fe_mul(l, r);
}

// P1 + P2, both XYTZ.
__device__ __forceinline__ fe quad_add(const fe& p1, const fe& p2v, const fe& p2) {
  const int q = quad_lane();
  fe X1 = qbcast<0>(p1), Y1 = qbcast<1>(p1);
  fe X2 = qbcast<0>(p2v), Y2 = qbcast<1>(p2v);
  fe l = qpick(q, fe_sub_plus(Y1, X1, p2), fe_add(Y1, X1), p1, p1);
  fe r = qpick(q, fe_sub_plus(Y2, X2, p2), fe_add(Y2, X2), p2v, p2v);
  fe m = fe_mul(l, r);                 // A, B, T1 T2, Z1 Z2
  fe s = (q == 2) ? fe_const(kK) : fe_const(kOne);
  m = fe_mul(m, s);                    // C = k T1 T2 on lane 2, unchanged elsewhere
  m = fe_select(q == 3, fe_add(m, m), m);
  return quad_finish(q, m, p2);
}

// T -> U = k T on lane 2 of the quad (XYTZ -> XYUZ); one phase.
__device__ __forceinline__ fe quad_to_u(const fe& pc) {
  const int q = quad_lane();
  fe s = (q == 2) ? fe_const(kK) : fe_const(kOne);
  return fe_mul(pc, s);
}

// identity (0, 1, 0, 1): coordinate q
__device__ __forceinline__ fe quad_identity() {
  const int q = quad_lane();
  return (q == 1 || q == 3) ? fe_const(kOne) : fe_zero();
}

// coordinate q of an XYTZ record
__device__ __forceinline__ fe quad_ld(const uint32_t* __restrict__ rec) {
  return ld_aos(rec, quad_lane());
}

__device__ __forceinline__ void quad_st(uint32_t* __restrict__ rec, const fe& v) {
  st_aos(rec, quad_lane(), v);
}

}  // namespace msm
