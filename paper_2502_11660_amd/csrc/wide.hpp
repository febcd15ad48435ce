// Wide field elements for latency-bound chains: one wave holds one element
// as 16 limbs of 24 bits, limb j in lane j (lanes 16..63 hold zero), the
// same Montgomery representation (R = 2^384 = 2^(16*24)) as the 12-word
// form, so every lazy-reduction bound of curve.hpp carries over.
//
// A lone wave issues about one VALU instruction per 4-10 cycles whatever the
// dependencies, so a dependent chain of products is as fast as the
// instruction count of one product.  Spread over lanes, a product takes 16
// multiply-adds per lane for a*b (one broadcast factor per step, the other
// shifted one lane per step) and 16 more for the reduction, whose digits
// m_k = -t_k mod 2^24 (p = 1 mod 2^46) are formed on the scalar unit from
// the column value read out of lane k.
#pragma once
#include "field.hpp"

namespace msm {

constexpr uint32_t kLimbMask = 0xffffffu;

struct wfe {
  uint32_t v;  // this lane's limb (zero above lane 15)
};

__device__ __forceinline__ uint32_t wlane() { return __lane_id(); }

// lane k's value (the builtin returns a signed int: keep it unsigned)
__device__ __forceinline__ uint32_t rlane(uint32_t v, int k) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, k);
}

// DPP wave shift by one lane towards higher lanes (lane 0 receives 0)
__device__ __forceinline__ uint32_t wave_shr1(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138, 0xF, 0xF, false);
}

// limb j of the 12-word value w (all lanes read; lanes >= 16 get 0)
__device__ __forceinline__ wfe wfe_from_words(const fe& w) {
  const uint32_t j = wlane();
  const uint32_t bit = 24 * j, wi = bit >> 5, sh = bit & 31;
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    lo = ((uint32_t)i == wi) ? w.v[i] : lo;
    hi = ((uint32_t)i == wi + 1) ? w.v[i] : hi;
  }
  const uint64_t two = ((uint64_t)hi << 32) | lo;
  wfe r;
  r.v = j < 16 ? (uint32_t)(two >> sh) & kLimbMask : 0u;
  return r;
}

// Carry-normalise limbs (each pass moves limb >> 24 one lane up).  With
// limbs below 2^32 three passes leave every limb below 2^24 + 2^9; the top
// limb keeps what reaches it (the value is below 2^384).
__device__ __forceinline__ uint32_t wnorm32(uint32_t x) {
#pragma unroll
  for (int pass = 0; pass < 3; ++pass) {
    const uint32_t c = wave_shr1(x >> 24);
    x = (wlane() < 15 ? (x & kLimbMask) : x) + (wlane() < 16 ? c : 0u);
    x = wlane() < 16 ? x : 0u;
  }
  return x;
}

// Fully reduced 12-word form of w (< 2^384) for storing: exact carry
// propagation on the scalar unit, then packing.
__device__ __forceinline__ fe wfe_to_words(const wfe& w) {
  uint64_t carry = 0;
  uint32_t limb[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const uint64_t t = (uint64_t)rlane(w.v, j) + carry;
    limb[j] = (uint32_t)t & kLimbMask;
    carry = t >> 24;
  }
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int bit = 32 * i, j = bit / 24, sh = bit % 24;
    uint64_t v = (uint64_t)limb[j] >> sh;
    if (j + 1 < 16) v |= (uint64_t)limb[j + 1] << (24 - sh);
    if (j + 2 < 16 && 48 - sh < 32) v |= (uint64_t)limb[j + 2] << (48 - sh);
    r.v[i] = (uint32_t)v;
  }
  return r;
}

// Montgomery product a b R^-1 (R = 2^384), lazily reduced (< 2p when
// a b < R p); limbs of a and b at most 2^27.
__device__ __forceinline__ wfe wfe_mul(const wfe& a, const wfe& b) {
  const uint32_t lane = wlane();
  // columns 0..31 of a*b, column j in lane j: sum_i a_i b_{j-i}
  uint64_t col = 0;
  uint32_t bs = b.v;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const uint32_t ai = rlane(a.v, i);
    col += (uint64_t)ai * bs;
    bs = wave_shr1(bs);
  }
  // reduction: m_k = -(column k + carry) mod 2^24; column k + j += m_k p_j
  uint32_t ps = wfe_from_words(fe_const(kP)).v;  // p_j in lane j
  uint64_t carry = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const uint64_t ck = ((uint64_t)rlane((uint32_t)(col >> 32), k) << 32) | rlane((uint32_t)col, k);
    const uint64_t t = ck + carry;
    uint32_t m = (0u - (uint32_t)t) & kLimbMask;
    // opaque to the optimiser: otherwise it treats the product as a 24-bit
    // multiply, drops the mask, and then emits a full 32-bit multiply-add
    asm volatile("" : "+s"(m));
    carry = (t + m) >> 24;
    col += (uint64_t)m * ps;  // lane k + j gets m p_j (lane k itself is retired)
    ps = wave_shr1(ps);
  }
  // result limbs: columns 16..31 (+ carry into column 16), moved to lanes 0..15
  const uint32_t lo = (uint32_t)col, hi = (uint32_t)(col >> 32);
  const uint32_t lo_d = (uint32_t)__builtin_amdgcn_ds_swizzle((int)lo, 0x401F);
  const uint32_t hi_d = (uint32_t)__builtin_amdgcn_ds_swizzle((int)hi, 0x401F);
  uint64_t r = lane < 16 ? (((uint64_t)hi_d << 32) | lo_d) : 0u;
  r += lane == 0 ? carry : 0u;
  // carry normalisation: two 64-bit passes bring the limbs below 2^32 (the
  // top limb keeps its carries: the value is below 2^384), then three more
  uint64_t x = r;
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const uint64_t c = (uint64_t)wave_shr1((uint32_t)(x >> 24)) |
                       ((uint64_t)wave_shr1((uint32_t)(x >> 56)) << 32);
    x = (lane < 15 ? (x & kLimbMask) : x) + (lane < 16 ? c : 0u);
  }
  wfe out;
  out.v = wnorm32(lane < 16 ? (uint32_t)x : 0u);
  return out;
}

}  // namespace msm
