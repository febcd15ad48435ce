// Wide field elements for latency-bound chains: one field element spread over
// 16 lanes as 16 limbs of 24 bits (limb j in lane j of its half-wave), in the
// same Montgomery representation as the 12-word form (R = 2^384 = 2^(16*24)).
//
// A lone wave issues one VALU instruction every few cycles whatever the
// dependencies, so a dependent chain of products runs at the instruction
// count of one product.  Spread over lanes, a product is 16 multiply-adds per
// lane for a b, 16 for the reduction digits and 16 for adding m p; a wave
// computes two products at once, one per 32-lane half (columns 0..31 of the
// half's product in its 32 lanes).  The reduction is separated from the
// product (no step waits on the previous digit):
//
//   T = a b                 m = (T mod R) q mod R  (q = -p^-1 mod R)
//   U = T + m p = 0 mod R   result = U / R
//
// Limbs are lazily normalised: an operand limb may be up to 2^28, values up
// to 8p; a product comes back with limbs at most 2^24 + 2^6 + 1 and value
// below a b / R + 1.001 p.
#pragma once
#include "field.hpp"

namespace msm {

constexpr uint32_t kLimbMask = 0xffffffu;

// 24-bit limbs of p and of q = -p^-1 mod 2^384
constexpr uint32_t kP24[16] = {0x000001u, 0xc00000u, 0x008508u, 0x300000u, 0x0b5d44u, 0x480017u,
                               0x2fba09u, 0x1ef362u, 0xf5138fu, 0xd9f300u, 0x3b1a22u, 0x6ca149u,
                               0x3b05c0u, 0x10eac6u, 0x4617c5u, 0x01ae3au};
constexpr uint32_t kQ24[16] = {0xffffffu, 0xbfffffu, 0x008508u, 0xa00000u, 0xe94577u, 0xebffd1u,
                               0x47970du, 0x35ed13u, 0xed7a13u, 0x5b86ccu, 0xec5b24u, 0x806a3cu,
                               0xf80141u, 0x2e3d22u, 0x5feec8u, 0xbfa520u};

__device__ __forceinline__ uint32_t wlane() { return __lane_id(); }

// shift by one lane towards higher lanes, lane 0 receiving 0 (bound_ctrl)
__device__ __forceinline__ uint32_t shr1z(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x138, 0xF, 0xF, true);
}

// one carry pass over 64-bit columns / 32-bit limbs: limb & mask plus the
// carry of the lane below
__device__ __forceinline__ uint64_t cpass64(uint64_t x) {
  const uint64_t c = x >> 24;
  return (x & kLimbMask) +
         ((uint64_t)shr1z((uint32_t)c) | ((uint64_t)shr1z((uint32_t)(c >> 32)) << 32));
}
__device__ __forceinline__ uint32_t cpass32(uint32_t x) { return (x & kLimbMask) + shr1z(x >> 24); }

// order this wave's LDS accesses (cross-lane exchange inside one wave)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS scratch of one wave for wmul2: words 0..63 hold the broadcast operands,
// then per half 16 zero words followed by the half's 32 shifted-operand words.
constexpr int WMUL2_WORDS = 160;

// zero the padding of a wmul2 scratch area (once, before its first use; the
// first wmul2 call orders it)
__device__ __forceinline__ void wmul2_init(uint32_t* lds) {
  const uint32_t lane = wlane();
  if (lane < 16) {
    lds[64 + lane] = 0u;
    lds[112 + lane] = 0u;
  }
}

// Two Montgomery products per wave: the half h = lane / 32 multiplies its own
// a and b, given as limbs in lanes 32h + j (j < 16) and zero in lanes
// 32h + 16 .. 32h + 31.  Limb j of the result comes back in lane 32h + 16 + j
// (zero in the half's lower 16 lanes).  Column j of a product is
// sum_i a_i b_{j-i}: a_i is an LDS broadcast, b_{j-i} an LDS read at a
// lane-shifted address (zero below the half's first lane).
__device__ __forceinline__ uint32_t wmul2_hi(uint32_t a, uint32_t b, uint32_t* lds) {
  const uint32_t lane = wlane(), h = lane >> 5, jj = lane & 31;
  const uint32_t* bc = lds + 16 * h;
  uint32_t* sh = lds + 80 + 48 * h;  // sh[jj - i] reaches the 16 zero words below
  wave_lds_sync();
  lds[16 * h + jj + (jj & 16)] = a;  // a of half h at words 16h .. 16h + 15
  sh[jj] = b;
  wave_lds_sync();
  uint32_t av[16], bv[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    av[i] = bc[i];
    bv[i] = sh[(int)jj - i];
  }
  uint64_t col = (uint64_t)av[0] * bv[0];
#pragma unroll
  for (int i = 1; i < 16; ++i) col += (uint64_t)av[i] * bv[i];
  // two passes: limbs below 2^24 + 2^12 (a column holds at most 2^60)
  const uint32_t t = (uint32_t)cpass64(cpass64(col));
  // m = (T mod R) q mod R: product columns 0..15 of the low half with q
  wave_lds_sync();
  sh[jj] = jj < 16 ? t : 0u;
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < 16; ++i) bv[i] = sh[(int)jj - i];
  uint64_t mc = (uint64_t)kQ24[0] * bv[0];
#pragma unroll
  for (int i = 1; i < 16; ++i) mc += (uint64_t)kQ24[i] * bv[i];
  mc = jj < 16 ? mc : 0u;  // mod R (and no carry into the other half)
  uint32_t m = cpass32((uint32_t)cpass64(mc));  // limbs below 2^24 + 2^6
  m = jj < 16 ? m : 0u;                          // m < R (1 + 2^-17)
  // U = T + m p (p_0 = 1)
  wave_lds_sync();
  sh[jj] = m;
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < 16; ++i) bv[i] = sh[(int)jj - i];
  uint64_t u = (uint64_t)t + bv[0];
#pragma unroll
  for (int i = 1; i < 16; ++i) u += (uint64_t)kP24[i] * bv[i];
  const uint32_t uv = cpass32((uint32_t)cpass64(u));  // limbs below 2^24 + 2^6
  // The low 16 limbs are 0 mod R and below 2R: all zero, or exactly R (then
  // one carry into limb 16).
  const uint64_t nz = __ballot(jj < 16 && uv != 0u);
  const bool carry = ((h ? (nz >> 32) : nz) & 0xffffu) != 0u;
  return jj >= 16 ? uv + ((jj == 16 && carry) ? 1u : 0u) : 0u;
}

// wmul2_hi with the result moved to the operand layout (lanes 32h + j)
__device__ __forceinline__ uint32_t wmul2(uint32_t a, uint32_t b, uint32_t* lds) {
  const uint32_t v = wmul2_hi(a, b, lds);
  // swap of the 16-lane groups within each 32 lanes
  const uint32_t r = (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);
  return (wlane() & 31u) < 16u ? r : 0u;
}

// The two words that hold limb j (bits 24j .. 24j + 23, j < 16) of a
// 12-word little-endian value, fetched without using them (so that a
// prefetch is not waited for until limb_extract); both loads stay inside the
// 12 words.
struct limb_src {
  uint32_t lo, hi;
};
__device__ __forceinline__ limb_src limb_fetch(const uint32_t* __restrict__ w, uint32_t j) {
  const uint32_t wi = (24u * j) >> 5;
  limb_src r;
  r.lo = w[wi];
  r.hi = w[wi + 1 < (uint32_t)NL ? wi + 1 : (uint32_t)NL - 1];  // unused when the limb fits in lo
  return r;
}
__device__ __forceinline__ uint32_t limb_extract(const limb_src& s, uint32_t j) {
  const uint32_t sh = (24u * j) & 31u;
  return (uint32_t)(((((uint64_t)s.hi) << 32) | s.lo) >> sh) & kLimbMask;
}

// limb j of a compile-time constant (selects, no memory)
__device__ __forceinline__ uint32_t limb_of_const(const uint32_t (&w)[NL], uint32_t j) {
  const uint32_t bit = 24u * j, wi = bit >> 5, sh = bit & 31u;
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (uint32_t i = 0; i < (uint32_t)NL; ++i) {
    lo = (i == wi) ? w[i] : lo;
    hi = (i == wi + 1) ? w[i] : hi;
  }
  return (uint32_t)(((((uint64_t)hi) << 32) | lo) >> sh) & kLimbMask;
}

// 12-word value of 16 lazily normalised limbs (value below 2^384), by an
// exact carry chain in one lane
__device__ __forceinline__ fe words_of_limbs(const uint32_t* limbs) {
  uint32_t n[16];
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const uint64_t t = (uint64_t)limbs[j] + c;
    n[j] = (uint32_t)t & kLimbMask;
    c = t >> 24;
  }
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int bit = 32 * i, j = bit / 24, sh = bit % 24;
    uint64_t v = (uint64_t)n[j] >> sh;
    if (j + 1 < 16) v |= (uint64_t)n[j + 1] << (24 - sh);
    if (j + 2 < 16 && 48 - sh < 32) v |= (uint64_t)n[j + 2] << (48 - sh);
    r.v[i] = (uint32_t)v;
  }
  return r;
}

}  // namespace msm
