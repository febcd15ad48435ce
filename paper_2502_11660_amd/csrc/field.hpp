// Base-field arithmetic for BLS12-377 on gfx950 (device code).
//
// An element is twelve little-endian 32-bit words held in VGPRs, in Montgomery
// form with R = 2^384.  The paper names Montgomery representation as the way
// to remove most exact carry propagation (Sec. V-C); its own design keeps
// intermediate values loosely reduced ("lazy" reduction, Sec. III-E).  The same
// idea is used here with Montgomery bounds instead of Barrett ones:
//
//   * REDC(a*b) < 2p whenever a*b < R*p.  Since R/p > 152, any operands with
//     a, b < 12p (or a product of bounds below 152 p^2) are safe.
//   * mul/sqr outputs are therefore kept in [0, 2p) and never conditionally
//     subtracted; add/sub results are left unreduced and the subtraction adds
//     2p so it never goes negative (the paper adds 3M for the same purpose).
//   * values are brought to canonical [0, p) only at the library boundary.
//
// Multiplication is product scanning with Montgomery reduction interleaved per
// column.  Each 32x32->64 product is added into a 64-bit column accumulator by
// one v_mad_u64_u32 whose carry-out is collected into a third word by one
// v_addc_co_u32: carries are saved per column and resolved once when the
// column retires, the carry-save idea of Sec. III-D applied to 32-bit words.
// p = 1 (mod 2^46) makes the per-word Montgomery factor -p^{-1} mod 2^32 equal
// to 0xffffffff and the low word of p equal to 1, so the reduction digit is
// m_k = -t_k and the m_k * p_0 product collapses to a borrow.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msm {

constexpr int NL = 12;  // 32-bit words per element

struct fe {
  uint32_t v[NL];
};

// p, 2p and Montgomery constants (little-endian words).
constexpr uint32_t kP[NL] = {0x00000001u, 0x8508c000u, 0x30000000u, 0x170b5d44u,
                             0xba094800u, 0x1ef3622fu, 0x00f5138fu, 0x1a22d9f3u,
                             0x6ca1493bu, 0xc63b05c0u, 0x17c510eau, 0x01ae3a46u};
constexpr uint32_t kP2[NL] = {0x00000002u, 0x0a118000u, 0x60000001u, 0x2e16ba88u,
                              0x74129000u, 0x3de6c45fu, 0x01ea271eu, 0x3445b3e6u,
                              0xd9429276u, 0x8c760b80u, 0x2f8a21d5u, 0x035c748cu};
constexpr uint32_t kP4[NL] = {0x00000004u, 0x14230000u, 0xc0000002u, 0x5c2d7510u,
                              0xe8252000u, 0x7bcd88beu, 0x03d44e3cu, 0x688b67ccu,
                              0xb28524ecu, 0x18ec1701u, 0x5f1443abu, 0x06b8e918u};
// R mod p: Montgomery form of 1.
constexpr uint32_t kOne[NL] = {0xffffff68u, 0x02cdffffu, 0x7fffffb1u, 0x51409f83u,
                               0x8a7d3ff2u, 0x9f7db3a9u, 0x6e7c6305u, 0x7b4e97b7u,
                               0x803c84e8u, 0x4cf495bfu, 0xe2fdf49au, 0x008d6661u};
// R^2 mod p: multiply-by to enter Montgomery form.
constexpr uint32_t kR2[NL] = {0x9400cd22u, 0xb786686cu, 0xb00431b1u, 0x0329fcaau,
                              0x62d6b46du, 0x22a5f111u, 0x827dc3acu, 0xbfdf7d03u,
                              0x41790bf9u, 0x837e92f0u, 0x1e914b88u, 0x006dfccbu};
// p - 2: the Fermat inversion exponent.
constexpr uint32_t kPm2[NL] = {0xffffffffu, 0x8508bfffu, 0x30000000u, 0x170b5d44u,
                               0xba094800u, 0x1ef3622fu, 0x00f5138fu, 0x1a22d9f3u,
                               0x6ca1493bu, 0xc63b05c0u, 0x17c510eau, 0x01ae3a46u};

__device__ __forceinline__ fe fe_const(const uint32_t (&c)[NL]) {
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.v[i] = c[i];
  return r;
}

__device__ __forceinline__ fe fe_zero() {
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.v[i] = 0u;
  return r;
}

// ---------------------------------------------------------------------------
// column multiply-accumulate primitives (acc: 64-bit column sum, hi: its
// deferred carry word)
// ---------------------------------------------------------------------------

// acc = a*b  (first product of column 0: no carry possible)
#define MSM_MUL0(acc, a, b) \
  asm("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(acc) : "v"(a), "v"(b) : "vcc")

// acc += a*b, hi = carry   (first product of a column)
#define MSM_MACF(acc, hi, a, b)                                       \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t"                          \
      "v_cndmask_b32_e64 %1, 0, 1, vcc"                                \
      : "+v"(acc), "=v"(hi)                                            \
      : "v"(a), "v"(b)                                                 \
      : "vcc")

// acc += a*b, hi += carry
#define MSM_MAC(acc, hi, a, b)                                        \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t"                          \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc"                          \
      : "+v"(acc), "+v"(hi)                                            \
      : "v"(a), "v"(b)                                                 \
      : "vcc")

// same with a scalar (wave-uniform) second operand
#define MSM_MACF_S(acc, hi, a, b)                                     \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t"                          \
      "v_cndmask_b32_e64 %1, 0, 1, vcc"                                \
      : "+v"(acc), "=v"(hi)                                            \
      : "v"(a), "s"(b)                                                 \
      : "vcc")
#define MSM_MAC_S(acc, hi, a, b)                                      \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t"                          \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc"                          \
      : "+v"(acc), "+v"(hi)                                            \
      : "v"(a), "s"(b)                                                 \
      : "vcc")

// Retire a reduction column (k < 12): m = -lo (mod 2^32); lo + m*p_0 = lo + m
// clears the low word with carry (lo != 0); the next column's accumulator is
// (acc_hi + carry) + (hi << 32).
__device__ __forceinline__ void redc_step(uint64_t& acc, uint32_t hi, uint32_t& m) {
  uint32_t lo = (uint32_t)acc, ah = (uint32_t)(acc >> 32);
  uint32_t nlo, nhi;
  asm("v_sub_co_u32_e32 %0, vcc, 0, %3\n\t"
      "v_addc_co_u32_e32 %1, vcc, 0, %4, vcc\n\t"
      "v_addc_co_u32_e32 %2, vcc, 0, %5, vcc"
      : "=&v"(m), "=&v"(nlo), "=&v"(nhi)
      : "v"(lo), "v"(ah), "v"(hi)
      : "vcc");
  acc = ((uint64_t)nhi << 32) | nlo;
}

// Column 0 variant: hi is known to be zero.
__device__ __forceinline__ void redc_step0(uint64_t& acc, uint32_t& m) {
  uint32_t lo = (uint32_t)acc, ah = (uint32_t)(acc >> 32);
  uint32_t nlo, nhi;
  asm("v_sub_co_u32_e32 %0, vcc, 0, %3\n\t"
      "v_addc_co_u32_e32 %1, vcc, 0, %4, vcc\n\t"
      "v_cndmask_b32_e64 %2, 0, 1, vcc"
      : "=&v"(m), "=&v"(nlo), "=&v"(nhi)
      : "v"(lo), "v"(ah)
      : "vcc");
  acc = ((uint64_t)nhi << 32) | nlo;
}

// Montgomery product r = a*b*R^{-1} mod p, lazily reduced.
// Requires a*b < R*p (e.g. a, b < 12p); returns r < 2p.
__device__ __forceinline__ fe fe_mul(const fe& a, const fe& b) {
  uint32_t m[NL];
  fe r;
  uint64_t acc;
  uint32_t hi;
  // column 0
  MSM_MUL0(acc, a.v[0], b.v[0]);
  redc_step0(acc, m[0]);
  // columns 1..11: a*b terms, m*p terms, then the reduction digit
#pragma unroll
  for (int k = 1; k < NL; ++k) {
    MSM_MACF(acc, hi, a.v[0], b.v[k]);
#pragma unroll
    for (int i = 1; i <= k; ++i) MSM_MAC(acc, hi, a.v[i], b.v[k - i]);
#pragma unroll
    for (int j = 0; j < k; ++j) MSM_MAC_S(acc, hi, m[j], kP[k - j]);
    redc_step(acc, hi, m[k]);
  }
  // columns 12..22 produce the result words
#pragma unroll
  for (int k = NL; k < 2 * NL - 1; ++k) {
    MSM_MACF(acc, hi, a.v[k - (NL - 1)], b.v[NL - 1]);
#pragma unroll
    for (int i = k - (NL - 1) + 1; i < NL; ++i) MSM_MAC(acc, hi, a.v[i], b.v[k - i]);
#pragma unroll
    for (int j = k - (NL - 1); j < NL; ++j) MSM_MAC_S(acc, hi, m[j], kP[k - j]);
    r.v[k - NL] = (uint32_t)acc;
    acc = ((uint64_t)hi << 32) | (acc >> 32);
  }
  r.v[NL - 1] = (uint32_t)acc;
  return r;
}

// Montgomery square.  With two VALU ops per product, the symmetric-product
// shortcut saves only a few percent once its doubling and merging work is
// counted, so squaring shares the multiply.
__device__ __forceinline__ fe fe_sqr(const fe& a) { return fe_mul(a, a); }

// ---------------------------------------------------------------------------
// unreduced add / subtract (12-word carry chains)
// ---------------------------------------------------------------------------

#define MSM_ADD0(r, cy, a, b) \
  asm("v_add_co_u32_e64 %0, %1, %2, %3" : "=v"(r), "=s"(cy) : "v"(a), "v"(b))
#define MSM_ADDC(r, cy, a, b, ci) \
  asm("v_addc_co_u32_e64 %0, %1, %2, %3, %4" : "=v"(r), "=s"(cy) : "v"(a), "v"(b), "s"(ci))
#define MSM_ADDC_LAST(r, a, b, ci) \
  asm("v_addc_co_u32_e64 %0, %1, %2, %3, %4" : "=v"(r), "=s"(dummy) : "v"(a), "v"(b), "s"(ci))
#define MSM_SUB0(r, cy, a, b) \
  asm("v_sub_co_u32_e64 %0, %1, %2, %3" : "=v"(r), "=s"(cy) : "v"(a), "v"(b))
#define MSM_SUBB(r, cy, a, b, ci) \
  asm("v_subb_co_u32_e64 %0, %1, %2, %3, %4" : "=v"(r), "=s"(cy) : "v"(a), "v"(b), "s"(ci))

// r = a + b (no reduction; caller guarantees a + b < 2^384)
__device__ __forceinline__ fe fe_add(const fe& a, const fe& b) {
  fe r;
  uint64_t cy, cy2, dummy;
  MSM_ADD0(r.v[0], cy, a.v[0], b.v[0]);
#pragma unroll
  for (int i = 1; i < NL - 1; ++i) {
    MSM_ADDC(r.v[i], cy2, a.v[i], b.v[i], cy);
    cy = cy2;
  }
  MSM_ADDC_LAST(r.v[NL - 1], a.v[NL - 1], b.v[NL - 1], cy);
  (void)dummy;
  return r;
}

// r = a - b + c where c is a constant multiple of p held in VGPRs and b <= c
// (so the result is non-negative); the caller guarantees a + c < 2^384.
__device__ __forceinline__ fe fe_sub_plus(const fe& a, const fe& b, const fe& c) {
  fe t, r;
  uint64_t cy, cy2, dummy;
  // t = c - b (no borrow out since b <= c)
  MSM_SUB0(t.v[0], cy, c.v[0], b.v[0]);
#pragma unroll
  for (int i = 1; i < NL; ++i) {
    MSM_SUBB(t.v[i], cy2, c.v[i], b.v[i], cy);
    cy = cy2;
  }
  // r = a + t
  MSM_ADD0(r.v[0], cy, a.v[0], t.v[0]);
#pragma unroll
  for (int i = 1; i < NL - 1; ++i) {
    MSM_ADDC(r.v[i], cy2, a.v[i], t.v[i], cy);
    cy = cy2;
  }
  MSM_ADDC_LAST(r.v[NL - 1], a.v[NL - 1], t.v[NL - 1], cy);
  (void)dummy;
  return r;
}

// r = a - b with the borrow returned as this wave's lane mask (bit set where
// a < b); consumed by fe_pick.
__device__ __forceinline__ fe fe_sub_mask(const fe& a, const fe& b, uint64_t& borrow) {
  fe r;
  uint64_t cy, cy2;
  MSM_SUB0(r.v[0], cy, a.v[0], b.v[0]);
#pragma unroll
  for (int i = 1; i < NL; ++i) {
    MSM_SUBB(r.v[i], cy2, a.v[i], b.v[i], cy);
    cy = cy2;
  }
  borrow = cy;
  return r;
}

// r = (lane bit of mask set) ? a : b
__device__ __forceinline__ fe fe_pick(uint64_t mask, const fe& a, const fe& b) {
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i)
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r.v[i]) : "v"(b.v[i]), "v"(a.v[i]), "s"(mask));
  return r;
}

__device__ __forceinline__ fe fe_select(bool c, const fe& a, const fe& b) {
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.v[i] = c ? a.v[i] : b.v[i];
  return r;
}

// Reduce any value < 8p to canonical [0, p).
__device__ __forceinline__ fe fe_canon(const fe& a) {
  fe x = a;
  uint64_t br;
  fe t = fe_sub_mask(x, fe_const(kP4), br);
  x = fe_pick(br, x, t);
  t = fe_sub_mask(x, fe_const(kP2), br);
  x = fe_pick(br, x, t);
  t = fe_sub_mask(x, fe_const(kP), br);
  x = fe_pick(br, x, t);
  return x;
}

__device__ __forceinline__ bool fe_is_zero_canon(const fe& a) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) o |= a.v[i];
  return o == 0;
}

__device__ __forceinline__ bool fe_eq_canon(const fe& a, const fe& b) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) o |= a.v[i] ^ b.v[i];
  return o == 0;
}

__device__ __forceinline__ fe fe_to_mont(const fe& a) { return fe_mul(a, fe_const(kR2)); }

__device__ __forceinline__ fe fe_from_mont(const fe& a) {
  fe one = fe_zero();
  one.v[0] = 1u;
  return fe_canon(fe_mul(a, one));
}

// Inverse by Fermat: a^(p-2), left-to-right square-and-multiply over the bits
// of p - 2.  Input in Montgomery form (any lazily reduced value < 12p), output
// in Montgomery form, < 2p.  Zero maps to zero.
__device__ __noinline__ fe fe_inv(const fe& a) {
  fe r = a;  // top bit of p-2 (bit 376) is set
  for (int bit = 375; bit >= 0; --bit) {
    r = fe_sqr(r);
    if ((kPm2[bit >> 5] >> (bit & 31)) & 1u) r = fe_mul(r, a);
  }
  return r;
}

}  // namespace msm
