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

// Grouped multiply-adds: n products of one column in one asm block.  The
// compiler separates consecutive asm blocks by a wait state, which a lone
// wave (the latency-bound aggregation chains) pays in full, so a column's
// products are issued a group of up to eight at a time.  MACN adds to the
// deferred carry word hi; MACFN starts it from the first product's carry.
// The first factor is a VGPR; CB is the second factor's constraint ("v" for
// a VGPR, "s" for an SGPR such as a constant of p).
#define MSM_MACN_1(CB, acc, hi, a0, b0) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "+v"(hi) \
      : "v"(a0), CB(b0) \
      : "vcc")

#define MSM_MACN_2(CB, acc, hi, a0, b0, a1, b1) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "+v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1) \
      : "vcc")

#define MSM_MACN_3(CB, acc, hi, a0, b0, a1, b1, a2, b2) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "+v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2) \
      : "vcc")

#define MSM_MACN_4(CB, acc, hi, a0, b0, a1, b1, a2, b2, a3, b3) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "+v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3) \
      : "vcc")

#define MSM_MACN_5(CB, acc, hi, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %10, %11, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "+v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4) \
      : "vcc")

#define MSM_MACN_6(CB, acc, hi, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4, a5, b5) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %10, %11, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %12, %13, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "+v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4), "v"(a5), CB(b5) \
      : "vcc")

#define MSM_MACN_7(CB, acc, hi, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4, a5, b5, a6, b6) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %10, %11, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %12, %13, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %14, %15, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "+v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4), "v"(a5), CB(b5), "v"(a6), CB(b6) \
      : "vcc")

#define MSM_MACN_8(CB, acc, hi, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4, a5, b5, a6, b6, a7, b7) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %10, %11, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %12, %13, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %14, %15, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %16, %17, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "+v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4), "v"(a5), CB(b5), "v"(a6), CB(b6), "v"(a7), CB(b7) \
      : "vcc")

#define MSM_MACFN_1(CB, acc, hi, a0, b0) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_cndmask_b32_e64 %1, 0, 1, vcc" \
      : "+v"(acc), "=&v"(hi) \
      : "v"(a0), CB(b0) \
      : "vcc")

#define MSM_MACFN_2(CB, acc, hi, a0, b0, a1, b1) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_cndmask_b32_e64 %1, 0, 1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "=&v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1) \
      : "vcc")

#define MSM_MACFN_3(CB, acc, hi, a0, b0, a1, b1, a2, b2) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_cndmask_b32_e64 %1, 0, 1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "=&v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2) \
      : "vcc")

#define MSM_MACFN_4(CB, acc, hi, a0, b0, a1, b1, a2, b2, a3, b3) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_cndmask_b32_e64 %1, 0, 1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "=&v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3) \
      : "vcc")

#define MSM_MACFN_5(CB, acc, hi, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_cndmask_b32_e64 %1, 0, 1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %10, %11, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "=&v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4) \
      : "vcc")

#define MSM_MACFN_6(CB, acc, hi, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4, a5, b5) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_cndmask_b32_e64 %1, 0, 1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %10, %11, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %12, %13, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "=&v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4), "v"(a5), CB(b5) \
      : "vcc")

#define MSM_MACFN_7(CB, acc, hi, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4, a5, b5, a6, b6) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_cndmask_b32_e64 %1, 0, 1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %10, %11, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %12, %13, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %14, %15, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "=&v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4), "v"(a5), CB(b5), "v"(a6), CB(b6) \
      : "vcc")

#define MSM_MACFN_8(CB, acc, hi, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4, a5, b5, a6, b6, a7, b7) \
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t" \
      "v_cndmask_b32_e64 %1, 0, 1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %4, %5, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %6, %7, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %10, %11, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %12, %13, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %14, %15, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc\n\t" \
      "v_mad_u64_u32 %0, vcc, %16, %17, %0\n\t" \
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc" \
      : "+v"(acc), "=&v"(hi) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4), "v"(a5), CB(b5), "v"(a6), CB(b6), "v"(a7), CB(b7) \
      : "vcc")

template <int N, bool SGPR_Y>
__device__ __forceinline__ void mac_group(uint64_t& acc, uint32_t& hi, const uint32_t* x,
                                          const uint32_t* y, bool first) {
#define MSM_G1 x[0], y[0]
#define MSM_G2 MSM_G1, x[1], y[1]
#define MSM_G3 MSM_G2, x[2], y[2]
#define MSM_G4 MSM_G3, x[3], y[3]
#define MSM_G5 MSM_G4, x[4], y[4]
#define MSM_G6 MSM_G5, x[5], y[5]
#define MSM_G7 MSM_G6, x[6], y[6]
#define MSM_G8 MSM_G7, x[7], y[7]
#define MSM_CALL(f, ...) f(__VA_ARGS__)
#define MSM_GROUP(n)                                      \
  if (first && SGPR_Y)                                    \
    MSM_CALL(MSM_MACFN_##n, "s", acc, hi, MSM_G##n);      \
  else if (first)                                         \
    MSM_CALL(MSM_MACFN_##n, "v", acc, hi, MSM_G##n);      \
  else if (SGPR_Y)                                        \
    MSM_CALL(MSM_MACN_##n, "s", acc, hi, MSM_G##n);       \
  else                                                    \
    MSM_CALL(MSM_MACN_##n, "v", acc, hi, MSM_G##n);
  if constexpr (N == 1) { MSM_GROUP(1) }
  if constexpr (N == 2) { MSM_GROUP(2) }
  if constexpr (N == 3) { MSM_GROUP(3) }
  if constexpr (N == 4) { MSM_GROUP(4) }
  if constexpr (N == 5) { MSM_GROUP(5) }
  if constexpr (N == 6) { MSM_GROUP(6) }
  if constexpr (N == 7) { MSM_GROUP(7) }
  if constexpr (N == 8) { MSM_GROUP(8) }
#undef MSM_GROUP
#undef MSM_CALL
#undef MSM_G8
#undef MSM_G7
#undef MSM_G6
#undef MSM_G5
#undef MSM_G4
#undef MSM_G3
#undef MSM_G2
#undef MSM_G1
}

// (acc, hi) += sum of the L products x[t] y[t] (y in SGPRs when SGPR_Y);
// first: hi starts from the first product's carry
template <int L, bool SGPR_Y>
__device__ __forceinline__ void mac_run(uint64_t& acc, uint32_t& hi, const uint32_t* x,
                                        const uint32_t* y, bool first) {
  if constexpr (L > 0) {
    constexpr int G = L < 8 ? L : 8;
    mac_group<G, SGPR_Y>(acc, hi, x, y, first);
    if constexpr (L > G) mac_run<L - G, SGPR_Y>(acc, hi, x + G, y + G, false);
  }
}

// column K < 12 of a*b + m*p: a_i b_{K-i} (i <= K), m_j p_{K-j} (j < K); then
// the reduction digit m_K
template <int K>
__device__ __forceinline__ void mont_low_column(const fe& a, const fe& b, uint32_t* m,
                                                uint64_t& acc) {
  uint32_t x[2 * K + 1], y[2 * K + 1];
#pragma unroll
  for (int i = 0; i <= K; ++i) {
    x[i] = a.v[i];
    y[i] = b.v[K - i];
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    x[K + 1 + j] = m[j];
    y[K + 1 + j] = kP[K - j];
  }
  uint32_t hi;
  mac_run<2 * K + 1, false>(acc, hi, x, y, true);
  redc_step(acc, hi, m[K]);
}

// column K >= 12: a_i b_{K-i} and m_i p_{K-i} for i = K-11 .. 11; the low
// word is result word K - 12
template <int K>
__device__ __forceinline__ uint32_t mont_high_column(const fe& a, const fe& b, const uint32_t* m,
                                                     uint64_t& acc) {
  constexpr int I0 = K - (NL - 1), L = NL - I0;
  uint32_t x[2 * L], y[2 * L];
#pragma unroll
  for (int i = I0; i < NL; ++i) {
    x[i - I0] = a.v[i];
    y[i - I0] = b.v[K - i];
    x[L + i - I0] = m[i];
    y[L + i - I0] = kP[K - i];
  }
  uint32_t hi;
  mac_run<2 * L, false>(acc, hi, x, y, true);
  const uint32_t w = (uint32_t)acc;
  acc = ((uint64_t)hi << 32) | (acc >> 32);
  return w;
}

// Montgomery product r = a*b*R^{-1} mod p, lazily reduced: product scanning
// with the reduction interleaved per column (the m_j p terms join column k
// once m_j is known).  Requires a*b < R*p (e.g. a, b < 12p); returns r < 2p.
__device__ __forceinline__ fe fe_mul(const fe& a, const fe& b) {
  uint32_t m[NL];
  fe r;
  uint64_t acc;
  MSM_MUL0(acc, a.v[0], b.v[0]);
  redc_step0(acc, m[0]);
  mont_low_column<1>(a, b, m, acc);
  mont_low_column<2>(a, b, m, acc);
  mont_low_column<3>(a, b, m, acc);
  mont_low_column<4>(a, b, m, acc);
  mont_low_column<5>(a, b, m, acc);
  mont_low_column<6>(a, b, m, acc);
  mont_low_column<7>(a, b, m, acc);
  mont_low_column<8>(a, b, m, acc);
  mont_low_column<9>(a, b, m, acc);
  mont_low_column<10>(a, b, m, acc);
  mont_low_column<11>(a, b, m, acc);
  r.v[0] = mont_high_column<12>(a, b, m, acc);
  r.v[1] = mont_high_column<13>(a, b, m, acc);
  r.v[2] = mont_high_column<14>(a, b, m, acc);
  r.v[3] = mont_high_column<15>(a, b, m, acc);
  r.v[4] = mont_high_column<16>(a, b, m, acc);
  r.v[5] = mont_high_column<17>(a, b, m, acc);
  r.v[6] = mont_high_column<18>(a, b, m, acc);
  r.v[7] = mont_high_column<19>(a, b, m, acc);
  r.v[8] = mont_high_column<20>(a, b, m, acc);
  r.v[9] = mont_high_column<21>(a, b, m, acc);
  r.v[10] = mont_high_column<22>(a, b, m, acc);
  r.v[11] = (uint32_t)acc;
  return r;
}

// Montgomery square.  With two VALU ops per product, the symmetric-product
// shortcut saves only a few percent once its doubling and merging work is
// counted, so squaring shares the multiply.
__device__ __forceinline__ fe fe_sqr(const fe& a) { return fe_mul(a, a); }

// ---------------------------------------------------------------------------
// unreduced add / subtract (12-word carry chains)
// ---------------------------------------------------------------------------

#define MSM_SUB0(r, cy, a, b) \
  asm("v_sub_co_u32_e64 %0, %1, %2, %3" : "=v"(r), "=s"(cy) : "v"(a), "v"(b))
#define MSM_SUBB(r, cy, a, b, ci) \
  asm("v_subb_co_u32_e64 %0, %1, %2, %3, %4" : "=v"(r), "=s"(cy) : "v"(a), "v"(b), "s"(ci))

// 12-word carry chains, each in a single asm block (the compiler separates
// asm blocks by a wait state; one block per word cost a lone wave 11 of them
// per chain).

// r = a + b (no reduction; caller guarantees a + b < 2^384)
__device__ __forceinline__ fe fe_add(const fe& a, const fe& b) {
  fe r;
  asm("v_add_co_u32_e32 %0, vcc, %12, %24\n\t"
      "v_addc_co_u32_e32 %1, vcc, %13, %25, vcc\n\t"
      "v_addc_co_u32_e32 %2, vcc, %14, %26, vcc\n\t"
      "v_addc_co_u32_e32 %3, vcc, %15, %27, vcc\n\t"
      "v_addc_co_u32_e32 %4, vcc, %16, %28, vcc\n\t"
      "v_addc_co_u32_e32 %5, vcc, %17, %29, vcc\n\t"
      "v_addc_co_u32_e32 %6, vcc, %18, %30, vcc\n\t"
      "v_addc_co_u32_e32 %7, vcc, %19, %31, vcc\n\t"
      "v_addc_co_u32_e32 %8, vcc, %20, %32, vcc\n\t"
      "v_addc_co_u32_e32 %9, vcc, %21, %33, vcc\n\t"
      "v_addc_co_u32_e32 %10, vcc, %22, %34, vcc\n\t"
      "v_addc_co_u32_e32 %11, vcc, %23, %35, vcc"
      : "=&v"(r.v[0]), "=&v"(r.v[1]), "=&v"(r.v[2]), "=&v"(r.v[3]), "=&v"(r.v[4]), "=&v"(r.v[5]), "=&v"(r.v[6]), "=&v"(r.v[7]), "=&v"(r.v[8]), "=&v"(r.v[9]), "=&v"(r.v[10]), "=&v"(r.v[11])
      : "v"(a.v[0]), "v"(a.v[1]), "v"(a.v[2]), "v"(a.v[3]), "v"(a.v[4]), "v"(a.v[5]), "v"(a.v[6]), "v"(a.v[7]), "v"(a.v[8]), "v"(a.v[9]), "v"(a.v[10]), "v"(a.v[11]),
        "v"(b.v[0]), "v"(b.v[1]), "v"(b.v[2]), "v"(b.v[3]), "v"(b.v[4]), "v"(b.v[5]), "v"(b.v[6]), "v"(b.v[7]), "v"(b.v[8]), "v"(b.v[9]), "v"(b.v[10]), "v"(b.v[11])
      : "vcc");
  return r;
}

// r = c - b for b <= c (no borrow out)
__device__ __forceinline__ fe fe_sub_nb(const fe& c, const fe& b) {
  fe r;
  asm("v_sub_co_u32_e32 %0, vcc, %12, %24\n\t"
      "v_subb_co_u32_e32 %1, vcc, %13, %25, vcc\n\t"
      "v_subb_co_u32_e32 %2, vcc, %14, %26, vcc\n\t"
      "v_subb_co_u32_e32 %3, vcc, %15, %27, vcc\n\t"
      "v_subb_co_u32_e32 %4, vcc, %16, %28, vcc\n\t"
      "v_subb_co_u32_e32 %5, vcc, %17, %29, vcc\n\t"
      "v_subb_co_u32_e32 %6, vcc, %18, %30, vcc\n\t"
      "v_subb_co_u32_e32 %7, vcc, %19, %31, vcc\n\t"
      "v_subb_co_u32_e32 %8, vcc, %20, %32, vcc\n\t"
      "v_subb_co_u32_e32 %9, vcc, %21, %33, vcc\n\t"
      "v_subb_co_u32_e32 %10, vcc, %22, %34, vcc\n\t"
      "v_subb_co_u32_e32 %11, vcc, %23, %35, vcc"
      : "=&v"(r.v[0]), "=&v"(r.v[1]), "=&v"(r.v[2]), "=&v"(r.v[3]), "=&v"(r.v[4]), "=&v"(r.v[5]), "=&v"(r.v[6]), "=&v"(r.v[7]), "=&v"(r.v[8]), "=&v"(r.v[9]), "=&v"(r.v[10]), "=&v"(r.v[11])
      : "v"(c.v[0]), "v"(c.v[1]), "v"(c.v[2]), "v"(c.v[3]), "v"(c.v[4]), "v"(c.v[5]), "v"(c.v[6]), "v"(c.v[7]), "v"(c.v[8]), "v"(c.v[9]), "v"(c.v[10]), "v"(c.v[11]),
        "v"(b.v[0]), "v"(b.v[1]), "v"(b.v[2]), "v"(b.v[3]), "v"(b.v[4]), "v"(b.v[5]), "v"(b.v[6]), "v"(b.v[7]), "v"(b.v[8]), "v"(b.v[9]), "v"(b.v[10]), "v"(b.v[11])
      : "vcc");
  return r;
}

// r = a - b + c where c is a constant multiple of p held in VGPRs and b <= c
// (so the result is non-negative); the caller guarantees a + c < 2^384.
__device__ __forceinline__ fe fe_sub_plus(const fe& a, const fe& b, const fe& c) {
  return fe_add(a, fe_sub_nb(c, b));
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


}  // namespace msm
