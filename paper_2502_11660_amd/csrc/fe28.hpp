// Carry-free base-field arithmetic for the one-lane throughput PADD unit
// (device code).
//
// An element is fourteen 28-bit limbs, each in its own 32-bit word, so a
// 32x32->64 multiply-add of two limbs leaves room above the product: a 64-bit
// column accumulator absorbs every product of a column with no carry word.
// The 12-word form of field.hpp pays one carry add per multiply-add (the carry
// out of a full 64-bit column sum); here the carries are resolved once per
// column by a shift, the carry-save idea of Sec. III-D with the saved carry
// bits inside each 64-bit column sum.
//
// Montgomery form with R' = 2^392 = 2^(14*28).  Stored data (HBM records,
// the C boundary) stays in the 12-word form with R = 2^384; a value w R mod p
// read in this arithmetic is the value w 2^-8 in R'-form.  Projective points
// are unchanged by a common factor of their coordinates, so extended points
// (X, Y, T, Z) carry over between the two forms as they are; the only
// affine inputs, prepared points (X, Y, U = kT with Z = 1), become the
// projective point with Z = 2^-8, which the mixed addition accounts for by
// D = 2 Z1 Z2 = Z1 2^-7 (an exact division by 2^7 mod p, f28_div128x2).
//
// Bounds.  p < 2^377, R'/p > 38996.  For operands with limbs below 2^30 the
// largest column sum is 14 (2^30)^2 + 13 (2^28)^2 + 2^36 < 2^64, and
// REDC(a b) < 2p whenever a b < R' p.  Products return limbs 0..12 below
// 2^28 ("normalised") and the value below 2p (limb 13 below 2^15).
// Additions are limb-wise (no carries); a subtraction adds a multiple of p
// whose limbs are raised by borrowing from the next limb, so that every limb
// difference is non-negative:
//   KS4 = 4p with limbs 0..12 in [2^28 - 1, 2^29): subtracts values with
//         normalised limbs and top limb <= 0x6b8c (values < 4p do).
// The per-formula bounds are written next to each point formula (curve28.hpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field.hpp"

namespace msm {

constexpr int NL28 = 14;
constexpr uint32_t M28 = 0x0fffffffu;

struct fe28 {
  uint32_t v[NL28];
};

// p in 28-bit limbs
constexpr uint32_t kP28[NL28] = {0x0000001u, 0x08c0000u, 0x0000085u, 0x5d44300u, 0x800170bu,
                                 0x2fba094u, 0xf1ef362u, 0x00f5138u, 0xa22d9f3u, 0xa1493b1u,
                                 0xb05c06cu, 0x10eac63u, 0xa4617c5u, 0x0001ae3u};
// 4p, limbs 0..12 raised by 2^28 and lowered by the borrow of the limb above
constexpr uint32_t kKS4[NL28] = {0x10000004u, 0x122fffffu, 0x10000213u, 0x17510bffu,
                                 0x10005c2cu, 0x1bee8251u, 0x1c7bcd87u, 0x103d44e2u,
                                 0x188b67cbu, 0x18524ec5u, 0x1c1701b1u, 0x143ab18du,
                                 0x19185f13u, 0x00006b8du};
// the curve constant k = 2d in R'-form (k 2^392 mod p)
constexpr uint32_t kK28[NL28] = {0x706c521u, 0xdf4444au, 0x8fa7e68u, 0x371b2aau, 0xdd6cd3du,
                                 0xebe579eu, 0x3577a6au, 0x1d3f1c6u, 0x2ada318u, 0x2a73d9du,
                                 0x7da6ef5u, 0xce09495u, 0xfed4ab8u, 0x0001813u};

__device__ __forceinline__ fe28 f28_const(const uint32_t (&c)[NL28]) {
  fe28 r;
#pragma unroll
  for (int i = 0; i < NL28; ++i) r.v[i] = c[i];
  return r;
}

__device__ __forceinline__ fe28 f28_small(uint32_t x) {
  fe28 r;
  r.v[0] = x;
#pragma unroll
  for (int i = 1; i < NL28; ++i) r.v[i] = 0u;
  return r;
}

// 12 words (value < 2^392) -> 14 limbs: limb i holds bits 28i .. 28i + 27.
__device__ __forceinline__ fe28 f28_from_words(const fe& x) {
  fe28 r;
#pragma unroll
  for (int i = 0; i < NL28; ++i) {
    const int b = 28 * i, w = b >> 5, s = b & 31;
    if (s + 28 <= 32)
      r.v[i] = s + 28 == 32 ? x.v[w] >> s : (x.v[w] >> s) & M28;
    else if (w + 1 < NL)
      r.v[i] = __builtin_amdgcn_alignbit(x.v[w + 1], x.v[w], s) & M28;
    else
      r.v[i] = x.v[w] >> s;
  }
  return r;
}

// 14 limbs with limbs 0..12 normalised (value < 2^384) -> 12 words.
__device__ __forceinline__ fe f28_to_words(const fe28& x) {
  fe r;
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const int b = 32 * j, i = b / 28, s = b % 28;
    uint32_t w = x.v[i] >> s;
    w |= x.v[i + 1] << (28 - s);
    if (56 - s < 32) w |= x.v[i + 2] << (56 - s);
    r.v[j] = w;
  }
  return r;
}

// Grouped multiply-adds without carry words: n products added into one 64-bit
// column accumulator by one asm block (written as asm so that the column's
// products are added in order onto the incoming carry: as plain C the
// compiler sums each column from zero and adds the carry afterwards, one
// extra 64-bit add per column).  The carry-out of v_mad_u64_u32 goes to a
// scratch SGPR pair (cc) that nothing reads.  CB is the second factor's
// constraint ("v" for a VGPR, "s" for an SGPR such as a limb of p).  cc is
// early-clobber ("=&s"): the block's first multiply-add writes it before the
// later ones read their factors, so it must not share a register with an
// SGPR factor (without the "&" the compiler may assign both to one register,
// and a limb of p would be overwritten by a carry-out mid-block).
#define MSM_MAD28_1(CB, acc, cc, a0, b0) \
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" \
      : "+v"(acc), "=&s"(cc) \
      : "v"(a0), CB(b0))

#define MSM_MAD28_2(CB, acc, cc, a0, b0, a1, b1) \
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %4, %5, %0" \
      : "+v"(acc), "=&s"(cc) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1))

#define MSM_MAD28_3(CB, acc, cc, a0, b0, a1, b1, a2, b2) \
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %4, %5, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %6, %7, %0" \
      : "+v"(acc), "=&s"(cc) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2))

#define MSM_MAD28_4(CB, acc, cc, a0, b0, a1, b1, a2, b2, a3, b3) \
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %4, %5, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %6, %7, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %8, %9, %0" \
      : "+v"(acc), "=&s"(cc) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3))

#define MSM_MAD28_5(CB, acc, cc, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4) \
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %4, %5, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %6, %7, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %8, %9, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %10, %11, %0" \
      : "+v"(acc), "=&s"(cc) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4))

#define MSM_MAD28_6(CB, acc, cc, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4, a5, b5) \
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %4, %5, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %6, %7, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %8, %9, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %10, %11, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %12, %13, %0" \
      : "+v"(acc), "=&s"(cc) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4), "v"(a5), CB(b5))

#define MSM_MAD28_7(CB, acc, cc, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4, a5, b5, a6, b6) \
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %4, %5, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %6, %7, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %8, %9, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %10, %11, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %12, %13, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %14, %15, %0" \
      : "+v"(acc), "=&s"(cc) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4), "v"(a5), CB(b5), "v"(a6), CB(b6))

#define MSM_MAD28_8(CB, acc, cc, a0, b0, a1, b1, a2, b2, a3, b3, a4, b4, a5, b5, a6, b6, a7, b7) \
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %4, %5, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %6, %7, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %8, %9, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %10, %11, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %12, %13, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %14, %15, %0\n\t" \
      "v_mad_u64_u32 %0, %1, %16, %17, %0" \
      : "+v"(acc), "=&s"(cc) \
      : "v"(a0), CB(b0), "v"(a1), CB(b1), "v"(a2), CB(b2), "v"(a3), CB(b3), "v"(a4), CB(b4), "v"(a5), CB(b5), "v"(a6), CB(b6), "v"(a7), CB(b7))

template <int N, bool SGPR_Y>
__device__ __forceinline__ void mad28_group(uint64_t& acc, const uint32_t* x, const uint32_t* y) {
  uint64_t cc;
#define MSM_G1 x[0], y[0]
#define MSM_G2 MSM_G1, x[1], y[1]
#define MSM_G3 MSM_G2, x[2], y[2]
#define MSM_G4 MSM_G3, x[3], y[3]
#define MSM_G5 MSM_G4, x[4], y[4]
#define MSM_G6 MSM_G5, x[5], y[5]
#define MSM_G7 MSM_G6, x[6], y[6]
#define MSM_G8 MSM_G7, x[7], y[7]
#define MSM_CALL(f, ...) f(__VA_ARGS__)
#define MSM_GROUP(n)                                  \
  if (SGPR_Y)                                         \
    MSM_CALL(MSM_MAD28_##n, "s", acc, cc, MSM_G##n);  \
  else                                                \
    MSM_CALL(MSM_MAD28_##n, "v", acc, cc, MSM_G##n);
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
  (void)cc;
}

// acc += sum of the L products x[t] y[t] (y in SGPRs when SGPR_Y)
template <int L, bool SGPR_Y>
__device__ __forceinline__ void mad28_run(uint64_t& acc, const uint32_t* x, const uint32_t* y) {
  if constexpr (L > 0) {
    constexpr int G = L < 8 ? L : 8;
    mad28_group<G, SGPR_Y>(acc, x, y);
    if constexpr (L > G) mad28_run<L - G, SGPR_Y>(acc, x + G, y + G);
  }
}

// column K of a b + m p: the products a_i b_{K-i} and m_j p_{K-j} whose
// indices lie in [0, 14) (j < K below column 14, where m_K is not known yet)
template <int K>
__device__ __forceinline__ void f28_column(const fe28& a, const fe28& b, const uint32_t* m,
                                           uint64_t& acc) {
  constexpr int I0 = K < NL28 ? 0 : K - (NL28 - 1);
  constexpr int I1 = K < NL28 ? K : NL28 - 1;
  constexpr int J1 = K < NL28 ? K - 1 : NL28 - 1;
  uint32_t x[NL28], y[NL28];
#pragma unroll
  for (int i = I0; i <= I1; ++i) {
    x[i - I0] = a.v[i];
    y[i - I0] = b.v[K - i];
  }
  mad28_run<I1 - I0 + 1, false>(acc, x, y);
  if constexpr (J1 >= I0) {
    uint32_t u[NL28], q[NL28];
#pragma unroll
    for (int j = I0; j <= J1; ++j) {
      u[j - I0] = m[j];
      q[j - I0] = kP28[K - j];
    }
    mad28_run<J1 - I0 + 1, true>(acc, u, q);
  }
}

// low column K < 14 with column sum t: the reduction digit m_K = -t mod 2^28
// (-p^-1 = -1 mod 2^28 since p = 1 mod 2^46) clears the column's low 28 bits
// when m_K p_0 = m_K is added, so the carry is (t + m_K) >> 28, which equals
// (t + 2^28 - 1) >> 28; with u = t + 2^28 - 1, m_K is also ~u mod 2^28 (one
// and-not of u's low word)
template <int K>
__device__ __forceinline__ void f28_low(const fe28& a, const fe28& b, uint32_t* m, uint64_t& acc) {
  f28_column<K>(a, b, m, acc);
  acc += M28;
  m[K] = ~(uint32_t)acc & M28;
  acc >>= 28;
}

// high column K >= 14: result limb K - 14
template <int K>
__device__ __forceinline__ void f28_high(const fe28& a, const fe28& b, const uint32_t* m,
                                         uint64_t& acc, fe28& r) {
  f28_column<K>(a, b, m, acc);
  r.v[K - NL28] = (uint32_t)acc & M28;
  acc >>= 28;
}

// Montgomery product a b 2^-392 mod p, product scanning with the reduction
// interleaved per column: column k's products are added onto the carry of
// column k - 1 in one 64-bit accumulator.  Operands: limbs < 2^30 and
// a b < R' p.  Result: limbs 0..12 normalised, value < 2p.
__device__ __forceinline__ fe28 f28_mul(const fe28& a, const fe28& b) {
  uint32_t m[NL28];
  fe28 r;
  uint64_t acc = 0;
  f28_low<0>(a, b, m, acc);
  f28_low<1>(a, b, m, acc);
  f28_low<2>(a, b, m, acc);
  f28_low<3>(a, b, m, acc);
  f28_low<4>(a, b, m, acc);
  f28_low<5>(a, b, m, acc);
  f28_low<6>(a, b, m, acc);
  f28_low<7>(a, b, m, acc);
  f28_low<8>(a, b, m, acc);
  f28_low<9>(a, b, m, acc);
  f28_low<10>(a, b, m, acc);
  f28_low<11>(a, b, m, acc);
  f28_low<12>(a, b, m, acc);
  f28_low<13>(a, b, m, acc);
  f28_high<14>(a, b, m, acc, r);
  f28_high<15>(a, b, m, acc, r);
  f28_high<16>(a, b, m, acc, r);
  f28_high<17>(a, b, m, acc, r);
  f28_high<18>(a, b, m, acc, r);
  f28_high<19>(a, b, m, acc, r);
  f28_high<20>(a, b, m, acc, r);
  f28_high<21>(a, b, m, acc, r);
  f28_high<22>(a, b, m, acc, r);
  f28_high<23>(a, b, m, acc, r);
  f28_high<24>(a, b, m, acc, r);
  f28_high<25>(a, b, m, acc, r);
  f28_high<26>(a, b, m, acc, r);
  r.v[NL28 - 1] = (uint32_t)acc;
  return r;
}

// limb-wise a + b (no carries)
__device__ __forceinline__ fe28 f28_add(const fe28& a, const fe28& b) {
  fe28 r;
#pragma unroll
  for (int i = 0; i < NL28; ++i) r.v[i] = a.v[i] + b.v[i];
  return r;
}

// a + 4p - b, limb-wise; b normalised with value < 4p (top limb <= 0x6b8c).
// Limbs of the result are below a's limbs + 2^29.
__device__ __forceinline__ fe28 f28_sub4(const fe28& a, const fe28& b) {
  fe28 r;
#pragma unroll
  for (int i = 0; i < NL28; ++i) r.v[i] = a.v[i] + (kKS4[i] - b.v[i]);
  return r;
}

// r = (lane condition) ? x : y
__device__ __forceinline__ fe28 f28_select(bool c, const fe28& x, const fe28& y) {
  fe28 r;
#pragma unroll
  for (int i = 0; i < NL28; ++i) r.v[i] = c ? x.v[i] : y.v[i];
  return r;
}

// 2 z 2^-8 = z 2^-7 mod p, exactly: with m = -z mod 2^7, z + m p is a
// multiple of 2^7 (p = 1 mod 2^46) and the quotient is taken limb by limb,
// each limb keeping its own bits above 7 and receiving the low 7 bits of the
// limb above.  z: normalised, value < 2p.  Result: limbs < 2^29,
// value < (2p + 127 p) / 128 < 1.01 p.
__device__ __forceinline__ fe28 f28_div128x2(const fe28& z) {
  const uint32_t m = (0u - z.v[0]) & 0x7fu;
  uint64_t w[NL28];
  w[0] = (uint64_t)(z.v[0] + m);
#pragma unroll
  for (int i = 1; i < NL28; ++i) w[i] = (uint64_t)m * kP28[i] + z.v[i];
  fe28 r;
#pragma unroll
  for (int i = 0; i < NL28 - 1; ++i) {
    const uint32_t lo = (uint32_t)w[i], hi = (uint32_t)(w[i] >> 32);
    r.v[i] = __builtin_amdgcn_alignbit(hi, lo, 7) + (((uint32_t)w[i + 1] & 0x7fu) << 21);
  }
  r.v[NL28 - 1] = (uint32_t)(w[NL28 - 1] >> 7);
  return r;
}

}  // namespace msm
