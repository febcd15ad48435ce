// Alternative field-multiplication cores, for comparison with the production
// Montgomery multiply of field.hpp (the paper proposes both directions as
// future work, Sec. V-C):
//
//  * fe_mul_barrett: plain residues with Barrett reduction for k = 378,
//    mu = floor(2^756 / p).  For t = x y < 2^756: q1 = t >> 377,
//    q3 = (q1 mu) >> 379, r = t - q3 p.  The columns of q1 mu below word 9
//    are skipped (their sum is < 2^324, so q3 is at most one below the exact
//    Barrett quotient, itself at most two below t / p): r < 4p.  Inputs
//    x < 4p and y < p keep t < 4 p^2 < 2^756 between chained products.
//  * fe_mul_karatsuba: Montgomery (R = 2^384) with the 12 x 12-word product
//    formed by one Karatsuba level over 6-word halves (three 6 x 6 products
//    instead of four, plus the sums and differences), then a separate
//    product-scanning reduction.  Same value and bounds as fe_mul.
#pragma once
#include "field.hpp"

namespace msm {

// floor(2^756 / p), 380 bits
constexpr uint32_t kBarrettMu[NL] = {0x7936bff3u, 0x7e7f5631u, 0x2710a964u, 0x43b5a1deu,
                                     0x6169b40bu, 0xabcb5223u, 0x9ddac681u, 0xeeeb4379u,
                                     0x60bbd3dcu, 0x5db0f281u, 0x3310183au, 0x09854234u};

// t[0 .. NA+NB) = a * b by product scanning (column sum + deferred carry word)
template <int NA, int NB>
__device__ __forceinline__ void mul_words(const uint32_t* a, const uint32_t* b, uint32_t* t) {
  uint64_t acc;
  uint32_t hi = 0;
  MSM_MUL0(acc, a[0], b[0]);
  t[0] = (uint32_t)acc;
  acc >>= 32;
#pragma unroll
  for (int k = 1; k < NA + NB - 1; ++k) {
    const int i0 = k - (NB - 1) > 0 ? k - (NB - 1) : 0;
    const int i1 = k < NA - 1 ? k : NA - 1;
    MSM_MACF(acc, hi, a[i0], b[k - i0]);
#pragma unroll
    for (int i = i0 + 1; i <= i1; ++i) MSM_MAC(acc, hi, a[i], b[k - i]);
    t[k] = (uint32_t)acc;
    acc = ((uint64_t)hi << 32) | (acc >> 32);
  }
  t[NA + NB - 1] = (uint32_t)acc;
}

__device__ __forceinline__ fe fe_mul_barrett(const fe& x, const fe& y) {
  uint32_t t[2 * NL];
  mul_words<NL, NL>(x.v, y.v, t);
  uint32_t q1[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i)
    q1[i] = __builtin_amdgcn_alignbit(i + 12 < 2 * NL ? t[i + 12] : 0u, t[i + 11], 25);
  // columns 9..22 of q1 * mu (words 9..23)
  uint32_t q2[2 * NL];
  {
    uint64_t acc = 0;
    uint32_t hi = 0;
#pragma unroll
    for (int k = 9; k < 2 * NL - 1; ++k) {
      const int i0 = k - (NL - 1) > 0 ? k - (NL - 1) : 0;
      const int i1 = k < NL - 1 ? k : NL - 1;
      MSM_MACF_S(acc, hi, q1[i0], kBarrettMu[k - i0]);
#pragma unroll
      for (int i = i0 + 1; i <= i1; ++i) MSM_MAC_S(acc, hi, q1[i], kBarrettMu[k - i]);
      q2[k] = (uint32_t)acc;
      acc = ((uint64_t)hi << 32) | (acc >> 32);
    }
    q2[2 * NL - 1] = (uint32_t)acc;
  }
  uint32_t q3[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i)
    q3[i] = __builtin_amdgcn_alignbit(i + 12 < 2 * NL ? q2[i + 12] : 0u, q2[i + 11], 27);
  // low 12 words of q3 * p
  uint32_t qp[NL];
  {
    uint64_t acc;
    uint32_t hi = 0;
    MSM_MUL0(acc, q3[0], kP[0]);
    qp[0] = (uint32_t)acc;
    acc >>= 32;
#pragma unroll
    for (int k = 1; k < NL; ++k) {
      MSM_MACF_S(acc, hi, q3[0], kP[k]);
#pragma unroll
      for (int i = 1; i <= k; ++i) MSM_MAC_S(acc, hi, q3[i], kP[k - i]);
      qp[k] = (uint32_t)acc;
      acc = ((uint64_t)hi << 32) | (acc >> 32);
    }
  }
  fe r;
  uint64_t cy, cy2;
  MSM_SUB0(r.v[0], cy, t[0], qp[0]);
#pragma unroll
  for (int i = 1; i < NL; ++i) {
    MSM_SUBB(r.v[i], cy2, t[i], qp[i], cy);
    cy = cy2;
  }
  return r;
}

__device__ __forceinline__ fe fe_mul_karatsuba(const fe& a, const fe& b) {
  constexpr int H = NL / 2;
  uint32_t z0[NL], z2[NL], zm[NL + 1];
  mul_words<H, H>(a.v, b.v, z0);
  mul_words<H, H>(a.v + H, b.v + H, z2);
  uint32_t sa[H], sb[H];
  uint64_t c = 0, d = 0;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    c = (uint64_t)a.v[i] + a.v[i + H] + (c >> 32);
    d = (uint64_t)b.v[i] + b.v[i + H] + (d >> 32);
    sa[i] = (uint32_t)c;
    sb[i] = (uint32_t)d;
  }
  const uint32_t ca = (uint32_t)(c >> 32), cb = (uint32_t)(d >> 32);
  mul_words<H, H>(sa, sb, zm);
  // (sa + ca 2^192)(sb + cb 2^192) = zm + (ca sb + cb sa) 2^192 + ca cb 2^384
  {
    uint64_t e = 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      e = (uint64_t)zm[i + H] + (ca ? sb[i] : 0u) + (cb ? sa[i] : 0u) + (e >> 32);
      zm[i + H] = (uint32_t)e;
    }
    zm[NL] = (uint32_t)(e >> 32) + (ca & cb);
  }
  // z1 = zm - z0 - z2 (13 words, non-negative)
  {
    int64_t e = 0;
#pragma unroll
    for (int i = 0; i <= NL; ++i) {
      e += (int64_t)zm[i] - (i < NL ? (int64_t)z0[i] + (int64_t)z2[i] : 0);
      zm[i] = (uint32_t)e;
      e >>= 32;
    }
  }
  // t = z0 + z1 2^192 + z2 2^384
  uint32_t t[2 * NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    t[i] = z0[i];
    t[i + NL] = z2[i];
  }
  {
    uint64_t e = 0;
#pragma unroll
    for (int i = H; i < 2 * NL; ++i) {
      e = (uint64_t)t[i] + (i - H <= NL ? zm[i - H] : 0u) + (e >> 32);
      t[i] = (uint32_t)e;
    }
  }
  // Montgomery reduction of t, product scanning: m_k = -(column k) mod 2^32
  uint32_t m[NL];
  fe r;
  uint64_t acc = t[0];
  uint32_t hi = 0;
  redc_step0(acc, m[0]);
#pragma unroll
  for (int k = 1; k < NL; ++k) {
    acc += t[k];
    MSM_MACF_S(acc, hi, m[0], kP[k]);
#pragma unroll
    for (int j = 1; j < k; ++j) MSM_MAC_S(acc, hi, m[j], kP[k - j]);
    redc_step(acc, hi, m[k]);
  }
#pragma unroll
  for (int k = NL; k < 2 * NL - 1; ++k) {
    acc += t[k];
    MSM_MACF_S(acc, hi, m[k - (NL - 1)], kP[NL - 1]);
#pragma unroll
    for (int j = k - (NL - 1) + 1; j < NL; ++j) MSM_MAC_S(acc, hi, m[j], kP[k - j]);
    r.v[k - NL] = (uint32_t)acc;
    acc = ((uint64_t)hi << 32) | (acc >> 32);
  }
  r.v[NL - 1] = (uint32_t)(acc + t[2 * NL - 1]);
  return r;
}

}  // namespace msm
