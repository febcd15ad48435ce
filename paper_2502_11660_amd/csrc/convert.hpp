// Field inversion and the Weierstrass <-> twisted-Edwards conversions (device).
#pragma once
#include "common.hpp"

namespace msm {

// Plain C++ multiword helpers for the data-dependent inversion loop (the
// carry sequences of field.hpp pass carries through wave-wide lane masks,
// which the compiler treats as uniform values).

// r = a - b; returns 1 if a < b
__device__ __forceinline__ uint32_t fe_sub_c(const fe& a, const fe& b, fe& r) {
  uint32_t borrow = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    uint64_t d = (uint64_t)a.v[i] - b.v[i] - borrow;
    r.v[i] = (uint32_t)d;
    borrow = (uint32_t)(d >> 63);
  }
  return borrow;
}

__device__ __forceinline__ fe fe_add_c(const fe& a, const fe& b) {
  fe r;
  uint64_t c = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    c = (uint64_t)a.v[i] + b.v[i] + (c >> 32);
    r.v[i] = (uint32_t)c;
  }
  return r;
}

// ---------------------------------------------------------------------------
// Modular inversion by the binary extended Euclidean algorithm with the
// divsteps batched 31 at a time (T. Pornin, "Optimized Binary GCD for Modular
// Inversion", 2020).  State: a, b >= 0 and u, v mod p with a = u y and
// b = v y (mod p), starting from (a, b, u, v) = (y, p, 1, 0).  One divstep:
// if a is odd, order the pair so that a >= b and replace a by a - b; then
// halve a.  Thirty-one divsteps only look at the low 31 bits of a and b
// (parity) and at their top bits (the comparisons), so they run on 64-bit
// approximations built from the low 31 bits and the 33 bits below the common
// bit length; their effect is a matrix [[f0, g0], [f1, g1]] with
// |f| + |g| <= 2^31, applied once to the full values:
//   a <- (f0 a + g0 b) / 2^31,  b <- (f1 a + g1 b) / 2^31
// (made non-negative by flipping the row's sign when needed), and likewise to
// u, v with the division by 2^31 done mod p (add m p with m = -x mod 2^31,
// valid because p = 1 mod 2^46).  After 2 * 377 - 1 divsteps a = 0 and
// b = gcd = 1, so v = y^-1; 26 rounds of 31 cover them (extra rounds leave
// the state unchanged once a = 0).  Plain C++ throughout: the loop is
// data-dependent per lane.
// ---------------------------------------------------------------------------

constexpr int INV_ROUNDS = 26;

// larger bit length of a and b
__device__ __forceinline__ uint32_t bitlen_max(const fe& a, const fe& b) {
  uint32_t n = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const uint32_t w = a.v[i] | b.v[i];
    n = w ? (uint32_t)(32 * i + 32) - (uint32_t)__builtin_clz(w) : n;
  }
  return n;
}

// the 64 bits of x starting at bit pos (0 <= pos < 384), zero-filled
__device__ __forceinline__ uint64_t bits_at(const fe& x, uint32_t pos) {
  const uint32_t wi = pos >> 5, sh = pos & 31;
  uint32_t w0 = 0, w1 = 0, w2 = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    w0 = ((uint32_t)i == wi) ? x.v[i] : w0;
    w1 = ((uint32_t)i == wi + 1) ? x.v[i] : w1;
    w2 = ((uint32_t)i == wi + 2) ? x.v[i] : w2;
  }
  const uint64_t lo = ((uint64_t)w1 << 32) | w0;
  uint64_t r = lo >> sh;
  if (sh) r |= (uint64_t)w2 << (64 - sh);
  return r;
}

// w[0..12] = x f + y g as a 13-word two's-complement value; needs
// |f| + |g| <= 2^31 so that every partial sum fits in int64
__device__ __forceinline__ void lin_comb(const fe& x, const fe& y, int64_t f, int64_t g,
                                         uint32_t* w) {
  int64_t carry = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int64_t t = (int64_t)x.v[i] * f + (int64_t)y.v[i] * g + carry;
    w[i] = (uint32_t)t;
    carry = t >> 32;
  }
  w[NL] = (uint32_t)carry;
}

// two's complement negation of a 12-word value
__device__ __forceinline__ fe fe_neg_words(const fe& x) {
  fe r;
  uint64_t c = 1;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    c += (uint64_t)(~x.v[i]);
    r.v[i] = (uint32_t)c;
    c >>= 32;
  }
  return r;
}

// (x f + y g) / 2^K for non-negative x, y whose combination is divisible by
// 2^K and below 2^384 in magnitude: returns the magnitude, neg = sign
template <int K>
__device__ __forceinline__ fe comb_shift(const fe& x, const fe& y, int64_t f, int64_t g,
                                         bool& neg) {
  uint32_t w[NL + 1];
  lin_comb(x, y, f, g, w);
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.v[i] = __builtin_amdgcn_alignbit(w[i + 1], w[i], K);
  neg = (int32_t)w[NL] < 0;
  return neg ? fe_neg_words(r) : r;
}

// (x f + y g) / 2^K mod p for canonical x, y; canonical result
template <int K>
__device__ __forceinline__ fe comb_shift_mod(const fe& x, const fe& y, int64_t f, int64_t g) {
  uint32_t w[NL + 1];
  lin_comb(x, y, f, g, w);
  const uint32_t m = (0u - w[0]) & ((1u << K) - 1u);  // makes the sum divisible by 2^K
  uint32_t r[NL];
  uint64_t c = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    c = (uint64_t)w[i] + (uint64_t)m * kP[i] + (c >> 32);
    r[i] = (uint32_t)c;
  }
  const int64_t top = (int64_t)(int32_t)w[NL] + (int64_t)(c >> 32);
  fe q;
#pragma unroll
  for (int i = 0; i < NL - 1; ++i) q.v[i] = __builtin_amdgcn_alignbit(r[i + 1], r[i], K);
  q.v[NL - 1] = __builtin_amdgcn_alignbit((uint32_t)top, r[NL - 1], K);
  // |x f + y g| <= 2^K p and m p < 2^K p, so q lies in (-p, 2p)
  const fe P = fe_const(kP);
  if ((top >> K) < 0) return fe_add_c(q, P);
  fe d;
  const uint32_t borrow = fe_sub_c(q, P, d);
  return borrow ? q : d;
}

// lane 0's value of x (for values that are the same in every lane)
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(x >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
}

// Out-of-line product for code that runs once per result (the conversion
// below): one wave runs it a single time from a cold instruction cache, where
// ten inlined copies of the multiply cost more in instruction fetch than in
// arithmetic.  The operands travel as 4-word vectors, which the calling
// convention keeps in registers (two 12-word structures exceed its register
// budget for aggregate arguments and would go through memory).
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__device__ __noinline__ fe fe_mul_outlined(u32x4_t a0, u32x4_t a1, u32x4_t a2, u32x4_t b0,
                                           u32x4_t b1, u32x4_t b2) {
  fe a, b;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    a.v[i] = a0[i];
    a.v[4 + i] = a1[i];
    a.v[8 + i] = a2[i];
    b.v[i] = b0[i];
    b.v[4 + i] = b1[i];
    b.v[8 + i] = b2[i];
  }
  return fe_mul(a, b);
}
__device__ __forceinline__ fe fe_mul_cold(const fe& a, const fe& b) {
  const uint32_t* x = a.v;
  const uint32_t* y = b.v;
  return fe_mul_outlined(u32x4_t{x[0], x[1], x[2], x[3]}, u32x4_t{x[4], x[5], x[6], x[7]},
                         u32x4_t{x[8], x[9], x[10], x[11]}, u32x4_t{y[0], y[1], y[2], y[3]},
                         u32x4_t{y[4], y[5], y[6], y[7]}, u32x4_t{y[8], y[9], y[10], y[11]});
}

// K divsteps of the uniform inversion on the scalar unit.  a = (a1:a0) and
// b = (b1:b0) are the 64-bit approximations; each matrix row travels packed as
// one 64-bit integer P = f + g 2^32 (p0: f0, g0; p1: f1, g1), on which the
// row operations (difference, doubling, swap) act as on the pair, so a divstep
// is a short run of scalar instructions whose selects all read the scalar
// condition code: set by the borrow of a - b (a < b), then by a odd and
// a < b (swap), then by a odd.
__device__ __forceinline__ void divstep_scalar(uint32_t& a0, uint32_t& a1, uint32_t& b0,
                                               uint32_t& b1, uint32_t& p0l, uint32_t& p0h,
                                               uint32_t& p1l, uint32_t& p1h) {
  uint32_t d0, d1, n0, n1, t, q0l, q0h, e0, e1;
  asm volatile(
      "s_sub_u32 %[d0], %[a0], %[b0]\n\t"
      "s_subb_u32 %[d1], %[a1], %[b1]\n\t"      // d = a - b, SCC = a < b
      "s_cselect_b32 %[t], 1, 0\n\t"
      "s_sub_u32 %[n0], 0, %[d0]\n\t"
      "s_subb_u32 %[n1], 0, %[d1]\n\t"          // n = b - a
      "s_and_b32 %[t], %[a0], %[t]\n\t"          // SCC = swap = a odd and a < b
      "s_cselect_b32 %[d0], %[n0], %[d0]\n\t"
      "s_cselect_b32 %[d1], %[n1], %[d1]\n\t"    // |a - b|
      "s_cselect_b32 %[q0l], %[p1l], %[p0l]\n\t"
      "s_cselect_b32 %[q0h], %[p1h], %[p0h]\n\t"
      "s_cselect_b32 %[p1l], %[p0l], %[p1l]\n\t"
      "s_cselect_b32 %[p1h], %[p0h], %[p1h]\n\t"  // rows swapped
      "s_cselect_b32 %[b0], %[a0], %[b0]\n\t"
      "s_cselect_b32 %[b1], %[a1], %[b1]\n\t"    // b = old a on a swap
      "s_sub_u32 %[e0], %[q0l], %[p1l]\n\t"
      "s_subb_u32 %[e1], %[q0h], %[p1h]\n\t"     // row difference
      "s_bitcmp1_b32 %[a0], 0\n\t"               // SCC = a odd
      "s_cselect_b32 %[a0], %[d0], %[a0]\n\t"
      "s_cselect_b32 %[a1], %[d1], %[a1]\n\t"
      "s_cselect_b32 %[p0l], %[e0], %[q0l]\n\t"
      "s_cselect_b32 %[p0h], %[e1], %[q0h]\n\t"
      "s_lshl_b32 %[t], %[a1], 31\n\t"
      "s_lshr_b32 %[a0], %[a0], 1\n\t"
      "s_or_b32 %[a0], %[a0], %[t]\n\t"
      "s_lshr_b32 %[a1], %[a1], 1\n\t"           // a / 2
      "s_add_u32 %[p1l], %[p1l], %[p1l]\n\t"
      "s_addc_u32 %[p1h], %[p1h], %[p1h]"          // row 1 doubled
      : [a0] "+s"(a0), [a1] "+s"(a1), [b0] "+s"(b0), [b1] "+s"(b1), [p0l] "+s"(p0l),
        [p0h] "+s"(p0h), [p1l] "+s"(p1l), [p1h] "+s"(p1h), [d0] "=&s"(d0), [d1] "=&s"(d1),
        [n0] "=&s"(n0), [n1] "=&s"(n1), [t] "=&s"(t), [q0l] "=&s"(q0l), [q0h] "=&s"(q0h),
        [e0] "=&s"(e0), [e1] "=&s"(e1)
      :
      : "scc");
}

// Plain modular inverse y^-1 mod p of a canonical y (0 for y = 0), by rounds of
// divsteps on 64-bit approximations (the low K bits and the top 64 - K bits of
// a, b), each round applying its 2x2 transition matrix to the full values.
// Per lane: 26 rounds of 31 divsteps, 64-bit matrix entries.  UNIFORM (y the
// same in every lane of the wave): rounds of 30 divsteps on the scalar unit
// (divstep_scalar; |entry| <= 2^30), at most 27 of them, ending early once
// a = 0 (b = gcd = 1 then, and v is the inverse): the round count depends on
// y, which is a public result where this form is used.
template <bool UNIFORM = false>
__device__ __noinline__ fe fe_inv_plain(const fe& y) {
  constexpr int K = UNIFORM ? 30 : 31;
  constexpr int ROUNDS = UNIFORM ? 27 : INV_ROUNDS;
  fe a = y, b = fe_const(kP), u = fe_zero(), v = fe_zero();
  u.v[0] = 1u;
  for (int round = 0; round < ROUNDS; ++round) {
    uint32_t n = bitlen_max(a, b);
    n = n < 64 ? 64u : n;
    const uint64_t lomask = (1ull << K) - 1, himask = (1ull << (64 - K)) - 1;
    uint64_t ab = (a.v[0] & lomask) | ((bits_at(a, n - (64 - K)) & himask) << K);
    uint64_t bb = (b.v[0] & lomask) | ((bits_at(b, n - (64 - K)) & himask) << K);
    if constexpr (UNIFORM) {
      ab = uniform64(ab);
      bb = uniform64(bb);
    }
    int64_t F0, G0, F1, G1;
    if constexpr (UNIFORM) {
      uint32_t a0 = (uint32_t)ab, a1 = (uint32_t)(ab >> 32), b0 = (uint32_t)bb,
               b1 = (uint32_t)(bb >> 32);
      uint32_t p0l = 1u, p0h = 0u, p1l = 0u, p1h = 1u;
#pragma unroll
      for (int j = 0; j < K; ++j) divstep_scalar(a0, a1, b0, b1, p0l, p0h, p1l, p1h);
      // unpack P = f + g 2^32 with |f|, |g| <= 2^30
      const int64_t P0 = (int64_t)(((uint64_t)p0h << 32) | p0l);
      const int64_t P1 = (int64_t)(((uint64_t)p1h << 32) | p1l);
      F0 = (int32_t)p0l;
      F1 = (int32_t)p1l;
      G0 = (P0 - F0) >> 32;
      G1 = (P1 - F1) >> 32;
    } else {
      int64_t f0 = 1, g0 = 0, f1 = 0, g1 = 1;
      for (int j = 0; j < K; ++j) {
        const bool odd = (ab & 1u) != 0;
        unsigned long long d;
        const bool lt = __builtin_usubll_overflow(ab, bb, &d);  // d = ab - bb, lt = ab < bb
        const bool sw = odd && lt;
        const int64_t tf0 = sw ? f1 : f0, tf1 = sw ? f0 : f1;
        const int64_t tg0 = sw ? g1 : g0, tg1 = sw ? g0 : g1;
        const uint64_t na = odd ? (sw ? (0ull - d) : (uint64_t)d) : ab;  // |ab - bb| or ab
        bb = sw ? ab : bb;
        ab = na >> 1;
        f0 = odd ? tf0 - tf1 : tf0;
        g0 = odd ? tg0 - tg1 : tg0;
        f1 = tf1 * 2;
        g1 = tg1 * 2;
      }
      F0 = f0;
      G0 = g0;
      F1 = f1;
      G1 = g1;
    }
    bool na, nb;
    const fe a2 = comb_shift<K>(a, b, F0, G0, na);
    const fe b2 = comb_shift<K>(a, b, F1, G1, nb);
    if (na) {
      F0 = -F0;
      G0 = -G0;
    }
    if (nb) {
      F1 = -F1;
      G1 = -G1;
    }
    const fe u2 = comb_shift_mod<K>(u, v, F0, G0);
    const fe v2 = comb_shift_mod<K>(u, v, F1, G1);
    a = a2;
    b = b2;
    u = u2;
    v = v2;
    if constexpr (UNIFORM) {
      uint32_t o = 0;
#pragma unroll
      for (int i = 0; i < NL; ++i) o |= a.v[i];
      if (__builtin_amdgcn_readfirstlane((int)o) == 0) break;
    }
  }
  return v;
}

// Inverse in Montgomery form: (aR)^-1 R^3 R^-1 = a^-1 R.  Input any value < 2p
// representing aR; output canonical.
template <bool UNIFORM = false>
__device__ __forceinline__ fe fe_inv_mont(const fe& am) {
  fe inv = fe_inv_plain<UNIFORM>(fe_canon(am));
  return fe_canon(fe_mul_cold(inv, fe_const(kR3)));
}

// Twisted-Edwards extended (Montgomery form) -> Weierstrass affine, ordinary
// form, canonical.  Returns false for the identity (x = y = 0 written).
template <bool UNIFORM = false>
__device__ __forceinline__ bool te_to_weierstrass(const xytz& q, fe& xw, fe& yw) {
  fe X = fe_canon(q.X);
  if (fe_is_zero_canon(X)) {
    xw = fe_zero();
    yw = fe_zero();
    return false;
  }
  const fe p2 = fe_const(kP2);
  fe zpy = fe_add(q.Z, q.Y);           // Z + Y
  fe zmy = fe_sub_plus(q.Z, q.Y, p2);  // Z - Y
  fe one = fe_zero();
  one.v[0] = 1u;
  fe inv = fe_inv_mont<UNIFORM>(fe_mul_cold(zmy, q.X));
  fe u = fe_mul_cold(fe_mul_cold(zpy, q.X), inv);  // (Z + Y) / (Z - Y)
  fe v = fe_mul_cold(fe_mul_cold(zpy, q.Z), inv);  // u / x_e
  fe au = fe_mul_cold(u, fe_const(kAlpha));
  xw = fe_canon(fe_mul_cold(fe_sub_plus(au, fe_const(kOne), p2), one));  // out of Montgomery form
  yw = fe_canon(fe_mul_cold(fe_mul_cold(v, fe_const(kBeta)), one));
  return true;
}

// ---------------------------------------------------------------------------
// scalars
// ---------------------------------------------------------------------------
struct scalar256 {
  uint32_t w[SCALAR_WORDS];
};

// Load scalar i; bits >= 253 are reported through *flags and ignored.
__device__ __forceinline__ scalar256 ld_scalar(const uint32_t* __restrict__ s, uint32_t i,
                                               uint32_t* __restrict__ flags) {
  const uint4* q = reinterpret_cast<const uint4*>(s + (size_t)i * SCALAR_WORDS);
  uint4 a = q[0], b = q[1];
  scalar256 r;
  r.w[0] = a.x; r.w[1] = a.y; r.w[2] = a.z; r.w[3] = a.w;
  r.w[4] = b.x; r.w[5] = b.y; r.w[6] = b.z; r.w[7] = b.w;
  if (r.w[7] >> (SCALAR_BITS - 224)) {
    if (flags) atomicOr(flags, MSM_FLAG_RANGE);
    r.w[7] &= (1u << (SCALAR_BITS - 224)) - 1u;
  }
  return r;
}

// c-bit digit starting at bit position pos (c <= 20, pos < 253)
// Endomorphism split (optional, not in the paper): lambda = x0^2 - 1 with
// lambda^2 + lambda + 1 = r; s = s1 lambda + s0 with 0 <= s0 < lambda and
// s1 < 2^127 for every s < 2^253.  q = floor(s mu / 2^380) with
// mu = floor(2^380 / lambda) is the quotient or one below it (the error
// s (2^380 / lambda - mu) / 2^380 is below 2^-127), fixed by one compare.
constexpr uint32_t kGlvLambda[4] = {0x00000000u, 0x0a118000u, 0x90000001u, 0x452217ccu};
constexpr uint32_t kGlvMu[8] = {0xb7b820d2u, 0x55cc5a03u, 0x76f25c6bu, 0xc3366fc8u,
                                0x2af90182u, 0x07f72ed3u, 0x69fd3716u, 0x3b3f7aa9u};

__device__ __forceinline__ void glv_split(const scalar256& s, scalar256& s0, scalar256& s1) {
  uint32_t prod[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) prod[k] = 0u;
#pragma unroll
  for (int i = 0; i < SCALAR_WORDS; ++i) {
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      c = (uint64_t)s.w[i] * kGlvMu[j] + prod[i + j] + (c >> 32);
      prod[i + j] = (uint32_t)c;
    }
    prod[i + 8] = (uint32_t)(c >> 32);
  }
  uint32_t q[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = __builtin_amdgcn_alignbit(prod[12 + k], prod[11 + k], 28);
  // r = s - q lambda (fits in 5 words: r < 2 lambda)
  uint32_t ql[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) ql[k] = 0u;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      c = (uint64_t)q[i] * kGlvLambda[j] + ql[i + j] + (c >> 32);
      ql[i + j] = (uint32_t)c;
    }
    ql[i + 4] = (uint32_t)(c >> 32);
  }
  uint32_t r[SCALAR_WORDS];
  uint32_t borrow = 0;
#pragma unroll
  for (int k = 0; k < SCALAR_WORDS; ++k) {
    const uint64_t d = (uint64_t)s.w[k] - ql[k] - borrow;
    r[k] = (uint32_t)d;
    borrow = (uint32_t)(d >> 63);
  }
  // r >= lambda: subtract once more and bump the quotient
  uint32_t t[SCALAR_WORDS];
  borrow = 0;
#pragma unroll
  for (int k = 0; k < SCALAR_WORDS; ++k) {
    const uint64_t d = (uint64_t)r[k] - (k < 4 ? kGlvLambda[k] : 0u) - borrow;
    t[k] = (uint32_t)d;
    borrow = (uint32_t)(d >> 63);
  }
  const bool ge = borrow == 0;
  uint64_t inc = ge ? 1u : 0u;
#pragma unroll
  for (int k = 0; k < SCALAR_WORDS; ++k) {
    s0.w[k] = ge ? t[k] : r[k];
    if (k < 4) {
      inc += q[k];
      s1.w[k] = (uint32_t)inc;
      inc >>= 32;
    } else {
      s1.w[k] = 0u;
    }
  }
}

__device__ __forceinline__ uint32_t digit_at(const scalar256& s, int pos, int c) {
  int wi = pos >> 5, sh = pos & 31;
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int j = 0; j < SCALAR_WORDS; ++j) {
    lo = (j == wi) ? s.w[j] : lo;
    hi = (j == wi + 1) ? s.w[j] : hi;
  }
  uint64_t two = ((uint64_t)hi << 32) | lo;
  return (uint32_t)(two >> sh) & ((1u << c) - 1u);
}

}  // namespace msm
