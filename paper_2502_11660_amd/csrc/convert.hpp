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
// the state unchanged once a = 0).  The per-lane form is plain C++ (the loop
// is data-dependent per lane); the form for one value per wave
// (fe_inv_lanes) spreads the words over the lanes and runs the divsteps on
// the scalar unit.
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

// Out-of-line product for code that runs once per result (the conversion
// below): inlined, its ten multiplies make a long straight-line kernel that
// each wave runs once from a cold instruction cache, where instruction fetch
// costs more than the arithmetic.  The operands travel as 4-word vectors, which the calling
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

// 30 divsteps of the uniform inversion on the scalar unit.  a and b are the
// 64-bit approximations; each matrix row travels packed as one 64-bit integer
// P = f + g 2^32 (P0: f0, g0; P1: f1, g1), on which the row operations
// (difference, doubling, swap) act as on the pair.  A divstep is 17 scalar
// instructions whose selects read the scalar condition code: set by the
// borrow of a - b (a < b), then by a odd and a < b (swap), then by a odd.
// The operands sit in fixed register pairs so that the 64-bit selects and
// shifts can name their halves.
__device__ __forceinline__ void divsteps30_scalar(uint64_t& a, uint64_t& b, uint64_t& P0,
                                                  uint64_t& P1) {
  asm volatile(
      ".rept 30\n\t"
      "s_sub_u32 s88, s80, s82\n\t"
      "s_subb_u32 s89, s81, s83\n\t"                  // d = a - b, SCC = a < b
      "s_cselect_b32 s96, 1, 0\n\t"
      "s_sub_u32 s90, 0, s88\n\t"
      "s_subb_u32 s91, 0, s89\n\t"                    // n = b - a
      "s_and_b32 s96, s80, s96\n\t"                   // SCC = swap: a odd, a < b
      "s_cselect_b64 s[88:89], s[90:91], s[88:89]\n\t"  // |a - b|
      "s_cselect_b64 s[92:93], s[86:87], s[84:85]\n\t"  // rows swapped: q0 ...
      "s_cselect_b64 s[86:87], s[84:85], s[86:87]\n\t"  // ... and P1
      "s_cselect_b64 s[82:83], s[80:81], s[82:83]\n\t"  // b = old a on a swap
      "s_sub_u32 s94, s92, s86\n\t"
      "s_subb_u32 s95, s93, s87\n\t"                  // row difference q0 - P1
      "s_bitcmp1_b32 s80, 0\n\t"                      // SCC = a odd
      "s_cselect_b64 s[80:81], s[88:89], s[80:81]\n\t"
      "s_cselect_b64 s[84:85], s[94:95], s[92:93]\n\t"
      "s_lshr_b64 s[80:81], s[80:81], 1\n\t"          // a / 2
      "s_lshl_b64 s[86:87], s[86:87], 1\n\t"          // row 1 doubled
      ".endr"
      : "+{s[80:81]}"(a), "+{s[82:83]}"(b), "+{s[84:85]}"(P0), "+{s[86:87]}"(P1)
      :
      : "s88", "s89", "s90", "s91", "s92", "s93", "s94", "s95", "s96", "scc");
}

// Plain modular inverse y^-1 mod p of a canonical y (0 for y = 0), per lane:
// 26 rounds of 31 divsteps on 64-bit approximations (the low 31 bits and the
// top 33 bits of a, b), each round applying its 2x2 transition matrix
// (64-bit entries) to the full values.
__device__ __noinline__ fe fe_inv_plain(const fe& y) {
  constexpr int K = 31;
  fe a = y, b = fe_const(kP), u = fe_zero(), v = fe_zero();
  u.v[0] = 1u;
  for (int round = 0; round < INV_ROUNDS; ++round) {
    uint32_t n = bitlen_max(a, b);
    n = n < 64 ? 64u : n;
    const uint64_t lomask = (1ull << K) - 1, himask = (1ull << (64 - K)) - 1;
    uint64_t ab = (a.v[0] & lomask) | ((bits_at(a, n - (64 - K)) & himask) << K);
    uint64_t bb = (b.v[0] & lomask) | ((bits_at(b, n - (64 - K)) & himask) << K);
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
    bool na, nb;
    const fe a2 = comb_shift<K>(a, b, f0, g0, na);
    const fe b2 = comb_shift<K>(a, b, f1, g1, nb);
    if (na) {
      f0 = -f0;
      g0 = -g0;
    }
    if (nb) {
      f1 = -f1;
      g1 = -g1;
    }
    const fe u2 = comb_shift_mod<K>(u, v, f0, g0);
    const fe v2 = comb_shift_mod<K>(u, v, f1, g1);
    a = a2;
    b = b2;
    u = u2;
    v = v2;
  }
  return v;
}

// ---------------------------------------------------------------------------
// The same inversion for a value held by every lane of a wave (one result per
// wave), with the lanes put to work: lane 16 s + i holds word i (i < 12;
// words 12..15 are zero) of segment s's operand pair, (a, b) in segments 0
// and 1, (u, v) in segments 2 and 3.  A round reads the approximations of a
// and b out of segment 0 (lane reads), runs its 30 divsteps on the scalar unit
// (divsteps30_scalar), and then each segment forms its own combination at once:
// 0: f0 a + g0 b, 1: f1 a + g1 b, 2: f0 u + g0 v + m p, 3: f1 u + g1 v + m p,
// one word per lane (64-bit column products), turned into two's complement
// words by two carry-lookahead passes over 16-lane rows, divided by 2^30 (a
// funnel shift with the next lane's word), then made non-negative (a, b) or
// reduced to [0, p) (u, v), and u, v negated mod p where the row of a, b
// changed sign.  The rounds end once a = 0 (then b = gcd = 1 and v is the
// inverse; at most 27 rounds cover the 753 divsteps): the round count depends
// on y, which is a public result where this form is used.
// ---------------------------------------------------------------------------

constexpr uint64_t kRowTops = 0x8000800080008000ull;  // lane 15 of each row

// Completes per-lane sums x < 2^33 (row-wise multiword additions, word i in
// lane 16 s + i) by carry lookahead: a lane generates a carry when x >= 2^32
// and passes one on when its word is all ones; no carry leaves a row.
__device__ __forceinline__ uint32_t row_carry(uint64_t x) {
  const uint64_t g = __ballot((x >> 32) != 0u) & ~kRowTops;
  const uint64_t pp = __ballot((uint32_t)x == 0xffffffffu) & ~kRowTops;
  const uint64_t gp = g | pp;
  const uint64_t c = (g + gp) ^ g ^ gp;  // bit l: carry into lane l
  return (uint32_t)x + (uint32_t)((c >> __lane_id()) & 1u);
}

// word of the lane below / above in the same row (0 past the row's ends)
__device__ __forceinline__ uint32_t row_from_below(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x111, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t row_from_above(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x101, 0xF, 0xF, true);
}

// word i of a 12-word constant (0 for i >= 12)
__device__ __forceinline__ uint32_t word_of_const(const uint32_t (&c)[NL], uint32_t i) {
  uint32_t r = 0u;
#pragma unroll
  for (uint32_t k = 0; k < (uint32_t)NL; ++k) r = (i == k) ? c[k] : r;
  return r;
}

__device__ __noinline__ fe fe_inv_lanes(fe y) {  // by value: kept in registers
  constexpr int K = 30;
  constexpr int ROUNDS = 27;
  const uint32_t l = __lane_id(), s = l >> 4, i = l & 15u, top = (l & 48u) | 12u;
  const uint32_t pw = word_of_const(kP, i);
  // -(2^31 sum_{j=1..13} 2^(32 j)) mod 2^512, the bias of the high halves
  const uint32_t negc = i == 0 ? 0u : (i == 1 ? 0x80000000u : (i < 14 ? 0x7fffffffu : ~0u));
  uint32_t yw = 0u;
#pragma unroll
  for (uint32_t k = 0; k < (uint32_t)NL; ++k) yw = (i == k) ? y.v[k] : yw;
  uint32_t X = s < 2 ? yw : (i == 0 ? 1u : 0u);  // a = y, u = 1
  uint32_t Y = s < 2 ? pw : 0u;                  // b = p, v = 0
  for (int round = 0; round < ROUNDS; ++round) {
    // 64-bit approximations of a and b: the low K bits and the 64 - K bits
    // below their common bit length
    const uint32_t w = X | Y;
    const uint64_t nzw = __ballot(l < 12u && w != 0u);
    uint32_t n = 0;
    if (nzw != 0u) {
      const uint32_t t = 63u - (uint32_t)__builtin_clzll(nzw);
      const uint32_t wt = (uint32_t)__builtin_amdgcn_readlane((int)w, (int)t);
      n = 32u * t + 32u - (uint32_t)__builtin_clz(wt);
    }
    n = n < 64u ? 64u : n;
    const uint32_t pos = n - (64 - K), i0 = pos >> 5, sh = pos & 31u;
    const uint32_t xa0 = (uint32_t)__builtin_amdgcn_readlane((int)X, (int)i0);
    const uint32_t xa1 = (uint32_t)__builtin_amdgcn_readlane((int)X, (int)i0 + 1);
    const uint32_t xa2 = (uint32_t)__builtin_amdgcn_readlane((int)X, (int)i0 + 2);
    const uint32_t xb0 = (uint32_t)__builtin_amdgcn_readlane((int)Y, (int)i0);
    const uint32_t xb1 = (uint32_t)__builtin_amdgcn_readlane((int)Y, (int)i0 + 1);
    const uint32_t xb2 = (uint32_t)__builtin_amdgcn_readlane((int)Y, (int)i0 + 2);
    const uint32_t alo = (uint32_t)__builtin_amdgcn_readlane((int)X, 0);
    const uint32_t blo = (uint32_t)__builtin_amdgcn_readlane((int)Y, 0);
    uint64_t ta = ((((uint64_t)xa1) << 32) | xa0) >> sh;
    uint64_t tb = ((((uint64_t)xb1) << 32) | xb0) >> sh;
    if (sh) {
      ta |= (uint64_t)xa2 << (64 - sh);
      tb |= (uint64_t)xb2 << (64 - sh);
    }
    const uint32_t lomask = (1u << K) - 1u;
    uint64_t ab = (alo & lomask) | (ta << K), bb = (blo & lomask) | (tb << K);
    uint64_t P0 = 1u, P1 = 1ull << 32;
    static_assert(K == 30, "divsteps30_scalar runs 30 divsteps");
    divsteps30_scalar(ab, bb, P0, P1);
    // this segment's row (f, g), unpacked from P = f + g 2^32 (|f|, |g| <= 2^30)
    const uint64_t P = (s & 1u) ? P1 : P0;
    const int32_t f = (int32_t)(uint32_t)P;
    const int32_t g = (int32_t)(((int64_t)P - f) >> 32);
    // column products x f + y g, exact in two's complement 64 bits
    uint64_t t = (uint64_t)X * (uint32_t)f + (uint64_t)Y * (uint32_t)g;
    // m p with m = -(x f + y g) mod 2^K makes the u, v sums divisible by 2^K
    const uint32_t m2 = (0u - (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)t, 32)) & lomask;
    const uint32_t m3 = (0u - (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)t, 48)) & lomask;
    t += (uint64_t)(s == 2 ? m2 : (s == 3 ? m3 : 0u)) * pw;
    const uint32_t hi = (uint32_t)(t >> 32) - (f < 0 ? X : 0u) - (g < 0 ? Y : 0u);
    // two's complement words: low halves plus the high halves of the column
    // below, biased by 2^31 to keep every word sum non-negative, then the
    // bias taken off
    const uint32_t hb = i < 13u ? (hi ^ 0x80000000u) : 0u;
    const uint32_t U = row_carry((uint64_t)(uint32_t)t + row_from_below(hb));
    const uint32_t V = row_carry((uint64_t)U + negc);
    // divided by 2^K; lane 12 holds the sign word
    const uint32_t Q = __builtin_amdgcn_alignbit(row_from_above(V), V, K);
    const uint64_t negm = __ballot(i == 12u && (int32_t)Q < 0);
    const bool neg = ((negm >> top) & 1u) != 0u;
    // a, b: magnitude (-Q = ~Q + 1); u, v: in (-p, 2p), so Q + p when
    // negative, else Q - p (= Q + ~p + 1) kept only without a borrow
    uint32_t xo = Q, yo = 0u;
    if (s < 2u) {
      xo = neg ? ~Q : Q;
      yo = (neg && i == 0u) ? 1u : 0u;
    } else {
      yo = neg ? pw : ~pw + (i == 0u ? 1u : 0u);
    }
    xo = i <= 12u ? xo : 0u;
    yo = i <= 12u ? yo : 0u;
    uint32_t R = row_carry((uint64_t)xo + yo);
    const uint64_t borm = __ballot(i == 12u && (int32_t)R < 0);
    R = (s >= 2u && !neg && ((borm >> top) & 1u)) ? Q : R;
    // u, v negated mod p (p - R, for R != 0) where a, b changed sign
    const uint64_t nzm = __ballot(i < 12u && R != 0u);
    const bool nz = ((nzm >> (l & 48u)) & 0xfffu) != 0u;
    const bool dn = s >= 2u && nz && ((negm >> (((s - 2u) << 4) | 12u)) & 1u);
    xo = i < 12u ? (dn ? ~R : R) : 0u;
    yo = (dn && i < 12u) ? pw + (i == 0u ? 1u : 0u) : 0u;
    R = row_carry((uint64_t)xo + yo);
    R = i < 12u ? R : 0u;
    // segment pairs exchange their results: (a, b) and (u, v) again
    const uint32_t Rp = (uint32_t)__builtin_amdgcn_ds_swizzle((int)R, 0x401F);
    X = (s & 1u) ? Rp : R;
    Y = (s & 1u) ? R : Rp;
    if (__ballot(l < 12u && X != 0u) == 0u) break;  // a = 0
  }
  fe r;
#pragma unroll
  for (int k = 0; k < NL; ++k) r.v[k] = (uint32_t)__builtin_amdgcn_readlane((int)Y, 32 + k);
  return r;
}

// Inverse in Montgomery form: (aR)^-1 R^3 R^-1 = a^-1 R.  Input any value < 2p
// representing aR; output canonical.
__device__ __forceinline__ fe fe_inv_mont(const fe& am) {
  fe inv = fe_inv_plain(fe_canon(am));
  return fe_canon(fe_mul_cold(inv, fe_const(kR3)));
}

// Twisted-Edwards extended (Montgomery form) -> Weierstrass affine, ordinary
// form, canonical.  Returns false for the identity (x = y = 0 written).
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
  fe inv = fe_inv_mont(fe_mul_cold(zmy, q.X));
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
