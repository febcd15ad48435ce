// Field inversion and the Weierstrass <-> twisted-Edwards conversions (device).
#pragma once
#include "common.hpp"

namespace msm {

__device__ __forceinline__ bool fe_is_one_plain(const fe& a) {
  uint32_t o = a.v[0] ^ 1u;
#pragma unroll
  for (int i = 1; i < NL; ++i) o |= a.v[i];
  return o == 0;
}

// a >> t for 0 <= t <= 31
__device__ __forceinline__ fe fe_shr(const fe& a, uint32_t t) {
  fe r;
#pragma unroll
  for (int i = 0; i < NL - 1; ++i) r.v[i] = __builtin_amdgcn_alignbit(a.v[i + 1], a.v[i], t);
  r.v[NL - 1] = a.v[NL - 1] >> t;
  return r;
}

// x * 2^-t mod p for canonical x and 1 <= t <= 31: adds m p with
// m = -x mod 2^t (p = 1 mod 2^46, so -p^-1 = -1 mod 2^t), making the sum
// divisible by 2^t; the quotient is < (x + (2^t - 1) p) / 2^t < p.
__device__ __forceinline__ fe fe_div_pow2(const fe& x, uint32_t t) {
  const uint32_t m = (0u - x.v[0]) & ((1u << t) - 1u);
  uint32_t y[NL + 1];
  uint64_t acc = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    acc = (uint64_t)m * kP[i] + x.v[i] + (acc >> 32);
    y[i] = (uint32_t)acc;
  }
  y[NL] = (uint32_t)(acc >> 32);
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.v[i] = __builtin_amdgcn_alignbit(y[i + 1], y[i], t);
  return r;
}

// Plain C++ multiword helpers for the data-dependent inversion loop.  The
// hand-scheduled carry sequences of field.hpp pass carries through wave-wide
// lane masks, which the compiler treats as uniform values; inside the
// divergent branches of this loop the compiler is left to derive the carry
// code itself.

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

// x - y mod p for canonical x, y
__device__ __forceinline__ fe fe_sub_mod(const fe& x, const fe& y) {
  fe d;
  uint32_t br = fe_sub_c(x, y, d);
  return br ? fe_add_c(d, fe_const(kP)) : d;
}

// Plain modular inverse a^-1 mod p of a canonical 0 < a < p by the binary
// extended Euclidean algorithm (invariants x1 a = u, x2 a = v mod p); factors
// of two are removed up to 31 at a time.  Returns 0 for a = 0.  Every pass
// removes at least one bit from u or v or makes one of them even, so 2048
// passes always suffice (at most ~600 are used) and the loop is bounded.
__device__ __noinline__ fe fe_inv_plain(const fe& a) {
  if (fe_is_zero_canon(a)) return fe_zero();
  fe u = a, v = fe_const(kP);
  fe x1 = fe_zero(), x2 = fe_zero();
  x1.v[0] = 1u;
  for (int guard = 0; guard < 2048; ++guard) {
    if (fe_is_one_plain(u)) return x1;
    if (fe_is_one_plain(v)) return x2;
    if ((u.v[0] & 1u) == 0u) {
      uint32_t t = u.v[0] ? (uint32_t)__builtin_ctz(u.v[0]) : 31u;
      u = fe_shr(u, t);
      x1 = fe_div_pow2(x1, t);
    } else if ((v.v[0] & 1u) == 0u) {
      uint32_t t = v.v[0] ? (uint32_t)__builtin_ctz(v.v[0]) : 31u;
      v = fe_shr(v, t);
      x2 = fe_div_pow2(x2, t);
    } else {
      fe d;
      if (!fe_sub_c(u, v, d)) {  // u >= v
        u = d;
        x1 = fe_sub_mod(x1, x2);
      } else {
        fe_sub_c(v, u, d);
        v = d;
        x2 = fe_sub_mod(x2, x1);
      }
    }
  }
  return fe_zero();
}

// Inverse in Montgomery form: (aR)^-1 R^3 R^-1 = a^-1 R.  Input any value < 2p
// representing aR; output canonical.
__device__ __forceinline__ fe fe_inv_mont(const fe& am) {
  fe inv = fe_inv_plain(fe_canon(am));
  return fe_canon(fe_mul(inv, fe_const(kR3)));
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
  fe inv = fe_inv_mont(fe_mul(zmy, q.X));
  fe u = fe_mul(fe_mul(zpy, q.X), inv);  // (Z + Y) / (Z - Y)
  fe v = fe_mul(fe_mul(zpy, q.Z), inv);  // u / x_e
  fe au = fe_mul(u, fe_const(kAlpha));
  xw = fe_from_mont(fe_sub_plus(au, fe_const(kOne), p2));
  yw = fe_from_mont(fe_mul(v, fe_const(kBeta)));
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
