// Twisted-Edwards point additions on the carry-free 28-bit field form
// (fe28.hpp): the one-lane throughput unit of bucket accumulation, the
// standalone PADD kernel and the split-bucket merges.
//
// Same unified law as curve.hpp (Hisil, Wong, Carter and Dawson 2008, a = -1,
// Sec. II-D):
//   A = (Y1 - X1)(Y2 - X2)   B = (Y1 + X1)(Y2 + X2)   C = T1 k T2   D = 2 Z1 Z2
//   E = B - A   F = D - C   G = D + C   H = B + A
//   X3 = E F    Y3 = G H    T3 = E H    Z3 = F G
// computed with R' = 2^392 products.  Extended points read from the 12-word
// form (R = 2^384) are the same projective points in R'-form (all four
// coordinates scaled by 2^-8), so they are used as they are.  A prepared
// point (X, Y, U = kT, Z = 1 in R-form) is, in R'-form, the point with
// Z2 = 2^-8 and U2 = k T2, hence D = 2 Z1 2^-8 (f28_div128x2) and C = T1 U2.
//
// Bounds (fe28.hpp conventions; "n" = normalised limbs, values in units of p):
//   inputs: n, < 2p (prepared inputs canonical, < p)
//   Y1 - X1 + 4p < 6p, limbs < 2^29 + 2^28    Y1 + X1 < 4p, limbs < 2^29
//   A, B, C: n, < 2p     D (mixed) < 1.01p, limbs < 2^29;  D (complete) < 4p, limbs < 2^29
//   E = B - A + 4p < 6p, limbs < 2^29 + 2^28   H = B + A < 4p, limbs < 2^29
//   F = D - C + 4p < 8p, limbs < 2^30          G = D + C < 6p, limbs < 2^29 + 2^28
// so every product operand has limbs < 2^30 and every product is below
// 48 p^2 < R' p; outputs are n and < 2p.
#pragma once
#include "curve.hpp"
#include "fe28.hpp"

namespace msm {

struct xytz28 {
  fe28 X, Y, T, Z;
};

struct xyu28 {
  fe28 X, Y, U;
};

// identity (0 : 1 : 0 : 1); any common non-zero Y = Z is the same point
__device__ __forceinline__ xytz28 pt28_identity() {
  xytz28 r;
  r.X = f28_small(0u);
  r.Y = f28_small(1u);
  r.T = f28_small(0u);
  r.Z = f28_small(1u);
  return r;
}

__device__ __forceinline__ xytz28 pt28_from(const xytz& p) {
  xytz28 r;
  r.X = f28_from_words(p.X);
  r.Y = f28_from_words(p.Y);
  r.T = f28_from_words(p.T);
  r.Z = f28_from_words(p.Z);
  return r;
}

__device__ __forceinline__ xyu28 pt28_from(const xyu& p) {
  xyu28 r;
  r.X = f28_from_words(p.X);
  r.Y = f28_from_words(p.Y);
  r.U = f28_from_words(p.U);
  return r;
}

// outputs of products only (normalised limbs, values < 2p < 2^384)
__device__ __forceinline__ xytz pt28_to_words(const xytz28& p) {
  xytz r;
  r.X = f28_to_words(p.X);
  r.Y = f28_to_words(p.Y);
  r.T = f28_to_words(p.T);
  r.Z = f28_to_words(p.Z);
  return r;
}

__device__ __forceinline__ xytz28 padd28_tail(const fe28& A, const fe28& B, const fe28& Fp,
                                              const fe28& Gp, bool swapFG) {
  const fe28 E = f28_sub4(B, A);
  const fe28 H = f28_add(B, A);
  const fe28 F = f28_select(swapFG, Gp, Fp);
  const fe28 G = f28_select(swapFG, Fp, Gp);
  xytz28 r;
  r.X = f28_mul(E, F);
  r.Y = f28_mul(G, H);
  r.T = f28_mul(E, H);
  r.Z = f28_mul(F, G);
  return r;
}

// a + b (neg = false) or a - b (neg = true), b prepared.  -b = (-X2, Y2, -U2)
// exchanges Y2 - X2 with Y2 + X2 and negates C, which exchanges F with G.
// 7 products.
__device__ __forceinline__ xytz28 padd28_mixed_signed(const xytz28& a, const xyu28& b, bool neg) {
  const fe28 bm = f28_sub4(b.Y, b.X);
  const fe28 bp = f28_add(b.Y, b.X);
  const fe28 A = f28_mul(f28_sub4(a.Y, a.X), f28_select(neg, bp, bm));
  const fe28 B = f28_mul(f28_add(a.Y, a.X), f28_select(neg, bm, bp));
  const fe28 C = f28_mul(a.T, b.U);
  const fe28 D = f28_div128x2(a.Z);
  return padd28_tail(A, B, f28_sub4(D, C), f28_add(D, C), neg);
}

__device__ __forceinline__ xytz28 padd28_mixed(const xytz28& a, const xyu28& b) {
  const fe28 A = f28_mul(f28_sub4(a.Y, a.X), f28_sub4(b.Y, b.X));
  const fe28 B = f28_mul(f28_add(a.Y, a.X), f28_add(b.Y, b.X));
  const fe28 C = f28_mul(a.T, b.U);
  const fe28 D = f28_div128x2(a.Z);
  return padd28_tail(A, B, f28_sub4(D, C), f28_add(D, C), false);
}

// a + b, both extended: 9 products (k T2 formed on the fly).
__device__ __forceinline__ xytz28 padd28_full(const xytz28& a, const xytz28& b) {
  const fe28 A = f28_mul(f28_sub4(a.Y, a.X), f28_sub4(b.Y, b.X));
  const fe28 B = f28_mul(f28_add(a.Y, a.X), f28_add(b.Y, b.X));
  const fe28 C = f28_mul(a.T, f28_mul(b.T, f28_const(kK28)));
  const fe28 Zp = f28_mul(a.Z, b.Z);
  const fe28 D = f28_add(Zp, Zp);
  return padd28_tail(A, B, f28_sub4(D, C), f28_add(D, C), false);
}

}  // namespace msm
