// Twisted-Edwards point arithmetic for BLS12-377 G1 (device code).
//
// Points live on -x^2 + y^2 = 1 + (k/2) x^2 y^2 in extended projective
// coordinates (X, Y, T, Z), x = X/Z, y = Y/Z, T = XY/Z (Sec. II-D).  Points
// entering bucket accumulation are "prepared": Z = 1 and T replaced by
// U = k T, so the mixed addition needs no multiplication by the curve constant
// (Sec. II-D).  Addition uses the unified extended-coordinate law of Hisil,
// Wong, Carter and Dawson (2008) for a = -1:
//
//   A = (Y1 - X1)(Y2 - X2)   B = (Y1 + X1)(Y2 + X2)   C = T1 k T2   D = 2 Z1 Z2
//   E = B - A   F = D - C   G = D + C   H = B + A
//   X3 = E F    Y3 = G H    T3 = E H    Z3 = F G
//
// The E/F/G/H additions are left unreduced and every subtraction adds 2p
// (Sec. III-E adds 3M for the same reason).  With inputs below 2p (and
// prepared inputs below p) every multiplication operand stays below 6p, so
// every product is below 36 p^2 < R p and each output is again below 2p:
//
//   (Y1-X1+2p) < 4p  (Y2-X2+2p) < 4p  (sums) < 4p   -> A, B, C < 2p
//   D < 4p   E < 4p   F < 6p   G < 6p   H < 4p      -> X3..Z3 < 2p
//
// The law is unified (it doubles correctly) and has no exceptional inputs
// inside the prime-order subgroup, so bucket sums need no special cases; the
// identity is (0, 1, 0, 1).
#pragma once
#include "field.hpp"

namespace msm {

// Montgomery form of the curve constant k = 2d.
constexpr uint32_t kK[NL] = {0x44a706c6u, 0xf24b7e84u, 0x80faa8fau, 0xeae02375u,
                             0x7ef38fa5u, 0x0f4d7cf2u, 0xc5f2bb26u, 0x5597097du,
                             0x0d95a93eu, 0x8bf6c1ddu, 0xfbff628au, 0x01784602u};

struct xytz {
  fe X, Y, T, Z;
};

struct xyu {
  fe X, Y, U;
};

__device__ __forceinline__ xytz pt_identity() {
  xytz r;
  r.X = fe_zero();
  r.Y = fe_const(kOne);
  r.T = fe_zero();
  r.Z = fe_const(kOne);
  return r;
}

// a + b, b prepared (Z2 = 1, U2 = k T2): 7 multiplications.
__device__ __forceinline__ xytz padd_mixed(const xytz& a, const xyu& b, const fe& p2) {
  fe A = fe_mul(fe_sub_plus(a.Y, a.X, p2), fe_sub_plus(b.Y, b.X, p2));
  fe B = fe_mul(fe_add(a.Y, a.X), fe_add(b.Y, b.X));
  fe C = fe_mul(a.T, b.U);
  fe D = fe_add(a.Z, a.Z);
  fe E = fe_sub_plus(B, A, p2);
  fe F = fe_sub_plus(D, C, p2);
  fe G = fe_add(D, C);
  fe H = fe_add(B, A);
  xytz r;
  r.X = fe_mul(E, F);
  r.Y = fe_mul(G, H);
  r.T = fe_mul(E, H);
  r.Z = fe_mul(F, G);
  return r;
}

// a + b or a - b, b prepared: -b = (-X2, Y2, -U2) exchanges Y2 - X2 with
// Y2 + X2 and negates C, which exchanges F with G.  Same bounds as
// padd_mixed; the sign costs selects only.
__device__ __forceinline__ xytz padd_mixed_signed(const xytz& a, const xyu& b, bool neg,
                                                 const fe& p2) {
  const fe bm = fe_sub_plus(b.Y, b.X, p2);
  const fe bp = fe_add(b.Y, b.X);
  fe A = fe_mul(fe_sub_plus(a.Y, a.X, p2), fe_select(neg, bp, bm));
  fe B = fe_mul(fe_add(a.Y, a.X), fe_select(neg, bm, bp));
  fe C = fe_mul(a.T, b.U);
  fe D = fe_add(a.Z, a.Z);
  fe E = fe_sub_plus(B, A, p2);
  const fe Fp = fe_sub_plus(D, C, p2);
  const fe Gp = fe_add(D, C);
  fe F = fe_select(neg, Gp, Fp);
  fe G = fe_select(neg, Fp, Gp);
  fe H = fe_add(B, A);
  xytz r;
  r.X = fe_mul(E, F);
  r.Y = fe_mul(G, H);
  r.T = fe_mul(E, H);
  r.Z = fe_mul(F, G);
  return r;
}

// a + b, both extended: 9 multiplications (k T2 formed on the fly).
__device__ __forceinline__ xytz padd_full(const xytz& a, const xytz& b, const fe& p2) {
  fe A = fe_mul(fe_sub_plus(a.Y, a.X, p2), fe_sub_plus(b.Y, b.X, p2));
  fe B = fe_mul(fe_add(a.Y, a.X), fe_add(b.Y, b.X));
  fe C = fe_mul(a.T, fe_mul(b.T, fe_const(kK)));
  fe Z = fe_mul(a.Z, b.Z);
  fe D = fe_add(Z, Z);
  fe E = fe_sub_plus(B, A, p2);
  fe F = fe_sub_plus(D, C, p2);
  fe G = fe_add(D, C);
  fe H = fe_add(B, A);
  xytz r;
  r.X = fe_mul(E, F);
  r.Y = fe_mul(G, H);
  r.T = fe_mul(E, H);
  r.Z = fe_mul(F, G);
  return r;
}

// 2a by the dedicated doubling for a = -1 (Hisil et al. 2008):
//   A = X^2  B = Y^2  C = 2 Z^2  E = (X+Y)^2 - A - B
//   G = B - A  F = G - C  H = -(A + B)
//   X3 = E F  Y3 = G H  T3 = E H  Z3 = F G
// with non-negative lazily reduced representatives
//   E = S - (A+B) + 4p in (0, 6p)   G = B - A + 2p in (0, 4p)
//   H = 4p - (A+B) in (0, 4p]        F = G - C + 4p in (0, 8p)
// so every product is below 48 p^2 < R p.
__device__ __forceinline__ xytz pdbl(const xytz& a, const fe& p2) {
  fe A = fe_sqr(a.X);
  fe B = fe_sqr(a.Y);
  fe Zs = fe_sqr(a.Z);
  fe C = fe_add(Zs, Zs);
  fe S = fe_sqr(fe_add(a.X, a.Y));
  fe AB = fe_add(A, B);
  fe p4 = fe_add(p2, p2);
  fe E = fe_sub_plus(S, AB, p4);
  fe G = fe_sub_plus(B, A, p2);
  fe H = fe_sub_plus(fe_zero(), AB, p4);
  fe F = fe_sub_plus(G, C, p4);
  xytz r;
  r.X = fe_mul(E, F);
  r.Y = fe_mul(G, H);
  r.T = fe_mul(E, H);
  r.Z = fe_mul(F, G);
  return r;
}

// ---------------------------------------------------------------------------
// memory layouts
// ---------------------------------------------------------------------------

// Structure of arrays, limb-major: word (coord*12 + limb)*count + i.
__device__ __forceinline__ fe ld_soa(const uint32_t* __restrict__ base, size_t count, int coord,
                                    size_t i) {
  fe r;
#pragma unroll
  for (int l = 0; l < NL; ++l) r.v[l] = base[(size_t)(coord * NL + l) * count + i];
  return r;
}

__device__ __forceinline__ void st_soa(uint32_t* __restrict__ base, size_t count, int coord, size_t i,
                                      const fe& x) {
#pragma unroll
  for (int l = 0; l < NL; ++l) base[(size_t)(coord * NL + l) * count + i] = x.v[l];
}

// Array of structures: element e of a record starting at rec (16-byte aligned).
__device__ __forceinline__ fe ld_aos(const uint32_t* __restrict__ rec, int coord) {
  const uint4* q = reinterpret_cast<const uint4*>(rec + coord * NL);
  fe r;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    uint4 w = q[j];
    r.v[4 * j + 0] = w.x;
    r.v[4 * j + 1] = w.y;
    r.v[4 * j + 2] = w.z;
    r.v[4 * j + 3] = w.w;
  }
  return r;
}

__device__ __forceinline__ void st_aos(uint32_t* __restrict__ rec, int coord, const fe& x) {
  uint4* q = reinterpret_cast<uint4*>(rec + coord * NL);
#pragma unroll
  for (int j = 0; j < 3; ++j)
    q[j] = make_uint4(x.v[4 * j + 0], x.v[4 * j + 1], x.v[4 * j + 2], x.v[4 * j + 3]);
}

constexpr int XYU_WORDS = 3 * NL;   // prepared point record: X, Y, U
constexpr int XYTZ_WORDS = 4 * NL;  // extended point record: X, Y, T, Z

__device__ __forceinline__ xyu ld_xyu(const uint32_t* __restrict__ rec) {
  xyu r;
  r.X = ld_aos(rec, 0);
  r.Y = ld_aos(rec, 1);
  r.U = ld_aos(rec, 2);
  return r;
}

__device__ __forceinline__ xytz ld_xytz(const uint32_t* __restrict__ rec) {
  xytz r;
  r.X = ld_aos(rec, 0);
  r.Y = ld_aos(rec, 1);
  r.T = ld_aos(rec, 2);
  r.Z = ld_aos(rec, 3);
  return r;
}

__device__ __forceinline__ void st_xytz(uint32_t* __restrict__ rec, const xytz& p) {
  st_aos(rec, 0, p.X);
  st_aos(rec, 1, p.Y);
  st_aos(rec, 2, p.T);
  st_aos(rec, 3, p.Z);
}

}  // namespace msm
