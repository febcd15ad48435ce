// Latency-oriented point arithmetic on wide elements: two waves per point.
//
// Bucket and group aggregation end in chains of dependent additions and
// doublings (Sec. II-C), served by a separate low-latency PADD mapping
// (Sec. V-A).  Here one point occupies two waves: every formula below has
// four independent products per phase, and the four 32-lane halves of the two
// waves each compute one of them with wmul2 (the half's index k = 2 wave +
// half picks the product).  Coordinates live in LDS between phases as 16
// limbs each; the additions between the products are one integer operation
// per limb.  Subtractions add a multiple of p whose limbs are pre-borrowed
// (2^26 added to limbs 0..14, 4 taken from limbs 1..15), so that every limb
// difference is non-negative.
//
// Lazy bounds (products come back below a b / R + 1.001 p, p / R < 0.0066):
// with every coordinate below 1.2p (inputs below 2p where noted),
//   addition   E = B - A + 3p < 4.2p   F = D - C + 3p < 5.4p
//              G = D + C < 3.6p        H = B + A < 2.4p
//   doubling   E = 2 T Z < 2.4p            G = B - A + 2p < 3.2p
//              H = 3p - A - B <= 3p        F = G - 2 Z^2 + 3p < 6.2p
// so every product operand stays below 8p and every product below 1.2p;
// limbs stay below 2^28.
#pragma once
#include "curve.hpp"
#include "wide.hpp"

namespace msm {

// LDS of one unit with `WAVES` waves (the first two compute; more waves may
// prepare operands)
template <int WAVES>
struct wunit_lds {
  uint32_t mul[WAVES][WMUL2_WORDS];
  uint32_t acc[64];      // X, Y, T, Z of the accumulator
  uint32_t prod[2][64];  // phase-1 products, alternating between operations
  uint32_t opd[2][64];  // second operands X, Y, U = kT, Z (two slots)
  uint32_t c2p[16], c3p[16];
};

// this lane's place in the unit: product k = 2 wave + half, limb j
struct wslot {
  uint32_t k, j;
  bool act;  // operand limb lanes (the lower 16 of each half; the upper 16
             // carry zero operands and receive the product's limbs)
};

__device__ __forceinline__ wslot wslot_here() {
  const uint32_t lane = wlane();
  wslot s;
  s.k = ((threadIdx.x >> 6) << 1) | (lane >> 5);
  s.j = lane & 15u;
  s.act = (lane & 31u) < 16u;
  return s;
}

// all waves of the block: LDS writes done, then meet (outstanding global
// loads are not waited for)
__device__ __forceinline__ void unit_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// constants and scratch padding; the accumulator set to the identity
// (0, 1, 0, 1).  Needs a unit_sync before use.
template <int WAVES>
__device__ __forceinline__ void wunit_init(wunit_lds<WAVES>& s) {
  const uint32_t t = threadIdx.x;
  wmul2_init(s.mul[t >> 6]);
  if (t < 16) {
    const uint32_t up = t < 15 ? (1u << 26) : 0u, down = t >= 1 ? 4u : 0u;
    s.c2p[t] = 2u * kP24[t] + up - down;
    s.c3p[t] = 3u * kP24[t] + up - down;
  }
  if (t < 64) {
    const uint32_t coord = t >> 4;
    s.acc[t] = (coord == 1 || coord == 3) ? limb_of_const(kOne, t & 15u) : 0u;
  }
}

// phase 2 shared by addition and doubling: (E F, G H, E H, F G) -> acc
template <int WAVES>
__device__ __forceinline__ void wu_products_out(wunit_lds<WAVES>& s, const wslot& q, uint32_t E,
                                                uint32_t F, uint32_t G, uint32_t H) {
  uint32_t l = (q.k == 0 || q.k == 2) ? E : (q.k == 1 ? G : F);
  uint32_t r = q.k == 0 ? F : (q.k == 3 ? G : H);
  l = q.act ? l : 0u;
  r = q.act ? r : 0u;
  const uint32_t v = wmul2_hi(l, r, s.mul[threadIdx.x >> 6]);
  if (!q.act) s.acc[16 * q.k + q.j] = v;  // result limb j sits in lane 16 + j
}

// Both operations below take two phases and meet the other computing wave
// once, in a unit_sync between the phases (other waves of the block must
// meet it too).  The first phase of either operation reads only coordinates
// its own wave wrote (wave 0: X, Y; wave 1: T, Z; the doubling forms
// 2XY as 2TZ) and writes the product buffer par, which alternates between
// operations: so no sync is needed after the second phase, while the other
// wave may still be reading the previous buffer.  A cross-wave read of the
// accumulator after the last operation needs a block barrier.

// acc + opd (X2, Y2, U2 = k T2, Z2; coordinates below 2p; each wave reads
// only its own coordinates of opd).
template <int WAVES>
__device__ __forceinline__ void wu_add_u(wunit_lds<WAVES>& s, const uint32_t* opd, const wslot& q,
                                         uint32_t& par) {
  uint32_t* prod = s.prod[par];
  par ^= 1u;
  {
    const uint32_t x1 = s.acc[q.j], y1 = s.acc[16 + q.j], o1 = s.acc[16 * q.k + q.j];
    const uint32_t x2 = opd[q.j], y2 = opd[16 + q.j], o2 = opd[16 * q.k + q.j];
    const uint32_t c = s.c3p[q.j];
    uint32_t l = q.k == 0 ? (y1 + c) - x1 : (q.k == 1 ? y1 + x1 : o1);
    uint32_t r = q.k == 0 ? (y2 + c) - x2 : (q.k == 1 ? y2 + x2 : o2);
    l = q.act ? l : 0u;
    r = q.act ? r : 0u;
    uint32_t v = wmul2_hi(l, r, s.mul[threadIdx.x >> 6]);  // A, B, C = T1 U2, Z1 Z2
    if (q.k == 3) v <<= 1;                                // D = 2 Z1 Z2
    if (!q.act) prod[16 * q.k + q.j] = v;
  }
  unit_sync();
  {
    const uint32_t A = prod[q.j], B = prod[16 + q.j], C = prod[32 + q.j], D = prod[48 + q.j],
                   c = s.c3p[q.j];
    wu_products_out(s, q, (B + c) - A, (D + c) - C, D + C, B + A);
  }
  wave_lds_sync();
}

// 2 acc by the dedicated doubling (a = -1), with E = 2XY taken as 2TZ:
// A = X^2, B = Y^2, T Z, 2 Z^2 in the first phase.
template <int WAVES>
__device__ __forceinline__ void wu_dbl(wunit_lds<WAVES>& s, const wslot& q, uint32_t& par) {
  uint32_t* prod = s.prod[par];
  par ^= 1u;
  {
    const uint32_t o = s.acc[16 * q.k + q.j];            // X, Y, T, Z
    const uint32_t r = q.k == 2 ? s.acc[48 + q.j] : o;   // X, Y, Z, Z
    const uint32_t v0 = wmul2_hi(q.act ? o : 0u, q.act ? r : 0u, s.mul[threadIdx.x >> 6]);
    const uint32_t v = q.k == 3 ? v0 << 1 : v0;          // 2 Z^2
    if (!q.act) prod[16 * q.k + q.j] = v;
  }
  unit_sync();
  {
    const uint32_t A = prod[q.j], B = prod[16 + q.j], TZ = prod[32 + q.j], Z2 = prod[48 + q.j];
    const uint32_t c2 = s.c2p[q.j], c3 = s.c3p[q.j], AB = A + B;
    const uint32_t G = (B + c2) - A;
    wu_products_out(s, q, TZ + TZ, (G + c3) - Z2, G, c3 - AB);
  }
  wave_lds_sync();
}

// the words of this lane's limb of coordinate `coord` of an AoS record (12
// words per coordinate)
__device__ __forceinline__ limb_src wu_fetch(const uint32_t* __restrict__ rec, uint32_t coord,
                                             uint32_t j) {
  return limb_fetch(rec + coord * NL, j);
}

// store the accumulator as one AoS XYTZ record (lanes 0..3 of the calling
// wave, one coordinate each; values stay lazily reduced, below 1.2p)
template <int WAVES>
__device__ __forceinline__ void wu_store_acc(const wunit_lds<WAVES>& s, uint32_t* __restrict__ rec) {
  const uint32_t lane = wlane();
  if (lane < 4) st_aos(rec, (int)lane, words_of_limbs(s.acc + 16 * lane));
}

}  // namespace msm
