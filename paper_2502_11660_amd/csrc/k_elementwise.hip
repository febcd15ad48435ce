// Elementwise kernels: batched field multiply, batched PADD (the paper's
// "task", Sec. II-D / V-A), point preparation and the synthetic point
// generator.
#include <algorithm>

#include "common.hpp"
#include "convert.hpp"
#include "curve28.hpp"

namespace msm {
namespace {

__global__ void __launch_bounds__(256) k_fe_mul(const uint32_t* __restrict__ a,
                                                const uint32_t* __restrict__ b,
                                                uint32_t* __restrict__ out, uint32_t count,
                                                int canonical) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  fe r = fe_mul(ld_soa(a, count, 0, i), ld_soa(b, count, 0, i));
  if (canonical) r = fe_canon(r);
  st_soa(out, count, 0, i, r);
}

// SoA rows through buffer instructions: row r of an array (word r count + i
// of element i) is a wave-uniform base, so its buffer descriptor lives in
// scalar registers and every load or store takes the one per-lane byte
// offset 4 i, with no per-access address arithmetic on the vector unit.
// Requires count < 2^29 (4 count fits a descriptor's 32-bit byte range).
constexpr uint32_t kBufferFlags = 0x00020000u;  // raw 32-bit buffer access

__device__ __forceinline__ fe ld_rows(const uint32_t* __restrict__ base, uint32_t count, int coord,
                                      uint32_t voff) {
  fe r;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    const uint32_t* row = base + (size_t)(coord * NL + l) * count;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)row, 0, (int)(count * 4u), kBufferFlags);
    r.v[l] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff, 0, 0);
  }
  return r;
}

__device__ __forceinline__ void st_rows(uint32_t* __restrict__ base, uint32_t count, int coord,
                                        uint32_t voff, const fe& x) {
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    uint32_t* row = base + (size_t)(coord * NL + l) * count;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)row, 0, (int)(count * 4u), kBufferFlags);
    __builtin_amdgcn_raw_buffer_store_b32(x.v[l], rs, voff, 0, 0);
  }
}

// canonical form of a product output (< 2p): one conditional subtraction
__device__ __forceinline__ fe canon_of_product(const fe28& x) {
  const fe w = f28_to_words(x);
  uint64_t br;
  const fe t = fe_sub_mask(w, fe_const(kP), br);
  return fe_pick(br, w, t);
}

// out_i = a_i + b_i, SoA limb-major operands; FORM selects the mixed
// (b prepared: X, Y, U, Z = 1) or the complete (b extended) addition.  On the
// carry-free 28-bit field form (curve28.hpp); outputs canonical.
template <int FORM>
__global__ void __launch_bounds__(256) k_padd(const uint32_t* __restrict__ a,
                                              const uint32_t* __restrict__ b,
                                              uint32_t* __restrict__ out, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t vo = 4u * i;
  xytz28 pa;
  pa.X = f28_from_words(ld_rows(a, count, 0, vo));
  pa.Y = f28_from_words(ld_rows(a, count, 1, vo));
  pa.T = f28_from_words(ld_rows(a, count, 2, vo));
  pa.Z = f28_from_words(ld_rows(a, count, 3, vo));
  xytz28 r;
  if (FORM == MSM_FORM_XYU) {
    xyu28 pb;
    pb.X = f28_from_words(ld_rows(b, count, 0, vo));
    pb.Y = f28_from_words(ld_rows(b, count, 1, vo));
    pb.U = f28_from_words(ld_rows(b, count, 2, vo));
    r = padd28_mixed(pa, pb);
  } else {
    xytz28 pb;
    pb.X = f28_from_words(ld_rows(b, count, 0, vo));
    pb.Y = f28_from_words(ld_rows(b, count, 1, vo));
    pb.T = f28_from_words(ld_rows(b, count, 2, vo));
    pb.Z = f28_from_words(ld_rows(b, count, 3, vo));
    r = padd28_full(pa, pb);
  }
  st_rows(out, count, 0, vo, canon_of_product(r.X));
  st_rows(out, count, 1, vo, canon_of_product(r.Y));
  st_rows(out, count, 2, vo, canon_of_product(r.T));
  st_rows(out, count, 3, vo, canon_of_product(r.Z));
}

// Weierstrass affine (ordinary form) -> prepared (X, Y, U = k x y), Z = 1
// (Sec. II-D: inputs enter as (X, Y, U, Z = 1)):
//   w = x + 1,  x_e = (beta/alpha) w / y,  y_e = (w - alpha) / (w + alpha)
// so each point needs the inverse of its denominator y (w + alpha).  The
// inverses come from one inversion per wave (Montgomery's trick, on two
// levels).  Each lane walks its points forward multiplying their
// denominators into a running product (each point's record slot keeps the
// product before it); the wave then forms prefix and suffix products of the
// 64 lane products (six shuffle-and-multiply steps each), inverts the wave's
// total once with all lanes cooperating (fe_inv_lanes), and gives each lane
// the inverse of its own product as total^-1 x prefix x suffix.  Walking
// back, the inverse of point j's denominator is (inverse of the product up to
// j) times (product before j), and multiplying by denominator j steps the
// inverse back.  With the image phi(P) = (omega x, y) the two denominators
// y (w + alpha) and y (omega x + 1 + alpha) of a point are multiplied first,
// so one entry serves both.  A zero denominator (an exceptional point,
// flagged; it cannot lie in the prime-order subgroup) enters the product as
// 1 so that it does not spoil the batch; its own record is then
// unspecified.

// Preparation runs once per point set, off the MSM's path; its products are
// the out-of-line multiply (fe_mul_cold), which keeps the kernel's register
// footprint small enough for several waves per SIMD.

// lane-to-lane moves of a field element (lanes without a source keep x)
__device__ __forceinline__ fe fe_shfl_up(const fe& x, int d) {
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.v[i] = (uint32_t)__shfl_up((int)x.v[i], d, 64);
  return r;
}

__device__ __forceinline__ fe fe_shfl_down(const fe& x, int d) {
  fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.v[i] = (uint32_t)__shfl_down((int)x.v[i], d, 64);
  return r;
}

// Every lane's v^-1 (Montgomery form, canonical) for non-zero v < 2p, with
// one inversion for the wave.  All 64 lanes of the wave must take part.
__device__ __forceinline__ fe wave_batch_inverse(const fe& v) {
  const int lane = (int)__lane_id();
  fe P = v, Q = v;  // inclusive prefix and suffix products over the lanes
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const fe pu = fe_mul_cold(P, fe_shfl_up(P, d));
    const fe qd = fe_mul_cold(Q, fe_shfl_down(Q, d));
    P = fe_select(lane >= d, pu, P);
    Q = fe_select(lane + d < 64, qd, Q);
  }
  const fe E = fe_select(lane == 0, fe_const(kOne), fe_shfl_up(P, 1));    // lanes below
  const fe S = fe_select(lane == 63, fe_const(kOne), fe_shfl_down(Q, 1)); // lanes above
  fe total;
#pragma unroll
  for (int i = 0; i < NL; ++i) total.v[i] = (uint32_t)__builtin_amdgcn_readlane((int)P.v[i], 63);
  const fe inv_total = fe_mul_cold(fe_inv_lanes(fe_canon(total)), fe_const(kR3));
  return fe_mul_cold(fe_mul_cold(inv_total, E), S);
}

// the denominator y (x + 1 + alpha)
__device__ __forceinline__ fe prep_den(const fe& x, const fe& y) {
  return fe_mul_cold(y, fe_add(fe_add(x, fe_const(kOne)), fe_const(kAlpha)));
}

// the record (x_e, y_e, k x_e y_e), canonical, given the inverse of the
// denominator
__device__ __forceinline__ void prep_record(const fe& x, const fe& y, const fe& inv,
                                            uint32_t* rec) {
  const fe p2 = fe_const(kP2);
  const fe w = fe_add(x, fe_const(kOne));                 // < 4p
  const fe wpa = fe_add(w, fe_const(kAlpha));             // < 6p
  const fe wma = fe_sub_plus(w, fe_const(kAlpha), p2);    // < 6p
  const fe xe = fe_mul_cold(fe_mul_cold(fe_mul_cold(w, wpa), inv), fe_const(kBetaOverAlpha));
  const fe ye = fe_mul_cold(fe_mul_cold(wma, y), inv);
  const fe u = fe_mul_cold(fe_mul_cold(xe, ye), fe_const(kK));
  st_aos(rec, 0, fe_canon(xe));
  st_aos(rec, 1, fe_canon(ye));
  st_aos(rec, 2, fe_canon(u));
}

__device__ __forceinline__ void prepare_identity(uint32_t* rec) {
  st_aos(rec, 0, fe_zero());
  st_aos(rec, 1, fe_const(kOne));
  st_aos(rec, 2, fe_zero());
}

// the point's factor of the batch product (1 for a zero denominator)
__device__ __forceinline__ fe batch_factor(const fe& den_a, const fe& den_b, bool endo,
                                           uint32_t& flags) {
  fe d = endo ? fe_mul_cold(den_a, den_b) : den_a;
  if (fe_is_zero_canon(fe_canon(d))) {
    flags |= MSM_FLAG_EXCEPT;
    d = fe_const(kOne);
  }
  return d;
}

// Thread t prepares points i = t + j T, j = 0 .. m-1 (i < n), T = threads;
// threads t >= T take part in the wave-wide inversion only.
// ENDO: records 2i and 2i + 1 hold point i and its image (omega x, y).
template <bool ENDO>
__global__ void __launch_bounds__(256) k_prepare(const uint32_t* __restrict__ xy,
                                                 const uint32_t* __restrict__ inf,
                                                 uint32_t* __restrict__ out, uint32_t n,
                                                 uint32_t T, uint32_t m,
                                                 uint32_t* __restrict__ status) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t mine = t < T ? m : 0u;
  uint32_t flags = 0;
  fe c = fe_const(kOne);  // product of the factors so far
  uint32_t last = 0;      // points of this thread
  for (uint32_t j = 0; j < mine; ++j) {
    const uint64_t i = (uint64_t)t + (uint64_t)j * T;
    if (i >= n) break;
    last = j + 1;
    if (inf && inf[i]) continue;
    const fe x = fe_mul_cold(ld_soa(xy, n, 0, (size_t)i), fe_const(kR2));
    const fe y = fe_mul_cold(ld_soa(xy, n, 1, (size_t)i), fe_const(kR2));
    const fe lhs = fe_canon(fe_mul_cold(y, y));
    const fe rhs = fe_canon(fe_add(fe_mul_cold(fe_mul_cold(x, x), x), fe_const(kOne)));
    if (!fe_eq_canon(lhs, rhs)) flags |= MSM_FLAG_OFFCURVE;
    const fe den_a = prep_den(x, y);
    const fe den_b = ENDO ? prep_den(fe_mul_cold(x, fe_const(kOmega)), y) : den_a;
    st_aos(out + (size_t)(ENDO ? 2 * i : i) * XYU_WORDS, 0, fe_canon(c));  // product before i
    c = fe_mul_cold(c, batch_factor(den_a, den_b, ENDO, flags));
  }
  fe tinv = wave_batch_inverse(c);  // inverse of this thread's product
  for (uint32_t jj = last; jj-- > 0;) {
    const uint64_t i = (uint64_t)t + (uint64_t)jj * T;
    uint32_t* rec = out + (size_t)(ENDO ? 2 * i : i) * XYU_WORDS;
    if (inf && inf[i]) {
      prepare_identity(rec);
      if (ENDO) prepare_identity(rec + XYU_WORDS);
      continue;
    }
    const fe x = fe_mul_cold(ld_soa(xy, n, 0, (size_t)i), fe_const(kR2));
    const fe y = fe_mul_cold(ld_soa(xy, n, 1, (size_t)i), fe_const(kR2));
    const fe den_a = prep_den(x, y);
    const fe xb = ENDO ? fe_mul_cold(x, fe_const(kOmega)) : x;
    const fe den_b = ENDO ? prep_den(xb, y) : den_a;
    uint32_t dummy = 0;
    const fe d = batch_factor(den_a, den_b, ENDO, dummy);
    const fe inv_d = fe_mul_cold(tinv, ld_aos(rec, 0));  // 1 / d
    tinv = fe_mul_cold(tinv, d);                          // 1 / (product before this point)
    if (ENDO) {
      prep_record(x, y, fe_mul_cold(inv_d, den_b), rec);
      prep_record(xb, y, fe_mul_cold(inv_d, den_a), rec + XYU_WORDS);
    } else {
      prep_record(x, y, inv_d, rec);
    }
  }
  if (flags) atomicOr(status, flags);
}

// P_i = k_i G: most-significant-bit-first double-and-add in twisted-Edwards
// coordinates, then mapped to Weierstrass affine.
__global__ void __launch_bounds__(256) k_gen_points(const uint32_t* __restrict__ kk,
                                                    uint32_t* __restrict__ xy,
                                                    uint32_t* __restrict__ inf, uint32_t n) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const fe p2 = fe_const(kP2);
  xyu g;
  g.X = fe_const(kGteX);
  g.Y = fe_const(kGteY);
  g.U = fe_const(kGteU);
  uint32_t kw[SCALAR_WORDS];
#pragma unroll
  for (int j = 0; j < SCALAR_WORDS; ++j) kw[j] = kk[(size_t)i * SCALAR_WORDS + j];
  xytz acc = pt_identity();
  for (int j = SCALAR_WORDS - 1; j >= 0; --j) {
    uint32_t word = kw[j];
    for (int bit = 31; bit >= 0; --bit) {
      acc = pdbl(acc, p2);
      if ((word >> bit) & 1u) acc = padd_mixed(acc, g, p2);
    }
  }
  fe xw, yw;
  bool fin = te_to_weierstrass(acc, xw, yw);
  st_soa(xy, n, 0, i, xw);
  st_soa(xy, n, 1, i, yw);
  inf[i] = fin ? 0u : 1u;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

}  // namespace

int launch_fe_mul(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t count,
                  int canonical, hipStream_t st) {
  k_fe_mul<<<grid_for(count, 256), 256, 0, st>>>(a, b, out, count, canonical);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int launch_padd(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t count, int form,
                hipStream_t st) {
  if (form == MSM_FORM_XYU)
    k_padd<MSM_FORM_XYU><<<grid_for(count, 256), 256, 0, st>>>(a, b, out, count);
  else
    k_padd<MSM_FORM_XYTZ><<<grid_for(count, 256), 256, 0, st>>>(a, b, out, count);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int launch_prepare(const uint32_t* xy, const uint32_t* inf, uint32_t* xyu, uint32_t n,
                   uint32_t* status, bool endo, hipStream_t st) {
  // points per thread: enough threads for four waves per SIMD
  // (256 CUs x 4 SIMDs x 64 lanes x 4), the rest of the points batched
  const uint32_t m = std::max<uint32_t>(1u, std::min<uint32_t>(64u, n / 262144u));
  const uint32_t T = (uint32_t)(((uint64_t)n + m - 1) / m);
  if (endo)
    k_prepare<true><<<grid_for(T, 256), 256, 0, st>>>(xy, inf, xyu, n, T, m, status);
  else
    k_prepare<false><<<grid_for(T, 256), 256, 0, st>>>(xy, inf, xyu, n, T, m, status);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int launch_gen_points(const uint32_t* k, uint32_t* xy, uint32_t* inf, uint32_t n, hipStream_t st) {
  k_gen_points<<<grid_for(n, 256), 256, 0, st>>>(k, xy, inf, n);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

int launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st) {
  unsigned g = grid_for(n, 256);
  if (g > 4096u) g = 4096u;
  if (g == 0) g = 1;
  k_fill_u32<<<g, 256, 0, st>>>(p, n, v);
  HIPCHK(hipGetLastError());
  return MSM_OK;
}

}  // namespace msm
