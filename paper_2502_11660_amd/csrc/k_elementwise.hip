// Elementwise kernels: batched field multiply, batched PADD (the paper's
// "task", Sec. II-D / V-A), point preparation and the synthetic point
// generator.
#include "common.hpp"
#include "convert.hpp"

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

// out_i = a_i + b_i, SoA limb-major operands; FORM selects the mixed
// (b prepared: X, Y, U, Z = 1) or the complete (b extended) addition.
template <int FORM>
__global__ void __launch_bounds__(256) k_padd(const uint32_t* __restrict__ a,
                                              const uint32_t* __restrict__ b,
                                              uint32_t* __restrict__ out, uint32_t count) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const fe p2 = fe_const(kP2);
  xytz pa;
  pa.X = ld_soa(a, count, 0, i);
  pa.Y = ld_soa(a, count, 1, i);
  pa.T = ld_soa(a, count, 2, i);
  pa.Z = ld_soa(a, count, 3, i);
  xytz r;
  if (FORM == MSM_FORM_XYU) {
    xyu pb;
    pb.X = ld_soa(b, count, 0, i);
    pb.Y = ld_soa(b, count, 1, i);
    pb.U = ld_soa(b, count, 2, i);
    r = padd_mixed(pa, pb, p2);
  } else {
    xytz pb;
    pb.X = ld_soa(b, count, 0, i);
    pb.Y = ld_soa(b, count, 1, i);
    pb.T = ld_soa(b, count, 2, i);
    pb.Z = ld_soa(b, count, 3, i);
    r = padd_full(pa, pb, p2);
  }
  st_soa(out, count, 0, i, fe_canon(r.X));
  st_soa(out, count, 1, i, fe_canon(r.Y));
  st_soa(out, count, 2, i, fe_canon(r.T));
  st_soa(out, count, 3, i, fe_canon(r.Z));
}

// Weierstrass affine (ordinary form) -> prepared (X, Y, U = k x y), Z = 1:
//   w = x + 1,  x_e = (beta/alpha) w / y,  y_e = (w - alpha) / (w + alpha)
// with one inversion of y (w + alpha) per point.
// prepared record (x_e, y_e, k x_e y_e) of the affine point (x, y), both in
// Montgomery form; flags for off-curve / map-exceptional inputs
__device__ __forceinline__ uint32_t prepare_one(const fe& x, const fe& y, uint32_t* rec) {
  const fe p2 = fe_const(kP2);
  uint32_t flags = 0;
  fe lhs = fe_canon(fe_sqr(y));
  fe rhs = fe_canon(fe_add(fe_mul(fe_sqr(x), x), fe_const(kOne)));
  if (!fe_eq_canon(lhs, rhs)) flags |= MSM_FLAG_OFFCURVE;
  fe w = fe_add(x, fe_const(kOne));               // < 4p
  fe wpa = fe_add(w, fe_const(kAlpha));           // < 6p
  fe wma = fe_sub_plus(w, fe_const(kAlpha), p2);  // < 6p
  fe den = fe_mul(y, wpa);
  if (fe_is_zero_canon(fe_canon(den))) flags |= MSM_FLAG_EXCEPT;
  fe inv = fe_inv_mont(den);
  fe xe = fe_mul(fe_mul(fe_mul(w, wpa), inv), fe_const(kBetaOverAlpha));
  fe ye = fe_mul(fe_mul(wma, y), inv);
  fe u = fe_mul(fe_mul(xe, ye), fe_const(kK));
  st_aos(rec, 0, fe_canon(xe));
  st_aos(rec, 1, fe_canon(ye));
  st_aos(rec, 2, fe_canon(u));
  return flags;
}

__device__ __forceinline__ void prepare_identity(uint32_t* rec) {
  st_aos(rec, 0, fe_zero());
  st_aos(rec, 1, fe_const(kOne));
  st_aos(rec, 2, fe_zero());
}

// ENDO: records 2i and 2i + 1 hold point i and its image (omega x, y)
template <bool ENDO>
__global__ void __launch_bounds__(256) k_prepare(const uint32_t* __restrict__ xy,
                                                 const uint32_t* __restrict__ inf,
                                                 uint32_t* __restrict__ out, uint32_t n,
                                                 uint32_t* __restrict__ status) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t* rec = out + (size_t)(ENDO ? 2 * i : i) * XYU_WORDS;
  uint32_t* rec2 = rec + XYU_WORDS;
  if (inf && inf[i]) {
    prepare_identity(rec);
    if (ENDO) prepare_identity(rec2);
    return;
  }
  const fe x = fe_to_mont(ld_soa(xy, n, 0, i));
  const fe y = fe_to_mont(ld_soa(xy, n, 1, i));
  uint32_t flags = prepare_one(x, y, rec);
  if (ENDO) flags |= prepare_one(fe_mul(x, fe_const(kOmega)), y, rec2);
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
  if (endo)
    k_prepare<true><<<grid_for(n, 256), 256, 0, st>>>(xy, inf, xyu, n, status);
  else
    k_prepare<false><<<grid_for(n, 256), 256, 0, st>>>(xy, inf, xyu, n, status);
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
