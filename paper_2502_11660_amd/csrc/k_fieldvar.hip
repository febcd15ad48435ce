// Chained field products for comparing field-multiplication cores: each lane
// loads a_i and b_i and multiplies x = a_i by b_i `rounds` times, one product
// waiting for the previous (so a launch of many lanes measures multiplication
// throughput and the value pins every product).
#include "common.hpp"
#include "field_variants.hpp"
#include "wide.hpp"

namespace msm {
namespace {

template <int V>
__device__ __forceinline__ fe mul_variant(const fe& x, const fe& y) {
  if constexpr (V == MSM_MUL_MONT) return fe_mul(x, y);
  if constexpr (V == MSM_MUL_BARRETT) return fe_mul_barrett(x, y);
  if constexpr (V == MSM_MUL_KARATSUBA) return fe_mul_karatsuba(x, y);
}

template <int V>
__global__ void __launch_bounds__(256) k_fe_mul_chain(const uint32_t* __restrict__ a,
                                                      const uint32_t* __restrict__ b,
                                                      uint32_t* __restrict__ out, uint32_t count,
                                                      uint32_t rounds) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  fe x = ld_soa(a, count, 0, i);
  const fe y = ld_soa(b, count, 0, i);
  for (uint32_t r = 0; r < rounds; ++r) x = mul_variant<V>(x, y);
  st_soa(out, count, 0, i, fe_canon(x));
}

// one wave per element: the same chain with the lane-parallel product
__global__ void __launch_bounds__(64) k_fe_mul_chain_wide(const uint32_t* __restrict__ a,
                                                          const uint32_t* __restrict__ b,
                                                          uint32_t* __restrict__ out,
                                                          uint32_t count, uint32_t rounds) {
  const uint32_t e = blockIdx.x;
  wfe x = wfe_from_words(ld_soa(a, count, 0, e));
  const wfe y = wfe_from_words(ld_soa(b, count, 0, e));
  for (uint32_t r = 0; r < rounds; ++r) x = wfe_mul(x, y);
  const fe w = fe_canon(wfe_to_words(x));
  if (threadIdx.x == 0) st_soa(out, count, 0, e, w);
}

}  // namespace
}  // namespace msm

using namespace msm;

extern "C" int msm_fe_mul_chain(const uint32_t* a, const uint32_t* b, uint32_t* out, size_t count,
                                int variant, int rounds, void* stream) {
  if (!a || !b || !out || count == 0 || count >= (1u << 31) || rounds < 1) return MSM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const unsigned grid = grid_for(count, 256);
  switch (variant) {
    case MSM_MUL_MONT:
      k_fe_mul_chain<MSM_MUL_MONT><<<grid, 256, 0, st>>>(a, b, out, (uint32_t)count, (uint32_t)rounds);
      break;
    case MSM_MUL_BARRETT:
      k_fe_mul_chain<MSM_MUL_BARRETT><<<grid, 256, 0, st>>>(a, b, out, (uint32_t)count,
                                                            (uint32_t)rounds);
      break;
    case MSM_MUL_KARATSUBA:
      k_fe_mul_chain<MSM_MUL_KARATSUBA><<<grid, 256, 0, st>>>(a, b, out, (uint32_t)count,
                                                              (uint32_t)rounds);
      break;
    case MSM_MUL_WIDE:
      k_fe_mul_chain_wide<<<(unsigned)count, 64, 0, st>>>(a, b, out, (uint32_t)count,
                                                           (uint32_t)rounds);
      break;
    default:
      return MSM_EINVAL;
  }
  HIPCHK(hipGetLastError());
  return MSM_OK;
}
