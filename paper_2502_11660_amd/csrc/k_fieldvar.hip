// Chained field products for comparing field-multiplication cores: each lane
// loads a_i and b_i and multiplies x = a_i by b_i `rounds` times, one product
// waiting for the previous (so a launch of many lanes measures multiplication
// throughput and the value pins every product).
#include "common.hpp"
#include "fe28.hpp"
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

// the carry-free 28-bit core (R' = 2^392): out = a b^rounds 2^(-392 rounds)
__global__ void __launch_bounds__(256) k_fe_mul_chain_f28(const uint32_t* __restrict__ a,
                                                          const uint32_t* __restrict__ b,
                                                          uint32_t* __restrict__ out,
                                                          uint32_t count, uint32_t rounds) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  fe28 x = f28_from_words(ld_soa(a, count, 0, i));
  const fe28 y = f28_from_words(ld_soa(b, count, 0, i));
  for (uint32_t r = 0; r < rounds; ++r) x = f28_mul(x, y);
  st_soa(out, count, 0, i, fe_canon(f28_to_words(x)));
}

// two elements per wave (one per 32-lane half): the same chain with the
// lane-parallel product
__global__ void __launch_bounds__(64) k_fe_mul_chain_wide(const uint32_t* __restrict__ a,
                                                          const uint32_t* __restrict__ b,
                                                          uint32_t* __restrict__ out,
                                                          uint32_t count, uint32_t rounds) {
  __shared__ uint32_t scratch[WMUL2_WORDS];
  __shared__ uint32_t res[32];
  wmul2_init(scratch);
  const uint32_t lane = wlane(), h = lane >> 5, jj = lane & 31;
  const uint32_t e = 2 * blockIdx.x + h;
  const bool act = jj < 16 && e < count;
  uint32_t x = 0, y = 0;
  if (act) {
    // limb jj of the SoA element e: bits 24 jj .. 24 jj + 23
    const uint32_t bit = 24u * jj, wi = bit >> 5, sh = bit & 31u;
    const uint32_t hi = sh > 8u;
    const uint64_t wa = ((uint64_t)(hi ? a[(size_t)(wi + 1) * count + e] : 0u) << 32) |
                        a[(size_t)wi * count + e];
    const uint64_t wb = ((uint64_t)(hi ? b[(size_t)(wi + 1) * count + e] : 0u) << 32) |
                        b[(size_t)wi * count + e];
    x = (uint32_t)(wa >> sh) & kLimbMask;
    y = (uint32_t)(wb >> sh) & kLimbMask;
  }
  for (uint32_t r = 0; r < rounds; ++r) x = wmul2(x, y, scratch);
  if (jj < 16) res[16 * h + jj] = x;
  wave_lds_sync();
  if (jj == 0 && e < count) st_soa(out, count, 0, e, fe_canon(words_of_limbs(res + 16 * h)));
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
    case MSM_MUL_F28:
      k_fe_mul_chain_f28<<<grid, 256, 0, st>>>(a, b, out, (uint32_t)count, (uint32_t)rounds);
      break;
    case MSM_MUL_WIDE:
      k_fe_mul_chain_wide<<<(unsigned)((count + 1) / 2), 64, 0, st>>>(a, b, out, (uint32_t)count,
                                                                       (uint32_t)rounds);
      break;
    default:
      return MSM_EINVAL;
  }
  HIPCHK(hipGetLastError());
  return MSM_OK;
}
