// Microbenchmarks that give the rooflines their denominators: the VALU issue
// rate of the 32x32->64 multiply-add the field core is built on (and of the
// carry add that accompanies it), and a plain HBM copy used both as the
// bandwidth reference and to calibrate memory-traffic counters; and the
// issue rate of a lone wave, which sets the latency of dependent chains.
#include "common.hpp"

namespace msm {
namespace {

constexpr int MB_BLOCKS = 256 * 8;  // 8 workgroups per CU
constexpr int MB_THREADS = 256;     // 4 waves each: 8 waves per SIMD

// 8 independent v_mad_u64_u32 chains per lane, 16 instructions per iteration
__global__ void __launch_bounds__(MB_THREADS) k_mb_mad64(uint64_t* __restrict__ out, uint32_t iters) {
  uint32_t a = 0x9e3779b9u + threadIdx.x, b = 0x7f4a7c15u ^ blockIdx.x;
  uint64_t c0 = 1, c1 = 2, c2 = 3, c3 = 4, c4 = 5, c5 = 6, c6 = 7, c7 = 8;
  for (uint32_t it = 0; it < iters; ++it) {
#define MB_MAD(c) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(c) : "v"(a), "v"(b) : "vcc");
    MB_MAD(c0) MB_MAD(c1) MB_MAD(c2) MB_MAD(c3) MB_MAD(c4) MB_MAD(c5) MB_MAD(c6) MB_MAD(c7)
    MB_MAD(c0) MB_MAD(c1) MB_MAD(c2) MB_MAD(c3) MB_MAD(c4) MB_MAD(c5) MB_MAD(c6) MB_MAD(c7)
#undef MB_MAD
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = c0 ^ c1 ^ c2 ^ c3 ^ c4 ^ c5 ^ c6 ^ c7;
}

// 8 independent add-with-carry chains per lane, 16 instructions per iteration
__global__ void __launch_bounds__(MB_THREADS) k_mb_addc(uint64_t* __restrict__ out, uint32_t iters) {
  uint32_t a = 0x9e3779b9u + threadIdx.x;
  uint32_t c0 = 1, c1 = 2, c2 = 3, c3 = 4, c4 = 5, c5 = 6, c6 = 7, c7 = 8;
  for (uint32_t it = 0; it < iters; ++it) {
#define MB_ADDC(c) asm volatile("v_addc_co_u32_e32 %0, vcc, %0, %1, vcc" : "+v"(c) : "v"(a) : "vcc");
    MB_ADDC(c0) MB_ADDC(c1) MB_ADDC(c2) MB_ADDC(c3) MB_ADDC(c4) MB_ADDC(c5) MB_ADDC(c6) MB_ADDC(c7)
    MB_ADDC(c0) MB_ADDC(c1) MB_ADDC(c2) MB_ADDC(c3) MB_ADDC(c4) MB_ADDC(c5) MB_ADDC(c6) MB_ADDC(c7)
#undef MB_ADDC
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = c0 ^ c1 ^ c2 ^ c3 ^ c4 ^ c5 ^ c6 ^ c7;
}

// one dependent v_mad_u64_u32 chain per lane, 16 instructions per iteration
__global__ void __launch_bounds__(64) k_mb_mad64_dep(uint64_t* __restrict__ out, uint32_t iters) {
  uint32_t a = 0x9e3779b9u + threadIdx.x, b = 0x7f4a7c15u;
  uint64_t c = 1;
  for (uint32_t it = 0; it < iters; ++it) {
#define MB_MAD(c) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(c) : "v"(a), "v"(b) : "vcc");
    MB_MAD(c) MB_MAD(c) MB_MAD(c) MB_MAD(c) MB_MAD(c) MB_MAD(c) MB_MAD(c) MB_MAD(c)
    MB_MAD(c) MB_MAD(c) MB_MAD(c) MB_MAD(c) MB_MAD(c) MB_MAD(c) MB_MAD(c) MB_MAD(c)
#undef MB_MAD
  }
  out[threadIdx.x] = c;
}

// a dependent chain of Montgomery products in one wave: x = x * y, iters times
__global__ void __launch_bounds__(64) k_mb_femul_dep(uint64_t* __restrict__ out, uint32_t iters) {
  fe x = fe_const(kR2), y = fe_const(kOne);
  x.v[0] ^= threadIdx.x;
  for (uint32_t it = 0; it < iters; ++it) x = fe_mul(x, y);
  uint64_t h = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) h = h * 31 + x.v[i];
  out[threadIdx.x] = h;
}

__global__ void __launch_bounds__(256) k_mb_copy(const uint4* __restrict__ in, uint4* __restrict__ out,
                                                 size_t n) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = in[i];
}

}  // namespace
}  // namespace msm

using namespace msm;

extern "C" int msm_microbench(int kind, size_t param, void* buf, size_t buf_bytes, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (!buf) return MSM_EINVAL;
  switch (kind) {
    case MSM_MB_MAD64:
    case MSM_MB_ADDC: {
      if (buf_bytes < (size_t)MB_BLOCKS * MB_THREADS * 8 || param == 0 || param >= (1u << 31))
        return MSM_EINVAL;
      if (kind == MSM_MB_MAD64)
        k_mb_mad64<<<MB_BLOCKS, MB_THREADS, 0, st>>>((uint64_t*)buf, (uint32_t)param);
      else
        k_mb_addc<<<MB_BLOCKS, MB_THREADS, 0, st>>>((uint64_t*)buf, (uint32_t)param);
      break;
    }
    case MSM_MB_MAD64_LONE:
    case MSM_MB_MAD64_DEP:
    case MSM_MB_FEMUL_DEP: {
      if (buf_bytes < 64 * 8 || param == 0 || param >= (1u << 31)) return MSM_EINVAL;
      if (kind == MSM_MB_MAD64_LONE)
        k_mb_mad64<<<1, 64, 0, st>>>((uint64_t*)buf, (uint32_t)param);
      else if (kind == MSM_MB_MAD64_DEP)
        k_mb_mad64_dep<<<1, 64, 0, st>>>((uint64_t*)buf, (uint32_t)param);
      else
        k_mb_femul_dep<<<1, 64, 0, st>>>((uint64_t*)buf, (uint32_t)param);
      break;
    }
    case MSM_MB_COPY: {
      // copy the first half of buf (param bytes) to the second half
      if (param == 0 || param % 16 != 0 || 2 * param > buf_bytes ||
          ((uintptr_t)buf % 16) != 0)
        return MSM_EINVAL;
      const uint4* in = (const uint4*)buf;
      uint4* out = (uint4*)((char*)buf + param);
      k_mb_copy<<<256 * 16, 256, 0, st>>>(in, out, param / 16);
      break;
    }
    default:
      return MSM_EINVAL;
  }
  HIPCHK(hipGetLastError());
  return MSM_OK;
}
