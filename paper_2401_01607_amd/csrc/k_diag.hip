// Diagnostics: the FP32 fused-multiply-add issue rate the gather kernels can
// reach on this device.  The published FP32 vector peak counts packed FP32
// instructions (two FMAs per lane per instruction); the library is built
// without them (-packed-fp32-ops), so its kernels issue one v_fmac_f32 per
// FMA and lane.  This kernel runs independent v_fmac_f32 chains with no
// memory traffic and reports the rate reached, the practical ceiling of the
// gather path.
#include "taches_internal.h"

namespace taches {
namespace {

constexpr int kChains = 32;
constexpr int kUnroll = 8;

__global__ __launch_bounds__(256) void k_fmac_ceiling(float* out, const float* in, int iters) {
  float acc[kChains], x[kChains];
  const float y = in[threadIdx.x & 255];
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    acc[i] = 0.f;
    x[i] = in[(threadIdx.x + i) & 255];
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int i = 0; i < kChains; ++i) acc[i] = __builtin_fmaf(x[i], y, acc[i]);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kChains; ++i) s += acc[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

hipError_t measure_fmac_ceiling(int device, double* tflops) {
  constexpr int blocks = 16384, iters = 400;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return e;
  float *in = nullptr, *out = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.f;
  e = hipMalloc(&in, 256 * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&out, (size_t)blocks * 256 * sizeof(float));
  if (e == hipSuccess) e = hipMemset(in, 0, 256 * sizeof(float));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fmac_ceiling, dim3(blocks), dim3(256), 0, st, out, in, 16);   // warm-up
    e = hipEventRecord(e0, st);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_fmac_ceiling, dim3(blocks), dim3(256), 0, st, out, in, iters);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  }
  if (e == hipSuccess) {
    const double flops = 2.0 * kChains * kUnroll * (double)iters * 256.0 * blocks;
    *tflops = ms > 0.f ? flops / (ms * 1e-3) / 1e12 : 0.0;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  (void)hipFree(in);
  (void)hipFree(out);
  return e;
}

}  // namespace taches
