// Measured peaks of the device, for reporting roofline fractions against
// what the chip delivers beside its published figures: a matrix-core loop
// per input type (FP32, BF16, FP16 MFMA with FP32 accumulation) on random
// register operands.  Not part of the method: a measurement aid.
#include <cstdint>

#include "internal.hpp"
#include "device_common.hpp"

namespace pftpie {
namespace {

constexpr int kChains = 8;  // independent accumulators per wave (hide MFMA latency)

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ float rnd(uint32_t k) { return (float)(hash32(k) & 0xFFFFu) * (1.f / 32768.f) - 1.f; }

// kind 0: v_mfma_f32_16x16x4_f32 (2048 flops); 1: 16x16x32 bf16 (16384);
// 2: 16x16x32 f16 (16384).  Every wave runs `iters` rounds of kChains
// products and stores a sum of its accumulators (so none is dropped).
template <int KIND>
__global__ __launch_bounds__(256) void k_mfma_loop(int iters, float* out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  f32x4 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = zero4();
  if constexpr (KIND == 0) {
    const float a = rnd(3 * t), b = rnd(3 * t + 1);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    }
  } else {
    using PR = typename std::conditional<KIND == 1, PrecBF16, PrecF16>::type;
    typename PR::V a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = (typename PR::T)rnd(16 * t + e);
      b[e] = (typename PR::T)rnd(16 * t + 8 + e);
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = PR::mfma(a, b, acc[c]);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[t] = s;
}

template <int KIND>
hipError_t time_loop(int blocks, int iters, float* out, hipStream_t st, hipEvent_t e0, hipEvent_t e1, float* ms) {
  hipLaunchKernelGGL(k_mfma_loop<KIND>, dim3(blocks), dim3(256), 0, st, iters / 8, out);  // warm-up
  hipError_t e = hipEventRecord(e0, st);
  hipLaunchKernelGGL(k_mfma_loop<KIND>, dim3(blocks), dim3(256), 0, st, iters, out);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  return e;
}

}  // namespace
}  // namespace pftpie

using namespace pftpie;

extern "C" pftpie_status pftpie_measure_mfma_peaks(double* fp32_tflops, double* bf16_tflops, double* fp16_tflops) {
  if (!fp32_tflops || !bf16_tflops || !fp16_tflops)
    return fail(PFTPIE_E_INVALID, "measure_mfma_peaks: NULL output");
  int dev = 0, cus = 256;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "measure_mfma_peaks: hipGetDevice");
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  const int blocks = cus * 8;  // 8 waves per SIMD
  float* out = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipMalloc((void**)&out, sizeof(float) * (size_t)blocks * 256);
  if (e == hipSuccess) e = hipStreamCreate(&st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float ms[3] = {0.f, 0.f, 0.f};
  const int iters[3] = {4096, 2048, 2048};
  if (e == hipSuccess) e = time_loop<0>(blocks, iters[0], out, st, e0, e1, &ms[0]);
  if (e == hipSuccess) e = time_loop<1>(blocks, iters[1], out, st, e0, e1, &ms[1]);
  if (e == hipSuccess) e = time_loop<2>(blocks, iters[2], out, st, e0, e1, &ms[2]);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  (void)hipFree(out);
  if (e != hipSuccess) return hip_fail(e, "measure_mfma_peaks");
  const double waves = (double)blocks * 4;
  const double flops[3] = {2048.0, 16384.0, 16384.0};
  double* res[3] = {fp32_tflops, bf16_tflops, fp16_tflops};
  for (int k = 0; k < 3; ++k)
    *res[k] = waves * kChains * (double)iters[k] * flops[k] / ((double)ms[k] * 1e-3) / 1e12;
  return PFTPIE_OK;
}
