// Device-side building blocks shared by the partial-transform, PIE and loss
// kernels: MFMA wrappers, the per-lane operand chunk, wave reductions.
//
// MFMA tile used throughout (v_mfma_f32_16x16x4_f32, wave64):
//   A operand: lane l supplies A[row = l % 16][k = l / 16]
//   B operand: lane l supplies B[k = l / 16][col = l % 16]
//   D result : lane l holds   D[row = 4 * (l / 16) + i][col = l % 16], i = 0..3
// The contraction index k of one instruction may be any bijection onto the
// four lane groups, provided A and B use the same one.  The kernels use
//   k = 16 * block + 4 * (l / 16) + s,   s = 0..3 (one instruction per s),
// so each lane streams 4 consecutive complex values (32 bytes) of a row, and
// the D layout of one product (rows 4*(l/16) + i) is directly the B operand
// of the next product contracting over those rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pftpie {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// Four consecutive complex values held by one lane.
struct c4 {
  float2 v[4];
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // conj(a) * b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Load one 2 KB twiddle block of the swizzled table: lane l receives the
// four complex entries of its (row, k) chunk.  Block layout: two 1 KB
// planes of float4, plane p holding entries s = 2p, 2p+1 of every lane.
__device__ __forceinline__ c4 load_tw(const float4* __restrict__ blk, int lane) {
  float4 a = blk[lane];
  float4 b = blk[64 + lane];
  c4 r;
  r.v[0] = make_float2(a.x, a.y);
  r.v[1] = make_float2(a.z, a.w);
  r.v[2] = make_float2(b.x, b.y);
  r.v[3] = make_float2(b.z, b.w);
  return r;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

}  // namespace pftpie
