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

// Workgroup barrier that orders LDS accesses only: global loads still in
// flight (prefetches) are not waited for, unlike __syncthreads.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

namespace pftpie {

// ---------------------------------------------------------------------------
// Split 16-bit operands (v_mfma_f32_16x16x32_{bf16,f16}): a lane supplies 8
// 16-bit values per operand; lane group g = l / 16 holds K-slots
// 8g .. 8g+7 for A and B alike.  The kernels pack 4 complex values per lane
// group as (re, im) pairs in those slots, the same complex index mapping as
// the FP32 engine (k = 16 block + 4 g + s).

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// pk(a, b): RNE(a) in the low half, RNE(b) in the high half of one dword;
// lo / hi: the float value of the low / high half.
struct PrecBF16 {
  typedef __bf16 T;
  typedef bf16x8 V;
  static __device__ __forceinline__ uint32_t pk(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2v){a, b}, bf16x2));
  }
  static __device__ __forceinline__ float lo(uint32_t p) { return __builtin_bit_cast(float, p << 16); }
  static __device__ __forceinline__ float hi(uint32_t p) { return __builtin_bit_cast(float, p & 0xffff0000u); }
  static __device__ __forceinline__ f32x4 mfma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
struct PrecF16 {
  typedef _Float16 T;
  typedef f16x8 V;
  static __device__ __forceinline__ uint32_t pk(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2v){a, b}, f16x2));
  }
  static __device__ __forceinline__ float lo(uint32_t p) { return (float)__builtin_bit_cast(f16x2, p).x; }
  static __device__ __forceinline__ float hi(uint32_t p) { return (float)__builtin_bit_cast(f16x2, p).y; }
  static __device__ __forceinline__ f32x4 mfma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// hi = RNE(x), lo = RNE(x - hi) for 8 floats (x - hi is exact in float).
template <class PR>
__device__ __forceinline__ void split8(const float (&x)[8], typename PR::V& hi, typename PR::V& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const typename PR::T h = (typename PR::T)x[e];
    hi[e] = h;
    lo[e] = (typename PR::T)(x[e] - (float)h);
  }
}

// Split twiddle block: plane 0 (1 KB) = hi parts, plane 1 = lo parts, each
// 8 x 16-bit per lane: (re_s, im_s) for s = 0..3.
template <class PR>
struct TwS {
  typename PR::V h, l;
};
template <class PR>
__device__ __forceinline__ TwS<PR> load_tws(const void* __restrict__ blk, int lane) {
  const typename PR::V* p = reinterpret_cast<const typename PR::V*>(blk);
  TwS<PR> r;
  r.h = p[lane];
  r.l = p[64 + lane];
  return r;
}

// acc += a * b with split operands: hi*hi + hi*lo + lo*hi
template <class PR>
__device__ __forceinline__ f32x4 mfma3(const typename PR::V& ah, const typename PR::V& al, const TwS<PR>& b,
                                       f32x4 c) {
  c = PR::mfma(ah, b.h, c);
  c = PR::mfma(ah, b.l, c);
  c = PR::mfma(al, b.h, c);
  return c;
}

}  // namespace pftpie

namespace pftpie {

// ---------------------------------------------------------------------------
// Twiddle-table accessors.  A table is an array of 2048-byte blocks (FP32:
// 128 float4 in two 1 KB planes; split: hi plane then lo plane).  TabG reads
// from global memory (L2-resident), TabL from a copy in LDS.

typedef const __attribute__((address_space(3))) char* lds_cptr;

struct TabG {
  const char* __restrict__ p;
  __device__ __forceinline__ c4 f32(size_t blk, int lane) const {
    return load_tw(reinterpret_cast<const float4*>(p + blk * 2048), lane);
  }
  template <class PR>
  __device__ __forceinline__ TwS<PR> s16(size_t blk, int lane) const {
    return load_tws<PR>(p + blk * 2048, lane);
  }
};

struct TabL {
  lds_cptr p;
  __device__ __forceinline__ c4 f32(size_t blk, int lane) const {
    typedef const __attribute__((address_space(3))) f32x4* q_t;
    const q_t q = reinterpret_cast<q_t>(p + blk * 2048);
    const f32x4 a = q[lane], b = q[64 + lane];
    c4 r;
    r.v[0] = make_float2(a.x, a.y);
    r.v[1] = make_float2(a.z, a.w);
    r.v[2] = make_float2(b.x, b.y);
    r.v[3] = make_float2(b.z, b.w);
    return r;
  }
  template <class PR>
  __device__ __forceinline__ TwS<PR> s16(size_t blk, int lane) const {
    typedef const __attribute__((address_space(3))) typename PR::V* q_t;
    const q_t q = reinterpret_cast<q_t>(p + blk * 2048);
    TwS<PR> r;
    r.h = q[lane];
    r.l = q[64 + lane];
    return r;
  }
};

}  // namespace pftpie

