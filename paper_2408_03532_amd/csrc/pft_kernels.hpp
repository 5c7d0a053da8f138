// Plain batched partial transform kernels (pft2d_forward / pft2d_adjoint)
// and their launchers, templated on the precision of the contraction; each
// precision is compiled in a translation unit of its own
// (kernels_pft_{f32,bf16,f16}.hip).
#pragma once

#include <type_traits>

#include "internal.hpp"
#include "pft_split.hpp"

namespace pftpie {
namespace {

// Forward: one workgroup of W waves per patch; wave w owns column tiles
// [w*CT, w*CT + CT).  Tiles at or beyond MT are computed on the zero rows of
// the padded table and not stored.
template <class PR, int MT, int CT, bool EXACT>
__global__ __launch_bounds__(64 * ((MT + CT - 1) / CT)) void k_forward(
    const float2* __restrict__ psi, float2* __restrict__ y, int n, int m, int nb,
    const void* __restrict__ fa) {
  const int64_t b = blockIdx.x;
  const int w = threadIdx.x >> 6;
  const int c2t0 = w * CT;
  PlainSrc<EXACT> src{psi + b * (int64_t)n * n, n};
  f32x4 Yre[MT][CT], Yim[MT][CT];
  fwd_engine<PR, MT, CT>(src, nb, TabG{static_cast<const char*>(fa)}, c2t0, Yre, Yim, 0, 1, (int)(b % nb));
  const int lane = lane_id();
  float2* out = y + b * (int64_t)m * m;
#pragma unroll
  for (int c1t = 0; c1t < MT; ++c1t)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int2 rc = tile_rc<Orient<PR>::TR>(c1t, c2t0 + ct, i, lane);
        if (rc.x < m && rc.y < m) out[(size_t)rc.x * m + rc.y] = make_float2(Yre[c1t][ct][i], Yim[c1t][ct][i]);
      }
    }
}

// Y source of the plain adjoint, m % 16 == 0 and 16-byte aligned: two
// 16-byte loads per chunk, every chunk in bounds.
struct CoefSrcExact {
  const float2* __restrict__ p;
  int m;
  __device__ __forceinline__ c4 load(int row, int col0) const {
    const float4* q = reinterpret_cast<const float4*>(p + (size_t)row * m + col0);
    const float4 a = q[0], b = q[1];
    c4 r;
    r.v[0] = make_float2(a.x, a.y);
    r.v[1] = make_float2(a.z, a.w);
    r.v[2] = make_float2(b.x, b.y);
    r.v[3] = make_float2(b.z, b.w);
    return r;
  }
};

// Y source of the plain adjoint (m x m blocks, masked).
struct CoefSrc {
  const float2* __restrict__ p;
  int m;
  __device__ __forceinline__ c4 load(int row, int col0) const {
    c4 r;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int col = col0 + s;
      r.v[s] = (row < m && col < m) ? p[(size_t)row * m + col] : make_float2(0.f, 0.f);
    }
    return r;
  }
};

struct StoreSink {
  float2* __restrict__ out;
  int n;
  template <bool TR>
  __device__ __forceinline__ void put(int k1t, int k2t, const f32x4& re, const f32x4& im) const {
    const int lane = lane_id();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int2 rc = tile_rc<TR>(k1t, k2t, i, lane);
      if (rc.x < n && rc.y < n) out[(size_t)rc.x * n + rc.y] = make_float2(re[i], im[i]);
    }
  }
};

// Sink of transposed-orientation tiles (element i of lane (r, g) at row
// 16 k1t + r, column 16 k2t + 4 g + i) for n % 16 == 0 and 16-byte aligned
// output.  Lanes r and r + 8 of each 16-lane row swap one half of their four
// values (row rotate by 8), so each of the two 16-byte-per-lane stores
// writes 8 whole 128-byte tile rows instead of half of 16.
struct StoreSinkRows {
  float2* __restrict__ out;
  int n;
  template <bool TR>
  __device__ __forceinline__ void put(int k1t, int k2t, const f32x4& re, const f32x4& im) const {
    static_assert(TR, "row stores serve the transposed tile orientation");
    const int lane = lane_id();
    const int r16 = lane & 15, g = lane >> 4;
    const bool upper = r16 >= 8;
    const float a[4] = {re[0], im[0], re[1], im[1]};  // columns 4g, 4g+1
    const float b[4] = {re[2], im[2], re[3], im[3]};  // columns 4g+2, 4g+3
    float r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float snd = upper ? a[k] : b[k];
      r[k] = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, snd), 0x128, 0xf, 0xf, false));
    }
    // lane r < 8: row r columns 4g.. (own a), row r + 8 columns 4g.. (partner's a)
    // lane r >= 8: row r - 8 columns 4g+2.. (partner's b), row r columns 4g+2.. (own b)
    const int row = k1t * 16 + (r16 & 7);
    const int col = k2t * 16 + 4 * g + 2 * (r16 >> 3);
    float4* q0 = reinterpret_cast<float4*>(out + (size_t)row * n + col);
    float4* q1 = reinterpret_cast<float4*>(out + (size_t)(row + 8) * n + col);
    *q0 = upper ? make_float4(r[0], r[1], r[2], r[3]) : make_float4(a[0], a[1], a[2], a[3]);
    *q1 = upper ? make_float4(b[0], b[1], b[2], b[3]) : make_float4(r[0], r[1], r[2], r[3]);
  }
};

// Adjoint: one workgroup of W waves per patch; wave w takes column tiles
// w, w + W, ...
template <class PR, int MT>
__global__ __launch_bounds__(256) void k_adjoint(const float2* __restrict__ y, float2* __restrict__ psi,
                                                 int n, int m, int nb, const void* __restrict__ ft) {
  const int64_t b = blockIdx.x;
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  CoefSrc src{y + b * (int64_t)m * m, m};
  StoreSink sink{psi + b * (int64_t)n * n, n};
  for (int kt2 = w; kt2 < nb; kt2 += nw) adj_engine<PR, MT>(src, nb, TabG{static_cast<const char*>(ft)}, kt2, sink);
}

// Persistent variants: one workgroup per compute unit copies the whole
// twiddle table into LDS once, then its waves pull work items (patch,
// column-tile group) / (patch, column tile) until the batch is done.
constexpr int kLdsThreads = 512;

__device__ __forceinline__ void copy_table_to_lds(f32x4* smem, const f32x4* __restrict__ tab, int n16) {
  for (int i = threadIdx.x; i < n16; i += blockDim.x) smem[i] = tab[i];
  __syncthreads();
}

template <class PR, int MT, int CT, int THREADS = kLdsThreads>
__global__ __launch_bounds__(THREADS) void k_forward_lds(const float2* __restrict__ psi, float2* __restrict__ y,
                                                             int n, int m, int nb, const f32x4* __restrict__ tab,
                                                             int tab16, int64_t batch) {
  extern __shared__ f32x4 smem[];
  copy_table_to_lds(smem, tab, tab16);
  const TabL T{(lds_cptr)smem};
  constexpr int W = (MT + CT - 1) / CT;
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int64_t items = batch * W;
  const int lane = lane_id();
  for (int64_t it = (int64_t)blockIdx.x * nwaves + wave; it < items; it += (int64_t)gridDim.x * nwaves) {
    const int64_t b = it / W;
    const int c2t0 = (int)(it % W) * CT;
    PlainSrc<true> src{psi + b * (int64_t)n * n, n};
    f32x4 Yre[MT][CT], Yim[MT][CT];
    fwd_engine<PR, MT, CT>(src, nb, T, c2t0, Yre, Yim, 0, 1, (int)(b % nb));
    float2* out = y + b * (int64_t)m * m;
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int2 rc = tile_rc<Orient<PR>::TR>(c1t, c2t0 + ct, i, lane);
          if (rc.x < m && rc.y < m) out[(size_t)rc.x * m + rc.y] = make_float2(Yre[c1t][ct][i], Yim[c1t][ct][i]);
        }
  }
}

template <class PR, int MT, bool EXACT, int K1, int THREADS = kLdsThreads>
__global__ __launch_bounds__(THREADS) void k_adjoint_lds(const float2* __restrict__ y, float2* __restrict__ psi,
                                                             int n, int m, int nb, const f32x4* __restrict__ tab,
                                                             int tab16, int64_t batch) {
  extern __shared__ f32x4 smem[];
  copy_table_to_lds(smem, tab, tab16);
  const TabL T{(lds_cptr)smem};
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int64_t items = batch * nb;
  for (int64_t it = (int64_t)blockIdx.x * nwaves + wave; it < items; it += (int64_t)gridDim.x * nwaves) {
    const int64_t b = it / nb;
    const int kt2 = (int)(it % nb);
    StoreSink sink{psi + b * (int64_t)n * n, n};
    if constexpr (EXACT) {
      CoefSrcExact src{y + b * (int64_t)m * m, m};
      adj_engine<PR, MT, CoefSrcExact, StoreSink, TabL, K1>(src, nb, T, kt2, sink);
    } else {
      CoefSrc src{y + b * (int64_t)m * m, m};
      adj_engine<PR, MT, CoefSrc, StoreSink, TabL, K1>(src, nb, T, kt2, sink);
    }
  }
}

// Split adjoint, whole patch per wave (m <= 64, m % 16 == 0, n % 16 == 0,
// 16-byte aligned).  At m = 48, 64 the split coefficients of a patch take
// most of the register file: 256-thread workgroups, one wave per SIMD; at
// m <= 32 two waves per SIMD fit.
template <int MT>
constexpr int adj_patch_threads() { return MT <= 2 ? 512 : 256; }
template <class PR, int MT, int THREADS = adj_patch_threads<MT>()>
__global__ __launch_bounds__(THREADS) void k_adjoint_patch_lds(const float2* __restrict__ y,
                                                                   float2* __restrict__ psi, int n, int m, int nb,
                                                                   const f32x4* __restrict__ tab, int tab16,
                                                                   int64_t batch) {
  extern __shared__ f32x4 smem[];
  copy_table_to_lds(smem, tab, tab16);
  const TabL T{(lds_cptr)smem};
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int64_t b = (int64_t)blockIdx.x * nwaves + wave; b < batch; b += (int64_t)gridDim.x * nwaves) {
    CoefSrcExact src{y + b * (int64_t)m * m, m};
    StoreSinkRows sink{psi + b * (int64_t)n * n, n};
    adj_patch_split<PR, MT>(src, nb, T, sink);
  }
}

// FP32 adjoint, whole patch per wave (m <= 64, m % 16 == 0): the raw
// coefficients take 8 MT^2 registers, so two waves per SIMD still fit.
template <int MT, int K1>
__global__ __launch_bounds__(512) void k_adjoint_patch_f32_lds(const float2* __restrict__ y, float2* __restrict__ psi,
                                                                 int n, int m, int nb, const f32x4* __restrict__ tab,
                                                                 int tab16, int64_t batch) {
  extern __shared__ f32x4 smem[];
  copy_table_to_lds(smem, tab, tab16);
  const TabL T{(lds_cptr)smem};
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int64_t b = (int64_t)blockIdx.x * nwaves + wave; b < batch; b += (int64_t)gridDim.x * nwaves) {
    CoefSrcExact src{y + b * (int64_t)m * m, m};
    StoreSink sink{psi + b * (int64_t)n * n, n};
    adj_patch_f32<MT, K1>(src, nb, T, sink);
  }
}

template <class K>
hipError_t launch_lds(K kernel, const pftpie_plan_s* p, size_t tab_bytes, int64_t items, hipStream_t st,
                             const float2* in, float2* out, const void* tab, int64_t batch,
                             int threads = kLdsThreads) {
  // every instantiation is allowed the table's dynamic LDS once
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)tab_bytes);
  if (e != hipSuccess) return e;
  const int64_t waves = threads / 64;
  int64_t grid = (items + waves - 1) / waves;
  if (grid > p->num_cu) grid = p->num_cu;
  hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(threads), tab_bytes, st, in, out, p->n, p->m, p->nb,
                     static_cast<const f32x4*>(tab), (int)(tab_bytes / 16), batch);
  return hipGetLastError();
}

template <class PR, int MT, int CT>
hipError_t fwd_mt_ct(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch, hipStream_t st) {
  constexpr int W = (MT + CT - 1) / CT;
  const bool exact = (p->n % 16 == 0) && ((uintptr_t)psi % 16 == 0);
  // CT = 4 needs more than the 256 registers a 512-thread workgroup leaves:
  // it runs in 256-thread workgroups (one wave per SIMD, 512 registers)
  if (exact && p->use_lds && p->fa_bytes <= kMaxLdsTable) {
    if constexpr (CT == 4)
      return launch_lds(k_forward_lds<PR, MT, CT, 256>, p, p->fa_bytes, batch * W, st, psi, y, p->fa, batch, 256);
    else
      return launch_lds(k_forward_lds<PR, MT, CT>, p, p->fa_bytes, batch * W, st, psi, y, p->fa, batch);
  }
  dim3 grid((unsigned)batch), block(64 * W);
  if (exact)
    hipLaunchKernelGGL((k_forward<PR, MT, CT, true>), grid, block, 0, st, psi, y, p->n, p->m, p->nb, p->fa);
  else
    hipLaunchKernelGGL((k_forward<PR, MT, CT, false>), grid, block, 0, st, psi, y, p->n, p->m, p->nb, p->fa);
  return hipGetLastError();
}

template <class PR, int MT>
hipError_t fwd_mt(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch, hipStream_t st) {
  if constexpr (!std::is_same<PR, PrecF32>::value) {
    // split: one wave takes all four column tiles when the plan asks for it
    // (the operand split is shared by twice the products)
    if constexpr (MT == 4) {
      if (p->fwd_ct == 4) return fwd_mt_ct<PR, 4, 4>(p, psi, y, batch, st);
    }
    return fwd_mt_ct<PR, MT, (MT < 2 ? MT : 2)>(p, psi, y, batch, st);
  } else {
    // FP32: column tiles per wave from the plan (4 only while the Y
    // accumulators stay within 128 registers)
    switch (p->fwd_ct) {
      case 1: return fwd_mt_ct<PrecF32, MT, 1>(p, psi, y, batch, st);
      case 2: if constexpr (MT >= 2) return fwd_mt_ct<PrecF32, MT, 2>(p, psi, y, batch, st); break;
      case 4: if constexpr (MT == 4) return fwd_mt_ct<PrecF32, MT, 4>(p, psi, y, batch, st); break;
      case 3: if constexpr (MT == 3) return fwd_mt_ct<PrecF32, MT, 3>(p, psi, y, batch, st); break;
    }
    return hipErrorInvalidValue;
  }
}

template <class PR>
hipError_t forward_prec(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch, hipStream_t st) {
  if (batch == 0) return hipSuccess;
  switch (p->mt) {
    case 1: return fwd_mt<PR, 1>(p, psi, y, batch, st);
    case 2: return fwd_mt<PR, 2>(p, psi, y, batch, st);
    case 3: return fwd_mt<PR, 3>(p, psi, y, batch, st);
    case 4: return fwd_mt<PR, 4>(p, psi, y, batch, st);
    case 5: return fwd_mt<PR, 5>(p, psi, y, batch, st);
    case 6: return fwd_mt<PR, 6>(p, psi, y, batch, st);
    case 7: return fwd_mt<PR, 7>(p, psi, y, batch, st);
    case 8: return fwd_mt<PR, 8>(p, psi, y, batch, st);
  }
  return hipErrorInvalidValue;
}

template <class PR, int MT>
hipError_t adj_mt(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch, hipStream_t st) {
  constexpr bool kF32 = std::is_same<PR, PrecF32>::value;
  if (p->use_lds_adj && p->ft_bytes <= kMaxLdsTable) {
    const int64_t items = batch * p->nb;
    const bool exact = (p->m % 16 == 0) && ((uintptr_t)y % 16 == 0);
    if constexpr (MT <= 4) {
      // (one stage-2 row tile per step: the three accumulator sets of two
      // would spill at m = 64)
      if constexpr (kF32) {
        if (exact && p->adj_patch)
          return launch_lds(k_adjoint_patch_f32_lds<MT, 1>, p, p->ft_bytes, batch, st, y, psi, p->ft, batch, 512);
      } else {
        if (exact && p->adj_patch && p->n % 16 == 0 && (uintptr_t)psi % 16 == 0)
          return launch_lds(k_adjoint_patch_lds<PR, MT>, p, p->ft_bytes, batch, st, y, psi, p->ft, batch,
                            adj_patch_threads<MT>());
      }
    }
    if constexpr (!kF32) {
      return exact ? launch_lds(k_adjoint_lds<PR, MT, true, 2>, p, p->ft_bytes, items, st, y, psi, p->ft, batch)
                   : launch_lds(k_adjoint_lds<PR, MT, false, 2>, p, p->ft_bytes, items, st, y, psi, p->ft, batch);
    } else {
      if (p->adj_threads == 768) {
        if (p->adj_k1 == 4)
          return exact ? launch_lds(k_adjoint_lds<PrecF32, MT, true, 4, 768>, p, p->ft_bytes, items, st, y, psi,
                                    p->ft, batch, 768)
                       : launch_lds(k_adjoint_lds<PrecF32, MT, false, 4, 768>, p, p->ft_bytes, items, st, y, psi,
                                    p->ft, batch, 768);
        return exact ? launch_lds(k_adjoint_lds<PrecF32, MT, true, 2, 768>, p, p->ft_bytes, items, st, y, psi,
                                  p->ft, batch, 768)
                     : launch_lds(k_adjoint_lds<PrecF32, MT, false, 2, 768>, p, p->ft_bytes, items, st, y, psi,
                                  p->ft, batch, 768);
      }
      if (p->adj_k1 == 4)
        return exact ? launch_lds(k_adjoint_lds<PrecF32, MT, true, 4>, p, p->ft_bytes, items, st, y, psi, p->ft, batch)
                     : launch_lds(k_adjoint_lds<PrecF32, MT, false, 4>, p, p->ft_bytes, items, st, y, psi, p->ft,
                                  batch);
      return exact ? launch_lds(k_adjoint_lds<PrecF32, MT, true, 2>, p, p->ft_bytes, items, st, y, psi, p->ft, batch)
                   : launch_lds(k_adjoint_lds<PrecF32, MT, false, 2>, p, p->ft_bytes, items, st, y, psi, p->ft, batch);
    }
  }
  dim3 grid((unsigned)batch), block(64 * adj_waves(p->nb));
  hipLaunchKernelGGL((k_adjoint<PR, MT>), grid, block, 0, st, y, psi, p->n, p->m, p->nb, p->ft);
  return hipGetLastError();
}

template <class PR>
hipError_t adjoint_prec(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch, hipStream_t st) {
  if (batch == 0) return hipSuccess;
  switch (p->mt) {
    case 1: return adj_mt<PR, 1>(p, y, psi, batch, st);
    case 2: return adj_mt<PR, 2>(p, y, psi, batch, st);
    case 3: return adj_mt<PR, 3>(p, y, psi, batch, st);
    case 4: return adj_mt<PR, 4>(p, y, psi, batch, st);
    case 5: return adj_mt<PR, 5>(p, y, psi, batch, st);
    case 6: return adj_mt<PR, 6>(p, y, psi, batch, st);
    case 7: return adj_mt<PR, 7>(p, y, psi, batch, st);
    case 8: return adj_mt<PR, 8>(p, y, psi, batch, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace
}  // namespace pftpie
