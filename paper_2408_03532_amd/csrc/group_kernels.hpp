// The persistent kernel of the uneven batch, templated on the precision of
// the contraction (each precision is compiled in a translation unit of its
// own, kernels_group_{f32,bf16,f16}.hip): every wave pulls work items from a
// device counter (items are sorted longest-first on the host) and runs the
// forward or adjoint engine of the item's class.  Every wave leaves the loop
// once the counter passes the item count, so the grid always drains.
#pragma once

#include "group.hpp"
#include "pft_split.hpp"

namespace pftpie {
namespace {

struct GCoefSrc {
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

struct GStoreSink {
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

template <class PR, int MT, int CT, bool EXACT>
__device__ __forceinline__ void fwd_item(const GroupClass& c, const GroupItem& it, const float2* in, float2* out) {
  const int c2t0 = it.slot * CT;
  PlainSrc<EXACT> src{in + it.in_off, c.n};
  f32x4 Yre[MT][CT], Yim[MT][CT];
  const TabG tab{static_cast<const char*>(c.tab)};
  if constexpr (Orient<PR>::TR)
    fwd_engine<PR, MT, CT>(src, c.nb, tab, c2t0, Yre, Yim);
  else  // FP32: three products for every block (the kernel runs one wave per SIMD)
    fwd_wave<MT, CT, PlainSrc<EXACT>, TabG, true>(src, c.nb, tab, c2t0, Yre, Yim);
  const int lane = lane_id();
  float2* o = out + it.out_off;
  const int m = c.m;
#pragma unroll
  for (int c1t = 0; c1t < MT; ++c1t)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int2 rc = tile_rc<Orient<PR>::TR>(c1t, c2t0 + ct, i, lane);
        if (rc.x < m && rc.y < m) o[(size_t)rc.x * m + rc.y] = make_float2(Yre[c1t][ct][i], Yim[c1t][ct][i]);
      }
}

template <class PR, int MT>
__device__ __forceinline__ void adj_item(const GroupClass& c, const GroupItem& it, const float2* in, float2* out) {
  GCoefSrc src{in + it.in_off, c.m};
  GStoreSink sink{out + it.out_off, c.n};
  const int k0 = it.slot * c.kpi;
  const int k1 = (k0 + c.kpi < c.nb) ? k0 + c.kpi : c.nb;
  for (int kt2 = k0; kt2 < k1; ++kt2) adj_engine<PR, MT>(src, c.nb, TabG{static_cast<const char*>(c.tab)}, kt2, sink);
}

template <class PR, int MT, int CT>
__device__ __forceinline__ void fwd_dispatch_exact(const GroupClass& c, const GroupItem& it, const float2* in,
                                                   float2* out) {
  if (c.exact)
    fwd_item<PR, MT, CT, true>(c, it, in, out);
  else
    fwd_item<PR, MT, CT, false>(c, it, in, out);
}

template <class PR, bool ADJ>
__global__ __launch_bounds__(kGroupThreads) void k_group(GroupArgs a) {
  const int lane = lane_id();
  for (;;) {
    unsigned long long i = 0;
    if (lane == 0) i = atomicAdd(a.counter, 1ull);
    i = __shfl(i, 0, 64);
    if (i >= (unsigned long long)a.nitems) break;
    const GroupItem it = a.items[i];
    const GroupClass c = a.cls[it.cls];
    if constexpr (ADJ) {
      switch (c.mt) {
        case 1: adj_item<PR, 1>(c, it, a.in, a.out); break;
        case 2: adj_item<PR, 2>(c, it, a.in, a.out); break;
        case 3: adj_item<PR, 3>(c, it, a.in, a.out); break;
        case 4: adj_item<PR, 4>(c, it, a.in, a.out); break;
        case 5: adj_item<PR, 5>(c, it, a.in, a.out); break;
        case 6: adj_item<PR, 6>(c, it, a.in, a.out); break;
        case 7: adj_item<PR, 7>(c, it, a.in, a.out); break;
        case 8: adj_item<PR, 8>(c, it, a.in, a.out); break;
        default: break;
      }
    } else {
      // column tiles per wave: ct = min(mt, 2) for mt <= 2, else 2 (or 1)
      switch (c.mt * 4 + c.ct) {
        case 1 * 4 + 1: fwd_dispatch_exact<PR, 1, 1>(c, it, a.in, a.out); break;
        case 2 * 4 + 1: fwd_dispatch_exact<PR, 2, 1>(c, it, a.in, a.out); break;
        case 2 * 4 + 2: fwd_dispatch_exact<PR, 2, 2>(c, it, a.in, a.out); break;
        case 3 * 4 + 1: fwd_dispatch_exact<PR, 3, 1>(c, it, a.in, a.out); break;
        case 3 * 4 + 2: fwd_dispatch_exact<PR, 3, 2>(c, it, a.in, a.out); break;
        case 4 * 4 + 1: fwd_dispatch_exact<PR, 4, 1>(c, it, a.in, a.out); break;
        case 4 * 4 + 2: fwd_dispatch_exact<PR, 4, 2>(c, it, a.in, a.out); break;
        case 5 * 4 + 1: fwd_dispatch_exact<PR, 5, 1>(c, it, a.in, a.out); break;
        case 5 * 4 + 2: fwd_dispatch_exact<PR, 5, 2>(c, it, a.in, a.out); break;
        case 6 * 4 + 1: fwd_dispatch_exact<PR, 6, 1>(c, it, a.in, a.out); break;
        case 6 * 4 + 2: fwd_dispatch_exact<PR, 6, 2>(c, it, a.in, a.out); break;
        case 7 * 4 + 1: fwd_dispatch_exact<PR, 7, 1>(c, it, a.in, a.out); break;
        case 7 * 4 + 2: fwd_dispatch_exact<PR, 7, 2>(c, it, a.in, a.out); break;
        case 8 * 4 + 1: fwd_dispatch_exact<PR, 8, 1>(c, it, a.in, a.out); break;
        case 8 * 4 + 2: fwd_dispatch_exact<PR, 8, 2>(c, it, a.in, a.out); break;
        default: break;
      }
    }
  }
}

}  // namespace
}  // namespace pftpie
