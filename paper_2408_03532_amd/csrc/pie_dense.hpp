// Dense-contraction kernels of the PIE sweep and their launchers, templated
// on the precision of the contraction; each precision is compiled in a
// translation unit of its own (kernels_pie_{f32,bf16,f16}.hip).
#pragma once

#include <atomic>
#include <type_traits>

#include "internal.hpp"
#include "pft_split.hpp"
#include "pie.hpp"

namespace pftpie {
namespace {

// Gather source that also tracks max |P|^2 and max |O|^2 over what it reads.
// (entries outside the patch are zeros and leave the maxima unchanged)
template <bool EXACT>
struct GatherTrackSrc {
  using Raw = GatherRaw;
  GatherSrc<EXACT> g;
  mutable float mp, mo;
  __device__ __forceinline__ Raw load_raw(int row, int col0) const { return g.load_raw(row, col0); }
  __device__ __forceinline__ c4 combine(const Raw& v) const {
    c4 z;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float2 p = v.p.v[s], o = v.o.v[s];
      mp = fmaxf(mp, p.x * p.x + p.y * p.y);
      mo = fmaxf(mo, o.x * o.x + o.y * o.y);
      z.v[s] = cmul(p, o);
    }
    return z;
  }
  __device__ __forceinline__ c4 load(int row, int col0) const { return combine(load_raw(row, col0)); }
};

// Magnitude projection (eq. (3)) of coefficient (c1, c2) of chunk entry q:
// stores the residual r = a u/|u| - u (theta(0) = 0; zero for an invalid
// entry) and returns the objective term (|u| - a)^2 (eq. (4)).
__device__ __forceinline__ double pie_project_one(const PieArgs& a, int q, int j, bool valid, int c1, int c2,
                                                  float ur, float ui) {
  const int m = a.m;
  const float av = a.amp[(size_t)j * m * m + (size_t)c1 * m + c2];
  const float mag = sqrtf(ur * ur + ui * ui);
  float2 r;
  if (!valid) {
    r = make_float2(0.f, 0.f);
  } else if (mag > 0.f) {
    const float s = av / mag - 1.f;  // a u/|u| - u = (a/|u| - 1) u
    r = make_float2(s * ur, s * ui);
  } else {
    r = make_float2(av - ur, -ui);  // theta(0) = 0
  }
  a.R[(size_t)q * m * m + (size_t)c1 * m + c2] = r;
  const double d = (double)mag - (double)av;
  return valid ? d * d : 0.0;
}

// Forward + projection.  Block = WR x WC waves: wave (wr, wc) runs strips
// g, g + G, ... (row group g = split * WR + wr, G = WR * splits) for
// column-tile group wc; partial spectra of wr > 0 are added to wr = 0
// through LDS, whose waves then apply the projection, or, when the
// position's strips are split over several workgroups (SPLIT, blockIdx.y),
// store the workgroup's partial spectrum for k_pie_project.
template <class PR, int MT, int CT, int WR, bool EXACT, bool TRACK, bool SPLIT, int RS = 1>
__global__ __launch_bounds__(64 * WR * ((MT + CT - 1) / CT)) void k_pie_forward(PieArgs a, int c0) {
  constexpr int WC = (MT + CT - 1) / CT;
  const int q = blockIdx.x;
  bool valid;
  const int j = pos_index(a.order, a.J, c0, q, &valid);
  const int w = threadIdx.x >> 6;
  const int wc = w % WC, wr = w / WC;
  const int c2t0 = wc * CT;
  const int2 ps = a.pos[j];
  const int lane = lane_id();
  const int g0 = SPLIT ? (int)blockIdx.y * WR + wr : wr;
  const int G = SPLIT ? (int)gridDim.y * WR : WR;
  f32x4 Yre[MT][CT], Yim[MT][CT];
  if constexpr (TRACK) {
    GatherTrackSrc<EXACT> src{{a.O, a.P, a.W, a.n, ps.x, ps.y}, 0.f, 0.f};
    fwd_engine<PR, MT, CT>(src, a.nb, TabG{static_cast<const char*>(a.fa)}, c2t0, Yre, Yim, g0, G);
    if (wc == 0) {
      const float mp = wave_max(src.mp), mo = wave_max(src.mo);
      if (lane == 0 && valid) {
        atomicMax(&a.winmax[2 * j], __float_as_uint(mp));
        atomicMax(&a.winmax[2 * j + 1], __float_as_uint(mo));
      }
    }
  } else {
    GatherSrc<EXACT> src{a.O, a.P, a.W, a.n, ps.x, ps.y};
    if constexpr (RS > 1)
      fwd_wave_rs<MT, CT, RS>(src, a.nb, TabG{static_cast<const char*>(a.fa)}, c2t0, Yre, Yim, g0, G);
    else
      fwd_engine<PR, MT, CT>(src, a.nb, TabG{static_cast<const char*>(a.fa)}, c2t0, Yre, Yim, g0, G);
  }
  if constexpr (WR > 1) {
    // partial spectra: [WR - 1][WC][MT * CT * 2][64 lanes] f32x4
    __shared__ f32x4 part[(WR - 1) * WC * MT * CT * 2 * 64];
    if (wr > 0) {
      f32x4* dst = part + ((size_t)((wr - 1) * WC + wc) * MT * CT * 2) * 64;
#pragma unroll
      for (int a1 = 0; a1 < MT; ++a1)
#pragma unroll
        for (int b1 = 0; b1 < CT; ++b1) {
          dst[((a1 * CT + b1) * 2 + 0) * 64 + lane] = Yre[a1][b1];
          dst[((a1 * CT + b1) * 2 + 1) * 64 + lane] = Yim[a1][b1];
        }
    }
    __syncthreads();
    if (wr > 0) return;
#pragma unroll
    for (int r = 1; r < WR; ++r) {
      const f32x4* src = part + ((size_t)((r - 1) * WC + wc) * MT * CT * 2) * 64;
#pragma unroll
      for (int a1 = 0; a1 < MT; ++a1)
#pragma unroll
        for (int b1 = 0; b1 < CT; ++b1) {
          Yre[a1][b1] += src[((a1 * CT + b1) * 2 + 0) * 64 + lane];
          Yim[a1][b1] += src[((a1 * CT + b1) * 2 + 1) * 64 + lane];
        }
    }
  }
  const int m = a.m;
  if constexpr (SPLIT) {
    float2* part = a.part + ((size_t)q * gridDim.y + blockIdx.y) * m * m;
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int2 rc = tile_rc<Orient<PR>::TR>(c1t, c2t0 + ct, i, lane);
          if (rc.x < m && rc.y < m) part[(size_t)rc.x * m + rc.y] = make_float2(Yre[c1t][ct][i], Yim[c1t][ct][i]);
        }
    return;
  }
  double phi = 0.0;
#pragma unroll
  for (int c1t = 0; c1t < MT; ++c1t)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int2 rc = tile_rc<Orient<PR>::TR>(c1t, c2t0 + ct, i, lane);
        if (rc.x < m && rc.y < m) phi += pie_project_one(a, q, j, valid, rc.x, rc.y, Yre[c1t][ct][i], Yim[c1t][ct][i]);
      }
    }
  phi = wave_sum(phi);
  if (lane == 0 && valid && !a.probe_pass) a.phi_part[(size_t)j * 4 + wc] = phi;
}

// Sum of the partial spectra of chunk entry q (fixed order over the splits)
// and the projection; blockIdx.y takes a quarter of the rows, its objective
// sum goes to that position's slot blockIdx.y.
__global__ __launch_bounds__(256) void k_pie_project(PieArgs a, int c0) {
  __shared__ double sh[4];
  const int q = blockIdx.x;
  bool valid;
  const int j = pos_index(a.order, a.J, c0, q, &valid);
  const int m = a.m, S = a.splits;
  const int rows = (m + 3) / 4, r0 = blockIdx.y * rows;
  const int r1 = r0 + rows < m ? r0 + rows : m;
  const float2* part = a.part + (size_t)q * S * m * m;
  double phi = 0.0;
  for (int t = r0 * m + threadIdx.x; t < r1 * m; t += blockDim.x) {
    float ur = 0.f, ui = 0.f;
    for (int s = 0; s < S; ++s) {
      const float2 v = part[(size_t)s * m * m + t];
      ur += v.x;
      ui += v.y;
    }
    phi += pie_project_one(a, q, j, valid, t / m, t % m, ur, ui);
  }
  phi = wave_sum(phi);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = phi;
  __syncthreads();
  if (threadIdx.x == 0 && valid && !a.probe_pass) a.phi_part[(size_t)j * 4 + blockIdx.y] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Residual source of the adjoint (m x m, masked).
struct ResSrc {
  const float2* __restrict__ p;
  int m;
  __device__ __forceinline__ c4 load(int row, int col0) const {
    c4 v;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int col = col0 + s;
      v.v[s] = (row < m && col < m) ? p[(size_t)row * m + col] : make_float2(0.f, 0.f);
    }
    return v;
  }
};

// Single-position chunk: O[window] += beta conj(P) dpsi / (|P|^2 + alpha max |P|^2)
// (denominator only with norm), and with a probe step
// P += gamma conj(O_j) dpsi / (|O_j|^2 + alpha max |O_j|^2), both from the
// values before this position's update.  probe_pass: the second pass of the
// probe step at the updated object (eq. (6) as printed): P += gamma conj(O_j)
// dpsi only, O unchanged.  Each pixel belongs to one lane.
struct UpdateSink {
  float2* __restrict__ O;
  float2* __restrict__ P;
  int n, W, r, c, norm, probe_step, valid, probe_pass;
  float inv, beta, gamma;
  double regP, regO;  // alpha * max |P|^2, alpha * max |O_j|^2
  template <bool TR>
  __device__ __forceinline__ void put(int k1t, int k2t, const f32x4& xre, const f32x4& xim) const {
    if (!valid) return;
    const int lane = lane_id();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int2 rc = tile_rc<TR>(k1t, k2t, i, lane);
      const int k1 = rc.x, k2 = rc.y;
      if (k1 < n && k2 < n) {
        const float2 d = make_float2(xre[i] * inv, xim[i] * inv);
        const size_t pi = (size_t)k1 * n + k2;
        const size_t o = (size_t)(r + k1) * W + (c + k2);
        const float2 p = P[pi];
        const float2 ov = O[o];
        if (probe_pass) {
          const float2 vp = cmulc(ov, d);
          P[pi] = make_float2(p.x + gamma * vp.x, p.y + gamma * vp.y);
          continue;
        }
        float so = beta;
        if (norm) {
          const double p2 = (double)p.x * p.x + (double)p.y * p.y;
          so = p2 > 0.0 ? (float)((double)beta / (p2 + regP)) : 0.f;
        }
        const float2 vo = cmulc(p, d);
        O[o] = make_float2(ov.x + so * vo.x, ov.y + so * vo.y);
        if (probe_step) {
          float sp = gamma;
          if (norm) {
            const double o2 = (double)ov.x * ov.x + (double)ov.y * ov.y;
            sp = o2 > 0.0 ? (float)((double)gamma / (o2 + regO)) : 0.f;
          }
          const float2 vp = cmulc(ov, d);
          P[pi] = make_float2(p.x + sp * vp.x, p.y + sp * vp.y);
        }
      }
    }
  }
};

// Larger chunks: store dpsi = X / n^2.
struct DeltaSink {
  float2* __restrict__ out;
  int n;
  float inv;
  template <bool TR>
  __device__ __forceinline__ void put(int k1t, int k2t, const f32x4& xre, const f32x4& xim) const {
    const int lane = lane_id();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int2 rc = tile_rc<TR>(k1t, k2t, i, lane);
      if (rc.x < n && rc.y < n) out[(size_t)rc.x * n + rc.y] = make_float2(xre[i] * inv, xim[i] * inv);
    }
  }
};

// K2 > 1 (FP32, long windows): each wave takes K2 neighbouring column tiles
// so the FT table streams once per K2 tiles.
template <class PR, int MT, bool SINGLE, int K2 = 1>
__global__ __launch_bounds__(256) void k_pie_adjoint(PieArgs a, int c0) {
  const int q = blockIdx.x;
  bool valid;
  const int j = pos_index(a.order, a.J, c0, q, &valid);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  ResSrc src{a.R + (size_t)q * a.m * a.m, a.m};
  const TabG T{static_cast<const char*>(a.ft)};
  if constexpr (SINGLE) {
    const int2 ps = a.pos[j];
    double regP = 0.0, regO = 0.0;
    if (a.norm) {
      regP = a.alpha * (double)__uint_as_float(a.winmax[2 * j]);
      regO = a.alpha * (double)__uint_as_float(a.winmax[2 * j + 1]);
    }
    UpdateSink sink{a.O, a.P, a.n, a.W, ps.x, ps.y, a.norm, a.probe_step, (int)valid, a.probe_pass,
                    a.inv_n2, a.beta, a.gamma, regP, regO};
    if constexpr (K2 > 1) {
      for (int gi = blockIdx.y * nw + w; gi * K2 < a.nb; gi += gridDim.y * nw)
        adj_tiles_f32<MT, K2>(src, a.nb, T, gi * K2, sink);
    } else {
      for (int kt2 = blockIdx.y * nw + w; kt2 < a.nb; kt2 += gridDim.y * nw)
        adj_engine<PR, MT>(src, a.nb, T, kt2, sink);
    }
  } else {
    DeltaSink sink{a.dpsi + (size_t)q * a.n * a.n, a.n, a.inv_n2};
    if constexpr (K2 > 1) {
      for (int gi = blockIdx.y * nw + w; gi * K2 < a.nb; gi += gridDim.y * nw)
        adj_tiles_f32<MT, K2>(src, a.nb, T, gi * K2, sink);
    } else {
      for (int kt2 = blockIdx.y * nw + w; kt2 < a.nb; kt2 += gridDim.y * nw)
        adj_engine<PR, MT>(src, a.nb, T, kt2, sink);
    }
  }
}

// Workgroups of Kernel at `threads` threads (a multiple of 64, at most 1024)
// that one compute unit holds at once; the first query of each kernel and
// block size asks the runtime, later ones read the cache.
template <auto Kernel>
static int blocks_per_cu(int threads) {
  static std::atomic<int> cache[17];
  const int w = threads >> 6;
  int n = cache[w].load(std::memory_order_relaxed);
  if (n == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, Kernel, threads, 0) != hipSuccess || n < 1) n = 1;
    cache[w].store(n, std::memory_order_relaxed);
  }
  return n;
}

// forward split: WR row groups per position, summed through LDS (WR - 1
// copies of the partial spectrum): two up to 64 kept coefficients (four
// groups at m <= 32 spent more on the partial sums and the epilogue than the
// extra waves gained), one above
template <int MT>
constexpr int pie_wr() {
  return MT <= 4 ? 2 : 1;
}

template <class PR, int MT, bool TRACK>
static void fwd_launch(const PieArgs& a, int c0, int cnt, hipStream_t st) {
  constexpr int CT = (MT <= 2) ? MT : 2;
  constexpr int WC = (MT + CT - 1) / CT;
  constexpr int WR = pie_wr<MT>();
  static_assert(CT == (MT <= 2 ? MT : 2) && WR == (MT <= 4 ? 2 : 1),
                "the host-side split count assumes this work split");
  dim3 grid(cnt, a.splits), block(64 * WR * WC);
  const bool exact = a.n % 16 == 0;
  if (a.splits > 1) {
    // long windows (>= 8 strips per row group, FP32, untracked): four strips
    // per pass share each twiddle block of the uncached table
    constexpr bool kRs = std::is_same<PR, PrecF32>::value && !TRACK;
    if (kRs && exact && pie_fwd_rs(a.nb, WR, a.splits))
      hipLaunchKernelGGL((k_pie_forward<PR, MT, CT, WR, true, TRACK, true, kRs ? 4 : 1>), grid, block, 0, st, a, c0);
    else if (exact)
      hipLaunchKernelGGL((k_pie_forward<PR, MT, CT, WR, true, TRACK, true>), grid, block, 0, st, a, c0);
    else
      hipLaunchKernelGGL((k_pie_forward<PR, MT, CT, WR, false, TRACK, true>), grid, block, 0, st, a, c0);
    hipLaunchKernelGGL(k_pie_project, dim3(cnt, 4), dim3(256), 0, st, a, c0);
  } else {
    if (exact)
      hipLaunchKernelGGL((k_pie_forward<PR, MT, CT, WR, true, TRACK, false>), grid, block, 0, st, a, c0);
    else
      hipLaunchKernelGGL((k_pie_forward<PR, MT, CT, WR, false, TRACK, false>), grid, block, 0, st, a, c0);
  }
}

template <class PR, int MT>
static void chunk_prec(const PieArgs& a, int c0, int cnt, hipStream_t st) {
  const bool single = (cnt == 1);
  if (single && (a.norm || a.probe_step))
    fwd_launch<PR, MT, true>(a, c0, cnt, st);
  else
    fwd_launch<PR, MT, false>(a, c0, cnt, st);
  // column tiles of the adjoint over a second grid dimension when the chunk
  // alone leaves compute units idle, balanced against the workgroups that
  // fit on the chip at once; long FP32 windows take K2 column tiles per wave
  // (the FT table then streams 1/K2 as often; K2 = 2 above 64 kept
  // coefficients, where four tiles' accumulators would spill)
  constexpr bool kF32 = std::is_same<PR, PrecF32>::value;
  constexpr int K2 = kF32 ? (MT <= 4 ? 4 : 2) : 1;
  const bool tiles4 = kF32 && a.nb >= 128;
  const int units = tiles4 ? (a.nb + K2 - 1) / K2 : a.nb;
  const int nw = adj_waves(a.nb);
  const int per = (units + nw - 1) / nw;
  int gy = 1;
  if ((long)cnt * nw < 4L * a.num_cu) {
    int occ;
    if (tiles4)
      occ = single ? blocks_per_cu<k_pie_adjoint<PR, MT, true, K2>>(64 * nw)
                   : blocks_per_cu<k_pie_adjoint<PR, MT, false, K2>>(64 * nw);
    else
      occ = single ? blocks_per_cu<k_pie_adjoint<PR, MT, true>>(64 * nw)
                   : blocks_per_cu<k_pie_adjoint<PR, MT, false>>(64 * nw);
    gy = pie_balanced_y(cnt, units, nw, per, (long)a.num_cu * occ);
  }
  dim3 grid(cnt, gy), block(64 * nw);
  if (tiles4) {
    if (single)
      hipLaunchKernelGGL((k_pie_adjoint<PR, MT, true, K2>), grid, block, 0, st, a, c0);
    else
      hipLaunchKernelGGL((k_pie_adjoint<PR, MT, false, K2>), grid, block, 0, st, a, c0);
  } else if (single) {
    hipLaunchKernelGGL((k_pie_adjoint<PR, MT, true>), grid, block, 0, st, a, c0);
  } else {
    hipLaunchKernelGGL((k_pie_adjoint<PR, MT, false>), grid, block, 0, st, a, c0);
  }
}

template <class PR, int MT>
static int fwd_split_blocks(bool rs) {
  constexpr int CT = (MT <= 2) ? MT : 2;
  constexpr int WC = (MT + CT - 1) / CT;
  constexpr int WR = pie_wr<MT>();
  constexpr bool kF32 = std::is_same<PR, PrecF32>::value;
  if (rs && kF32) return blocks_per_cu<k_pie_forward<PR, MT, CT, WR, true, false, true, kF32 ? 4 : 1>>(64 * WR * WC);
  return blocks_per_cu<k_pie_forward<PR, MT, CT, WR, true, false, true>>(64 * WR * WC);
}

template <class PR>
static int fwd_split_blocks_mt(int mt, bool rs) {
  switch (mt) {
    case 1: return fwd_split_blocks<PR, 1>(rs);
    case 2: return fwd_split_blocks<PR, 2>(rs);
    case 3: return fwd_split_blocks<PR, 3>(rs);
    case 4: return fwd_split_blocks<PR, 4>(rs);
    case 5: return fwd_split_blocks<PR, 5>(rs);
    case 6: return fwd_split_blocks<PR, 6>(rs);
    case 7: return fwd_split_blocks<PR, 7>(rs);
    case 8: return fwd_split_blocks<PR, 8>(rs);
    default: return 1;
  }
}

template <class PR>
void chunk_dense(const PieArgs& a, int c0, int cnt, hipStream_t st) {
  switch (a.mt) {
    case 1: chunk_prec<PR, 1>(a, c0, cnt, st); break;
    case 2: chunk_prec<PR, 2>(a, c0, cnt, st); break;
    case 3: chunk_prec<PR, 3>(a, c0, cnt, st); break;
    case 4: chunk_prec<PR, 4>(a, c0, cnt, st); break;
    case 5: chunk_prec<PR, 5>(a, c0, cnt, st); break;
    case 6: chunk_prec<PR, 6>(a, c0, cnt, st); break;
    case 7: chunk_prec<PR, 7>(a, c0, cnt, st); break;
    case 8: chunk_prec<PR, 8>(a, c0, cnt, st); break;
    default: break;
  }
}

}  // namespace
}  // namespace pftpie
