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

// The projection of pie_project_one with the amplitude already loaded.
__device__ __forceinline__ double pie_project_amp(const PieArgs& a, int q, bool valid, int c1, int c2, float ur,
                                                  float ui, float av) {
  const int m = a.m;
  const float mag = sqrtf(ur * ur + ui * ui);
  float2 r;
  if (!valid) {
    r = make_float2(0.f, 0.f);
  } else if (mag > 0.f) {
    const float s = av / mag - 1.f;
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
    GatherTrackSrc<EXACT> src{{a.O, a.P, a.W, a.n, ps.x, ps.y, a.n}, 0.f, 0.f};
    fwd_engine<PR, MT, CT>(src, a.nb, TabG{static_cast<const char*>(a.fa)}, c2t0, Yre, Yim, g0, G);
    if (wc == 0) {
      const float mp = wave_max(src.mp), mo = wave_max(src.mo);
      if (lane == 0 && valid) {
        atomicMax(&a.winmax[2 * j], __float_as_uint(mp));
        atomicMax(&a.winmax[2 * j + 1], __float_as_uint(mo));
      }
    }
  } else {
    GatherSrc<EXACT> src{a.O, a.P, a.W, a.n, ps.x, ps.y, a.n};
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
  int ldp;            // row stride of P (n, or padded in LDS)
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
        const size_t pi = (size_t)k1 * ldp + k2;
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

// Larger chunks: store dpsi = X / n^2 (rows of `stride`, from dpsi_base).
struct DeltaSink {
  float2* __restrict__ out;
  int n, stride;
  float inv;
  template <bool TR>
  __device__ __forceinline__ void put(int k1t, int k2t, const f32x4& xre, const f32x4& xim) const {
    const int lane = lane_id();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int2 rc = tile_rc<TR>(k1t, k2t, i, lane);
      if (rc.x < n && rc.y < n) out[(size_t)rc.x * stride + rc.y] = make_float2(xre[i] * inv, xim[i] * inv);
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
                    a.inv_n2, a.beta, a.gamma, regP, regO, a.n};
    if constexpr (K2 > 1) {
      for (int gi = blockIdx.y * nw + w; gi * K2 < a.nb; gi += gridDim.y * nw)
        adj_tiles_f32<MT, K2>(src, a.nb, T, gi * K2, sink);
    } else {
      for (int kt2 = blockIdx.y * nw + w; kt2 < a.nb; kt2 += gridDim.y * nw)
        adj_engine<PR, MT>(src, a.nb, T, kt2, sink);
    }
  } else {
    const int c = valid ? a.pos[j].y : a.bb_c0;
    DeltaSink sink{a.dpsi + dpsi_base(a, q, c), a.n, a.dstride, a.inv_n2};
    if constexpr (MT <= 4 && K2 == 1) {
      // whole residual per wave (split, or the three-product first stage in
      // FP32), the position's column tiles shared by its waves
      const int first = blockIdx.y * nw + w, step = gridDim.y * nw;
      if constexpr (Orient<PR>::TR)
        adj_patch_split<PR, MT>(src, a.nb, T, sink, first, step);
      else
        adj_patch_f32<MT, 2>(src, a.nb, T, sink, first, step);
    } else if constexpr (K2 > 1) {
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

// Sequential sweep (chunks of one position, eq. (5)) for small windows in
// one persistent workgroup of kSeqWaves waves: for each position of the
// order in turn, the forward (its row groups over waves, partial spectra
// summed through LDS) and projection, a barrier, the adjoint column tiles
// over all waves updating O (and P) in place, a barrier.  One workgroup runs
// on one compute unit, so the barriers alone order each position's reads
// after the previous position's writes; the launch replaces two launches
// per position.  Literal probe steps (eq. (6) as printed) run their second
// pass at the updated object inside the same loop.
constexpr int kSeqWaves = 4;

template <class PR, int MT, bool EXACT>
__global__ __launch_bounds__(64 * kSeqWaves) void k_pie_sequential(PieArgs a) {
  constexpr int CT = (MT <= 2) ? MT : 2;
  constexpr int WC = (MT + CT - 1) / CT;
  constexpr int WR = pie_wr<MT>();
  static_assert(WR * WC <= kSeqWaves, "the forward's waves must fit the workgroup");
  __shared__ f32x4 part[(WR > 1 ? (WR - 1) * WC : 1) * MT * CT * 2 * 64];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  const int wc = w % WC, wr = w / WC;
  const bool fwd_wave = w < WR * WC;
  const TabG FA{static_cast<const char*>(a.fa)};
  const TabG FT{static_cast<const char*>(a.ft)};
  const int passes = a.probe_literal ? 2 : 1;
  for (int t = 0; t < a.J; ++t) {
    bool valid;
    const int j = pos_index(a.order, a.J, t, 0, &valid);
    const int2 ps = a.pos[j];
    for (int pass = 0; pass < passes; ++pass) {
      PieArgs b = a;
      if (a.probe_literal) {
        b.probe_step = pass;  // object pass first, then the probe pass
        b.probe_pass = pass;
      }
      const bool track = b.norm || b.probe_step;
      // forward: Y of this wave's column-tile group over its row group
      f32x4 Yre[MT][CT], Yim[MT][CT];
      if (fwd_wave) {
        if (track) {
          GatherTrackSrc<EXACT> src{{b.O, b.P, b.W, b.n, ps.x, ps.y, b.n}, 0.f, 0.f};
          fwd_engine<PR, MT, CT>(src, b.nb, FA, wc * CT, Yre, Yim, wr, WR);
          if (wc == 0) {
            const float mp = wave_max(src.mp), mo = wave_max(src.mo);
            if (lane == 0 && valid) {
              atomicMax(&b.winmax[2 * j], __float_as_uint(mp));
              atomicMax(&b.winmax[2 * j + 1], __float_as_uint(mo));
            }
          }
        } else {
          GatherSrc<EXACT> src{b.O, b.P, b.W, b.n, ps.x, ps.y, b.n};
          fwd_engine<PR, MT, CT>(src, b.nb, FA, wc * CT, Yre, Yim, wr, WR);
        }
        if (WR > 1 && wr > 0) {
          f32x4* dst = part + ((size_t)((wr - 1) * WC + wc) * MT * CT * 2) * 64;
#pragma unroll
          for (int a1 = 0; a1 < MT; ++a1)
#pragma unroll
            for (int b1 = 0; b1 < CT; ++b1) {
              dst[((a1 * CT + b1) * 2 + 0) * 64 + lane] = Yre[a1][b1];
              dst[((a1 * CT + b1) * 2 + 1) * 64 + lane] = Yim[a1][b1];
            }
        }
      }
      __syncthreads();
      if (fwd_wave && wr == 0) {
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
        double phi = 0.0;
#pragma unroll
        for (int c1t = 0; c1t < MT; ++c1t)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int2 rc = tile_rc<Orient<PR>::TR>(c1t, wc * CT + ct, i, lane);
              if (rc.x < b.m && rc.y < b.m)
                phi += pie_project_one(b, 0, j, valid, rc.x, rc.y, Yre[c1t][ct][i], Yim[c1t][ct][i]);
            }
        phi = wave_sum(phi);
        if (lane == 0 && valid && !b.probe_pass) b.phi_part[(size_t)j * 4 + wc] = phi;
      }
      __syncthreads();
      // adjoint and in-place update, column tiles over every wave
      double regP = 0.0, regO = 0.0;
      if (b.norm) {
        regP = b.alpha * (double)__uint_as_float(b.winmax[2 * j]);
        regO = b.alpha * (double)__uint_as_float(b.winmax[2 * j + 1]);
      }
      UpdateSink sink{b.O, b.P, b.n, b.W, ps.x, ps.y, b.norm, b.probe_step, (int)valid, b.probe_pass,
                      b.inv_n2, b.beta, b.gamma, regP, regO, b.n};
      ResSrc rsrc{b.R, b.m};
      for (int kt2 = w; kt2 < b.nb; kt2 += kSeqWaves) adj_engine<PR, MT>(rsrc, b.nb, FT, kt2, sink);
      __syncthreads();
    }
  }
}

// The same sequential sweep with everything it touches held in LDS: the
// object over the scan's bounding box, the probe, the residual and both
// twiddle tables are loaded once, every position reads and updates them
// there, and the end of the sweep computes the statistics (against the
// object still in global memory) before writing the box back.  One launch
// per sweep; used when these fit the compute unit's LDS.
//
// Without probe step a position changes the object only inside its own
// window, so eq. (5) in sweep order gives the same result whenever every
// pair of overlapping positions runs in sweep order.  TEAMS > 1: the sweep
// is cut into dependency levels (a position's level is one more than the
// highest level of the earlier positions whose windows overlap it, so the
// positions of one level have disjoint windows) and TEAMS groups of
// kSeqWaves waves take the positions of a level side by side.  Every pixel
// then sees the same updates in the same order as in the one-by-one sweep.
struct SeqLdsLayout {
  size_t obj, probe, res, fa, ft, pos, jidx, lvl, sched, lstart, rtab, total;
  int ldo, ldp;  // row strides of the object box and the probe
};

// LDS row stride for rows of `w` complex values: rows read down a column
// then start 8 banks apart (stride = 4 mod 32 complex values).
__host__ __device__ inline int seq_lds_stride(int w) { return w + ((36 - w % 32) % 32); }

__host__ __device__ inline SeqLdsLayout seq_lds_layout(int bb_h, int bb_w, int n, int m, int J, size_t fa_bytes,
                                                         size_t ft_bytes, int teams) {
  SeqLdsLayout L;
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  L.ldo = seq_lds_stride(bb_w);
  L.ldp = seq_lds_stride(n);
  L.fa = 0;
  L.ft = up(fa_bytes);
  L.obj = L.ft + up(ft_bytes);
  L.probe = L.obj + up((size_t)bb_h * L.ldo * 8);
  L.res = L.probe + up((size_t)n * L.ldp * 8);
  L.pos = L.res + (size_t)teams * up((size_t)m * m * 8);
  L.jidx = L.pos + up((size_t)J * 8);
  // levels: each step's level, the steps in level order, where each level
  // starts (J + 1), and each round's step per team (-1: none)
  const size_t lv = teams > 1 ? up((size_t)J * 4) : 0;
  L.lvl = L.jidx + up((size_t)J * 4);
  L.sched = L.lvl + lv;
  L.lstart = L.sched + lv;
  L.rtab = L.lstart + (teams > 1 ? up((size_t)(J + 1) * 4) : 0);
  L.total = L.rtab + (teams > 1 ? up((size_t)J * teams * 4) : 0);
  return L;
}

constexpr int kSeqLevelMaxJ = 2048;  // positions for which the levels are worth finding (O(J^2 / 64) steps)

template <class PR, int MT, bool EXACT, int TEAMS>
__global__ __launch_bounds__(64 * kSeqWaves * TEAMS) void k_pie_sequential_lds(PieArgs a, size_t fa_bytes,
                                                                               size_t ft_bytes) {
  constexpr int CT = (MT <= 2) ? MT : 2;
  constexpr int WC = (MT + CT - 1) / CT;
  constexpr int WR = pie_wr<MT>();
  // FP32: the waves the row groups leave over split each strip's column
  // blocks (KS partial sums per row group)
  constexpr int KS = Orient<PR>::TR ? 1 : kSeqWaves / (WR * WC);
  constexpr int NP = WR * KS;  // partial spectra per column group
  constexpr int PART = NP * WC * MT * CT * 2 * 64;  // every forward wave's partial spectrum
  // projection elements per lane, e = ((wc * MT + c1t) * CT + ct) * 4 + i,
  // shared out over the team's waves (element e to role e mod kSeqWaves)
  constexpr int NE = WC * MT * CT * 4;
  constexpr int EPW = (NE + kSeqWaves - 1) / kSeqWaves;
  static_assert(WR * WC <= kSeqWaves && KS >= 1, "the forward's waves must fit the team");
  extern __shared__ f32x4 dyn[];
  __shared__ f32x4 part[TEAMS][PART];
  __shared__ double red[kSeqWaves * TEAMS][4];
  __shared__ unsigned wmx[TEAMS][2][2];  // per-position max |P|^2, max |O_j|^2 (double-buffered by round parity)
  __shared__ int nlev, nrounds;
  char* base = reinterpret_cast<char*>(dyn);
  const SeqLdsLayout L = seq_lds_layout(a.bb_h, a.bb_w, a.n, a.m, a.J, fa_bytes, ft_bytes, TEAMS);
  float2* Ol = reinterpret_cast<float2*>(base + L.obj);
  float2* Pl = reinterpret_cast<float2*>(base + L.probe);
  int2* posl = reinterpret_cast<int2*>(base + L.pos);  // window corner in the box, x < 0: no position
  int* jl = reinterpret_cast<int*>(base + L.jidx);     // position index of each step
  int* lvl = reinterpret_cast<int*>(base + L.lvl);
  int* sched = reinterpret_cast<int*>(base + L.sched);
  int* lstart = reinterpret_cast<int*>(base + L.lstart);
  int* rtab = reinterpret_cast<int*>(base + L.rtab);
  const int ldo = L.ldo, ldp = L.ldp;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int w = tid >> 6;
  const int lane = lane_id();
  // wave w runs on SIMD w % 4; the second team's roles are rotated by two so
  // that the two teams' forward waves (roles 0 and 1) sit on different SIMDs
  const int team = w / kSeqWaves, wl = (w + team * (kSeqWaves / 2)) % kSeqWaves;
  float2* Rl = reinterpret_cast<float2*>(base + L.res + (size_t)team * (((size_t)a.m * a.m * 8 + 255) & ~size_t(255)));
  // load: tables (verbatim), probe, object box, the order's positions;
  // clear the per-position slots
  {
    const f32x4* fa = static_cast<const f32x4*>(a.fa);
    const f32x4* ft = static_cast<const f32x4*>(a.ft);
    f32x4* fal = reinterpret_cast<f32x4*>(base + L.fa);
    f32x4* ftl = reinterpret_cast<f32x4*>(base + L.ft);
    for (size_t i = tid; i < fa_bytes / 16; i += nt) fal[i] = fa[i];
    for (size_t i = tid; i < ft_bytes / 16; i += nt) ftl[i] = ft[i];
    for (int i = tid; i < a.n * a.n; i += nt) Pl[(i / a.n) * ldp + i % a.n] = a.P[i];
    for (int i = tid; i < a.bb_h * a.bb_w; i += nt)
      Ol[(i / a.bb_w) * ldo + i % a.bb_w] = a.O[(size_t)(a.bb_r0 + i / a.bb_w) * a.W + a.bb_c0 + i % a.bb_w];
    for (int t = tid; t < a.J; t += nt) {
      bool valid;
      const int j = pos_index(a.order, a.J, t, 0, &valid);
      const int2 ps = a.pos[j];
      posl[t] = valid ? make_int2(ps.x - a.bb_r0, ps.y - a.bb_c0) : make_int2(-1, 0);
      jl[t] = j;
    }
    if (tid < 4 * TEAMS) (&wmx[0][0][0])[tid] = 0u;
    if constexpr (TEAMS > 1)
      for (int i = tid; i <= a.J; i += nt) lstart[i] = 0;
  }
  __syncthreads();
  if constexpr (TEAMS > 1) {
    // levels, by the first wave in sweep order; a skipped entry touches
    // nothing and takes level 0
    if (w == 0) {
      volatile int* lev = lvl;
      int top = 0;
      for (int t = 0; t < a.J; ++t) {
        const int2 pt = posl[t];
        int l = 0;
        if (pt.x >= 0)
          for (int u = lane; u < t; u += 64) {
            const int2 pu = posl[u];
            if (pu.x >= 0 && abs(pu.x - pt.x) < a.n && abs(pu.y - pt.y) < a.n) l = max(l, lev[u] + 1);
          }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) l = max(l, __shfl_xor(l, off, 64));
        if (lane == 0) lev[t] = l;
        top = max(top, l);
      }
      if (lane == 0) nlev = top + 1;
    }
    __syncthreads();
    // stable counting sort of the steps by level (sweep order inside a
    // level, so that each team's share of the sweep is fixed)
    for (int t = tid; t < a.J; t += nt) atomicAdd(&lstart[lvl[t] + 1], 1);
    __syncthreads();
    if (tid == 0)
      for (int l = 1; l <= nlev; ++l) lstart[l] += lstart[l - 1];
    __syncthreads();
    for (int t = tid; t < a.J; t += nt) {
      const int l = lvl[t];
      int before = 0;
      for (int u = 0; u < t; ++u) before += lvl[u] == l;
      sched[lstart[l] + before] = t;
    }
    __syncthreads();
    // the levels as rounds of up to TEAMS steps
    if (tid == 0) {
      int r = 0;
      for (int l = 0; l < nlev; ++l)
        for (int sb = lstart[l]; sb < lstart[l + 1]; sb += TEAMS, ++r)
          for (int k = 0; k < TEAMS; ++k) rtab[r * TEAMS + k] = sb + k < lstart[l + 1] ? sched[sb + k] : -1;
      nrounds = r;
    }
    __syncthreads();
  } else {
    if (tid == 0) nrounds = a.J;
    __syncthreads();
  }
  const TabL FA{(lds_cptr)(base + L.fa)};
  const TabL FT{(lds_cptr)(base + L.ft)};
  const int wc = wl % WC, wr = (wl / WC) % WR, kh = wl / (WC * WR);
  const bool fwd_role = wl < WR * WC * KS;
  const int pslot = kh * WR + wr;                         // partial index (0: the projecting wave)
  auto forward = [&](const auto& src, f32x4(&Yre)[MT][CT], f32x4(&Yim)[MT][CT]) {
    if constexpr (Orient<PR>::TR)
      fwd_engine<PR, MT, CT>(src, a.nb, FA, wc * CT, Yre, Yim, wr, WR);
    else
      fwd_wave<MT, CT>(src, a.nb, FA, wc * CT, Yre, Yim, wr, WR, kh, KS);
  };
  const int passes = a.probe_literal ? 2 : 1;
  const int m = a.m;
  // this team's step of each round (-1: idle), and the projection's
  // amplitudes, requested one round ahead
  auto step_of = [&](int rd) { return TEAMS > 1 ? rtab[rd * TEAMS + team] : rd; };
  // element e of this lane: its (row, column) of the window's spectrum and
  // the partial-spectrum slot and component holding it
  auto element = [&](int e, int& slot, int& comp) {
    const int i = e & 3, blk = e >> 2;  // blk = (wc * MT + c1t) * CT + ct
    const int ct = blk % CT, c1t = (blk / CT) % MT, wce = blk / (CT * MT);
    slot = (wce * MT + c1t) * CT + ct;
    comp = i;
    return tile_rc<Orient<PR>::TR>(c1t, wce * CT + ct, i, lane);
  };
  float avn[EPW];
  auto load_amp = [&](int t) {
    const int j = t >= 0 ? jl[t] : 0;
#pragma unroll
    for (int k = 0; k < EPW; ++k) {
      const int e = wl + k * kSeqWaves;
      int slot, comp;
      const int2 rc = element(e < NE ? e : 0, slot, comp);
      avn[k] = (t >= 0 && e < NE && rc.x < m && rc.y < m) ? a.amp[(size_t)j * m * m + (size_t)rc.x * m + rc.y] : 0.f;
    }
  };
  // (the rounds exchange data through LDS only, so their barriers leave the
  // amplitude prefetch in flight)
  load_amp(step_of(0));
  double phi_acc = 0.0;  // this lane's objective terms over the sweep (summed once at the end)
  for (int round = 0; round < nrounds; ++round) {
    {
      const int t = step_of(round);
      const bool active = t >= 0;  // uniform over the team
      float av[EPW];
#pragma unroll
      for (int k = 0; k < EPW; ++k) av[k] = avn[k];
      if (round + 1 < nrounds) load_amp(step_of(round + 1));
      const int2 rc0 = posl[active ? t : 0];
      const bool valid = active && rc0.x >= 0;
      const int r = valid ? rc0.x : 0, c = valid ? rc0.y : 0;
      unsigned* mx = wmx[team][round & 1];
      if (wl == 0 && lane == 0) {  // the next round's maxima start from zero (last read two rounds ago)
        wmx[team][(round + 1) & 1][0] = 0u;
        wmx[team][(round + 1) & 1][1] = 0u;
      }
      for (int pass = 0; pass < passes; ++pass) {
        PieArgs b = a;
        b.R = Rl;
        if (a.probe_literal) {
          b.probe_step = pass;
          b.probe_pass = pass;
        }
        const bool track = b.norm || b.probe_step;
        f32x4 Yre[MT][CT], Yim[MT][CT];
        if (active && fwd_role) {
          if (track) {
            GatherTrackSrc<EXACT> src{{Ol, Pl, ldo, b.n, r, c, ldp}, 0.f, 0.f};
            forward(src, Yre, Yim);
            if (wc == 0) {
              const float mp = wave_max(src.mp), mo = wave_max(src.mo);
              if (lane == 0) {
                atomicMax(&mx[0], __float_as_uint(mp));
                atomicMax(&mx[1], __float_as_uint(mo));
              }
            }
          } else {
            GatherSrc<EXACT> src{Ol, Pl, ldo, b.n, r, c, ldp};
            forward(src, Yre, Yim);
          }
          {
            f32x4* dst = part[team] + ((size_t)(pslot * WC + wc) * MT * CT * 2) * 64;
#pragma unroll
            for (int a1 = 0; a1 < MT; ++a1)
#pragma unroll
              for (int b1 = 0; b1 < CT; ++b1) {
                dst[((a1 * CT + b1) * 2 + 0) * 64 + lane] = Yre[a1][b1];
                dst[((a1 * CT + b1) * 2 + 1) * 64 + lane] = Yim[a1][b1];
              }
          }
        }
        lds_barrier();
        if (active) {
          // this wave's share of the projection: each element summed over
          // the partial spectra in slot order
          const float* pf = reinterpret_cast<const float*>(part[team]);
          double phi = 0.0;
#pragma unroll
          for (int k = 0; k < EPW; ++k) {
            const int e = wl + k * kSeqWaves;
            if (e >= NE) break;
            int slot, comp;
            const int2 rc = element(e, slot, comp);
            float ur = 0.f, ui = 0.f;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
              const float* q = pf + (size_t)p * WC * MT * CT * 2 * 64 * 4;
              ur += q[((slot * 2 + 0) * 64 + lane) * 4 + comp];
              ui += q[((slot * 2 + 1) * 64 + lane) * 4 + comp];
            }
            if (rc.x < m && rc.y < m) phi += pie_project_amp(b, 0, valid, rc.x, rc.y, ur, ui, av[k]);
          }
          if (!b.probe_pass) phi_acc += phi;
        }
        lds_barrier();
        if (active) {
          double regP = 0.0, regO = 0.0;
          if (b.norm) {
            regP = b.alpha * (double)__uint_as_float(mx[0]);
            regO = b.alpha * (double)__uint_as_float(mx[1]);
          }
          UpdateSink sink{Ol, Pl, b.n, ldo, r, c, b.norm, b.probe_step, (int)valid, b.probe_pass,
                          b.inv_n2, b.beta, b.gamma, regP, regO, ldp};
          ResSrc rsrc{Rl, m};
          bool shared_tiles = false;
          if constexpr (!Orient<PR>::TR) {
            // few column tiles (FP32): two waves per tile, each taking every
            // other row tile of it
            if (2 * b.nb <= kSeqWaves) {
              shared_tiles = true;
              const int kt2 = wl % b.nb, half = wl / b.nb;
              if (half < 2) adj_wave_tile<MT, ResSrc, UpdateSink, TabL, 1>(rsrc, b.nb, FT, kt2, sink, half, 2);
            }
          }
          if (!shared_tiles)
            for (int kt2 = wl; kt2 < b.nb; kt2 += kSeqWaves) adj_engine<PR, MT>(rsrc, b.nb, FT, kt2, sink);
        }
        lds_barrier();
      }
    }
  }
  __syncthreads();
  // statistics against the object still in global memory, then write back:
  // {Phi, ||O_after - O_before||^2, ||O_before||^2, non-finite}
  double v[4] = {phi_acc, 0.0, 0.0, 0.0};
  const int total = a.H * a.W;  // at most kSeqLdsMaxObject
  for (int i = tid; i < total; i += nt) {
    const int y = i / a.W, x = i - y * a.W;
    const float2 z = a.O[i];
    float2 o = z;
    const int yy = y - a.bb_r0, xx = x - a.bb_c0;
    if (yy >= 0 && yy < a.bb_h && xx >= 0 && xx < a.bb_w) o = Ol[yy * ldo + xx];
    const double dx = (double)o.x - z.x, dy = (double)o.y - z.y;
    v[1] += dx * dx + dy * dy;
    v[2] += (double)z.x * z.x + (double)z.y * z.y;
    v[3] += (isfinite(o.x) && isfinite(o.y)) ? 0.0 : 1.0;
  }
  if (a.probe_step)
    for (int i = tid; i < a.n * a.n; i += nt) {
      const float2 pv = Pl[(i / a.n) * ldp + i % a.n];
      v[3] += (isfinite(pv.x) && isfinite(pv.y)) ? 0.0 : 1.0;
    }
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) red[w][k] = v[k];
  __syncthreads();
  if (tid == 0) {
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < kSeqWaves * TEAMS; ++k)
      for (int q = 0; q < 4; ++q) s4[q] += red[k][q];
    a.stats[0] = s4[0] / ((double)a.J * a.period * a.period);
    a.stats[1] = s4[1];
    a.stats[2] = s4[2];
    a.stats[3] = s4[3];
  }
  for (int i = tid; i < a.bb_h * a.bb_w; i += nt)
    a.O[(size_t)(a.bb_r0 + i / a.bb_w) * a.W + a.bb_c0 + i % a.bb_w] = Ol[(i / a.bb_w) * ldo + i % a.bb_w];
  if (a.probe_step)
    for (int i = tid; i < a.n * a.n; i += nt) a.P[i] = Pl[(i / a.n) * ldp + i % a.n];
}

template <class PR, int MT>
bool sequential_lds_prec(const PieArgs& a, size_t fa_bytes, size_t ft_bytes, hipStream_t st) {
  // (the statistics read the whole object from one workgroup)
  if ((size_t)a.H * a.W > kSeqLdsMaxObject) return false;
  // launches `kernel` when its static LDS and the layout for `nteams` fit
  // the compute unit's LDS
  auto launch = [&](auto kernel, int nteams) {
    const SeqLdsLayout L = seq_lds_layout(a.bb_h, a.bb_w, a.n, a.m, a.J, fa_bytes, ft_bytes, nteams);
    hipFuncAttributes attr{};
    if (L.total > kSeqLdsBytes ||
        hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(kernel)) != hipSuccess ||
        L.total + attr.sharedSizeBytes > kMaxLdsTable ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)L.total) != hipSuccess)
      return false;
    hipLaunchKernelGGL(kernel, dim3(1), dim3(64 * kSeqWaves * nteams), L.total, st, a, fa_bytes, ft_bytes);
    return true;
  };
  // side-by-side teams only without probe step (which couples every
  // position) and for one tile of kept coefficients per axis (two tiles need
  // more registers than two waves per SIMD leave); else one team
  if constexpr (MT == 1) {
    if (!a.probe_step && a.J <= kSeqLevelMaxJ &&
        (a.n % 16 == 0 ? launch(k_pie_sequential_lds<PR, MT, true, 2>, 2)
                       : launch(k_pie_sequential_lds<PR, MT, false, 2>, 2)))
      return true;
  }
  return a.n % 16 == 0 ? launch(k_pie_sequential_lds<PR, MT, true, 1>, 1)
                       : launch(k_pie_sequential_lds<PR, MT, false, 1>, 1);
}

template <class PR, int MT>
void sequential_prec(const PieArgs& a, hipStream_t st) {
  if (a.n % 16 == 0)
    hipLaunchKernelGGL((k_pie_sequential<PR, MT, true>), dim3(1), dim3(64 * kSeqWaves), 0, st, a);
  else
    hipLaunchKernelGGL((k_pie_sequential<PR, MT, false>), dim3(1), dim3(64 * kSeqWaves), 0, st, a);
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
bool sequential_lds_dense(const PieArgs& a, size_t fa_bytes, size_t ft_bytes, hipStream_t st) {
  switch (a.mt) {
    case 1: return sequential_lds_prec<PR, 1>(a, fa_bytes, ft_bytes, st);
    case 2: return sequential_lds_prec<PR, 2>(a, fa_bytes, ft_bytes, st);
    default: return false;
  }
}

template <class PR>
void sequential_dense(const PieArgs& a, hipStream_t st) {
  switch (a.mt) {
    case 1: sequential_prec<PR, 1>(a, st); break;
    case 2: sequential_prec<PR, 2>(a, st); break;
    default: break;
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
