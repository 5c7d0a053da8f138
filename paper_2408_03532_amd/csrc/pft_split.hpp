// Split-precision (hi + lo in bf16 or fp16, FP32 accumulation) wave engines
// of the partial DFT and its adjoint, and the precision-generic entry points
// the kernels call.
//
// Complex products as real 16 x 16 x 32 MFMAs: each lane group carries 4
// complex values as (re, im) pairs along K.  With B = F in natural (re, im)
// order, a product x * F is
//   re: A = (xr, -xi) . B      im: A = (xi, xr) . B
// and x * conj(F) is
//   re: A = (xr, xi) . B       im: A = (xi, -xr) . B
// so only the variable operand is rearranged (in registers, once per block)
// and one twiddle table per direction serves both stages.
//
// Stage 2 is computed transposed (Y^T = T^T F^T, X^T = S^T conj(F)^T): the
// stage-1 accumulators (rows 4*(l/16) + i, column l % 16) are then exactly
// the A operand of stage 2, so nothing goes through LDS.  The finished tiles
// come out transposed: element i of lane l is (row 16 t_r + l % 16,
// column 16 t_c + 4 (l/16) + i); tile_rc<true> gives those coordinates.
//
// Split twiddle tables (same block grid as the FP32 FA / FT tables, 2 KB per
// block): plane 0 = hi parts, plane 1 = lo parts, 8 16-bit values per lane:
//   FA block (ct, kb), lane l: F[16 ct + l%16][16 kb + 4(l/16) + s], s = 0..3
//   FT block (kt, cb), lane l: F[16 cb + 4(l/16) + s][16 kt + l%16]
#pragma once

#include "device_common.hpp"
#include "pft_engine.hpp"

namespace pftpie {

struct PrecF32 {};

template <class PR>
struct Orient {
  static constexpr bool TR = true;
};
template <>
struct Orient<PrecF32> {
  static constexpr bool TR = false;
};

// (row, col) of element i of lane `lane` in tile (tr, tc).
template <bool TR>
__device__ __forceinline__ int2 tile_rc(int tr, int tc, int i, int lane) {
  const int r16 = lane & 15, g = lane >> 4;
  return TR ? make_int2(tr * 16 + r16, tc * 16 + 4 * g + i) : make_int2(tr * 16 + 4 * g + i, tc * 16 + r16);
}

// 8 floats (re, im interleaved) of a c4 chunk in the two product variants.
__device__ __forceinline__ void variants_mul(const c4& a, float (&re)[8], float (&im)[8]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    re[2 * s] = a.v[s].x;
    re[2 * s + 1] = -a.v[s].y;
    im[2 * s] = a.v[s].y;
    im[2 * s + 1] = a.v[s].x;
  }
}
__device__ __forceinline__ void variants_mulconj(const c4& a, float (&re)[8], float (&im)[8]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    re[2 * s] = a.v[s].x;
    re[2 * s + 1] = a.v[s].y;
    im[2 * s] = a.v[s].y;
    im[2 * s + 1] = -a.v[s].x;
  }
}

template <class PR>
struct SplitOp {
  typename PR::V reh, rel, imh, iml;
};

template <class PR>
__device__ __forceinline__ SplitOp<PR> make_op(const float (&re)[8], const float (&im)[8]) {
  SplitOp<PR> o;
  split8<PR>(re, o.reh, o.rel);
  split8<PR>(im, o.imh, o.iml);
  return o;
}

// Forward, split: Y^T tiles [MT][CT] for the wave's CT column tiles.  The
// patch chunks are fetched three blocks ahead (a 16x16x32 MFMA block is only
// ~200 cycles of work, far shorter than a memory round trip); twiddles one
// block ahead.
template <class PR, int MT, int CT, class Src, class Tab>
__device__ __forceinline__ void fwd_wave_split(const Src& src, int NB, const Tab& FA, int c2t0,
                                               f32x4 (&Yre)[MT][CT], f32x4 (&Yim)[MT][CT], int strip0 = 0,
                                               int sstep = 1) {
  const int lane = lane_id();
  const int r16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      Yre[a][b] = zero4();
      Yim[a][b] = zero4();
    }
  for (int strip = strip0; strip < NB; strip += sstep) {
    const int row = strip * 16 + r16;
    f32x4 Tre[CT], Tim[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      Tre[ct] = zero4();
      Tim[ct] = zero4();
    }
    auto stage1 = [&](const c4& a, const TwS<PR>(&f)[CT]) {
      float re[8], im[8];
      variants_mul(a, re, im);
      const SplitOp<PR> op = make_op<PR>(re, im);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        Tre[ct] = PR::mfma(op.reh, f[ct].h, Tre[ct]);
        Tim[ct] = PR::mfma(op.imh, f[ct].h, Tim[ct]);
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        Tre[ct] = PR::mfma(op.reh, f[ct].l, Tre[ct]);
        Tim[ct] = PR::mfma(op.imh, f[ct].l, Tim[ct]);
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        Tre[ct] = PR::mfma(op.rel, f[ct].h, Tre[ct]);
        Tim[ct] = PR::mfma(op.iml, f[ct].h, Tim[ct]);
      }
    };
    auto load_a = [&](int kb) { return src.load(row, (kb < NB ? kb : NB - 1) * 16 + 4 * g); };
    auto load_f = [&](int kb, TwS<PR>(&f)[CT]) {
      const int k = kb < NB ? kb : NB - 1;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) f[ct] = FA.template s16<PR>((size_t)(c2t0 + ct) * NB + k, lane);
    };
    c4 a[4];
    TwS<PR> f[2][CT];
    a[0] = load_a(0);
    a[1] = load_a(1);
    a[2] = load_a(2);
    load_f(0, f[0]);
    for (int kb = 0; kb < NB; kb += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (kb + u < NB) {
          a[(u + 3) & 3] = load_a(kb + u + 3);
          load_f(kb + u + 1, f[(u + 1) & 1]);
          __builtin_amdgcn_sched_barrier(0);
          stage1(a[u], f[u & 1]);
        }
      }
    }
    // stage 2 (transposed): Y^T[c2][c1] += sum_{k1 in strip} T[k1][c2] F[c1][k1]
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      float re[8], im[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        re[2 * i] = Tre[ct][i];
        re[2 * i + 1] = -Tim[ct][i];
        im[2 * i] = Tim[ct][i];
        im[2 * i + 1] = Tre[ct][i];
      }
      const SplitOp<PR> op = make_op<PR>(re, im);
#pragma unroll
      for (int c1t = 0; c1t < MT; ++c1t) {
        const TwS<PR> fb = FA.template s16<PR>((size_t)c1t * NB + strip, lane);
        Yre[c1t][ct] = PR::mfma(op.reh, fb.h, Yre[c1t][ct]);
        Yim[c1t][ct] = PR::mfma(op.imh, fb.h, Yim[c1t][ct]);
        Yre[c1t][ct] = PR::mfma(op.reh, fb.l, Yre[c1t][ct]);
        Yim[c1t][ct] = PR::mfma(op.imh, fb.l, Yim[c1t][ct]);
        Yre[c1t][ct] = PR::mfma(op.rel, fb.h, Yre[c1t][ct]);
        Yim[c1t][ct] = PR::mfma(op.iml, fb.h, Yim[c1t][ct]);
      }
    }
  }
}

// Adjoint, split, one column tile kt2: sink.put<true> receives X^T tiles.
template <class PR, int MT, class YSrc, class Sink, class Tab>
__device__ __forceinline__ void adj_wave_tile_split(const YSrc& ysrc, int NB, const Tab& FT, int kt2,
                                                    Sink& sink) {
  const int lane = lane_id();
  const int r16 = lane & 15, g = lane >> 4;
  f32x4 Sre[MT], Sim[MT];
#pragma unroll
  for (int a = 0; a < MT; ++a) {
    Sre[a] = zero4();
    Sim[a] = zero4();
  }
  // stage 1: S[c1][k2] = sum_c2 Y[c1][c2] conj(F[c2][k2])
#pragma unroll
  for (int kb = 0; kb < MT; ++kb) {
    const TwS<PR> f = FT.template s16<PR>((size_t)kt2 * MT + kb, lane);
    c4 y[MT];
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) y[c1t] = ysrc.load(c1t * 16 + r16, kb * 16 + 4 * g);
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) {
      float re[8], im[8];
      variants_mulconj(y[c1t], re, im);
      const SplitOp<PR> op = make_op<PR>(re, im);
      Sre[c1t] = PR::mfma(op.reh, f.h, Sre[c1t]);
      Sim[c1t] = PR::mfma(op.imh, f.h, Sim[c1t]);
      Sre[c1t] = PR::mfma(op.reh, f.l, Sre[c1t]);
      Sim[c1t] = PR::mfma(op.imh, f.l, Sim[c1t]);
      Sre[c1t] = PR::mfma(op.rel, f.h, Sre[c1t]);
      Sim[c1t] = PR::mfma(op.iml, f.h, Sim[c1t]);
    }
  }
  // stage-2 operands from the accumulators: S^T rows (k2) x c1, times conj(F)
  SplitOp<PR> ops[MT];
#pragma unroll
  for (int c1t = 0; c1t < MT; ++c1t) {
    float re[8], im[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      re[2 * i] = Sre[c1t][i];
      re[2 * i + 1] = Sim[c1t][i];
      im[2 * i] = Sim[c1t][i];
      im[2 * i + 1] = -Sre[c1t][i];
    }
    ops[c1t] = make_op<PR>(re, im);
  }
  // stage 2 (transposed): X^T[k2][k1] = sum_c1 S[c1][k2] conj(F[c1][k1]),
  // two row tiles at a time, ping-pong twiddle fetches
  auto fetch2 = [&](int k1t, int c1t, TwS<PR>& fa, TwS<PR>& fb) {
    const int k1b = (k1t + 1 < NB) ? k1t + 1 : k1t;
    fa = FT.template s16<PR>((size_t)k1t * MT + c1t, lane);
    fb = FT.template s16<PR>((size_t)k1b * MT + c1t, lane);
  };
  TwS<PR> fa[2], fb[2];
  fetch2(0, 0, fa[0], fb[0]);
  for (int k1t = 0; k1t < NB; k1t += 2) {
    const bool two = (k1t + 1 < NB);
    const int k1n = (k1t + 2 < NB) ? k1t + 2 : k1t;
    f32x4 Xre0 = zero4(), Xim0 = zero4(), Xre1 = zero4(), Xim1 = zero4();
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) {
      const int cur = c1t & 1;
      if (c1t + 1 < MT)
        fetch2(k1t, c1t + 1, fa[cur ^ 1], fb[cur ^ 1]);
      else if ((MT & 1) == 0)
        fetch2(k1n, 0, fa[cur ^ 1], fb[cur ^ 1]);
      __builtin_amdgcn_sched_barrier(0);
      const SplitOp<PR>& o = ops[c1t];
      Xre0 = PR::mfma(o.reh, fa[cur].h, Xre0);
      Xim0 = PR::mfma(o.imh, fa[cur].h, Xim0);
      Xre1 = PR::mfma(o.reh, fb[cur].h, Xre1);
      Xim1 = PR::mfma(o.imh, fb[cur].h, Xim1);
      Xre0 = PR::mfma(o.reh, fa[cur].l, Xre0);
      Xim0 = PR::mfma(o.imh, fa[cur].l, Xim0);
      Xre1 = PR::mfma(o.reh, fb[cur].l, Xre1);
      Xim1 = PR::mfma(o.imh, fb[cur].l, Xim1);
      Xre0 = PR::mfma(o.rel, fa[cur].h, Xre0);
      Xim0 = PR::mfma(o.iml, fa[cur].h, Xim0);
      Xre1 = PR::mfma(o.rel, fb[cur].h, Xre1);
      Xim1 = PR::mfma(o.iml, fb[cur].h, Xim1);
    }
    if constexpr ((MT & 1) != 0) fetch2(k1n, 0, fa[0], fb[0]);
    sink.template put<true>(k1t, kt2, Xre0, Xim0);
    if (two) sink.template put<true>(k1t + 1, kt2, Xre1, Xim1);
  }
}

// ---------------------------------------------------------------------------
// precision-generic entry points used by the kernels

template <class PR, int MT, int CT, class Src, class Tab>
__device__ __forceinline__ void fwd_engine(const Src& src, int NB, const Tab& FA, int c2t0,
                                           f32x4 (&Yre)[MT][CT], f32x4 (&Yim)[MT][CT], int strip0 = 0,
                                           int sstep = 1) {
  if constexpr (Orient<PR>::TR)
    fwd_wave_split<PR, MT, CT>(src, NB, FA, c2t0, Yre, Yim, strip0, sstep);
  else
    fwd_wave<MT, CT>(src, NB, FA, c2t0, Yre, Yim, strip0, sstep);
}

template <class PR, int MT, class YSrc, class Sink, class Tab>
__device__ __forceinline__ void adj_engine(const YSrc& ysrc, int NB, const Tab& FT, int kt2, Sink& sink) {
  if constexpr (Orient<PR>::TR)
    adj_wave_tile_split<PR, MT>(ysrc, NB, FT, kt2, sink);
  else
    adj_wave_tile<MT>(ysrc, NB, FT, kt2, sink);
}

template <class Tab>
__device__ __forceinline__ Tab tab_global(const void* p) {
  return Tab{static_cast<const char*>(p)};
}

}  // namespace pftpie
