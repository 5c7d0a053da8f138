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

template <class PR>
struct SplitOp {
  typename PR::V reh, rel, imh, iml;
};

template <class PR>
__device__ __forceinline__ typename PR::V pack4(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  return __builtin_bit_cast(typename PR::V, (u32x4){w0, w1, w2, w3});
}

// Split operands of the two product variants of 4 complex values x:
//   CONJ = false (x * F):        re (xr, -xi)   im (xi, xr)
//   CONJ = true  (x * conj(F)):  re (xr, xi)    im (xi, -xr)
// hi = RNE(v), lo = RNE(v - hi) per value (v - hi is exact in float).  Both
// variants hold the same two numbers per dword, swapped and with one sign
// flipped, and RNE(-v) = -RNE(v): one conversion per (xr, xi) pair, then a
// 16-bit rotate and a sign-bit xor give the variants.
__device__ __forceinline__ uint32_t swap16(uint32_t p) { return __builtin_amdgcn_alignbit(p, p, 16); }
template <class PR, bool CONJ>
__device__ __forceinline__ SplitOp<PR> split_c4(const c4& x) {
  constexpr uint32_t kHiSign = 0x80000000u;
  uint32_t rh[4], ih[4], rl[4], il[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float xr = x.v[s].x, xi = x.v[s].y;
    const uint32_t h = PR::pk(xr, xi);
    const uint32_t l = PR::pk(xr - PR::lo(h), xi - PR::hi(h));
    if constexpr (!CONJ) {
      rh[s] = h ^ kHiSign;
      ih[s] = swap16(h);
      rl[s] = l ^ kHiSign;
      il[s] = swap16(l);
    } else {
      rh[s] = h;
      ih[s] = swap16(h) ^ kHiSign;
      rl[s] = l;
      il[s] = swap16(l) ^ kHiSign;
    }
  }
  SplitOp<PR> o;
  o.reh = pack4<PR>(rh[0], rh[1], rh[2], rh[3]);
  o.imh = pack4<PR>(ih[0], ih[1], ih[2], ih[3]);
  o.rel = pack4<PR>(rl[0], rl[1], rl[2], rl[3]);
  o.iml = pack4<PR>(il[0], il[1], il[2], il[3]);
  return o;
}

// 4 complex values from the re / im accumulator quads.
__device__ __forceinline__ c4 c4_of(const f32x4& re, const f32x4& im) {
  c4 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.v[i] = make_float2(re[i], im[i]);
  return r;
}

// Forward, split: Y^T tiles [MT][CT] for the wave's CT column tiles, rows
// strips strip0, strip0 + sstep, ...  The wave's patch chunks form one
// sequence q = (strip index) * NB + column block, fetched kSplitRing - 1
// chunks ahead (a chunk is ~400 cycles of products, far shorter than a
// memory round trip); twiddles one chunk ahead.  The operand split of chunk
// q + 1 is issued between the products of chunk q, so the vector ALU work
// runs beside the matrix cores instead of before them.  When NB is a
// multiple of the ring the sequence runs on across strips (no refill at a
// strip start); otherwise the ring restarts per strip.  The ring size must
// be even (twiddle and operand ping-pong).
#ifndef PFTPIE_SPLIT_RING
#define PFTPIE_SPLIT_RING 8
#endif
constexpr int kSplitRing = PFTPIE_SPLIT_RING;
template <class PR, int MT, int CT, class Src, class Tab>
__device__ __forceinline__ void fwd_wave_split_pass(const Src& src, int NB, const Tab& FA, int c2t0,
                                                    f32x4 (&Yre)[MT][CT], f32x4 (&Yim)[MT][CT], int strip0,
                                                    int sstep, int rot) {
  static_assert(kSplitRing % 4 == 0, "ring size must be a multiple of 4");
  // raw exit-wave operands (probe and object values, twice the registers of
  // a formed block) take half the ring depth
  using Raw = typename RawOf<Src>::type;
  constexpr int RING = RawOf<Src>::split ? kSplitRing / 2 : kSplitRing;
  const int lane = lane_id();
  const int r16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      Yre[a][b] = zero4();
      Yim[a][b] = zero4();
    }
  const int nstrips = strip0 < NB ? (NB - strip0 + sstep - 1) / sstep : 0;
  if (nstrips == 0) return;
  f32x4 Tre[CT], Tim[CT];
  auto products = [&](const SplitOp<PR>& op, const TwS<PR>(&f)[CT]) {
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
  // stage 2 (transposed): Y^T[c2][c1] += sum_{k1 in strip} T[k1][c2] F[c1][k1]
  auto stage2 = [&](int strip) {
    TwS<PR> fb[MT];
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) fb[c1t] = FA.template s16<PR>((size_t)c1t * NB + strip, lane);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const SplitOp<PR> op = split_c4<PR, false>(c4_of(Tre[ct], Tim[ct]));
#pragma unroll
      for (int c1t = 0; c1t < MT; ++c1t) {
        Yre[c1t][ct] = PR::mfma(op.reh, fb[c1t].h, Yre[c1t][ct]);
        Yim[c1t][ct] = PR::mfma(op.imh, fb[c1t].h, Yim[c1t][ct]);
        Yre[c1t][ct] = PR::mfma(op.reh, fb[c1t].l, Yre[c1t][ct]);
        Yim[c1t][ct] = PR::mfma(op.imh, fb[c1t].l, Yim[c1t][ct]);
        Yre[c1t][ct] = PR::mfma(op.rel, fb[c1t].h, Yre[c1t][ct]);
        Yim[c1t][ct] = PR::mfma(op.iml, fb[c1t].h, Yim[c1t][ct]);
      }
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      Tre[ct] = zero4();
      Tim[ct] = zero4();
    }
  };
  Raw a[RING];
  TwS<PR> f[2][CT];
  SplitOp<PR> op[2];
  // one chunk step of a ring turn starting at chunk q0 (q0 % RING == 0 within
  // the sequence the loaders index): request chunk q0 + u + RING - 1 and the
  // next twiddles, split chunk q0 + u + 1, multiply chunk q0 + u
  auto run = [&](auto load_a, auto load_f, int q0, int u) {
    a[(u + RING - 1) % RING] = load_a(q0 + u + RING - 1);
    load_f(q0 + u + 1, f[(u + 1) & 1]);
    __builtin_amdgcn_sched_barrier(0);
    op[(u + 1) & 1] = split_c4<PR, false>(combine(src, a[(u + 1) % RING]));
    products(op[u & 1], f[u & 1]);
    // one wave per SIMD: its vector work overlaps the matrix products only
    // when issued between them, so the scheduler alternates one product
    // with two vector instructions of the next chunk's split
#pragma unroll
    for (int k = 0; k < 6 * CT; ++k) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
    }
  };
  auto start = [&](auto load_a, auto load_f) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      Tre[ct] = zero4();
      Tim[ct] = zero4();
    }
#pragma unroll
    for (int u = 0; u < RING - 1; ++u) a[u] = load_a(u);
    load_f(0, f[0]);
    op[0] = split_c4<PR, false>(combine(src, a[0]));
  };
  if (NB % RING == 0) {
    // one sequence over all the wave's strips; whole ring turns carry no
    // guard (a guarded load makes the wait-count analysis assume the loads
    // after it were skipped and drain the ring every turn)
    // column blocks in the order rot, rot + 1, ... (mod NB): waves that start
    // at different offsets of their patches spread over the memory channels
    // The loaders take chunk offsets q < 2 RING <= NB from the start of the
    // current ring turn (strip tj, column block tk), so a chunk is at most
    // one strip ahead: no division per chunk.
    int tj = 0, tk = 0;
    auto chunk = [&](int q, int& j, int& k) {
      j = tj;
      k = tk + q;
      if (k >= NB) {
        k -= NB;
        ++j;
      }
      if (j >= nstrips) {  // past the wave's last chunk: reload it
        j = nstrips - 1;
        k = NB - 1;
      }
      k += rot;
      k = k < NB ? k : k - NB;
    };
    auto load_a = [&](int q) {
      int j, k;
      chunk(q, j, k);
      return load_raw(src, (strip0 + j * sstep) * 16 + r16, k * 16 + 4 * g);
    };
    auto load_f = [&](int q, TwS<PR>(&fr)[CT]) {
      int j, k;
      chunk(q, j, k);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) fr[ct] = FA.template s16<PR>((size_t)(c2t0 + ct) * NB + k, lane);
    };
    start(load_a, load_f);
    for (int j = 0; j < nstrips; ++j) {
      for (int k0 = 0; k0 < NB; k0 += RING) {
        tj = j;
        tk = k0;
#pragma unroll
        for (int u = 0; u < RING; ++u) run(load_a, load_f, 0, u);
      }
      stage2(strip0 + j * sstep);
    }
  } else {
    for (int strip = strip0; strip < NB; strip += sstep) {
      const int row = strip * 16 + r16;
      auto load_a = [&](int kb) { return load_raw(src, row, (kb < NB ? kb : NB - 1) * 16 + 4 * g); };
      auto load_f = [&](int kb, TwS<PR>(&fr)[CT]) {
        const int k = kb < NB ? kb : NB - 1;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) fr[ct] = FA.template s16<PR>((size_t)(c2t0 + ct) * NB + k, lane);
      };
      start(load_a, load_f);
      int kb = 0;
      for (; kb + RING <= NB; kb += RING) {
#pragma unroll
        for (int u = 0; u < RING; ++u) run(load_a, load_f, kb, u);
      }
      if (kb < NB) {
#pragma unroll
        for (int u = 0; u < RING; ++u)
          if (kb + u < NB) run(load_a, load_f, kb, u);
      }
      stage2(strip);
    }
  }
}

// ---------------------------------------------------------------------------
// FP16 range guard.  FP16 holds magnitudes up to 65504: an operand component,
// or a component of the stage-1 intermediate (T in the forward, S in the
// adjoint), beyond it turns into inf when it is split, and the products then
// leave non-finite accumulators.  The engines detect that (a wave vote over
// the accumulators, before anything is stored), find the largest operand
// component c of the wave's input, and run the work again on the input
// times s = 2^e, the largest power of two with 2 K c s <= 2^15, where K is
// the length of a stage-1 sum (each intermediate component is a sum of K
// products with |Re|, |Im| <= 2 c |F| = 2 c).  The results are then
// multiplied by 1/s.  Both scalings are exact (they move exponents only), so
// a rescued patch carries the same relative error as any other.  BF16 has
// the FP32 exponent range and needs no guard.
template <class PR>
constexpr bool kRangeGuard = std::is_same<PR, PrecF16>::value;

constexpr float kF16Max = 65504.f;

// s = 2^e, the largest power of two with 2 K c s <= 2^15; 0 when c is not
// finite (an inf or NaN input has nothing to rescue).
__device__ __forceinline__ float guard_scale(float c, int K) {
  if (!(c <= 3.0e38f)) return 0.f;
  if (c == 0.f) return 1.f;
  int e;
  (void)frexpf(32768.f / (2.f * (float)K * c), &e);
  return ldexpf(1.f, e - 1);
}

__device__ __forceinline__ float absmax_c4(float acc, const c4& v) {
#pragma unroll
  for (int i = 0; i < 4; ++i) acc = fmaxf(acc, fmaxf(fabsf(v.v[i].x), fabsf(v.v[i].y)));
  return acc;
}

// True on every lane when some lane holds a component outside [-lim, lim]
// or a NaN.
template <int N>
__device__ __forceinline__ bool wave_any_beyond(const f32x4 (&re)[N], const f32x4 (&im)[N], float lim) {
  float mx = 0.f;
  int bad = 0;
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      mx = fmaxf(mx, fmaxf(fabsf(re[a][i]), fabsf(im[a][i])));
      bad |= (re[a][i] != re[a][i]) | (im[a][i] != im[a][i]);
    }
  return __ballot(bad || !(mx <= lim)) != 0;
}

// Operand source whose values are multiplied by k (a power of two).
template <class Src>
struct ScaledSrc {
  using Raw = typename RawOf<Src>::type;
  Src s;
  float k;
  __device__ __forceinline__ Raw load_raw(int row, int col0) const { return ::pftpie::load_raw(s, row, col0); }
  __device__ __forceinline__ c4 combine(const Raw& r) const {
    c4 z = ::pftpie::combine(s, r);
#pragma unroll
    for (int i = 0; i < 4; ++i) z.v[i] = make_float2(z.v[i].x * k, z.v[i].y * k);
    return z;
  }
  __device__ __forceinline__ c4 load(int row, int col0) const { return combine(load_raw(row, col0)); }
};

// Forward, split: fwd_wave_split_pass, and for FP16 the range guard over the
// wave's strips (K = NB * 16 terms per stage-1 sum).
template <class PR, int MT, int CT, class Src, class Tab>
__device__ __forceinline__ void fwd_wave_split(const Src& src, int NB, const Tab& FA, int c2t0,
                                               f32x4 (&Yre)[MT][CT], f32x4 (&Yim)[MT][CT], int strip0 = 0,
                                               int sstep = 1, int rot = 0) {
  fwd_wave_split_pass<PR, MT, CT>(src, NB, FA, c2t0, Yre, Yim, strip0, sstep, rot);
  if constexpr (kRangeGuard<PR>) {
    f32x4 fr[MT * CT], fi[MT * CT];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int b = 0; b < CT; ++b) {
        fr[a * CT + b] = Yre[a][b];
        fi[a * CT + b] = Yim[a][b];
      }
    if (wave_any_beyond(fr, fi, 3.0e38f)) {
      const int lane = lane_id();
      const int r16 = lane & 15, g = lane >> 4;
      float c = 0.f;
      for (int strip = strip0; strip < NB; strip += sstep)
        for (int kb = 0; kb < NB; ++kb) {
          const int row = strip * 16 + r16, col0 = kb * 16 + 4 * g;
          c = absmax_c4(c, combine(src, load_raw(src, row, col0)));
        }
      const float sc = guard_scale(wave_max(c), NB * 16);
      if (sc > 0.f) {
        const ScaledSrc<Src> scaled{src, sc};
        fwd_wave_split_pass<PR, MT, CT>(scaled, NB, FA, c2t0, Yre, Yim, strip0, sstep, rot);
        const float inv = 1.f / sc;
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
          for (int b = 0; b < CT; ++b) {
            Yre[a][b] *= inv;
            Yim[a][b] *= inv;
          }
      }
    }
  }
}

// Split adjoint, stage 2 (transposed) of column tile kt2 from the split
// stage-1 operands: X^T[k2][k1] = sum_c1 S[c1][k2] conj(F[c1][k1]), two row
// tiles at a time with ping-pong twiddle fetches; sink.put<true> receives
// the X^T tiles.
template <class PR, int MT, class Sink, class Tab>
__device__ __forceinline__ void adj_stage2_split(const SplitOp<PR> (&ops)[MT], int NB, const Tab& FT, int kt2,
                                                 Sink& sink, float inv = 1.f) {
  const int lane = lane_id();
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
    if (inv != 1.f) {  // range-guarded input (FP16): undo its scale
      Xre0 *= inv;
      Xim0 *= inv;
      Xre1 *= inv;
      Xim1 *= inv;
    }
    sink.template put<true>(k1t, kt2, Xre0, Xim0);
    if (two) sink.template put<true>(k1t + 1, kt2, Xre1, Xim1);
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
  // stage 1: S[c1][k2] = sum_c2 Y[c1][c2] conj(F[c2][k2]); coefficient
  // chunks of the next column block are fetched while this block's products
  // issue (ping-pong for MT <= 4)
  auto stage1 = [&](const TwS<PR>& f, const c4(&y)[MT]) {
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) {
      const SplitOp<PR> op = split_c4<PR, true>(y[c1t]);
      Sre[c1t] = PR::mfma(op.reh, f.h, Sre[c1t]);
      Sim[c1t] = PR::mfma(op.imh, f.h, Sim[c1t]);
      Sre[c1t] = PR::mfma(op.reh, f.l, Sre[c1t]);
      Sim[c1t] = PR::mfma(op.imh, f.l, Sim[c1t]);
      Sre[c1t] = PR::mfma(op.rel, f.h, Sre[c1t]);
      Sim[c1t] = PR::mfma(op.iml, f.h, Sim[c1t]);
    }
  };
  auto fetch1 = [&](int kb, TwS<PR>& f, c4(&y)[MT]) {
    f = FT.template s16<PR>((size_t)kt2 * MT + kb, lane);
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) y[c1t] = ysrc.load(c1t * 16 + r16, kb * 16 + 4 * g);
  };
  if constexpr (MT <= 4) {
    TwS<PR> f[2];
    c4 y[2][MT];
    fetch1(0, f[0], y[0]);
#pragma unroll
    for (int kb = 0; kb < MT; ++kb) {
      if (kb + 1 < MT) fetch1(kb + 1, f[(kb + 1) & 1], y[(kb + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);
      stage1(f[kb & 1], y[kb & 1]);
    }
  } else {
#pragma unroll
    for (int kb = 0; kb < MT; ++kb) {
      TwS<PR> f;
      c4 y[MT];
      fetch1(kb, f, y);
      stage1(f, y);
    }
  }
  float inv = 1.f;
  if constexpr (kRangeGuard<PR>) {
    // S is split next: every component must fit FP16 (an inf or NaN here
    // also reports an input component beyond it)
    if (wave_any_beyond(Sre, Sim, kF16Max)) {
      float c = 0.f;
      for (int kb = 0; kb < MT; ++kb)
        for (int c1t = 0; c1t < MT; ++c1t) c = absmax_c4(c, ysrc.load(c1t * 16 + r16, kb * 16 + 4 * g));
      const float sc = guard_scale(wave_max(c), MT * 16);
      if (sc > 0.f) {
#pragma unroll
        for (int a = 0; a < MT; ++a) {
          Sre[a] = zero4();
          Sim[a] = zero4();
        }
        for (int kb = 0; kb < MT; ++kb) {
          const TwS<PR> f = FT.template s16<PR>((size_t)kt2 * MT + kb, lane);
          c4 y[MT];
#pragma unroll
          for (int c1t = 0; c1t < MT; ++c1t) {
            const c4 v = ysrc.load(c1t * 16 + r16, kb * 16 + 4 * g);
#pragma unroll
            for (int i = 0; i < 4; ++i) y[c1t].v[i] = make_float2(v.v[i].x * sc, v.v[i].y * sc);
          }
          stage1(f, y);
        }
        inv = 1.f / sc;
      }
    }
  }
  // stage-2 operands from the accumulators: S^T rows (k2) x c1, times conj(F)
  SplitOp<PR> ops[MT];
#pragma unroll
  for (int c1t = 0; c1t < MT; ++c1t) {
    ops[c1t] = split_c4<PR, true>(c4_of(Sre[c1t], Sim[c1t]));
  }
  adj_stage2_split<PR, MT>(ops, NB, FT, kt2, sink, inv);
}

// ---------------------------------------------------------------------------
// Split adjoint, one whole patch per wave (MT <= 4): the m x m coefficients
// are loaded and split once (MT * MT operands, 256 registers at MT = 4) and
// serve every column tile kt2, so the wave issues no memory loads between
// its output stores and the stage-1 operand split is not repeated per tile.
template <class PR, int MT, class YSrc, class Sink, class Tab>
__device__ __forceinline__ void adj_patch_split(const YSrc& ysrc, int NB, const Tab& FT, Sink& sink, int kt_first = 0,
                                                int kt_step = 1) {
  static_assert(MT <= 4, "the split coefficients of larger windows do not fit in registers");
  const int lane = lane_id();
  const int r16 = lane & 15, g = lane >> 4;
  SplitOp<PR> ys[MT][MT];  // [column block kb][row tile c1t]
  float cmax = 0.f;
#pragma unroll
  for (int kb = 0; kb < MT; ++kb)
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) {
      const c4 v = ysrc.load(c1t * 16 + r16, kb * 16 + 4 * g);
      if constexpr (kRangeGuard<PR>) cmax = absmax_c4(cmax, v);
      ys[kb][c1t] = split_c4<PR, true>(v);
    }
  float inv = 1.f;
  if constexpr (kRangeGuard<PR>) {
    // every S component is bounded by 2 (MT 16) cmax: scale the coefficients
    // down when that bound passes 2^15 (never for data of ordinary range)
    const float sc = guard_scale(wave_max(cmax), MT * 16);
    if (sc > 0.f && sc < 1.f) {
#pragma unroll
      for (int kb = 0; kb < MT; ++kb)
#pragma unroll
        for (int c1t = 0; c1t < MT; ++c1t) {
          const c4 v = ysrc.load(c1t * 16 + r16, kb * 16 + 4 * g);
          c4 w;
#pragma unroll
          for (int i = 0; i < 4; ++i) w.v[i] = make_float2(v.v[i].x * sc, v.v[i].y * sc);
          ys[kb][c1t] = split_c4<PR, true>(w);
        }
      inv = 1.f / sc;
    }
  }
  // column tiles kt_first, kt_first + kt_step, ... (several waves may share
  // a window)
  for (int kt2 = kt_first; kt2 < NB; kt2 += kt_step) {
    // stage 1: S[c1][k2] = sum_c2 Y[c1][c2] conj(F[c2][k2]) for this tile
    f32x4 Sre[MT], Sim[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      Sre[a] = zero4();
      Sim[a] = zero4();
    }
    TwS<PR> f[2];
    f[0] = FT.template s16<PR>((size_t)kt2 * MT, lane);
#pragma unroll
    for (int kb = 0; kb < MT; ++kb) {
      if (kb + 1 < MT) f[(kb + 1) & 1] = FT.template s16<PR>((size_t)kt2 * MT + kb + 1, lane);
      const TwS<PR>& fc = f[kb & 1];
#pragma unroll
      for (int c1t = 0; c1t < MT; ++c1t) {
        const SplitOp<PR>& op = ys[kb][c1t];
        Sre[c1t] = PR::mfma(op.reh, fc.h, Sre[c1t]);
        Sim[c1t] = PR::mfma(op.imh, fc.h, Sim[c1t]);
        Sre[c1t] = PR::mfma(op.reh, fc.l, Sre[c1t]);
        Sim[c1t] = PR::mfma(op.imh, fc.l, Sim[c1t]);
        Sre[c1t] = PR::mfma(op.rel, fc.h, Sre[c1t]);
        Sim[c1t] = PR::mfma(op.iml, fc.h, Sim[c1t]);
      }
    }
    SplitOp<PR> ops[MT];
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) ops[c1t] = split_c4<PR, true>(c4_of(Sre[c1t], Sim[c1t]));
    adj_stage2_split<PR, MT>(ops, NB, FT, kt2, sink, inv);
  }
}

// precision-generic entry points used by the kernels

template <class PR, int MT, int CT, class Src, class Tab>
__device__ __forceinline__ void fwd_engine(const Src& src, int NB, const Tab& FA, int c2t0,
                                           f32x4 (&Yre)[MT][CT], f32x4 (&Yim)[MT][CT], int strip0 = 0,
                                           int sstep = 1, int rot = 0) {
  if constexpr (Orient<PR>::TR)
    fwd_wave_split<PR, MT, CT>(src, NB, FA, c2t0, Yre, Yim, strip0, sstep, rot);
  else
    fwd_wave<MT, CT>(src, NB, FA, c2t0, Yre, Yim, strip0, sstep);
}

template <class PR, int MT, class YSrc, class Sink, class Tab, int K1 = 2>
__device__ __forceinline__ void adj_engine(const YSrc& ysrc, int NB, const Tab& FT, int kt2, Sink& sink) {
  if constexpr (Orient<PR>::TR)
    adj_wave_tile_split<PR, MT>(ysrc, NB, FT, kt2, sink);
  else
    adj_wave_tile<MT, YSrc, Sink, Tab, K1>(ysrc, NB, FT, kt2, sink);
}

template <class Tab>
__device__ __forceinline__ Tab tab_global(const void* p) {
  return Tab{static_cast<const char*>(p)};
}

}  // namespace pftpie
