// Wave-level FP32 MFMA engines of the 2-D partial DFT and its adjoint.
//
// Forward   Y = F T,       T = psi F^T       (Appendix A, 2-D DFT restricted
//                                             to the kept window)
// Adjoint   X = F^H S,     S = Y conj(F)^T   (exact adjoint, no scaling)
// with F = F_m the m x n partial DFT matrix.
//
// Forward: one wave owns CT column tiles (16 output columns each) of Y for
// one patch.  It streams psi in 16-row strips; for each strip it contracts
// the strip against F^T over all n columns (stage 1, T strip in MFMA
// accumulators), then immediately contracts F[:, strip] against that T strip
// into its Y accumulators (stage 2).  The accumulator layout of stage 1 is
// the B-operand layout of stage 2, so T never leaves registers.
//
// Adjoint: one wave owns one 16-column tile of X at a time: stage 1 forms
// S[:, tile] = Y conj(F)[:, tile] over the m kept columns, stage 2 emits
// X[row tile, tile] = F^H S for every row tile, handing each finished 16 x 16
// tile to a sink (plain store, or the PIE scatter).
//
// Twiddle tables (built on the host in double, rounded once):
//   FA block (ct, kb), lane l, entry s = F[16 ct + l%16][16 kb + 4(l/16) + s]
//   FT block (kt, cb), lane l, entry s = F[16 cb + 4(l/16) + s][16 kt + l%16]
// zero outside the m x n matrix.  Each block is 2 KB (see load_tw).
#pragma once

#include <type_traits>

#include "device_common.hpp"

namespace pftpie {

// Operand sources may split a load into its memory part (load_raw, whose
// result sits in the prefetch registers) and the arithmetic on it (combine,
// applied just before the block's products), so that a prefetched block is
// not waited for when it is fetched.  Sources without that split (plain
// patches, coefficients) load in full.
template <class S, class = void>
struct RawOf {
  using type = c4;
  static constexpr bool split = false;
};
template <class S>
struct RawOf<S, std::void_t<typename S::Raw>> {
  using type = typename S::Raw;
  static constexpr bool split = true;
};

template <class S>
__device__ __forceinline__ typename RawOf<S>::type load_raw(const S& src, int row, int col0) {
  if constexpr (RawOf<S>::split)
    return src.load_raw(row, col0);
  else
    return src.load(row, col0);
}

template <class S>
__device__ __forceinline__ c4 combine(const S& src, const typename RawOf<S>::type& r) {
  if constexpr (RawOf<S>::split)
    return src.combine(r);
  else
    return r;
}

// psi source of the plain transform: patch p, side n.  EXACT: n % 16 == 0
// and 16-byte aligned base, so every lane chunk is in bounds and aligned.
template <bool EXACT>
struct PlainSrc {
  const float2* __restrict__ p;
  int n;
  __device__ __forceinline__ c4 load(int row, int col0) const {
    c4 r;
    if (EXACT) {
      const float4* q = reinterpret_cast<const float4*>(p + (size_t)row * n + col0);
      float4 a = q[0], b = q[1];
      r.v[0] = make_float2(a.x, a.y);
      r.v[1] = make_float2(a.z, a.w);
      r.v[2] = make_float2(b.x, b.y);
      r.v[3] = make_float2(b.z, b.w);
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        int col = col0 + s;
        r.v[s] = (row < n && col < n) ? p[(size_t)row * n + col] : make_float2(0.f, 0.f);
      }
    }
    return r;
  }
};

// Complex products in three real MFMA products (Gauss): for data a + ib and
// twiddle c + id,
//   k1 = a (c + d),  k2 = d (a + b),  k3 = c (b - a),
//   re = k1 - k2,    im = k1 + k3,
// each k accumulated over the contraction in its own registers.  The two
// data-side sums are formed once per data element (shared by every twiddle
// tile that element meets), c + d once per twiddle element.

// Forward engine, three products per complex product (output blocks of up
// to 8 tiles per wave, whose three accumulator sets fit the registers).
template <int MT, int CT, class Src, class Tab>
__device__ __forceinline__ void fwd_wave_gauss(const Src& src, int NB, const Tab& FA, int c2t0, f32x4 (&Yre)[MT][CT],
                                         f32x4 (&Yim)[MT][CT], int strip0, int sstep, int kb0 = 0, int kbs = 1) {
  const int lane = lane_id();
  const int r16 = lane & 15, g = lane >> 4;
  // Yre accumulates k1, Yim k3, Y2 k2 of the stage-2 products
  f32x4 Y2[MT][CT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      Yre[a][b] = zero4();
      Yim[a][b] = zero4();
      Y2[a][b] = zero4();
    }
  for (int strip = strip0; strip < NB; strip += sstep) {
    const int row = strip * 16 + r16;
    f32x4 T1[CT], T2[CT], T3[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      T1[ct] = zero4();
      T2[ct] = zero4();
      T3[ct] = zero4();
    }
    // stage 1 over column blocks (data psi, twiddle F^T), two register sets
    // in ping-pong so the loads of one block are in flight while the other
    // block's products issue
    using Raw = typename RawOf<Src>::type;
    auto stage1 = [&](const Raw& raw, const c4(&f)[CT]) {
      const c4 a = combine(src, raw);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float ar = a.v[s].x, ai = a.v[s].y;
        const float sab = ar + ai, dba = ai - ar;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const float fr = f[ct].v[s].x, fi = f[ct].v[s].y;
          T1[ct] = mfma4(ar, fr + fi, T1[ct]);
          T2[ct] = mfma4(sab, fi, T2[ct]);
          T3[ct] = mfma4(dba, fr, T3[ct]);
        }
      }
    };
    auto fetch = [&](int kb, Raw& a, c4(&f)[CT]) {
      a = load_raw(src, row, kb * 16 + 4 * g);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) f[ct] = FA.f32((size_t)(c2t0 + ct) * NB + kb, lane);
    };
    Raw a0, a1;
    c4 f0[CT], f1[CT];
    if (kb0 < NB) {
      // column blocks kb0, kb0 + kbs, ... (all of them unless several waves
      // share the strip's sum)
      fetch(kb0, a0, f0);
      int kb = kb0;
      for (; kb + kbs < NB; kb += 2 * kbs) {
        fetch(kb + kbs, a1, f1);
        __builtin_amdgcn_sched_barrier(0);
        stage1(a0, f0);
        fetch(kb + 2 * kbs < NB ? kb + 2 * kbs : kb + kbs, a0, f0);
        __builtin_amdgcn_sched_barrier(0);
        stage1(a1, f1);
      }
      if (kb < NB) stage1(a0, f0);
    }
    // T strip = a + ib with a = k1 - k2, b = k1 + k3; stage 2 takes T as the
    // data side: a in T1, a + b in T2, b - a in T3
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const f32x4 tr = T1[ct] - T2[ct], ti = T1[ct] + T3[ct];
      T1[ct] = tr;
      T2[ct] = tr + ti;
      T3[ct] = ti - tr;
    }
    // stage 2: Y[c1 tile][own tiles] += F[c1 tile, strip] * T[strip, own tiles]
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) {
      c4 fb = FA.f32((size_t)c1t * NB + strip, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float fr = fb.v[i].x, fi = fb.v[i].y, cd = fr + fi;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          Yre[c1t][ct] = mfma4(cd, T1[ct][i], Yre[c1t][ct]);
          Y2[c1t][ct] = mfma4(fi, T2[ct][i], Y2[c1t][ct]);
          Yim[c1t][ct] = mfma4(fr, T3[ct][i], Yim[c1t][ct]);
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      const f32x4 k1 = Yre[a][b];
      Yre[a][b] = k1 - Y2[a][b];
      Yim[a][b] = k1 + Yim[a][b];
    }
}

// Forward engine, four products per complex product (the negated operand
// formed in a register), for wider output blocks.
template <int MT, int CT, class Src, class Tab>
__device__ __forceinline__ void fwd_wave_four(const Src& src, int NB, const Tab& FA, int c2t0, f32x4 (&Yre)[MT][CT],
                                              f32x4 (&Yim)[MT][CT], int strip0, int sstep) {
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
    using Raw = typename RawOf<Src>::type;
    auto stage1 = [&](const Raw& raw, const c4(&f)[CT]) {
      const c4 a = combine(src, raw);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float ar = a.v[s].x, ai = a.v[s].y, nai = -ai;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          Tre[ct] = mfma4(ar, f[ct].v[s].x, Tre[ct]);
          Tim[ct] = mfma4(ar, f[ct].v[s].y, Tim[ct]);
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          Tre[ct] = mfma4(nai, f[ct].v[s].y, Tre[ct]);
          Tim[ct] = mfma4(ai, f[ct].v[s].x, Tim[ct]);
        }
      }
    };
    auto fetch = [&](int kb, Raw& a, c4(&f)[CT]) {
      a = load_raw(src, row, kb * 16 + 4 * g);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) f[ct] = FA.f32((size_t)(c2t0 + ct) * NB + kb, lane);
    };
    Raw a0, a1;
    c4 f0[CT], f1[CT];
    fetch(0, a0, f0);
    int kb = 0;
    for (; kb + 1 < NB; kb += 2) {
      fetch(kb + 1, a1, f1);
      __builtin_amdgcn_sched_barrier(0);
      stage1(a0, f0);
      fetch(kb + 2 < NB ? kb + 2 : kb + 1, a0, f0);
      __builtin_amdgcn_sched_barrier(0);
      stage1(a1, f1);
    }
    if (kb < NB) stage1(a0, f0);
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) {
      c4 fb = FA.f32((size_t)c1t * NB + strip, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float fr = fb.v[i].x, fi = fb.v[i].y, nfi = -fi;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          Yre[c1t][ct] = mfma4(fr, Tre[ct][i], Yre[c1t][ct]);
          Yim[c1t][ct] = mfma4(fr, Tim[ct][i], Yim[c1t][ct]);
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          Yre[c1t][ct] = mfma4(nfi, Tim[ct][i], Yre[c1t][ct]);
          Yim[c1t][ct] = mfma4(fi, Tre[ct][i], Yim[c1t][ct]);
        }
      }
    }
  }
}

// Forward engine.  NB = ceil(n/16) row strips / column blocks.  FA holds
// ctiles x NB blocks.  c2t0: first column tile this wave owns; the wave
// runs strips strip0, strip0 + sstep, ...
// With kbs > 1 (three-product form only) the wave sums column blocks kb0,
// kb0 + kbs, ... only: kbs waves then hold partial results whose sum is the
// transform.  WIDE: three
// products also for up to 16 output tiles (about 440 registers, one wave
// per SIMD; for kernels that run at that occupancy anyway).
template <int MT, int CT, class Src, class Tab, bool WIDE = false>
__device__ __forceinline__ void fwd_wave(const Src& src, int NB, const Tab& FA, int c2t0, f32x4 (&Yre)[MT][CT],
                                         f32x4 (&Yim)[MT][CT], int strip0 = 0, int sstep = 1, int kb0 = 0,
                                         int kbs = 1) {
  if constexpr (MT * CT <= (WIDE ? 16 : 8))
    fwd_wave_gauss<MT, CT>(src, NB, FA, c2t0, Yre, Yim, strip0, sstep, kb0, kbs);
  else
    fwd_wave_four<MT, CT>(src, NB, FA, c2t0, Yre, Yim, strip0, sstep);  // (kbs == 1 only)
}

// Forward engine for long windows whose twiddle table does not stay in the
// caches (n in the thousands): RS row strips per pass share every twiddle
// block fetched, so the table streams NB / RS instead of NB times per wave.
// The wave's strips are strip0, strip0 + sstep, ... taken RS at a time;
// strips past NB in the last pass load rows of the pass's first strip and
// their products are dropped.
template <int MT, int CT, int RS, class Src, class Tab>
__device__ __forceinline__ void fwd_wave_rs(const Src& src, int NB, const Tab& FA, int c2t0, f32x4 (&Yre)[MT][CT],
                                            f32x4 (&Yim)[MT][CT], int strip0, int sstep) {
  const int lane = lane_id();
  const int r16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      Yre[a][b] = zero4();
      Yim[a][b] = zero4();
    }
  for (int base = strip0; base < NB; base += sstep * RS) {
    int rows[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int sr = base + r * sstep;
      rows[r] = (sr < NB ? sr : base) * 16 + r16;
    }
    // stage 1 in three products (Gauss): k1 in T1, k2 in Tre, k3 in Tim
    // until the strip is done
    f32x4 T1[RS][CT], Tre[RS][CT], Tim[RS][CT];
#pragma unroll
    for (int r = 0; r < RS; ++r)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        T1[r][ct] = zero4();
        Tre[r][ct] = zero4();
        Tim[r][ct] = zero4();
      }
    using Raw = typename RawOf<Src>::type;
    auto stage1 = [&](const Raw(&raw)[RS], const c4(&f)[CT]) {
      c4 a[RS];
#pragma unroll
      for (int r = 0; r < RS; ++r) a[r] = combine(src, raw[r]);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        float fs[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) fs[ct] = f[ct].v[s].x + f[ct].v[s].y;
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          const float ar = a[r].v[s].x, ai = a[r].v[s].y, sab = ar + ai, dba = ai - ar;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            T1[r][ct] = mfma4(ar, fs[ct], T1[r][ct]);
            Tre[r][ct] = mfma4(sab, f[ct].v[s].y, Tre[r][ct]);
            Tim[r][ct] = mfma4(dba, f[ct].v[s].x, Tim[r][ct]);
          }
        }
      }
    };
    auto fetch = [&](int kb, Raw(&a)[RS], c4(&f)[CT]) {
#pragma unroll
      for (int r = 0; r < RS; ++r) a[r] = load_raw(src, rows[r], kb * 16 + 4 * g);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) f[ct] = FA.f32((size_t)(c2t0 + ct) * NB + kb, lane);
    };
    Raw a0[RS], a1[RS];
    c4 f0[CT], f1[CT];
    fetch(0, a0, f0);
    int kb = 0;
    for (; kb + 1 < NB; kb += 2) {
      fetch(kb + 1, a1, f1);
      __builtin_amdgcn_sched_barrier(0);
      stage1(a0, f0);
      fetch(kb + 2 < NB ? kb + 2 : kb + 1, a0, f0);
      __builtin_amdgcn_sched_barrier(0);
      stage1(a1, f1);
    }
    if (kb < NB) stage1(a0, f0);
    // T = (k1 - k2) + i (k1 + k3)
#pragma unroll
    for (int r = 0; r < RS; ++r)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        Tre[r][ct] = T1[r][ct] - Tre[r][ct];
        Tim[r][ct] = T1[r][ct] + Tim[r][ct];
      }
    // stage 2 per live strip: Y[c1 tile][own tiles] += F[c1 tile, strip] * T
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int sr = base + r * sstep;
      if (sr >= NB) break;
#pragma unroll
      for (int c1t = 0; c1t < MT; ++c1t) {
        const c4 fb = FA.f32((size_t)c1t * NB + sr, lane);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float fr = fb.v[i].x, fi = fb.v[i].y, nfi = -fi;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            Yre[c1t][ct] = mfma4(fr, Tre[r][ct][i], Yre[c1t][ct]);
            Yim[c1t][ct] = mfma4(fr, Tim[r][ct][i], Yim[c1t][ct]);
          }
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            Yre[c1t][ct] = mfma4(nfi, Tim[r][ct][i], Yre[c1t][ct]);
            Yim[c1t][ct] = mfma4(fi, Tre[r][ct][i], Yim[c1t][ct]);
          }
        }
      }
    }
  }
}

// FP32 adjoint, stage 2 of column tile kt2 from the stage-1 accumulators S,
// four products per complex product.
template <int MT, int K1, class Sink, class Tab>
__device__ __forceinline__ void adj_stage2_four(const f32x4 (&Sre)[MT], const f32x4 (&Sim)[MT], int NB, const Tab& FT,
                                                int kt2, Sink& sink, int k1_first = 0, int k1_step = 1) {
  const int lane = lane_id();
  // stage 2: X[k1][k2] = sum_c1 conj(F[c1][k1]) S[c1][k2], K1 row tiles at a
  // time; the twiddle blocks of the next step are fetched while the current
  // step's products issue (ping-pong buffers, no register copies).
  auto fetch2 = [&](int k1t, int c1t, c4(&f)[K1]) {
#pragma unroll
    for (int u = 0; u < K1; ++u) {
      const int kt = (k1t + u < NB) ? k1t + u : NB - 1;
      f[u] = FT.f32((size_t)kt * MT + c1t, lane);
    }
  };
  c4 fb[2][K1];
  const int k1s = K1 * k1_step;
  fetch2(K1 * k1_first, 0, fb[0]);
  for (int k1t = K1 * k1_first; k1t < NB; k1t += k1s) {
    const int k1n = (k1t + k1s < NB) ? k1t + k1s : k1t;
    f32x4 Xre[K1], Xim[K1];
#pragma unroll
    for (int u = 0; u < K1; ++u) {
      Xre[u] = zero4();
      Xim[u] = zero4();
    }
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) {
      const int cur = c1t & 1;
      if (c1t + 1 < MT)
        fetch2(k1t, c1t + 1, fb[cur ^ 1]);
      else if ((MT & 1) == 0)
        fetch2(k1n, 0, fb[cur ^ 1]);  // cur ^ 1 == 0 here
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float sr = Sre[c1t][i], si = Sim[c1t][i];
#pragma unroll
        for (int u = 0; u < K1; ++u) {
          Xre[u] = mfma4(fb[cur][u].v[i].x, sr, Xre[u]);
          Xim[u] = mfma4(fb[cur][u].v[i].x, si, Xim[u]);
        }
#pragma unroll
        for (int u = 0; u < K1; ++u) {
          Xre[u] = mfma4(fb[cur][u].v[i].y, si, Xre[u]);
          Xim[u] = mfma4(-fb[cur][u].v[i].y, sr, Xim[u]);
        }
      }
    }
    if constexpr ((MT & 1) != 0) fetch2(k1n, 0, fb[0]);
#pragma unroll
    for (int u = 0; u < K1; ++u)
      if (k1t + u < NB) sink.template put<false>(k1t + u, kt2, Xre[u], Xim[u]);
  }
}

// FP32 adjoint, stage 2 of column tile kt2, three products per complex
// product: conj(F) = c + id with c = Re F, d = -Im F, data S = a + ib, so
//   k1 = a (Re F - Im F),  k2' = Im F (a + b),  k3 = Re F (b - a),
//   Re X = k1 + k2',       Im X = k1 + k3
// (k2' = -k2 of the Gauss form).  a + b and b - a are formed once per tile.
template <int MT, int K1, class Sink, class Tab>
__device__ __forceinline__ void adj_stage2_gauss(const f32x4 (&Sre)[MT], const f32x4 (&Sim)[MT], int NB,
                                                 const Tab& FT, int kt2, Sink& sink, int k1_first = 0,
                                                 int k1_step = 1) {
  const int lane = lane_id();
  f32x4 Ssum[MT], Sdif[MT];
#pragma unroll
  for (int c = 0; c < MT; ++c) {
    Ssum[c] = Sre[c] + Sim[c];
    Sdif[c] = Sim[c] - Sre[c];
  }
  auto fetch2 = [&](int k1t, int c1t, c4(&f)[K1]) {
#pragma unroll
    for (int u = 0; u < K1; ++u) {
      const int kt = (k1t + u < NB) ? k1t + u : NB - 1;
      f[u] = FT.f32((size_t)kt * MT + c1t, lane);
    }
  };
  c4 fb[2][K1];
  const int k1s = K1 * k1_step;
  fetch2(K1 * k1_first, 0, fb[0]);
  for (int k1t = K1 * k1_first; k1t < NB; k1t += k1s) {
    const int k1n = (k1t + k1s < NB) ? k1t + k1s : k1t;
    f32x4 X1[K1], X2[K1], X3[K1];
#pragma unroll
    for (int u = 0; u < K1; ++u) {
      X1[u] = zero4();
      X2[u] = zero4();
      X3[u] = zero4();
    }
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) {
      const int cur = c1t & 1;
      if (c1t + 1 < MT)
        fetch2(k1t, c1t + 1, fb[cur ^ 1]);
      else if ((MT & 1) == 0)
        fetch2(k1n, 0, fb[cur ^ 1]);  // cur ^ 1 == 0 here
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int u = 0; u < K1; ++u) {
          const float fr = fb[cur][u].v[i].x, fi = fb[cur][u].v[i].y;
          X1[u] = mfma4(fr - fi, Sre[c1t][i], X1[u]);
          X2[u] = mfma4(fi, Ssum[c1t][i], X2[u]);
          X3[u] = mfma4(fr, Sdif[c1t][i], X3[u]);
        }
      }
    }
    if constexpr ((MT & 1) != 0) fetch2(k1n, 0, fb[0]);
#pragma unroll
    for (int u = 0; u < K1; ++u)
      if (k1t + u < NB) sink.template put<false>(k1t + u, kt2, X1[u] + X2[u], X1[u] + X3[u]);
  }
}

// FP32 adjoint, stage 2 of column tile kt2 from the stage-1 accumulators S.
// Row tiles k1_first * K1, (k1_first + k1_step) * K1, ... (K1 at a time) only
// when several waves share the tile's rows.
template <int MT, int K1, class Sink, class Tab>
__device__ __forceinline__ void adj_stage2_f32(const f32x4 (&Sre)[MT], const f32x4 (&Sim)[MT], int NB, const Tab& FT,
                                               int kt2, Sink& sink, int k1_first = 0, int k1_step = 1) {
  if constexpr (MT <= 4 && K1 <= 2)
    adj_stage2_gauss<MT, K1>(Sre, Sim, NB, FT, kt2, sink, k1_first, k1_step);
  else
    adj_stage2_four<MT, K1>(Sre, Sim, NB, FT, kt2, sink, k1_first, k1_step);
}

// Adjoint engine for one 16-column tile kt2 of X.  ysrc.load(row, col0)
// returns Y[row][col0..col0+3] (zeros outside m x m).  FT holds NB x MT
// blocks.  sink.put<false>(k1t, kt2, Xre, Xim) receives each finished tile.
template <int MT, class YSrc, class Sink, class Tab, int K1 = 2>
__device__ __forceinline__ void adj_wave_tile(const YSrc& ysrc, int NB, const Tab& FT, int kt2, Sink& sink,
                                              int k1_first = 0, int k1_step = 1) {
  const int lane = lane_id();
  const int r16 = lane & 15, g = lane >> 4;
  f32x4 Sre[MT], Sim[MT];
#pragma unroll
  for (int a = 0; a < MT; ++a) {
    Sre[a] = zero4();
    Sim[a] = zero4();
  }
  // stage 1: S[c1][k2 in tile] = sum_c2 Y[c1][c2] conj(F[c2][k2])
  auto stage1 = [&](const c4& f, const c4(&y)[MT]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float fr = f.v[s].x, fi = f.v[s].y;
#pragma unroll
      for (int c1t = 0; c1t < MT; ++c1t) {
        Sre[c1t] = mfma4(y[c1t].v[s].x, fr, Sre[c1t]);
        Sim[c1t] = mfma4(y[c1t].v[s].y, fr, Sim[c1t]);
      }
#pragma unroll
      for (int c1t = 0; c1t < MT; ++c1t) {
        Sre[c1t] = mfma4(y[c1t].v[s].y, fi, Sre[c1t]);
        Sim[c1t] = mfma4(-y[c1t].v[s].x, fi, Sim[c1t]);
      }
    }
  };
  auto fetch1 = [&](int kb, c4& f, c4(&y)[MT]) {
    f = FT.f32((size_t)kt2 * MT + kb, lane);
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) y[c1t] = ysrc.load(c1t * 16 + r16, kb * 16 + 4 * g);
  };
  if constexpr (MT <= 4) {
    c4 f[2], y[2][MT];
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
      c4 f, y[MT];
      fetch1(kb, f, y);
      stage1(f, y);
    }
  }
  adj_stage2_f32<MT, K1>(Sre, Sim, NB, FT, kt2, sink, k1_first, k1_step);
}

// FP32 adjoint for long windows: K2 neighbouring column tiles kt2_0 ..
// kt2_0 + K2 - 1 per wave.  Stage 1 shares each coefficient chunk between
// the K2 tiles; stage 2 fetches each FT block (k1t, c1t) once for all K2
// tiles, so the table (megabytes when n is in the thousands, past the
// caches) streams NB / K2 instead of NB times per patch.  Tiles at or past
// NB are computed on the last tile's twiddles and not stored.
template <int MT, int K2, class YSrc, class Sink, class Tab>
__device__ __forceinline__ void adj_tiles_f32(const YSrc& ysrc, int NB, const Tab& FT, int kt2_0, Sink& sink) {
  const int lane = lane_id();
  const int r16 = lane & 15, g = lane >> 4;
  f32x4 Sre[K2][MT], Sim[K2][MT];
#pragma unroll
  for (int u = 0; u < K2; ++u)
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      Sre[u][a] = zero4();
      Sim[u][a] = zero4();
    }
  int kt[K2];
#pragma unroll
  for (int u = 0; u < K2; ++u) kt[u] = kt2_0 + u < NB ? kt2_0 + u : NB - 1;
  // stage 1: S_u[c1][k2] = sum_c2 Y[c1][c2] conj(F[c2][k2]) for every tile u
#pragma unroll
  for (int kb = 0; kb < MT; ++kb) {
    c4 y[MT], f[K2];
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) y[c1t] = ysrc.load(c1t * 16 + r16, kb * 16 + 4 * g);
#pragma unroll
    for (int u = 0; u < K2; ++u) f[u] = FT.f32((size_t)kt[u] * MT + kb, lane);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int u = 0; u < K2; ++u) {
        const float fr = f[u].v[s].x, fi = f[u].v[s].y;
#pragma unroll
        for (int c1t = 0; c1t < MT; ++c1t) {
          Sre[u][c1t] = mfma4(y[c1t].v[s].x, fr, Sre[u][c1t]);
          Sim[u][c1t] = mfma4(y[c1t].v[s].y, fr, Sim[u][c1t]);
          Sre[u][c1t] = mfma4(y[c1t].v[s].y, fi, Sre[u][c1t]);
          Sim[u][c1t] = mfma4(-y[c1t].v[s].x, fi, Sim[u][c1t]);
        }
      }
  }
  // stage 2: X_u[k1][k2] = sum_c1 conj(F[c1][k1]) S_u[c1][k2], one row tile
  // at a time, the next block fetched while this one's products issue; three
  // products per complex product as in adj_stage2_gauss (S = a + ib:
  // k1 = a (Re F - Im F), k2' = Im F (a + b), k3 = Re F (b - a),
  // Re X = k1 + k2', Im X = k1 + k3), so Sim is turned into a + b and Sre
  // keeps a beside b - a
  f32x4 Sdif[K2][MT];
#pragma unroll
  for (int u = 0; u < K2; ++u)
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      Sdif[u][a] = Sim[u][a] - Sre[u][a];
      Sim[u][a] = Sim[u][a] + Sre[u][a];
    }
  c4 fb[2];
  fb[0] = FT.f32(0, lane);
  for (int k1t = 0; k1t < NB; ++k1t) {
    f32x4 X1[K2], X2[K2], X3[K2];
#pragma unroll
    for (int u = 0; u < K2; ++u) {
      X1[u] = zero4();
      X2[u] = zero4();
      X3[u] = zero4();
    }
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) {
      const int cur = c1t & 1;
      const int nk = c1t + 1 < MT ? k1t : (k1t + 1 < NB ? k1t + 1 : k1t);
      const int nc = c1t + 1 < MT ? c1t + 1 : 0;
      fb[cur ^ 1] = FT.f32((size_t)nk * MT + nc, lane);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float fr = fb[cur].v[i].x, fi = fb[cur].v[i].y, fd = fr - fi;
#pragma unroll
        for (int u = 0; u < K2; ++u) {
          X1[u] = mfma4(fd, Sre[u][c1t][i], X1[u]);
          X2[u] = mfma4(fi, Sim[u][c1t][i], X2[u]);
          X3[u] = mfma4(fr, Sdif[u][c1t][i], X3[u]);
        }
      }
    }
    if constexpr ((MT & 1) != 0) fb[0] = fb[1];
#pragma unroll
    for (int u = 0; u < K2; ++u)
      if (kt2_0 + u < NB) sink.template put<false>(k1t, kt2_0 + u, X1[u] + X2[u], X1[u] + X3[u]);
  }
}

// FP32 adjoint, one whole patch per wave (MT <= 4): the m x m coefficients
// stay in registers (128 at MT = 4) for every column tile kt2, so the wave
// issues no memory loads between its output stores.
template <int MT, int K1, class YSrc, class Sink, class Tab>
__device__ __forceinline__ void adj_patch_f32(const YSrc& ysrc, int NB, const Tab& FT, Sink& sink, int kt_first = 0,
                                              int kt_step = 1) {
  static_assert(MT <= 4, "larger windows do not fit in registers");
  const int lane = lane_id();
  const int r16 = lane & 15, g = lane >> 4;
  c4 y[MT][MT];  // [column block kb][row tile c1t]
#pragma unroll
  for (int kb = 0; kb < MT; ++kb)
#pragma unroll
    for (int c1t = 0; c1t < MT; ++c1t) y[kb][c1t] = ysrc.load(c1t * 16 + r16, kb * 16 + 4 * g);
  // column tiles kt_first, kt_first + kt_step, ... (several waves may share
  // a window)
  for (int kt2 = kt_first; kt2 < NB; kt2 += kt_step) {
    // stage 1, S = Y conj(F), in three products: data y = a + ib, twiddle
    // conj(F) = c + id (c = Re F, d = -Im F):
    //   k1 = c (a + b),  k2' = a (Re F + Im F),  k3 = b (Re F - Im F),
    //   Re S = k1 - k3,  Im S = k1 - k2'
    // (k2' = -a (d - c) of the Gauss form); the two twiddle sums serve every
    // row tile, a + b takes the place of the negation of the four-product form
    f32x4 S1[MT], S2[MT], S3[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      S1[a] = zero4();
      S2[a] = zero4();
      S3[a] = zero4();
    }
    c4 f[2];
    f[0] = FT.f32((size_t)kt2 * MT, lane);
#pragma unroll
    for (int kb = 0; kb < MT; ++kb) {
      if (kb + 1 < MT) f[(kb + 1) & 1] = FT.f32((size_t)kt2 * MT + kb + 1, lane);
      const c4& fc = f[kb & 1];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float fr = fc.v[s].x, fi = fc.v[s].y;
        const float fsum = fr + fi, fdif = fr - fi;
#pragma unroll
        for (int c1t = 0; c1t < MT; ++c1t) {
          const float ya = y[kb][c1t].v[s].x, yb = y[kb][c1t].v[s].y;
          S1[c1t] = mfma4(ya + yb, fr, S1[c1t]);
          S2[c1t] = mfma4(ya, fsum, S2[c1t]);
          S3[c1t] = mfma4(yb, fdif, S3[c1t]);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      const f32x4 k1 = S1[a];
      S1[a] = k1 - S3[a];
      S2[a] = k1 - S2[a];
    }
    adj_stage2_f32<MT, K1>(S1, S2, NB, FT, kt2, sink);
  }
}

}  // namespace pftpie
