// PIE / ePIE sweep kernels (Sec. 2.1: projection eq. (3), objective eq. (4),
// iterates eqs. (5)-(6)), built on the MFMA partial-transform engines.
//
// Per chunk of positions:
//   k_pie_forward  gather psi = P * O[window] in the operand loader, forward
//                  partial DFT, magnitude projection in the epilogue; writes
//                  the residual r = u' - u ([chunk][m][m]) and per-wave
//                  partial sums of (|u| - a)^2.
//   k_pie_adjoint  dpsi = F^H r conj(F) / n^2, scattered in the epilogue:
//                  O (or numO) += conj(P) dpsi, D += |P|^2 (double),
//                  numP += conj(O_j) dpsi, E += |O_j|^2 (double).
//   k_pie_max      max D (and max E) for the overlap-normalised step.
//   k_pie_apply    O += beta numO / (D + alpha max D) (or beta numO), same
//                  for P; clears the accumulators it read.
// Per sweep: k_pie_begin (copy O, clear accumulators / stats) and
// k_pie_stats (||dO||^2, ||O||^2, non-finite count, Phi).
#include "internal.hpp"
#include "pft_split.hpp"
#include "pie.hpp"

namespace pftpie {

// Position of entry q of the chunk starting at c0.  An order entry outside
// [0, J) is clamped for addressing and reported through `valid` so that the
// kernels contribute nothing for it.
__device__ __forceinline__ int pos_index(const int32_t* __restrict__ order, int J, int c0, int q, bool* valid) {
  int j = order ? order[c0 + q] : c0 + q;
  const bool ok = (j >= 0 && j < J);
  if (valid) *valid = ok;
  return ok ? j : 0;
}

template <class PR, int MT, int CT, bool EXACT>
__global__ __launch_bounds__(64 * ((MT + CT - 1) / CT)) void k_pie_forward(PieArgs a, int c0) {
  const int q = blockIdx.x;
  bool valid;
  const int j = pos_index(a.order, a.J, c0, q, &valid);
  const int w = threadIdx.x >> 6;
  const int c2t0 = w * CT;
  const int2 ps = a.pos[j];
  GatherSrc<EXACT> src{a.O, a.P, a.W, a.n, ps.x, ps.y};
  f32x4 Yre[MT][CT], Yim[MT][CT];
  fwd_engine<PR, MT, CT>(src, a.nb, TabG{static_cast<const char*>(a.fa)}, c2t0, Yre, Yim);
  const int lane = lane_id();
  const int m = a.m;
  const float* amp = a.amp + (size_t)j * m * m;
  float2* res = a.R + (size_t)q * m * m;
  double phi = 0.0;
#pragma unroll
  for (int c1t = 0; c1t < MT; ++c1t)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int2 rc = tile_rc<Orient<PR>::TR>(c1t, c2t0 + ct, i, lane);
        const int c1 = rc.x, c2 = rc.y;
        if (c1 < m && c2 < m) {
          const float ur = Yre[c1t][ct][i], ui = Yim[c1t][ct][i];
          const float av = amp[(size_t)c1 * m + c2];
          const float mag = sqrtf(ur * ur + ui * ui);
          float2 r;
          if (!valid) {
            r = make_float2(0.f, 0.f);
          } else if (mag > 0.f) {
            const float s = av / mag - 1.f;  // a u/|u| - u = (a/|u| - 1) u
            r = make_float2(s * ur, s * ui);
          } else {
            r = make_float2(av - ur, -ui);    // theta(0) = 0
          }
          res[(size_t)c1 * m + c2] = r;
          const double d = (double)mag - (double)av;
          phi += valid ? d * d : 0.0;
        }
      }
    }
  phi = wave_sum(phi);
  if (lane == 0 && valid) a.phi_part[(size_t)j * 4 + w] = phi;
}

// Scatter of dpsi = X / n^2 for one finished 16 x 16 tile.  Holds copies of
// the fields it needs (never the address of a kernel argument).
struct ScatterSink {
  float2* __restrict__ O;
  const float2* __restrict__ P;
  float2* __restrict__ numO;
  double* __restrict__ D;
  float2* __restrict__ numP;
  double* __restrict__ E;
  int n, W, r, c, mode, norm, probe_step;
  float inv, beta;
  template <bool TR>
  __device__ __forceinline__ void put(int k1t, int k2t, const f32x4& xre, const f32x4& xim) const {
    const int lane = lane_id();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int2 rc = tile_rc<TR>(k1t, k2t, i, lane);
      const int k1 = rc.x, k2 = rc.y;
      if (k1 < n && k2 < n) {
        const float2 d = make_float2(xre[i] * inv, xim[i] * inv);
        const float2 p = P[(size_t)k1 * n + k2];
        const size_t o = (size_t)(r + k1) * W + (c + k2);
        const float2 v = cmulc(p, d);  // conj(P) dpsi
        if (mode == kModeDirect) {
          unsafeAtomicAdd(&O[o].x, beta * v.x);
          unsafeAtomicAdd(&O[o].y, beta * v.y);
        } else {
          unsafeAtomicAdd(&numO[o].x, v.x);
          unsafeAtomicAdd(&numO[o].y, v.y);
          if (norm) unsafeAtomicAdd(&D[o], (double)p.x * p.x + (double)p.y * p.y);
          if (probe_step) {
            const float2 ob = O[o];   // unchanged until the apply pass
            const float2 vp = cmulc(ob, d);  // conj(O_j) dpsi
            const size_t pi = (size_t)k1 * n + k2;
            unsafeAtomicAdd(&numP[pi].x, vp.x);
            unsafeAtomicAdd(&numP[pi].y, vp.y);
            if (norm) unsafeAtomicAdd(&E[pi], (double)ob.x * ob.x + (double)ob.y * ob.y);
          }
        }
      }
    }
  }
};

template <class PR, int MT>
__global__ __launch_bounds__(256) void k_pie_adjoint(PieArgs a, int c0) {
  const int q = blockIdx.x;
  const int j = pos_index(a.order, a.J, c0, q, nullptr);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int2 ps = a.pos[j];
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
  } src{a.R + (size_t)q * a.m * a.m, a.m};
  ScatterSink sink{a.O, a.P, a.numO, a.D, a.numP, a.E, a.n, a.W, ps.x, ps.y,
                   a.mode, a.norm, a.probe_step, a.inv_n2, a.beta};
  for (int kt2 = w; kt2 < a.nb; kt2 += nw) adj_engine<PR, MT>(src, a.nb, TabG{static_cast<const char*>(a.ft)}, kt2, sink);
}

// ---------------------------------------------------------------------------
// element-wise passes

// Region of one apply pass: the window of the single position of a chunk
// (read on the device), or the scan's bounding box.
struct Region {
  int r0, c0, h, w;
};

__device__ __forceinline__ Region region_of(const PieArgs& a, int chunk0, int single) {
  if (single) {
    const int j = pos_index(a.order, a.J, chunk0, 0, nullptr);
    const int2 ps = a.pos[j];
    return {ps.x, ps.y, a.n, a.n};
  }
  return {a.bb_r0, a.bb_c0, a.bb_h, a.bb_w};
}

__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }

// max over the region of D (and over the probe of E) -> a.maxes[0], [1]
// (non-negative doubles compare like their bit patterns).
__global__ __launch_bounds__(256) void k_pie_max(PieArgs a, int chunk0, int single) {
  const Region rg = region_of(a, chunk0, single);
  const size_t total = (size_t)rg.h * rg.w;
  double mD = 0.0, mE = 0.0;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int rr = (int)(t / rg.w), cc = (int)(t % rg.w);
    mD = fmax(mD, a.D[(size_t)(rg.r0 + rr) * a.W + rg.c0 + cc]);
  }
  if (a.probe_step) {
    const size_t nn = (size_t)a.n * a.n;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < nn; t += (size_t)gridDim.x * blockDim.x)
      mE = fmax(mE, a.E[t]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    mD = fmax(mD, __shfl_xor(mD, off, 64));
    mE = fmax(mE, __shfl_xor(mE, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(reinterpret_cast<unsigned long long*>(&a.maxes[0]), dbits(mD));
    atomicMax(reinterpret_cast<unsigned long long*>(&a.maxes[1]), dbits(mE));
  }
}

__global__ __launch_bounds__(256) void k_pie_apply(PieArgs a, int chunk0, int single) {
  const Region rg = region_of(a, chunk0, single);
  const size_t total = (size_t)rg.h * rg.w;
  const double regO = a.alpha * a.maxes[0];
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int rr = (int)(t / rg.w), cc = (int)(t % rg.w);
    const size_t o = (size_t)(rg.r0 + rr) * a.W + rg.c0 + cc;
    const float2 num = a.numO[o];
    float sc = a.beta;
    if (a.norm) {
      const double d = a.D[o];
      sc = (d > 0.0) ? (float)((double)a.beta / (d + regO)) : 0.f;
      a.D[o] = 0.0;
    }
    float2 ov = a.O[o];
    ov.x += sc * num.x;
    ov.y += sc * num.y;
    a.O[o] = ov;
    a.numO[o] = make_float2(0.f, 0.f);
  }
  if (a.probe_step) {
    const size_t nn = (size_t)a.n * a.n;
    const double regP = a.alpha * a.maxes[1];
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < nn; t += (size_t)gridDim.x * blockDim.x) {
      const float2 num = a.numP[t];
      float sc = a.gamma;
      if (a.norm) {
        const double e = a.E[t];
        sc = (e > 0.0) ? (float)((double)a.gamma / (e + regP)) : 0.f;
        a.E[t] = 0.0;
      }
      float2 pv = a.P[t];
      pv.x += sc * num.x;
      pv.y += sc * num.y;
      a.P[t] = pv;
      a.numP[t] = make_float2(0.f, 0.f);
    }
  }
}

__global__ void k_pie_clear_max(PieArgs a) {
  if (threadIdx.x < 2) a.maxes[threadIdx.x] = 0.0;
}

// Sweep start: O0 = O; clear the object and probe accumulators and stats.
__global__ __launch_bounds__(256) void k_pie_begin(PieArgs a) {
  const size_t total = (size_t)a.H * a.W;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    a.O0[t] = a.O[t];
    if (a.numO) a.numO[t] = make_float2(0.f, 0.f);
    if (a.D) a.D[t] = 0.0;
  }
  const size_t nn = (size_t)a.n * a.n;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < nn; t += (size_t)gridDim.x * blockDim.x) {
    if (a.numP) a.numP[t] = make_float2(0.f, 0.f);
    if (a.E) a.E[t] = 0.0;
  }
  const size_t np = (size_t)a.J * 4;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < np; t += (size_t)gridDim.x * blockDim.x)
    a.phi_part[t] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x < 4) a.stats[threadIdx.x] = 0.0;
}

// Sweep end: stats = {Phi, ||O - O0||^2, ||O0||^2, non-finite count}.
__global__ __launch_bounds__(256) void k_pie_stats(PieArgs a) {
  const size_t total = (size_t)a.H * a.W;
  double d2 = 0.0, o2 = 0.0, bad = 0.0;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const float2 o = a.O[t], z = a.O0[t];
    const double dx = (double)o.x - z.x, dy = (double)o.y - z.y;
    d2 += dx * dx + dy * dy;
    o2 += (double)z.x * z.x + (double)z.y * z.y;
    bad += (isfinite(o.x) && isfinite(o.y)) ? 0.0 : 1.0;
  }
  if (a.probe_step) {
    const size_t nn = (size_t)a.n * a.n;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < nn; t += (size_t)gridDim.x * blockDim.x) {
      const float2 p = a.P[t];
      bad += (isfinite(p.x) && isfinite(p.y)) ? 0.0 : 1.0;
    }
  }
  d2 = wave_sum(d2);
  o2 = wave_sum(o2);
  bad = wave_sum(bad);
  if ((threadIdx.x & 63) == 0) {
    unsafeAtomicAdd(&a.stats[1], d2);
    unsafeAtomicAdd(&a.stats[2], o2);
    unsafeAtomicAdd(&a.stats[3], bad);
  }
  if (blockIdx.x == 0) {
    // Phi: the per-position partials summed in a fixed order by one wave
    if (threadIdx.x < 64) {
      const size_t np = (size_t)a.J * 4;
      double s = 0.0;
      for (size_t t = threadIdx.x; t < np; t += 64) s += a.phi_part[t];
      s = wave_sum(s);
      if (threadIdx.x == 0) unsafeAtomicAdd(&a.stats[0], s / ((double)a.J * a.n * a.n));
    }
  }
}

// amp[j][c1][c2] = sqrt(I[j][s + c1][s + c2]), s = floor(n/2) - floor(m/2)
__global__ __launch_bounds__(256) void k_crop_amp(const float* __restrict__ I, int J, int n, int m,
                                                  float* __restrict__ amp) {
  const size_t total = (size_t)J * m * m;
  const int s = n / 2 - m / 2;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const size_t j = t / ((size_t)m * m);
    const int rem = (int)(t % ((size_t)m * m));
    const int c1 = rem / m, c2 = rem % m;
    amp[t] = sqrtf(fmaxf(I[(j * n + s + c1) * n + s + c2], 0.f));
  }
}

// ---------------------------------------------------------------------------
// launch

template <class PR, int MT, int CT>
static void fwd_launch(const PieArgs& a, int c0, int cnt, hipStream_t st) {
  constexpr int W = (MT + CT - 1) / CT;
  dim3 grid(cnt), block(64 * W);
  if (a.n % 16 == 0)
    hipLaunchKernelGGL((k_pie_forward<PR, MT, CT, true>), grid, block, 0, st, a, c0);
  else
    hipLaunchKernelGGL((k_pie_forward<PR, MT, CT, false>), grid, block, 0, st, a, c0);
}

template <class PR, int MT>
static void chunk_prec(const PieArgs& a, int c0, int cnt, hipStream_t st) {
  // forward: at most 4 waves per patch so phi_part has a slot per wave
  constexpr int CT = (MT <= 2) ? MT : 2;
  fwd_launch<PR, MT, CT>(a, c0, cnt, st);
  dim3 grid(cnt), block(64 * adj_waves(a.nb));
  hipLaunchKernelGGL((k_pie_adjoint<PR, MT>), grid, block, 0, st, a, c0);
}

template <int MT>
static void chunk_mt(const PieArgs& a, int c0, int cnt, hipStream_t st) {
  if (a.prec == PFTPIE_SPLIT_BF16)
    chunk_prec<PrecBF16, MT>(a, c0, cnt, st);
  else if (a.prec == PFTPIE_SPLIT_FP16)
    chunk_prec<PrecF16, MT>(a, c0, cnt, st);
  else
    chunk_prec<PrecF32, MT>(a, c0, cnt, st);
}

static int ew_blocks(size_t work) {
  size_t b = (work + 255) / 256;
  if (b > 4096) b = 4096;
  return b < 1 ? 1 : (int)b;
}

hipError_t launch_crop_amp(const float* I, int J, int n, int m, float* amp, hipStream_t st) {
  hipLaunchKernelGGL(k_crop_amp, dim3(ew_blocks((size_t)J * m * m)), dim3(256), 0, st, I, J, n, m, amp);
  return hipGetLastError();
}

hipError_t launch_pie_sweep(const PieArgs& a, int batch, hipStream_t st) {
  const size_t obj = (size_t)a.H * a.W;
  hipLaunchKernelGGL(k_pie_begin, dim3(ew_blocks(obj)), dim3(256), 0, st, a);
  for (int c0 = 0; c0 < a.J; c0 += batch) {
    const int cnt = (a.J - c0 < batch) ? a.J - c0 : batch;
    switch (a.mt) {
      case 1: chunk_mt<1>(a, c0, cnt, st); break;
      case 2: chunk_mt<2>(a, c0, cnt, st); break;
      case 3: chunk_mt<3>(a, c0, cnt, st); break;
      case 4: chunk_mt<4>(a, c0, cnt, st); break;
      case 5: chunk_mt<5>(a, c0, cnt, st); break;
      case 6: chunk_mt<6>(a, c0, cnt, st); break;
      case 7: chunk_mt<7>(a, c0, cnt, st); break;
      case 8: chunk_mt<8>(a, c0, cnt, st); break;
      default: return hipErrorInvalidValue;
    }
    if (a.mode != kModeDirect) {
      const int single = (cnt == 1);
      const size_t area = single ? (size_t)a.n * a.n : (size_t)a.bb_h * a.bb_w;
      if (a.norm) {
        hipLaunchKernelGGL(k_pie_clear_max, dim3(1), dim3(64), 0, st, a);
        hipLaunchKernelGGL(k_pie_max, dim3(ew_blocks(area)), dim3(256), 0, st, a, c0, single);
      }
      hipLaunchKernelGGL(k_pie_apply, dim3(ew_blocks(area)), dim3(256), 0, st, a, c0, single);
    }
  }
  hipLaunchKernelGGL(k_pie_stats, dim3(ew_blocks(obj)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace pftpie
