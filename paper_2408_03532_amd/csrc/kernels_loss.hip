// Amplitude loss L = sum_j || |F_m (P * O_j) F_m^T| - a_j ||^2 and its
// hand-written gradient with respect to object and probe.
//
// Gradient (grad = dL/dRe + i dL/dIm): with u_j = F_m psi_j F_m^T,
//   G_j = 2 (u_j - a_j sgn(u_j)),   R_j = F_m^H G_j conj(F_m),
//   dL/dO[window j] += conj(P) R_j,  dL/dP += conj(O_j) R_j.
// k_loss_forward   gathers psi_j in its operand loader, transforms, writes
//                  u_j (optional) and per-wave partial losses.
// k_loss_adjoint   forms G_j from u_j and a_j in its operand loader, applies
//                  the adjoint and scatters both gradients in its epilogue;
//                  the exit waves are never stored.
#include "internal.hpp"
#include "loss.hpp"
#include "pft_split.hpp"

namespace pftpie {

template <class PR, int MT, int CT, bool EXACT>
__global__ __launch_bounds__(64 * ((MT + CT - 1) / CT)) void k_loss_forward(LossArgs a) {
  const int j = blockIdx.x;
  const int w = threadIdx.x >> 6;
  const int c2t0 = w * CT;
  const int2 ps = a.pos[j];
  GatherSrc<EXACT> src{a.O, a.P, a.W, a.n, ps.x, ps.y};
  f32x4 Yre[MT][CT], Yim[MT][CT];
  fwd_engine<PR, MT, CT>(src, a.nb, TabG{static_cast<const char*>(a.fa)}, c2t0, Yre, Yim);
  const int lane = lane_id();
  const int m = a.m;
  const float* amp = a.amp + (size_t)j * m * m;
  float2* u = a.U ? a.U + (size_t)j * m * m : nullptr;
  double part = 0.0;
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
          if (u) u[(size_t)c1 * m + c2] = make_float2(ur, ui);
          const double d = (double)sqrtf(ur * ur + ui * ui) - (double)amp[(size_t)c1 * m + c2];
          part += d * d;
        }
      }
    }
  part = wave_sum(part);
  if (lane == 0) a.part[(size_t)j * 4 + w] = part;
}

// G = 2 (u - a sgn(u)) built on the fly from u_j and a_j (sgn(0) = 0).
struct GradSrc {
  const float2* __restrict__ u;
  const float* __restrict__ amp;
  int m;
  __device__ __forceinline__ c4 load(int row, int col0) const {
    c4 v;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int col = col0 + s;
      if (row < m && col < m) {
        const float2 z = u[(size_t)row * m + col];
        const float av = amp[(size_t)row * m + col];
        const float mag = sqrtf(z.x * z.x + z.y * z.y);
        const float sc = (mag > 0.f) ? 2.f * (1.f - av / mag) : 2.f;  // 2(u - a u/|u|)
        v.v[s] = make_float2(sc * z.x, sc * z.y);
      } else {
        v.v[s] = make_float2(0.f, 0.f);
      }
    }
    return v;
  }
};

struct GradSink {
  const float2* __restrict__ O;
  const float2* __restrict__ P;
  float2* __restrict__ gO;
  float2* __restrict__ gP;
  int n, W, r, c;
  float scale;
  template <bool TR>
  __device__ __forceinline__ void put(int k1t, int k2t, const f32x4& xre, const f32x4& xim) const {
    const int lane = lane_id();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int2 rc = tile_rc<TR>(k1t, k2t, i, lane);
      const int k1 = rc.x, k2 = rc.y;
      if (k1 < n && k2 < n) {
        const float2 R = make_float2(scale * xre[i], scale * xim[i]);
        const size_t pi = (size_t)k1 * n + k2;
        const size_t o = (size_t)(r + k1) * W + (c + k2);
        const float2 vo = cmulc(P[pi], R);  // conj(P) R
        unsafeAtomicAdd(&gO[o].x, vo.x);
        unsafeAtomicAdd(&gO[o].y, vo.y);
        if (gP) {
          const float2 vp = cmulc(O[o], R);  // conj(O_j) R
          unsafeAtomicAdd(&gP[pi].x, vp.x);
          unsafeAtomicAdd(&gP[pi].y, vp.y);
        }
      }
    }
  }
};

template <class PR, int MT>
__global__ __launch_bounds__(256) void k_loss_adjoint(LossArgs a) {
  const int j = blockIdx.x;
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int2 ps = a.pos[j];
  const size_t mm = (size_t)a.m * a.m;
  GradSrc src{a.Uc + (size_t)j * mm, a.amp + (size_t)j * mm, a.m};
  const float scale = a.scale_dev ? (float)a.scale_dev[0] : 1.f;
  GradSink sink{a.O, a.P, a.gO, a.gP, a.n, a.W, ps.x, ps.y, scale};
  for (int kt2 = w; kt2 < a.nb; kt2 += nw) adj_engine<PR, MT>(src, a.nb, TabG{static_cast<const char*>(a.ft)}, kt2, sink);
}

__global__ __launch_bounds__(256) void k_loss_reduce(LossArgs a) {
  // one wave, fixed summation order
  const size_t np = (size_t)a.J * 4;
  double s = 0.0;
  for (size_t t = threadIdx.x; t < np; t += 64) s += a.part[t];
  s = wave_sum(s);
  if (threadIdx.x == 0) a.loss[0] = s;
}

__global__ __launch_bounds__(256) void k_loss_clear(LossArgs a) {
  const size_t total = (size_t)a.H * a.W;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x)
    a.gO[t] = make_float2(0.f, 0.f);
  if (a.gP) {
    const size_t nn = (size_t)a.n * a.n;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < nn; t += (size_t)gridDim.x * blockDim.x)
      a.gP[t] = make_float2(0.f, 0.f);
  }
  if (a.part) {
    const size_t np = (size_t)a.J * 4;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < np; t += (size_t)gridDim.x * blockDim.x)
      a.part[t] = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_loss_clear_parts(LossArgs a) {
  const size_t np = (size_t)a.J * 4;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < np; t += (size_t)gridDim.x * blockDim.x)
    a.part[t] = 0.0;
}

template <class PR, int MT>
static void fwd_prec(const LossArgs& a, hipStream_t st) {
  constexpr int CT = (MT <= 2) ? MT : 2;
  constexpr int W = (MT + CT - 1) / CT;
  if (a.n % 16 == 0)
    hipLaunchKernelGGL((k_loss_forward<PR, MT, CT, true>), dim3(a.J), dim3(64 * W), 0, st, a);
  else
    hipLaunchKernelGGL((k_loss_forward<PR, MT, CT, false>), dim3(a.J), dim3(64 * W), 0, st, a);
}

template <int MT>
static void fwd_mt(const LossArgs& a, hipStream_t st) {
  if (a.prec == PFTPIE_SPLIT_BF16)
    fwd_prec<PrecBF16, MT>(a, st);
  else if (a.prec == PFTPIE_SPLIT_FP16)
    fwd_prec<PrecF16, MT>(a, st);
  else
    fwd_prec<PrecF32, MT>(a, st);
}

template <int MT>
static void adj_mt(const LossArgs& a, hipStream_t st) {
  dim3 grid(a.J), block(64 * adj_waves(a.nb));
  if (a.prec == PFTPIE_SPLIT_BF16)
    hipLaunchKernelGGL((k_loss_adjoint<PrecBF16, MT>), grid, block, 0, st, a);
  else if (a.prec == PFTPIE_SPLIT_FP16)
    hipLaunchKernelGGL((k_loss_adjoint<PrecF16, MT>), grid, block, 0, st, a);
  else
    hipLaunchKernelGGL((k_loss_adjoint<PrecF32, MT>), grid, block, 0, st, a);
}

static hipError_t fwd_dispatch(const LossArgs& a, hipStream_t st) {
  switch (a.mt) {
    case 1: fwd_mt<1>(a, st); break;
    case 2: fwd_mt<2>(a, st); break;
    case 3: fwd_mt<3>(a, st); break;
    case 4: fwd_mt<4>(a, st); break;
    case 5: fwd_mt<5>(a, st); break;
    case 6: fwd_mt<6>(a, st); break;
    case 7: fwd_mt<7>(a, st); break;
    case 8: fwd_mt<8>(a, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipSuccess;
}

static int blocks_for(size_t work) {
  size_t b = (work + 255) / 256;
  if (b > 4096) b = 4096;
  return b < 1 ? 1 : (int)b;
}

hipError_t launch_loss_forward(const LossArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_clear_parts, dim3(blocks_for((size_t)a.J * 4)), dim3(256), 0, st, a);
  if (hipError_t e = fwd_dispatch(a, st)) return e;
  hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_loss_backward(const LossArgs& a, bool recompute, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_clear, dim3(blocks_for((size_t)a.H * a.W)), dim3(256), 0, st, a);
  if (recompute)
    if (hipError_t e = fwd_dispatch(a, st)) return e;
  switch (a.mt) {
    case 1: adj_mt<1>(a, st); break;
    case 2: adj_mt<2>(a, st); break;
    case 3: adj_mt<3>(a, st); break;
    case 4: adj_mt<4>(a, st); break;
    case 5: adj_mt<5>(a, st); break;
    case 6: adj_mt<6>(a, st); break;
    case 7: adj_mt<7>(a, st); break;
    case 8: adj_mt<8>(a, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pftpie
