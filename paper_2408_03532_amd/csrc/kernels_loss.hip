// Amplitude loss L = sum_j || |F_m (P * O_j) F_m^T| - a_j ||^2 and its
// hand-written gradient with respect to object and probe.
//
// Gradient (grad = dL/dRe + i dL/dIm): with u_j = F_m psi_j F_m^T,
//   G_j = 2 (u_j - a_j sgn(u_j)),   R_j = F_m^H G_j conj(F_m),
//   dL/dO[window j] += conj(P) R_j,  dL/dP += conj(O_j) R_j.
// k_loss_forward   gathers psi_j in its operand loader, transforms, writes
//                  u_j (optional) and per-wave partial losses.
// k_loss_adjoint   forms G_j from u_j and a_j in its operand loader, applies
//                  the adjoint and stores scale * R_j; the exit waves are
//                  never stored.
// k_loss_object_gather  per 16 x 16 object tile, sums conj(P) R_j over the
//                  positions of the tile's cover list (no atomics).
// k_loss_probe_gather   per probe pixel, sums conj(O_j) R_j over positions.
#include "internal.hpp"
#include "loss.hpp"
#include "pft_split.hpp"

namespace pftpie {

// Forward of position j for column-tile group wslot (tiles wslot * CT ...):
// u_j (optional) and the group's partial loss at part[j][wslot].
template <class PR, int MT, int CT, bool EXACT, class Tab>
__device__ __forceinline__ void loss_fwd_item(const LossArgs& a, const Tab& T, int j, int wslot) {
  const int c2t0 = wslot * CT;
  const int2 ps = a.pos[j];
  GatherSrc<EXACT> src{a.O, a.P, a.W, a.n, ps.x, ps.y, a.n};
  f32x4 Yre[MT][CT], Yim[MT][CT];
  fwd_engine<PR, MT, CT>(src, a.nb, T, c2t0, Yre, Yim, 0, 1, j % a.nb);
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
  if (lane == 0) a.part[(size_t)j * 4 + wslot] = part;
}

template <class PR, int MT, int CT, bool EXACT>
__global__ __launch_bounds__(64 * ((MT + CT - 1) / CT)) void k_loss_forward(LossArgs a) {
  loss_fwd_item<PR, MT, CT, EXACT>(a, TabG{static_cast<const char*>(a.fa)}, blockIdx.x, threadIdx.x >> 6);
}

// Persistent forms: one workgroup per compute unit copies the twiddle table
// into LDS, then its waves pull work items (position, column-tile group) or
// positions.  Used when the table fits LDS and the windows are whole
// 16-pixel tiles.
__device__ __forceinline__ void loss_table_to_lds(f32x4* smem, const void* tab, size_t bytes) {
  const f32x4* t = static_cast<const f32x4*>(tab);
  for (size_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) smem[i] = t[i];
  __syncthreads();
}

template <class PR, int MT, int CT, int THREADS>
__global__ __launch_bounds__(THREADS) void k_loss_forward_lds(LossArgs a) {
  extern __shared__ f32x4 smem[];
  loss_table_to_lds(smem, a.fa, a.fa_bytes);
  const TabL T{(lds_cptr)smem};
  constexpr int W = (MT + CT - 1) / CT;
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int64_t items = (int64_t)a.J * W;
  for (int64_t it = (int64_t)blockIdx.x * nwaves + wave; it < items; it += (int64_t)gridDim.x * nwaves)
    loss_fwd_item<PR, MT, CT, true>(a, T, (int)(it / W), (int)(it % W));
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

struct RSink {
  float2* __restrict__ out;
  int n;
  float scale;
  template <bool TR>
  __device__ __forceinline__ void put(int k1t, int k2t, const f32x4& xre, const f32x4& xim) const {
    const int lane = lane_id();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int2 rc = tile_rc<TR>(k1t, k2t, i, lane);
      if (rc.x < n && rc.y < n) out[(size_t)rc.x * n + rc.y] = make_float2(scale * xre[i], scale * xim[i]);
    }
  }
};

// Whole window per wave (m <= 64 in 16-pixel tiles): the gradient
// coefficients stay in registers for every column tile.  FP32 with `share`
// = 2: two waves per window, each taking every other column tile (work
// items (position, half)), so that fewer positions than twice the wave
// slots still fill the compute units.
template <class PR, int MT, int THREADS>
__global__ __launch_bounds__(THREADS) void k_loss_adjoint_lds(LossArgs a, int share) {
  extern __shared__ f32x4 smem[];
  loss_table_to_lds(smem, a.ft, a.ft_bytes);
  const TabL T{(lds_cptr)smem};
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const size_t mm = (size_t)a.m * a.m;
  const float scale = a.scale_dev ? (float)a.scale_dev[0] : 1.f;
  const int items = a.J * share;
  for (int it = blockIdx.x * nwaves + wave; it < items; it += gridDim.x * nwaves) {
    const int j = it / share, part = it % share;
    GradSrc src{a.Uc + (size_t)j * mm, a.amp + (size_t)j * mm, a.m};
    RSink sink{a.Rbuf + (size_t)j * a.n * a.n, a.n, scale};
    if constexpr (Orient<PR>::TR)
      adj_patch_split<PR, MT>(src, a.nb, T, sink);
    else
      adj_patch_f32<MT, 1>(src, a.nb, T, sink, part, share);
  }
}

template <class PR, int MT>
__global__ __launch_bounds__(256) void k_loss_adjoint(LossArgs a) {
  const int j = blockIdx.x;
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const size_t mm = (size_t)a.m * a.m;
  GradSrc src{a.Uc + (size_t)j * mm, a.amp + (size_t)j * mm, a.m};
  const float scale = a.scale_dev ? (float)a.scale_dev[0] : 1.f;
  RSink sink{a.Rbuf + (size_t)j * a.n * a.n, a.n, scale};
  for (int kt2 = w; kt2 < a.nb; kt2 += nw)
    adj_engine<PR, MT>(src, a.nb, TabG{static_cast<const char*>(a.ft)}, kt2, sink);
}

// dL/dO over the bounding box: per 16 x 16 tile, every position of its cover
// list whose window holds the pixel contributes conj(P) R_j.
__global__ __launch_bounds__(256) void k_loss_object_gather(LossArgs a) {
  const int tile = blockIdx.x;
  const int ty = tile / a.tiles_x, tx = tile % a.tiles_x;
  const int py = a.bb_r0 + ty * 16 + (threadIdx.x >> 4);
  const int px = a.bb_c0 + tx * 16 + (threadIdx.x & 15);
  if (py >= a.bb_r0 + a.bb_h || px >= a.bb_c0 + a.bb_w) return;
  const size_t nn = (size_t)a.n * a.n;
  float2 acc = make_float2(0.f, 0.f);
  const int e0 = a.tile_ptr[tile], e1 = a.tile_ptr[tile + 1];
  for (int e = e0; e < e1; ++e) {
    const int j = a.tile_pos[e];
    const int2 ps = a.pos[j];
    const int dy = py - ps.x, dx = px - ps.y;
    if (dy < 0 || dy >= a.n || dx < 0 || dx >= a.n) continue;
    const size_t k = (size_t)dy * a.n + dx;
    const float2 v = cmulc(a.P[k], a.Rbuf[(size_t)j * nn + k]);
    acc.x += v.x;
    acc.y += v.y;
  }
  a.gO[(size_t)py * a.W + px] = acc;
}

// dL/dP: per probe pixel, partial sums of conj(O_j) R_j over chunks of
// kLossChunk positions (blockIdx.y), then a fixed-order sum of the partials.
constexpr int kLossChunk = 64;

__global__ __launch_bounds__(256) void k_loss_probe_gather(LossArgs a) {
  const size_t nn = (size_t)a.n * a.n;
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const int k1 = (int)(k / a.n), k2 = (int)(k % a.n);
  const int j0 = blockIdx.y * kLossChunk;
  const int j1 = (j0 + kLossChunk < a.J) ? j0 + kLossChunk : a.J;
  float2 acc = make_float2(0.f, 0.f);
  for (int j = j0; j < j1; ++j) {
    const int2 ps = a.pos[j];
    const float2 v = cmulc(a.O[(size_t)(ps.x + k1) * a.W + ps.y + k2], a.Rbuf[(size_t)j * nn + k]);
    acc.x += v.x;
    acc.y += v.y;
  }
  a.gPpart[(size_t)blockIdx.y * nn + k] = acc;
}

__global__ __launch_bounds__(256) void k_loss_probe_sum(LossArgs a, int nchunks) {
  const size_t nn = (size_t)a.n * a.n;
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  float2 acc = make_float2(0.f, 0.f);
  for (int c = 0; c < nchunks; ++c) {
    const float2 v = a.gPpart[(size_t)c * nn + k];
    acc.x += v.x;
    acc.y += v.y;
  }
  a.gP[k] = acc;
}

__global__ __launch_bounds__(256) void k_loss_reduce(LossArgs a) {
  // one wave, fixed summation order
  const size_t np = (size_t)a.J * 4;
  double s = 0.0;
  for (size_t t = threadIdx.x; t < np; t += 64) s += a.part[t];
  s = wave_sum(s);
  if (threadIdx.x == 0) a.loss[0] = s;
}

// dL/dO is zero outside the bounding box of the windows.
__global__ __launch_bounds__(256) void k_loss_clear(LossArgs a) {
  const size_t total = (size_t)a.H * a.W;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(t / a.W), c = (int)(t % a.W);
    if (r < a.bb_r0 || r >= a.bb_r0 + a.bb_h || c < a.bb_c0 || c >= a.bb_c0 + a.bb_w)
      a.gO[t] = make_float2(0.f, 0.f);
  }
}

__global__ __launch_bounds__(256) void k_loss_clear_parts(LossArgs a) {
  const size_t np = (size_t)a.J * 4;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < np; t += (size_t)gridDim.x * blockDim.x)
    a.part[t] = 0.0;
}

// Persistent launch of `kernel` with `tab_bytes` of dynamic LDS: at most one
// workgroup per compute unit, fewer when the items are few.
template <class K, class... Extra>
static bool launch_lds(K kernel, const LossArgs& a, size_t tab_bytes, int64_t items, int threads, hipStream_t st,
                       Extra... extra) {
  if (tab_bytes > kMaxLdsTable ||
      hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)tab_bytes) != hipSuccess)
    return false;
  const int64_t waves = threads / 64;
  int64_t grid = (items + waves - 1) / waves;
  if (grid > a.num_cu) grid = a.num_cu;
  hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(threads), tab_bytes, st, a, extra...);
  return true;
}

// windows of whole 16-pixel tiles (the persistent forward runs the
// unchecked operand loads)
static bool loss_tiles_exact(const LossArgs& a) { return a.n % 16 == 0; }

template <class PR, int MT>
static void fwd_prec(const LossArgs& a, hipStream_t st) {
  constexpr int CT = (MT <= 2) ? MT : 2;
  constexpr int W = (MT + CT - 1) / CT;
  if (loss_tiles_exact(a) &&
      launch_lds(k_loss_forward_lds<PR, MT, CT, 512>, a, a.fa_bytes, (int64_t)a.J * W, 512, st))
    return;
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
  if constexpr (MT <= 4) {
    if (a.m % 16 == 0 && a.n % 16 == 0) {
      // whole window per wave: the split coefficients of m = 48, 64 take
      // most of the registers (one wave per SIMD); otherwise two fit
      constexpr int TH = MT <= 2 ? 512 : 256;
      bool done = false;
      if (a.prec == PFTPIE_SPLIT_BF16) {
        done = launch_lds(k_loss_adjoint_lds<PrecBF16, MT, TH>, a, a.ft_bytes, a.J, TH, st, 1);
      } else if (a.prec == PFTPIE_SPLIT_FP16) {
        done = launch_lds(k_loss_adjoint_lds<PrecF16, MT, TH>, a, a.ft_bytes, a.J, TH, st, 1);
      } else {
        // two waves per window while the positions alone leave wave slots idle
        const int share = (a.J < 2 * 8 * a.num_cu && a.nb >= 2) ? 2 : 1;
        done = launch_lds(k_loss_adjoint_lds<PrecF32, MT, 512>, a, a.ft_bytes, (int64_t)a.J * share, 512, st, share);
      }
      if (done) return;
    }
  }
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
  hipLaunchKernelGGL(k_loss_object_gather, dim3(a.tiles_x * a.tiles_y), dim3(256), 0, st, a);
  if (a.gP) {
    const unsigned pb = (unsigned)(((size_t)a.n * a.n + 255) / 256);
    const int nch = (a.J + kLossChunk - 1) / kLossChunk;
    hipLaunchKernelGGL(k_loss_probe_gather, dim3(pb, nch), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_loss_probe_sum, dim3(pb), dim3(256), 0, st, a, nch);
  }
  return hipGetLastError();
}

}  // namespace pftpie
