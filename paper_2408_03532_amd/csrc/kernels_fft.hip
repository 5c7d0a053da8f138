// Full-window (m = n) kernels on the in-LDS fast transform (fft.hpp): the
// plain forward / adjoint of a plan whose method is the fast transform, and
// the fused PIE step of one scan position (exit wave, forward transform,
// magnitude projection of eq. (3) and objective of eq. (4), inverse
// transform, then the in-place update of eqs. (5)-(6) for a single-position
// chunk or the stored correction for a larger chunk), used by the second
// phase of the hybrid method (Algorithm 3) at full resolution.
//
// With m = n the centred window index c holds frequency (c - n/2) mod n
// (the kept frequencies t_c = c - floor(m/2) of the partial transform), so
// the outputs are the fast transform in centred order.  One workgroup owns
// one block of n x n complex values in LDS (n = 128: 136 KB).
#include "fft.hpp"
#include "internal.hpp"
#include "pie.hpp"

namespace pftpie {

// n = 128: the block takes most of the LDS, one workgroup per compute
// unit, so it brings four waves per SIMD itself to hide LDS latency.
template <class G>
constexpr int fft_threads() {
  return G::N >= 128 ? 1024 : (G::N == 64 ? 256 : (G::N == 32 ? 128 : 64));
}
template <class G>
constexpr size_t fft_lds_bytes() {
  return (size_t)(G::N + G::ELEMS) * sizeof(float2);
}

__device__ __forceinline__ void load_twiddles(float2* tw, const float2* __restrict__ tw_g, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = tw_g[i];
}

// centred window index -> stored slot of its frequency
template <class G>
__device__ __forceinline__ int centred_slot(int c) {
  return G::slot((c + G::N / 2) & (G::N - 1));
}

// y_b = centred-order 2-D transform of psi_b.
template <class G>
__global__ __launch_bounds__(fft_threads<G>()) void k_fft_forward(const float2* __restrict__ psi,
                                                                   float2* __restrict__ y,
                                                                   const float2* __restrict__ tw_g, int64_t batch) {
  extern __shared__ float2 sm[];
  float2* tw = sm;
  float2* buf = sm + G::N;
  constexpr int N = G::N;
  load_twiddles(tw, tw_g, N);
  __syncthreads();
  for (int64_t b = blockIdx.x; b < batch; b += gridDim.x) {
    const float2* __restrict__ x = psi + b * (int64_t)N * N;
    for (int it = threadIdx.x; it < N * G::R2; it += blockDim.x) {
      const int row = it / G::R2, n2 = it % G::R2;
      float2 v[G::R1];
#pragma unroll
      for (int n1 = 0; n1 < G::R1; ++n1) v[n1] = x[(size_t)row * N + G::R2 * n1 + n2];
      pass_a_values<G, false>(v, n2, tw);
#pragma unroll
      for (int k1 = 0; k1 < G::R1; ++k1) buf[G::at(row, G::R2 * k1 + n2)] = v[k1];
    }
    fft2_rest_forward<G>(buf, tw);
    float2* __restrict__ out = y + b * (int64_t)N * N;
    for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
      const int c1 = t / N, c2 = t % N;
      out[t] = buf[G::at(centred_slot<G>(c1), centred_slot<G>(c2))];
    }
    __syncthreads();
  }
}

// psi_b = F^H y_b conj(F) (unnormalised inverse of the centred-order y_b).
template <class G>
__global__ __launch_bounds__(fft_threads<G>()) void k_fft_adjoint(const float2* __restrict__ y,
                                                                   float2* __restrict__ psi,
                                                                   const float2* __restrict__ tw_g, int64_t batch) {
  extern __shared__ float2 sm[];
  float2* tw = sm;
  float2* buf = sm + G::N;
  constexpr int N = G::N;
  load_twiddles(tw, tw_g, N);
  for (int64_t b = blockIdx.x; b < batch; b += gridDim.x) {
    const float2* __restrict__ in = y + b * (int64_t)N * N;
    for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
      const int c1 = t / N, c2 = t % N;
      buf[G::at(centred_slot<G>(c1), centred_slot<G>(c2))] = in[t];
    }
    fft2_inverse_head<G>(buf, tw);
    float2* __restrict__ out = psi + b * (int64_t)N * N;
    for (int it = threadIdx.x; it < N * G::R2; it += blockDim.x) {
      const int row = it / G::R2, n2 = it % G::R2;
      float2 v[G::R1];
#pragma unroll
      for (int k1 = 0; k1 < G::R1; ++k1) v[k1] = buf[G::at(row, G::R2 * k1 + n2)];
      pass_a_values<G, true>(v, n2, tw);
#pragma unroll
      for (int n1 = 0; n1 < G::R1; ++n1) out[(size_t)row * N + G::R2 * n1 + n2] = v[n1];
    }
    __syncthreads();
  }
}

// Position of entry q of the chunk starting at c0 (order entries outside
// [0, J) contribute nothing).
__device__ __forceinline__ int fft_pos_index(const int32_t* __restrict__ order, int J, int c0, int q, bool* valid) {
  const int j = order ? order[c0 + q] : c0 + q;
  *valid = (j >= 0 && j < J);
  return *valid ? j : 0;
}

// One PIE position per workgroup (chunk entry q = blockIdx.x).  SINGLE: the
// chunk is this one position, updated in place (every pixel belongs to one
// thread, values before the update); TRACK: also the window maxima of |P|^2
// and |O_j|^2 for the overlap-normalised single-position step.
template <class G, bool SINGLE, bool TRACK>
__global__ __launch_bounds__(fft_threads<G>()) void k_pie_fft(PieArgs a, int c0) {
  extern __shared__ float2 sm[];
  float2* tw = sm;
  float2* buf = sm + G::N;
  __shared__ double red_phi[16];
  __shared__ float red_max[2][16];
  constexpr int N = G::N;
  load_twiddles(tw, a.fft_tw, N);
  __syncthreads();
  const int q = blockIdx.x;
  bool valid;
  const int j = fft_pos_index(a.order, a.J, c0, q, &valid);
  const int2 ps = a.pos[j];
  [[maybe_unused]] const size_t dbase = dpsi_base(a, q, valid ? ps.y : a.bb_c0);
  // exit wave psi = P * O[window] and the row pass A
  float mp = 0.f, mo = 0.f;
  for (int it = threadIdx.x; it < N * G::R2; it += blockDim.x) {
    const int row = it / G::R2, n2 = it % G::R2;
    const float2* orow = a.O + (size_t)(ps.x + row) * a.W + ps.y;
    float2 v[G::R1];
#pragma unroll
    for (int n1 = 0; n1 < G::R1; ++n1) {
      const int col = G::R2 * n1 + n2;
      const float2 p = a.P[(size_t)row * N + col], o = orow[col];
      if constexpr (TRACK) {
        mp = fmaxf(mp, p.x * p.x + p.y * p.y);
        mo = fmaxf(mo, o.x * o.x + o.y * o.y);
      }
      v[n1] = cmul(p, o);
    }
    pass_a_values<G, false>(v, n2, tw);
#pragma unroll
    for (int k1 = 0; k1 < G::R1; ++k1) buf[G::at(row, G::R2 * k1 + n2)] = v[k1];
  }
  fft2_rest_forward<G>(buf, tw);
  // projection: residual r = a u/|u| - u (theta(0) = 0) in place, objective
  const float* __restrict__ amp = a.amp + (size_t)j * N * N;
  double phi = 0.0;
  for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
    const int c1 = t / N, c2 = t % N;
    const int ad = G::at(centred_slot<G>(c1), centred_slot<G>(c2));
    const float2 u = buf[ad];
    const float av = amp[t];
    const float mag = sqrtf(u.x * u.x + u.y * u.y);
    float2 r;
    if (!valid) {
      r = make_float2(0.f, 0.f);
    } else if (mag > 0.f) {
      const float s = av / mag - 1.f;
      r = make_float2(s * u.x, s * u.y);
    } else {
      r = make_float2(av - u.x, -u.y);
    }
    buf[ad] = r;
    const double d = (double)mag - (double)av;
    phi += valid ? d * d : 0.0;
  }
  phi = wave_sum(phi);
  if constexpr (TRACK) {
    mp = wave_max(mp);
    mo = wave_max(mo);
  }
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red_phi[w] = phi;
    red_max[0][w] = mp;
    red_max[1][w] = mo;
  }
  fft2_inverse_head<G>(buf, tw);  // starts with a barrier: the partials are visible
  if (threadIdx.x == 0 && valid && !a.probe_pass) {
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red_phi[k];
    a.phi_part[(size_t)j * 4] = s;
  }
  double regP = 0.0, regO = 0.0;
  if constexpr (SINGLE && TRACK) {
    if (a.norm) {
      float xp = 0.f, xo = 0.f;
      for (int k = 0; k < nw; ++k) {
        xp = fmaxf(xp, red_max[0][k]);
        xo = fmaxf(xo, red_max[1][k]);
      }
      regP = a.alpha * (double)xp;
      regO = a.alpha * (double)xo;
    }
  }
  // last row pass A^H: dpsi = F^H r conj(F) / n^2 into the update or store
  for (int it = threadIdx.x; it < N * G::R2; it += blockDim.x) {
    const int row = it / G::R2, n2 = it % G::R2;
    float2 v[G::R1];
#pragma unroll
    for (int k1 = 0; k1 < G::R1; ++k1) v[k1] = buf[G::at(row, G::R2 * k1 + n2)];
    pass_a_values<G, true>(v, n2, tw);
#pragma unroll
    for (int n1 = 0; n1 < G::R1; ++n1) {
      const int col = G::R2 * n1 + n2;
      const float2 d = make_float2(v[n1].x * a.inv_n2, v[n1].y * a.inv_n2);
      if constexpr (SINGLE) {
        if (!valid) continue;
        const size_t pi = (size_t)row * N + col;
        const size_t oi = (size_t)(ps.x + row) * a.W + ps.y + col;
        const float2 p = a.P[pi];
        const float2 ov = a.O[oi];
        if (a.probe_pass) {  // probe step at the updated object, O unchanged
          const float2 vp = cmulc(ov, d);
          a.P[pi] = make_float2(p.x + a.gamma * vp.x, p.y + a.gamma * vp.y);
          continue;
        }
        float so = a.beta;
        if (a.norm) {
          const double p2 = (double)p.x * p.x + (double)p.y * p.y;
          so = p2 > 0.0 ? (float)((double)a.beta / (p2 + regP)) : 0.f;
        }
        const float2 vo = cmulc(p, d);
        a.O[oi] = make_float2(ov.x + so * vo.x, ov.y + so * vo.y);
        if (a.probe_step) {
          float sp = a.gamma;
          if (a.norm) {
            const double o2 = (double)ov.x * ov.x + (double)ov.y * ov.y;
            sp = o2 > 0.0 ? (float)((double)a.gamma / (o2 + regO)) : 0.f;
          }
          const float2 vp = cmulc(ov, d);
          a.P[pi] = make_float2(p.x + sp * vp.x, p.y + sp * vp.y);
        }
      } else {
        a.dpsi[dbase + (size_t)row * a.dstride + col] = valid ? d : make_float2(0.f, 0.f);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launch

template <class K>
static hipError_t set_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <class G>
static hipError_t fft_fwd(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch, hipStream_t st) {
  const size_t lds = fft_lds_bytes<G>();
  hipError_t e = set_lds(k_fft_forward<G>, lds);
  if (e != hipSuccess) return e;
  const int64_t grid = batch < (int64_t)p->num_cu * 8 ? batch : (int64_t)p->num_cu * 8;
  hipLaunchKernelGGL(k_fft_forward<G>, dim3((unsigned)grid), dim3(fft_threads<G>()), lds, st, psi, y,
                     static_cast<const float2*>(p->fft_tw), batch);
  return hipGetLastError();
}

template <class G>
static hipError_t fft_adj(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch, hipStream_t st) {
  const size_t lds = fft_lds_bytes<G>();
  hipError_t e = set_lds(k_fft_adjoint<G>, lds);
  if (e != hipSuccess) return e;
  const int64_t grid = batch < (int64_t)p->num_cu * 8 ? batch : (int64_t)p->num_cu * 8;
  hipLaunchKernelGGL(k_fft_adjoint<G>, dim3((unsigned)grid), dim3(fft_threads<G>()), lds, st, y, psi,
                     static_cast<const float2*>(p->fft_tw), batch);
  return hipGetLastError();
}

template <class G>
static hipError_t pie_fft(const PieArgs& a, int c0, int cnt, hipStream_t st) {
  const size_t lds = fft_lds_bytes<G>();
  const dim3 grid(cnt), block(fft_threads<G>());
  hipError_t e;
  if (cnt == 1 && (a.norm || a.probe_step)) {
    if ((e = set_lds(k_pie_fft<G, true, true>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_pie_fft<G, true, true>), grid, block, lds, st, a, c0);
  } else if (cnt == 1) {
    if ((e = set_lds(k_pie_fft<G, true, false>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_pie_fft<G, true, false>), grid, block, lds, st, a, c0);
  } else {
    if ((e = set_lds(k_pie_fft<G, false, false>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_pie_fft<G, false, false>), grid, block, lds, st, a, c0);
  }
  return hipGetLastError();
}

bool fft_supported(int n, int m) { return n == m && (n == 16 || n == 32 || n == 64 || n == 128); }

hipError_t launch_fft_forward(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch, hipStream_t st) {
  if (batch == 0) return hipSuccess;
  switch (p->n) {
    case 16: return fft_fwd<FftGeom<4, 4>>(p, psi, y, batch, st);
    case 32: return fft_fwd<FftGeom<4, 8>>(p, psi, y, batch, st);
    case 64: return fft_fwd<FftGeom<8, 8>>(p, psi, y, batch, st);
    case 128: return fft_fwd<FftGeom<8, 16>>(p, psi, y, batch, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fft_adjoint(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch, hipStream_t st) {
  if (batch == 0) return hipSuccess;
  switch (p->n) {
    case 16: return fft_adj<FftGeom<4, 4>>(p, y, psi, batch, st);
    case 32: return fft_adj<FftGeom<4, 8>>(p, y, psi, batch, st);
    case 64: return fft_adj<FftGeom<8, 8>>(p, y, psi, batch, st);
    case 128: return fft_adj<FftGeom<8, 16>>(p, y, psi, batch, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pie_fft_chunk(const PieArgs& a, int c0, int cnt, hipStream_t st) {
  switch (a.n) {
    case 16: return pie_fft<FftGeom<4, 4>>(a, c0, cnt, st);
    case 32: return pie_fft<FftGeom<4, 8>>(a, c0, cnt, st);
    case 64: return pie_fft<FftGeom<8, 8>>(a, c0, cnt, st);
    case 128: return pie_fft<FftGeom<8, 16>>(a, c0, cnt, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace pftpie
