// PIE / ePIE sweep kernels (Sec. 2.1: projection eq. (3), objective eq. (4),
// iterates eqs. (5)-(6)), built on the MFMA partial-transform engines.
//
// Per chunk of positions (all seeing the object and probe of the chunk start):
//   k_pie_forward   gathers psi = P * O[window] in the operand loader, runs
//                   the forward transform (its row strips split over WR
//                   waves, partial spectra summed through LDS) and applies the
//                   magnitude projection in the epilogue: residual
//                   r = u' - u ([chunk][m][m]) and per-wave sums of
//                   (|u| - a)^2.
//   k_pie_adjoint   dpsi = F^H r conj(F) / n^2.  A single-position chunk (the
//                   sequential iterate of eq. (5)) updates O (and P) in place
//                   in the epilogue: every pixel belongs to exactly one lane,
//                   so no atomics.  Larger chunks store dpsi.
//   k_pie_probe_gather   numP = sum_j conj(O_j) dpsi_j, E = sum_j |O_j|^2 per
//                   probe pixel (ePIE, larger chunks).
//   k_pie_object_gather  per 16 x 16 object tile, the positions of its cover
//                   list that belong to the chunk contribute conj(P) dpsi_j
//                   and |P|^2 (FP64); the plain step is applied at once, the
//                   overlap-normalised one is stored with per-tile maxima.
//   k_pie_reduce_max, k_pie_apply   maxima and the normalised updates.
// Per sweep: k_pie_begin (object copy, ranks, clears) and the statistics
// pair k_pie_stats_part / k_pie_stats_final (fixed-order sums).
#include <atomic>
#include <type_traits>

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

// ---------------------------------------------------------------------------
// gathers of a chunk's corrections

__device__ __forceinline__ double block_max(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r = fmax(r, sh[k]);
  return r;
}

// Per probe pixel: numP = sum_q conj(O_j) dpsi_q, E = sum_q |O_j|^2 over the
// chunk (O as at the chunk start).  Stores both and per-block maxima of E.
__global__ __launch_bounds__(256) void k_pie_probe_gather(PieArgs a, int c0, int cnt) {
  __shared__ double sh[4];
  const size_t nn = (size_t)a.n * a.n;
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (k < nn) {
    const int k1 = (int)(k / a.n), k2 = (int)(k % a.n);
    float2 acc = make_float2(0.f, 0.f);
    // U positions at a time: the loads of the group's valid entries all
    // issue before any is used; contributions are added in chunk order
    constexpr int U = 8;
    for (int qb = 0; qb < cnt; qb += U) {
      float2 ov[U], dv[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = qb + u;
        bool valid = false;
        int2 ps = make_int2(0, 0);
        if (q < cnt) {
          const int j = pos_index(a.order, a.J, c0, q, &valid);
          ps = a.pos[j];
        }
        ok[u] = valid;
        ov[u] = dv[u] = make_float2(0.f, 0.f);
        if (valid) {
          ov[u] = a.O[(size_t)(ps.x + k1) * a.W + ps.y + k2];
          dv[u] = a.dpsi[(size_t)q * nn + k];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!ok[u]) continue;
        const float2 v = cmulc(ov[u], dv[u]);
        acc.x += v.x;
        acc.y += v.y;
        e += (double)ov[u].x * ov[u].x + (double)ov[u].y * ov[u].y;
      }
    }
    a.numP[k] = acc;
    if (a.norm) a.E[k] = e;
  }
  if (a.norm) {
    const double mx = block_max(e, sh);
    if (threadIdx.x == 0) a.maxpart[a.tiles_x * a.tiles_y + blockIdx.x] = mx;
  }
}

// Per 16 x 16 object tile of the bounding box: sum over the chunk's positions
// in the tile's cover list.  norm 0: O += beta numO at once; norm 1: store
// numO and D with the tile's maximum of D.
__global__ __launch_bounds__(256) void k_pie_object_gather(PieArgs a, int c0, int cnt) {
  __shared__ double sh[4];
  const int tile = blockIdx.x;
  const int ty = tile / a.tiles_x, tx = tile % a.tiles_x;
  const int py = a.bb_r0 + ty * 16 + (threadIdx.x >> 4);
  const int px = a.bb_c0 + tx * 16 + (threadIdx.x & 15);
  const bool inside = (py < a.bb_r0 + a.bb_h) && (px < a.bb_c0 + a.bb_w);
  const size_t nn = (size_t)a.n * a.n;
  if (a.norm && tile == 0 && threadIdx.x == 0) {
    // the maxima that k_pie_reduce_max collects next start from zero
    a.maxes[0] = 0.0;
    a.maxes[1] = 0.0;
  }
  float2 acc = make_float2(0.f, 0.f);
  double D = 0.0;
  const int e0 = a.tile_ptr[tile], e1 = a.tile_ptr[tile + 1];
  // U cover-list entries at a time: the loads of the group's entries that
  // reach this pixel are all issued before any is used, then the
  // contributions are added in list order
  constexpr int U = 8;
  for (int eb = e0; eb < e1; eb += U) {
    int qv[U];
    int2 cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      qv[u] = -1;
      cv[u] = make_int2(0, 0);
      if (eb + u < e1) {
        const int j = a.tile_pos[eb + u];
        const int rk = a.rank[j];
        if (rk >= c0 && rk - c0 < cnt) qv[u] = rk - c0;
        cv[u] = a.pos[j];
      }
    }
    float2 pv[U], dv[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int dy = py - cv[u].x, dx = px - cv[u].y;
      ok[u] = inside && qv[u] >= 0 && dy >= 0 && dy < a.n && dx >= 0 && dx < a.n;
      pv[u] = dv[u] = make_float2(0.f, 0.f);
      if (ok[u]) {
        const size_t k = (size_t)dy * a.n + dx;
        pv[u] = a.P[k];
        dv[u] = a.dpsi[(size_t)qv[u] * nn + k];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!ok[u]) continue;
      const float2 v = cmulc(pv[u], dv[u]);
      acc.x += v.x;
      acc.y += v.y;
      D += (double)pv[u].x * pv[u].x + (double)pv[u].y * pv[u].y;
    }
  }
  const size_t o = (size_t)py * a.W + px;
  if (!a.norm) {
    if (inside && (acc.x != 0.f || acc.y != 0.f)) {
      const float2 ov = a.O[o];
      a.O[o] = make_float2(ov.x + a.beta * acc.x, ov.y + a.beta * acc.y);
    }
    return;
  }
  if (inside) {
    a.numO[o] = acc;
    a.D[o] = D;
  }
  const double mx = block_max(inside ? D : 0.0, sh);
  if (threadIdx.x == 0) a.maxpart[tile] = mx;
}

// maxes[0] = max D over the tile maxima, maxes[1] = max E over the probe
// blocks (both cleared by k_pie_object_gather).  The maxima are of
// non-negative doubles, whose bit patterns order as unsigned integers, so
// the blocks combine them with integer atomic maxima: exact, and the same
// in any order.
__global__ __launch_bounds__(256) void k_pie_reduce_max(PieArgs a, int nprobe_blocks) {
  __shared__ double sh[4];
  const int ntiles = a.tiles_x * a.tiles_y;
  double mD = 0.0, mE = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x)
    mD = fmax(mD, a.maxpart[t]);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nprobe_blocks; t += gridDim.x * blockDim.x)
    mE = fmax(mE, a.maxpart[ntiles + t]);
  mD = block_max(mD, sh);
  __syncthreads();
  mE = block_max(mE, sh);
  if (threadIdx.x == 0) {
    unsigned long long* bits = reinterpret_cast<unsigned long long*>(a.maxes);
    if (mD > 0.0) atomicMax(&bits[0], (unsigned long long)__double_as_longlong(mD));
    if (mE > 0.0) atomicMax(&bits[1], (unsigned long long)__double_as_longlong(mE));
  }
}

// Normalised object update over the bounding box and the probe update.
__global__ __launch_bounds__(256) void k_pie_apply(PieArgs a, int object_part) {
  if (object_part) {
    const double regO = a.alpha * a.maxes[0];
    // rows of the bounding box over blockIdx.y, columns over blockIdx.x
    for (int rr = blockIdx.y; rr < a.bb_h; rr += gridDim.y)
    for (int cc = blockIdx.x * blockDim.x + threadIdx.x; cc < a.bb_w; cc += gridDim.x * blockDim.x) {
      const size_t o = (size_t)(a.bb_r0 + rr) * a.W + a.bb_c0 + cc;
      const double d = a.D[o];
      if (d > 0.0) {
        const float sc = (float)((double)a.beta / (d + regO));
        const float2 num = a.numO[o];
        const float2 ov = a.O[o];
        a.O[o] = make_float2(ov.x + sc * num.x, ov.y + sc * num.y);
      }
    }
  }
  if (a.probe_step) {
    const size_t nn = (size_t)a.n * a.n;
    const double regP = a.alpha * a.maxes[1];
    const size_t nthreads = (size_t)gridDim.x * gridDim.y * blockDim.x;
    const size_t t0 = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
    for (size_t t = t0; t < nn; t += nthreads) {
      const float2 num = a.numP[t];
      float sc = a.gamma;
      if (a.norm) {
        const double e = a.E[t];
        sc = (e > 0.0) ? (float)((double)a.gamma / (e + regP)) : 0.f;
      }
      const float2 pv = a.P[t];
      a.P[t] = make_float2(pv.x + sc * num.x, pv.y + sc * num.y);
    }
  }
}

// Sweep start: O0 = O, cleared per-position slots, and the ranks: the scan
// order's own (no order), else every rank cleared to "absent" for
// k_pie_rank to fill, so that a position the order leaves out is never
// gathered from a stale workspace slot.
__global__ __launch_bounds__(256) void k_pie_begin(PieArgs a) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t total = (size_t)a.H * a.W;
  for (size_t t = t0; t < total; t += stride) a.O0[t] = a.O[t];
  for (size_t t = t0; t < (size_t)a.J; t += stride) {
    a.rank[t] = a.order ? kRankAbsent : (int)t;
    a.winmax[2 * t] = 0u;
    a.winmax[2 * t + 1] = 0u;
  }
  for (size_t t = t0; t < (size_t)a.J * 4; t += stride) a.phi_part[t] = 0.0;
}

// rank[order[t]] = t for the entries of the order inside [0, J); a position
// listed twice keeps its first place (the least t), whatever the order in
// which the threads run.
__global__ __launch_bounds__(256) void k_pie_rank(PieArgs a) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < (size_t)a.J; t += stride) {
    const int j = a.order[t];
    if (j >= 0 && j < a.J) atomicMin(&a.rank[j], (int)t);
  }
}

// Statistics partials per block: ||O - O0||^2, ||O0||^2, non-finite count.
__global__ __launch_bounds__(256) void k_pie_stats_part(PieArgs a) {
  __shared__ double sh[3][4];
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
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = d2;
    sh[1][w] = o2;
    sh[2][w] = bad;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[threadIdx.x][k];
    a.red[(size_t)blockIdx.x * 3 + threadIdx.x] = s;
  }
}

// stats = {Phi, ||dO||^2, ||O||^2, non-finite}: one wave, fixed order.
__global__ __launch_bounds__(1024) void k_pie_stats_final(PieArgs a, int nblocks) {
  __shared__ double sh[4][16];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const size_t np = (size_t)a.J * 4;
  for (size_t t = threadIdx.x; t < np; t += blockDim.x) v[0] += a.phi_part[t];
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
    for (int c = 0; c < 3; ++c) v[c + 1] += a.red[(size_t)b * 3 + c];
  for (int c = 0; c < 4; ++c) v[c] = wave_sum(v[c]);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int c = 0; c < 4; ++c) sh[c][w] = v[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nw; ++k)
      for (int c = 0; c < 4; ++c) s[c] += sh[c][k];
    a.stats[0] = s[0] / ((double)a.J * a.period * a.period);
    a.stats[1] = s[1];
    a.stats[2] = s[2];
    a.stats[3] = s[3];
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

static int ew_blocks(size_t work) {
  size_t b = (work + 255) / 256;
  if (b > 4096) b = 4096;
  return b < 1 ? 1 : (int)b;
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

int pie_fwd_split_blocks_per_cu(pftpie_precision prec, int mt, bool rs) {
  if (prec == PFTPIE_SPLIT_BF16) return fwd_split_blocks_mt<PrecBF16>(mt, rs);
  if (prec == PFTPIE_SPLIT_FP16) return fwd_split_blocks_mt<PrecF16>(mt, rs);
  return fwd_split_blocks_mt<PrecF32>(mt, rs);
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

int pie_probe_blocks(int n) { return (int)(((size_t)n * n + 255) / 256); }

hipError_t launch_crop_amp(const float* I, int J, int n, int m, float* amp, hipStream_t st) {
  hipLaunchKernelGGL(k_crop_amp, dim3(ew_blocks((size_t)J * m * m)), dim3(256), 0, st, I, J, n, m, amp);
  return hipGetLastError();
}

hipError_t launch_pie_sweep(const PieArgs& a, int batch, hipStream_t st) {
  const size_t obj = (size_t)a.H * a.W;
  hipLaunchKernelGGL(k_pie_begin, dim3(ew_blocks(obj)), dim3(256), 0, st, a);
  if (a.order) hipLaunchKernelGGL(k_pie_rank, dim3(ew_blocks((size_t)a.J)), dim3(256), 0, st, a);
  const int ntiles = a.tiles_x * a.tiles_y;
  const int pblocks = pie_probe_blocks(a.n);
  auto run_chunk = [&](const PieArgs& ca, int c0, int cnt) -> hipError_t {
    if (ca.fft_tw) return launch_pie_fft_chunk(ca, c0, cnt, st);
    switch (ca.mt) {
      case 1: chunk_mt<1>(ca, c0, cnt, st); break;
      case 2: chunk_mt<2>(ca, c0, cnt, st); break;
      case 3: chunk_mt<3>(ca, c0, cnt, st); break;
      case 4: chunk_mt<4>(ca, c0, cnt, st); break;
      case 5: chunk_mt<5>(ca, c0, cnt, st); break;
      case 6: chunk_mt<6>(ca, c0, cnt, st); break;
      case 7: chunk_mt<7>(ca, c0, cnt, st); break;
      case 8: chunk_mt<8>(ca, c0, cnt, st); break;
      default: return hipErrorInvalidValue;
    }
    return hipSuccess;
  };
  // eq. (6) as printed (single positions): the object step, then a second
  // transform pair at the updated object for the probe step
  PieArgs obj_pass = a, probe_pass = a;
  obj_pass.probe_step = 0;
  probe_pass.probe_pass = 1;
  for (int c0 = 0; c0 < a.J; c0 += batch) {
    const int cnt = (a.J - c0 < batch) ? a.J - c0 : batch;
    hipError_t e;
    if (a.probe_literal) {
      if ((e = run_chunk(obj_pass, c0, cnt)) != hipSuccess) return e;
      if ((e = run_chunk(probe_pass, c0, cnt)) != hipSuccess) return e;
    } else if ((e = run_chunk(a, c0, cnt)) != hipSuccess) {
      return e;
    }
    if (cnt == 1) continue;  // updated in place
    if (a.probe_step) hipLaunchKernelGGL(k_pie_probe_gather, dim3(pblocks), dim3(256), 0, st, a, c0, cnt);
    hipLaunchKernelGGL(k_pie_object_gather, dim3(ntiles), dim3(256), 0, st, a, c0, cnt);
    if (a.norm) {
      const int items = ntiles > pblocks ? ntiles : pblocks;
      int rb = (items + 255) / 256;
      if (rb > 1024) rb = 1024;
      hipLaunchKernelGGL(k_pie_reduce_max, dim3(rb), dim3(256), 0, st, a, a.probe_step ? pblocks : 0);
    }
    if (a.norm || a.probe_step) {
      // object part: columns of the bounding box over x, rows over y; the
      // probe part runs over the flattened grid
      int gx = 1, gy = 1;
      if (a.norm) {
        gx = (a.bb_w + 255) / 256;
        gy = a.bb_h;
        if (gx > 64) gx = 64;
        if (gy > 4096 / gx) gy = 4096 / gx;
      }
      const int pb = a.probe_step ? ew_blocks((size_t)a.n * a.n) : 1;
      if (gx * gy < pb) gy = (pb + gx - 1) / gx;
      hipLaunchKernelGGL(k_pie_apply, dim3(gx, gy), dim3(256), 0, st, a, a.norm);
    }
  }
  hipLaunchKernelGGL(k_pie_stats_part, dim3(kStatBlocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_pie_stats_final, dim3(1), dim3(1024), 0, st, a, kStatBlocks);
  return hipGetLastError();
}

}  // namespace pftpie
