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
//                   The gathers combine their maxima of D and E with
//                   integer atomic maxima (per chunk parity).
//   k_pie_apply     the normalised updates.
// Per sweep: k_pie_begin (object copy, ranks, clears) and the statistics
// pair k_pie_stats_part / k_pie_stats_final (fixed-order sums); for one
// overlap-normalised chunk without probe step k_pie_apply covers the whole
// object and k_pie_stats_final alone follows.
#include "internal.hpp"
#include "pie.hpp"

namespace pftpie {

// the dense-contraction chunk of each precision (kernels_pie_{f32,bf16,f16}.hip)
void pie_chunk_dense_f32(const PieArgs& a, int c0, int cnt, hipStream_t st);
void pie_chunk_dense_bf16(const PieArgs& a, int c0, int cnt, hipStream_t st);
void pie_chunk_dense_f16(const PieArgs& a, int c0, int cnt, hipStream_t st);
int pie_fwd_split_blocks_f32(int mt, bool rs);
int pie_fwd_split_blocks_bf16(int mt, bool rs);
int pie_fwd_split_blocks_f16(int mt, bool rs);
// the whole sequential sweep in one workgroup (kernels_pie_{f32,bf16,f16}.hip)
void pie_sequential_dense_f32(const PieArgs& a, hipStream_t st);
void pie_sequential_dense_bf16(const PieArgs& a, hipStream_t st);
void pie_sequential_dense_f16(const PieArgs& a, hipStream_t st);
// ... with the box, probe, residual and tables in LDS and the statistics in
// the same launch; false when they do not fit
bool pie_sequential_lds_f32(const PieArgs& a, hipStream_t st);
bool pie_sequential_lds_bf16(const PieArgs& a, hipStream_t st);
bool pie_sequential_lds_f16(const PieArgs& a, hipStream_t st);

// ---------------------------------------------------------------------------
// gathers of a chunk's corrections

// Sums of three doubles over the workgroup (fixed order), stored by thread 0
// at out[0..2].
__device__ __forceinline__ void block_sum3(double v0, double v1, double v2, double* out) {
  __shared__ double sh3[3][16];
  v0 = wave_sum(v0);
  v1 = wave_sum(v1);
  v2 = wave_sum(v2);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh3[0][w] = v0;
    sh3[1][w] = v1;
    sh3[2][w] = v2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh3[threadIdx.x][k];
    out[threadIdx.x] = s;
  }
}

// ||new - old||^2, ||old||^2 and non-finite count of one pixel's update.
__device__ __forceinline__ void pixel_stats(float2 ov, float2 nv, double& d2, double& o2, double& bad) {
  const double dx = (double)nv.x - ov.x, dy = (double)nv.y - ov.y;
  d2 += dx * dx + dy * dy;
  o2 += (double)ov.x * ov.x + (double)ov.y * ov.y;
  bad += (isfinite(nv.x) && isfinite(nv.y)) ? 0.0 : 1.0;
}

// max over the workgroup of non-negative doubles into *dst, whose bit
// patterns order as unsigned integers: an integer atomic maximum, exact and
// the same in any order (skipped when *dst is already as large).
__device__ __forceinline__ void atomic_max_nonneg(double* dst, double v) {
  unsigned long long* bits = reinterpret_cast<unsigned long long*>(dst);
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  if (v > 0.0 && __hip_atomic_load(bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < b) atomicMax(bits, b);
}

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
__global__ __launch_bounds__(256) void k_pie_probe_gather(PieArgs a, int c0, int cnt, int par) {
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
          dv[u] = a.dpsi[dpsi_base(a, q, ps.y) + (size_t)k1 * a.dstride + k2];
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
    if (threadIdx.x == 0) atomic_max_nonneg(&a.maxes[2 * par + 1], mx);
  }
}

// Per 16 x 16 object tile of the bounding box: sum over the chunk's positions
// in the tile's cover list.  norm 0: O += beta numO at once; norm 1: store
// numO and D with the tile's maximum of D.
__global__ __launch_bounds__(256) void k_pie_object_gather(PieArgs a, int c0, int cnt, int par) {
  __shared__ double sh[4];
  const int tile = blockIdx.x;
  const int ty = tile / a.tiles_x, tx = tile % a.tiles_x;
  const int py = a.bb_r0 + ty * 16 + (threadIdx.x >> 4);
  const int px = a.bb_c0 + tx * 16 + (threadIdx.x & 15);
  const bool inside = (py < a.bb_r0 + a.bb_h) && (px < a.bb_c0 + a.bb_w);
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
        pv[u] = a.P[(size_t)dy * a.n + dx];
        dv[u] = a.dpsi[dpsi_base(a, qv[u], cv[u].y) + (size_t)dy * a.dstride + dx];
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
    if (a.fuse_stats) {
      double d2 = 0.0, o2 = 0.0, bad = 0.0;
      if (inside) {
        const float2 ov = a.O[o];
        float2 nv = ov;
        if (acc.x != 0.f || acc.y != 0.f) {
          nv = make_float2(ov.x + a.beta * acc.x, ov.y + a.beta * acc.y);
          a.O[o] = nv;
        }
        pixel_stats(ov, nv, d2, o2, bad);
      }
      block_sum3(d2, o2, bad, a.fred + (size_t)tile * 3);
    } else if (inside && (acc.x != 0.f || acc.y != 0.f)) {
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
  if (threadIdx.x == 0) atomic_max_nonneg(&a.maxes[2 * par], mx);
}

// stats = {Phi, ||dO||^2, ||O||^2, non-finite}: the objective parts, `nred`
// statistics partials at red and `nfused` at fred, added in a fixed order by
// one workgroup.
__device__ void stats_sum(const PieArgs& a, int nred, int nfused) {
  __shared__ double sh[4][16];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const size_t np = (size_t)a.J * 4;
  for (size_t t = threadIdx.x; t < np; t += blockDim.x) v[0] += a.phi_part[t];
  auto parts = [&](const double* src, int nb) {
    // four partials per thread in flight, added in block order
    for (int b0 = threadIdx.x; b0 < nb; b0 += 4 * blockDim.x) {
      double t[4][3];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = b0 + u * blockDim.x;
#pragma unroll
        for (int c = 0; c < 3; ++c) t[u][c] = b < nb ? src[(size_t)b * 3 + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c + 1] += t[u][c];
    }
  };
  parts(a.red, nred);
  parts(a.fred, nfused);
  for (int c = 0; c < 4; ++c) v[c] = wave_sum(v[c]);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int c = 0; c < 4; ++c) sh[c][w] = v[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nw; ++k)
      for (int c = 0; c < 4; ++c) t[c] += sh[c][k];
    a.stats[0] = t[0] / ((double)a.J * a.period * a.period);
    a.stats[1] = t[1];
    a.stats[2] = t[2];
    a.stats[3] = t[3];
  }
}

// Normalised object update over the bounding box and the probe update of
// one chunk, with the maxima of the chunk's parity `par` (the other pair is
// cleared for the next chunk).  fold_stats (one chunk, no probe step): the
// object part runs over the whole object, outside the box only summing the
// statistics, so that no statistics pass over the object follows.
__global__ __launch_bounds__(256) void k_pie_apply(PieArgs a, int object_part, int par) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    a.maxes[2 * (par ^ 1)] = 0.0;
    a.maxes[2 * (par ^ 1) + 1] = 0.0;
  }
  if (object_part) {
    const double regO = a.alpha * a.maxes[2 * par];
    double d2 = 0.0, o2 = 0.0, bad = 0.0;
    const bool fold = a.fold_stats;
    const int r0 = fold ? 0 : a.bb_r0, c0 = fold ? 0 : a.bb_c0;
    const int hh = fold ? a.H : a.bb_h, ww = fold ? a.W : a.bb_w;
    // rows over blockIdx.y, columns over blockIdx.x
    for (int rr = blockIdx.y; rr < hh; rr += gridDim.y) {
      const int y = r0 + rr;
      const bool in_rows = y >= a.bb_r0 && y < a.bb_r0 + a.bb_h;
      for (int cc = blockIdx.x * blockDim.x + threadIdx.x; cc < ww; cc += gridDim.x * blockDim.x) {
        const int x = c0 + cc;
        const size_t o = (size_t)y * a.W + x;
        const double d = (in_rows && x >= a.bb_c0 && x < a.bb_c0 + a.bb_w) ? a.D[o] : 0.0;
        if (d > 0.0) {
          const float sc = (float)((double)a.beta / (d + regO));
          const float2 num = a.numO[o];
          const float2 ov = a.O[o];
          const float2 nv = make_float2(ov.x + sc * num.x, ov.y + sc * num.y);
          a.O[o] = nv;
          if (a.fuse_stats) pixel_stats(ov, nv, d2, o2, bad);
        } else if (a.fuse_stats) {
          const float2 ov = a.O[o];
          pixel_stats(ov, ov, d2, o2, bad);
        }
      }
    }
    if (a.fuse_stats) block_sum3(d2, o2, bad, a.fred + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 3);
  }
  if (a.probe_step) {
    const size_t nn = (size_t)a.n * a.n;
    const double regP = a.alpha * a.maxes[2 * par + 1];
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
  if (!a.fuse_stats)
    for (size_t t = t0; t < total; t += stride) a.O0[t] = a.O[t];
  for (size_t t = t0; t < (size_t)a.J; t += stride) {
    a.rank[t] = a.order ? kRankAbsent : (int)t;
    a.winmax[2 * t] = 0u;
    a.winmax[2 * t + 1] = 0u;
  }
  for (size_t t = t0; t < (size_t)a.J * 4; t += stride) a.phi_part[t] = 0.0;
  if (t0 == 0)
    for (int k = 0; k < 4; ++k) a.maxes[k] = 0.0;
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
  if (a.fuse_stats) {
    // the box was summed by the update; outside it the object is unchanged:
    // rows over workgroups, and in the box's rows only the columns beside it
    for (int y = blockIdx.x; y < a.H; y += gridDim.x) {
      const float2* row = a.O + (size_t)y * a.W;
      const bool in_rows = y >= a.bb_r0 && y < a.bb_r0 + a.bb_h;
      const int xa = in_rows ? a.bb_c0 : a.W, xb = in_rows ? a.bb_c0 + a.bb_w : a.W;
      for (int x = threadIdx.x; x < xa; x += blockDim.x) pixel_stats(row[x], row[x], d2, o2, bad);
      for (int x = xb + threadIdx.x; x < a.W; x += blockDim.x) pixel_stats(row[x], row[x], d2, o2, bad);
    }
  } else {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
      const float2 o = a.O[t], z = a.O0[t];
      pixel_stats(z, o, d2, o2, bad);
    }
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

// stats after the statistics partials (kStatBlocks at red, nfused at fred).
__global__ __launch_bounds__(1024) void k_pie_stats_final(PieArgs a, int nblocks, int nfused) {
  stats_sum(a, nblocks, nfused);
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

int pie_fwd_split_blocks_per_cu(pftpie_precision prec, int mt, bool rs) {
  if (prec == PFTPIE_SPLIT_BF16) return pie_fwd_split_blocks_bf16(mt, rs);
  if (prec == PFTPIE_SPLIT_FP16) return pie_fwd_split_blocks_f16(mt, rs);
  return pie_fwd_split_blocks_f32(mt, rs);
}

int pie_probe_blocks(int n) { return (int)(((size_t)n * n + 255) / 256); }

hipError_t launch_crop_amp(const float* I, int J, int n, int m, float* amp, hipStream_t st) {
  hipLaunchKernelGGL(k_crop_amp, dim3(ew_blocks((size_t)J * m * m)), dim3(256), 0, st, I, J, n, m, amp);
  return hipGetLastError();
}

hipError_t launch_pie_sweep(const PieArgs& a, int batch, hipStream_t st) {
  const size_t obj = (size_t)a.H * a.W;
  if (batch == 1 && !a.fft_tw && a.nb <= kSeqMaxNb && a.mt <= 2) {
    // sequential sweep of small windows held in LDS: one launch per sweep
    bool done;
    if (a.prec == PFTPIE_SPLIT_BF16)
      done = pie_sequential_lds_bf16(a, st);
    else if (a.prec == PFTPIE_SPLIT_FP16)
      done = pie_sequential_lds_f16(a, st);
    else
      done = pie_sequential_lds_f32(a, st);
    if (done) return hipGetLastError();
  }
  // (the object copy only where the statistics need it; else the per-position
  // slots alone)
  hipLaunchKernelGGL(k_pie_begin, dim3(ew_blocks(a.fuse_stats ? (size_t)a.J * 4 : obj)), dim3(256), 0, st, a);
  if (a.order) hipLaunchKernelGGL(k_pie_rank, dim3(ew_blocks((size_t)a.J)), dim3(256), 0, st, a);
  const int ntiles = a.tiles_x * a.tiles_y;
  const int pblocks = pie_probe_blocks(a.n);
  auto run_chunk = [&](const PieArgs& ca, int c0, int cnt) -> hipError_t {
    if (ca.fft_tw) return launch_pie_fft_chunk(ca, c0, cnt, st);
    if (ca.mt < 1 || ca.mt > 8) return hipErrorInvalidValue;
    if (ca.prec == PFTPIE_SPLIT_BF16)
      pie_chunk_dense_bf16(ca, c0, cnt, st);
    else if (ca.prec == PFTPIE_SPLIT_FP16)
      pie_chunk_dense_f16(ca, c0, cnt, st);
    else
      pie_chunk_dense_f32(ca, c0, cnt, st);
    return hipSuccess;
  };
  if (batch == 1 && !a.fft_tw && a.nb <= kSeqMaxNb && a.mt <= 2) {
    // sequential sweep of small windows: one persistent workgroup
    if (a.prec == PFTPIE_SPLIT_BF16)
      pie_sequential_dense_bf16(a, st);
    else if (a.prec == PFTPIE_SPLIT_FP16)
      pie_sequential_dense_f16(a, st);
    else
      pie_sequential_dense_f32(a, st);
    hipLaunchKernelGGL(k_pie_stats_part, dim3(kStatBlocks), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_pie_stats_final, dim3(1), dim3(1024), 0, st, a, kStatBlocks, 0);
    return hipGetLastError();
  }
  // eq. (6) as printed (single positions): the object step, then a second
  // transform pair at the updated object for the probe step
  PieArgs obj_pass = a, probe_pass = a;
  obj_pass.probe_step = 0;
  probe_pass.probe_pass = 1;
  int nfused = 0;  // statistics partials written by the update (single-chunk sweeps)
  bool stats_done = false;
  for (int c0 = 0; c0 < a.J; c0 += batch) {
    const int cnt = (a.J - c0 < batch) ? a.J - c0 : batch;
    const int par = (c0 / batch) & 1;  // maxima pair of this chunk
    hipError_t e;
    if (a.probe_literal) {
      if ((e = run_chunk(obj_pass, c0, cnt)) != hipSuccess) return e;
      if ((e = run_chunk(probe_pass, c0, cnt)) != hipSuccess) return e;
    } else if ((e = run_chunk(a, c0, cnt)) != hipSuccess) {
      return e;
    }
    if (cnt == 1) continue;  // updated in place
    if (a.probe_step) hipLaunchKernelGGL(k_pie_probe_gather, dim3(pblocks), dim3(256), 0, st, a, c0, cnt, par);
    hipLaunchKernelGGL(k_pie_object_gather, dim3(ntiles), dim3(256), 0, st, a, c0, cnt, par);
    if (a.fuse_stats && !a.norm) nfused = ntiles;
    if (a.norm || a.probe_step) {
      // object part: columns (of the bounding box, or of the whole object
      // when the statistics are folded in) over x, rows over y; the probe
      // part runs over the flattened grid
      int gx = 1, gy = 1;
      if (a.norm) {
        gx = ((a.fold_stats ? a.W : a.bb_w) + 255) / 256;
        gy = a.fold_stats ? a.H : a.bb_h;
        if (gx > 64) gx = 64;
        if (gy > 4096 / gx) gy = 4096 / gx;
      }
      const int pb = a.probe_step ? ew_blocks((size_t)a.n * a.n) : 1;
      if (gx * gy < pb) gy = (pb + gx - 1) / gx;
      hipLaunchKernelGGL(k_pie_apply, dim3(gx, gy), dim3(256), 0, st, a, a.norm, par);
      if (a.fuse_stats && a.norm) nfused = gx * gy;
      stats_done = a.fold_stats;
    }
  }
  if (!stats_done) hipLaunchKernelGGL(k_pie_stats_part, dim3(kStatBlocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_pie_stats_final, dim3(1), dim3(1024), 0, st, a, stats_done ? 0 : kStatBlocks, nfused);
  return hipGetLastError();
}

}  // namespace pftpie
