// Kernel-side argument block of the PIE sweep and the amplitude loss, and
// the scan object.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "internal.hpp"
#ifdef __HIPCC__
#include "device_common.hpp"
#endif

namespace pftpie {

constexpr int kModeDirect = 0;  // norm 0, probe fixed: scatter beta conj(P) dpsi into O
constexpr int kModeAccum = 1;   // accumulate numO (D, numP, E), then apply

struct PieArgs {
  // problem
  int n, m, nb, mt, J, H, W;
  int bb_r0, bb_c0, bb_h, bb_w;  // bounding box of all windows
  int tiles_x, tiles_y;          // 16 x 16 pixel tiles over the bounding box
  const int2* pos;               // [J] (row, col)
  const int32_t* order;          // [J] or null
  const int32_t* tile_ptr;       // [tiles + 1] cover lists (CSR): positions whose window meets the tile
  const int32_t* tile_pos;
  const void* fa;
  const void* ft;
  const float2* fft_tw;  // full-window fast transform twiddles (null: dense contraction)
  size_t fa_bytes, ft_bytes;  // bytes of the twiddle tables
  int prec;
  int period;       // DFT length: n, or the masked field's size
  float inv_n2;     // 1 / period^2 (inverse DFT of the band change)
  // parameters
  int norm, probe_step;
  int probe_literal;  // probe step of eq. (6) at the updated object (second pass)
  int probe_pass;     // 1: this launch is that second pass (probe only, no objective)
  float beta, gamma;
  double alpha;
  // data
  float2* O;        // [H][W]
  float2* P;        // [n][n]
  const float* amp; // [J][m][m]
  // workspace
  float2* R;        // [batch][m][m] residuals u' - u
  float2* part;     // [batch][splits][m][m] partial spectra (row groups split over workgroups)
  int splits;       // workgroups per position in the forward (1: whole window in one)
  int num_cu;       // compute units of the device
  float2* dpsi;     // [batch][n][dstride] corrections (chunks of more than one position), see dpsi_base
  int dstride;      // row stride of a stored correction (complex elements, a multiple of 16)
  double* phi_part; // [J][4]
  int32_t* rank;    // [J] place of each position in the sweep order
  unsigned* winmax; // [J][2] float bits of max |P|^2, max |O_j|^2 over the window (single-position chunks)
  float2* O0;       // [H][W] object at sweep start
  float2* numO;     // [H][W] (norm 1, multi-position chunks)
  double* D;        // [H][W]
  float2* numP;     // [n][n] (probe step, multi-position chunks)
  double* E;        // [n][n]
  double* maxes;    // [2][2] max D, max E of even / odd chunks (combined by integer atomic maxima)
  double* red;      // [kStatBlocks][3] statistics partials
  double* stats;    // [4]
  // single-chunk sweeps: the kernels that update the object also sum
  // ||dO||^2, ||O||^2 and the non-finite count over the bounding box into
  // fred[block][3], so no object copy is taken at the sweep start and the
  // statistics pass reads only the pixels outside the box
  int fuse_stats;
  int fold_stats;   // ... and, overlap-normalised without probe step, k_pie_apply covers the whole object
  double* fred;     // [kFusedRedBlocks or tiles][3]
};

constexpr int kStatBlocks = 2048;
constexpr int kFusedRedBlocks = 4096 + 64;  // the most workgroups k_pie_apply launches
constexpr int32_t kRankAbsent = 0x7fffffff;  // rank of a position the sweep order leaves out
// Sequential sweeps (chunks of one position) of windows up to kSeqMaxNb
// tiles of 16 per axis and up to 32 kept coefficients run in one
// persistent workgroup.
constexpr int kSeqMaxNb = 4;
// LDS a sequential sweep may hold (object box, probe, residual, tables).
constexpr size_t kSeqLdsBytes = 144 * 1024;
constexpr size_t kSeqLdsMaxObject = 1 << 16;  // object pixels

// Forward work split of the dense sweep for MT = ceil(m/16) tiles per axis:
// CT column tiles per wave, WC column groups, WR row groups per workgroup.
inline int pie_ct(int mt) { return mt <= 2 ? mt : 2; }
inline int pie_wc(int mt) { return (mt + pie_ct(mt) - 1) / pie_ct(mt); }
inline int pie_wr_rt(int mt) { return mt <= 4 ? 2 : 1; }
// Long windows split over several workgroups pass four strips at a time over
// each twiddle block when every row group keeps at least eight strips.
inline bool pie_fwd_rs(int nb, int wr, int splits) { return splits > 1 && nb >= 8 * wr * splits; }

// Workgroups per position in the forward for chunks of `batch` positions.
// Few large windows split their row strips over several workgroups (partial
// spectra summed by a projection kernel) while the chunk alone has fewer than
// four waves per compute unit.  The split count s minimises (rounds of
// co-resident workgroups) x (strips per row group), with `slots_plain` /
// `slots_rs` workgroups of the one-strip / four-strip kernels resident on
// the chip at once and strips counted in whole passes of four where those
// apply (rs_ok: FP32, whole tiles); ties keep the smaller s.  Every row group
// keeps at least one strip, and on long windows (nb >= 128) at least eight.
inline int pie_row_splits(int nb, int mt, int batch, int num_cu, long slots_plain, long slots_rs, bool rs_ok) {
  const int wr = pie_wr_rt(mt);
  const long waves = (long)batch * pie_wc(mt) * wr;
  if (waves >= 4L * num_cu) return 1;
  long cap = nb >= 128 ? nb / (8 * wr) : nb / wr;
  if (cap < 1) cap = 1;
  int best = 1;
  long best_cost = -1;
  for (int s = 1; s <= cap; ++s) {
    const bool rs = rs_ok && pie_fwd_rs(nb, wr, s);
    const long slots = std::max(1L, rs ? slots_rs : slots_plain);
    const long rounds = ((long)batch * s + slots - 1) / slots;
    long strips = (nb + (long)wr * s - 1) / ((long)wr * s);
    if (rs) strips = (strips + 3) / 4 * 4;
    const long cost = rounds * strips;
    if (best_cost < 0 || cost < best_cost) {
      best = s;
      best_cost = cost;
    }
  }
  return best;
}

// The least g in [1, gmax] minimising (rounds of co-resident workgroups,
// `slots` at once) x (work units per wave) for `items` x g workgroups of
// `nw` waves sharing `units` units of work per item.
inline int pie_balanced_y(long items, long units, int nw, int gmax, long slots) {
  slots = std::max(1L, slots);
  int best = 1;
  long best_cost = -1;
  for (int g = 1; g <= gmax; ++g) {
    const long rounds = (items * g + slots - 1) / slots;
    const long per = (units + (long)g * nw - 1) / ((long)g * nw);
    const long cost = rounds * per;
    if (best_cost < 0 || cost < best_cost) {
      best = g;
      best_cost = cost;
    }
  }
  return best;
}

// Split-forward workgroups of the one-strip (rs = false) or four-strip
// kernel that one compute unit holds at once (HIP occupancy query).
int pie_fwd_split_blocks_per_cu(pftpie_precision prec, int mt, bool rs);

hipError_t launch_pie_sweep(const PieArgs& a, int batch, hipStream_t st);
hipError_t launch_crop_amp(const float* I, int J, int n, int m, float* amp, hipStream_t st);
hipError_t launch_pie_fft_chunk(const PieArgs& a, int c0, int cnt, hipStream_t st);
int pie_probe_blocks(int n);
// Row stride of a stored correction: n columns after a shift of up to 15.
inline int dpsi_stride(int n) { return (n + 30) / 16 * 16; }

#ifdef __HIPCC__
// Position of entry q of the chunk starting at c0.  An order entry outside
// [0, J) is clamped for addressing and reported through `valid` so that the
// kernels contribute nothing for it.
__device__ __forceinline__ int pos_index(const int32_t* __restrict__ order, int J, int c0, int q, bool* valid) {
  int j = order ? order[c0 + q] : c0 + q;
  const bool ok = (j >= 0 && j < J);
  if (valid) *valid = ok;
  return ok ? j : 0;
}

// Stored correction of chunk entry q at window column c: row k1, column k2
// at dpsi_base + k1 * dstride + k2.  The row is shifted right by
// (c - bb_c0) mod 16 so that each 16-pixel row segment of an object tile
// (tiles start at bb_c0 + 16 t) begins on a 128-byte line; the object gather
// then reads whole lines.
__host__ __device__ __forceinline__ size_t dpsi_base(const PieArgs& a, int q, int c) {
  return (size_t)q * a.n * a.dstride + ((c - a.bb_c0) & 15);
}
// psi[k1][k2] = P[k1][k2] * O[r + k1][c + k2]; zero outside the n x n patch.
// The engines prefetch the raw probe and object values (load_raw) and form
// the products (combine) just before the block's MFMA products.
struct GatherRaw {
  c4 p, o;
};

template <bool EXACT>
struct GatherSrc {
  using Raw = GatherRaw;
  const float2* __restrict__ O;
  const float2* __restrict__ P;
  int W, n, r, c;
  int ldp;  // row stride of P (n, or padded in LDS)
  __device__ __forceinline__ Raw load_raw(int row, int col0) const {
    Raw v;
    const float2* orow = O + (size_t)(r + row) * W + c + col0;
    const float2* prow = P + (size_t)row * ldp + col0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int col = col0 + s;
      if (EXACT || (row < n && col < n)) {
        v.p.v[s] = prow[s];
        v.o.v[s] = orow[s];
      } else {
        v.p.v[s] = v.o.v[s] = make_float2(0.f, 0.f);
      }
    }
    return v;
  }
  __device__ __forceinline__ c4 combine(const Raw& v) const {
    c4 z;
#pragma unroll
    for (int s = 0; s < 4; ++s) z.v[s] = cmul(v.p.v[s], v.o.v[s]);
    return z;
  }
  __device__ __forceinline__ c4 load(int row, int col0) const { return combine(load_raw(row, col0)); }
};

#endif

}  // namespace pftpie

struct pie_scan_s {
  pftpie_plan_s* plan;
  int32_t J, H, W;
  int bb_r0, bb_c0, bb_h, bb_w;
  int tiles_x, tiles_y;
  int2* pos;           // device [J]
  int32_t* tile_ptr;   // device [tiles + 1]
  int32_t* tile_pos;   // device [nnz]
  int64_t nnz;
};
