// Kernel-side argument block of the PIE sweep and the amplitude loss, and
// the scan object.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
  float2* dpsi;     // [batch][n][n] corrections (chunks of more than one position)
  double* phi_part; // [J][4]
  int32_t* rank;    // [J] place of each position in the sweep order
  unsigned* winmax; // [J][2] float bits of max |P|^2, max |O_j|^2 over the window (single-position chunks)
  float2* O0;       // [H][W] object at sweep start
  float2* numO;     // [H][W] (norm 1, multi-position chunks)
  double* D;        // [H][W]
  float2* numP;     // [n][n] (probe step, multi-position chunks)
  double* E;        // [n][n]
  double* maxpart;  // [tiles + probe blocks] per-block maxima of D and E
  double* maxes;    // [2]
  double* red;      // [kStatBlocks][3] statistics partials
  double* stats;    // [4]
};

constexpr int kStatBlocks = 512;

// Forward work split of the dense sweep for MT = ceil(m/16) tiles per axis:
// CT column tiles per wave, WC column groups, WR row groups per workgroup.
inline int pie_ct(int mt) { return mt <= 2 ? mt : 2; }
inline int pie_wc(int mt) { return (mt + pie_ct(mt) - 1) / pie_ct(mt); }
inline int pie_wr_rt(int mt) { return mt <= 2 ? 4 : (mt <= 4 ? 2 : 1); }
// Workgroups per position in the forward for chunks of `batch` positions:
// few large windows split their row strips over more workgroups (partial
// spectra summed by a projection kernel) until the chunk has about four
// waves per compute unit, keeping at least one strip per row group, and
// for long windows (nb >= 128) at least eight, so that passes of several
// strips can share the twiddle blocks of the uncached table.
inline int pie_row_splits(int nb, int mt, int batch, int num_cu) {
  const long waves = (long)batch * pie_wc(mt) * pie_wr_rt(mt);
  const long target = 4L * num_cu;
  if (waves >= target) return 1;
  long s = (target + waves - 1) / waves;
  const long cap = nb >= 128 ? nb / (8 * pie_wr_rt(mt)) : nb / pie_wr_rt(mt);
  if (s > cap) s = cap;
  return s < 1 ? 1 : (int)s;
}

hipError_t launch_pie_sweep(const PieArgs& a, int batch, hipStream_t st);
hipError_t launch_crop_amp(const float* I, int J, int n, int m, float* amp, hipStream_t st);
hipError_t launch_pie_fft_chunk(const PieArgs& a, int c0, int cnt, hipStream_t st);
int pie_probe_blocks(int n);

#ifdef __HIPCC__
// psi[k1][k2] = P[k1][k2] * O[r + k1][c + k2]; zero outside the n x n patch.
template <bool EXACT>
struct GatherSrc {
  const float2* __restrict__ O;
  const float2* __restrict__ P;
  int W, n, r, c;
  __device__ __forceinline__ c4 load(int row, int col0) const {
    c4 v;
    const float2* orow = O + (size_t)(r + row) * W + c + col0;
    const float2* prow = P + (size_t)row * n + col0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int col = col0 + s;
      if (EXACT || (row < n && col < n)) {
        v.v[s] = cmul(prow[s], orow[s]);
      } else {
        v.v[s] = make_float2(0.f, 0.f);
      }
    }
    return v;
  }
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
