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
  float inv_n2;
  // parameters
  int norm, probe_step;
  float beta, gamma;
  double alpha;
  // data
  float2* O;        // [H][W]
  float2* P;        // [n][n]
  const float* amp; // [J][m][m]
  // workspace
  float2* R;        // [batch][m][m] residuals u' - u
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
