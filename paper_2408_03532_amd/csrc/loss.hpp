// Kernel argument block of the amplitude loss and its gradient.
#pragma once

#include "pie.hpp"

namespace pftpie {

struct LossArgs {
  int n, m, nb, mt, J, H, W;
  const int2* pos;
  const void* fa;
  const void* ft;
  size_t fa_bytes, ft_bytes;  // twiddle table sizes (the persistent kernels hold them in LDS)
  int num_cu;
  int prec;
  const float2* O;
  const float2* P;
  const float* amp;
  float2* U;              // forward: where u_j are written (or null)
  const float2* Uc;       // backward: where u_j are read
  double* part;           // [J][4] partial losses
  double* loss;           // [1] or null
  const double* scale_dev;
  float2* gO;
  float2* gP;
  float2* Rbuf;           // [J][n][n] back-projected residuals (backward)
  float2* gPpart;         // [ceil(J / 64)][n][n] partial probe gradients
  int bb_r0, bb_c0, bb_h, bb_w, tiles_x, tiles_y;
  const int32_t* tile_ptr;
  const int32_t* tile_pos;
};

hipError_t launch_loss_forward(const LossArgs& a, hipStream_t st);
hipError_t launch_loss_backward(const LossArgs& a, bool recompute, hipStream_t st);

}  // namespace pftpie
