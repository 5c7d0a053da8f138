// Host-side internals shared by the runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pftpie.h"
#include "twiddle.hpp"

namespace pftpie {

constexpr int kMaxN = 8192;             // window pixels per axis
constexpr int kMaxPeriod = 1 << 20;     // DFT length (masked larger fields)
constexpr int kMaxM = 128;  // 8 accumulator tiles per axis
constexpr size_t kMaxLdsTable = 160 * 1024;  // LDS per compute unit on gfx950

// Forward work split for MT = ceil(m/16) output tiles per axis: each wave
// owns CT column tiles, W = ceil(MT / CT) waves per patch.  Valid CT: 1, 2
// (MT >= 2), 3 (MT == 3), 4 (MT == 4).
inline int fwd_ct_default(int mt) { return mt <= 2 ? mt : 2; }
// split precisions: all four column tiles in one wave when m <= 64 (the
// operand split is shared by twice the products)
inline int fwd_ct_default_split(int mt) { return mt == 4 ? 4 : fwd_ct_default(mt); }
inline bool fwd_ct_valid(int mt, int ct) {
  return ct == 1 || (ct == 2 && mt >= 2) || (ct == 3 && mt == 3) || (ct == 4 && mt == 4);
}
// Column tiles allocated in the FA table: enough for every valid split.
inline int fa_ctiles_for(int mt) { return ((mt + 3) / 4) * 4; }
// Adjoint: waves per patch, each taking every W-th column tile.
inline int adj_waves(int nb) { return nb >= 4 ? 4 : nb; }

}  // namespace pftpie

struct pftpie_plan_s {
  int32_t n, m;
  int32_t period;    // DFT length (n, or the size of a masked larger field)
  pftpie_precision prec;
  int nb, mt;        // ceil(n/16), ceil(m/16)
  int fa_ctiles;     // column tiles allocated in FA (covers every forward split)
  int fwd_ct;        // forward column tiles per wave
  int use_lds;       // persistent LDS-table kernel for the plain forward
  int use_lds_adj;   // persistent LDS-table kernel for the plain adjoint
  int adj_k1;        // FP32 adjoint: row tiles per stage-2 step (2 or 4)
  int adj_threads;   // FP32 persistent adjoint: threads per workgroup (512 or 768)
  int adj_patch;     // split adjoint: whole patch per wave when m <= 64 (else tile per wave)
  int method;        // PFTPIE_METHOD_DENSE or PFTPIE_METHOD_FFT (resolved)
  void* fft_tw;      // device W_n^k, k < n (float2), fast-transform plans only
  int num_cu;        // compute units of the plan's device
  int device;
  void* fa;          // device FA table (float4 blocks, or split 16-bit blocks)
  void* ft;          // device FT table
  size_t fa_bytes, ft_bytes;
};

namespace pftpie {

// Live plans, for the per-call grouped transforms: a plan registers at
// creation and leaves at destruction.  find_plan returns a live plan of
// (n, m, prec) with DFT length n on `device`, or null.
void register_plan(pftpie_plan_s* p);
void unregister_plan(pftpie_plan_s* p);
pftpie_plan_s* find_plan(int n, int m, pftpie_precision prec, int device);

// Fills x[0, count) with float pairs uniform in [-1, 1) (timing operands of
// the autotuners; zeros would run the matrix cores at another clock).
hipError_t tune_fill(float2* x, size_t count, uint32_t salt, hipStream_t st);

// Thread-local error message plumbing.
pftpie_status fail(pftpie_status s, const std::string& msg);
pftpie_status hip_fail(hipError_t e, const char* where);

// Launchers (kernels_pft.hip).  Shapes validated by the caller.
hipError_t launch_forward(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch,
                          hipStream_t st);
hipError_t launch_adjoint(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch,
                          hipStream_t st);
// Full-window fast transform (kernels_fft.hip): n = m in {16, 32, 64, 128}.
bool fft_supported(int n, int m);
hipError_t launch_fft_forward(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch,
                              hipStream_t st);
hipError_t launch_fft_adjoint(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch,
                              hipStream_t st);

}  // namespace pftpie
