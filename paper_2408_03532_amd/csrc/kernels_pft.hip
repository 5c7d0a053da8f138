// Plain batched partial transform: the choice of the kernels by precision
// (kernels_pft_{f32,bf16,f16}.hip).
#include "internal.hpp"

namespace pftpie {

hipError_t launch_forward_f32(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch, hipStream_t st);
hipError_t launch_forward_bf16(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch, hipStream_t st);
hipError_t launch_forward_f16(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch, hipStream_t st);
hipError_t launch_adjoint_f32(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch, hipStream_t st);
hipError_t launch_adjoint_bf16(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch, hipStream_t st);
hipError_t launch_adjoint_f16(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch, hipStream_t st);

hipError_t launch_forward(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch, hipStream_t st) {
  if (p->prec == PFTPIE_SPLIT_BF16) return launch_forward_bf16(p, psi, y, batch, st);
  if (p->prec == PFTPIE_SPLIT_FP16) return launch_forward_f16(p, psi, y, batch, st);
  return launch_forward_f32(p, psi, y, batch, st);
}

hipError_t launch_adjoint(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch, hipStream_t st) {
  if (p->prec == PFTPIE_SPLIT_BF16) return launch_adjoint_bf16(p, y, psi, batch, st);
  if (p->prec == PFTPIE_SPLIT_FP16) return launch_adjoint_f16(p, y, psi, batch, st);
  return launch_adjoint_f32(p, y, psi, batch, st);
}

}  // namespace pftpie
