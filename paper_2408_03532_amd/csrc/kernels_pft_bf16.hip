// Plain partial transform kernels in BF16 (forward and adjoint).
#include "pft_kernels.hpp"

namespace pftpie {

hipError_t launch_forward_bf16(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch, hipStream_t st) {
  return forward_prec<PrecBF16>(p, psi, y, batch, st);
}

hipError_t launch_adjoint_bf16(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch, hipStream_t st) {
  return adjoint_prec<PrecBF16>(p, y, psi, batch, st);
}

}  // namespace pftpie
