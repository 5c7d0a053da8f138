// Plain partial transform kernels in F16 (forward and adjoint).
#include "pft_kernels.hpp"

namespace pftpie {

hipError_t launch_forward_f16(const pftpie_plan_s* p, const float2* psi, float2* y, int64_t batch, hipStream_t st) {
  return forward_prec<PrecF16>(p, psi, y, batch, st);
}

hipError_t launch_adjoint_f16(const pftpie_plan_s* p, const float2* y, float2* psi, int64_t batch, hipStream_t st) {
  return adjoint_prec<PrecF16>(p, y, psi, batch, st);
}

}  // namespace pftpie
