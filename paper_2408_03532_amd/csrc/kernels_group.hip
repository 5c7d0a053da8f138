// Uneven batch: the counter reset kernel and the choice of the persistent
// kernel by precision (kernels_group_{f32,bf16,f16}.hip).
#include "group.hpp"

namespace pftpie {

void* group_kernel_f32(int adjoint);
void* group_kernel_bf16(int adjoint);
void* group_kernel_f16(int adjoint);

namespace {

__global__ void k_group_reset(unsigned long long* counter) {
  if (threadIdx.x == 0) *counter = 0ull;
}

}  // namespace

void* group_kernel(int prec, int adjoint) {
  if (prec == PFTPIE_SPLIT_BF16) return group_kernel_bf16(adjoint);
  if (prec == PFTPIE_SPLIT_FP16) return group_kernel_f16(adjoint);
  return group_kernel_f32(adjoint);
}

void* group_reset_kernel() { return reinterpret_cast<void*>(&k_group_reset); }

}  // namespace pftpie
