// Uneven-batch persistent kernels in BF16 (forward and adjoint).
#include "group_kernels.hpp"

namespace pftpie {

void* group_kernel_bf16(int adjoint) {
  return adjoint ? reinterpret_cast<void*>(&k_group<PrecBF16, true>) : reinterpret_cast<void*>(&k_group<PrecBF16, false>);
}

}  // namespace pftpie
