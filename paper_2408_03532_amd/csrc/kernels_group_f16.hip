// Uneven-batch persistent kernels in F16 (forward and adjoint).
#include "group_kernels.hpp"

namespace pftpie {

void* group_kernel_f16(int adjoint) {
  return adjoint ? reinterpret_cast<void*>(&k_group<PrecF16, true>) : reinterpret_cast<void*>(&k_group<PrecF16, false>);
}

}  // namespace pftpie
