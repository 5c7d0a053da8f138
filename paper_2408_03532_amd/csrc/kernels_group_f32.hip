// Uneven-batch persistent kernels in F32 (forward and adjoint).
#include "group_kernels.hpp"

namespace pftpie {

void* group_kernel_f32(int adjoint) {
  return adjoint ? reinterpret_cast<void*>(&k_group<PrecF32, true>) : reinterpret_cast<void*>(&k_group<PrecF32, false>);
}

}  // namespace pftpie
