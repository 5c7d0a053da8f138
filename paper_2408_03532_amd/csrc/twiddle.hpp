// Host-only declarations of the twiddle-table builder (no HIP dependency).
#pragma once

#include <vector>

namespace pftpie {

inline int ceil16(int x) { return (x + 15) / 16; }

// Twiddle tables in kernel tile order (see pft_engine.hpp).  Built in double
// on the host, rounded to float once.  FA: fa_ctiles x NB blocks, FT: NB x MT
// blocks, 512 floats (128 float4) per block.
void build_twiddle_tables(int n, int m, int fa_ctiles, std::vector<float>& fa, std::vector<float>& ft);

}  // namespace pftpie
