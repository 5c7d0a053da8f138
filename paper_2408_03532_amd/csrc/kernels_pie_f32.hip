// PIE sweep, dense contraction in F32: the per-chunk forward / projection
// and adjoint / update kernels of this precision.
#include "pie_dense.hpp"

namespace pftpie {

void pie_chunk_dense_f32(const PieArgs& a, int c0, int cnt, hipStream_t st) { chunk_dense<PrecF32>(a, c0, cnt, st); }

int pie_fwd_split_blocks_f32(int mt, bool rs) { return fwd_split_blocks_mt<PrecF32>(mt, rs); }

void pie_sequential_dense_f32(const PieArgs& a, hipStream_t st) { sequential_dense<PrecF32>(a, st); }

bool pie_sequential_lds_f32(const PieArgs& a, hipStream_t st) {
  return sequential_lds_dense<PrecF32>(a, a.fa_bytes, a.ft_bytes, st);
}

}  // namespace pftpie
