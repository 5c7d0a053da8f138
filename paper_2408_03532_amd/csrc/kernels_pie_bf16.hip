// PIE sweep, dense contraction in BF16: the per-chunk forward / projection
// and adjoint / update kernels of this precision.
#include "pie_dense.hpp"

namespace pftpie {

void pie_chunk_dense_bf16(const PieArgs& a, int c0, int cnt, hipStream_t st) { chunk_dense<PrecBF16>(a, c0, cnt, st); }

int pie_fwd_split_blocks_bf16(int mt, bool rs) { return fwd_split_blocks_mt<PrecBF16>(mt, rs); }

void pie_sequential_dense_bf16(const PieArgs& a, hipStream_t st) { sequential_dense<PrecBF16>(a, st); }

bool pie_sequential_lds_bf16(const PieArgs& a, hipStream_t st) {
  return sequential_lds_dense<PrecBF16>(a, a.fa_bytes, a.ft_bytes, st);
}

}  // namespace pftpie
