// Host-only declarations of the twiddle-table builder (no HIP dependency).
#pragma once

#include <cstdint>
#include <vector>

namespace pftpie {

inline int ceil16(int x) { return (x + 15) / 16; }

// Twiddle tables in kernel tile order (see pft_engine.hpp) for windows of n
// pixels per axis and DFT length `period` (>= n).  Built in double on the
// host, rounded to float once.  FA: fa_ctiles x NB blocks, FT: NB x MT
// blocks, 512 floats (128 float4) per block.
void build_twiddle_tables(int n, int m, int period, int fa_ctiles, std::vector<float>& fa,
                          std::vector<float>& ft);

// Split tables for the 16-bit MFMA path: same block grid, 2048 bytes per
// block = two planes (hi parts, lo parts) of 64 lanes x 8 values
// (re_s, im_s), s = 0..3.  kind: 1 = bfloat16, 2 = IEEE half.  Each twiddle
// is rounded to float first; hi = RNE16(f), lo = RNE16(f - hi).
void build_split_tables(int n, int m, int period, int fa_ctiles, int kind, std::vector<uint16_t>& fa,
                        std::vector<uint16_t>& ft);

// Twiddles of the full-window fast transform: tw[2k], tw[2k+1] = re, im of
// exp(-2 pi i k / n), k < n, computed in double and rounded once.
void build_fft_twiddles(int n, std::vector<float>& tw);

// Round-to-nearest-even conversions used by the split tables.
uint16_t f32_to_bf16_rne(float x);
float bf16_to_f32(uint16_t h);
uint16_t f32_to_f16_rne(float x);
float f16_to_f32(uint16_t h);

}  // namespace pftpie
