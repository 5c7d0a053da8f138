// In-LDS 2-D discrete Fourier transforms of n x n complex blocks for the
// full-window case m = n (the second phase of the hybrid method, Algorithm 3,
// Sec. 3.2, where the data are used at full resolution).  There the kept
// window is the whole spectrum and the dense contraction F_m psi F_m^T costs
// 8 n^3 flops per patch against ~5 n^2 log2 n for a fast transform.
//
// Length n = R1 * R2 (16 = 4 x 4, 32 = 4 x 8, 64 = 8 x 8, 128 = 8 x 16) by
// one Cooley-Tukey split per axis:
//   X[k1 + R1 k2] = sum_n2 W_R2^(n2 k2) W_n^(n2 k1) sum_n1 x[R2 n1 + n2] W_R1^(n1 k1)
// Pass A: for each n2, an R1-point transform over n1, times W_n^(n2 k1),
//         written back to the slots R2 k1 + n2 it was read from.
// Pass B: for each k1, an R2-point transform over the slots R2 k1 + n2,
//         written back in place: slot R2 k1 + k2 then holds X[k1 + R1 k2]
//         (digit-reversed order; freq() / slot() convert).
// The unnormalised inverse (the adjoint F^H) runs the conjugate passes in
// the reverse order, B^H then A^H, taking the digit-reversed order back to
// natural order.  Every pass reads and writes the same slots per work item,
// so a pass needs no staging; passes are separated by barriers.  Rows carry
// one pad element per R2 block so the strided slots of pass B along a row
// fall on different LDS banks.
#pragma once

#include "device_common.hpp"

namespace pftpie {

template <int R1_, int R2_>
struct FftGeom {
  static constexpr int R1 = R1_, R2 = R2_, N = R1 * R2;
  static constexpr int LOG_R2 = R2 == 4 ? 2 : (R2 == 8 ? 3 : 4);
  static constexpr int STRIDE = N + N / R2;  // row stride in float2
  static constexpr int ELEMS = N * STRIDE;   // LDS elements of one block
  static_assert((1 << LOG_R2) == R2, "R2 must be 4, 8 or 16");
  __device__ static int at(int r, int c) { return r * STRIDE + c + (c >> LOG_R2); }
  // frequency held in slot p after the forward passes, and its inverse
  __device__ static int freq(int p) { return (p >> LOG_R2) + R1 * (p & (R2 - 1)); }
  __device__ static int slot(int f) { return R2 * (f % R1) + f / R1; }
};

template <int R>
constexpr int bit_reverse(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 conj2(float2 a) { return make_float2(a.x, -a.y); }

// In-register R-point transform (radix-2, decimation in time) with
// W_R^j = tw[j * (N / R)] from the block's twiddle table tw[k] = W_N^k;
// INV uses the conjugate twiddles (unnormalised inverse).
template <int R, int N, bool INV>
__device__ __forceinline__ void dft_small(float2 (&v)[R], const float2* __restrict__ tw) {
  float2 t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) t[bit_reverse<R>(i)] = v[i];
#pragma unroll
  for (int span = 2; span <= R; span *= 2) {
    const int half = span / 2;
#pragma unroll
    for (int k = 0; k < R; k += span)
#pragma unroll
      for (int j = 0; j < half; ++j) {
        float2 b = t[k + j + half];
        if (j != 0) {
          const float2 w = tw[j * (N / span)];
          b = cmul(INV ? conj2(w) : w, b);
        }
        const float2 a = t[k + j];
        t[k + j] = cadd(a, b);
        t[k + j + half] = csub(a, b);
      }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = t[i];
}

// Pass A on the R1 values of sub-sequence n2 (forward: transform, then
// twiddle; inverse: conjugate twiddle, then inverse transform).
template <class G, bool INV>
__device__ __forceinline__ void pass_a_values(float2 (&v)[G::R1], int n2, const float2* __restrict__ tw) {
  if constexpr (!INV) dft_small<G::R1, G::N, false>(v, tw);
#pragma unroll
  for (int k1 = 1; k1 < G::R1; ++k1) {
    const float2 w = tw[(n2 * k1) & (G::N - 1)];
    v[k1] = cmul(INV ? conj2(w) : w, v[k1]);
  }
  if constexpr (INV) dft_small<G::R1, G::N, true>(v, tw);
}

// LDS address of element e of line `line` (a row, or a column).
template <class G, bool ROWS>
__device__ __forceinline__ int line_at(int line, int e) {
  return ROWS ? G::at(line, e) : G::at(e, line);
}

// Work item -> (line, sub-sequence).  Rows: sub-sequences of one line on
// neighbouring lanes; columns: lines on neighbouring lanes (contiguous).
template <class G, bool ROWS, int SUB>
__device__ __forceinline__ void item_split(int it, int& line, int& sub) {
  if (ROWS) {
    line = it / SUB;
    sub = it % SUB;
  } else {
    line = it % G::N;
    sub = it / G::N;
  }
}

template <class G, bool ROWS, bool INV>
__device__ __forceinline__ void lds_pass_a(float2* buf, const float2* __restrict__ tw) {
  constexpr int items = G::N * G::R2;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    int line, n2;
    item_split<G, ROWS, G::R2>(it, line, n2);
    float2 v[G::R1];
#pragma unroll
    for (int n1 = 0; n1 < G::R1; ++n1) v[n1] = buf[line_at<G, ROWS>(line, G::R2 * n1 + n2)];
    pass_a_values<G, INV>(v, n2, tw);
#pragma unroll
    for (int k1 = 0; k1 < G::R1; ++k1) buf[line_at<G, ROWS>(line, G::R2 * k1 + n2)] = v[k1];
  }
}

template <class G, bool ROWS, bool INV>
__device__ __forceinline__ void lds_pass_b(float2* buf, const float2* __restrict__ tw) {
  constexpr int items = G::N * G::R1;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    int line, k1;
    item_split<G, ROWS, G::R1>(it, line, k1);
    float2 v[G::R2];
#pragma unroll
    for (int n2 = 0; n2 < G::R2; ++n2) v[n2] = buf[line_at<G, ROWS>(line, G::R2 * k1 + n2)];
    dft_small<G::R2, G::N, INV>(v, tw);
#pragma unroll
    for (int k2 = 0; k2 < G::R2; ++k2) buf[line_at<G, ROWS>(line, G::R2 * k1 + k2)] = v[k2];
  }
}

// Forward passes after the row pass A (done by the caller from its source):
// row pass B, then both column passes.
template <class G>
__device__ __forceinline__ void fft2_rest_forward(float2* buf, const float2* __restrict__ tw) {
  __syncthreads();
  lds_pass_b<G, true, false>(buf, tw);
  __syncthreads();
  lds_pass_a<G, false, false>(buf, tw);
  __syncthreads();
  lds_pass_b<G, false, false>(buf, tw);
  __syncthreads();
}

// Inverse passes up to the last row pass A^H (done by the caller into its
// sink): column B^H, column A^H, row B^H.
template <class G>
__device__ __forceinline__ void fft2_inverse_head(float2* buf, const float2* __restrict__ tw) {
  __syncthreads();
  lds_pass_b<G, false, true>(buf, tw);
  __syncthreads();
  lds_pass_a<G, false, true>(buf, tw);
  __syncthreads();
  lds_pass_b<G, true, true>(buf, tw);
  __syncthreads();
}

}  // namespace pftpie
