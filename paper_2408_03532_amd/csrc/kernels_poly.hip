// The paper's polynomial partial Fourier transform on the device (Sec. 3.1,
// Algorithms 2 and 5): an alternative to the exact dense contraction, kept
// for comparison of error and speed.
//
// With n = p q, window corners split k = q k' + j per axis:
//   C[k1'][k2'][l1][l2] = sum_{j1, j2} Z[q k1' + j1][q k2' + j2] B[j1][l1] B[j2][l2]
//   C^[., ., l1, l2]    = the p x p 2-D DFT over (k1', k2')
//   y[c1][c2]           = sum_{l1, l2} C^[t1 mod p][t2 mod p][l1][l2] W[c1][l1] W[c2][l2]
// for the kept frequencies t_c = c - floor(m/2).  C and C^ live in a
// workspace as [batch][l1][l2][p][p] planes; the 2-D DFTs are the in-LDS fast
// transform (which stores its output in centred order, t at (t + p/2) mod p).
#include "internal.hpp"
#include "poly.hpp"

namespace pftpie {

// One thread per (patch, k1', k2', l1): the row contraction over j1 for this
// l1, then every l2.  Consecutive threads take consecutive k2', so each
// store of a (l1, l2) plane row is contiguous.
__global__ __launch_bounds__(256) void k_poly_expand(const float2* __restrict__ psi, float2* __restrict__ C,
                                                     const float2* __restrict__ B, int n, int p, int q, int r,
                                                     int64_t batch) {
  const int64_t per_patch = (int64_t)r * p * p;
  const int64_t total = batch * per_patch;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = it / per_patch;
    int rem = (int)(it - b * per_patch);
    const int l1 = rem / (p * p);
    rem -= l1 * p * p;
    const int k1 = rem / p, k2 = rem - (rem / p) * p;
    const float2* __restrict__ z = psi + b * (int64_t)n * n + (size_t)(q * k1) * n + q * k2;
    float2 t[kPolyMaxQ];
    for (int j2 = 0; j2 < q; ++j2) t[j2] = make_float2(0.f, 0.f);
    for (int j1 = 0; j1 < q; ++j1) {
      const float2 bw = B[j1 * r + l1];
      const float2* row = z + (size_t)j1 * n;
      for (int j2 = 0; j2 < q; ++j2) {
        const float2 v = row[j2];
        t[j2].x += v.x * bw.x - v.y * bw.y;
        t[j2].y += v.x * bw.y + v.y * bw.x;
      }
    }
    float2* __restrict__ out = C + b * (int64_t)r * r * p * p + (size_t)l1 * r * p * p + (size_t)k1 * p + k2;
    for (int l2 = 0; l2 < r; ++l2) {
      float2 acc = make_float2(0.f, 0.f);
      for (int j2 = 0; j2 < q; ++j2) {
        const float2 bw = B[j2 * r + l2];
        acc.x += t[j2].x * bw.x - t[j2].y * bw.y;
        acc.y += t[j2].x * bw.y + t[j2].y * bw.x;
      }
      out[(size_t)l2 * p * p] = acc;
    }
  }
}

// One thread per (patch, c1, c2): the weighted sum over (l1, l2) of the
// transformed planes at (t1 mod p, t2 mod p); W staged in LDS.
__global__ __launch_bounds__(256) void k_poly_combine(const float2* __restrict__ Ch, float2* __restrict__ y,
                                                      const float2* __restrict__ W, int m, int p, int r,
                                                      int64_t batch) {
  __shared__ float2 w[kPolyMaxM * kPolyMaxR];
  for (int i = threadIdx.x; i < m * r; i += blockDim.x) w[i] = W[i];
  __syncthreads();
  const int64_t total = batch * (int64_t)m * m;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = it / ((int64_t)m * m);
    const int c = (int)(it - b * (int64_t)m * m);
    const int c1 = c / m, c2 = c - (c / m) * m;
    // centred storage of the p-point transform: frequency t sits at (t + p/2) mod p
    const int i1 = ((c1 - m / 2 + p / 2) % p + p) % p;
    const int i2 = ((c2 - m / 2 + p / 2) % p + p) % p;
    const float2* __restrict__ plane = Ch + b * (int64_t)r * r * p * p + (size_t)i1 * p + i2;
    float2 acc = make_float2(0.f, 0.f);
    for (int l1 = 0; l1 < r; ++l1) {
      const float2 w1 = w[c1 * r + l1];
      float2 part = make_float2(0.f, 0.f);
      for (int l2 = 0; l2 < r; ++l2) {
        const float2 v = plane[((size_t)l1 * r + l2) * p * p];
        const float2 w2 = w[c2 * r + l2];
        part.x += v.x * w2.x - v.y * w2.y;
        part.y += v.x * w2.y + v.y * w2.x;
      }
      acc.x += part.x * w1.x - part.y * w1.y;
      acc.y += part.x * w1.y + part.y * w1.x;
    }
    y[it] = acc;
  }
}

static unsigned grid_for(int64_t work) {
  int64_t g = (work + 255) / 256;
  if (g > 65536) g = 65536;
  return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_poly_forward(const pftpie_poly_s* pl, const float2* psi, float2* y, int64_t batch, float2* C,
                               float2* Ch, hipStream_t st) {
  if (batch == 0) return hipSuccess;
  const int p = pl->p, q = pl->q, r = pl->r, n = pl->n, m = pl->m;
  hipLaunchKernelGGL(k_poly_expand, dim3(grid_for(batch * r * p * p)), dim3(256), 0, st, psi, C,
                     static_cast<const float2*>(pl->B), n, p, q, r, batch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_fft_forward(pl->fft, C, Ch, batch * r * r, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_poly_combine, dim3(grid_for(batch * m * m)), dim3(256), 0, st, Ch, y,
                     static_cast<const float2*>(pl->W), m, p, r, batch);
  return hipGetLastError();
}

}  // namespace pftpie
