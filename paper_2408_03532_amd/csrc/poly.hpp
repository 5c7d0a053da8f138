// The polynomial partial Fourier transform object (Sec. 3.1, Algorithms 1-2;
// Appendix A, Algorithms 4-5): host configuration and device tables.
#pragma once

#include "internal.hpp"

constexpr int kPolyMaxQ = 32;   // window block side q = n / p handled per thread
constexpr int kPolyMaxR = 25;   // polynomial terms (the paper's range 1 <= r <= 25)
constexpr int kPolyMaxM = 128;  // kept coefficients per axis

struct pftpie_poly_s {
  int32_t n, m, p, q, r;
  double eps, xi;
  pftpie_plan fft;  // p x p fast transform of the expanded planes
  void* B;          // device float2 [q][r]: w_l (1 - 2j/q)^l
  void* W;          // device float2 [m][r]: (t/p)^l exp(-pi i t / p), t = c - floor(m/2)
};

namespace pftpie {
hipError_t launch_poly_forward(const pftpie_poly_s* pl, const float2* psi, float2* y, int64_t batch, float2* C,
                               float2* Ch, hipStream_t st);
}  // namespace pftpie
