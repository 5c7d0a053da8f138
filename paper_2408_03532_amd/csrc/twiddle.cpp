// Partial DFT matrix F_m[c][k] = exp(-2 pi i t_c k / n), t_c = c - floor(m/2)
// (the DFT kernel of Sec. 3.1.1 restricted to the kept window), built in
// double and laid out in the kernels' tile order.  The phase t_c * k is
// reduced modulo n in 64-bit integers before the trigonometric call so the
// angle stays in [0, 2 pi) whatever the sizes.
#include <cmath>
#include <cstdint>
#include <vector>

#include "twiddle.hpp"

namespace pftpie {

namespace {

struct cd {
  double re, im;
};

cd twiddle(int n, int m, int c, int k) {
  if (c >= m || k >= n) return {0.0, 0.0};
  const int64_t t = (int64_t)c - (int64_t)(m / 2);
  int64_t p = (t * (int64_t)k) % n;
  if (p < 0) p += n;
  const double ang = 2.0 * M_PI * (double)p / (double)n;
  return {std::cos(ang), -std::sin(ang)};
}

// One 2 KB block: lane l gets entries s = 0..3; plane (s / 2) holds float4
// {re_s, im_s, re_{s+1}, im_{s+1}} for s even, lane-major.
template <class F>
void put_block(float* blk, F entry) {
  for (int lane = 0; lane < 64; ++lane) {
    for (int s = 0; s < 4; ++s) {
      cd v = entry(lane & 15, lane >> 4, s);
      float* q = blk + ((s / 2) * 64 + lane) * 4 + (s % 2) * 2;
      q[0] = (float)v.re;  // round to nearest even
      q[1] = (float)v.im;
    }
  }
}

}  // namespace

void build_twiddle_tables(int n, int m, int fa_ctiles, std::vector<float>& fa, std::vector<float>& ft) {
  const int nb = ceil16(n), mt = ceil16(m);
  fa.assign((size_t)fa_ctiles * nb * 128 * 4, 0.f);
  ft.assign((size_t)nb * mt * 128 * 4, 0.f);
  for (int ct = 0; ct < fa_ctiles; ++ct)
    for (int kb = 0; kb < nb; ++kb)
      put_block(&fa[((size_t)ct * nb + kb) * 512], [&](int r16, int g, int s) {
        return twiddle(n, m, ct * 16 + r16, kb * 16 + 4 * g + s);
      });
  for (int kt = 0; kt < nb; ++kt)
    for (int cb = 0; cb < mt; ++cb)
      put_block(&ft[((size_t)kt * mt + cb) * 512], [&](int r16, int g, int s) {
        return twiddle(n, m, cb * 16 + 4 * g + s, kt * 16 + r16);
      });
}

}  // namespace pftpie
