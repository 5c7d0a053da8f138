// Partial DFT matrix F_m[c][k] = exp(-2 pi i t_c k / N), t_c = c - floor(m/2),
// k < n (the DFT kernel of Sec. 3.1.1 restricted to the kept window; N = n,
// or the DFT length of a masked larger field, Sec. 4.1.3), built in double and
// laid out in the kernels' tile order.  The phase t_c * k is reduced modulo
// N in 64-bit integers before the trigonometric call so the angle stays in
// [0, 2 pi) whatever the sizes.
#include <cmath>
#include <cstring>
#include <cstdint>
#include <vector>

#include "twiddle.hpp"

namespace pftpie {

namespace {

struct cd {
  double re, im;
};

// Entry (c, k) of the n-column partial DFT matrix of DFT length `period`
// (period > n: the window of a masked larger field).
cd twiddle(int n, int m, int period, int c, int k) {
  if (c >= m || k >= n) return {0.0, 0.0};
  const int64_t t = (int64_t)c - (int64_t)(m / 2);
  int64_t p = (t * (int64_t)k) % period;
  if (p < 0) p += period;
  const double ang = 2.0 * M_PI * (double)p / (double)period;
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

void build_twiddle_tables(int n, int m, int period, int fa_ctiles, std::vector<float>& fa,
                          std::vector<float>& ft) {
  const int nb = ceil16(n), mt = ceil16(m);
  fa.assign((size_t)fa_ctiles * nb * 128 * 4, 0.f);
  ft.assign((size_t)nb * mt * 128 * 4, 0.f);
  for (int ct = 0; ct < fa_ctiles; ++ct)
    for (int kb = 0; kb < nb; ++kb)
      put_block(&fa[((size_t)ct * nb + kb) * 512], [&](int r16, int g, int s) {
        return twiddle(n, m, period, ct * 16 + r16, kb * 16 + 4 * g + s);
      });
  for (int kt = 0; kt < nb; ++kt)
    for (int cb = 0; cb < mt; ++cb)
      put_block(&ft[((size_t)kt * mt + cb) * 512], [&](int r16, int g, int s) {
        return twiddle(n, m, period, cb * 16 + 4 * g + s, kt * 16 + r16);
      });
}

void build_fft_twiddles(int n, std::vector<float>& tw) {
  tw.assign((size_t)2 * n, 0.f);
  for (int k = 0; k < n; ++k) {
    const double ang = 2.0 * M_PI * (double)k / (double)n;
    tw[2 * k] = (float)std::cos(ang);
    tw[2 * k + 1] = (float)-std::sin(ang);
  }
}

uint16_t f32_to_bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

uint16_t f32_to_f16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  const uint32_t sign = (u >> 16) & 0x8000u;
  const int32_t e = (int32_t)((u >> 23) & 0xff) - 127 + 15;
  uint32_t mant = u & 0x7fffffu;
  if (((u >> 23) & 0xff) == 0xff) return (uint16_t)(sign | 0x7c00u | (mant ? 0x200u : 0u));
  if (e >= 31) return (uint16_t)(sign | 0x7c00u);  // overflow to infinity
  if (e <= 0) {                                     // subnormal half (or zero)
    if (e < -10) return (uint16_t)sign;
    mant |= 0x800000u;
    const int shift = 14 - e;  // 24-bit significand down to the subnormal grid
    uint32_t h = mant >> shift;
    const uint32_t rem = mant & ((1u << shift) - 1u), half = 1u << (shift - 1);
    if (rem > half || (rem == half && (h & 1u))) ++h;
    return (uint16_t)(sign | h);
  }
  uint32_t h = sign | ((uint32_t)e << 10) | (mant >> 13);
  const uint32_t rem = mant & 0x1fffu;
  if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;  // carry may round up the exponent
  return (uint16_t)h;
}

float f16_to_f32(uint16_t h) {
  const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
  const uint32_t e = (h >> 10) & 0x1fu, mant = h & 0x3ffu;
  uint32_t u;
  if (e == 0) {
    if (mant == 0) {
      u = sign;
    } else {  // subnormal: value = mant * 2^-24, exact in float
      float v = std::ldexp((float)mant, -24);
      std::memcpy(&u, &v, 4);
      u |= sign;
    }
  } else if (e == 31) {
    u = sign | 0x7f800000u | (mant << 13);
  } else {
    u = sign | ((e - 15 + 127) << 23) | (mant << 13);
  }
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

namespace {

template <class F>
void put_split_block(uint16_t* blk, int kind, F entry) {
  for (int lane = 0; lane < 64; ++lane) {
    for (int s = 0; s < 4; ++s) {
      const cd v = entry(lane & 15, lane >> 4, s);
      const float parts[2] = {(float)v.re, (float)v.im};
      for (int c = 0; c < 2; ++c) {
        const float f = parts[c];
        uint16_t hi, lo;
        if (kind == 1) {
          hi = f32_to_bf16_rne(f);
          lo = f32_to_bf16_rne(f - bf16_to_f32(hi));
        } else {
          hi = f32_to_f16_rne(f);
          lo = f32_to_f16_rne(f - f16_to_f32(hi));
        }
        blk[lane * 8 + 2 * s + c] = hi;
        blk[512 + lane * 8 + 2 * s + c] = lo;
      }
    }
  }
}

}  // namespace

void build_split_tables(int n, int m, int period, int fa_ctiles, int kind, std::vector<uint16_t>& fa,
                        std::vector<uint16_t>& ft) {
  const int nb = ceil16(n), mt = ceil16(m);
  fa.assign((size_t)fa_ctiles * nb * 1024, 0);
  ft.assign((size_t)nb * mt * 1024, 0);
  for (int ct = 0; ct < fa_ctiles; ++ct)
    for (int kb = 0; kb < nb; ++kb)
      put_split_block(&fa[((size_t)ct * nb + kb) * 1024], kind, [&](int r16, int g, int s) {
        return twiddle(n, m, period, ct * 16 + r16, kb * 16 + 4 * g + s);
      });
  for (int kt = 0; kt < nb; ++kt)
    for (int cb = 0; cb < mt; ++cb)
      put_split_block(&ft[((size_t)kt * mt + cb) * 1024], kind, [&](int r16, int g, int s) {
        return twiddle(n, m, period, cb * 16 + 4 * g + s, kt * 16 + r16);
      });
}

}  // namespace pftpie
