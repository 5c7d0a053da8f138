// C ABI of the polynomial partial Fourier transform: configuration on the
// host in double (Algorithm 1 per axis), device tables, launch.
#include <cmath>
#include <complex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"
#include "poly.hpp"

namespace pftpie {
namespace {

typedef std::complex<double> cplx;

// Interpolant of exp(i pi x) at the r Chebyshev points of [-xi, xi], as
// monomial coefficients: the Vandermonde system solved by Gaussian
// elimination with partial pivoting.
std::vector<cplx> chebyshev_poly(double xi, int r) {
  std::vector<cplx> A((size_t)r * r), f(r);
  for (int i = 0; i < r; ++i) {
    const double x = xi * std::cos(M_PI * (i + 0.5) / r);
    double pw = 1.0;
    for (int k = 0; k < r; ++k) {
      A[(size_t)i * r + k] = pw;
      pw *= x;
    }
    f[i] = cplx(std::cos(M_PI * x), std::sin(M_PI * x));
  }
  for (int c = 0; c < r; ++c) {
    int piv = c;
    for (int i = c + 1; i < r; ++i)
      if (std::abs(A[(size_t)i * r + c]) > std::abs(A[(size_t)piv * r + c])) piv = i;
    if (piv != c) {
      for (int k = 0; k < r; ++k) std::swap(A[(size_t)c * r + k], A[(size_t)piv * r + k]);
      std::swap(f[c], f[piv]);
    }
    for (int i = c + 1; i < r; ++i) {
      const cplx g = A[(size_t)i * r + c] / A[(size_t)c * r + c];
      for (int k = c; k < r; ++k) A[(size_t)i * r + k] -= g * A[(size_t)c * r + k];
      f[i] -= g * f[c];
    }
  }
  std::vector<cplx> w(r);
  for (int i = r - 1; i >= 0; --i) {
    cplx s = f[i];
    for (int k = i + 1; k < r; ++k) s -= A[(size_t)i * r + k] * w[k];
    w[i] = s / A[(size_t)i * r + i];
  }
  return w;
}

// max |P(x) - exp(i pi x)| on 4001 equispaced points of [-xi, xi] (Horner)
double poly_error(const std::vector<cplx>& w, double xi) {
  double worst = 0.0;
  const int npts = 4001;
  for (int i = 0; i < npts; ++i) {
    const double x = -xi + 2.0 * xi * i / (npts - 1);
    cplx v = 0.0;
    for (int k = (int)w.size() - 1; k >= 0; --k) v = v * x + w[k];
    worst = std::max(worst, std::abs(v - cplx(std::cos(M_PI * x), std::sin(M_PI * x))));
  }
  return worst;
}

// xi(eps, r): the largest scope whose interpolant stays within eps (bisection)
double xi_of(double eps, int r) {
  double lo = 0.0, hi = 64.0;
  if (poly_error(chebyshev_poly(hi, r), hi) <= eps) return hi;
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (poly_error(chebyshev_poly(mid, r), mid) <= eps)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

pftpie_status check_poly(const pftpie_poly_s* pl) {
  if (!pl) return fail(PFTPIE_E_INVALID, "poly: object is NULL");
  return PFTPIE_OK;
}

}  // namespace
}  // namespace pftpie

using namespace pftpie;

extern "C" {

pftpie_status pftpie_poly_create(int32_t n, int32_t m, int32_t p, double eps, pftpie_poly* out) {
  if (!out) return fail(PFTPIE_E_INVALID, "poly_create: out is NULL");
  *out = nullptr;
  if (!(eps > 0.0 && eps < 1.0)) return fail(PFTPIE_E_INVALID, "poly_create: need 0 < eps < 1");
  if (n < 1 || n > kMaxN || m < 1 || m > n) return fail(PFTPIE_E_INVALID, "poly_create: need 1 <= m <= n <= 8192");
  if (p != 16 && p != 32 && p != 64 && p != 128)
    return fail(PFTPIE_E_UNSUPPORTED, "poly_create: p must be 16, 32, 64 or 128");
  if (n % p) return fail(PFTPIE_E_INVALID, "poly_create: p must divide n");
  const int q = n / p;
  if (q > kPolyMaxQ) return fail(PFTPIE_E_UNSUPPORTED, "poly_create: n / p above 32 is not supported");
  if (m > kPolyMaxM) return fail(PFTPIE_E_UNSUPPORTED, "poly_create: m above 128 is not supported");
  // Algorithm 1, line 2: the least r with xi(eps, r) >= m~ / p, m~ = floor(m/2)
  const double ratio = (double)(m / 2) / p;
  int r = 0;
  double xi = 0.0;
  for (int rr = 1; rr <= kPolyMaxR; ++rr) {
    xi = xi_of(eps, rr);
    if (xi >= ratio) {
      r = rr;
      break;
    }
  }
  if (r == 0) return fail(PFTPIE_E_UNSUPPORTED, "poly_create: no r <= 25 reaches eps for m/2 / p");
  const std::vector<cplx> w = chebyshev_poly(xi, r);
  std::vector<float> B((size_t)q * r * 2), W((size_t)m * r * 2);
  for (int j = 0; j < q; ++j) {
    const double x = 1.0 - 2.0 * j / q;
    double pw = 1.0;
    for (int l = 0; l < r; ++l) {
      const cplx v = w[l] * pw;
      B[((size_t)j * r + l) * 2] = (float)v.real();
      B[((size_t)j * r + l) * 2 + 1] = (float)v.imag();
      pw *= x;
    }
  }
  for (int c = 0; c < m; ++c) {
    const double t = (double)(c - m / 2);
    const cplx ph(std::cos(M_PI * t / p), -std::sin(M_PI * t / p));
    double pw = 1.0;
    for (int l = 0; l < r; ++l) {
      const cplx v = ph * pw;
      W[((size_t)c * r + l) * 2] = (float)v.real();
      W[((size_t)c * r + l) * 2 + 1] = (float)v.imag();
      pw *= t / p;
    }
  }
  pftpie_poly_s* pl = new (std::nothrow) pftpie_poly_s();
  if (!pl) return fail(PFTPIE_E_NOMEM, "poly_create: host allocation failed");
  pl->n = n;
  pl->m = m;
  pl->p = p;
  pl->q = q;
  pl->r = r;
  pl->eps = eps;
  pl->xi = xi;
  if (pftpie_status s = pftpie_plan_create_method(p, p, PFTPIE_FP32, PFTPIE_METHOD_FFT, &pl->fft)) {
    delete pl;
    return s;
  }
  hipError_t e = hipMalloc(&pl->B, B.size() * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&pl->W, W.size() * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(pl->B, B.data(), B.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pl->W, W.data(), W.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(pl->B);
    (void)hipFree(pl->W);
    pftpie_plan_destroy(pl->fft);
    delete pl;
    return hip_fail(e, "poly_create: tables");
  }
  *out = pl;
  return PFTPIE_OK;
}

pftpie_status pftpie_poly_destroy(pftpie_poly poly) {
  if (!poly) return PFTPIE_OK;
  (void)hipFree(poly->B);
  (void)hipFree(poly->W);
  pftpie_plan_destroy(poly->fft);
  delete poly;
  return PFTPIE_OK;
}

pftpie_status pftpie_poly_info(pftpie_poly poly, int32_t* r, double* xi) {
  if (pftpie_status s = check_poly(poly)) return s;
  if (r) *r = poly->r;
  if (xi) *xi = poly->xi;
  return PFTPIE_OK;
}

pftpie_status pftpie_poly_workspace_size(pftpie_poly poly, int64_t batch, size_t* bytes) {
  if (pftpie_status s = check_poly(poly)) return s;
  if (!bytes) return fail(PFTPIE_E_INVALID, "poly_workspace_size: bytes is NULL");
  if (batch < 0) return fail(PFTPIE_E_INVALID, "poly_workspace_size: batch must be >= 0");
  *bytes = (size_t)2 * batch * poly->r * poly->r * poly->p * poly->p * 8;
  return PFTPIE_OK;
}

pftpie_status pft2d_poly_forward(pftpie_poly poly, const void* psi, void* y, int64_t batch, void* ws,
                                 size_t ws_bytes, void* stream) {
  if (pftpie_status s = check_poly(poly)) return s;
  if (batch < 0) return fail(PFTPIE_E_INVALID, "pft2d_poly_forward: batch must be >= 0");
  if (batch == 0) return PFTPIE_OK;
  if (!psi || !y || !ws) return fail(PFTPIE_E_INVALID, "pft2d_poly_forward: NULL pointer");
  if (((uintptr_t)psi | (uintptr_t)y | (uintptr_t)ws) % 8)
    return fail(PFTPIE_E_INVALID, "pft2d_poly_forward: pointers must be 8-byte aligned");
  const size_t plane = (size_t)batch * poly->r * poly->r * poly->p * poly->p;
  if (ws_bytes < 2 * plane * 8) return fail(PFTPIE_E_INVALID, "pft2d_poly_forward: workspace too small");
  const char* a0 = static_cast<const char*>(psi);
  const char* a1 = a0 + (size_t)batch * poly->n * poly->n * 8;
  const char* b0 = static_cast<const char*>(y);
  const char* b1 = b0 + (size_t)batch * poly->m * poly->m * 8;
  if (a0 < b1 && b0 < a1) return fail(PFTPIE_E_INVALID, "pft2d_poly_forward: psi and y overlap");
  float2* C = static_cast<float2*>(ws);
  hipError_t e = launch_poly_forward(poly, static_cast<const float2*>(psi), static_cast<float2*>(y), batch, C,
                                     C + plane, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PFTPIE_OK : hip_fail(e, "pft2d_poly_forward: launch");
}

}  // extern "C"
