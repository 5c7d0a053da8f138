// C ABI: plans, validation, error plumbing and dispatch of the partial
// transform.  Every argument check happens here, on the host, before any
// work is enqueued.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

namespace pftpie {

static thread_local std::string g_last_error;

pftpie_status fail(pftpie_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

pftpie_status hip_fail(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return PFTPIE_E_DEVICE;
}

static std::mutex g_plans_mu;
static std::vector<pftpie_plan_s*> g_plans;

void register_plan(pftpie_plan_s* p) {
  std::lock_guard<std::mutex> lock(g_plans_mu);
  g_plans.push_back(p);
}

void unregister_plan(pftpie_plan_s* p) {
  std::lock_guard<std::mutex> lock(g_plans_mu);
  g_plans.erase(std::remove(g_plans.begin(), g_plans.end(), p), g_plans.end());
}

pftpie_plan_s* find_plan(int n, int m, pftpie_precision prec, int device) {
  std::lock_guard<std::mutex> lock(g_plans_mu);
  for (pftpie_plan_s* p : g_plans)
    if (p->n == n && p->m == m && p->prec == prec && p->device == device && p->period == n) return p;
  return nullptr;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

static pftpie_status check_plan(const pftpie_plan_s* p) {
  if (!p) return fail(PFTPIE_E_INVALID, "plan is NULL");
  return PFTPIE_OK;
}

static pftpie_status check_batch_io(const pftpie_plan_s* p, const void* in, size_t in_elems, const void* out,
                                    size_t out_elems, int64_t batch, const char* what) {
  if (batch < 0) return fail(PFTPIE_E_INVALID, std::string(what) + ": batch < 0");
  if (batch > 0x7fffffff) return fail(PFTPIE_E_INVALID, std::string(what) + ": batch exceeds 2^31 - 1");
  if (batch == 0) return PFTPIE_OK;
  if (!in || !out) return fail(PFTPIE_E_INVALID, std::string(what) + ": NULL data pointer");
  if ((uintptr_t)in % 8 || (uintptr_t)out % 8)
    return fail(PFTPIE_E_INVALID, std::string(what) + ": data pointers must be 8-byte aligned");
  if (overlaps(in, in_elems * batch * 8, out, out_elems * batch * 8))
    return fail(PFTPIE_E_INVALID, std::string(what) + ": input and output overlap");
  return PFTPIE_OK;
}

// Fills x[i] with float pairs uniform in [-1, 1) from a counter-based hash
// of i (timing operands only: zeros would run the matrix cores at a higher
// clock than real data do).
__global__ __launch_bounds__(256) void k_tune_fill(float2* __restrict__ x, size_t count, uint32_t salt) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u ^ (uint32_t)(i >> 32) ^ salt;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    const float a = (float)(h & 0xFFFFu) * (1.f / 32768.f) - 1.f;
    const float b = (float)(h >> 16) * (1.f / 32768.f) - 1.f;
    x[i] = make_float2(a, b);
  }
}

hipError_t tune_fill(float2* x, size_t count, uint32_t salt, hipStream_t st) {
  size_t blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_tune_fill, dim3((unsigned)blocks), dim3(256), 0, st, x, count, salt);
  return hipGetLastError();
}

}  // namespace pftpie

using namespace pftpie;

extern "C" {

const char* pftpie_status_string(pftpie_status s) {
  switch (s) {
    case PFTPIE_OK: return "ok";
    case PFTPIE_E_INVALID: return "invalid argument";
    case PFTPIE_E_UNSUPPORTED: return "unsupported";
    case PFTPIE_E_NOMEM: return "out of memory";
    case PFTPIE_E_DEVICE: return "device error";
  }
  return "unknown status";
}

const char* pftpie_last_error(void) { return g_last_error.c_str(); }

pftpie_status pftpie_plan_create(int32_t n, int32_t m, pftpie_precision prec, pftpie_plan* out) {
  return pftpie_plan_create_period(n, m, n, prec, PFTPIE_METHOD_AUTO, out);
}

pftpie_status pftpie_plan_create_method(int32_t n, int32_t m, pftpie_precision prec, pftpie_method method,
                                        pftpie_plan* out) {
  return pftpie_plan_create_period(n, m, n, prec, method, out);
}

pftpie_status pftpie_plan_create_period(int32_t n, int32_t m, int32_t period, pftpie_precision prec,
                                        pftpie_method method, pftpie_plan* out) {
  if (!out) return fail(PFTPIE_E_INVALID, "plan_create: out is NULL");
  *out = nullptr;
  if (method != PFTPIE_METHOD_AUTO && method != PFTPIE_METHOD_DENSE && method != PFTPIE_METHOD_FFT)
    return fail(PFTPIE_E_INVALID, "plan_create: unknown method");
  if (n < 1 || n > kMaxN) return fail(PFTPIE_E_INVALID, "plan_create: need 1 <= n <= 8192");
  if (m < 1 || m > n) return fail(PFTPIE_E_INVALID, "plan_create: need 1 <= m <= n");
  if (period < n || period > kMaxPeriod)
    return fail(PFTPIE_E_INVALID, "plan_create: need n <= period <= 2^20");
  if (prec != PFTPIE_FP32 && prec != PFTPIE_SPLIT_BF16 && prec != PFTPIE_SPLIT_FP16)
    return fail(PFTPIE_E_INVALID, "plan_create: unknown precision");
  if (m > kMaxM) return fail(PFTPIE_E_UNSUPPORTED, "plan_create: m > 128 is not supported");
  const bool fft_ok = fft_supported(n, m) && period == n;
  if (method == PFTPIE_METHOD_FFT && !fft_ok)
    return fail(PFTPIE_E_UNSUPPORTED,
                "plan_create: the fast transform needs m = n = period in {16, 32, 64, 128}");
  const bool use_fft = method == PFTPIE_METHOD_FFT || (method == PFTPIE_METHOD_AUTO && fft_ok);
  pftpie_plan_s* p = new (std::nothrow) pftpie_plan_s();
  if (!p) return fail(PFTPIE_E_NOMEM, "plan_create: host allocation failed");
  p->n = n;
  p->m = m;
  p->period = period;
  p->prec = prec;
  p->nb = ceil16(n);
  p->mt = ceil16(m);
  p->fa_ctiles = fa_ctiles_for(p->mt);
  p->method = use_fft ? PFTPIE_METHOD_FFT : PFTPIE_METHOD_DENSE;
  p->fft_tw = nullptr;
  p->fwd_ct = prec == PFTPIE_FP32 ? fwd_ct_default(p->mt) : fwd_ct_default_split(p->mt);
  // launch choices; pftpie_plan_autotune may replace them by measured ones
  p->use_lds = 1;
  p->use_lds_adj = 1;
  p->adj_k1 = 2;
  p->adj_patch = 1;
  p->adj_threads = 512;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "plan_create: hipGetDevice");
  }
  e = hipDeviceGetAttribute(&p->num_cu, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess || p->num_cu < 1) p->num_cu = 256;
  std::vector<float> fa, ft;
  std::vector<uint16_t> fa16, ft16;
  const void* fa_src;
  const void* ft_src;
  if (prec == PFTPIE_FP32) {
    build_twiddle_tables(n, m, period, p->fa_ctiles, fa, ft);
    p->fa_bytes = fa.size() * sizeof(float);
    p->ft_bytes = ft.size() * sizeof(float);
    fa_src = fa.data();
    ft_src = ft.data();
  } else {
    build_split_tables(n, m, period, p->fa_ctiles, prec == PFTPIE_SPLIT_BF16 ? 1 : 2, fa16, ft16);
    p->fa_bytes = fa16.size() * sizeof(uint16_t);
    p->ft_bytes = ft16.size() * sizeof(uint16_t);
    fa_src = fa16.data();
    ft_src = ft16.data();
  }
  e = hipMalloc((void**)&p->fa, p->fa_bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&p->ft, p->ft_bytes);
  if (e != hipSuccess) {
    (void)hipFree(p->fa);
    delete p;
    return fail(PFTPIE_E_NOMEM, std::string("plan_create: hipMalloc: ") + hipGetErrorString(e));
  }
  e = hipMemcpy(p->fa, fa_src, p->fa_bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->ft, ft_src, p->ft_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(p->fa);
    (void)hipFree(p->ft);
    delete p;
    return hip_fail(e, "plan_create: upload");
  }
  if (use_fft) {
    std::vector<float> tw;
    build_fft_twiddles(n, tw);
    e = hipMalloc((void**)&p->fft_tw, tw.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(p->fft_tw, tw.data(), tw.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(p->fa);
      (void)hipFree(p->ft);
      (void)hipFree(p->fft_tw);
      delete p;
      return hip_fail(e, "plan_create: fast-transform twiddles");
    }
  }
  register_plan(p);
  *out = p;
  return PFTPIE_OK;
}

pftpie_status pftpie_plan_destroy(pftpie_plan plan) {
  if (!plan) return PFTPIE_OK;
  unregister_plan(plan);
  (void)hipFree(plan->fa);
  (void)hipFree(plan->ft);
  if (plan->fft_tw) (void)hipFree(plan->fft_tw);
  delete plan;
  return PFTPIE_OK;
}

pftpie_status pftpie_plan_period(pftpie_plan plan, int32_t* period) {
  if (pftpie_status s = check_plan(plan)) return s;
  if (!period) return fail(PFTPIE_E_INVALID, "plan_period: period is NULL");
  *period = plan->period;
  return PFTPIE_OK;
}

pftpie_status pftpie_plan_method(pftpie_plan plan, pftpie_method* method) {
  if (pftpie_status s = check_plan(plan)) return s;
  if (!method) return fail(PFTPIE_E_INVALID, "plan_method: method is NULL");
  *method = (pftpie_method)plan->method;
  return PFTPIE_OK;
}

pftpie_status pftpie_plan_info(pftpie_plan plan, int32_t* n, int32_t* m, pftpie_precision* prec) {
  if (pftpie_status s = check_plan(plan)) return s;
  if (n) *n = plan->n;
  if (m) *m = plan->m;
  if (prec) *prec = plan->prec;
  return PFTPIE_OK;
}

pftpie_status pft2d_forward(pftpie_plan plan, const void* psi, void* y, int64_t batch, void* stream) {
  if (pftpie_status s = check_plan(plan)) return s;
  if (pftpie_status s = check_batch_io(plan, psi, (size_t)plan->n * plan->n, y, (size_t)plan->m * plan->m,
                                       batch, "pft2d_forward"))
    return s;
  const float2* in = static_cast<const float2*>(psi);
  float2* out = static_cast<float2*>(y);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = plan->method == PFTPIE_METHOD_FFT ? launch_fft_forward(plan, in, out, batch, st)
                                                   : launch_forward(plan, in, out, batch, st);
  return e == hipSuccess ? PFTPIE_OK : hip_fail(e, "pft2d_forward: launch");
}

pftpie_status pft2d_adjoint(pftpie_plan plan, const void* y, void* psi, int64_t batch, void* stream) {
  if (pftpie_status s = check_plan(plan)) return s;
  if (pftpie_status s = check_batch_io(plan, y, (size_t)plan->m * plan->m, psi, (size_t)plan->n * plan->n,
                                       batch, "pft2d_adjoint"))
    return s;
  const float2* in = static_cast<const float2*>(y);
  float2* out = static_cast<float2*>(psi);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = plan->method == PFTPIE_METHOD_FFT ? launch_fft_adjoint(plan, in, out, batch, st)
                                                   : launch_adjoint(plan, in, out, batch, st);
  return e == hipSuccess ? PFTPIE_OK : hip_fail(e, "pft2d_adjoint: launch");
}

pftpie_status pftpie_plan_autotune(pftpie_plan plan, int64_t sample, double* best_ms) {
  if (pftpie_status s = check_plan(plan)) return s;
  if (sample < 1 || sample > 1 << 20) return fail(PFTPIE_E_INVALID, "plan_autotune: need 1 <= sample <= 2^20");
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, plan->device);
  if (e != hipSuccess) return hip_fail(e, "plan_autotune: device properties");
  const std::string key = std::string(prop.gcnArchName) + " " + std::to_string(plan->n) + " " +
                          std::to_string(plan->m) + " " + std::to_string((int)plan->prec);
  const char* cache = std::getenv("PFTPIE_TUNE_CACHE");
  if (cache) {
    // "<arch> <n> <m> <prec> <fwd_ct> <lds_fwd> <lds_adj> <adj_patch> <adj_k1> <adj_threads> <ms>" per line
    if (FILE* f = std::fopen(cache, "r")) {
      char arch[128];
      int n, m, pr, ct, lf, la, ap, k1, th;
      double ms;
      while (std::fscanf(f, "%127s %d %d %d %d %d %d %d %d %d %lf", arch, &n, &m, &pr, &ct, &lf, &la, &ap, &k1, &th,
                         &ms) == 11) {
        const std::string k2 = std::string(arch) + " " + std::to_string(n) + " " + std::to_string(m) + " " +
                               std::to_string(pr);
        if (k2 == key && fwd_ct_valid(plan->mt, ct) && (k1 == 2 || k1 == 4) && (th == 512 || th == 768)) {
          plan->fwd_ct = ct;
          plan->use_lds = lf != 0;
          plan->use_lds_adj = la != 0;
          plan->adj_patch = ap != 0;
          plan->adj_k1 = k1;
          plan->adj_threads = th;
          if (best_ms) *best_ms = ms;
          std::fclose(f);
          return PFTPIE_OK;
        }
      }
      std::fclose(f);
    }
  }
  const size_t nin = (size_t)sample * plan->n * plan->n, nout = (size_t)sample * plan->m * plan->m;
  float2 *x = nullptr, *y = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipMalloc((void**)&x, nin * 8);
  if (e == hipSuccess) e = hipMalloc((void**)&y, nout * 8);
  if (e == hipSuccess) e = hipStreamCreate(&st);
  if (e == hipSuccess) e = tune_fill(x, nin, 0x1234567u, st);
  if (e == hipSuccess) e = tune_fill(y, nout, 0x89abcdefu, st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(x);
    (void)hipFree(y);
  };
  if (e != hipSuccess) {
    cleanup();
    return fail(PFTPIE_E_NOMEM, std::string("plan_autotune: scratch: ") + hipGetErrorString(e));
  }
  // each candidate runs on random operands: the adjoint writes x, so the
  // forward candidates, which read x, are all timed first
  auto time_ms = [&](bool fwd) -> double {
    double best = 1e30;
    for (int rep = 0; rep < 4; ++rep) {
      (void)hipEventRecord(e0, st);
      hipError_t le = fwd ? launch_forward(plan, x, y, sample, st) : launch_adjoint(plan, y, x, sample, st);
      (void)hipEventRecord(e1, st);
      if (le != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1e30;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) best = std::min(best, (double)ms);  // first run warms up
    }
    return best;
  };
  double best_f = 1e30, best_a = 1e30;
  int best_ct = plan->fwd_ct, best_lf = plan->use_lds;
  for (int ct = 1; ct <= 4; ++ct) {
    if (!fwd_ct_valid(plan->mt, ct)) continue;
    for (int lf = 1; lf >= 0; --lf) {
      plan->fwd_ct = ct;
      plan->use_lds = lf;
      const double t = time_ms(true);
      if (t < best_f) {
        best_f = t;
        best_ct = ct;
        best_lf = lf;
      }
    }
  }
  plan->fwd_ct = best_ct;
  plan->use_lds = best_lf;
  // the forward's output y is the adjoint's input: refill it with random data
  if (tune_fill(y, nout, 0x89abcdefu, st) != hipSuccess) {
    cleanup();
    return fail(PFTPIE_E_DEVICE, "plan_autotune: fill");
  }
  // adjoint: LDS or L2 table, whole patch per wave or tile per wave, and for
  // FP32 the stage-2 row tiles per step and the workgroup size
  const bool f32 = plan->prec == PFTPIE_FP32;
  int best_la = plan->use_lds_adj, best_ap = plan->adj_patch, best_k1 = plan->adj_k1, best_th = plan->adj_threads;
  for (int la = 1; la >= 0; --la)
    for (int ap = 1; ap >= 0; --ap)
      for (int k1 = 2; k1 <= (f32 ? 4 : 2); k1 += 2)
        for (int th = 512; th <= (f32 ? 768 : 512); th += 256) {
          // duplicates: the whole-patch kernels (m <= 64) take neither k1
          // nor the workgroup size, and above m = 64 there is no whole-patch kernel
          if (ap && (plan->mt > 4 || k1 != 2 || th != 512)) continue;
          plan->use_lds_adj = la;
          plan->adj_patch = ap;
          plan->adj_k1 = k1;
          plan->adj_threads = th;
          const double t = time_ms(false);
          if (t < best_a) {
            best_a = t;
            best_la = la;
            best_ap = ap;
            best_k1 = k1;
            best_th = th;
          }
        }
  plan->use_lds_adj = best_la;
  plan->adj_patch = best_ap;
  plan->adj_k1 = best_k1;
  plan->adj_threads = best_th;
  cleanup();
  if (best_f >= 1e30 || best_a >= 1e30) return fail(PFTPIE_E_DEVICE, "plan_autotune: every candidate failed");
  if (best_ms) *best_ms = best_f + best_a;
  if (cache) {
    if (FILE* f = std::fopen(cache, "a")) {
      std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %.6f\n", prop.gcnArchName, plan->n, plan->m, (int)plan->prec,
                   best_ct, best_lf, best_la, best_ap, best_k1, best_th, best_f + best_a);
      std::fclose(f);
    }
  }
  return PFTPIE_OK;
}

}  // extern "C"
