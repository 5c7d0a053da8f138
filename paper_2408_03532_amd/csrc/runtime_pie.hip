// C ABI of the PIE sweep: scans, workspace sizing, validation, dispatch.
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"
#include "pie.hpp"

namespace pftpie {

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace carve-up of one sweep; sizes in bytes, offsets 256-aligned.
struct PieLayout {
  size_t R, phi, O0, numO, D, numP, E, maxes, stats, total;
};

PieLayout pie_layout(const pie_scan_s* s, int batch, int mode, int norm, int probe_step) {
  const pftpie_plan_s* p = s->plan;
  const size_t obj = (size_t)s->H * s->W, nn = (size_t)p->n * p->n;
  PieLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.R = take((size_t)batch * p->m * p->m * 8);
  L.phi = take((size_t)s->J * 4 * 8);
  L.O0 = take(obj * 8);
  L.numO = (mode == kModeAccum) ? take(obj * 8) : SIZE_MAX;
  L.D = norm ? take(obj * 8) : SIZE_MAX;
  L.numP = probe_step ? take(nn * 8) : SIZE_MAX;
  L.E = (probe_step && norm) ? take(nn * 8) : SIZE_MAX;
  L.maxes = take(16);
  L.stats = take(32);
  L.total = off;
  return L;
}

pftpie_status check_params(const pie_scan_s* s, const pie_params* p) {
  if (!s) return fail(PFTPIE_E_INVALID, "pie: scan is NULL");
  if (!p) return fail(PFTPIE_E_INVALID, "pie: params is NULL");
  if (p->batch < 1) return fail(PFTPIE_E_INVALID, "pie: batch must be >= 1");
  if (p->norm != 0 && p->norm != 1) return fail(PFTPIE_E_INVALID, "pie: norm must be 0 or 1");
  if (!std::isfinite(p->beta) || !std::isfinite(p->gamma) || !std::isfinite(p->alpha))
    return fail(PFTPIE_E_INVALID, "pie: non-finite step or regulariser");
  if (p->gamma < 0.f || p->alpha < 0.f) return fail(PFTPIE_E_INVALID, "pie: gamma and alpha must be >= 0");
  return PFTPIE_OK;
}

int mode_of(const pie_params* p) { return (p->norm == 0 && p->gamma == 0.f) ? kModeDirect : kModeAccum; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

}  // namespace

}  // namespace pftpie

using namespace pftpie;

extern "C" {

pftpie_status pie_scan_create(pftpie_plan plan, const int32_t* host_pos, int32_t J, int32_t H, int32_t W,
                              pie_scan* out) {
  if (!out) return fail(PFTPIE_E_INVALID, "pie_scan_create: out is NULL");
  *out = nullptr;
  if (!plan) return fail(PFTPIE_E_INVALID, "pie_scan_create: plan is NULL");
  if (J < 1) return fail(PFTPIE_E_INVALID, "pie_scan_create: need J >= 1");
  if (!host_pos) return fail(PFTPIE_E_INVALID, "pie_scan_create: positions are NULL");
  const int n = plan->n;
  if (H < n || W < n) return fail(PFTPIE_E_INVALID, "pie_scan_create: object smaller than the window");
  if ((int64_t)H * W > (int64_t)1 << 31) return fail(PFTPIE_E_INVALID, "pie_scan_create: object too large");
  int r0 = H, c0 = W, r1 = 0, c1 = 0;
  std::vector<int32_t> pos(2 * (size_t)J);
  for (int32_t j = 0; j < J; ++j) {
    const int32_t r = host_pos[2 * j], c = host_pos[2 * j + 1];
    if (r < 0 || c < 0 || r > H - n || c > W - n)
      return fail(PFTPIE_E_INVALID, "pie_scan_create: position " + std::to_string(j) + " = (" +
                                        std::to_string(r) + ", " + std::to_string(c) +
                                        ") puts its window outside the object");
    pos[2 * j] = r;
    pos[2 * j + 1] = c;
    r0 = std::min(r0, r);
    c0 = std::min(c0, c);
    r1 = std::max(r1, r + n);
    c1 = std::max(c1, c + n);
  }
  pie_scan_s* s = new (std::nothrow) pie_scan_s();
  if (!s) return fail(PFTPIE_E_NOMEM, "pie_scan_create: host allocation failed");
  s->plan = plan;
  s->J = J;
  s->H = H;
  s->W = W;
  s->bb_r0 = r0;
  s->bb_c0 = c0;
  s->bb_h = r1 - r0;
  s->bb_w = c1 - c0;
  hipError_t e = hipMalloc((void**)&s->pos, sizeof(int2) * (size_t)J);
  if (e != hipSuccess) {
    delete s;
    return fail(PFTPIE_E_NOMEM, std::string("pie_scan_create: hipMalloc: ") + hipGetErrorString(e));
  }
  e = hipMemcpy(s->pos, pos.data(), sizeof(int2) * (size_t)J, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(s->pos);
    delete s;
    return hip_fail(e, "pie_scan_create: upload");
  }
  *out = s;
  return PFTPIE_OK;
}

pftpie_status pie_scan_destroy(pie_scan scan) {
  if (!scan) return PFTPIE_OK;
  (void)hipFree(scan->pos);
  delete scan;
  return PFTPIE_OK;
}

pftpie_status pie_workspace_size(pie_scan scan, const pie_params* p, size_t* bytes) {
  if (pftpie_status st = check_params(scan, p)) return st;
  if (!bytes) return fail(PFTPIE_E_INVALID, "pie_workspace_size: bytes is NULL");
  const int batch = p->batch < scan->J ? p->batch : scan->J;
  *bytes = pie_layout(scan, batch, mode_of(p), p->norm, p->gamma > 0.f).total;
  return PFTPIE_OK;
}

pftpie_status pie_sweep(pie_scan scan, void* object, void* probe, const float* amp, const int32_t* order_dev,
                        const pie_params* p, void* workspace, size_t ws_bytes, double* stats_dev, void* stream) {
  if (pftpie_status st = check_params(scan, p)) return st;
  if (!object || !probe || !amp) return fail(PFTPIE_E_INVALID, "pie_sweep: NULL object, probe or amplitudes");
  if ((uintptr_t)object % 8 || (uintptr_t)probe % 8 || (uintptr_t)amp % 4)
    return fail(PFTPIE_E_INVALID, "pie_sweep: misaligned object, probe or amplitudes");
  if (order_dev && (uintptr_t)order_dev % 4) return fail(PFTPIE_E_INVALID, "pie_sweep: misaligned order");
  if (stats_dev && (uintptr_t)stats_dev % 8) return fail(PFTPIE_E_INVALID, "pie_sweep: misaligned stats");
  const pftpie_plan_s* pl = scan->plan;
  const int batch = p->batch < scan->J ? p->batch : scan->J;
  const int mode = mode_of(p), probe_step = p->gamma > 0.f;
  const PieLayout L = pie_layout(scan, batch, mode, p->norm, probe_step);
  if (!workspace || ws_bytes < L.total)
    return fail(PFTPIE_E_INVALID, "pie_sweep: workspace smaller than pie_workspace_size (" +
                                      std::to_string(L.total) + " bytes)");
  if ((uintptr_t)workspace % 256) return fail(PFTPIE_E_INVALID, "pie_sweep: workspace must be 256-byte aligned");
  const size_t ob = (size_t)scan->H * scan->W * 8, pb = (size_t)pl->n * pl->n * 8;
  const size_t ab = (size_t)scan->J * pl->m * pl->m * 4;
  if (overlaps(object, ob, probe, pb) || overlaps(object, ob, workspace, L.total) ||
      overlaps(probe, pb, workspace, L.total) || overlaps(amp, ab, object, ob) || overlaps(amp, ab, probe, pb) ||
      overlaps(amp, ab, workspace, L.total))
    return fail(PFTPIE_E_INVALID, "pie_sweep: object, probe, amplitudes and workspace must not overlap");
  char* ws = static_cast<char*>(workspace);
  PieArgs a{};
  a.n = pl->n;
  a.m = pl->m;
  a.nb = pl->nb;
  a.mt = pl->mt;
  a.J = scan->J;
  a.H = scan->H;
  a.W = scan->W;
  a.bb_r0 = scan->bb_r0;
  a.bb_c0 = scan->bb_c0;
  a.bb_h = scan->bb_h;
  a.bb_w = scan->bb_w;
  a.pos = scan->pos;
  a.order = order_dev;
  a.fa = pl->fa;
  a.ft = pl->ft;
  a.prec = pl->prec;
  a.inv_n2 = (float)(1.0 / ((double)pl->n * pl->n));
  a.mode = mode;
  a.norm = p->norm;
  a.probe_step = probe_step;
  a.beta = p->beta;
  a.gamma = p->gamma;
  a.alpha = p->alpha;
  a.O = static_cast<float2*>(object);
  a.P = static_cast<float2*>(probe);
  a.amp = amp;
  a.R = reinterpret_cast<float2*>(ws + L.R);
  a.phi_part = reinterpret_cast<double*>(ws + L.phi);
  a.O0 = reinterpret_cast<float2*>(ws + L.O0);
  a.numO = L.numO != SIZE_MAX ? reinterpret_cast<float2*>(ws + L.numO) : nullptr;
  a.D = L.D != SIZE_MAX ? reinterpret_cast<double*>(ws + L.D) : nullptr;
  a.numP = L.numP != SIZE_MAX ? reinterpret_cast<float2*>(ws + L.numP) : nullptr;
  a.E = L.E != SIZE_MAX ? reinterpret_cast<double*>(ws + L.E) : nullptr;
  a.maxes = reinterpret_cast<double*>(ws + L.maxes);
  a.stats = stats_dev ? stats_dev : reinterpret_cast<double*>(ws + L.stats);
  hipError_t e = launch_pie_sweep(a, batch, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PFTPIE_OK : hip_fail(e, "pie_sweep: launch");
}

pftpie_status pie_crop_amplitudes(const float* intensity, int32_t J, int32_t n, int32_t m, float* amp,
                                  void* stream) {
  if (J < 0) return fail(PFTPIE_E_INVALID, "pie_crop_amplitudes: J < 0");
  if (n < 1 || m < 1 || m > n) return fail(PFTPIE_E_INVALID, "pie_crop_amplitudes: need 1 <= m <= n");
  if (J == 0) return PFTPIE_OK;
  if (!intensity || !amp) return fail(PFTPIE_E_INVALID, "pie_crop_amplitudes: NULL pointer");
  if ((uintptr_t)intensity % 4 || (uintptr_t)amp % 4)
    return fail(PFTPIE_E_INVALID, "pie_crop_amplitudes: misaligned pointer");
  if (overlaps(intensity, (size_t)J * n * n * 4, amp, (size_t)J * m * m * 4))
    return fail(PFTPIE_E_INVALID, "pie_crop_amplitudes: input and output overlap");
  hipError_t e = launch_crop_amp(intensity, J, n, m, amp, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PFTPIE_OK : hip_fail(e, "pie_crop_amplitudes: launch");
}

}  // extern "C"
