// C ABI of the PIE sweep: scans, workspace sizing, validation, dispatch.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"
#include "pie.hpp"

namespace pftpie {

// Device scratch of pie_sweep_noalloc: one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host the name is a stand-in, not a device address); it uses the address
// hipGetSymbolAddress returns for the device, looked up once per device.
constexpr size_t kNoAllocBytes = (size_t)PFTPIE_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace carve-up of one sweep; sizes in bytes, offsets 256-aligned.
struct PieLayout {
  size_t R, part, dpsi, phi, rank, winmax, O0, numO, D, numP, E, maxes, red, stats, fred, total;
  int fuse;
  int splits;
};

PieLayout pie_layout(const pie_scan_s* s, int batch, int norm, int probe_step) {
  const pftpie_plan_s* p = s->plan;
  const size_t obj = (size_t)s->H * s->W, nn = (size_t)p->n * p->n;
  const bool multi = batch > 1;
  PieLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.R = take((size_t)batch * p->m * p->m * 8);
  if (p->method == PFTPIE_METHOD_FFT) {
    L.splits = 1;
  } else {
    const long plain = (long)p->num_cu * pie_fwd_split_blocks_per_cu(p->prec, p->mt, false);
    const long rs = (long)p->num_cu * pie_fwd_split_blocks_per_cu(p->prec, p->mt, true);
    L.splits = pie_row_splits(p->nb, p->mt, batch, p->num_cu, plain, rs,
                              p->prec == PFTPIE_FP32 && p->n % 16 == 0);
  }
  L.part = L.splits > 1 ? take((size_t)batch * L.splits * p->m * p->m * 8) : SIZE_MAX;
  L.dpsi = multi ? take((size_t)batch * p->n * dpsi_stride(p->n) * 8) : SIZE_MAX;
  L.phi = take((size_t)s->J * 4 * 8);
  L.rank = take((size_t)s->J * 4);
  L.winmax = take((size_t)s->J * 8);
  // one chunk of several positions: statistics fused into the update, no
  // object copy (one position alone is updated in place, with the copy)
  L.fuse = multi && batch >= s->J && s->J > 1;
  L.O0 = L.fuse ? SIZE_MAX : take(obj * 8);
  L.numO = (multi && norm) ? take(obj * 8) : SIZE_MAX;
  L.D = (multi && norm) ? take(obj * 8) : SIZE_MAX;
  L.numP = (multi && probe_step) ? take(nn * 8) : SIZE_MAX;
  L.E = (multi && probe_step && norm) ? take(nn * 8) : SIZE_MAX;
  L.maxes = take(32);
  L.red = take((size_t)kStatBlocks * 3 * 8);
  L.stats = take(32);
  L.fred = L.fuse ? take((size_t)std::max<size_t>((size_t)s->tiles_x * s->tiles_y, kFusedRedBlocks) * 3 * 8) : SIZE_MAX;
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
  if (p->probe_update != 0 && p->probe_update != 1) return fail(PFTPIE_E_INVALID, "pie: probe_update must be 0 or 1");
  if (p->probe_update == 1 && p->gamma > 0.f && (p->batch != 1 || p->norm != 0))
    return fail(PFTPIE_E_INVALID, "pie: the probe update at the updated object needs batch == 1 and norm == 0");
  return PFTPIE_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch address on `device`, looked up with that device current.
pftpie_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(PFTPIE_E_UNSUPPORTED, "pie_sweep_noalloc: device index");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "pie_sweep_noalloc: hipGetDevice");
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "pie_sweep_noalloc: hipSetDevice");
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "pie_sweep_noalloc: hipGetSymbolAddress");
    if (!p || (uintptr_t)p % 256) return fail(PFTPIE_E_DEVICE, "pie_sweep_noalloc: scratch address unusable");
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return PFTPIE_OK;
}

// Body of pie_sweep and pie_sweep_noalloc: validation, then the launches.
pftpie_status sweep(pie_scan scan, void* object, void* probe, const float* amp, const int32_t* order_dev,
                    const pie_params* p, void* workspace, size_t ws_bytes, double* stats_dev, void* stream,
                    const char* who) {
  if (pftpie_status st = check_params(scan, p)) return st;
  const std::string name(who);
  if (!object || !probe || !amp) return fail(PFTPIE_E_INVALID, name + ": NULL object, probe or amplitudes");
  if ((uintptr_t)object % 8 || (uintptr_t)probe % 8 || (uintptr_t)amp % 4)
    return fail(PFTPIE_E_INVALID, name + ": misaligned object, probe or amplitudes");
  if (order_dev && (uintptr_t)order_dev % 4) return fail(PFTPIE_E_INVALID, name + ": misaligned order");
  if (stats_dev && (uintptr_t)stats_dev % 8) return fail(PFTPIE_E_INVALID, name + ": misaligned stats");
  const pftpie_plan_s* pl = scan->plan;
  const int batch = p->batch < scan->J ? p->batch : scan->J;
  const int probe_step = p->gamma > 0.f;
  const PieLayout L = pie_layout(scan, batch, p->norm, probe_step);
  if (!workspace || ws_bytes < L.total)
    return fail(PFTPIE_E_INVALID, name + ": workspace smaller than pie_workspace_size (" +
                                      std::to_string(L.total) + " bytes)");
  if ((uintptr_t)workspace % 256) return fail(PFTPIE_E_INVALID, name + ": workspace must be 256-byte aligned");
  const size_t ob = (size_t)scan->H * scan->W * 8, pb = (size_t)pl->n * pl->n * 8;
  const size_t ab = (size_t)scan->J * pl->m * pl->m * 4;
  if (overlaps(object, ob, probe, pb) || overlaps(object, ob, workspace, L.total) ||
      overlaps(probe, pb, workspace, L.total) || overlaps(amp, ab, object, ob) || overlaps(amp, ab, probe, pb) ||
      overlaps(amp, ab, workspace, L.total))
    return fail(PFTPIE_E_INVALID, name + ": object, probe, amplitudes and workspace must not overlap");
  char* ws = static_cast<char*>(workspace);
  auto at = [&](size_t off) -> void* { return off == SIZE_MAX ? nullptr : ws + off; };
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
  a.tiles_x = scan->tiles_x;
  a.tiles_y = scan->tiles_y;
  a.pos = scan->pos;
  a.order = order_dev;
  a.tile_ptr = scan->tile_ptr;
  a.tile_pos = scan->tile_pos;
  a.fa = pl->fa;
  a.ft = pl->ft;
  a.fft_tw = pl->method == PFTPIE_METHOD_FFT ? static_cast<const float2*>(pl->fft_tw) : nullptr;
  a.fa_bytes = pl->fa_bytes;
  a.ft_bytes = pl->ft_bytes;
  a.prec = pl->prec;
  a.period = pl->period;
  a.inv_n2 = (float)(1.0 / ((double)pl->period * pl->period));
  a.norm = p->norm;
  a.probe_step = probe_step;
  a.probe_literal = probe_step && p->probe_update == 1;
  a.probe_pass = 0;
  a.beta = p->beta;
  a.gamma = p->gamma;
  a.alpha = p->alpha;
  a.O = static_cast<float2*>(object);
  a.P = static_cast<float2*>(probe);
  a.amp = amp;
  a.R = static_cast<float2*>(at(L.R));
  a.part = static_cast<float2*>(at(L.part));
  a.splits = L.splits;
  a.num_cu = pl->num_cu;
  a.dpsi = static_cast<float2*>(at(L.dpsi));
  a.dstride = dpsi_stride(pl->n);
  a.phi_part = static_cast<double*>(at(L.phi));
  a.rank = static_cast<int32_t*>(at(L.rank));
  a.winmax = static_cast<unsigned*>(at(L.winmax));
  a.O0 = static_cast<float2*>(at(L.O0));
  a.numO = static_cast<float2*>(at(L.numO));
  a.D = static_cast<double*>(at(L.D));
  a.numP = static_cast<float2*>(at(L.numP));
  a.E = static_cast<double*>(at(L.E));
  a.maxes = static_cast<double*>(at(L.maxes));
  a.red = static_cast<double*>(at(L.red));
  a.stats = stats_dev ? stats_dev : static_cast<double*>(at(L.stats));
  a.fuse_stats = L.fuse;
  a.fold_stats = L.fuse && p->norm && !probe_step;
  a.fred = static_cast<double*>(at(L.fred));
  hipError_t e = launch_pie_sweep(a, batch, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PFTPIE_OK : hip_fail(e, (name + ": launch").c_str());
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
  // cover lists: for each 16 x 16 tile of the bounding box, the positions
  // whose window meets it (CSR, positions in increasing order)
  s->tiles_y = (s->bb_h + 15) / 16;
  s->tiles_x = (s->bb_w + 15) / 16;
  const size_t ntiles = (size_t)s->tiles_x * s->tiles_y;
  std::vector<int32_t> cnt(ntiles + 1, 0);
  auto tile_range = [&](int32_t j, int& ty0, int& ty1, int& tx0, int& tx1) {
    ty0 = (pos[2 * j] - r0) / 16;
    ty1 = (pos[2 * j] + n - 1 - r0) / 16;
    tx0 = (pos[2 * j + 1] - c0) / 16;
    tx1 = (pos[2 * j + 1] + n - 1 - c0) / 16;
  };
  for (int32_t j = 0; j < J; ++j) {
    int ty0, ty1, tx0, tx1;
    tile_range(j, ty0, ty1, tx0, tx1);
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) ++cnt[(size_t)ty * s->tiles_x + tx + 1];
  }
  for (size_t t = 0; t < ntiles; ++t) cnt[t + 1] += cnt[t];
  std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1), lists((size_t)cnt[ntiles]);
  for (int32_t j = 0; j < J; ++j) {
    int ty0, ty1, tx0, tx1;
    tile_range(j, ty0, ty1, tx0, tx1);
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) lists[(size_t)fill[(size_t)ty * s->tiles_x + tx]++] = j;
  }
  s->nnz = (int64_t)lists.size();
  hipError_t e = hipMalloc((void**)&s->pos, sizeof(int2) * (size_t)J);
  if (e == hipSuccess) e = hipMalloc((void**)&s->tile_ptr, sizeof(int32_t) * (ntiles + 1));
  if (e == hipSuccess) e = hipMalloc((void**)&s->tile_pos, sizeof(int32_t) * std::max<size_t>(1, lists.size()));
  if (e != hipSuccess) {
    (void)hipFree(s->pos);
    (void)hipFree(s->tile_ptr);
    delete s;
    return fail(PFTPIE_E_NOMEM, std::string("pie_scan_create: hipMalloc: ") + hipGetErrorString(e));
  }
  e = hipMemcpy(s->pos, pos.data(), sizeof(int2) * (size_t)J, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->tile_ptr, cnt.data(), sizeof(int32_t) * (ntiles + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && !lists.empty())
    e = hipMemcpy(s->tile_pos, lists.data(), sizeof(int32_t) * lists.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(s->pos);
    (void)hipFree(s->tile_ptr);
    (void)hipFree(s->tile_pos);
    delete s;
    return hip_fail(e, "pie_scan_create: upload");
  }
  *out = s;
  return PFTPIE_OK;
}

pftpie_status pie_scan_destroy(pie_scan scan) {
  if (!scan) return PFTPIE_OK;
  (void)hipFree(scan->pos);
  (void)hipFree(scan->tile_ptr);
  (void)hipFree(scan->tile_pos);
  delete scan;
  return PFTPIE_OK;
}

pftpie_status pie_workspace_size(pie_scan scan, const pie_params* p, size_t* bytes) {
  if (pftpie_status st = check_params(scan, p)) return st;
  if (!bytes) return fail(PFTPIE_E_INVALID, "pie_workspace_size: bytes is NULL");
  const int batch = p->batch < scan->J ? p->batch : scan->J;
  *bytes = pie_layout(scan, batch, p->norm, p->gamma > 0.f).total;
  return PFTPIE_OK;
}

pftpie_status pie_sweep(pie_scan scan, void* object, void* probe, const float* amp, const int32_t* order_dev,
                        const pie_params* p, void* workspace, size_t ws_bytes, double* stats_dev, void* stream) {
  return sweep(scan, object, probe, amp, order_dev, p, workspace, ws_bytes, stats_dev, stream, "pie_sweep");
}

pftpie_status pie_sweep_noalloc(pie_scan scan, void* object, void* probe, const float* amp,
                                const int32_t* order_dev, const pie_params* p, double* stats_dev, void* stream) {
  if (pftpie_status st = check_params(scan, p)) return st;
  const int batch = p->batch < scan->J ? p->batch : scan->J;
  const size_t need = pie_layout(scan, batch, p->norm, p->gamma > 0.f).total;
  if (need > kNoAllocBytes)
    return fail(PFTPIE_E_INVALID, "pie_sweep_noalloc: this sweep needs " + std::to_string(need) +
                                      " bytes of workspace, above the library's fixed scratch of " +
                                      std::to_string(kNoAllocBytes) + " bytes (use a smaller batch or pie_sweep)");
  void* ws = nullptr;
  if (pftpie_status st = scratch_address(scan->plan->device, &ws)) return st;
  return sweep(scan, object, probe, amp, order_dev, p, ws, kNoAllocBytes, stats_dev, stream, "pie_sweep_noalloc");
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
