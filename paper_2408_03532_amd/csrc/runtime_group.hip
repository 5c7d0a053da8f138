// C ABI of the uneven batch: descriptor validation, longest-first work list,
// one persistent launch.  Two forms: a group object (work list uploaded and
// a hipGraph instantiated once, replayed per run) and per-call grouped
// transforms over host descriptors and a caller workspace.
#include <algorithm>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "group.hpp"

namespace pftpie {
namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool ranges_overlap(int64_t a0, int64_t a1, int64_t b0, int64_t b1) { return a0 < b1 && b0 < a1; }

// Forward items per descriptor of a class: one per column-tile group.
int fwd_items(const GroupClass& c) { return c.w; }
// Adjoint items per descriptor: one per chunk of kpi column tiles.
int adj_items(const GroupClass& c) { return (c.nb + c.kpi - 1) / c.kpi; }

struct Work {
  GroupArgs args{};
  std::vector<GroupItem> items;
  int64_t in_extent = 0, out_extent = 0;  // complex elements the descriptors reach
};

// Classes from the plans, descriptor checks, and the work items sorted by
// cost, longest first (stable: equal costs keep descriptor order).
// in_len / out_len < 0: no packed-array lengths given; the extents the
// descriptors reach are returned instead.
pftpie_status build_work(const pftpie_plan_s* const* plans, int nplans, const pft2d_desc* desc, int64_t count,
                         int64_t in_len, int64_t out_len, int adjoint, const std::string& who, Work& w,
                         const int* ct_choice = nullptr, const int* kpi_choice = nullptr) {
  if (nplans < 1 || nplans > kGroupMaxClasses) return fail(PFTPIE_E_INVALID, who + ": need 1..8 (n, m) classes");
  for (int k = 0; k < nplans; ++k) {
    if (!plans[k]) return fail(PFTPIE_E_INVALID, who + ": NULL plan");
    if (plans[k]->prec != plans[0]->prec) return fail(PFTPIE_E_INVALID, who + ": plans differ in precision");
    if (plans[k]->device != plans[0]->device) return fail(PFTPIE_E_INVALID, who + ": plans on different devices");
    if (plans[k]->period != plans[k]->n)
      return fail(PFTPIE_E_INVALID, who + ": uneven batches take plans of DFT length n");
    for (int q = 0; q < k; ++q)
      if (plans[q]->n == plans[k]->n && plans[q]->m == plans[k]->m)
        return fail(PFTPIE_E_INVALID, who + ": two plans with the same (n, m)");
  }
  GroupArgs& args = w.args;
  std::vector<int> exact(nplans, 1);
  for (int k = 0; k < nplans; ++k) {
    const pftpie_plan_s* p = plans[k];
    GroupClass& c = args.cls[k];
    c.n = p->n;
    c.m = p->m;
    c.nb = p->nb;
    c.mt = p->mt;
    c.ct = (p->fwd_ct == 1 || p->mt == 1) ? 1 : 2;
    if (ct_choice && ct_choice[k] > 0) c.ct = (ct_choice[k] == 2 && p->mt >= 2) ? 2 : 1;
    c.w = (c.mt + c.ct - 1) / c.ct;
    c.kpi = 4;
    if (kpi_choice && kpi_choice[k] > 0) c.kpi = kpi_choice[k];
    c.tab = adjoint ? p->ft : p->fa;
    if (p->n % 16) exact[k] = 0;
  }
  std::vector<int> cls(count);
  std::vector<std::pair<int64_t, int64_t>> outs(count);
  for (int64_t i = 0; i < count; ++i) {
    const pft2d_desc& d = desc[i];
    int k = -1;
    for (int q = 0; q < nplans; ++q)
      if (plans[q]->n == d.n && plans[q]->m == d.m) k = q;
    if (k < 0) return fail(PFTPIE_E_INVALID, who + ": descriptor " + std::to_string(i) + " has no matching plan");
    const int64_t nin = adjoint ? (int64_t)d.m * d.m : (int64_t)d.n * d.n;
    const int64_t nout = adjoint ? (int64_t)d.n * d.n : (int64_t)d.m * d.m;
    if (d.in_offset < 0 || d.out_offset < 0 || (in_len >= 0 && d.in_offset + nin > in_len) ||
        (out_len >= 0 && d.out_offset + nout > out_len))
      return fail(PFTPIE_E_INVALID, who + ": descriptor " + std::to_string(i) + " outside the packed arrays");
    w.in_extent = std::max(w.in_extent, d.in_offset + nin);
    w.out_extent = std::max(w.out_extent, d.out_offset + nout);
    if (!adjoint && d.in_offset % 2) exact[k] = 0;
    cls[i] = k;
    outs[i] = {d.out_offset, d.out_offset + nout};
  }
  std::sort(outs.begin(), outs.end());
  for (size_t i = 1; i < outs.size(); ++i)
    if (ranges_overlap(outs[i - 1].first, outs[i - 1].second, outs[i].first, outs[i].second))
      return fail(PFTPIE_E_INVALID, who + ": output blocks overlap");
  for (int k = 0; k < nplans; ++k) args.cls[k].exact = exact[k];
  // work items, longest first (cost in MFMA issues of one item)
  std::vector<std::pair<double, GroupItem>> work;
  for (int64_t i = 0; i < count; ++i) {
    const GroupClass& c = args.cls[cls[i]];
    const pft2d_desc& d = desc[i];
    if (!adjoint) {
      const double cost = (double)c.nb * ((double)c.nb * c.ct + (double)c.mt * c.ct);
      for (int s = 0; s < fwd_items(c); ++s) work.push_back({cost, GroupItem{d.in_offset, d.out_offset, cls[i], s}});
    } else {
      for (int s = 0; s < adj_items(c); ++s) {
        const int tiles = std::min(c.kpi, c.nb - s * c.kpi);
        const double cost = (double)tiles * ((double)c.mt * c.mt + (double)c.nb * c.mt);
        work.push_back({cost, GroupItem{d.in_offset, d.out_offset, cls[i], s}});
      }
    }
  }
  std::stable_sort(work.begin(), work.end(),
                   [](const std::pair<double, GroupItem>& a, const std::pair<double, GroupItem>& b) {
                     return a.first > b.first;
                   });
  w.items.resize(work.size());
  for (size_t i = 0; i < work.size(); ++i) w.items[i] = work[i].second;
  args.nitems = (int64_t)w.items.size();
  return PFTPIE_OK;
}

unsigned grid_for(int num_cu, int64_t nitems, int wg_per_cu = 2) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)num_cu * wg_per_cu, (nitems + 3) / 4));
}

// The most work items any launch choice gives these descriptors: forward
// one per column tile, adjoint one per column tile.
size_t items_bound(const pft2d_desc* desc, int64_t count) {
  size_t items = 0;
  for (int64_t i = 0; i < count; ++i) items += (size_t)std::max(ceil16(desc[i].m), ceil16(desc[i].n));
  return items;
}

hipKernelNodeParams kernel_node(pft2d_group_s* g, void** kargs) {
  hipKernelNodeParams kp{};
  kp.func = group_kernel(g->prec, g->adjoint);
  kp.gridDim = dim3(g->grid);
  kp.blockDim = dim3(kGroupThreads);
  kp.sharedMemBytes = 0;
  kp.kernelParams = kargs;
  kp.extra = nullptr;
  return kp;
}

void destroy_group(pft2d_group_s* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  (void)hipFree(g->items);
  (void)hipFree(g->counter);
  delete g;
}

// reset node (counter = 0, a kernel: no memset node) -> persistent kernel
// node, instantiated once; runs only update the kernel node's buffers.
hipError_t build_graph(pft2d_group_s* g) {
  hipError_t e = hipGraphCreate(&g->graph, 0);
  if (e != hipSuccess) return e;
  hipKernelNodeParams rp{};
  void* rargs[] = {&g->counter};
  rp.func = group_reset_kernel();
  rp.gridDim = dim3(1);
  rp.blockDim = dim3(64);
  rp.sharedMemBytes = 0;
  rp.kernelParams = rargs;
  rp.extra = nullptr;
  hipGraphNode_t rn;
  e = hipGraphAddKernelNode(&rn, g->graph, nullptr, 0, &rp);
  if (e != hipSuccess) return e;
  void* kargs[] = {&g->args};
  hipKernelNodeParams kp = kernel_node(g, kargs);
  e = hipGraphAddKernelNode(&g->kernel_node, g->graph, &rn, 1, &kp);
  if (e != hipSuccess) return e;
  return hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
}

pftpie_status grouped(const pft2d_desc* desc, int64_t count, const void* in, void* out, pftpie_precision prec,
                      void* workspace, size_t ws_bytes, void* stream, int adjoint, const char* who_c) {
  const std::string who(who_c);
  if (count < 0) return fail(PFTPIE_E_INVALID, who + ": count < 0");
  if (count == 0) return PFTPIE_OK;
  if (!desc) return fail(PFTPIE_E_INVALID, who + ": descriptors are NULL");
  if (prec != PFTPIE_FP32 && prec != PFTPIE_SPLIT_BF16 && prec != PFTPIE_SPLIT_FP16)
    return fail(PFTPIE_E_INVALID, who + ": unknown precision");
  if (!in || !out) return fail(PFTPIE_E_INVALID, who + ": NULL data pointer");
  if ((uintptr_t)in % 16 || (uintptr_t)out % 16)
    return fail(PFTPIE_E_INVALID, who + ": packed arrays must be 16-byte aligned");
  if (!workspace || (uintptr_t)workspace % 256)
    return fail(PFTPIE_E_INVALID, who + ": workspace must be non-NULL and 256-byte aligned");
  int device = -1;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return hip_fail(e, (who + ": hipGetDevice").c_str());
  std::vector<const pftpie_plan_s*> plans;
  for (int64_t i = 0; i < count; ++i) {
    bool seen = false;
    for (const pftpie_plan_s* p : plans) seen = seen || (p->n == desc[i].n && p->m == desc[i].m);
    if (seen) continue;
    const pftpie_plan_s* p = find_plan(desc[i].n, desc[i].m, prec, device);
    if (!p)
      return fail(PFTPIE_E_INVALID, who + ": no live plan of (n, m) = (" + std::to_string(desc[i].n) + ", " +
                                        std::to_string(desc[i].m) +
                                        ") in this precision on the current device (create one first)");
    if ((int)plans.size() == kGroupMaxClasses) return fail(PFTPIE_E_INVALID, who + ": more than 8 (n, m) classes");
    plans.push_back(p);
  }
  Work w;
  if (pftpie_status st = build_work(plans.data(), (int)plans.size(), desc, count, -1, -1, adjoint, who, w))
    return st;
  const char* pi = static_cast<const char*>(in);
  const char* po = static_cast<const char*>(out);
  const char* pw = static_cast<const char*>(workspace);
  const size_t ib = (size_t)w.in_extent * 8, ob = (size_t)w.out_extent * 8;
  const size_t need = 256 + align256(w.items.size() * sizeof(GroupItem));
  if (ws_bytes < need)
    return fail(PFTPIE_E_INVALID, who + ": workspace smaller than pft2d_grouped_workspace_size (" +
                                      std::to_string(need) + " bytes)");
  if (pi < po + ob && po < pi + ib) return fail(PFTPIE_E_INVALID, who + ": input and output overlap");
  if ((pw < pi + ib && pi < pw + need) || (pw < po + ob && po < pw + need))
    return fail(PFTPIE_E_INVALID, who + ": workspace overlaps the data");
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned long long* counter = reinterpret_cast<unsigned long long*>(workspace);
  GroupItem* items = reinterpret_cast<GroupItem*>(static_cast<char*>(workspace) + 256);
  // a host-to-device copy from pageable memory returns once the runtime has
  // taken the source, so the item list may go out of scope after the call
  e = hipMemcpyAsync(items, w.items.data(), w.items.size() * sizeof(GroupItem), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, (who + ": work list upload").c_str());
  hipLaunchKernelGGL(reinterpret_cast<void (*)(unsigned long long*)>(group_reset_kernel()), dim3(1), dim3(64), 0, st,
                     counter);
  w.args.items = items;
  w.args.counter = counter;
  w.args.in = static_cast<const float2*>(in);
  w.args.out = static_cast<float2*>(out);
  void* kargs[] = {&w.args};
  e = hipLaunchKernel(group_kernel(prec, adjoint), dim3(grid_for(plans[0]->num_cu, w.args.nitems)),
                      dim3(kGroupThreads), kargs, 0, st);
  if (e == hipSuccess) e = hipGetLastError();
  return e == hipSuccess ? PFTPIE_OK : hip_fail(e, (who + ": launch").c_str());
}

}  // namespace
}  // namespace pftpie

using namespace pftpie;

extern "C" {

pftpie_status pftpie_group_create(const pftpie_plan* plans, int32_t nplans, const pft2d_desc* host_desc,
                                  int64_t count, int64_t in_len, int64_t out_len, int32_t adjoint,
                                  pft2d_group* out) {
  if (!out) return fail(PFTPIE_E_INVALID, "group_create: out is NULL");
  *out = nullptr;
  if (!plans || nplans < 1 || nplans > kGroupMaxClasses)
    return fail(PFTPIE_E_INVALID, "group_create: need 1..8 plans");
  if (count < 0 || (count > 0 && !host_desc)) return fail(PFTPIE_E_INVALID, "group_create: bad descriptor list");
  if (in_len < 0 || out_len < 0) return fail(PFTPIE_E_INVALID, "group_create: negative array length");
  if (adjoint != 0 && adjoint != 1) return fail(PFTPIE_E_INVALID, "group_create: adjoint must be 0 or 1");
  Work w;
  if (pftpie_status st = build_work(plans, nplans, host_desc, count, in_len, out_len, adjoint, "group_create", w))
    return st;
  pft2d_group_s* g = new (std::nothrow) pft2d_group_s();
  if (!g) return fail(PFTPIE_E_NOMEM, "group_create: host allocation failed");
  g->prec = plans[0]->prec;
  g->adjoint = adjoint;
  g->device = plans[0]->device;
  g->num_cu = plans[0]->num_cu;
  g->nitems = (int64_t)w.items.size();
  g->in_len = in_len;
  g->out_len = out_len;
  g->wg_per_cu = 2;
  for (int k = 0; k < kGroupMaxClasses; ++k) g->ct_choice[k] = g->kpi_choice[k] = 0;
  g->descs.assign(host_desc, host_desc + count);
  g->plans.assign(plans, plans + nplans);
  g->items_cap = std::max<size_t>(1, items_bound(host_desc, count));
  g->grid = grid_for(g->num_cu, g->nitems, g->wg_per_cu);
  hipError_t e = hipMalloc((void**)&g->items, sizeof(GroupItem) * g->items_cap);
  if (e == hipSuccess) e = hipMalloc((void**)&g->counter, sizeof(unsigned long long));
  if (e != hipSuccess) {
    destroy_group(g);
    return fail(PFTPIE_E_NOMEM, std::string("group_create: hipMalloc: ") + hipGetErrorString(e));
  }
  if (!w.items.empty())
    e = hipMemcpy(g->items, w.items.data(), sizeof(GroupItem) * w.items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    destroy_group(g);
    return hip_fail(e, "group_create: upload");
  }
  g->args = w.args;
  g->args.items = g->items;
  g->args.counter = g->counter;
  g->args.in = nullptr;
  g->args.out = nullptr;
  g->graph_in = nullptr;
  g->graph_out = nullptr;
  if (g->nitems > 0 && (e = build_graph(g)) != hipSuccess) {
    destroy_group(g);
    return hip_fail(e, "group_create: graph");
  }
  *out = g;
  return PFTPIE_OK;
}

pftpie_status pftpie_group_destroy(pft2d_group group) {
  destroy_group(group);
  return PFTPIE_OK;
}

pftpie_status pft2d_group_run(pft2d_group g, const void* in, void* out, void* stream) {
  if (!g) return fail(PFTPIE_E_INVALID, "group_run: group is NULL");
  if (g->nitems == 0) return PFTPIE_OK;
  if (!in || !out) return fail(PFTPIE_E_INVALID, "group_run: NULL data pointer");
  if ((uintptr_t)in % 16 || (uintptr_t)out % 16)
    return fail(PFTPIE_E_INVALID, "group_run: packed arrays must be 16-byte aligned");
  const char* pi = static_cast<const char*>(in);
  const char* po = static_cast<const char*>(out);
  if (pi < po + g->out_len * 8 && po < pi + g->in_len * 8)
    return fail(PFTPIE_E_INVALID, "group_run: input and output overlap");
  hipError_t e;
  if (g->graph_in != in || g->graph_out != out) {
    g->args.in = static_cast<const float2*>(in);
    g->args.out = static_cast<float2*>(out);
    void* kargs[] = {&g->args};
    hipKernelNodeParams kp = kernel_node(g, kargs);
    e = hipGraphExecKernelNodeSetParams(g->exec, g->kernel_node, &kp);
    if (e != hipSuccess) return hip_fail(e, "group_run: graph update");
    g->graph_in = in;
    g->graph_out = out;
  }
  e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PFTPIE_OK : hip_fail(e, "group_run: graph launch");
}

pftpie_status pftpie_group_autotune(pft2d_group g, double* best_ms) {
  if (!g) return fail(PFTPIE_E_INVALID, "group_autotune: group is NULL");
  if (g->nitems == 0) {
    if (best_ms) *best_ms = 0.0;
    return PFTPIE_OK;
  }
  const int nplans = (int)g->plans.size();
  float2 *x = nullptr, *y = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void**)&x, std::max<int64_t>(1, g->in_len) * 8);
  if (e == hipSuccess) e = hipMalloc((void**)&y, std::max<int64_t>(1, g->out_len) * 8);
  if (e == hipSuccess) e = hipStreamCreate(&st);
  if (e == hipSuccess) e = tune_fill(x, (size_t)g->in_len, 0x2468aceu, st);
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
    return fail(PFTPIE_E_NOMEM, std::string("group_autotune: scratch: ") + hipGetErrorString(e));
  }
  // time the batch with launch choices (ct, kpi, wg): rebuild the work
  // list, upload it, run reset + kernel directly (best of 3 after a warm-up)
  auto time_with = [&](const int* ct, const int* kpi, int wg, Work& w) -> double {
    w = Work{};
    if (build_work(g->plans.data(), nplans, g->descs.data(), (int64_t)g->descs.size(), g->in_len, g->out_len,
                   g->adjoint, "group_autotune", w, ct, kpi) != PFTPIE_OK)
      return 1e30;
    if (w.items.size() > g->items_cap) return 1e30;
    if (hipMemcpyAsync(g->items, w.items.data(), sizeof(GroupItem) * w.items.size(), hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return 1e30;
    w.args.items = g->items;
    w.args.counter = g->counter;
    w.args.in = x;
    w.args.out = y;
    void* kargs[] = {&w.args};
    const unsigned grid = grid_for(g->num_cu, w.args.nitems, wg);
    double best = 1e30;
    for (int rep = 0; rep < 4; ++rep) {
      (void)hipEventRecord(e0, st);
      hipLaunchKernelGGL(reinterpret_cast<void (*)(unsigned long long*)>(group_reset_kernel()), dim3(1), dim3(64), 0,
                         st, g->counter);
      hipError_t le = hipLaunchKernel(group_kernel(g->prec, g->adjoint), dim3(grid), dim3(kGroupThreads), kargs, 0, st);
      (void)hipEventRecord(e1, st);
      if (le != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1e30;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) best = std::min(best, (double)ms);
    }
    return best;
  };
  int ct[kGroupMaxClasses], kpi[kGroupMaxClasses];
  for (int k = 0; k < kGroupMaxClasses; ++k) {
    ct[k] = g->ct_choice[k];
    kpi[k] = g->kpi_choice[k];
  }
  int wg = g->wg_per_cu;
  Work w;
  double best = time_with(ct, kpi, wg, w);
  // classes in order of their work (longest first), one choice at a time
  std::vector<std::pair<double, int>> order;
  for (int k = 0; k < nplans; ++k) {
    double work = 0.0;
    for (const pft2d_desc& d : g->descs)
      if (d.n == g->plans[k]->n && d.m == g->plans[k]->m) work += (double)d.n * d.m * (d.n + d.m);
    order.push_back({-work, k});
  }
  std::sort(order.begin(), order.end());
  for (const auto& o : order) {
    const int k = o.second;
    static const int kAdjOpts[] = {1, 2, 4, 8};
    static const int kFwdOpts[] = {1, 2};
    const int* opts = g->adjoint ? kAdjOpts : kFwdOpts;
    const int nopts = g->adjoint ? 4 : 2;
    for (int i = 0; i < nopts; ++i) {
      int* choice = g->adjoint ? kpi : ct;
      const int keep = choice[k];
      choice[k] = opts[i];
      const double t = time_with(ct, kpi, wg, w);
      if (t < best) {
        best = t;
      } else {
        choice[k] = keep;
      }
    }
  }
  for (int cand : {1, 2, 3, 4}) {
    const double t = time_with(ct, kpi, cand, w);
    if (t < best) {
      best = t;
      wg = cand;
    }
  }
  // keep the best choices: work list, grid and graph
  for (int k = 0; k < kGroupMaxClasses; ++k) {
    g->ct_choice[k] = ct[k];
    g->kpi_choice[k] = kpi[k];
  }
  g->wg_per_cu = wg;
  Work fin;
  pftpie_status rs = build_work(g->plans.data(), nplans, g->descs.data(), (int64_t)g->descs.size(), g->in_len,
                                g->out_len, g->adjoint, "group_autotune", fin, ct, kpi);
  if (rs == PFTPIE_OK &&
      (e = hipMemcpy(g->items, fin.items.data(), sizeof(GroupItem) * fin.items.size(), hipMemcpyHostToDevice)) != hipSuccess)
    rs = hip_fail(e, "group_autotune: upload");
  cleanup();
  if (rs != PFTPIE_OK) return rs;
  g->args = fin.args;
  g->args.items = g->items;
  g->args.counter = g->counter;
  g->nitems = (int64_t)fin.items.size();
  g->grid = grid_for(g->num_cu, g->nitems, g->wg_per_cu);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
  g->graph_in = nullptr;
  g->graph_out = nullptr;
  if ((e = build_graph(g)) != hipSuccess) return hip_fail(e, "group_autotune: graph");
  if (best >= 1e30) return fail(PFTPIE_E_DEVICE, "group_autotune: every candidate failed");
  if (best_ms) *best_ms = best;
  return PFTPIE_OK;
}

pftpie_status pft2d_grouped_workspace_size(const pft2d_desc* host_desc, int64_t count, int32_t adjoint,
                                           size_t* bytes) {
  if (!bytes) return fail(PFTPIE_E_INVALID, "grouped_workspace_size: bytes is NULL");
  if (count < 0 || (count > 0 && !host_desc))
    return fail(PFTPIE_E_INVALID, "grouped_workspace_size: bad descriptor list");
  if (adjoint != 0 && adjoint != 1) return fail(PFTPIE_E_INVALID, "grouped_workspace_size: adjoint must be 0 or 1");
  // an upper bound on the work items whatever the plans' launch choices:
  // forward at most ceil(m / 16) column-tile groups per descriptor, adjoint
  // ceil(ceil(n / 16) / 4) chunks
  size_t items = 0;
  for (int64_t i = 0; i < count; ++i) {
    const int n = host_desc[i].n, m = host_desc[i].m;
    if (n < 1 || m < 1 || m > n || n > kMaxN)
      return fail(PFTPIE_E_INVALID, "grouped_workspace_size: descriptor " + std::to_string(i) + " needs 1 <= m <= n <= 8192");
    items += adjoint ? (size_t)((ceil16(n) + 3) / 4) : (size_t)ceil16(m);
  }
  *bytes = 256 + align256(items * sizeof(GroupItem));
  return PFTPIE_OK;
}

pftpie_status pft2d_forward_grouped(const pft2d_desc* host_desc, int64_t count, const void* in, void* out,
                                    pftpie_precision prec, void* workspace, size_t ws_bytes, void* stream) {
  return grouped(host_desc, count, in, out, prec, workspace, ws_bytes, stream, 0, "pft2d_forward_grouped");
}

pftpie_status pft2d_adjoint_grouped(const pft2d_desc* host_desc, int64_t count, const void* in, void* out,
                                    pftpie_precision prec, void* workspace, size_t ws_bytes, void* stream) {
  return grouped(host_desc, count, in, out, prec, workspace, ws_bytes, stream, 1, "pft2d_adjoint_grouped");
}

}  // extern "C"
