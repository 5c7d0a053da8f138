// C ABI of the uneven batch: descriptor validation, longest-first work list,
// persistent launch through an explicitly built hipGraph.
#include <algorithm>
#include <cstdlib>
#include <new>
#include <string>
#include <vector>

#include "group.hpp"

namespace pftpie {
namespace {

bool ranges_overlap(int64_t a0, int64_t a1, int64_t b0, int64_t b1) { return a0 < b1 && b0 < a1; }

void destroy_group(pft2d_group_s* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  (void)hipFree(g->items);
  (void)hipFree(g->counter);
  delete g;
}

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
  hipKernelNodeParams kp{};
  void* kargs[] = {&g->args};
  kp.func = group_kernel(g->prec, g->adjoint);
  kp.gridDim = dim3(g->grid);
  kp.blockDim = dim3(kGroupThreads);
  kp.sharedMemBytes = 0;
  kp.kernelParams = kargs;
  kp.extra = nullptr;
  e = hipGraphAddKernelNode(&g->kernel_node, g->graph, &rn, 1, &kp);
  if (e != hipSuccess) return e;
  return hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
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
  for (int k = 0; k < nplans; ++k) {
    if (!plans[k]) return fail(PFTPIE_E_INVALID, "group_create: NULL plan");
    if (plans[k]->prec != plans[0]->prec) return fail(PFTPIE_E_INVALID, "group_create: plans differ in precision");
    if (plans[k]->device != plans[0]->device) return fail(PFTPIE_E_INVALID, "group_create: plans on different devices");
    for (int q = 0; q < k; ++q)
      if (plans[q]->n == plans[k]->n && plans[q]->m == plans[k]->m)
        return fail(PFTPIE_E_INVALID, "group_create: two plans with the same (n, m)");
  }
  // classes
  GroupArgs args{};
  std::vector<int> exact(nplans, 1);
  for (int k = 0; k < nplans; ++k) {
    const pftpie_plan_s* p = plans[k];
    GroupClass& c = args.cls[k];
    c.n = p->n;
    c.m = p->m;
    c.nb = p->nb;
    c.mt = p->mt;
    c.ct = (p->fwd_ct == 1 || p->mt == 1) ? 1 : 2;
    c.w = (c.mt + c.ct - 1) / c.ct;
    c.kpi = 4;
    c.tab = adjoint ? p->ft : p->fa;
    if (p->n % 16) exact[k] = 0;
  }
  // descriptors: class, bounds, disjoint outputs
  std::vector<int> cls(count);
  std::vector<std::pair<int64_t, int64_t>> outs(count);
  for (int64_t i = 0; i < count; ++i) {
    const pft2d_desc& d = host_desc[i];
    int k = -1;
    for (int q = 0; q < nplans; ++q)
      if (plans[q]->n == d.n && plans[q]->m == d.m) k = q;
    if (k < 0)
      return fail(PFTPIE_E_INVALID, "group_create: descriptor " + std::to_string(i) + " has no matching plan");
    const int64_t nin = adjoint ? (int64_t)d.m * d.m : (int64_t)d.n * d.n;
    const int64_t nout = adjoint ? (int64_t)d.n * d.n : (int64_t)d.m * d.m;
    if (d.in_offset < 0 || d.out_offset < 0 || d.in_offset + nin > in_len || d.out_offset + nout > out_len)
      return fail(PFTPIE_E_INVALID, "group_create: descriptor " + std::to_string(i) + " outside the packed arrays");
    if (!adjoint && d.in_offset % 2) exact[k] = 0;
    cls[i] = k;
    outs[i] = {d.out_offset, d.out_offset + nout};
  }
  std::vector<std::pair<int64_t, int64_t>> so(outs);
  std::sort(so.begin(), so.end());
  for (size_t i = 1; i < so.size(); ++i)
    if (ranges_overlap(so[i - 1].first, so[i - 1].second, so[i].first, so[i].second))
      return fail(PFTPIE_E_INVALID, "group_create: output blocks overlap");
  for (int k = 0; k < nplans; ++k) args.cls[k].exact = exact[k];
  // work items, longest first (cost in MFMA issues of one item)
  std::vector<std::pair<double, GroupItem>> work;
  for (int64_t i = 0; i < count; ++i) {
    const GroupClass& c = args.cls[cls[i]];
    const pft2d_desc& d = host_desc[i];
    if (!adjoint) {
      const double cost = (double)c.nb * ((double)c.nb * c.ct + (double)c.mt * c.ct);
      for (int s = 0; s < c.w; ++s) work.push_back({cost, GroupItem{d.in_offset, d.out_offset, cls[i], s}});
    } else {
      const int slots = (c.nb + c.kpi - 1) / c.kpi;
      for (int s = 0; s < slots; ++s) {
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
  std::vector<GroupItem> items(work.size());
  for (size_t i = 0; i < work.size(); ++i) items[i] = work[i].second;

  pft2d_group_s* g = new (std::nothrow) pft2d_group_s();
  if (!g) return fail(PFTPIE_E_NOMEM, "group_create: host allocation failed");
  g->prec = plans[0]->prec;
  g->adjoint = adjoint;
  g->device = plans[0]->device;
  g->num_cu = plans[0]->num_cu;
  g->nitems = (int64_t)items.size();
  g->in_len = in_len;
  g->out_len = out_len;
  g->use_graph = 1;
  if (const char* env = std::getenv("PFTPIE_GROUP_GRAPH")) g->use_graph = std::atoi(env) != 0;
  g->grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)g->num_cu * 2, (g->nitems + 3) / 4));
  hipError_t e = hipMalloc((void**)&g->items, sizeof(GroupItem) * std::max<size_t>(1, items.size()));
  if (e == hipSuccess) e = hipMalloc((void**)&g->counter, sizeof(unsigned long long));
  if (e != hipSuccess) {
    destroy_group(g);
    return fail(PFTPIE_E_NOMEM, std::string("group_create: hipMalloc: ") + hipGetErrorString(e));
  }
  if (!items.empty()) e = hipMemcpy(g->items, items.data(), sizeof(GroupItem) * items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    destroy_group(g);
    return hip_fail(e, "group_create: upload");
  }
  args.items = g->items;
  args.nitems = g->nitems;
  args.counter = g->counter;
  g->args = args;
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
  hipStream_t st = static_cast<hipStream_t>(stream);
  g->args.in = static_cast<const float2*>(in);
  g->args.out = static_cast<float2*>(out);
  hipError_t e;
  if (!g->use_graph) {
    hipLaunchKernelGGL(reinterpret_cast<void (*)(unsigned long long*)>(group_reset_kernel()), dim3(1), dim3(64), 0,
                       st, g->counter);
    void* kargs[] = {&g->args};
    e = hipLaunchKernel(group_kernel(g->prec, g->adjoint), dim3(g->grid), dim3(kGroupThreads), kargs, 0, st);
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? PFTPIE_OK : hip_fail(e, "group_run: launch");
  }
  if (!g->exec) {
    e = build_graph(g);
    if (e != hipSuccess) return hip_fail(e, "group_run: graph build");
    g->graph_in = in;
    g->graph_out = out;
  } else if (g->graph_in != in || g->graph_out != out) {
    hipKernelNodeParams kp{};
    void* kargs[] = {&g->args};
    kp.func = group_kernel(g->prec, g->adjoint);
    kp.gridDim = dim3(g->grid);
    kp.blockDim = dim3(kGroupThreads);
    kp.sharedMemBytes = 0;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    e = hipGraphExecKernelNodeSetParams(g->exec, g->kernel_node, &kp);
    if (e != hipSuccess) return hip_fail(e, "group_run: graph update");
    g->graph_in = in;
    g->graph_out = out;
  }
  e = hipGraphLaunch(g->exec, st);
  return e == hipSuccess ? PFTPIE_OK : hip_fail(e, "group_run: graph launch");
}

}  // extern "C"
