// Uneven batches: many patches of different sizes in one persistent launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "internal.hpp"

namespace pftpie {

constexpr int kGroupMaxClasses = 8;

// One (n, m) class of the batch: the plan's sizes, tile split and table.
struct GroupClass {
  int n, m, nb, mt, ct, w;  // forward: ct column tiles per wave, w waves per patch
  int kpi;                  // adjoint: column tiles per work item
  int exact;                // every block of this class is 16-byte aligned and n % 16 == 0
  const void* tab;          // FA (forward) or FT (adjoint) table
};

// One work item: a descriptor's block offsets, its class and its slot
// (forward: which column-tile group; adjoint: which column-tile chunk).
struct GroupItem {
  int64_t in_off, out_off;
  int32_t cls, slot;
};

struct GroupArgs {
  GroupClass cls[kGroupMaxClasses];
  const GroupItem* items;
  int64_t nitems;
  unsigned long long* counter;
  const float2* in;
  float2* out;
};

// kernels (kernels_group.hip)
void* group_kernel(int prec, int adjoint);
void* group_reset_kernel();
constexpr int kGroupThreads = 256;

}  // namespace pftpie

struct pft2d_group_s {
  int prec, adjoint, device, num_cu;
  // descriptors and plans (kept for the autotuner) and the per-class launch
  // choices it may change: forward column tiles per wave, adjoint column
  // tiles per item (0: the default), workgroups per compute unit
  std::vector<pft2d_desc> descs;
  std::vector<pftpie_plan_s*> plans;
  int ct_choice[pftpie::kGroupMaxClasses];
  int kpi_choice[pftpie::kGroupMaxClasses];
  int wg_per_cu;
  size_t items_cap;                // work items the device list can hold
  pftpie::GroupArgs args;      // in / out filled at run time
  pftpie::GroupItem* items;    // device
  unsigned long long* counter; // device
  int64_t nitems, in_len, out_len;
  // graph built and instantiated at creation: reset node -> persistent
  // kernel node; runs update the kernel node's buffers when they change
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipGraphNode_t kernel_node;
  const void* graph_in;
  void* graph_out;
  unsigned grid;
};
