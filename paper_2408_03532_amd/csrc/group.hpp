// Uneven batches: many patches of different sizes in one persistent launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
