// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>

#include "odp.h"

namespace odp {

// Digest geometry of ODP-D64 v1.
constexpr uint32_t kLeaf = 4096;              // leaf bytes
constexpr uint32_t kFanIn = 64;               // children per tree node
constexpr uint64_t kNodeBytes = uint64_t(kLeaf) * kFanIn;  // bytes under one level-1 node

// Error plumbing (thread-local message, codes from odp.h).
int set_error(int code, const char* fmt, ...);
int check_hip(hipError_t e, const char* what);
#define ODP_HIP(call)                                   \
  do {                                                  \
    hipError_t odp_e_ = (call);                         \
    if (odp_e_ != hipSuccess) return ::odp::check_hip(odp_e_, #call); \
  } while (0)

// Grow-only device buffer.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  int ensure(size_t need);  // may synchronise the device before freeing the old block
  void release();
};

// Control block of one batched digest call (device memory).
struct DigestCtl {
  uint64_t n_node_items;  // level-1 node work items
  uint64_t n_small;       // buffers of at most one leaf
  uint64_t n_items;       // node items + small groups
  uint64_t tree_total;    // tree scratch slots needed
  uint64_t tk_total;      // ticket slots needed
  uint64_t n_med;         // level-1 nodes small enough for one wavefront
  uint32_t head;          // work-queue head
  uint32_t overflow;      // 1 when the plan did not fit the workspace
};

struct Workspace {
  int device = -1;
  hipStream_t stream = nullptr;
  // batched digest
  DevBuf node_off, tree_off, tk_off, small_list, blk, ctl, item_buf, item_rec, med_rec, tree, tickets;
  size_t cap_buffers = 0;
  uint64_t cap_items = 0, cap_tree = 0, cap_tk = 0;
  // plain digest (one buffer at a time)
  DevBuf p_tree, p_tickets;
  uint64_t p_cap_tree = 0, p_cap_tk = 0;
  // analysis: the allocation path runs on a second stream of this workspace,
  // forked from and joined to the caller's stream with events
  DevBuf a_bufs[24];
  size_t a_cap_events = 0;
  hipStream_t a_side = nullptr;
  hipEvent_t a_fork = nullptr, a_join = nullptr;
  // graph of the analysis launches for repeated calls with the same arguments
  hipGraphExec_t a_graph = nullptr;
  const void* ag_ev = nullptr;  // arguments of the graph (a_graph set) or of the last direct call
  size_t ag_n = 0;
  void* ag_flags = nullptr;
  void* ag_rep = nullptr;
  // graph cache of the batched digest
  hipGraphExec_t graph = nullptr;
  const void* g_ptrs = nullptr;
  const void* g_sizes = nullptr;
  void* g_out = nullptr;
  size_t g_n = 0;
  uint32_t g_grid = 0;
  uint32_t g_split = 0;
  uint32_t g_chunk = 0;
};

Workspace* workspace_for(hipStream_t stream, int* err);
// Frees the workspace of (device, stream), if any, after the stream is idle
// (for owners of a stream that is about to be destroyed).
void workspace_drop(int device, hipStream_t stream);
uint32_t* device_status_word(int device);  // device-visible sticky status (host-mapped)
int current_device(int* dev);
int cu_count(int device);

// Defaults: the autotuner's choice on MI355X (registers admit four of the
// batched digest's workgroups per compute unit, so more only queue; with the
// batched kernel's 256-byte steps, small level-1 nodes are no faster on one
// wavefront than on a whole workgroup).
struct Tuning {
  uint32_t blocks_per_cu = 4;
  uint32_t use_graph = 1;
  uint32_t split_bytes = 0;
  uint32_t chunk_nodes = 1;
};
Tuning& tuning();

int digest_reserve(Workspace* ws, size_t max_buffers, uint64_t max_total_bytes);
// Device bytes that digest_reserve / digest_plain_reserve allocate for these sizes.
uint64_t digest_workspace_bytes(size_t max_buffers, uint64_t max_total_bytes);
uint64_t digest_plain_workspace_bytes(uint64_t max_bytes);
// Workspace of the per-buffer form for buffers of up to max_bytes (grow-only).
int digest_plain_reserve(Workspace* ws, uint64_t max_bytes);
// Batched digest enqueued with direct launches (workspace reserved
// beforehand); total_bytes, the sum of the sizes, sizes the grids.
int digest_batched_direct(const void* const* ptrs, const uint64_t* sizes, size_t n, uint64_t* out, hipStream_t stream,
                          uint64_t total_bytes);
int analyze_reserve(Workspace* ws, size_t max_events);
// Reads and clears the status word of the no-allocation digest on `dev`
// (ODP_OK when that entry point never ran there). Synchronous.
int noalloc_take_status(int dev);
void analyze_release(Workspace* ws);

}  // namespace odp
