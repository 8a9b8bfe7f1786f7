// Library runtime: error reporting, per-(device, stream) workspaces, the
// host-mapped status word, tuning knobs and the helper entry points.
#include <cstdarg>
#include <cstdio>
#include <map>
#include <utility>
#include <vector>

#include "internal.h"

namespace odp {

namespace {
thread_local std::string g_last_error;
std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;
std::map<int, uint32_t*> g_status_host;  // host pointer of each device's status word
std::map<int, uint32_t*> g_status_dev;
std::map<int, int> g_cus;
Tuning g_tuning;
}  // namespace

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return ODP_OK;
  return set_error(e == hipErrorOutOfMemory ? ODP_ENOMEM : ODP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int DevBuf::ensure(size_t need) {
  if (need <= bytes) return ODP_OK;
  if (ptr) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return check_hip(e, "hipDeviceSynchronize before workspace growth");
    (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  hipError_t e = hipMalloc(&ptr, need);
  if (e != hipSuccess) {
    ptr = nullptr;
    return set_error(ODP_ENOMEM, "workspace allocation of %zu bytes failed: %s", need, hipGetErrorString(e));
  }
  bytes = need;
  return ODP_OK;
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

int current_device(int* dev) {
  hipError_t e = hipGetDevice(dev);
  return e == hipSuccess ? ODP_OK : check_hip(e, "hipGetDevice");
}

int cu_count(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cus.find(device);
  if (it != g_cus.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0) cus = 256;
  g_cus[device] = cus;
  return cus;
}

Tuning& tuning() { return g_tuning; }

uint32_t* device_status_word(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_status_dev.find(device);
  if (it != g_status_dev.end()) return it->second;
  uint32_t* h = nullptr;
  uint32_t* d = nullptr;
  if (hipHostMalloc(reinterpret_cast<void**>(&h), sizeof(uint32_t), hipHostMallocMapped) != hipSuccess) return nullptr;
  *h = 0;
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&d), h, 0) != hipSuccess) {
    (void)hipHostFree(h);
    return nullptr;
  }
  g_status_host[device] = h;
  g_status_dev[device] = d;
  return d;
}

Workspace* workspace_for(hipStream_t stream, int* err) {
  int dev = 0;
  if ((*err = current_device(&dev))) return nullptr;
  if (!device_status_word(dev)) {
    *err = set_error(ODP_ENOMEM, "could not allocate the host-mapped status word");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, stream);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) return it->second;
  Workspace* ws = new Workspace();
  ws->device = dev;
  ws->stream = stream;
  g_ws[key] = ws;
  return ws;
}

}  // namespace odp

using namespace odp;

extern "C" int odp_version(void) { return 100; }

extern "C" const char* odp_last_error_string(void) { return g_last_error.c_str(); }

extern "C" int odp_reserve(size_t max_buffers, uint64_t max_total_bytes, size_t max_events, odp_stream_t stream) {
  if (max_buffers > 0xFFFFFFFFull || max_events > 0xFFFFFFFFull)
    return set_error(ODP_ERANGE, "odp_reserve: sizes above 2^32 - 1");
  int err = 0;
  Workspace* ws = workspace_for(static_cast<hipStream_t>(stream), &err);
  if (!ws) return err;
  if (max_buffers || max_total_bytes) {
    int e = digest_reserve(ws, max_buffers, max_total_bytes);
    if (e) return e;
  }
  if (max_events) {
    int e = analyze_reserve(ws, max_events);
    if (e) return e;
  }
  return ODP_OK;
}

namespace odp {
// Frees one workspace (its device must be current and idle for its stream).
static void free_workspace(Workspace* ws) {
  if (ws->graph) (void)hipGraphExecDestroy(ws->graph);
  DevBuf* bufs[] = {&ws->node_off, &ws->tree_off, &ws->tk_off, &ws->small_list, &ws->blk, &ws->ctl,
                    &ws->item_buf, &ws->item_rec, &ws->med_rec, &ws->tree, &ws->tickets, &ws->p_tree, &ws->p_tickets};
  for (DevBuf* b : bufs) b->release();
  analyze_release(ws);
  delete ws;
}

void workspace_drop(int device, hipStream_t stream) {
  Workspace* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find(std::make_pair(device, stream));
    if (it == g_ws.end()) return;
    ws = it->second;
    g_ws.erase(it);
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(device);
  (void)hipStreamSynchronize(stream);
  free_workspace(ws);
  (void)hipSetDevice(cur);
}
}  // namespace odp

extern "C" int odp_release(void) {
  std::vector<Workspace*> all;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_ws) all.push_back(kv.second);
    g_ws.clear();
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (Workspace* ws : all) {
    (void)hipSetDevice(ws->device);
    (void)hipDeviceSynchronize();
    free_workspace(ws);
  }
  (void)hipSetDevice(cur);
  return ODP_OK;
}

extern "C" int odp_device_status(void) {
  int dev = 0;
  int e = current_device(&dev);
  if (e) return e;
  uint32_t* d = device_status_word(dev);
  if (!d) return set_error(ODP_ENOMEM, "status word unavailable");
  ODP_HIP(hipDeviceSynchronize());
  uint32_t* h;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    h = g_status_host[dev];
  }
  const uint32_t v = __atomic_exchange_n(h, 0u, __ATOMIC_SEQ_CST);
  const int na = noalloc_take_status(dev);
  if (v) return -(int)v;
  return na;
}

extern "C" int odp_get_tuning(odp_tuning* out) {
  if (!out) return set_error(ODP_EINVAL, "odp_get_tuning: null");
  *out = odp_tuning{};
  out->blocks_per_cu = g_tuning.blocks_per_cu;
  out->use_graph = g_tuning.use_graph;
  out->split_bytes = g_tuning.split_bytes;
  out->chunk_nodes = g_tuning.chunk_nodes;
  return ODP_OK;
}

extern "C" int odp_set_tuning(const odp_tuning* in) {
  if (!in) return set_error(ODP_EINVAL, "odp_set_tuning: null");
  if (in->blocks_per_cu < 1 || in->blocks_per_cu > 8)
    return set_error(ODP_EINVAL, "odp_set_tuning: blocks_per_cu %u outside 1..8", in->blocks_per_cu);
  if (in->use_graph > 1) return set_error(ODP_EINVAL, "odp_set_tuning: use_graph must be 0 or 1");
  if (in->split_bytes != 0 && (in->split_bytes < 4096 || in->split_bytes > 65536))
    return set_error(ODP_EINVAL, "odp_set_tuning: split_bytes %u not 0 or in 4096..65536", in->split_bytes);
  if (in->chunk_nodes > 16)
    return set_error(ODP_EINVAL, "odp_set_tuning: chunk_nodes %u outside 1..16", in->chunk_nodes);
  g_tuning.blocks_per_cu = in->blocks_per_cu;
  g_tuning.use_graph = in->use_graph;
  g_tuning.split_bytes = in->split_bytes;
  g_tuning.chunk_nodes = in->chunk_nodes ? in->chunk_nodes : 1u;
  return ODP_OK;
}
