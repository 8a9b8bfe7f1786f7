// Serving: mapping-event requests classified as they arrive.
//
// A request is one event record plus, for a transfer, the device-resident
// bytes it moved. The host loop admits arrived requests into ticks, bounded by
// a slot count and a budget of in-flight payload bytes; each tick is one
// batched digest of its payloads followed by one classification kernel that
// works against device-resident per-key state and appends the records to a
// device-resident log. The flags known at arrival are exact at once:
//   DD     (digest, receiver) already seen                     (Def. 1)
//   RT_RX  latest earlier transfer of the digest between the same endpoints
//          went the other way                                   (Def. 2)
//   PAIRED a DELETE meeting an ALLOC just before it at its (device, address)
// The remaining flags depend on later records (a later return, a later
// repeat, a later kernel); draining the server runs the full analysis over
// the logged records, whose result equals the analysis of the arrival-ordered
// log.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <vector>

#include "internal.h"

namespace odp {
namespace {

constexpr int kTickMax = 1024;     // records per tick (one workgroup)
// staged bytes per request: the record, the payload pointer and size, a flag
constexpr size_t kStageBytes = sizeof(odp_event) + 8 + 8 + 1;
constexpr uint32_t kEmpty = 0;
// Set in every second key word: an unwritten (zeroed) slot never matches.
constexpr uint64_t kMark = 1ull << 63;

// Open-addressing table entry; keys are two words, values two words. state is
// kEmpty or the tag of the tick that claimed the slot (never kEmpty), so a
// thread tells a slot claimed earlier (keys complete and visible) from one
// another thread of its own tick is still filling in.
struct Slot {
  uint32_t state;
  uint32_t v0;
  uint64_t k0, k1;
  uint64_t v1;
};

struct Table {
  Slot* slots;
  uint64_t mask;  // capacity - 1 (power of two)
};

__device__ __forceinline__ uint64_t mix64(uint64_t a, uint64_t b) {
  uint64_t h = a * 0x9E3779B97F4A7C15ull ^ (b + 0x632BE59BD9B4E019ull);
  h ^= h >> 31;
  h *= 0xC2B2AE3D27D4EB4Full;
  h ^= h >> 29;
  return h;
}

// Lookup (no insertion; every slot was claimed by an earlier tick). Returns the slot or null.
__device__ Slot* tfind(const Table& T, uint64_t k0, uint64_t k1) {
  uint64_t i = mix64(k0, k1) & T.mask;
  for (uint64_t probe = 0; probe <= T.mask; ++probe) {
    Slot* s = &T.slots[i];
    if (s->state == kEmpty) return nullptr;
    if (s->k0 == k0 && s->k1 == k1) return s;
    i = (i + 1) & T.mask;
  }
  return nullptr;
}

// Find or insert. Within one tick a key is updated by one thread only, so a
// slot carrying this tick's tag holds another key (possibly half written):
// it is skipped without reading its keys.
__device__ Slot* tupsert(const Table& T, uint64_t k0, uint64_t k1, uint32_t tag, bool* inserted) {
  uint64_t i = mix64(k0, k1) & T.mask;
  for (uint64_t probe = 0; probe <= T.mask; ++probe) {
    Slot* s = &T.slots[i];
    uint32_t st = __hip_atomic_load(&s->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (st == kEmpty) st = atomicCAS(&s->state, kEmpty, tag);
    if (st == kEmpty) {
      s->k0 = k0;
      s->k1 = k1;
      s->v0 = 0;
      s->v1 = 0;
      *inserted = true;
      return s;
    }
    if (st != tag && s->k0 == k0 && s->k1 == k1) {
      *inserted = false;
      return s;
    }
    i = (i + 1) & T.mask;
  }
  *inserted = false;
  return nullptr;  // table full: reported through the server status
}

struct ServeState {
  uint64_t last_t_start;  // t_start of the last logged record
  uint64_t n_logged;
  uint32_t overflow;      // a table ran full
  uint32_t pad;
};

struct TickArgs {
  const odp_event* tick_ev;     // m records
  const uint64_t* tick_dig;     // m digests of the payloads (or the record's own digest)
  const uint8_t* tick_haspay;   // 1 when the digest came from a payload
  uint32_t m;
  uint64_t base_id;             // arrival index of the first record of the tick
  uint32_t tag;                 // nonzero, distinct for every tick of the server's life
  odp_event* log;               // all records in arrival order
  uint8_t* imm;                 // flags known at arrival (per arrival index)
  Table t_dd, t_rx, t_ad;
  ServeState* st;
};

__device__ __forceinline__ bool dev_ok(int d) { return d >= -1 && d <= ODP_MAX_DEVICE; }

__global__ __launch_bounds__(kTickMax) void serve_tick_kernel(TickArgs A) {
  __shared__ uint64_t s_dig[kTickMax];
  __shared__ uint64_t s_addr[kTickMax];
  __shared__ int16_t s_src[kTickMax], s_dst[kTickMax];
  __shared__ uint8_t s_kind[kTickMax];   // 0 invalid, 1 transfer, 2 alloc/delete, 3 kernel
  __shared__ uint8_t s_op[kTickMax];
  __shared__ uint64_t s_ts[kTickMax];
  const uint32_t t = threadIdx.x;
  const bool in = t < A.m;
  const uint64_t id = A.base_id + t;
  odp_event e;
  if (in) {
    e = A.tick_ev[t];
    if (A.tick_haspay[t]) e.digest = A.tick_dig[t];
    A.log[id] = e;
    s_ts[t] = e.t_start;
  }
  __syncthreads();
  uint8_t kind = 0;
  if (in) {
    const uint64_t prev = t ? s_ts[t - 1] : A.st->last_t_start;
    const bool first_ever = id == 0;
    const bool is_tx = e.op == ODP_H2D || e.op == ODP_D2H || e.op == ODP_D2D;
    const bool valid = e.op >= ODP_ALLOC && e.op <= ODP_KERNEL && e.t_end >= e.t_start &&
                       (first_ever || e.t_start >= prev) && dev_ok(e.dst_dev) && (!is_tx || dev_ok(e.src_dev));
    kind = !valid ? 0 : is_tx ? 1 : (e.op == ODP_KERNEL ? 3 : 2);
    s_dig[t] = e.digest;
    s_addr[t] = e.dst_addr;
    s_src[t] = e.src_dev;
    s_dst[t] = e.dst_dev;
    s_kind[t] = kind;
    s_op[t] = e.op;
  }
  __syncthreads();
  // Phase 1: predecessors inside the tick, else the state of earlier ticks.
  uint8_t f = kind == 0 && in ? ODP_F_INVALID : 0;
  int dd_first = -1, rx_pred = -1, rx_last = 1, ad_pred = -1, ad_last = 1;
  bool dd_last_occ = true;
  if (kind == 1) {
    const uint64_t h = e.digest;
    const int s = e.src_dev, d = e.dst_dev;
    const int lo = min(s, d), hi = max(s, d);
    for (uint32_t u = 0; u < A.m; ++u) {
      if (s_kind[u] != 1 || s_dig[u] != h) continue;
      if (u < t) {
        if (s_dst[u] == d && dd_first < 0) dd_first = (int)u;
        if (s != d && s_src[u] != s_dst[u] && min((int)s_src[u], (int)s_dst[u]) == lo &&
            max((int)s_src[u], (int)s_dst[u]) == hi)
          rx_pred = (int)u;
      } else if (u > t) {
        if (s_dst[u] == d) dd_last_occ = false;
        if (s != d && s_src[u] != s_dst[u] && min((int)s_src[u], (int)s_dst[u]) == lo &&
            max((int)s_src[u], (int)s_dst[u]) == hi)
          rx_last = 0;
      }
    }
    if (dd_first >= 0) {
      f |= ODP_F_DD;
    } else if (tfind(A.t_dd, h, kMark | (uint64_t)(d + 1))) {
      f |= ODP_F_DD;
    }
    if (s != d) {
      int pdir = -1;  // direction of the predecessor: 1 = lo -> hi
      if (rx_pred >= 0) {
        pdir = s_src[rx_pred] == lo ? 1 : 0;
      } else {
        const Slot* sl = tfind(A.t_rx, h, kMark | ((uint64_t)(lo + 1) << 8) | (uint64_t)(hi + 1));
        if (sl) pdir = (int)sl->v0;
      }
      const int mydir = s == lo ? 1 : 0;
      if (pdir >= 0 && pdir != mydir) f |= ODP_F_RT_RX;
    }
  } else if (kind == 2) {
    const uint64_t a = e.dst_addr;
    const int d = e.dst_dev;
    for (uint32_t u = 0; u < A.m; ++u) {
      if (s_kind[u] != 2 || s_addr[u] != a || s_dst[u] != d) continue;
      if (u < t) ad_pred = (int)u;
      else if (u > t) ad_last = 0;
    }
    uint8_t pop = 0;
    uint64_t pid = 0;
    if (ad_pred >= 0) {
      pop = s_op[ad_pred];
      pid = A.base_id + ad_pred;
    } else {
      const Slot* sl = tfind(A.t_ad, a, kMark | (uint64_t)(d + 1));
      if (sl) {
        pop = (uint8_t)sl->v0;
        pid = sl->v1;
      }
    }
    if (e.op == ODP_DELETE && pop == ODP_ALLOC) {
      f |= ODP_F_PAIRED;
      A.imm[pid] = ODP_F_PAIRED;  // the ALLOC this DELETE completes (its only writer)
    }
  }
  __syncthreads();
  // Phase 2: state updates, one thread per key.
  if (kind == 1) {
    const uint64_t h = e.digest;
    const int s = e.src_dev, d = e.dst_dev;
    bool ins;
    if (dd_first < 0) {
      Slot* sl = tupsert(A.t_dd, h, kMark | (uint64_t)(d + 1), A.tag, &ins);
      if (!sl) A.st->overflow = 1;
    }
    if (s != d && rx_last) {
      const int lo = min(s, d), hi = max(s, d);
      Slot* sl = tupsert(A.t_rx, h, kMark | ((uint64_t)(lo + 1) << 8) | (uint64_t)(hi + 1), A.tag, &ins);
      if (sl) sl->v0 = s == lo ? 1u : 0u;
      else A.st->overflow = 1;
    }
  } else if (kind == 2 && ad_last) {
    bool ins;
    Slot* sl = tupsert(A.t_ad, e.dst_addr, kMark | (uint64_t)(e.dst_dev + 1), A.tag, &ins);
    if (sl) {
      sl->v0 = e.op;
      sl->v1 = id;
    } else {
      A.st->overflow = 1;
    }
  }
  (void)dd_last_occ;
  if (in) A.imm[id] = (uint8_t)(A.imm[id] | f);
  __syncthreads();
  if (t == 0) {
    A.st->last_t_start = s_ts[A.m - 1];
    A.st->n_logged = A.base_id + A.m;
  }
}

__global__ void zero_bytes_kernel(uint8_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace
}  // namespace odp

using namespace odp;

struct odp_server {
  int device = 0;
  hipStream_t stream = nullptr;
  odp_server_config cfg{};
  // device state
  odp_event* log = nullptr;
  uint8_t* imm = nullptr;
  Table t_dd{}, t_rx{}, t_ad{};
  ServeState* st = nullptr;
  // tick staging, double-buffered: one pinned host block and one device block
  // per buffer, packed as records[m] | payload pointers[m] | sizes[m] | has[m]
  uint8_t* h_stage[2] = {nullptr, nullptr};
  uint8_t* d_stage[2] = {nullptr, nullptr};
  uint64_t* d_dig[2] = {nullptr, nullptr};
  hipEvent_t done[2] = {nullptr, nullptr};
  uint64_t n_logged = 0;
  uint64_t n_ticks = 0;
};

static int server_alloc(odp_server* s) {
  const odp_server_config& c = s->cfg;
  ODP_HIP(hipMalloc(&s->log, c.max_events * sizeof(odp_event)));
  ODP_HIP(hipMalloc(&s->imm, c.max_events));
  const uint64_t tcap = pow2_at_least(std::max<uint64_t>(1024, 2 * c.max_events));
  for (Table* T : {&s->t_dd, &s->t_rx, &s->t_ad}) {
    ODP_HIP(hipMalloc(&T->slots, tcap * sizeof(Slot)));
    ODP_HIP(hipMemset(T->slots, 0, tcap * sizeof(Slot)));
    T->mask = tcap - 1;
  }
  ODP_HIP(hipMalloc(&s->st, sizeof(ServeState)));
  ODP_HIP(hipMemset(s->st, 0, sizeof(ServeState)));
  ODP_HIP(hipMemset(s->imm, 0, c.max_events));
  for (int b = 0; b < 2; ++b) {
    ODP_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->h_stage[b]), kTickMax * kStageBytes, hipHostMallocDefault));
    ODP_HIP(hipMalloc(&s->d_stage[b], kTickMax * kStageBytes));
    ODP_HIP(hipMalloc(&s->d_dig[b], kTickMax * 8));
    ODP_HIP(hipEventCreateWithFlags(&s->done[b], hipEventDisableTiming));
  }
  return ODP_OK;
}

static void server_free(odp_server* s) {
  if (s->stream) {
    (void)hipStreamSynchronize(s->stream);
    // the digest and analysis workspace the library keeps for this stream
    workspace_drop(s->device, s->stream);
  }
  (void)hipFree(s->log);
  (void)hipFree(s->imm);
  for (Table* T : {&s->t_dd, &s->t_rx, &s->t_ad}) (void)hipFree(T->slots);
  (void)hipFree(s->st);
  for (int b = 0; b < 2; ++b) {
    (void)hipHostFree(s->h_stage[b]);
    (void)hipFree(s->d_stage[b]);
    (void)hipFree(s->d_dig[b]);
    if (s->done[b]) (void)hipEventDestroy(s->done[b]);
  }
  if (s->stream) (void)hipStreamDestroy(s->stream);
}

extern "C" int odp_server_create(const odp_server_config* cfg, odp_server** out) {
  if (!cfg || !out) return set_error(ODP_EINVAL, "odp_server_create: null argument");
  if (cfg->max_events == 0 || cfg->max_events > 0xFFFFFFFFull)
    return set_error(ODP_ERANGE, "odp_server_create: max_events must be in 1 .. 2^32 - 1");
  if (cfg->max_tick == 0 || cfg->max_tick > kTickMax)
    return set_error(ODP_EINVAL, "odp_server_create: max_tick must be in 1 .. %d", kTickMax);
  if (cfg->max_inflight == 0) return set_error(ODP_EINVAL, "odp_server_create: max_inflight must be positive");
  if (cfg->mode != ODP_SERVER_BATCHED && cfg->mode != ODP_SERVER_PLAIN)
    return set_error(ODP_EINVAL, "odp_server_create: unknown mode %u", cfg->mode);
  odp_server* s = new odp_server();
  s->cfg = *cfg;
  if (cfg->mode == ODP_SERVER_PLAIN) s->cfg.max_tick = s->cfg.max_inflight = 1;
  int e = current_device(&s->device);
  if (!e) {
    hipError_t he = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (he != hipSuccess) e = check_hip(he, "hipStreamCreate");
  }
  if (!e) e = server_alloc(s);
  if (!e) {
    int err = 0;
    Workspace* ws = workspace_for(s->stream, &err);
    e = ws ? digest_reserve(ws, kTickMax, cfg->budget_bytes + (uint64_t)kTickMax * kNodeBytes) : err;
    // one-request ticks take the per-buffer launch: its workspace too, up front
    if (!e) e = digest_plain_reserve(ws, cfg->budget_bytes);
  }
  if (e) {
    server_free(s);
    delete s;
    return e;
  }
  *out = s;
  return ODP_OK;
}

extern "C" int odp_server_destroy(odp_server* s) {
  if (!s) return ODP_OK;
  server_free(s);
  delete s;
  return ODP_OK;
}

struct StageView {
  odp_event* ev;
  uint64_t* ptr;
  uint64_t* size;
  uint8_t* has;
};

// The packed layout of a staging block holding m requests.
StageView stage_view(uint8_t* base, uint32_t m) {
  StageView v;
  v.ev = reinterpret_cast<odp_event*>(base);
  v.ptr = reinterpret_cast<uint64_t*>(base + (size_t)m * sizeof(odp_event));
  v.size = v.ptr + m;
  v.has = reinterpret_cast<uint8_t*>(v.size + m);
  return v;
}

// Enqueues one tick: one staging copy, the digest of the payloads (one
// persistent batched launch, or per-buffer launches in the plain mode), the
// classification.
static int launch_tick(odp_server* s, int b, uint32_t m, uint64_t bytes) {
  hipStream_t st = s->stream;
  ODP_HIP(hipMemcpyAsync(s->d_stage[b], s->h_stage[b], m * kStageBytes, hipMemcpyHostToDevice, st));
  const StageView hv = stage_view(s->h_stage[b], m), dv = stage_view(s->d_stage[b], m);
  // Tick sizes change every tick: direct launches rather than a captured
  // graph. A tick of one request takes the per-buffer launch (one kernel
  // instead of the plan, the persistent digest and the tree kernels).
  int e = s->cfg.mode == ODP_SERVER_PLAIN || m == 1
              ? odp_digest_buffers_plain(reinterpret_cast<const void* const*>(hv.ptr), hv.size, m, s->d_dig[b], st)
              : digest_batched_direct(reinterpret_cast<const void* const*>(dv.ptr), dv.size, m, s->d_dig[b], st, bytes);
  if (e) return e;
  TickArgs A;
  A.tick_ev = dv.ev;
  A.tick_dig = s->d_dig[b];
  A.tick_haspay = dv.has;
  A.m = m;
  A.base_id = s->n_logged;
  // at most max_events < 2^32 ticks: tags never repeat
  A.tag = (uint32_t)(s->n_ticks % 0xFFFFFFFFull) + 1;
  A.log = s->log;
  A.imm = s->imm;
  A.t_dd = s->t_dd;
  A.t_rx = s->t_rx;
  A.t_ad = s->t_ad;
  A.st = s->st;
  hipLaunchKernelGGL(serve_tick_kernel, dim3(1), dim3(kTickMax), 0, st, A);
  ODP_HIP(hipGetLastError());
  ODP_HIP(hipEventRecord(s->done[b], st));
  s->n_logged += m;
  s->n_ticks++;
  return ODP_OK;
}

extern "C" int odp_server_run(odp_server* s, const odp_event* events, const uint64_t* payload_ptrs,
                              const uint64_t* payload_bytes, const uint64_t* arrival_ns, size_t n,
                              uint64_t* complete_ns, odp_server_stats* stats) {
  if (!s || (n && (!events || !payload_ptrs || !payload_bytes || !arrival_ns || !complete_ns)))
    return set_error(ODP_EINVAL, "odp_server_run: null argument");
  if (s->n_logged + n > s->cfg.max_events)
    return set_error(ODP_ERANGE, "odp_server_run: %zu more records exceed max_events", n);
  for (size_t i = 0; i < n; ++i) {
    if (i && arrival_ns[i] < arrival_ns[i - 1])
      return set_error(ODP_EINVAL, "odp_server_run: arrival times must not decrease (request %zu)", i);
    if (payload_bytes[i] > s->cfg.budget_bytes)
      return set_error(ODP_EINVAL, "odp_server_run: request %zu payload above the memory budget", i);
    if (payload_bytes[i] && !payload_ptrs[i]) return set_error(ODP_EINVAL, "odp_server_run: request %zu null payload", i);
  }
  odp_server_stats lst{};
  const double t0 = now_s();
  size_t next_arrival = 0;             // first request not yet arrived
  std::deque<size_t> waiting;          // arrived, not admitted
  struct Inflight {
    int buf;
    size_t first, count;
    uint64_t bytes;
  };
  std::deque<Inflight> inflight;
  uint64_t inflight_bytes = 0;
  uint64_t inflight_reqs = 0;
  int next_buf = 0;
  size_t done = 0;
  size_t last_deferred = SIZE_MAX;
  while (done < n) {
    const double now = now_s() - t0;
    const uint64_t now_ns = (uint64_t)(now * 1e9);
    while (next_arrival < n && arrival_ns[next_arrival] <= now_ns) waiting.push_back(next_arrival++);
    // completions (in order)
    while (!inflight.empty()) {
      hipError_t q = hipEventQuery(s->done[inflight.front().buf]);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return check_hip(q, "odp_server_run: tick");
      const Inflight f = inflight.front();
      inflight.pop_front();
      const uint64_t tn = (uint64_t)((now_s() - t0) * 1e9);
      for (size_t k = 0; k < f.count; ++k) complete_ns[f.first + k] = tn;
      done += f.count;
      inflight_bytes -= f.bytes;
      inflight_reqs -= f.count;
    }
    // admission: a tick when a staging buffer is free (at most two ticks in flight)
    if (!waiting.empty() && inflight.size() < 2) {
      const int b = next_buf;
      uint32_t m = 0;
      uint64_t bytes = 0;
      const size_t first = waiting.front();
      const uint32_t cap = (uint32_t)std::min<size_t>(waiting.size(), s->cfg.max_tick);
      // admitted requests are packed for a tick of `cap`; a shorter tick is repacked below
      StageView v = stage_view(s->h_stage[b], cap);
      while (!waiting.empty() && m < cap && inflight_reqs + m < s->cfg.max_inflight) {
        const size_t i = waiting.front();
        if (inflight_bytes + bytes + payload_bytes[i] > s->cfg.budget_bytes) {
          if (i != last_deferred) lst.budget_waits++;  // each deferred request once
          last_deferred = i;
          break;
        }
        v.ev[m] = events[i];
        v.ptr[m] = payload_ptrs[i];
        v.size[m] = payload_bytes[i];
        v.has[m] = payload_bytes[i] || payload_ptrs[i] ? 1 : 0;
        bytes += payload_bytes[i];
        ++m;
        waiting.pop_front();
      }
      if (m && m < cap) {
        const StageView w = stage_view(s->h_stage[b], m);
        std::memmove(w.ptr, v.ptr, m * 8);
        std::memmove(w.size, v.size, m * 8);
        std::memmove(w.has, v.has, m);
      }
      if (m) {
        int e = launch_tick(s, b, m, bytes);
        if (e) return e;
        inflight.push_back({b, first, m, bytes});
        inflight_bytes += bytes;
        inflight_reqs += m;
        next_buf ^= 1;
        lst.ticks++;
        lst.max_tick = std::max<uint64_t>(lst.max_tick, m);
        lst.bytes += bytes;
      }
    }
  }
  lst.seconds = now_s() - t0;
  if (stats) *stats = lst;
  return ODP_OK;
}

extern "C" int odp_server_drain(odp_server* s, uint8_t* out_imm, uint8_t* out_flags, odp_report* out_report) {
  if (!s) return set_error(ODP_EINVAL, "odp_server_drain: null server");
  ODP_HIP(hipStreamSynchronize(s->stream));
  ServeState hs;
  ODP_HIP(hipMemcpy(&hs, s->st, sizeof(hs), hipMemcpyDeviceToHost));
  if (hs.overflow) return set_error(ODP_ECAPACITY, "odp_server_drain: a state table ran full");
  const uint64_t n = s->n_logged;
  if (out_imm && n) ODP_HIP(hipMemcpyAsync(out_imm, s->imm, n, hipMemcpyDeviceToDevice, s->stream));
  if (out_flags || out_report) {
    if (!out_flags || !out_report) return set_error(ODP_EINVAL, "odp_server_drain: flags and report go together");
    int e = odp_analyze_trace(s->log, n, out_flags, out_report, s->stream);
    if (e) return e;
  }
  ODP_HIP(hipStreamSynchronize(s->stream));
  return ODP_OK;
}

extern "C" int odp_server_log(odp_server* s, odp_event* out_events, size_t* n) {
  if (!s || !n) return set_error(ODP_EINVAL, "odp_server_log: null argument");
  ODP_HIP(hipStreamSynchronize(s->stream));
  *n = s->n_logged;
  if (out_events && s->n_logged)
    ODP_HIP(hipMemcpy(out_events, s->log, s->n_logged * sizeof(odp_event), hipMemcpyDeviceToDevice));
  return ODP_OK;
}
