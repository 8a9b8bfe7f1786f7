// Serving: mapping-event requests classified as they arrive.
//
// A request is one event record plus, for a transfer, the device-resident
// bytes it moved. The host loop admits arrived requests into ticks, bounded by
// a slot count and the memory budget; each tick is one batched digest of its
// payloads (on the server's digest stream) followed by one classification
// kernel (on its classification stream, ordered after the digest by an event)
// that works against device-resident per-key state and appends the records to
// a device-resident log. With two ticks in flight, the digest of tick k+1 runs
// while tick k is classified; a tick submitted while none is in flight is
// classified on the digest stream, right after its digest.
//
// Every flag of a record is set as soon as the records that decide it have
// arrived (Sec. 4, Defs. 1-4; the paper analyses post mortem, so this is an
// extension), into the per-record "known" flags:
//   DD, RT_RX, PAIRED  at the record's own arrival
//   RT_TX              when a later transfer carries the digest back: every
//                      earlier transfer of the reversed endpoint pair not yet
//                      marked is marked (a per-key list of unmarked records)
//   RA                 when the ALLOC is paired: the smallest paired ALLOC
//                      index per (host address, device, bytes) is kept, and
//                      whichever of the two is larger is repeated
//   UA, UT             once a record starting after the window's end has
//                      arrived, no later kernel can meet the window: the
//                      window is [ALLOC start, DELETE end] for UA and
//                      [copy start, next copy start] for UT. The kernels on a
//                      device are kept in arrival order (their starts, and the
//                      running maximum of their ends), so "a kernel meets the
//                      window" is one prefix maximum and one binary search.
//                      This rests on a chronological log: after a rejected
//                      record these two bits wait for the drain, and a record
//                      rejected later (which may let a later record start
//                      earlier) can contradict a bit already set.
// A copy with no later copy of its place, and RT_TX of a transfer never sent
// back, stay open until the drain, which runs the full analysis over the
// logged records; its result equals the analysis of the arrival-ordered log.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <vector>

#include "internal.h"

namespace odp {
namespace {

constexpr int kTickMax = 1024;     // records per tick (one workgroup)
constexpr uint32_t kPerBufferTick = 3;  // ticks of at most this many requests digest per buffer
// staged bytes per request: the record, the payload pointer and size, a flag
constexpr size_t kStageBytes = sizeof(odp_event) + 8 + 8 + 1;
constexpr uint32_t kEmpty = 0;
// Set in every second key word: an unwritten (zeroed) slot never matches.
constexpr uint64_t kMark = 1ull << 63;
constexpr int kDev = ODP_MAX_DEVICE + 2;  // device codes: host (-1) .. ODP_MAX_DEVICE, shifted by one
constexpr uint64_t kNone64 = ~0ull;

// Open-addressing table entry; keys are three words, values two. state is
// kEmpty or the tag of the tick that claimed the slot (never kEmpty), so a
// thread tells a slot claimed earlier (keys complete and visible) from one
// another thread of its own tick is still filling in.
struct Slot {
  uint32_t state;
  uint32_t v0;
  uint64_t k0, k1, k2;
  uint64_t v1;
};

struct Table {
  Slot* slots;
  uint64_t mask;  // capacity - 1 (power of two)
};

__device__ __forceinline__ uint64_t mix64(uint64_t a, uint64_t b, uint64_t c) {
  uint64_t h = a * 0x9E3779B97F4A7C15ull ^ (b + 0x632BE59BD9B4E019ull);
  h ^= h >> 31;
  h = (h ^ c) * 0xC2B2AE3D27D4EB4Full;
  h ^= h >> 29;
  return h;
}

// Lookup (no insertion; every slot was claimed by an earlier tick). Returns the slot or null.
__device__ Slot* tfind(const Table& T, uint64_t k0, uint64_t k1, uint64_t k2 = 0) {
  uint64_t i = mix64(k0, k1, k2) & T.mask;
  for (uint64_t probe = 0; probe <= T.mask; ++probe) {
    Slot* s = &T.slots[i];
    if (s->state == kEmpty) return nullptr;
    if (s->k0 == k0 && s->k1 == k1 && s->k2 == k2) return s;
    i = (i + 1) & T.mask;
  }
  return nullptr;
}

// Find or insert. Within one tick a key is updated by one thread only, so a
// slot carrying this tick's tag holds another key (possibly half written):
// it is skipped without reading its keys. A new slot's v1 starts at `init`.
__device__ Slot* tupsert(const Table& T, uint64_t k0, uint64_t k1, uint64_t k2, uint32_t tag, uint64_t init,
                         bool* inserted) {
  uint64_t i = mix64(k0, k1, k2) & T.mask;
  for (uint64_t probe = 0; probe <= T.mask; ++probe) {
    Slot* s = &T.slots[i];
    uint32_t st = __hip_atomic_load(&s->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (st == kEmpty) st = atomicCAS(&s->state, kEmpty, tag);
    if (st == kEmpty) {
      s->k0 = k0;
      s->k1 = k1;
      s->k2 = k2;
      s->v0 = 0;
      s->v1 = init;
      *inserted = true;
      return s;
    }
    if (st != tag && s->k0 == k0 && s->k1 == k1 && s->k2 == k2) {
      *inserted = false;
      return s;
    }
    i = (i + 1) & T.mask;
  }
  *inserted = false;
  return nullptr;  // table full: reported through the server status
}

// A window waiting for its deadline (UA: an ALLOC and its DELETE; UT: a copy
// and the next copy of its place). The kernels on `dev` that meet
// [lo, deadline] are those among the first `kc` (logged before the window
// opened) whose end reaches lo, and those logged later that start by the
// deadline.
struct Pending {
  uint64_t lo, deadline;
  uint32_t id;    // the record that gets the flag
  uint32_t kc;    // kernels on dev logged before it
  uint32_t dev;   // device code (device + 1)
  uint32_t flag;  // ODP_F_UA or ODP_F_UT
};

struct ServeState {
  uint64_t last_t_start;  // t_start of the last logged record
  uint64_t n_logged;
  uint32_t overflow;      // a table ran full
  uint32_t any_invalid;   // some record was rejected: UA/UT wait for the drain
  uint32_t kcount[kDev];  // valid KERNEL records per device code
  uint32_t pend_n;        // windows waiting in pend[pend_cur]
  uint32_t pend_cur;
};

struct TickArgs {
  const odp_event* tick_ev;     // m records
  const uint64_t* tick_dig;     // m digests of the payloads (or the record's own digest)
  const uint8_t* tick_haspay;   // 1 when the digest came from a payload
  uint32_t m;
  uint64_t base_id;             // arrival index of the first record of the tick
  uint32_t tag;                 // nonzero, distinct for every tick of the server's life
  odp_event* log;               // all records in arrival order
  uint8_t* known;               // flags decided so far (per arrival index; 4-byte padded)
  uint32_t* link;               // per record: the next older unmarked record of its RT_TX list (+1)
  uint32_t* kc_at;              // per record: kernels on its device logged before it
  uint64_t* kstart;             // [kDev][cap]: kernel starts per device, in arrival order
  uint64_t* kmaxend;            // [kDev][cap]: running maximum of their ends
  uint64_t cap;                 // log capacity
  Pending* pend[2];             // [cap] each: waiting windows (ping-pong)
  Table t_dd, t_rx, t_ad, t_tx, t_ra, t_ut;
  ServeState* st;
};

__device__ __forceinline__ bool dev_ok(int d) { return d >= -1 && d <= ODP_MAX_DEVICE; }

// ORs flag bits into a record's byte of the known flags (several threads may
// set bits of one word).
__device__ __forceinline__ void known_or(uint8_t* known, uint64_t id, uint32_t bits) {
  if (!bits) return;
  uint32_t* w = reinterpret_cast<uint32_t*>(known + (id & ~3ull));
  atomicOr(w, bits << (8 * (uint32_t)(id & 3)));
}

// Entries of a sorted array (the starts of a device's kernels, in arrival
// order, which is time order in a chronological log) that are at most x.
__device__ uint32_t count_upto(const uint64_t* ks, uint32_t n, uint64_t x) {
  uint32_t a = 0, b = n;
  while (a < b) {
    const uint32_t mid = (a + b) / 2;
    if (ks[mid] <= x) a = mid + 1; else b = mid;
  }
  return a;
}

enum : uint8_t { K_INVALID = 0, K_TRANSFER = 1, K_ALLOCDEL = 2, K_KERNEL = 3 };

__device__ __forceinline__ uint64_t tx_key(int s, int d) { return kMark | ((uint64_t)(s + 1) << 8) | (uint64_t)(d + 1); }

__global__ __launch_bounds__(kTickMax) void serve_tick_kernel(TickArgs A) {
  __shared__ uint64_t s_dig[kTickMax];
  __shared__ uint64_t s_addr[kTickMax];   // dst_addr (ALLOC/DELETE: device address)
  __shared__ uint64_t s_saddr[kTickMax];  // src_addr (copies: source; ALLOC: host address)
  __shared__ uint64_t s_ts[kTickMax];
  __shared__ uint64_t s_te[kTickMax];
  __shared__ uint64_t s_pid[kTickMax];    // DELETE: the ALLOC it pairs (arrival index), else none
  __shared__ uint64_t s_xchg[kTickMax];   // RT_TX list head taken by a key's last element; RA tick minimum
  __shared__ int16_t s_src[kTickMax], s_dst[kTickMax];
  __shared__ uint8_t s_kind[kTickMax];
  __shared__ uint8_t s_op[kTickMax];
  __shared__ uint8_t s_unmarked[kTickMax];  // transfer not sent back later in this tick
  __shared__ uint32_t s_kc0[kDev];          // kernels per device before this tick
  __shared__ uint32_t s_kc1[kDev];          // ... and after it
  __shared__ uint32_t s_pend_n, s_keep;
  const uint32_t t = threadIdx.x;
  const bool in = t < A.m;
  const uint64_t id = A.base_id + t;
  ServeState* st = A.st;
  odp_event e;
  if (t < kDev) s_kc0[t] = st->kcount[t];
  if (t == 0) {
    s_pend_n = st->pend_n;
    s_keep = 0;
  }
  if (in) {
    e = A.tick_ev[t];
    if (A.tick_haspay[t]) e.digest = A.tick_dig[t];
    A.log[id] = e;
    s_ts[t] = e.t_start;
  }
  __syncthreads();
  uint8_t kind = K_INVALID;
  if (in) {
    const uint64_t prev = t ? s_ts[t - 1] : st->last_t_start;
    const bool first_ever = id == 0;
    const bool is_tx = e.op == ODP_H2D || e.op == ODP_D2H || e.op == ODP_D2D;
    const bool valid = e.op >= ODP_ALLOC && e.op <= ODP_KERNEL && e.t_end >= e.t_start &&
                       (first_ever || e.t_start >= prev) && dev_ok(e.dst_dev) && (!is_tx || dev_ok(e.src_dev));
    kind = !valid ? K_INVALID : is_tx ? K_TRANSFER : (e.op == ODP_KERNEL ? K_KERNEL : K_ALLOCDEL);
    s_dig[t] = e.digest;
    s_addr[t] = e.dst_addr;
    s_saddr[t] = e.src_addr;
    s_te[t] = e.t_end;
    s_src[t] = e.src_dev;
    s_dst[t] = e.dst_dev;
    s_kind[t] = kind;
    s_op[t] = e.op;
    s_pid[t] = kNone64;
    s_unmarked[t] = 0;
  }
  // UA and UT are decided early only while the log is chronological.
  const bool tick_invalid = __syncthreads_or(in && kind == K_INVALID);
  const bool windows_on = !st->any_invalid && !tick_invalid;
  // Kernels on my device logged before me (earlier ticks and earlier in this one).
  uint32_t kc_me = 0;
  if (in && kind != K_INVALID) {
    const int dv = e.dst_dev;
    uint32_t c = 0;
    for (uint32_t u = 0; u < t; ++u) c += s_kind[u] == K_KERNEL && s_dst[u] == dv;
    kc_me = s_kc0[dv + 1] + c;
  }
  // Phase 1: predecessors inside the tick, else the state of earlier ticks.
  uint8_t f = kind == K_INVALID && in ? ODP_F_INVALID : 0;
  int dd_first = -1, rx_pred = -1, rx_last = 1, ad_pred = -1, ad_last = 1;
  bool tx_first = true, tx_last = true, ut_last = true, is_copyin = false;
  int ut_prev = -1;
  uint64_t ut_prev_id = kNone64;  // the copy this one closes (its next copy is this one)
  if (kind == K_TRANSFER) {
    const uint64_t h = e.digest;
    const int s = e.src_dev, d = e.dst_dev;
    const int lo = min(s, d), hi = max(s, d);
    is_copyin = e.op != ODP_D2H && d >= 0;
    bool sent_back = false;
    for (uint32_t u = 0; u < A.m; ++u) {
      if (s_kind[u] != K_TRANSFER) continue;
      if (is_copyin && u != t && s_op[u] != ODP_D2H && s_dst[u] == d && s_src[u] == s && s_saddr[u] == e.src_addr) {
        if (u < t) ut_prev = (int)u; else ut_last = false;
      }
      if (s_dig[u] != h) continue;
      const int su = s_src[u], du = s_dst[u];
      const bool same_pair = s != d && su != du && min(su, du) == lo && max(su, du) == hi;
      if (u < t) {
        if (du == d && dd_first < 0) dd_first = (int)u;
        if (same_pair) rx_pred = (int)u;
        if (su == s && du == d) tx_first = false;
      } else if (u > t) {
        if (same_pair) rx_last = 0;
        if (s != d && su == d && du == s) sent_back = true;
        if (su == s && du == d) tx_last = false;
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
      if (sent_back) f |= ODP_F_RT_TX;
      // The first transfer of my ordered pair in this tick takes the list of
      // earlier ticks' transfers that went the other way and marks them all:
      // it carries their data back.
      if (tx_first) {
        Slot* sl = tfind(A.t_tx, h, tx_key(d, s));
        if (sl) {
          uint64_t head = atomicExch(reinterpret_cast<unsigned long long*>(&sl->v1), 0ull);
          while (head) {
            const uint64_t rid = head - 1;
            known_or(A.known, rid, ODP_F_RT_TX);
            head = A.link[rid];
          }
        }
      }
      s_unmarked[t] = !sent_back;
    }
    if (is_copyin) {
      if (ut_prev >= 0) {
        ut_prev_id = A.base_id + (uint64_t)ut_prev;
      } else {
        const Slot* sl = tfind(A.t_ut, e.src_addr, tx_key(s, d));
        if (sl && sl->v1) ut_prev_id = sl->v1 - 1;
      }
    }
  } else if (kind == K_ALLOCDEL) {
    const uint64_t a = e.dst_addr;
    const int d = e.dst_dev;
    for (uint32_t u = 0; u < A.m; ++u) {
      if (s_kind[u] != K_ALLOCDEL || s_addr[u] != a || s_dst[u] != d) continue;
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
      known_or(A.known, pid, ODP_F_PAIRED);  // the ALLOC this DELETE completes
      s_pid[t] = pid;
    }
  }
  if (in) {
    known_or(A.known, id, f);
    A.kc_at[id] = kc_me;
  }
  __syncthreads();
  // Phase 2: state updates, one thread per key.
  const uint32_t tag = A.tag;
  bool ins;
  if (kind == K_TRANSFER) {
    const uint64_t h = e.digest;
    const int s = e.src_dev, d = e.dst_dev;
    if (dd_first < 0) {
      Slot* sl = tupsert(A.t_dd, h, kMark | (uint64_t)(d + 1), 0, tag, 0, &ins);
      if (!sl) st->overflow = 1;
    }
    if (s != d && rx_last) {
      const int lo = min(s, d), hi = max(s, d);
      Slot* sl = tupsert(A.t_rx, h, kMark | ((uint64_t)(lo + 1) << 8) | (uint64_t)(hi + 1), 0, tag, 0, &ins);
      if (sl) sl->v0 = s == lo ? 1u : 0u;
      else st->overflow = 1;
    }
    // The unmarked transfers of my ordered pair in this tick join its list:
    // the pair's last transfer of the tick swaps the newest unmarked one in as
    // the head; each links to the next older unmarked one of the tick, the
    // oldest to the old head (phase 2b).
    if (s != d && tx_last) {
      int newest = -1;
      for (uint32_t u = 0; u <= t; ++u)
        if (s_kind[u] == K_TRANSFER && s_unmarked[u] && s_dig[u] == h && s_src[u] == s && s_dst[u] == d) newest = (int)u;
      s_xchg[t] = 0;
      if (newest >= 0) {
        Slot* sl = tupsert(A.t_tx, h, tx_key(s, d), 0, tag, 0, &ins);
        if (sl) s_xchg[t] = atomicExch(reinterpret_cast<unsigned long long*>(&sl->v1), A.base_id + newest + 1);
        else st->overflow = 1;
      }
    }
    if (is_copyin && ut_last) {
      Slot* sl = tupsert(A.t_ut, e.src_addr, tx_key(s, d), 0, tag, 0, &ins);
      if (sl) sl->v1 = id + 1;  // open: no later copy of this place yet
      else st->overflow = 1;
    }
    // The copy this one follows is closed: its window ends at my start.
    if (is_copyin && ut_prev_id != kNone64 && windows_on) {
      const uint64_t pid = ut_prev_id;
      Pending p;
      p.lo = A.log[pid].t_start;
      p.deadline = e.t_start;
      p.id = (uint32_t)pid;
      p.kc = A.kc_at[pid];
      p.dev = (uint32_t)(d + 1);
      p.flag = ODP_F_UT;
      A.pend[st->pend_cur][atomicAdd(&s_pend_n, 1u)] = p;
    }
  } else if (kind == K_ALLOCDEL) {
    if (ad_last) {
      Slot* sl = tupsert(A.t_ad, e.dst_addr, kMark | (uint64_t)(e.dst_dev + 1), 0, tag, 0, &ins);
      if (sl) {
        sl->v0 = e.op;
        sl->v1 = id;
      } else {
        st->overflow = 1;
      }
    }
    s_xchg[t] = kNone64;
    if (s_pid[t] != kNone64) {
      // Repeated allocation, keyed by the paired ALLOC's (host address,
      // device, bytes): the pairings of this key in this tick all read the
      // table's smallest ALLOC index before the tick; the first one then
      // stores the tick's smallest (phase 2b).
      const uint64_t pid = s_pid[t];
      const odp_event& a = A.log[pid];
      const uint64_t k0 = a.src_addr, k1 = kMark | (uint64_t)(a.dst_dev + 1), k2 = a.bytes;
      bool first = true;
      uint64_t tick_min = pid;
      for (uint32_t u = 0; u < A.m; ++u) {
        if (u == t || s_pid[u] == kNone64) continue;
        const odp_event& b = A.log[s_pid[u]];
        if (b.src_addr == k0 && b.dst_dev == a.dst_dev && b.bytes == k2) {
          if (u < t) first = false;
          tick_min = min(tick_min, s_pid[u]);
        }
      }
      const Slot* found = tfind(A.t_ra, k0, k1, k2);
      const uint64_t before = found ? found->v1 : kNone64;
      if (pid > min(before, tick_min)) known_or(A.known, pid, ODP_F_RA);
      if (first && before != kNone64 && before > tick_min) known_or(A.known, before, ODP_F_RA);
      if (first) s_xchg[t] = tick_min;
      // unused allocation: the window [ALLOC start, DELETE end]
      if (windows_on) {
        Pending p;
        p.lo = a.t_start;
        p.deadline = e.t_end;
        p.id = (uint32_t)pid;
        p.kc = A.kc_at[pid];
        p.dev = (uint32_t)(a.dst_dev + 1);
        p.flag = ODP_F_UA;
        A.pend[st->pend_cur][atomicAdd(&s_pend_n, 1u)] = p;
      }
    }
  } else if (kind == K_KERNEL) {
    // my place in my device's kernel list and the running maximum of the ends
    const int dv = e.dst_dev;
    const uint64_t row = (uint64_t)(dv + 1) * A.cap;
    const uint32_t k0 = s_kc0[dv + 1];
    uint64_t mx = k0 ? A.kmaxend[row + k0 - 1] : 0;
    for (uint32_t u = 0; u <= t; ++u)
      if (s_kind[u] == K_KERNEL && s_dst[u] == dv) mx = max(mx, s_te[u]);
    A.kstart[row + kc_me] = e.t_start;
    A.kmaxend[row + kc_me] = mx;
  }
  __syncthreads();
  // Phase 2b: the RA table and the RT_TX links (after every head swap).
  if (kind == K_ALLOCDEL && s_pid[t] != kNone64 && s_xchg[t] != kNone64) {
    const odp_event& a = A.log[s_pid[t]];
    Slot* sl = tupsert(A.t_ra, a.src_addr, kMark | (uint64_t)(a.dst_dev + 1), a.bytes, tag, kNone64, &ins);
    if (sl) atomicMin(reinterpret_cast<unsigned long long*>(&sl->v1), (unsigned long long)s_xchg[t]);
    else st->overflow = 1;
  }
  if (kind == K_TRANSFER && s_unmarked[t]) {
    const uint64_t h = e.digest;
    const int s = e.src_dev, d = e.dst_dev;
    int older = -1, last = -1;
    for (uint32_t u = 0; u < A.m; ++u) {
      if (!(s_kind[u] == K_TRANSFER && s_dig[u] == h && s_src[u] == s && s_dst[u] == d)) continue;
      if (u < t && s_unmarked[u]) older = (int)u;
      last = (int)u;  // the pair's last transfer of the tick took the old head
    }
    A.link[id] = older >= 0 ? (uint32_t)(A.base_id + older + 1) : (uint32_t)s_xchg[last];
  }
  if (t < kDev) {
    uint32_t c = 0;
    for (uint32_t u = 0; u < A.m; ++u) c += s_kind[u] == K_KERNEL && s_dst[u] == (int)t - 1;
    s_kc1[t] = s_kc0[t] + c;
  }
  __syncthreads();
  // Phase 3: the windows whose deadline has passed (a record starting after
  // it is logged, so no kernel still to come can meet the window) get their
  // flag when no kernel met them; the others wait for later ticks.
  const uint64_t now_ts = s_ts[A.m - 1];
  const uint32_t cur = st->pend_cur, np = s_pend_n;
  const Pending* P = A.pend[cur];
  Pending* Q = A.pend[cur ^ 1];
  for (uint32_t base = 0; base < np; base += kTickMax) {
    const uint32_t j = base + t;
    if (j >= np || !windows_on) continue;  // after a rejected record these bits wait for the drain
    const Pending p = P[j];
    if (p.deadline < now_ts) {
      const uint64_t row = (uint64_t)p.dev * A.cap;
      const bool before = p.kc > 0 && A.kmaxend[row + p.kc - 1] >= p.lo;
      const bool after = count_upto(A.kstart + row, s_kc1[p.dev], p.deadline) > p.kc;
      if (!before && !after) known_or(A.known, p.id, p.flag);
    } else {
      Q[atomicAdd(&s_keep, 1u)] = p;
    }
  }
  __syncthreads();
  if (t < kDev) st->kcount[t] = s_kc1[t];
  if (t == 0) {
    st->pend_n = s_keep;
    st->pend_cur = cur ^ 1;
    st->any_invalid |= tick_invalid ? 1u : 0u;
    st->last_t_start = now_ts;
    st->n_logged = A.base_id + A.m;
  }
}

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kTables = 6;

// Device bytes of a server's state for a log of `cap` records.
uint64_t state_bytes_for(uint64_t cap) {
  const uint64_t tcap = pow2_at_least(std::max<uint64_t>(1024, 2 * cap));
  return cap * (sizeof(odp_event) + 4 + 4) + ((cap + 8) & ~3ull) + 2ull * kDev * cap * 8 + 2 * cap * sizeof(Pending) +
         kTables * tcap * sizeof(Slot) + sizeof(ServeState) + 2ull * kTickMax * (kStageBytes + 8);
}

}  // namespace
}  // namespace odp

using namespace odp;

struct odp_server {
  int device = 0;
  hipStream_t stream = nullptr;   // classification (and every call's ordering point)
  hipStream_t dstream = nullptr;  // payload staging and digests
  odp_server_config cfg{};
  uint64_t state_bytes = 0;       // device memory of the server's state and digest workspace
  uint64_t payload_budget = 0;    // budget_bytes - state_bytes
  // device state
  odp_event* log = nullptr;
  uint8_t* known = nullptr;
  uint32_t* link = nullptr;
  uint32_t* kc_at = nullptr;
  uint64_t* kstart = nullptr;
  uint64_t* kmaxend = nullptr;
  Pending* pend[2] = {nullptr, nullptr};
  Table t_dd{}, t_rx{}, t_ad{}, t_tx{}, t_ra{}, t_ut{};
  ServeState* st = nullptr;
  // tick staging, double-buffered: one pinned host block and one device block
  // per buffer, packed as records[m] | payload pointers[m] | sizes[m] | has[m]
  uint8_t* h_stage[2] = {nullptr, nullptr};
  uint8_t* d_stage[2] = {nullptr, nullptr};
  uint64_t* d_dig[2] = {nullptr, nullptr};
  hipEvent_t digested[2] = {nullptr, nullptr};
  hipEvent_t done[2] = {nullptr, nullptr};
  uint64_t n_logged = 0;
  uint64_t n_ticks = 0;
};

static Table* table_at(odp_server* s, int i) {
  Table* t[kTables] = {&s->t_dd, &s->t_rx, &s->t_ad, &s->t_tx, &s->t_ra, &s->t_ut};
  return t[i];
}

static int server_alloc(odp_server* s) {
  const uint64_t cap = s->cfg.max_events;
  ODP_HIP(hipMalloc(&s->log, cap * sizeof(odp_event)));
  ODP_HIP(hipMalloc(&s->known, (cap + 8) & ~3ull));
  ODP_HIP(hipMalloc(&s->link, cap * 4));
  ODP_HIP(hipMalloc(&s->kc_at, cap * 4));
  ODP_HIP(hipMalloc(&s->kstart, (uint64_t)kDev * cap * 8));
  ODP_HIP(hipMalloc(&s->kmaxend, (uint64_t)kDev * cap * 8));
  for (int b = 0; b < 2; ++b) ODP_HIP(hipMalloc(&s->pend[b], cap * sizeof(Pending)));
  const uint64_t tcap = pow2_at_least(std::max<uint64_t>(1024, 2 * cap));
  for (int i = 0; i < kTables; ++i) {
    Table* T = table_at(s, i);
    ODP_HIP(hipMalloc(&T->slots, tcap * sizeof(Slot)));
    ODP_HIP(hipMemset(T->slots, 0, tcap * sizeof(Slot)));
    T->mask = tcap - 1;
  }
  ODP_HIP(hipMalloc(&s->st, sizeof(ServeState)));
  ODP_HIP(hipMemset(s->st, 0, sizeof(ServeState)));
  ODP_HIP(hipMemset(s->known, 0, (cap + 8) & ~3ull));
  for (int b = 0; b < 2; ++b) {
    ODP_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->h_stage[b]), kTickMax * kStageBytes, hipHostMallocDefault));
    ODP_HIP(hipMalloc(&s->d_stage[b], kTickMax * kStageBytes));
    ODP_HIP(hipMalloc(&s->d_dig[b], kTickMax * 8));
    ODP_HIP(hipEventCreateWithFlags(&s->digested[b], hipEventDisableTiming));
    ODP_HIP(hipEventCreateWithFlags(&s->done[b], hipEventDisableTiming));
  }
  return ODP_OK;
}

static void server_free(odp_server* s) {
  for (hipStream_t q : {s->dstream, s->stream}) {
    if (!q) continue;
    (void)hipStreamSynchronize(q);
    // the digest and analysis workspace the library keeps for this stream
    workspace_drop(s->device, q);
  }
  (void)hipFree(s->log);
  (void)hipFree(s->known);
  (void)hipFree(s->link);
  (void)hipFree(s->kc_at);
  (void)hipFree(s->kstart);
  (void)hipFree(s->kmaxend);
  for (int b = 0; b < 2; ++b) (void)hipFree(s->pend[b]);
  for (int i = 0; i < kTables; ++i) (void)hipFree(table_at(s, i)->slots);
  (void)hipFree(s->st);
  for (int b = 0; b < 2; ++b) {
    (void)hipHostFree(s->h_stage[b]);
    (void)hipFree(s->d_stage[b]);
    (void)hipFree(s->d_dig[b]);
    if (s->digested[b]) (void)hipEventDestroy(s->digested[b]);
    if (s->done[b]) (void)hipEventDestroy(s->done[b]);
  }
  if (s->dstream) (void)hipStreamDestroy(s->dstream);
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
  // The budget covers the server's state, its digest workspace and the
  // payload bytes of the requests in flight. The workspace is sized for
  // payload batches of at most the whole budget, so it is known up front.
  const uint64_t fixed = state_bytes_for(cfg->max_events) +
                         digest_workspace_bytes(kTickMax, cfg->budget_bytes + (uint64_t)kTickMax * kNodeBytes) +
                         digest_plain_workspace_bytes(cfg->budget_bytes);
  if (cfg->budget_bytes <= fixed)
    return set_error(ODP_EINVAL, "odp_server_create: a budget of %llu bytes does not cover the server's state and "
                                 "workspace (%llu bytes)", (unsigned long long)cfg->budget_bytes,
                     (unsigned long long)fixed);
  odp_server* s = new odp_server();
  s->cfg = *cfg;
  s->state_bytes = fixed;
  s->payload_budget = cfg->budget_bytes - fixed;
  if (cfg->mode == ODP_SERVER_PLAIN) s->cfg.max_tick = s->cfg.max_inflight = 1;
  int e = current_device(&s->device);
  if (!e) {
    hipError_t he = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&s->dstream, hipStreamNonBlocking);
    if (he != hipSuccess) e = check_hip(he, "hipStreamCreate");
  }
  if (!e) e = server_alloc(s);
  if (!e) {
    int err = 0;
    Workspace* ws = workspace_for(s->dstream, &err);
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

// Enqueues one tick: the staging copy and the digest of the payloads (one
// persistent batched launch, or per-buffer launches in the plain mode) on the
// digest stream; the classification on the server stream, after the digest.
// The digest of the next tick then runs during this classification. A tick
// submitted while none is in flight (`idle`) has nothing to overlap: its
// classification follows the digest on the digest stream itself, without the
// hop between streams. A later tick's classification stays ordered after it:
// its digest, which it waits for, follows it on the digest stream.
static int launch_tick(odp_server* s, int b, uint32_t m, uint64_t bytes, bool idle) {
  hipStream_t ds = s->dstream;
  hipStream_t cs = idle ? ds : s->stream;
  ODP_HIP(hipMemcpyAsync(s->d_stage[b], s->h_stage[b], m * kStageBytes, hipMemcpyHostToDevice, ds));
  const StageView hv = stage_view(s->h_stage[b], m), dv = stage_view(s->d_stage[b], m);
  // Tick sizes change every tick: direct launches rather than a captured
  // graph. A tick of up to kPerBufferTick requests takes per-buffer launches
  // (one kernel each instead of the plan, the persistent digest and the tree
  // kernels: fewer launches and a shorter chain on the device).
  int e = s->cfg.mode == ODP_SERVER_PLAIN || m <= kPerBufferTick
              ? odp_digest_buffers_plain(reinterpret_cast<const void* const*>(hv.ptr), hv.size, m, s->d_dig[b], ds)
              : digest_batched_direct(reinterpret_cast<const void* const*>(dv.ptr), dv.size, m, s->d_dig[b], ds, bytes);
  if (e) return e;
  if (!idle) {
    ODP_HIP(hipEventRecord(s->digested[b], ds));
    ODP_HIP(hipStreamWaitEvent(s->stream, s->digested[b], 0));
  }
  TickArgs A;
  A.tick_ev = dv.ev;
  A.tick_dig = s->d_dig[b];
  A.tick_haspay = dv.has;
  A.m = m;
  A.base_id = s->n_logged;
  // at most max_events < 2^32 ticks: tags never repeat
  A.tag = (uint32_t)(s->n_ticks % 0xFFFFFFFFull) + 1;
  A.log = s->log;
  A.known = s->known;
  A.link = s->link;
  A.kc_at = s->kc_at;
  A.kstart = s->kstart;
  A.kmaxend = s->kmaxend;
  A.cap = s->cfg.max_events;
  A.pend[0] = s->pend[0];
  A.pend[1] = s->pend[1];
  A.t_dd = s->t_dd;
  A.t_rx = s->t_rx;
  A.t_ad = s->t_ad;
  A.t_tx = s->t_tx;
  A.t_ra = s->t_ra;
  A.t_ut = s->t_ut;
  A.st = s->st;
  hipLaunchKernelGGL(serve_tick_kernel, dim3(1), dim3(kTickMax), 0, cs, A);
  ODP_HIP(hipGetLastError());
  ODP_HIP(hipEventRecord(s->done[b], cs));
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
    if (payload_bytes[i] > s->payload_budget)
      return set_error(ODP_EINVAL, "odp_server_run: request %zu payload above the budget left after the server's "
                                   "state (%llu bytes)", i, (unsigned long long)s->payload_budget);
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
        if (inflight_bytes + bytes + payload_bytes[i] > s->payload_budget) {
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
        int e = launch_tick(s, b, m, bytes, inflight.empty());
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
  lst.state_bytes = s->state_bytes;
  if (stats) *stats = lst;
  return ODP_OK;
}

extern "C" int odp_server_drain(odp_server* s, uint8_t* out_known, uint8_t* out_flags, odp_report* out_report) {
  if (!s) return set_error(ODP_EINVAL, "odp_server_drain: null server");
  ODP_HIP(hipStreamSynchronize(s->dstream));
  ODP_HIP(hipStreamSynchronize(s->stream));
  ServeState hs;
  ODP_HIP(hipMemcpy(&hs, s->st, sizeof(hs), hipMemcpyDeviceToHost));
  if (hs.overflow) return set_error(ODP_ECAPACITY, "odp_server_drain: a state table ran full");
  const uint64_t n = s->n_logged;
  if (out_known && n) ODP_HIP(hipMemcpyAsync(out_known, s->known, n, hipMemcpyDeviceToDevice, s->stream));
  if (out_flags || out_report) {
    if (!out_flags || !out_report) return set_error(ODP_EINVAL, "odp_server_drain: flags and report go together");
    int e = odp_analyze_trace(s->log, n, out_flags, out_report, s->stream);
    if (e) return e;
  }
  ODP_HIP(hipStreamSynchronize(s->dstream));
  ODP_HIP(hipStreamSynchronize(s->stream));
  return ODP_OK;
}

extern "C" int odp_server_log(odp_server* s, odp_event* out_events, size_t* n) {
  if (!s || !n) return set_error(ODP_EINVAL, "odp_server_log: null argument");
  ODP_HIP(hipStreamSynchronize(s->dstream));
  ODP_HIP(hipStreamSynchronize(s->stream));
  *n = s->n_logged;
  if (out_events && s->n_logged)
    ODP_HIP(hipMemcpy(out_events, s->log, s->n_logged * sizeof(odp_event), hipMemcpyDeviceToDevice));
  return ODP_OK;
}
