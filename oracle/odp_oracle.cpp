// Serial CPU oracle for the content digest and the mapping-trace analysis of
// "Dynamic Detection of Inefficient Data Mapping Patterns in Heterogeneous
// OpenMP Applications" (PPoPP '26).
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
// loads this file; only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark do. It shares no code, header or table with the GPU
// path: the event layout is re-declared here from the documented format.
//
// Everything here is plain, serial and written for checking by eye:
//   * xxh64      : XXH64 from the public xxHash specification (the paper's
//                  hash study, Appendix B, evaluates XXH64 among its 19 hashes).
//   * d64        : the chunked, tree-combined digest ODP-D64 v1 built on XXH64
//                  (leaves of 4096 bytes, fan-in 64, per-level seeds). The
//                  paper hashes each transfer whole (Sec. 5.1 and App. B); the
//                  tree form is this project's parallel definition.
//   * analyze    : the detection rules of Sec. 5 (Defs. 1-4 of Sec. 4 with the
//                  keys of Algorithms 1-5), computed by chronological passes
//                  over per-key state, and the optimization-potential sums of
//                  Sec. 7.6.
//   * alg2_pairs : the pairs Alg. 2 records, restated over per-endpoint
//                  arrival lists, to compare that algorithm with the
//                  round-trip rule where they differ (three or more endpoints).
// Parity status of each part is listed in the header of oracle/__init__.py.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <tuple>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

namespace {

// ----------------------------------------------------------------------------
// XXH64, public xxHash specification (five 64-bit primes, 32-byte stripes over
// four accumulators, then the remaining 8/4/1-byte pieces, then avalanche).
// ----------------------------------------------------------------------------
const uint64_t PRIME1 = 0x9E3779B185EBCA87ULL;
const uint64_t PRIME2 = 0xC2B2AE3D27D4EB4FULL;
const uint64_t PRIME3 = 0x165667B19E3779F9ULL;
const uint64_t PRIME4 = 0x85EBCA77C2B2AE63ULL;
const uint64_t PRIME5 = 0x27D4EB2F165667C5ULL;

uint64_t rotl(uint64_t x, int r) { return (x << r) | (x >> (64 - r)); }

uint64_t read_le64(const uint8_t* p) {
  uint64_t v = 0;
  for (int i = 0; i < 8; ++i) v |= (uint64_t)p[i] << (8 * i);
  return v;
}
uint32_t read_le32(const uint8_t* p) {
  uint32_t v = 0;
  for (int i = 0; i < 4; ++i) v |= (uint32_t)p[i] << (8 * i);
  return v;
}

uint64_t xxh_round(uint64_t acc, uint64_t input) {
  acc += input * PRIME2;
  acc = rotl(acc, 31);
  acc *= PRIME1;
  return acc;
}
uint64_t xxh_merge(uint64_t h, uint64_t acc) {
  h ^= xxh_round(0, acc);
  h = h * PRIME1 + PRIME4;
  return h;
}

uint64_t xxh64(const uint8_t* p, uint64_t len, uint64_t seed) {
  const uint8_t* end = p + len;
  uint64_t h;
  if (len >= 32) {
    uint64_t v1 = seed + PRIME1 + PRIME2;
    uint64_t v2 = seed + PRIME2;
    uint64_t v3 = seed;
    uint64_t v4 = seed - PRIME1;
    const uint8_t* limit = end - 32;
    do {
      v1 = xxh_round(v1, read_le64(p));
      v2 = xxh_round(v2, read_le64(p + 8));
      v3 = xxh_round(v3, read_le64(p + 16));
      v4 = xxh_round(v4, read_le64(p + 24));
      p += 32;
    } while (p <= limit);
    h = rotl(v1, 1) + rotl(v2, 7) + rotl(v3, 12) + rotl(v4, 18);
    h = xxh_merge(h, v1);
    h = xxh_merge(h, v2);
    h = xxh_merge(h, v3);
    h = xxh_merge(h, v4);
  } else {
    h = seed + PRIME5;
  }
  h += len;
  while (p + 8 <= end) {
    h ^= xxh_round(0, read_le64(p));
    h = rotl(h, 27) * PRIME1 + PRIME4;
    p += 8;
  }
  if (p + 4 <= end) {
    h ^= (uint64_t)read_le32(p) * PRIME1;
    h = rotl(h, 23) * PRIME2 + PRIME3;
    p += 4;
  }
  while (p < end) {
    h ^= (uint64_t)(*p) * PRIME5;
    h = rotl(h, 11) * PRIME1;
    p += 1;
  }
  h ^= h >> 33;
  h *= PRIME2;
  h ^= h >> 29;
  h *= PRIME3;
  h ^= h >> 32;
  return h;
}

// ----------------------------------------------------------------------------
// ODP-D64 v1: leaves of L = 4096 bytes hashed with seed 0; then, level by
// level, groups of up to F = 64 child digests serialised little-endian and
// hashed with seed = level number, until one digest remains. Inputs of at most
// one leaf are hashed directly (the empty input included).
// ----------------------------------------------------------------------------
const uint64_t LEAF = 4096;
const uint64_t FANIN = 64;

uint64_t d64(const uint8_t* p, uint64_t n) {
  if (n <= LEAF) return xxh64(p, n, 0);
  std::vector<uint64_t> level;
  for (uint64_t off = 0; off < n; off += LEAF) level.push_back(xxh64(p + off, std::min(LEAF, n - off), 0));
  uint64_t seed = 0;
  while (level.size() > 1) {
    seed += 1;
    std::vector<uint64_t> parent;
    for (size_t first = 0; first < level.size(); first += FANIN) {
      size_t last = std::min(level.size(), (size_t)(first + FANIN));
      std::vector<uint8_t> bytes;
      for (size_t c = first; c < last; ++c)
        for (int b = 0; b < 8; ++b) bytes.push_back((uint8_t)(level[c] >> (8 * b)));
      parent.push_back(xxh64(bytes.data(), bytes.size(), seed));
    }
    level.swap(parent);
  }
  return level[0];
}

}  // namespace

// ----------------------------------------------------------------------------
// Event log record and report, re-declared from the documented 64-byte layout.
// ----------------------------------------------------------------------------
extern "C" {

struct orc_event {
  uint64_t digest;    // transfers: digest of the bytes moved
  uint64_t src_addr;  // transfers: source address; ALLOC/DELETE: host address
  uint64_t dst_addr;  // transfers: destination address; ALLOC/DELETE: device address
  uint64_t bytes;
  uint64_t t_start, t_end;
  uint64_t codeptr;
  int16_t src_dev, dst_dev;  // -1 = host; ALLOC/DELETE/KERNEL use dst_dev
  uint8_t op, rsv0;
  uint16_t rsv1;
};
static_assert(sizeof(orc_event) == 64, "event record is 64 bytes");

struct orc_report {
  uint64_t n_events, n_invalid, n_transfers, n_kernels;
  uint64_t n_alloc_pairs, n_unpaired_alloc, n_unpaired_delete;
  uint64_t dd_events, dd_groups, dd_members, dd_bytes, dd_time_ns;
  uint64_t rt_pairs, rt_rx_events, rt_bytes, rt_time_ns;
  uint64_t ra_events, ra_groups, ra_members, ra_bytes, ra_time_ns;
  uint64_t ua_events, ua_bytes, ua_time_ns;
  uint64_t ut_events, ut_bytes, ut_time_ns;
  uint64_t span_ns, elim_ns;
  double predicted_speedup;
  int32_t status;
  uint32_t first_bad_event;
};
static_assert(sizeof(orc_report) == 248, "report is 248 bytes");

enum { OP_ALLOC = 1, OP_H2D = 2, OP_D2H = 3, OP_D2D = 4, OP_DELETE = 5, OP_KERNEL = 6 };
enum { F_DD = 1, F_RT_TX = 2, F_RT_RX = 4, F_RA = 8, F_UA = 16, F_PAIRED = 32, F_UT = 64, F_INVALID = 128 };
const int MAX_DEVICE = 9;  // device numbers -1 (host) .. 9 are accepted

uint64_t orc_xxh64(const uint8_t* p, uint64_t n, uint64_t seed) { return xxh64(p, n, seed); }
uint64_t orc_d64(const uint8_t* p, uint64_t n) { return d64(p, n); }
void orc_d64_many(const uint8_t* const* ptrs, const uint64_t* sizes, uint64_t n, uint64_t* out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = d64(ptrs[i], sizes[i]);
}

// Hash of a small tuple of integers, for the per-key state of the rules.
struct KeyHash {
  size_t operator()(const std::pair<uint64_t, int>& k) const { return mix(k.first, (uint64_t)k.second, 0); }
  size_t operator()(const std::pair<int, uint64_t>& k) const { return mix((uint64_t)k.first, k.second, 0); }
  size_t operator()(const std::tuple<uint64_t, int, int>& k) const {
    return mix(std::get<0>(k), (uint64_t)std::get<1>(k), (uint64_t)std::get<2>(k));
  }
  size_t operator()(const std::tuple<uint64_t, int, uint64_t>& k) const {
    return mix(std::get<0>(k), (uint64_t)std::get<1>(k), std::get<2>(k));
  }
  size_t operator()(const std::tuple<int, int, uint64_t>& k) const {
    return mix((uint64_t)std::get<0>(k), (uint64_t)std::get<1>(k), std::get<2>(k));
  }
  static size_t mix(uint64_t a, uint64_t b, uint64_t c) {
    uint64_t h = a * 0x9E3779B97F4A7C15ULL;
    h ^= (b + 0x632BE59BD9B4E019ULL + (h << 6) + (h >> 2)) * 0xC2B2AE3D27D4EB4FULL;
    h ^= (c + 0x27D4EB2F165667C5ULL + (h << 6) + (h >> 2)) * 0x9E3779B97F4A7C15ULL;
    return (size_t)(h ^ (h >> 29));
  }
};

static bool is_transfer(uint8_t op) { return op == OP_H2D || op == OP_D2H || op == OP_D2D; }
static bool dev_ok(int d) { return d >= -1 && d <= MAX_DEVICE; }
static uint64_t dur(const orc_event& e) { return e.t_end - e.t_start; }

// Validity: known op code, t_end >= t_start, t_start not below the previous
// record's (the log is chronological), and the device numbers the record uses
// within range. Invalid records take part in no rule.
static bool event_valid(const orc_event* ev, uint64_t i) {
  const orc_event& e = ev[i];
  if (e.op < OP_ALLOC || e.op > OP_KERNEL) return false;
  if (e.t_end < e.t_start) return false;
  if (i > 0 && e.t_start < ev[i - 1].t_start) return false;
  if (!dev_ok(e.dst_dev)) return false;
  if (is_transfer(e.op) && !dev_ok(e.src_dev)) return false;
  return true;
}

// Kernel intervals of one device, as two sorted lists. The number of kernels
// whose closed interval [t_start, t_end] meets the closed interval [lo, hi]
// (lo <= hi) is
//   #{kernels with t_start <= hi} - #{kernels with t_end < lo},
// because a kernel that ends before lo also starts before hi; what remains
// are the kernels that start by hi and end at or after lo.
struct DeviceKernels {
  std::vector<uint64_t> starts, ends;
  uint64_t meeting(uint64_t lo, uint64_t hi) const {
    const uint64_t started = std::upper_bound(starts.begin(), starts.end(), hi) - starts.begin();
    const uint64_t ended = std::lower_bound(ends.begin(), ends.end(), lo) - ends.begin();
    return started - ended;
  }
};

// The detection rules, one chronological pass per rule. flags[i] receives the
// F_* bits of record i; *rep receives the counts and sums.
int orc_analyze(const orc_event* ev, uint64_t n, uint8_t* flags, orc_report* rep) {
  std::memset(rep, 0, sizeof(*rep));
  rep->n_events = n;
  rep->first_bad_event = 0xFFFFFFFFu;
  std::vector<char> valid(n);
  for (uint64_t i = 0; i < n; ++i) {
    valid[i] = event_valid(ev, i);
    flags[i] = valid[i] ? 0 : F_INVALID;
    if (!valid[i]) {
      rep->n_invalid++;
      if (rep->status == 0) { rep->status = 1; rep->first_bad_event = (uint32_t)i; }
    }
  }
  std::vector<uint64_t> transfers, allocdel, kernels;
  for (uint64_t i = 0; i < n; ++i) {
    if (!valid[i]) continue;
    if (is_transfer(ev[i].op)) transfers.push_back(i);
    else if (ev[i].op == OP_ALLOC || ev[i].op == OP_DELETE) allocdel.push_back(i);
    else kernels.push_back(i);
  }
  rep->n_transfers = transfers.size();
  rep->n_kernels = kernels.size();

  // Duplicate transfer (Def. 1, key <hash, receiving device> of Alg. 1): a
  // transfer is a duplicate when the same receiver already got the same digest.
  {
    std::unordered_map<std::pair<uint64_t, int>, uint64_t, KeyHash> count;
    for (uint64_t i : transfers) {
      auto key = std::make_pair(ev[i].digest, (int)ev[i].dst_dev);
      if (count[key] > 0) {
        flags[i] |= F_DD;
        rep->dd_events++;
        rep->dd_bytes += ev[i].bytes;
        rep->dd_time_ns += dur(ev[i]);
      }
      count[key]++;
    }
    for (auto& kv : count)
      if (kv.second >= 2) { rep->dd_groups++; rep->dd_members += kv.second; }
  }

  // Round trip (Def. 2). Self-transfers (src == dst) take no part.
  //   RT_TX: a strictly later transfer carries the same digest in the reverse
  //          direction (A sent to B; later A gets the same data back from B).
  //   RT_RX: the latest earlier transfer with the same digest between the same
  //          two endpoints went the other way (this record is a return leg).
  {
    std::unordered_set<std::tuple<uint64_t, int, int>, KeyHash> later;
    for (size_t k = transfers.size(); k-- > 0;) {
      const orc_event& e = ev[transfers[k]];
      if (e.src_dev == e.dst_dev) continue;
      if (later.count(std::make_tuple(e.digest, (int)e.dst_dev, (int)e.src_dev))) {
        flags[transfers[k]] |= F_RT_TX;
        rep->rt_pairs++;
      }
      later.insert(std::make_tuple(e.digest, (int)e.src_dev, (int)e.dst_dev));
    }
    std::unordered_map<std::tuple<uint64_t, int, int>, std::pair<int, int>, KeyHash> last_dir;
    for (uint64_t i : transfers) {
      const orc_event& e = ev[i];
      if (e.src_dev == e.dst_dev) continue;
      int lo = std::min((int)e.src_dev, (int)e.dst_dev), hi = std::max((int)e.src_dev, (int)e.dst_dev);
      auto key = std::make_tuple(e.digest, lo, hi);
      auto it = last_dir.find(key);
      if (it != last_dir.end() && it->second == std::make_pair((int)e.dst_dev, (int)e.src_dev)) {
        flags[i] |= F_RT_RX;
        rep->rt_rx_events++;
        rep->rt_bytes += e.bytes;
        rep->rt_time_ns += dur(e);
      }
      last_dir[key] = std::make_pair((int)e.src_dev, (int)e.dst_dev);
    }
  }

  // Allocation/deletion pairing (the helper the paper calls in Algs. 3 and 4):
  // records grouped by (device, device address) in log order; a DELETE pairs
  // with the record just before it in its group when that record is an ALLOC.
  std::vector<std::pair<uint64_t, uint64_t>> pairs;  // (alloc, delete), in delete order
  {
    std::unordered_map<std::pair<int, uint64_t>, uint64_t, KeyHash> prev;
    for (uint64_t i : allocdel) {
      auto key = std::make_pair((int)ev[i].dst_dev, ev[i].dst_addr);
      auto it = prev.find(key);
      if (ev[i].op == OP_DELETE && it != prev.end() && ev[it->second].op == OP_ALLOC) {
        pairs.emplace_back(it->second, i);
        flags[it->second] |= F_PAIRED;
        flags[i] |= F_PAIRED;
      }
      prev[key] = i;
    }
    std::sort(pairs.begin(), pairs.end());  // alloc order
    rep->n_alloc_pairs = pairs.size();
    for (uint64_t i : allocdel) {
      if (flags[i] & F_PAIRED) continue;
      if (ev[i].op == OP_ALLOC) rep->n_unpaired_alloc++; else rep->n_unpaired_delete++;
    }
  }

  // Repeated allocation (Def. 3, key <host address, device, bytes> of Alg. 3):
  // every paired allocation after the first of its key. Its bytes are the
  // ALLOC's; its time is the ALLOC's and the paired DELETE's durations.
  {
    std::unordered_map<std::tuple<uint64_t, int, uint64_t>, uint64_t, KeyHash> count;
    for (auto& pr : pairs) {
      const orc_event& a = ev[pr.first];
      auto key = std::make_tuple(a.src_addr, (int)a.dst_dev, a.bytes);
      if (count[key] > 0) {
        flags[pr.first] |= F_RA;
        rep->ra_events++;
        rep->ra_bytes += a.bytes;
        rep->ra_time_ns += dur(a) + dur(ev[pr.second]);
      }
      count[key]++;
    }
    for (auto& kv : count)
      if (kv.second >= 2) { rep->ra_groups++; rep->ra_members += kv.second; }
  }

  // Kernel intervals per device, for both unused-mapping rules.
  std::map<int, DeviceKernels> dk;
  for (uint64_t k : kernels) {
    dk[ev[k].dst_dev].starts.push_back(ev[k].t_start);
    dk[ev[k].dst_dev].ends.push_back(ev[k].t_end);
  }
  for (auto& kv : dk) {
    std::sort(kv.second.starts.begin(), kv.second.starts.end());
    std::sort(kv.second.ends.begin(), kv.second.ends.end());
  }
  auto kernels_meeting = [&](int dev, uint64_t lo, uint64_t hi) -> uint64_t {
    auto it = dk.find(dev);
    return it == dk.end() ? 0 : it->second.meeting(lo, hi);
  };

  // Unused allocation (Def. 4, allocation half; Alg. 4): the closed interval
  // [alloc.t_start, delete.t_end] meets no kernel's [t_start, t_end] on the
  // same device.
  for (auto& pr : pairs) {
    const orc_event& a = ev[pr.first];
    const orc_event& d = ev[pr.second];
    if (kernels_meeting(a.dst_dev, a.t_start, d.t_end) == 0) {
      flags[pr.first] |= F_UA;
      rep->ua_events++;
      rep->ua_bytes += a.bytes;
      rep->ua_time_ns += dur(a) + dur(d);
    }
  }

  // Unused transfer (Def. 4, transfer half; Alg. 5): data copied into device
  // memory that no kernel on that device can read before the next copy to the
  // same place overwrites it, or ever, when no such copy follows. Readings:
  //   * the device a transfer writes is its dst_dev, for an H2D or a D2D; a
  //     D2H writes host memory, which the definition does not cover;
  //   * "the same place" is the transfer's (dst_dev, src_dev, src_addr):
  //     Alg. 5 keys by the host address, the same key when every copy into a
  //     device comes from the host; a D2D source address is device memory;
  //   * a kernel can read the copy when its closed interval meets
  //     [copy.t_start, next.t_start], where next is the next copy of the same
  //     key in log order (no upper end when there is none): the kernel is
  //     still running or not yet started when the copy begins, and starts no
  //     later than the overwrite begins. With kernels that do not overlap
  //     this is Alg. 5's pointer and candidate rule; it also holds when
  //     kernels on a device overlap (the count form above).
  {
    std::unordered_map<std::tuple<int, int, uint64_t>, uint64_t, KeyHash> next_of_key;
    std::vector<uint64_t> nxt(n, UINT64_MAX);
    for (size_t k = transfers.size(); k-- > 0;) {
      const uint64_t i = transfers[k];
      const orc_event& t = ev[i];
      if (!(t.op == OP_H2D || t.op == OP_D2D) || t.dst_dev < 0) continue;
      const auto key = std::make_tuple((int)t.dst_dev, (int)t.src_dev, t.src_addr);
      auto it = next_of_key.find(key);
      if (it != next_of_key.end()) nxt[i] = it->second;
      next_of_key[key] = i;
    }
    for (uint64_t i : transfers) {
      const orc_event& t = ev[i];
      if (!(t.op == OP_H2D || t.op == OP_D2D) || t.dst_dev < 0) continue;
      const uint64_t hi = nxt[i] == UINT64_MAX ? UINT64_MAX : ev[nxt[i]].t_start;
      if (kernels_meeting(t.dst_dev, t.t_start, hi) == 0) {
        flags[i] |= F_UT;
        rep->ut_events++;
        rep->ut_bytes += t.bytes;
        rep->ut_time_ns += dur(t);
      }
    }
  }

  // Optimization potential (Sec. 7.6): the time that removing the flagged
  // mappings would save, each record counted once whatever flags it carries.
  // A transfer flagged as a duplicate, a round-trip return leg or unused is
  // removable; a repeated or unused allocation removes its ALLOC and its
  // DELETE. The run's total time is the log's span, from the earliest valid
  // start to the latest valid end; the predicted speedup is
  // span / (span - eliminable), +infinity when nothing would be left, 1 for an
  // empty span.
  {
    for (uint64_t i : transfers)
      if (flags[i] & (F_DD | F_RT_RX | F_UT)) rep->elim_ns += dur(ev[i]);
    for (auto& pr : pairs)
      if (flags[pr.first] & (F_RA | F_UA)) rep->elim_ns += dur(ev[pr.first]) + dur(ev[pr.second]);
    bool any = false;
    uint64_t first = 0, last = 0;
    for (uint64_t i = 0; i < n; ++i) {
      if (!valid[i]) continue;
      first = any ? std::min(first, ev[i].t_start) : ev[i].t_start;
      last = any ? std::max(last, ev[i].t_end) : ev[i].t_end;
      any = true;
    }
    rep->span_ns = any ? last - first : 0;
    if (rep->span_ns == 0) rep->predicted_speedup = 1.0;
    else if (rep->elim_ns >= rep->span_ns) rep->predicted_speedup = INFINITY;
    else rep->predicted_speedup = (double)rep->span_ns / (double)(rep->span_ns - rep->elim_ns);
  }
  return 0;
}

// The pairs Alg. 2 records, for comparing that algorithm with the round-trip
// rule above (they differ with three or more endpoints; see the readings).
// Alg. 2 matches each transfer, in log order, against the transfers received
// by its source endpoint: for a digest h and an endpoint d, let R(h, d) be
// the transfers of h received by d, in log order, and c(h, d) how many of
// them have been used up. A transfer tx of h is matched to element
// c(h, tx.src) of R(h, tx.src) when that exists; a matched transfer uses up
// one element of R(h, tx.dst), the list that holds tx itself.
// `idx` lists the transfers (positions in the event array, log order).
// Output: tx_pos[p], rx_pos[p] (positions in idx) in match order. Returns the
// number of pairs.
int64_t orc_alg2_pairs(const orc_event* ev, const uint64_t* idx, uint64_t m, int64_t* tx_pos, int64_t* rx_pos) {
  std::map<std::pair<uint64_t, int>, std::vector<uint64_t>> received;  // R(h, d): positions in idx
  std::map<std::pair<uint64_t, int>, uint64_t> used;                   // c(h, d)
  for (uint64_t k = 0; k < m; ++k) received[std::make_pair(ev[idx[k]].digest, (int)ev[idx[k]].dst_dev)].push_back(k);
  int64_t np = 0;
  for (uint64_t k = 0; k < m; ++k) {
    const orc_event& tx = ev[idx[k]];
    const auto from = std::make_pair(tx.digest, (int)tx.src_dev);
    auto r = received.find(from);
    const uint64_t c = used[from];
    if (r == received.end() || c >= r->second.size()) continue;
    tx_pos[np] = (int64_t)k;
    rx_pos[np] = (int64_t)r->second[c];
    np++;
    used[std::make_pair(tx.digest, (int)tx.dst_dev)]++;
  }
  return np;
}

}  // extern "C"
