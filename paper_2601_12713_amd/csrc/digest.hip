// ODP-D64 v1 content digest on gfx950.
//
// The paper hashes every transferred buffer with one serial 64-bit hash on the
// host (Sec. 5.1, App. B). Here every 4096-byte leaf is hashed by four lanes of
// a wavefront (one per XXH64 accumulator); leaves are staged through LDS from
// coalesced 128-bit nontemporal loads, and leaf digests are combined into
// level-1 node digests (64 leaves, 256 KiB) inside the workgroup or wavefront.
//
// Plain form (one launch per buffer): one workgroup per level-1 node; the
// upper levels are finished by whichever workgroup completes the last level-1
// node (one atomic ticket per buffer up to 1 GiB, one per node above that).
//
// Batched form (one persistent launch for n buffers): a device-side plan
// splits the buffers into work items: level-1 nodes hashed by a whole
// workgroup, groups of four small level-1 nodes (at most `split` bytes, one per
// wavefront), and groups of 64 buffers of at most one leaf. Workgroups claim
// items ahead of time and carry their load pipeline from one node into the
// next; level-1 digests are stored without waiting, and a second kernel climbs
// the levels above.
#include "internal.h"
#include "xxh64_dev.h"

namespace odp {
namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kRows = 64;                  // rows per item
constexpr int kRowsPerWave = kRows / kWaves;
constexpr int kPad = 16;                   // LDS row padding (bank spread)
// Bytes of each row staged per step: 512 in the one-launch-per-buffer kernel,
// 256 in the persistent batched kernel, whose loop keeps more state live (the
// smaller step frees the load registers that the larger one spills there).
constexpr int kSlabOne = 512;
constexpr int kSlabBatch = 256;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct RowDesc {
  const uint8_t* base;
  uint32_t len;
  uint32_t present;
};

template <int SLAB>
struct Smem {
  uint8_t slab[kWaves][kRowsPerWave * (SLAB + kPad)];
  RowDesc rows[kRows];
  uint64_t leafdig[2][kRows];  // leaf digests of the current and the previous item
  uint32_t outidx[kRows];
  uint32_t ring[3];            // claimed work items, two ahead of the one in progress
};

// Work record of one level-1 node item, written by the plan.
struct NodeRec {
  const uint8_t* base;  // first byte of the node
  uint64_t* dst;        // where the node digest goes: out[i] for a one-node buffer, else its level-1 tree slot
  uint32_t len;         // bytes in the node, 1 .. kNodeBytes
  uint32_t buf;         // buffer index i
};

__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

__host__ __device__ __forceinline__ uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Tree slots below the root and ticket slots (levels >= 2) of a buffer with
// n1 level-1 nodes.
__host__ __device__ inline void tree_need(uint64_t n1, uint64_t& tree_slots, uint64_t& tk_slots) {
  tree_slots = 0;
  tk_slots = 0;
  uint64_t nj = n1;
  while (nj > 1) {
    tree_slots += nj;
    nj = (nj + kFanIn - 1) / kFanIn;
    tk_slots += nj;
  }
}

typedef __attribute__((address_space(1))) const u32x4 gu32x4;

__device__ __forceinline__ u32x4 ld_global_nt(const uint8_t* p) {
  return __builtin_nontemporal_load(reinterpret_cast<gu32x4*>(reinterpret_cast<uintptr_t>(p)));
}

template <typename T>
__device__ __forceinline__ T uniform(T v) {
  static_assert(sizeof(T) == 8 || sizeof(T) == 4, "");
  if constexpr (sizeof(T) == 4) {
    return (T)__builtin_amdgcn_readfirstlane((int)v);
  } else {
    uint64_t x = (uint64_t)v;
    uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return (T)(((uint64_t)hi << 32) | lo);
  }
}

__device__ __forceinline__ const uint8_t* uniform_ptr(const uint8_t* p) {
  return reinterpret_cast<const uint8_t*>(uniform(reinterpret_cast<uint64_t>(p)));
}

// Finishes the XXH64 of one row from its four lane accumulators; the result
// is valid in lane 4r (accumulator 0) of row r.
__device__ __forceinline__ uint64_t finish_row(uint64_t acc, const RowDesc& hrow) {
  const int a = threadIdx.x & 3;
  uint64_t v1, v2, v3, v4;
  xx_gather4(acc, v1, v2, v3, v4);
  uint64_t h = 0;
  if (a == 0 && hrow.present) {
    const uint32_t nstripes = hrow.len >> 5;
    h = nstripes ? xx_converge(v1, v2, v3, v4) : kP5;
    h += hrow.len;
    h = xx_tail_bytes(h, hrow.base + nstripes * 32, hrow.len - nstripes * 32);
    h = xx_avalanche(h);
  }
  return h;
}

// Fast path as one stage of a wavefront's continuous stream of items: 16
// whole, 16-byte aligned leaves at leaf_base + r*4096 (leaf_base wave-uniform).
// Each step stages 64*NL bytes of every leaf (512 bytes, 8 KiB per wavefront,
// in the per-buffer kernel; 256 in the batched one) through the wavefront's
// LDS slab with NL 128-bit nontemporal loads per lane; load k
// covers 128 contiguous bytes of 8 leaves (lane L: leaf L/8 + 8*(k%2), bytes
// 128*(k/2) + 16*(L%8)), so every address is one of two per-lane offsets from
// the uniform base plus an immediate. Lane 4r+a then folds accumulator a's
// words of leaf r. Two steps are in flight while one is hashed.
// On entry, `pre` says whether RA/RB already hold the first two steps (loaded
// while the previous item was hashed). When `next` (the next item's leaves
// for this wavefront, same shape) is non-null, its first two steps are loaded
// during the last two steps here and `pre` is set, so the loads in flight do
// not drain between items. Returns the leaf digest in lane 4r.
// Buffer resource over a wave-uniform base (raw addressing, no stride, no
// range limit below 4 GiB): keeps every address of a step as one scalar base
// plus a 32-bit lane offset and an immediate.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wave_rsrc(const uint8_t* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(base), (short)0, -1, 0x00020000);
}

template <int NL>
__device__ __forceinline__ void fast_load(u32x4 (&R)[NL], const uint8_t* base, uint32_t step_off) {
  const int lane = threadIdx.x & 63;
  const __amdgpu_buffer_rsrc_t rs = wave_rsrc(base);
  const uint32_t o = (uint32_t)(lane >> 3) * kLeaf + (uint32_t)(lane & 7) * 16;
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const uint32_t vo = o + (uint32_t)(8 * (k & 1)) * kLeaf + (uint32_t)(k >> 1) * 128;
    R[k] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)vo, (int)step_off, 2 /* nt */));
  }
}

template <int NL>
__device__ __forceinline__ void fast_stage(const u32x4 (&R)[NL], uint8_t* slab) {
  constexpr int kStride = NL * 64 + kPad;
  const int lane = threadIdx.x & 63;
  uint8_t* const wr = slab + (lane >> 3) * kStride + (lane & 7) * 16;
#pragma unroll
  for (int k = 0; k < NL; ++k) *reinterpret_cast<u32x4*>(wr + 8 * (k & 1) * kStride + (k >> 1) * 128) = R[k];
}

template <int SLAB>
__device__ __forceinline__ uint64_t fast_fold(uint64_t acc, const uint8_t* slab) {
  constexpr int kStride = SLAB + kPad;
  const int lane = threadIdx.x & 63;
  const uint8_t* const rd = slab + (lane >> 2) * kStride + (lane & 3) * 8;
#pragma unroll
  for (int h2 = 0; h2 < SLAB / 128; ++h2) {
    uint64_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = *reinterpret_cast<const uint64_t*>(rd + (h2 * 4 + q) * 32);
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = xx_round(acc, w[q]);
  }
  return acc;
}

template <int NL>
__device__ __forceinline__ uint64_t hash_wave_leaves_pipe(const uint8_t* leaf_base, const uint8_t* next, bool& pre,
                                                          u32x4 (&RA)[NL], u32x4 (&RB)[NL], uint8_t* slab) {
  constexpr int kSlab = NL * 64;  // NL 128-bit loads per lane cover one step
  constexpr uint32_t NS = kLeaf / kSlab;
  const int lane = threadIdx.x & 63;
  uint64_t acc = xx_acc_init(0, lane & 3);
  if (!pre) {
    fast_load(RA, leaf_base, 0);
    fast_load(RB, leaf_base, kSlab);
  }
#pragma unroll 1
  for (uint32_t s = 0; s < NS; s += 2) {
    fast_stage(RA, slab);
    if (s + 2 < NS) fast_load(RA, leaf_base, (s + 2) * kSlab);
    else if (next) fast_load(RA, next, 0);
    wave_fence();
    acc = fast_fold<kSlab>(acc, slab);
    wave_fence();
    fast_stage(RB, slab);
    if (s + 3 < NS) fast_load(RB, leaf_base, (s + 3) * kSlab);
    else if (next) fast_load(RB, next, kSlab);
    wave_fence();
    acc = fast_fold<kSlab>(acc, slab);
    wave_fence();
  }
  pre = next != nullptr;
  RowDesc full;
  full.base = leaf_base + (lane >> 2) * kLeaf;
  full.len = kLeaf;
  full.present = 1;
  return finish_row(acc, full);
}

// General path: 16 rows of any length (<= 4096) and presence. When every
// present row is 16-byte aligned, rows are staged through LDS like the fast
// path (same lane mapping, two steps in flight) with loads predicated on each
// row's length; a 16-byte load that crosses a row's end stays inside the
// row's last 16-byte granule, so inside the same page. Otherwise every lane
// reads its words straight from memory at any alignment, eight stripes per
// batch of independent loads. Returns the row digest in lane 4r.
// A 16-byte granule that row loads past a row's end read instead.
__device__ __align__(16) uint8_t g_no_row[16];

// In the per-buffer kernel every lane issues every load of the step, without
// a branch: a load under a branch makes the compiler wait for all loads in
// flight at the next stage, which serialised the two steps kept in flight (a
// partial node of 2-16 leaves took 9.8 us per launch). An offset at or past
// the row's end (or an absent row) reads g_no_row instead; those bytes are
// staged but never folded. The batched kernel keeps predicated loads: the
// address selects cost it a register spill.
template <int kSlab>
__device__ __forceinline__ void rows_load(u32x4 (&R)[kSlab / 64], const RowDesc& ra, const RowDesc& rb, uint32_t step_off) {
  const int lane = threadIdx.x & 63;
  const uint32_t lc = (uint32_t)(lane & 7) * 16;
#pragma unroll
  for (int k = 0; k < kSlab / 64; ++k) {
    const RowDesc& d = (k & 1) ? rb : ra;
    const uint32_t o = step_off + (uint32_t)(k >> 1) * 128 + lc;
    if constexpr (kSlab == kSlabOne) {
      R[k] = ld_global_nt(o < d.len ? d.base + o : g_no_row);
    } else {
      if (o < d.len) R[k] = ld_global_nt(d.base + o);
    }
  }
}

// One staged step of a row: lane 4r+a folds accumulator a's words of row r
// for the step's stripes q0.. that lie below the row's nstripes. In the
// per-buffer kernel the step's words are read from LDS four at a time ahead
// of their rounds, so the serial rounds wait on LDS once per four stripes,
// not once each (a one-leaf buffer: 9.0 instead of 13.2 us per launch); reads
// past a short row's end stay inside its slab row and are not folded. The
// batched kernel keeps one read per round: there the held words push it past
// its register budget, and it ran 2% slower.
template <int kSlab>
__device__ __forceinline__ uint64_t rows_fold(uint64_t acc, const uint8_t* rd, uint32_t q0, uint32_t nstripes,
                                              bool whole) {
  if constexpr (kSlab != kSlabOne) {
#pragma unroll
    for (int q = 0; q < kSlab / 32; ++q)
      if (q0 + q < nstripes) acc = xx_round(acc, *reinterpret_cast<const uint64_t*>(rd + q * 32));
    return acc;
  } else {
    if (whole) {
      // every present row covers the whole step: no per-round predicate
      uint64_t w[kSlab / 32];
#pragma unroll
      for (int q = 0; q < kSlab / 32; ++q) w[q] = *reinterpret_cast<const uint64_t*>(rd + q * 32);
#pragma unroll
      for (int q = 0; q < kSlab / 32; ++q) acc = xx_round(acc, w[q]);
      return acc;
    }
#pragma unroll
    for (int g = 0; g < kSlab / 128; ++g) {
      uint64_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) w[q] = *reinterpret_cast<const uint64_t*>(rd + (g * 4 + q) * 32);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint64_t folded = xx_round(acc, w[q]);
        acc = q0 + g * 4 + q < nstripes ? folded : acc;
      }
    }
    return acc;
  }
}

template <int kSlab>
__device__ __forceinline__ uint64_t hash_wave_rows(const RowDesc* rows, uint8_t* slab) {
  constexpr int kStride = kSlab + kPad;
  const int lane = threadIdx.x & 63;
  const RowDesc mine = rows[lane & 15];
  const bool aligned = !mine.present || ((reinterpret_cast<uintptr_t>(mine.base) & 15) == 0);
  const bool all_aligned = __all(aligned);
  uint32_t mlen = mine.present ? mine.len : 0u;
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) mlen = max(mlen, (uint32_t)__shfl_xor((int)mlen, o, 64));
  mlen = uniform(mlen);

  const int hr = lane >> 2, a = lane & 3;
  const RowDesc hrow = rows[hr];
  const uint32_t nstripes = hrow.present ? hrow.len >> 5 : 0u;
  uint64_t acc = xx_acc_init(0, a);

  if (all_aligned) {
    // lane L loads for rows L/8 and L/8 + 8 (absent rows count as length 0)
    RowDesc ra = rows[lane >> 3], rb = rows[(lane >> 3) + 8];
    if (!ra.present) ra.len = 0;
    if (!rb.present) rb.len = 0;
    const uint8_t* rd = slab + hr * kStride + a * 8;
    const uint32_t nslab = (mlen + kSlab - 1) / kSlab;
    u32x4 R0[kSlab / 64], R1[kSlab / 64];
#pragma unroll
    for (int k = 0; k < kSlab / 64; ++k) R0[k] = R1[k] = u32x4{0u, 0u, 0u, 0u};
    rows_load<kSlab>(R0, ra, rb, 0);
    // keeps the first step's loads ahead of the second's, so the first stage
    // can wait for its own loads only
    if constexpr (kSlab == kSlabOne) __builtin_amdgcn_sched_barrier(0);
    rows_load<kSlab>(R1, ra, rb, kSlab);
#pragma unroll 1
    for (uint32_t s = 0; s < nslab; s += 2) {
      fast_stage(R0, slab);
      if (s + 2 < nslab) rows_load<kSlab>(R0, ra, rb, (s + 2) * kSlab);
      wave_fence();
      uint32_t q0 = s * (kSlab / 32);
      bool whole = false;
      if constexpr (kSlab == kSlabOne) whole = __all(!hrow.present || nstripes >= q0 + 2 * (kSlab / 32));
      acc = rows_fold<kSlab>(acc, rd, q0, nstripes, whole);
      wave_fence();
      if (s + 1 < nslab) {
        fast_stage(R1, slab);
        if (s + 3 < nslab) rows_load<kSlab>(R1, ra, rb, (s + 3) * kSlab);
        wave_fence();
        q0 += kSlab / 32;
        acc = rows_fold<kSlab>(acc, rd, q0, nstripes, whole);
        wave_fence();
      }
    }
  } else {
#pragma unroll 1
    for (uint32_t s0 = 0; s0 < nstripes; s0 += 8) {
      uint64_t wv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) wv[j] = s0 + j < nstripes ? load64_any(hrow.base + (s0 + j) * 32 + a * 8) : 0ull;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (s0 + j < nstripes) acc = xx_round(acc, wv[j]);
    }
  }
  return finish_row(acc, hrow);
}

// Cross-workgroup hand-off of tree digests. Each XCD has its own L2, so a
// digest stored by one workgroup must reach the device-coherent level before
// the ticket that announces it, and the last arriver must read past its own
// L2. Agent-scope relaxed atomic stores and loads do exactly that per access;
// waiting for the stores to complete orders them before the ticket. This
// avoids agent-scope fences, which write back and invalidate a whole L2.
__device__ __forceinline__ void store_coherent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t load_coherent(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// XXH64 of `nw` (<= 64) child digests written by other workgroups, by one
// whole wavefront: lane i fetches child i (all fetches in flight at once),
// then lanes 4g+a fold accumulator a's words, taken by cross-lane shuffles.
// Every lane returns the digest.
__device__ __forceinline__ uint64_t xx_words64_coherent(const uint64_t* w, uint32_t nw, uint64_t seed) {
  const int lane = threadIdx.x & 63, a = lane & 3;
  const uint64_t v = (uint32_t)lane < nw ? load_coherent(w + lane) : 0ull;
  const uint32_t nstripes = nw / 4;
  uint64_t acc = xx_acc_init(seed, a);
  for (uint32_t s = 0; s < nstripes; ++s) acc = xx_round(acc, __shfl(v, (int)(s * 4) + a, 64));
  uint64_t v1, v2, v3, v4;
  xx_gather4(acc, v1, v2, v3, v4);
  uint64_t h = nstripes ? xx_converge(v1, v2, v3, v4) : seed + kP5;
  h += uint64_t(nw) * 8;
  for (uint32_t i = nstripes * 4; i < nw; ++i) h = xx_step8(h, __shfl(v, (int)i, 64));
  return xx_avalanche(h);
}

// Called by one whole wavefront after it computed the digest `h` (lane 0) of
// node m of tree level `level`, which holds nj nodes. Stores it, and while
// this wavefront completes the last missing child of the parent, climbs:
// hashes the parent (seed = its level) and repeats; the root goes to *out.
//   tree: the buffer's node slots, level by level (level 1 first); loff is
//         where this level's slots start
//   tk:   the buffer's tickets, one per node of level 2 and above, level by
//         level; tkoff is where the tickets of this level's parents start.
//         Each is reset to 0 by its last user.
__device__ __forceinline__ void tree_up(uint64_t h, uint64_t m, uint64_t nj, uint64_t level, uint64_t loff,
                                        uint64_t tkoff, uint64_t* out, uint64_t* tree, uint32_t* tk) {
  const int lane = threadIdx.x & 63;
  h = __shfl(h, 0, 64);
  for (;;) {
    if (nj == 1) {
      if (lane == 0) *out = h;
      return;
    }
    if (lane == 0) store_coherent(tree + loff + m, h);
    wait_stores_done();
    const uint64_t p = m / kFanIn;
    const uint32_t nchild = (uint32_t)min<uint64_t>(kFanIn, nj - p * kFanIn);
    const uint64_t nnext = ceil_div(nj, kFanIn);
    uint32_t old = 0;
    if (lane == 0) old = __hip_atomic_fetch_add(tk + tkoff + p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    old = __shfl(old, 0, 64);
    if (old != nchild - 1) return;
    if (lane == 0) __hip_atomic_store(tk + tkoff + p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    h = xx_words64_coherent(tree + loff + p * kFanIn, nchild, level + 1);
    h = __shfl(h, 0, 64);
    ++level;
    m = p;
    loff += nj;
    tkoff += nnext;
    nj = nnext;
  }
}

// Buffers of up to kOneTicketNodes level-1 nodes (1 GiB) share one ticket:
// the workgroup that completes the last level-1 node reads all of their
// digests into LDS (every load in flight at once) and hashes the levels above
// there, level 2 with four lanes per node and the root (level 3) with four
// lanes, instead of a store, a wait, a ticket and a coherent load per level.
constexpr uint32_t kOneTicketNodes = kFanIn * kFanIn;
constexpr int kGatherPer = kOneTicketNodes / kThreads;

__device__ __forceinline__ void finish_upper(Smem<kSlabOne>& sm, uint32_t n1, uint64_t* tree, uint32_t* tk, uint64_t* out) {
  static_assert(sizeof(sm.slab) >= kOneTicketNodes * sizeof(uint64_t), "level-1 digests fit the staging slabs");
  uint64_t* lv1 = reinterpret_cast<uint64_t*>(&sm.slab[0][0]);
  const int t = threadIdx.x;
  if (t == 0) __hip_atomic_store(tk, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint64_t v[kGatherPer];
#pragma unroll
  for (int k = 0; k < kGatherPer; ++k) {
    const uint32_t i = (uint32_t)t + (uint32_t)k * kThreads;
    v[k] = i < n1 ? load_coherent(tree + i) : 0ull;
  }
#pragma unroll
  for (int k = 0; k < kGatherPer; ++k) {
    const uint32_t i = (uint32_t)t + (uint32_t)k * kThreads;
    if (i < n1) lv1[i] = v[k];
  }
  __syncthreads();
  const uint32_t n2 = (n1 + kFanIn - 1) / kFanIn;
  const uint32_t g = (uint32_t)t >> 2;
  if (g < n2) {
    const uint64_t h2 = n1 % kFanIn == 0 ? xx_words4_full64(lv1 + g * kFanIn, 2)
                                         : xx_words4(lv1 + g * kFanIn, min<uint32_t>(kFanIn, n1 - g * kFanIn), 2);
    if ((t & 3) == 0) sm.leafdig[1][g] = h2;
  }
  __syncthreads();
  if (t < 64) {
    const uint64_t root = n2 == 1 ? sm.leafdig[1][0] : xx_words4(sm.leafdig[1], n2, 3);
    if (t == 0) *out = root;
  }
}

// XXH64 (seed 0) of a buffer of at most one leaf at a 16-byte aligned address,
// by one whole wavefront. Every lane issues its four 16-byte loads at once
// (lane L, load k: bytes 1024k + 16L), so the leaf arrives in one memory round
// trip instead of eight staged steps; a load starting below `len` may end past
// it, inside the same aligned 16-byte granule. The leaf lands contiguously in
// the LDS slab, lanes 4g+a fold accumulator a's words sixteen stripes per LDS
// wait, and the remainder bytes are read from the slab too. Returns the
// digest in lane 0 (and every lane 4g).
__device__ __forceinline__ uint64_t hash_one_leaf(const uint8_t* p, uint32_t len, uint8_t* slab) {
  const int lane = threadIdx.x & 63, a = lane & 3;
  u32x4 R[kLeaf / 1024];
#pragma unroll
  for (int k = 0; k < kLeaf / 1024; ++k) {
    const uint32_t o = (uint32_t)k * 1024 + (uint32_t)lane * 16;
    if (o < len) R[k] = ld_global_nt(p + o);
  }
#pragma unroll
  for (int k = 0; k < kLeaf / 1024; ++k) {
    const uint32_t o = (uint32_t)k * 1024 + (uint32_t)lane * 16;
    if (o < len) *reinterpret_cast<u32x4*>(slab + o) = R[k];
  }
  wave_fence();
  const uint32_t nstripes = len >> 5;
  uint64_t acc = xx_acc_init(0, a);
  const uint8_t* rd = slab + a * 8;
  // whole chunks of 16 stripes (one LDS wait each), then the remaining
  // stripes with selects
  constexpr uint32_t kChunk = 16;
  uint32_t s = 0;
#pragma unroll 1
  for (; s + kChunk <= nstripes; s += kChunk) {
    uint64_t w[kChunk];
#pragma unroll
    for (uint32_t q = 0; q < kChunk; ++q) w[q] = *reinterpret_cast<const uint64_t*>(rd + (s + q) * 32);
#pragma unroll
    for (uint32_t q = 0; q < kChunk; ++q) acc = xx_round(acc, w[q]);
  }
  if (s < nstripes) {
    uint64_t w[kChunk];
#pragma unroll
    for (uint32_t q = 0; q < kChunk; ++q) w[q] = *reinterpret_cast<const uint64_t*>(rd + (s + q) * 32);
#pragma unroll
    for (uint32_t q = 0; q < kChunk; ++q) {
      const uint64_t folded = xx_round(acc, w[q]);
      acc = s + q < nstripes ? folded : acc;
    }
  }
  RowDesc staged;
  staged.base = slab;
  staged.len = len;
  staged.present = 1;
  return finish_row(acc, staged);
}

// One level-1 node of a buffer larger than one leaf. `buf`, `size`, `node`
// and the tree pointers are wave-uniform.
__device__ __forceinline__ void run_node(Smem<kSlabOne>& sm, const uint8_t* buf, uint64_t size, uint64_t node, uint64_t* out,
                         uint64_t* tree, uint32_t* tk) {
  const int t = threadIdx.x;
  const int w = t >> 6, r = (t & 63) >> 2;
  const uint64_t nleaves = ceil_div(size, kLeaf);
  const uint64_t n1 = ceil_div(nleaves, kFanIn);
  const uint64_t first = node * kFanIn;
  const uint32_t nl = (uint32_t)min<uint64_t>(kFanIn, nleaves - first);
  // leaves [first + 16w, first + 16w + 16) belong to this wavefront
  const uint64_t wfirst = first + (uint64_t)w * kRowsPerWave;
  const bool wave_full = ((reinterpret_cast<uintptr_t>(buf) & 15) == 0) &&
                         (wfirst + kRowsPerWave) * kLeaf <= size;
  // The buffer's last leaf, when shorter than a leaf (and the buffer 16-byte
  // aligned), is hashed on its own by hash_one_leaf, so that every row the
  // wavefronts fold is a whole leaf and folds without per-round predicates:
  // wavefront 3 takes it when it holds no leaves of this node, else the
  // wavefront that owns it, after its rows.
  const bool has_short = ((reinterpret_cast<uintptr_t>(buf) & 15) == 0) && (size % kLeaf) != 0 && node == n1 - 1;
  const uint32_t short_row = (uint32_t)(nleaves - 1 - first);  // its index in the node
  const int short_wave = !has_short ? -1 : nl <= 3 * kRowsPerWave ? 3 : (int)(short_row / kRowsPerWave);
  uint64_t h;
  if (wave_full) {
    constexpr int NL = kSlabOne / 64;
    u32x4 RA[NL], RB[NL];
    bool pre = false;
    h = hash_wave_leaves_pipe<NL>(uniform_ptr(buf + wfirst * kLeaf), nullptr, pre, RA, RB, sm.slab[w]);
  } else {
    RowDesc* rows = sm.rows + w * kRowsPerWave;
    if ((t & 63) < kRowsPerWave) {
      const uint32_t rr = t & 63;
      RowDesc d;
      const uint64_t leaf = wfirst + rr;
      const uint64_t off = leaf * kLeaf;
      d.present = leaf < first + nl && !(has_short && leaf == nleaves - 1);
      d.base = buf + (d.present ? off : 0);
      d.len = d.present ? (uint32_t)min<uint64_t>(kLeaf, size - off) : 0u;
      rows[rr] = d;
    }
    wave_fence();
    h = hash_wave_rows<kSlabOne>(rows, sm.slab[w]);
    if (w == short_wave) {
      const uint64_t off = (nleaves - 1) * kLeaf;
      const uint64_t hs = hash_one_leaf(buf + off, (uint32_t)(size - off), sm.slab[w]);
      if ((t & 63) == 0) sm.leafdig[0][short_row] = hs;
    }
  }
  const uint32_t my_row = (uint32_t)(w * kRowsPerWave + r);
  if ((t & 3) == 0 && my_row < nl && !(has_short && my_row == short_row)) sm.leafdig[0][my_row] = h;
  __syncthreads();
  if (n1 > kOneTicketNodes) {
    if (w == 0) {
      const uint64_t d = xx_words4(sm.leafdig[0], nl, 1);
      tree_up(d, node, n1, 1, 0, 0, out, tree, tk);
    }
    __syncthreads();
    return;
  }
  if (w == 0) {
    const int lane = t & 63;
    const uint64_t d =
        __shfl(nl == kFanIn ? xx_words4_full64(sm.leafdig[0], 1) : xx_words4(sm.leafdig[0], nl, 1), 0, 64);
    uint32_t last = 0;
    if (n1 == 1) {
      if (lane == 0) *out = d;
    } else {
      if (lane == 0) store_coherent(tree + node, d);
      wait_stores_done();
      if (lane == 0) last = __hip_atomic_fetch_add(tk, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == n1 - 1;
    }
    if (lane == 0) sm.outidx[0] = last;
  }
  __syncthreads();
  if (sm.outidx[0]) finish_upper(sm, (uint32_t)n1, tree, tk, out);
}

// ---------------------------------------------------------------------------
// Plain form: one launch per buffer, one workgroup per level-1 node.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void digest_one_kernel(const uint8_t* p, uint64_t size, uint64_t* out,
                                                             uint64_t* tree, uint32_t* tk) {
  __shared__ Smem<kSlabOne> sm;
  if (size <= kLeaf) {
    const int t = threadIdx.x;
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
      if (t < 64) {
        const uint64_t h = hash_one_leaf(p, (uint32_t)size, sm.slab[0]);
        if (t == 0) *out = h;
      }
      return;
    }
    if (t < kRows) {
      RowDesc d;
      d.present = t == 0;
      d.base = p;
      d.len = t == 0 ? (uint32_t)size : 0u;
      sm.rows[t] = d;
    }
    __syncthreads();
    if (t < 64) {
      const uint64_t h = hash_wave_rows<kSlabOne>(sm.rows, sm.slab[0]);
      if (t == 0) *out = h;
    }
    return;
  }
  run_node(sm, p, size, blockIdx.x, out, tree, tk);
}

// ---------------------------------------------------------------------------
// Batched form: device-side work plan, then one persistent launch.
// ---------------------------------------------------------------------------
struct PlanArgs {
  const void* const* ptrs;
  const uint64_t* sizes;
  uint64_t* out;
  uint64_t* tree;
  NodeRec* rec;         // [node items]
  uint64_t n;
  uint64_t* node_off;   // [n] first node item of buffer i
  uint64_t* tree_off;   // [n]
  uint64_t* tk_off;     // [n]
  uint32_t* small_list; // [n]
  NodeRec* med_rec;     // [n] level-1 nodes of at most `split` bytes (one per buffer at most: its last)
  uint32_t split;       // bytes; 0: none
  uint64_t* blk;        // [kQ * nblk] per-tile sums, then exclusive prefixes
  uint64_t nblk;
  DigestCtl* ctl;
  uint64_t cap_items, cap_tree, cap_tk;
  uint64_t cap_nodes;   // level-1 nodes of buffers above one leaf, at most (the fixed array's limit)
};

constexpr int kPlanThreads = 256;
constexpr int kPlanPer = 8;  // buffers per thread
constexpr int kPlanTile = kPlanThreads * kPlanPer;

// Per-buffer plan quantities: [0] level-1 nodes hashed by a whole workgroup
// (node items), [1] 1 for a buffer of at most one leaf, [2] tree slots,
// [3] tickets, [4] 1 when the buffer's last level-1 node has at most `split`
// bytes and is hashed by one wavefront instead.
constexpr int kQ = 5;

__device__ __forceinline__ void buffer_counts(uint64_t size, uint32_t split, uint64_t c[kQ]) {
#pragma unroll
  for (int q = 0; q < kQ; ++q) c[q] = 0;
  if (size <= kLeaf) {
    c[1] = 1;
    return;
  }
  const uint64_t n1 = ceil_div(ceil_div(size, kLeaf), kFanIn);
  const bool med = size - (n1 - 1) * kNodeBytes <= split;
  c[0] = n1 - (med ? 1 : 0);
  c[4] = med ? 1 : 0;
  tree_need(n1, c[2], c[3]);
}

// Exclusive scan of kQ u64 quantities over the threads of a block; returns
// the block totals in tot[].
__device__ void block_scan4(uint64_t v[kQ], uint64_t tot[kQ]) {
  __shared__ uint64_t sh[kPlanThreads / 64][kQ];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    uint64_t x = v[q];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      uint64_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) sh[w][q] = x;
    v[q] = x - v[q];  // exclusive within the wavefront
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    uint64_t before = 0, all = 0;
    for (int j = 0; j < kPlanThreads / 64; ++j) {
      if (j < w) before += sh[j][q];
      all += sh[j][q];
    }
    v[q] += before;
    tot[q] = all;
  }
  __syncthreads();
}

// Totals of the plan (node items, small buffers, tree and ticket slots) into
// the control block; flags a plan that does not fit the workspace.
__device__ void finalize_plan(const PlanArgs& A, const uint64_t carry[kQ]) {
  DigestCtl* c = A.ctl;
  c->n_node_items = carry[0];
  c->n_small = carry[1];
  c->n_med = carry[4];
  c->n_items = carry[0] + ceil_div(carry[4], kWaves) + ceil_div(carry[1], kRows);
  c->tree_total = carry[2];
  c->tk_total = carry[3];
  c->head = 0;
  // item numbers run past n_items by up to (3 * workgroups + 2) * chunk, at
  // most 2^20 for 2^14 workgroups and chunks of 16
  c->overflow = (carry[0] > A.cap_items || carry[2] > A.cap_tree || carry[3] > A.cap_tk ||
                 carry[0] + carry[4] > A.cap_nodes || c->n_items >= 0xFFFF0000ull - (1ull << 20)) ? 1u : 0u;
}

__global__ __launch_bounds__(kPlanThreads) void plan_count_kernel(PlanArgs A) {
  const uint64_t base = (uint64_t)blockIdx.x * kPlanTile + threadIdx.x * kPlanPer;
  uint64_t s[kQ] = {0, 0, 0, 0, 0};
  for (int j = 0; j < kPlanPer; ++j) {
    const uint64_t i = base + j;
    if (i < A.n) {
      uint64_t c[kQ];
      buffer_counts(A.sizes[i], A.split, c);
#pragma unroll
      for (int q = 0; q < kQ; ++q) s[q] += c[q];
    }
  }
  uint64_t tot[kQ];
  block_scan4(s, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) A.blk[kQ * blockIdx.x + q] = tot[q];
  }
}

__global__ __launch_bounds__(kPlanThreads) void plan_scan_kernel(PlanArgs A) {
  __shared__ uint64_t carry[kQ];
  if (threadIdx.x < kQ) carry[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t b0 = 0; b0 < A.nblk; b0 += kPlanThreads) {
    const uint64_t b = b0 + threadIdx.x;
    uint64_t v[kQ] = {0, 0, 0, 0, 0};
    if (b < A.nblk) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) v[q] = A.blk[kQ * b + q];
    }
    uint64_t tot[kQ];
    block_scan4(v, tot);
    if (b < A.nblk) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) A.blk[kQ * b + q] = v[q] + carry[q];
    }
    __syncthreads();
    if (threadIdx.x < kQ) carry[threadIdx.x] += tot[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) finalize_plan(A, carry);
}

__global__ __launch_bounds__(kPlanThreads) void plan_write_kernel(PlanArgs A) {
  const uint64_t base = (uint64_t)blockIdx.x * kPlanTile + threadIdx.x * kPlanPer;
  uint64_t c[kPlanPer][kQ];
  uint64_t s[kQ] = {0, 0, 0, 0, 0};
  for (int j = 0; j < kPlanPer; ++j) {
    const uint64_t i = base + j;
    if (i < A.n) {
      buffer_counts(A.sizes[i], A.split, c[j]);
    } else {
#pragma unroll
      for (int q = 0; q < kQ; ++q) c[j][q] = 0;
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) s[q] += c[j][q];
  }
  uint64_t tot[kQ];
  block_scan4(s, tot);
  if (A.nblk == 1) {
    // one tile: its own scan is the whole plan (no count and scan launches)
    if (threadIdx.x == 0) finalize_plan(A, tot);
  } else {
#pragma unroll
    for (int q = 0; q < kQ; ++q) s[q] += A.blk[kQ * blockIdx.x + q];
  }
  for (int j = 0; j < kPlanPer; ++j) {
    const uint64_t i = base + j;
    if (i < A.n) {
      A.node_off[i] = s[0];
      A.tree_off[i] = s[2];
      A.tk_off[i] = s[3];
      if (c[j][1]) A.small_list[s[1]] = (uint32_t)i;
      if (c[j][4]) {
        const uint64_t size = A.sizes[i], n1 = c[j][0] + 1;
        NodeRec r;
        r.base = static_cast<const uint8_t*>(A.ptrs[i]) + (n1 - 1) * kNodeBytes;
        r.dst = n1 == 1 ? A.out + i : A.tree + s[2] + (n1 - 1);
        r.len = (uint32_t)(size - (n1 - 1) * kNodeBytes);
        r.buf = (uint32_t)i;
        A.med_rec[s[4]] = r;
      }
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) s[q] += c[j][q];
  }
}

// item_buf[k] = buffer owning node item k (largest i with node_off[i] <= k),
// rec[k] = the node's address, length and digest destination.
__global__ __launch_bounds__(kPlanThreads) void plan_items_kernel(PlanArgs A, uint32_t* item_buf) {
  const DigestCtl* c = A.ctl;
  if (c->overflow) return;
  const uint64_t total = c->n_node_items;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t lo = 0, hi = A.n;  // invariant: node_off[lo] <= k < node_off[hi] (node_off[n] = total)
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) / 2;
      if (A.node_off[mid] <= k) lo = mid; else hi = mid;
    }
    item_buf[k] = (uint32_t)lo;
    const uint64_t size = A.sizes[lo], node = k - A.node_off[lo];
    const uint64_t n1 = ceil_div(ceil_div(size, kLeaf), kFanIn);
    NodeRec r;
    r.base = static_cast<const uint8_t*>(A.ptrs[lo]) + node * kNodeBytes;
    r.dst = n1 == 1 ? A.out + lo : A.tree + A.tree_off[lo] + node;
    r.len = (uint32_t)min<uint64_t>(kNodeBytes, size - node * kNodeBytes);
    r.buf = (uint32_t)lo;
    A.rec[k] = r;
  }
}

struct BatchArgs {
  const void* const* ptrs;
  const uint64_t* sizes;
  uint64_t n;
  uint64_t* out;
  const uint64_t* node_off;
  const uint64_t* tree_off;
  const uint64_t* tk_off;
  const uint32_t* small_list;
  const uint32_t* item_buf;
  const NodeRec* rec;
  const NodeRec* med_rec;
  uint64_t* tree;
  uint32_t* tickets;
  DigestCtl* ctl;
  uint32_t* status;  // host-mapped sticky status word
  uint32_t chunk;    // items per claim
};

__device__ __forceinline__ bool aligned16(const uint8_t* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// The work record of queue item `item` (node items only; zeros otherwise).
__device__ __forceinline__ NodeRec load_rec(const BatchArgs& A, uint32_t item, uint64_t n_node) {
  NodeRec r;
  r.base = nullptr;
  r.dst = nullptr;
  r.len = 0;
  r.buf = 0;
  if (item < n_node) r = A.rec[item];
  return r;
}

// First leaf of wavefront w's rows in a node when they are 16 whole, 16-byte
// aligned leaves (the fast path), else null.
__device__ __forceinline__ const uint8_t* fast_rows(const uint8_t* base, uint32_t len, int w) {
  const uint32_t end = (uint32_t)(w + 1) * kRowsPerWave * kLeaf;
  return aligned16(base) && end <= len ? base + (uint32_t)w * kRowsPerWave * kLeaf : nullptr;
}

// Persistent batched digest. Workgroups take the items in chunks of
// A.chunk consecutive ones: workgroup b starts with chunks b and b + grid,
// then claims chunks from the queue (numbered from 2 * grid on). The item two
// ahead of the one being hashed is settled during it (a claim when it opens a
// chunk), so the claim and the item's record arrive while the current item
// streams; each wavefront carries its load pipeline from one node item into
// the next. Per item there is one barrier: after it, one
// wavefront (rotating) folds the 64 leaf digests into the level-1 digest and
// stores it without waiting (out[i] for one-node buffers, else the tree slot
// that the tree kernel climbs from).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void digest_batched_kernel(BatchArgs A) {
  __shared__ Smem<kSlabBatch> sm;
  const DigestCtl* c = A.ctl;
  if (c->overflow) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += (uint64_t)gridDim.x * blockDim.x)
      A.out[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && A.status) *reinterpret_cast<volatile uint32_t*>(A.status) = (uint32_t)(-ODP_ECAPACITY);
    return;
  }
  const uint64_t n_node = c->n_node_items, n_items = c->n_items, n_small = c->n_small, n_med = c->n_med;
  const uint64_t med_end = n_node + ceil_div(n_med, kWaves);
  const int t = threadIdx.x, w = uniform(t >> 6), lane = t & 63, r = lane >> 2;
  // items blockIdx.x and blockIdx.x + gridDim.x are this workgroup's; later
  // ones come from the queue, numbered from 2 * gridDim.x on. A workgroup
  // with nothing to do leaves without touching the queue.
  const uint32_t C = A.chunk, first_queued = 2u * gridDim.x;
  // item i of this workgroup's sequence, for the two preassigned chunks (i < 2C)
  auto pre_item = [&](uint32_t i) { return i < C ? blockIdx.x * C + i : (blockIdx.x + gridDim.x) * C + (i - C); };
  uint32_t cur = pre_item(0), nxt = pre_item(1);
  NodeRec rc = load_rec(A, cur, n_node), rn = load_rec(A, nxt, n_node);
  constexpr int NL = kSlabBatch / 64;
  u32x4 RA[NL], RB[NL];
  bool pre = false;
  RowDesc* rows = sm.rows + w * kRowsPerWave;
  for (uint32_t k = 0; cur < n_items; ++k) {
    // the item two ahead: the next of nxt's chunk, or the first of a new one
    uint32_t claim = 0;
    if (t == 0) {
      if (k + 2 < 2 * C) claim = pre_item(k + 2);
      else if ((k + 2) % C == 0) claim = (first_queued + atomicAdd(&A.ctl->head, 1u)) * C;
      else claim = nxt + 1;
    }
    const bool is_node = cur < n_node;
    const bool is_med = !is_node && cur < med_end;
    const uint8_t* base = uniform_ptr(rc.base);
    const uint32_t len = uniform(rc.len);
    const uint32_t nl = (len + kLeaf - 1) / kLeaf;
    const uint8_t* mine = is_node ? fast_rows(base, len, w) : nullptr;
    uint64_t h;
    if (mine) {
      const uint8_t* next = nxt < n_node ? fast_rows(uniform_ptr(rn.base), uniform(rn.len), w) : nullptr;
      h = hash_wave_leaves_pipe<NL>(mine, next, pre, RA, RB, sm.slab[w]);
    } else {
      // Nothing is in flight for this path (pre is false after it): constant
      // stage registers are rematerialised instead of kept across it.
#pragma unroll
      for (int j = 0; j < NL; ++j) RA[j] = RB[j] = u32x4{0u, 0u, 0u, 0u};
      // This wavefront's medium node (a whole level-1 node of at most 16 leaves).
      const uint64_t qm = (uint64_t)(cur - n_node) * kWaves + w;
      const bool has_med = is_med && qm < n_med;
      const uint8_t* mbase = nullptr;
      uint64_t* mdst = nullptr;
      uint32_t mlen = 0;
      if (has_med) {
        mbase = uniform_ptr(A.med_rec[qm].base);
        mdst = reinterpret_cast<uint64_t*>(uniform(reinterpret_cast<uint64_t>(A.med_rec[qm].dst)));
        mlen = uniform(A.med_rec[qm].len);
      }
      const uint32_t mnl = (mlen + kLeaf - 1) / kLeaf;
      // rows of a partial or unaligned node, of a medium node, or of up to 64
      // buffers of at most one leaf each (digest = XXH64 seed 0), 16 per wavefront
      if (lane < kRowsPerWave) {
        RowDesc d;
        if (is_node) {
          const uint32_t leaf = w * kRowsPerWave + lane;
          d.present = leaf < nl;
          d.base = base + (d.present ? leaf * kLeaf : 0u);
          d.len = d.present ? min<uint32_t>(kLeaf, len - leaf * kLeaf) : 0u;
        } else if (is_med) {
          const uint32_t leaf = lane;
          d.present = leaf < mnl;
          d.base = d.present ? mbase + leaf * kLeaf : nullptr;
          d.len = d.present ? min<uint32_t>(kLeaf, mlen - leaf * kLeaf) : 0u;
        } else {
          const uint64_t q = (uint64_t)(cur - med_end) * kRows + w * kRowsPerWave + lane;
          d.present = q < n_small;
          const uint32_t idx = d.present ? A.small_list[q] : 0u;
          d.base = d.present ? static_cast<const uint8_t*>(A.ptrs[idx]) : nullptr;
          d.len = d.present ? (uint32_t)A.sizes[idx] : 0u;
          sm.outidx[w * kRowsPerWave + lane] = idx;
        }
        rows[lane] = d;
      }
      wave_fence();
      h = hash_wave_rows<kSlabBatch>(rows, sm.slab[w]);
      pre = false;
      if (is_med) {
        // level-1 combine inside the wavefront, in its own slice of the leaf-digest buffer
        uint64_t* ld = sm.leafdig[k & 1] + w * kRowsPerWave;
        if ((lane & 3) == 0 && (uint32_t)r < mnl) ld[r] = h;
        wave_fence();
        if (has_med) {
          const uint64_t d = xx_words4(ld, mnl, 1);
          if (lane == 0) *mdst = d;
        }
      }
    }
    if ((lane & 3) == 0) {
      if (is_node) {
        if ((uint32_t)(w * kRowsPerWave + r) < nl) sm.leafdig[k & 1][w * kRowsPerWave + r] = h;
      } else if (!is_med && rows[r].present) {
        A.out[sm.outidx[w * kRowsPerWave + r]] = h;
      }
    }
    if (t == 0) sm.ring[(k + 2) % 3] = claim;
    __syncthreads();
    if (cur < n_node && w == (int)(k & 3)) {
      const uint64_t d = xx_words4(sm.leafdig[k & 1], nl, 1);
      if (lane == 0) *reinterpret_cast<uint64_t*>(uniform(reinterpret_cast<uint64_t>(rc.dst))) = d;
    }
    cur = nxt;
    rc = rn;
    nxt = uniform(sm.ring[(k + 2) % 3]);
    rn = load_rec(A, nxt, n_node);
  }
}

// Levels 2 and up of every buffer with more than one level-1 node: one
// wavefront per level-2 node hashes its (up to 64) level-1 digests, then
// climbs with tickets like the per-buffer form.
__global__ __launch_bounds__(kThreads) void digest_tree_kernel(BatchArgs A) {
  const DigestCtl* c = A.ctl;
  if (c->overflow) return;
  const uint64_t n_node = c->n_node_items;
  const int lane = threadIdx.x & 63;
  const uint64_t wave = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const uint64_t nwaves = (uint64_t)gridDim.x * kWaves;
  for (uint64_t base = wave * 64; base < n_node; base += nwaves * 64) {
    const uint64_t k = base + lane;
    bool first = false;
    if (k < n_node) {
      const uint32_t b = A.item_buf[k];
      const uint64_t node = k - A.node_off[b];
      const uint64_t n1 = ceil_div(ceil_div(A.sizes[b], kLeaf), kFanIn);
      first = n1 > 1 && node % kFanIn == 0;
    }
    uint64_t mask = __ballot(first);
    while (mask) {
      const uint64_t kk = base + (uint64_t)__builtin_ctzll(mask);
      mask &= mask - 1;
      const uint32_t b = uniform(A.item_buf[kk]);
      const uint64_t n1 = ceil_div(ceil_div(uniform(A.sizes[b]), kLeaf), kFanIn);
      const uint64_t n2 = ceil_div(n1, kFanIn);
      const uint64_t p = (kk - uniform(A.node_off[b])) / kFanIn;
      uint64_t* tree = A.tree + uniform(A.tree_off[b]);
      const uint32_t nchild = (uint32_t)min<uint64_t>(kFanIn, n1 - p * kFanIn);
      const uint64_t h = xx_words4(tree + p * kFanIn, nchild, 2);
      tree_up(h, p, n2, 2, n1, n2, A.out + b, tree, A.tickets + uniform(A.tk_off[b]));
    }
  }
  // a level-2 node whose only child is a buffer's last node, hashed as a medium node
  const uint64_t n_med = c->n_med;
  for (uint64_t base = wave * 64; base < n_med; base += nwaves * 64) {
    const uint64_t j = base + lane;
    bool alone = false;
    if (j < n_med) {
      const uint32_t b = A.med_rec[j].buf;
      const uint64_t n1 = ceil_div(ceil_div(A.sizes[b], kLeaf), kFanIn);
      alone = n1 > 1 && (n1 - 1) % kFanIn == 0;
    }
    uint64_t mask = __ballot(alone);
    while (mask) {
      const uint64_t jj = base + (uint64_t)__builtin_ctzll(mask);
      mask &= mask - 1;
      const uint32_t b = uniform(A.med_rec[jj].buf);
      const uint64_t n1 = ceil_div(ceil_div(uniform(A.sizes[b]), kLeaf), kFanIn);
      const uint64_t n2 = ceil_div(n1, kFanIn);
      const uint64_t p = (n1 - 1) / kFanIn;
      uint64_t* tree = A.tree + uniform(A.tree_off[b]);
      const uint64_t h = xx_words4(tree + p * kFanIn, 1, 2);
      tree_up(h, p, n2, 2, n1, n2, A.out + b, tree, A.tickets + uniform(A.tk_off[b]));
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
uint64_t digest_workspace_bytes(size_t max_buffers, uint64_t max_total_bytes) {
  const uint64_t nb = max_buffers < 1024 ? 1024 : max_buffers;
  const uint64_t nblk = (nb + kPlanTile - 1) / kPlanTile;
  const uint64_t items = max_total_bytes / kNodeBytes + nb;
  const uint64_t tree = items + items / 32 + 4 * nb, tk = items / 32 + 4 * nb;
  return (nb + 1) * 8 + 2 * nb * 8 + nb * 4 + nblk * kQ * 8 + nb * sizeof(NodeRec) + sizeof(DigestCtl) +
         items * (4 + sizeof(NodeRec)) + tree * 8 + tk * 4;
}

int digest_reserve(Workspace* ws, size_t max_buffers, uint64_t max_total_bytes) {
  // A captured graph holds workspace addresses: drop it before anything moves.
  if (ws->graph) {
    ODP_HIP(hipDeviceSynchronize());
    ODP_HIP(hipGraphExecDestroy(ws->graph));
    ws->graph = nullptr;
  }
  size_t nb = max_buffers < 1024 ? 1024 : max_buffers;
  if (nb > ws->cap_buffers) {
    const size_t nblk = (nb + kPlanTile - 1) / kPlanTile;
    int e;
    if ((e = ws->node_off.ensure((nb + 1) * 8)) || (e = ws->tree_off.ensure(nb * 8)) ||
        (e = ws->tk_off.ensure(nb * 8)) || (e = ws->small_list.ensure(nb * 4)) ||
        (e = ws->blk.ensure(nblk * kQ * 8)) || (e = ws->med_rec.ensure(nb * sizeof(NodeRec))))
      return e;
    ws->cap_buffers = nb;
  }
  if (!ws->ctl.ptr) {
    int e = ws->ctl.ensure(sizeof(DigestCtl));
    if (e) return e;
    ODP_HIP(hipMemset(ws->ctl.ptr, 0, sizeof(DigestCtl)));
  }
  uint64_t items = max_total_bytes / kNodeBytes + nb;
  if (items > ws->cap_items) {
    const uint64_t tree = items + items / 32 + 4 * (uint64_t)nb;
    const uint64_t tk = items / 32 + 4 * (uint64_t)nb;
    int e;
    if ((e = ws->item_buf.ensure(items * 4)) || (e = ws->item_rec.ensure(items * sizeof(NodeRec))) ||
        (e = ws->tree.ensure(tree * 8)) || (e = ws->tickets.ensure(tk * 4)))
      return e;
    ODP_HIP(hipMemset(ws->tickets.ptr, 0, tk * 4));
    ws->cap_items = items;
    ws->cap_tree = tree;
    ws->cap_tk = tk;
  }
  return ODP_OK;
}

// Device memory one batched call works in: the grow-only workspace of a
// (device, stream) pair, or the fixed array of the no-allocation entry point.
struct BatchedSpace {
  int device;
  uint64_t* node_off;   // [cap_buffers + 1]
  uint64_t* tree_off;   // [cap_buffers]
  uint64_t* tk_off;     // [cap_buffers]
  uint32_t* small_list; // [cap_buffers]
  uint64_t* blk;        // [kQ * tiles of cap_buffers]
  NodeRec* med_rec;     // [cap_buffers]
  DigestCtl* ctl;
  uint32_t* item_buf;   // [cap_items]
  NodeRec* item_rec;    // [cap_items]
  uint64_t* tree;       // [cap_tree]
  uint32_t* tickets;    // [cap_tk], zero between calls
  uint64_t cap_items, cap_tree, cap_tk;
  uint64_t cap_nodes;   // level-1 nodes of buffers above one leaf, at most
  uint32_t* status;     // sticky status word (ODP_ECAPACITY on overflow)
};

BatchedSpace space_of(Workspace* ws) {
  BatchedSpace S;
  S.device = ws->device;
  S.node_off = static_cast<uint64_t*>(ws->node_off.ptr);
  S.tree_off = static_cast<uint64_t*>(ws->tree_off.ptr);
  S.tk_off = static_cast<uint64_t*>(ws->tk_off.ptr);
  S.small_list = static_cast<uint32_t*>(ws->small_list.ptr);
  S.blk = static_cast<uint64_t*>(ws->blk.ptr);
  S.med_rec = static_cast<NodeRec*>(ws->med_rec.ptr);
  S.ctl = static_cast<DigestCtl*>(ws->ctl.ptr);
  S.item_buf = static_cast<uint32_t*>(ws->item_buf.ptr);
  S.item_rec = static_cast<NodeRec*>(ws->item_rec.ptr);
  S.tree = static_cast<uint64_t*>(ws->tree.ptr);
  S.tickets = static_cast<uint32_t*>(ws->tickets.ptr);
  S.cap_items = ws->cap_items;
  S.cap_tree = ws->cap_tree;
  S.cap_tk = ws->cap_tk;
  S.cap_nodes = ~0ull;  // bounded by the item, tree and ticket capacities
  S.status = device_status_word(ws->device);
  return S;
}

// item_hint: an upper bound on the work items when the caller knows one
// (0: unknown), to size the grids of small batches.
static int enqueue_batched(const BatchedSpace& S, const void* const* ptrs, const uint64_t* sizes, size_t n,
                           uint64_t* out, hipStream_t stream, uint64_t item_hint = 0) {
  PlanArgs P;
  P.ptrs = ptrs;
  P.sizes = sizes;
  P.out = out;
  P.tree = S.tree;
  P.rec = S.item_rec;
  P.med_rec = S.med_rec;
  P.split = tuning().split_bytes;
  P.n = n;
  P.node_off = S.node_off;
  P.tree_off = S.tree_off;
  P.tk_off = S.tk_off;
  P.small_list = S.small_list;
  P.blk = S.blk;
  P.nblk = (n + kPlanTile - 1) / kPlanTile;
  P.ctl = S.ctl;
  P.cap_items = S.cap_items;
  P.cap_tree = S.cap_tree;
  P.cap_tk = S.cap_tk;
  P.cap_nodes = S.cap_nodes;
  if (P.nblk > 1) {
    hipLaunchKernelGGL(plan_count_kernel, dim3((unsigned)P.nblk), dim3(kPlanThreads), 0, stream, P);
    hipLaunchKernelGGL(plan_scan_kernel, dim3(1), dim3(kPlanThreads), 0, stream, P);
  }
  hipLaunchKernelGGL(plan_write_kernel, dim3((unsigned)P.nblk), dim3(kPlanThreads), 0, stream, P);
  const uint64_t cus = (uint64_t)cu_count(S.device);
  auto sized = [&](uint64_t full, uint64_t per) {
    return (unsigned)(item_hint ? std::max<uint64_t>(1, std::min<uint64_t>(full, ceil_div(item_hint, per))) : full);
  };
  hipLaunchKernelGGL(plan_items_kernel, dim3(sized(cus * 4, kPlanThreads)), dim3(kPlanThreads), 0, stream, P,
                     S.item_buf);
  BatchArgs B;
  B.ptrs = ptrs;
  B.sizes = sizes;
  B.n = n;
  B.out = out;
  B.node_off = P.node_off;
  B.tree_off = P.tree_off;
  B.tk_off = P.tk_off;
  B.small_list = P.small_list;
  B.item_buf = S.item_buf;
  B.rec = P.rec;
  B.med_rec = P.med_rec;
  B.tree = S.tree;
  B.tickets = S.tickets;
  B.ctl = P.ctl;
  B.status = S.status;
  B.chunk = std::max<uint32_t>(1, tuning().chunk_nodes);
  const uint64_t bpc = tuning().blocks_per_cu;
  hipLaunchKernelGGL(digest_batched_kernel, dim3(sized(cus * bpc, 1)), dim3(kThreads), 0, stream, B);
  hipLaunchKernelGGL(digest_tree_kernel, dim3(sized(cus * 4, 64 * kWaves)), dim3(kThreads), 0, stream, B);
  return check_hip(hipGetLastError(), "digest launch");
}

}  // namespace odp

using namespace odp;

extern "C" int odp_digest_buffers(const void* const* ptrs, const uint64_t* sizes, size_t n, uint64_t* out,
                                  odp_stream_t stream_) {
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  if (n == 0) return ODP_OK;
  if (!ptrs || !sizes || !out) return set_error(ODP_EINVAL, "odp_digest_buffers: null array with n = %zu", n);
  if (n > 0xFFFFFFFFull) return set_error(ODP_ERANGE, "odp_digest_buffers: n = %zu above 2^32 - 1", n);
  int err = 0;
  Workspace* ws = workspace_for(stream, &err);
  if (!ws) return err;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  ODP_HIP(hipStreamIsCapturing(stream, &cap));
  const bool capturing = cap != hipStreamCaptureStatusNone;
  if (n > ws->cap_buffers || !ws->cap_items) {
    if (capturing)
      return set_error(ODP_ENOMEM, "odp_digest_buffers: workspace for %zu buffers not reserved before capture", n);
    hipDeviceProp_t prop;
    ODP_HIP(hipGetDeviceProperties(&prop, ws->device));
    int e = digest_reserve(ws, n, (uint64_t)prop.totalGlobalMem * 4);
    if (e) return e;
  }
  const Tuning& tn = tuning();
  if (!tn.use_graph || capturing) return enqueue_batched(space_of(ws), ptrs, sizes, n, out, stream);
  const uint32_t grid = cu_count(ws->device) * tn.blocks_per_cu;
  if (!(ws->graph && ws->g_ptrs == ptrs && ws->g_sizes == sizes && ws->g_out == out && ws->g_n == n &&
        ws->g_grid == grid && ws->g_split == tn.split_bytes && ws->g_chunk == tn.chunk_nodes)) {
    if (ws->graph) {
      ODP_HIP(hipGraphExecDestroy(ws->graph));
      ws->graph = nullptr;
    }
    hipStream_t cs;
    ODP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int e = ODP_OK;
    if (he == hipSuccess) {
      e = enqueue_batched(space_of(ws), ptrs, sizes, n, out, cs);
      he = hipStreamEndCapture(cs, &g);
    }
    (void)hipStreamDestroy(cs);
    if (he != hipSuccess) return check_hip(he, "graph capture");
    if (e) {
      if (g) (void)hipGraphDestroy(g);
      return e;
    }
    he = hipGraphInstantiate(&ws->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (he != hipSuccess) {
      ws->graph = nullptr;
      return check_hip(he, "graph instantiate");
    }
    ws->g_ptrs = ptrs;
    ws->g_sizes = sizes;
    ws->g_out = out;
    ws->g_n = n;
    ws->g_grid = grid;
    ws->g_split = tn.split_bytes;
    ws->g_chunk = tn.chunk_nodes;
  }
  ODP_HIP(hipGraphLaunch(ws->graph, stream));
  return ODP_OK;
}

namespace odp {
// Tree and ticket slots of the per-buffer form (grow-only; tickets zeroed).
int plain_reserve_slots(Workspace* ws, uint64_t need_tree, uint64_t need_tk) {
  if (need_tree <= ws->p_cap_tree && need_tk <= ws->p_cap_tk && ws->p_tickets.ptr) return ODP_OK;
  const uint64_t tr = std::max<uint64_t>(need_tree, 1024), tk = std::max<uint64_t>(need_tk, 256);
  int e;
  if ((e = ws->p_tree.ensure(tr * 8)) || (e = ws->p_tickets.ensure(tk * 4))) return e;
  ODP_HIP(hipMemset(ws->p_tickets.ptr, 0, tk * 4));
  ws->p_cap_tree = tr;
  ws->p_cap_tk = tk;
  return ODP_OK;
}

uint64_t digest_plain_workspace_bytes(uint64_t max_bytes) {
  uint64_t tr = 0, tk = 0;
  if (max_bytes > kLeaf) tree_need(ceil_div(ceil_div(max_bytes, kLeaf), kFanIn), tr, tk);
  return std::max<uint64_t>(tr, 1024) * 8 + std::max<uint64_t>(tk, 256) * 4;
}

int digest_plain_reserve(Workspace* ws, uint64_t max_bytes) {
  uint64_t tr = 0, tk = 0;
  if (max_bytes > kLeaf) tree_need(ceil_div(ceil_div(max_bytes, kLeaf), kFanIn), tr, tk);
  return plain_reserve_slots(ws, tr, tk);
}

int digest_batched_direct(const void* const* ptrs, const uint64_t* sizes, size_t n, uint64_t* out, hipStream_t stream,
                          uint64_t total_bytes) {
  if (n == 0) return ODP_OK;
  int err = 0;
  Workspace* ws = workspace_for(stream, &err);
  if (!ws) return err;
  if (n > ws->cap_buffers || !ws->cap_items)
    return set_error(ODP_ENOMEM, "digest: workspace for %zu buffers not reserved", n);
  // node items <= total_bytes / node + n; small groups <= n / 64 + 1
  const uint64_t hint = total_bytes / kNodeBytes + n + n / kRows + 1;
  return enqueue_batched(space_of(ws), ptrs, sizes, n, out, stream, hint);
}
}  // namespace odp

// ---------------------------------------------------------------------------
// The batched digest without allocation: every workspace byte lives in one
// fixed device array, `scratch`, laid out like the grow-only workspace for at
// most ODP_NOALLOC_MAX_BUFFERS buffers and ODP_NOALLOC_MAX_NODES level-1
// nodes. Each device holds its own copy of the array, at its own address,
// from load to process end; host code reaches it only through that address.
// ---------------------------------------------------------------------------
namespace odp {
namespace {
constexpr uint64_t kNaBuffers = ODP_NOALLOC_MAX_BUFFERS;
constexpr uint64_t kNaTiles = (kNaBuffers + kPlanTile - 1) / kPlanTile;
constexpr uint64_t kNaItems = uint64_t(ODP_NOALLOC_MAX_NODES) + kNaBuffers;  // as digest_reserve
constexpr uint64_t kNaTree = kNaItems + kNaItems / 32 + 4 * kNaBuffers;
constexpr uint64_t kNaTk = kNaItems / 32 + 4 * kNaBuffers;
constexpr uint64_t al256(uint64_t x) { return (x + 255) & ~uint64_t(255); }
constexpr uint64_t kOffNodeOff = 0;
constexpr uint64_t kOffTreeOff = al256(kOffNodeOff + (kNaBuffers + 1) * 8);
constexpr uint64_t kOffTkOff = al256(kOffTreeOff + kNaBuffers * 8);
constexpr uint64_t kOffSmall = al256(kOffTkOff + kNaBuffers * 8);
constexpr uint64_t kOffBlk = al256(kOffSmall + kNaBuffers * 4);
constexpr uint64_t kOffMed = al256(kOffBlk + kNaTiles * kQ * 8);
constexpr uint64_t kOffCtl = al256(kOffMed + kNaBuffers * sizeof(NodeRec));
constexpr uint64_t kOffItemBuf = al256(kOffCtl + sizeof(DigestCtl));
constexpr uint64_t kOffItemRec = al256(kOffItemBuf + kNaItems * 4);
constexpr uint64_t kOffTree = al256(kOffItemRec + kNaItems * sizeof(NodeRec));
constexpr uint64_t kOffTk = al256(kOffTree + kNaTree * 8);
constexpr uint64_t kOffStatus = al256(kOffTk + kNaTk * 4);
constexpr uint64_t kScratchBytes = al256(kOffStatus + 4);
static_assert(kScratchBytes == ODP_NOALLOC_SCRATCH_BYTES, "header states the array's size");
}  // namespace
}  // namespace odp

static __device__ __align__(256) unsigned char scratch[odp::kScratchBytes];

namespace odp {
namespace {
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
unsigned char* g_na_ptr[kNaMaxDevices];  // device address of `scratch` on each device, once set up

// Zeroes what must start at zero: the tickets (each is also reset by its last
// user, so calls leave them zero) and the status word.
__global__ void na_clear_kernel(uint32_t* tickets, uint64_t ntk, uint32_t* status) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ntk; i += (uint64_t)gridDim.x * blockDim.x)
    tickets[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
}

// Once per device, with that device current: the array's device address, and
// the clear. Later calls read the cached address only.
int na_base(int dev, hipStream_t stream, unsigned char** base) {
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return check_hip(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    unsigned char* b = static_cast<unsigned char*>(p);
    hipLaunchKernelGGL(na_clear_kernel, dim3(64), dim3(256), 0, stream, reinterpret_cast<uint32_t*>(b + kOffTk), kNaTk,
                       reinterpret_cast<uint32_t*>(b + kOffStatus));
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) return check_hip(le, "no-allocation digest set-up");
    (void)cu_count(dev);  // cached before the first launch sizes its grids
    g_na_ptr[dev] = b;
  }
  *base = g_na_ptr[dev];
  return ODP_OK;
}
}  // namespace

int noalloc_take_status(int dev) {
  unsigned char* b = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (dev < 0 || dev >= kNaMaxDevices || !g_na_ptr[dev]) return ODP_OK;
    b = g_na_ptr[dev];
  }
  uint32_t v = 0;
  ODP_HIP(hipMemcpy(&v, b + kOffStatus, sizeof(v), hipMemcpyDeviceToHost));
  if (v) {
    const uint32_t zero = 0;
    ODP_HIP(hipMemcpy(b + kOffStatus, &zero, sizeof(zero), hipMemcpyHostToDevice));
  }
  return v ? -(int)v : ODP_OK;
}
}  // namespace odp

extern "C" int odp_digest_buffers_noalloc(const void* const* ptrs, const uint64_t* sizes, size_t n, uint64_t* out,
                                          odp_stream_t stream_) {
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  if (n == 0) return ODP_OK;
  if (!ptrs || !sizes || !out)
    return set_error(ODP_EINVAL, "odp_digest_buffers_noalloc: null array with n = %zu", n);
  if (n > (size_t)ODP_NOALLOC_MAX_BUFFERS)
    return set_error(ODP_ERANGE, "odp_digest_buffers_noalloc: n = %zu above the maximum of %d buffers", n,
                     ODP_NOALLOC_MAX_BUFFERS);
  int dev = 0;
  int e = current_device(&dev);
  if (e) return e;
  if (dev < 0 || dev >= kNaMaxDevices)
    return set_error(ODP_ERANGE, "odp_digest_buffers_noalloc: device %d above %d", dev, kNaMaxDevices - 1);
  unsigned char* b = nullptr;
  if ((e = na_base(dev, stream, &b))) return e;
  BatchedSpace S;
  S.device = dev;
  S.node_off = reinterpret_cast<uint64_t*>(b + kOffNodeOff);
  S.tree_off = reinterpret_cast<uint64_t*>(b + kOffTreeOff);
  S.tk_off = reinterpret_cast<uint64_t*>(b + kOffTkOff);
  S.small_list = reinterpret_cast<uint32_t*>(b + kOffSmall);
  S.blk = reinterpret_cast<uint64_t*>(b + kOffBlk);
  S.med_rec = reinterpret_cast<NodeRec*>(b + kOffMed);
  S.ctl = reinterpret_cast<DigestCtl*>(b + kOffCtl);
  S.item_buf = reinterpret_cast<uint32_t*>(b + kOffItemBuf);
  S.item_rec = reinterpret_cast<NodeRec*>(b + kOffItemRec);
  S.tree = reinterpret_cast<uint64_t*>(b + kOffTree);
  S.tickets = reinterpret_cast<uint32_t*>(b + kOffTk);
  S.cap_items = kNaItems;
  S.cap_tree = kNaTree;
  S.cap_tk = kNaTk;
  S.cap_nodes = ODP_NOALLOC_MAX_NODES;
  S.status = reinterpret_cast<uint32_t*>(b + kOffStatus);
  return enqueue_batched(S, ptrs, sizes, n, out, stream);
}

extern "C" int odp_digest_buffers_plain(const void* const* host_ptrs, const uint64_t* host_sizes, size_t n,
                                        uint64_t* out, odp_stream_t stream_) {
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  if (n == 0) return ODP_OK;
  if (!host_ptrs || !host_sizes || !out)
    return set_error(ODP_EINVAL, "odp_digest_buffers_plain: null array with n = %zu", n);
  if (n > 0xFFFFFFFFull) return set_error(ODP_ERANGE, "odp_digest_buffers_plain: n = %zu above 2^32 - 1", n);
  uint64_t need_tree = 0, need_tk = 0;
  for (size_t i = 0; i < n; ++i) {
    if (!host_ptrs[i] && host_sizes[i] > 0)
      return set_error(ODP_EINVAL, "odp_digest_buffers_plain: buffer %zu is null with size %llu", i,
                       (unsigned long long)host_sizes[i]);
    if (host_sizes[i] > kLeaf) {
      uint64_t tr, tk;
      tree_need(ceil_div(ceil_div(host_sizes[i], kLeaf), kFanIn), tr, tk);
      need_tree = std::max(need_tree, tr);
      need_tk = std::max(need_tk, tk);
    }
  }
  int err = 0;
  Workspace* ws = workspace_for(stream, &err);
  if (!ws) return err;
  if (need_tree > ws->p_cap_tree || need_tk > ws->p_cap_tk || !ws->p_tickets.ptr) {
    ODP_HIP(hipStreamSynchronize(stream));
    int e = plain_reserve_slots(ws, need_tree, need_tk);
    if (e) return e;
  }
  uint64_t* tree = static_cast<uint64_t*>(ws->p_tree.ptr);
  uint32_t* tk = static_cast<uint32_t*>(ws->p_tickets.ptr);
  for (size_t i = 0; i < n; ++i) {
    const uint64_t s = host_sizes[i];
    const unsigned grid = s <= kLeaf ? 1u : (unsigned)ceil_div(ceil_div(s, kLeaf), kFanIn);
    hipLaunchKernelGGL(digest_one_kernel, dim3(grid), dim3(kThreads), 0, stream,
                       static_cast<const uint8_t*>(host_ptrs[i]), s, out + i, tree, tk);
  }
  return check_hip(hipGetLastError(), "digest_one launch");
}
