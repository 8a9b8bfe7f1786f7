/*
 * odp.h -- C ABI of the MI355X (gfx950) content-digest and mapping-trace
 * analysis library: the data-parallel hot path of "Dynamic Detection of
 * Inefficient Data Mapping Patterns in Heterogeneous OpenMP Applications"
 * (PPoPP '26).
 *
 * The paper's detector (Sec. 5) takes a chronological log of OpenMP target
 * events, each carrying start/end time, a hash of the data it moved, source and
 * destination device numbers, a code pointer, a byte count and an operation
 * type, and finds four inefficient mapping patterns (Sec. 4, Defs. 1-4):
 * duplicate transfers, round-trip transfers, repeated device allocations and
 * unused device allocations. This library computes the two data-parallel
 * parts of that method on one GPU:
 *
 *   odp_digest_buffers   the content digest of every transferred or mapped
 *                        buffer (the paper hashes each transfer, Sec. 5.1 and
 *                        App. B; here the digest is ODP-D64 v1, defined below)
 *   odp_analyze_trace    one pass over the event log that flags the four
 *                        patterns from those digests and addresses (both
 *                        halves of Def. 4: unused allocations and unused
 *                        transfers), and the optimization-potential estimate
 *                        of Sec. 7.6
 *   odp_server_*         the two combined for requests that arrive over
 *                        time: each is digested and classified as it comes,
 *                        with continuous batching (an extension; the paper
 *                        analyses post mortem)
 *
 * Conventions for every entry point
 *   - All pointers marked DEVICE must be device-accessible: hipMalloc memory,
 *     or pinned host memory mapped into the device address space. HOST marks
 *     ordinary host memory read during the call.
 *   - The caller owns every array. The library keeps only its own workspace
 *     (grow-only, per device and stream), released by odp_release().
 *   - Calls only enqueue work on `stream` (a hipStream_t; NULL means the
 *     default stream) and return; results are valid once the stream reaches
 *     that point. odp_digest_buffers_plain is the exception noted there.
 *   - Return value: ODP_OK (0) or a negative ODP_E* code. Nothing throws
 *     across the ABI. odp_last_error_string() describes the last failure of
 *     the calling thread.
 *   - Calls on different streams may run concurrently; calls on one stream are
 *     ordered by the stream.
 */
#ifndef ODP_H
#define ODP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* odp_stream_t; /* a hipStream_t */

enum {
  ODP_OK = 0,
  ODP_EINVAL = -1,  /* null array with n > 0, null buffer with size > 0, bad tuning */
  ODP_ERANGE = -2,  /* n above the supported maximum (2^32 - 1 events or buffers) */
  ODP_ENOMEM = -3,  /* workspace could not be allocated */
  ODP_EHIP = -4,    /* HIP launch or runtime failure (see odp_last_error_string) */
  ODP_ECAPACITY = -5 /* digest tree workspace too small for the call (see odp_reserve) */
};

/* ---------------------------------------------------------------------------
 * ODP-D64 v1, the content digest (this library's definition).
 *
 * The paper hashes every transferred buffer whole with a 64-bit
 * non-cryptographic hash and assumes no collisions (Sec. 5.1; App. B studies 19
 * such hashes, XXH64 among them). A whole-buffer serial hash cannot use a GPU,
 * so the digest is defined as a tree of XXH64 calls (XXH64 as in the public
 * xxHash specification, input read little-endian):
 *
 *   n <= 4096 bytes:  D64(b) = XXH64(b, seed 0)            (also for n = 0)
 *   n  > 4096 bytes:  leaves  = XXH64 of each 4096-byte piece (last one
 *                               shorter), seed 0
 *                     level s = groups of up to 64 consecutive digests of
 *                               level s-1, serialised as little-endian u64,
 *                               each group hashed with XXH64(seed = s),
 *                               s = 1, 2, ... until one digest remains.
 *
 * Only the bytes matter: the same bytes at any address or alignment give the
 * same digest, and no tuning choice changes it. Duplicate and round-trip
 * detection need digest equality only, so under the paper's collision-free
 * assumption the flags do not depend on which 64-bit hash is used.
 * ------------------------------------------------------------------------ */

/* Batched digest: one persistent launch over all buffers.
 *   ptrs   DEVICE, n entries: start address of buffer i (device memory; any
 *          alignment; buffers may overlap or alias; they are only read).
 *   sizes  DEVICE, n entries: byte length of buffer i (0 allowed).
 *   out    DEVICE, n entries: receives D64(buffer i). Must not overlap the
 *          inputs.
 * Work plan, leaf hashing, level-1 combine and upper levels all run on the
 * device; the host reads no size. The sum over buffers of ceil(size/262144)
 * must fit the tree workspace (odp_reserve; by default sized for four times
 * the device's memory in distinct buffers). When it does not, every out[i] of
 * the call is set to 0 and odp_device_status() reports ODP_ECAPACITY once the
 * stream has completed. n = 0 returns ODP_OK and enqueues nothing.
 * Capture-safe (no allocation, no memset node) once odp_reserve covered n. */
int odp_digest_buffers(const void* const* ptrs, const uint64_t* sizes, size_t n, uint64_t* out,
                       odp_stream_t stream);

/* Batched digest that allocates nothing, for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, harnesses
 * that forbid allocation). Same arguments and result as odp_digest_buffers;
 * its workspace is one fixed array of ODP_NOALLOC_SCRATCH_BYTES in the
 * library's device code, which each GPU the library runs on holds from load
 * until the process ends. The call makes no device or pinned allocation and
 * builds no graph (its launches go straight onto `stream`).
 *   n > ODP_NOALLOC_MAX_BUFFERS returns ODP_ERANGE and enqueues nothing.
 *   The buffers larger than 4096 bytes may hold at most ODP_NOALLOC_MAX_NODES
 *   level-1 nodes in all (the sum of ceil(size / 262144) over them; 16 GiB
 *   of data in large buffers). The sizes are read on the device, so a call
 *   over that limit is found there: every out[i] is set to 0 and
 *   odp_device_status() reports ODP_ECAPACITY. Check it before handing the
 *   digests to the analysis.
 * Every call on one GPU shares that GPU's array and leaves the last call's
 * contents in it: calls that overlap on one GPU (on different streams, or
 * from different threads) race and must be ordered by the caller. */
#define ODP_NOALLOC_MAX_BUFFERS 16384
#define ODP_NOALLOC_MAX_NODES 65536
#define ODP_NOALLOC_SCRATCH_BYTES 4619520
int odp_digest_buffers_noalloc(const void* const* ptrs, const uint64_t* sizes, size_t n, uint64_t* out,
                               odp_stream_t stream);

/* Per-buffer digest: the plain form, one kernel launch per buffer.
 *   host_ptrs   HOST, n entries: device start address of buffer i.
 *   host_sizes  HOST, n entries: byte length of buffer i.
 *   out         DEVICE, n entries: receives D64(buffer i).
 * Same result as odp_digest_buffers. May allocate (grow) workspace before the
 * first launch; not capture-safe when it has to grow. */
int odp_digest_buffers_plain(const void* const* host_ptrs, const uint64_t* host_sizes, size_t n,
                             uint64_t* out, odp_stream_t stream);

/* ---------------------------------------------------------------------------
 * Event log record (64 bytes, 8-byte aligned). The paper's tool logs 72 bytes
 * per data operation and 24 per target launch (Sec. 7.4) with the fields its
 * detector needs (Sec. 5); this record carries the same fields, and a target
 * launch is a record with op = ODP_KERNEL.
 * ------------------------------------------------------------------------ */
enum {
  ODP_ALLOC = 1,  /* device allocation: host address in src_addr, device address in dst_addr */
  ODP_H2D = 2,    /* host -> device transfer */
  ODP_D2H = 3,    /* device -> host transfer */
  ODP_D2D = 4,    /* device -> device transfer */
  ODP_DELETE = 5, /* device deallocation: addresses as for ALLOC */
  ODP_KERNEL = 6  /* target kernel execution on device dst_dev */
};

typedef struct odp_event {
  uint64_t digest;   /* transfers: D64 of the bytes moved; ignored otherwise */
  uint64_t src_addr; /* transfers: source address; ALLOC/DELETE: host address */
  uint64_t dst_addr; /* transfers: destination address; ALLOC/DELETE: device address */
  uint64_t bytes;    /* bytes moved or allocated */
  uint64_t t_start;  /* ns; must not decrease along the array (the log is chronological) */
  uint64_t t_end;    /* ns; must be >= t_start */
  uint64_t codeptr;  /* opaque return address (kept, not used by the rules) */
  int16_t src_dev;   /* transfers: sending device, -1 = host */
  int16_t dst_dev;   /* transfers: receiving device; ALLOC/DELETE/KERNEL: the device */
  uint8_t op;        /* ODP_ALLOC .. ODP_KERNEL */
  uint8_t rsv0;
  uint16_t rsv1;
} odp_event;

#define ODP_MAX_DEVICE 9 /* device numbers -1 (host) .. 9 are accepted */

/* Per-event flag bits written to out_flags. */
enum {
  ODP_F_DD = 1,      /* duplicate transfer: the receiver already got this digest (Def. 1, Alg. 1) */
  ODP_F_RT_TX = 2,   /* round trip, outbound: a later transfer carries this digest back (Def. 2, Alg. 2) */
  ODP_F_RT_RX = 4,   /* round trip, return leg: the latest earlier transfer of this digest
                        between the same two endpoints went the other way */
  ODP_F_RA = 8,      /* repeated allocation: an earlier paired ALLOC had the same
                        (host address, device, bytes) (Def. 3, Alg. 3) */
  ODP_F_UA = 16,     /* unused allocation: no kernel on the device meets the closed interval
                        [ALLOC.t_start, DELETE.t_end] (Def. 4, Alg. 4) */
  ODP_F_PAIRED = 32, /* ALLOC/DELETE matched into a pair (see below) */
  ODP_F_UT = 64,     /* unused transfer: no kernel on the receiving device can read the copy before
                        the next copy to the same place begins (Def. 4, Alg. 5) */
  ODP_F_INVALID = 128 /* record rejected: unknown op, t_end < t_start, t_start below the
                         previous record's, or a device number outside -1..ODP_MAX_DEVICE */
};

/* Counts and sums over one log (248 bytes). Filled on the device; valid after
 * the stream completes. *_bytes and *_time_ns sum `bytes` and
 * (t_end - t_start) over the flagged records (round trips: over return legs;
 * RA/UA: the ALLOC plus its DELETE's duration), the inputs of the paper's
 * savings estimate (Sec. 7.6), which the last three fields complete:
 *   span_ns            latest t_end minus earliest t_start over the valid
 *                      records (0 when there is none): the run's total time
 *   elim_ns            the time removing the flagged mappings would save, each
 *                      record counted once whatever flags it carries: a
 *                      transfer flagged DD, RT_RX or UT, and the ALLOC and
 *                      DELETE of a pair flagged RA or UA
 *   predicted_speedup  span_ns / (span_ns - elim_ns); 1.0 when span_ns is 0,
 *                      +infinity when elim_ns >= span_ns */
typedef struct odp_report {
  uint64_t n_events, n_invalid, n_transfers, n_kernels;
  uint64_t n_alloc_pairs, n_unpaired_alloc, n_unpaired_delete;
  uint64_t dd_events, dd_groups, dd_members, dd_bytes, dd_time_ns;
  uint64_t rt_pairs, rt_rx_events, rt_bytes, rt_time_ns;
  uint64_t ra_events, ra_groups, ra_members, ra_bytes, ra_time_ns;
  uint64_t ua_events, ua_bytes, ua_time_ns;
  uint64_t ut_events, ut_bytes, ut_time_ns;
  uint64_t span_ns, elim_ns;
  double predicted_speedup;
  int32_t status;           /* 0, or 1 when some record was rejected */
  uint32_t first_bad_event; /* index of the first rejected record, 0xFFFFFFFF if none */
} odp_report;

/* Mapping-trace analysis (Sec. 5, Algs. 1-5; Sec. 7.6) over a chronological log.
 *   events      DEVICE, n records in log order (array order is time order; the
 *               index breaks ties).
 *   out_flags   DEVICE, n bytes: ODP_F_* bits of each record.
 *   out_report  DEVICE, one odp_report.
 * Rules (transfers are valid records with op H2D/D2H/D2D, in log order):
 *   DD     some earlier transfer has the same digest and the same dst_dev.
 *   RT_TX  src_dev != dst_dev, and some later transfer has the same digest with
 *          (src_dev, dst_dev) swapped. rt_pairs counts these.
 *   RT_RX  src_dev != dst_dev, and the latest earlier transfer with the same
 *          digest between the same two endpoints went the other way.
 *   Pairing (the allocation/deletion pairing the paper's Algs. 3-4 use but do
 *          not define): ALLOC/DELETE records grouped by (dst_dev, dst_addr) in
 *          log order; a DELETE pairs with the record just before it in its
 *          group when that record is an ALLOC.
 *   RA     a paired ALLOC with an earlier paired ALLOC of the same
 *          (src_addr, dst_dev, bytes).
 *   UA     a paired ALLOC on device d whose [t_start, DELETE.t_end] meets no
 *          KERNEL record's [t_start, t_end] on d (closed intervals).
 *   UT     a transfer with op H2D or D2D into device d = dst_dev >= 0 whose
 *          [t_start, next.t_start] meets no KERNEL record's [t_start, t_end]
 *          on d, where next is the next such transfer in log order with the
 *          same (dst_dev, src_dev, src_addr), the copy that overwrites it (no
 *          upper end when there is none).
 * Data-dependent problems do not fail the call: rejected records get
 * ODP_F_INVALID, take part in no rule, and set report.status.
 * n = 0 writes an empty report. n > 2^32 - 1 returns ODP_ERANGE.
 * Logs of at most 512 records are analysed by one workgroup in one launch and
 * need no workspace. For longer logs the allocation rules run on a side
 * stream of the workspace that is forked from `stream` and joined back before
 * the report is written, so the call remains ordered on `stream` (and
 * capturable as one unit). Capture-safe once odp_reserve covered n (always for
 * n <= 512). */
int odp_analyze_trace(const odp_event* events, size_t n, uint8_t* out_flags, odp_report* out_report,
                      odp_stream_t stream);

/* Comparison mode for logs with three or more endpoints (Sec. 5, Alg. 2;
 * Sec. 7.8): the analysis above (same flags and report) plus the <tx, rx>
 * pairs that Algorithm 2 records when followed literally. For each digest h
 * and endpoint d the algorithm keeps the list R(h, d) of all valid transfers
 * of h into d, over the whole log in log order, and a count c(h, d); walking
 * the valid transfers (H2D, D2H, D2D; self-transfers included) in log order,
 * it records a transfer tx of h out of s, with rx = R(h, s)[c(h, s)], when
 * c(h, s) < |R(h, s)|, and then adds one to c(h, dst(tx)). On two endpoints
 * these pairs are the round trips of the rule above; on more, rx can precede
 * tx or come from a third endpoint, which the definitional rule never pairs.
 *   out_rx      device, n uint32: for a recorded tx, the record index of its rx;
 *               0xFFFFFFFF for every other record (written for all n)
 *   out_npairs  device, one uint64: the number of recorded pairs
 * Always runs on the workspace (any n, also n <= 512); never replayed from
 * the analysis graph cache. Errors as odp_analyze_trace, and ODP_EINVAL for a
 * null out_npairs, or a null out_rx with n > 0. */
int odp_analyze_trace_alg2(const odp_event* events, size_t n, uint8_t* out_flags, odp_report* out_report,
                           uint32_t* out_rx, uint64_t* out_npairs, odp_stream_t stream);

/* ---------------------------------------------------------------------------
 * Serving: mapping-event requests classified as they arrive.
 *
 * A request is one odp_event plus, for a transfer, the device-resident bytes it
 * moved (the digest field is then filled from those bytes). Requests are
 * admitted into ticks as slots and the memory budget allow; a tick is one
 * batched digest of its payloads (on the server's digest stream) and one
 * classification against device-resident per-key state (on its classification
 * stream, after that digest), appended to a device-resident log; the digest of
 * the next tick overlaps the classification of the current one (a tick
 * submitted while none is in flight is classified on the digest stream).
 * Every flag is set in the server's "known" flags as soon as the records that
 * decide it have arrived (the rules of Sec. 4, Defs. 1-4, and Sec. 5; the
 * paper analyses post mortem, serving is an extension):
 *   DD, RT_RX, PAIRED, INVALID  at the record's arrival;
 *   RT_TX  when a later transfer carries the digest back;
 *   RA     when the ALLOC is paired (or when an earlier ALLOC of its key is);
 *   UA     once a record starting after the DELETE's end has arrived;
 *   UT     once a record starting after the next copy's start has arrived.
 * UA and UT are set early only while no record has been rejected: they rest on
 * the log being chronological, and a record rejected later can let a later
 * record start earlier than one already logged. A transfer never sent back and
 * a copy never overwritten are decided by the drain, which runs the full
 * analysis of the whole log in arrival order.
 * Errors: every call returns an ODP_* code; on failure the message is in
 * odp_last_error_string(). A server belongs to one host thread.
 * ------------------------------------------------------------------------ */
typedef struct odp_server odp_server;

enum {
  ODP_SERVER_BATCHED = 0, /* continuous batching: ticks of up to max_tick requests */
  ODP_SERVER_PLAIN = 1    /* one request per tick, one tick in flight, per-buffer digest launches */
};

typedef struct odp_server_config {
  uint64_t max_events;   /* records over the server's life (log capacity), 1 .. 2^32 - 1 */
  uint64_t budget_bytes; /* device memory budget: the server's state and digest workspace
                            (odp_server_stats.state_bytes, fixed at creation) plus the payload
                            bytes of the requests in flight */
  uint32_t max_inflight; /* in-flight requests admitted at most (slots) */
  uint32_t max_tick;     /* records per tick, 1 .. 1024 */
  uint32_t mode;         /* ODP_SERVER_BATCHED or ODP_SERVER_PLAIN */
  uint32_t reserved;     /* 0 */
} odp_server_config;

typedef struct odp_server_stats {
  double seconds;        /* wall time of the run */
  uint64_t ticks;        /* ticks launched */
  uint64_t max_tick;     /* largest tick */
  uint64_t bytes;        /* payload bytes digested */
  uint64_t budget_waits; /* requests whose admission waited for the byte budget */
  uint64_t state_bytes;  /* device bytes of the server's state and digest workspace */
} odp_server_stats;

/* Creates a server on the current device with its own two streams; allocates
 * the log (64 B per record), the per-record flags and links (9 B), the
 * per-device kernel lists (176 B per record), the waiting windows (64 B per
 * record), six state tables (40 B x 2 x max_events each, rounded up to a
 * power of two) and the digest workspace for payload batches up to
 * budget_bytes. ODP_EINVAL when budget_bytes does not exceed what that
 * takes. *out is owned by the caller until odp_server_destroy. */
int odp_server_create(const odp_server_config* cfg, odp_server** out);

/* Runs an open-loop schedule to completion. All arrays are HOST arrays of n:
 *   events         the records (arrival order)
 *   payload_ptrs   device address of the bytes each record moved, or 0
 *   payload_bytes  their length (a request above budget_bytes - state_bytes is rejected)
 *   arrival_ns     scheduled arrival, ns after the call starts, non-decreasing
 *   complete_ns    out: when the request's tick was seen complete, ns after start
 * Blocks until every request is complete. Requests keep arrival order in the
 * log across calls. */
int odp_server_run(odp_server* s, const odp_event* events, const uint64_t* payload_ptrs, const uint64_t* payload_bytes,
                   const uint64_t* arrival_ns, size_t n, uint64_t* complete_ns, odp_server_stats* stats);

/* Waits for the server, then (each optional, DEVICE arrays of the logged count):
 * out_known gets the flags decided so far (see above); out_flags/out_report
 * get the analysis of the whole log (both or neither). ODP_ECAPACITY if a
 * state table ran full. */
int odp_server_drain(odp_server* s, uint8_t* out_known, uint8_t* out_flags, odp_report* out_report);

/* Copies the logged records (digests filled in) to DEVICE out_events (may be
 * NULL) and their count to *n. */
int odp_server_log(odp_server* s, odp_event* out_events, size_t* n);

/* Waits for the server and frees everything it holds; NULL is a no-op. */
int odp_server_destroy(odp_server* s);

/* ---------------------------------------------------------------------------
 * Helpers (workspace, tuning, status). Not part of the method.
 * ------------------------------------------------------------------------ */

/* Library version as 10000*major + 100*minor + patch. */
int odp_version(void);

/* Text of the calling thread's last error ("" if none). Owned by the library. */
const char* odp_last_error_string(void);

/* Pre-size the workspace of the current device for `stream`: up to max_buffers
 * buffers totalling max_total_bytes for odp_digest_buffers, and up to
 * max_events records for odp_analyze_trace (which also creates the
 * workspace's side stream and the two events that fork and join it).
 * Synchronous; allocates. Call it before capturing calls into a hipGraph. */
int odp_reserve(size_t max_buffers, uint64_t max_total_bytes, size_t max_events, odp_stream_t stream);

/* Frees every workspace the library holds (all devices and streams), the
 * analysis side streams included. Waits for the device first. Graphs that
 * captured library calls and live servers keep pointers into these
 * workspaces: destroy them first (a later call simply reserves again). */
int odp_release(void);

/* Sticky device-side status of the current device: ODP_OK or ODP_ECAPACITY
 * when a batched digest call (odp_digest_buffers or
 * odp_digest_buffers_noalloc) found its tree workspace too small. Reading it
 * synchronises the device and clears it. */
int odp_device_status(void);

/* Launch parameters of the batched digest. They change speed, never results. */
typedef struct odp_tuning {
  uint32_t blocks_per_cu;   /* persistent workgroups per compute unit, 1..8 */
  uint32_t use_graph;       /* 1: replay the work plan + digest launch as a hipGraph */
  uint32_t split_bytes;     /* level-1 nodes of at most this many bytes (0 or 4096..65536) are
                               hashed and combined by one wavefront, four per work item;
                               larger nodes take a whole workgroup */
  uint32_t chunk_nodes;     /* work items a workgroup claims at once from the queue, 1..16
                               (0 reads as 1): consecutive items, so a chunk of node items is
                               64 * chunk_nodes consecutive leaves (256 KiB each node) */
  uint32_t reserved[4];
} odp_tuning;

int odp_get_tuning(odp_tuning* out);
int odp_set_tuning(const odp_tuning* in);

#ifdef __cplusplus
}
#endif

#endif /* ODP_H */
