/*
 * rd.h -- scoped happens-before race checking of recorded GPU event traces on MI355X (gfx950).
 *
 * The problem (paper Section 2.2): a kernel trace is a sequence of per-thread events in the order
 * the GPU executed them.  Two events race when they access the same global word, or the same
 * shared word of one block (Section 4.1, "shared memory"), at least one writes, they are not both
 * atomics whose scopes overlap (Section 4, Section 5.1), and neither happens before the other
 * (Section 1 race definition).  Happens-before is the scoped HB relation of Section 2.2: program
 * order (rule i), block and warp barriers (rule iii; Section 5.1 for __syncwarp), and a release
 * followed by an acquire of the same sync variable unless both are block scoped in different
 * blocks (rule iv).  Releases and acquires are explicit lock events, or atomics next to a fence in
 * program order (Section 2.1 lock idiom, scope taken from the fence as in Section 5.1).  A fence
 * orders nothing by itself.  The report is every racing pair (first, second), first < second,
 * sorted ascending.
 *
 * Record format (16 bytes, little endian; trace index = position in the array):
 *   addr  4-byte word address; WBAR: warp-barrier id; FENCE and BAR: 0
 *   tid   block * threads_per_block + thread_in_block
 *   meta  kind (bits 0-3) | scope << 4 | space << 6; bits 7-31 must be zero
 *   aux   WBAR: lane mask (bit l = lane l of the warp); otherwise opaque (e.g. a site id)
 *
 * Validity (a trace that breaks a rule is rejected with RD_ETRACE and the first offending index):
 *   record rules, checked first: kind <= 7, scope <= 2, reserved meta bits zero;
 *     tid < n_blocks * threads_per_block; FENCE, BAR and WBAR are in global space.
 *   barrier rules, checked when every record is well formed:
 *     a thread emits nothing after its k-th BAR until every active thread of its block (a thread
 *     with at least one event) has emitted its k-th BAR;
 *     a WBAR's mask contains the emitting lane and equals the mask of the earliest arrival of the
 *     same instance (warp, id, occurrence of that id in the lane's program order); a lane emits
 *     nothing after a WBAR until every lane of the mask has arrived at that instance.
 *   The first offending index is the smallest index of an event that breaks a record rule, or,
 *   when there is none, the smallest index of an event that breaks a barrier rule.
 *
 * Memory: every device buffer is owned by the caller.  rd_workspace_bytes() sizes one workspace
 * per trace; the library never allocates device memory.  The one exception is the fixed array that
 * rd_check_static uses as its workspace (RD_STATIC_SCRATCH_BYTES per GPU, part of the library's
 * code object, held until the process ends).
 *
 * Errors: every call returns an rd_status; nothing throws across this interface.  Errors found on
 * the device during rd_check (trace errors, capacity overflows) are reported by rd_races().
 */
#ifndef RD_H
#define RD_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rd_status;
enum {
    RD_OK = 0,
    RD_EINVAL = -1, /* bad argument: null pointer, bad grid, size out of range */
    RD_ENOMEM = -2, /* workspace, clock pool or internal pair buffer too small */
    RD_ETRACE = -3, /* the trace breaks a validity rule; rd_last_error() gives the event index */
    RD_ETRUNC = -4, /* rd_races: more pairs than the caller's capacity; *n_races has the total */
    RD_EHIP = -5,   /* a HIP runtime call failed */
    RD_ESTATE = -6  /* call out of order (e.g. rd_races before rd_check) */
};

/* event kinds (meta bits 0-3) */
enum { RD_READ = 0, RD_WRITE = 1, RD_ATOMIC = 2, RD_FENCE = 3, RD_BAR = 4, RD_WBAR = 5, RD_ACQ = 6, RD_REL = 7 };
/* scopes (meta bits 4-5); system scope behaves as device scope on one GPU */
enum { RD_BLOCK = 0, RD_DEVICE = 1, RD_SYSTEM = 2 };
/* spaces (meta bit 6) */
enum { RD_GLOBAL = 0, RD_SHARED = 1 };

typedef struct {
    uint32_t addr, tid, meta, aux;
} rd_event;

typedef struct {
    uint32_t n_blocks;          /* >= 1 */
    uint32_t threads_per_block; /* 1 .. 1024 */
    uint32_t warp_size;         /* 1 .. 32, 0 means 32; only warp barriers use it */
    uint32_t reserved;          /* must be 0 */
} rd_grid;

typedef struct {
    uint32_t first, second; /* trace indices, first < second */
} rd_pair;

/* Capacity limits of one workspace.  Zero fields take defaults:
 *   max_pairs    internal race-pair buffer (default max(2^20, n_events / 4));
 *   clock_bytes  pool for knowledge vectors of release/acquire and warp-barrier traces
 *                (default 256 MiB); traces with only block barriers do not use it. */
typedef struct {
    uint64_t max_pairs;
    uint64_t clock_bytes;
} rd_limits;

typedef struct rd_ctx_s *rd_ctx;
typedef struct rd_trace_s *rd_trace;

/* Context on one HIP device.  Thread safe: distinct traces may be used concurrently. */
rd_status rd_init(int hip_device, rd_ctx *out);
rd_status rd_shutdown(rd_ctx ctx);

/* Bytes of device workspace one trace of this shape needs (limits may be NULL). */
rd_status rd_workspace_bytes(rd_ctx ctx, const rd_grid *grid, uint64_t n_events,
                             const rd_limits *limits, uint64_t *bytes);

/* Binds a trace to a caller-owned workspace of at least rd_workspace_bytes() bytes (256-byte
 * aligned).  events_on_device = 0: `events` is host memory; it is copied into the workspace on
 * `stream` and may be freed when the call returns.  events_on_device = 1: `events` is device
 * memory the library reads until rd_trace_free().  No validation of the contents happens here.
 * With events_on_device = 1 the workspace may be NULL: such a trace can only be checked as a member
 * of rd_check_many (rd_check returns RD_ESTATE); when its batch cannot answer for it, it is checked
 * alone in the batch's workspace. */
rd_status rd_trace_upload(rd_ctx ctx, const rd_grid *grid, const rd_event *events, uint64_t n_events,
                          int events_on_device, void *workspace, uint64_t workspace_bytes,
                          const rd_limits *limits, hipStream_t stream, rd_trace *out);

/* Enqueues the whole check on `stream` and returns without waiting; the report is sorted on the
 * device as part of it.  The workspace and the events must stay valid until rd_races() returns or
 * the stream is synchronised.  The first check of a trace is enqueued kernel by kernel; from the
 * second on, the pass is captured once (on a stream of the context) into a HIP graph and each check
 * is one graph launch on `stream`, captured again when the sort variant or the profiled kernels
 * change (rd_set_tuning, rd_profile_enable).  The graph reads the events and the workspace at
 * launch time, so device events rewritten in place are checked anew.  Checks of one trace must
 * not overlap (they share its workspace). */
rd_status rd_check(rd_ctx ctx, rd_trace trace, hipStream_t stream);

/* Waits for the check and copies the report: min(capacity, total) pairs in canonical order into
 * `out` (may be NULL to query the count), *n_races = total.  Returns RD_ETRACE for an invalid
 * trace, RD_ENOMEM when a device-side capacity overflowed, RD_ETRUNC when capacity < total.
 * The check leaves the report on the device in this layout, and as many pairs as the trace's
 * previous report held are copied together with the check's state (one wait when the report is no
 * longer than the last one): entries of `out` past the returned pairs, up to `capacity`, may be
 * overwritten, and so may `out` when an error is returned. */
rd_status rd_races(rd_ctx ctx, rd_trace trace, rd_pair *out, uint64_t capacity, uint64_t *n_races);

/* For callers that cannot allocate device memory -- code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation: rd_trace_upload (events_on_device = 1) + rd_check +
 * rd_races + rd_trace_free of one trace in one synchronous call, with the workspace taken from a
 * fixed device array inside the library instead of a caller buffer.  The array is
 * RD_STATIC_SCRATCH_BYTES on every GPU the library runs on (held until the process ends; its address
 * is looked up by rd_init); the call allocates nothing (no hipMalloc or hipFree, no graph, no
 * events, no page-locked staging) and makes no capture of its own.
 *   events   device memory, n_events records, read during the call;
 *   limits   as for rd_workspace_bytes (may be NULL), except that a zero clock_bytes means
 *            RD_STATIC_CLOCK_BYTES here;
 *   out      host memory for `capacity` pairs (NULL with capacity 0 asks for the count only);
 *            min(capacity, total) pairs in canonical order, *n_races = total;
 *   stream   the check runs on it; the call returns when it has ended.
 * Results and errors are those of the four calls it stands for (RD_ETRACE with the first offending
 * index in rd_last_error, RD_ETRUNC, ...).  RD_ENOMEM, before anything runs, when the workspace
 * of such a check (rd_workspace_bytes(grid, n_events, limits as above) less the event copy and
 * the race-kind scratch it does not need) exceeds RD_STATIC_SCRATCH_BYTES: about 400,000 events
 * with the default limits.  Every call on one GPU uses that GPU's one array and
 * leaves its contents behind (the check clears what it needs at its start): calls that overlap on
 * one GPU -- from other threads or on other streams -- race with each other and give wrong results,
 * so the caller runs them one at a time per GPU. */
#define RD_STATIC_SCRATCH_BYTES (128ull << 20)
#define RD_STATIC_CLOCK_BYTES (8ull << 20)
rd_status rd_check_static(rd_ctx ctx, const rd_grid *grid, const rd_event *events, uint64_t n_events,
                          const rd_limits *limits, rd_pair *out, uint64_t capacity, uint64_t *n_races,
                          hipStream_t stream);

/* One unique race kind: the unordered pair of the two racing accesses' site ids (the records'
 * aux words, site_lo <= site_hi) and the number of racing pairs of that kind.  The paper counts
 * unique kinds of races (Table 2, Section 6) without defining a kind; this is the reading taken. */
typedef struct {
    uint32_t site_lo, site_hi, count;
} rd_race_kind;

/* The unique race kinds of a checked trace, built on the device from its report: min(capacity,
 * total) kinds in ascending (site_lo, site_hi) order into `out` (may be NULL with capacity 0 to
 * query the count), *n_kinds = total.  Call after rd_check (rd_races need not come first); the
 * events and the workspace must still be valid.  Waits for the check.  The scratch (32 bytes per
 * race pair) is part of the trace's workspace, over memory the check no longer reads once it has
 * ended, so the call allocates nothing; it runs on the trace's stream and must not overlap another
 * call on the same trace.  Errors: those of rd_races for the check itself, RD_ETRUNC when
 * capacity < total, RD_ESTATE for a batch member without a workspace of its own (a member with
 * one is checked alone first). */
rd_status rd_race_kinds(rd_ctx ctx, rd_trace trace, rd_race_kind *out, uint64_t capacity, uint64_t *n_kinds);

/* The lockset pass the paper describes for ScoRD (Section 2.2, Section 3; Eraser's analysis), a
 * second workload over the same trace.  Every access carries the locks its thread holds at it: an
 * acquire (explicit, or an atomic right before a fence) of a word the thread does not hold opens a
 * critical section with the acquire's scope, the thread's next release of that word closes it.
 * Each access that is not a lock operation is compared with the previous such access of its
 * location in trace order, and the pair (previous, current) is reported when they conflict, at
 * least one of the two holds a lock, and no word is held by both with overlapping scopes (either
 * device/system scoped, or both in one block).  Unlike the happens-before report this is a
 * heuristic: it misses races of two unprotected accesses and flags correctly published data read
 * under a lock.
 * Runs a check of the trace and the pass on the trace's stream and waits: min(capacity, total)
 * pairs, sorted, into `out` (host memory; NULL with capacity 0 for the count), *n_pairs = total.
 * The pass keeps its tables in the trace's knowledge-vector pool (24 bytes per rd_limits.max_pairs
 * pair, 516 bytes per lock operation).  Errors: those of the check (RD_ETRACE ...), RD_ENOMEM when a
 * thread holds more than 64 locks at once, the pool is too small, or the pairs exceed max_pairs,
 * RD_ETRUNC when capacity < total, RD_ESTATE for a trace bound without a workspace.  Afterwards
 * rd_races returns that check's report. */
rd_status rd_lockset(rd_ctx ctx, rd_trace trace, rd_pair *out, uint64_t capacity, uint64_t *n_pairs);

/* The predictive relation GWCP (Section 4, Algorithms 1 and 2), a third workload over the same
 * trace: the races a reordering of the trace's critical sections could expose, a superset of the
 * happens-before report.  Each thread t keeps a local time N_t and clocks P_t (GWCP) and H_t (scoped
 * happens-before) with one word per program thread; lock operations (explicit, or atomics inferred
 * from fences; the critical sections as rd_lockset defines them) update them by Algorithm 1 with
 * scoped lock clocks, rule (ii)'s release-time joins and the read / write clocks L^r, L^w; reads and
 * writes inside critical sections by Algorithm 2; barrier and warp-barrier completions give every
 * participant the join of their clocks.  A pair (a, b) of conflicting accesses of different threads,
 * a before b in the trace (conflict and atomic scopes as for rd_races), is reported when a's local
 * time is above P_t at b for b's thread t.
 * Runs a check of the trace and the pass on the trace's stream and waits: min(capacity, total)
 * pairs, sorted, into `out` (host memory; NULL with capacity 0 for the count), *n_pairs = total.
 * The pass keeps its clocks in the trace's knowledge-vector pool: 8 T^2 bytes for the dense clocks
 * of T threads, 24 bytes per rd_limits.max_pairs pair, 4 T bytes per clock it keeps (lock clocks,
 * L^r / L^w per lock and location, the acquire and release times of each critical section, a copy
 * of P per event that changes it) and tables of about 100 bytes per lock operation and 20 bytes per
 * (access, held lock) pair.  Errors: those of the check (RD_ETRACE ...), RD_EINVAL for more than 4096
 * threads, RD_ENOMEM when a thread holds more than 64 locks at once, the pool is too small, or the
 * pairs exceed max_pairs, RD_ETRUNC when capacity < total, RD_ESTATE for a trace bound without a
 * workspace.  Afterwards rd_races returns that check's report. */
rd_status rd_gwcp(rd_ctx ctx, rd_trace trace, rd_pair *out, uint64_t capacity, uint64_t *n_pairs);

/* Batched form (the same check, many traces per pass).  The members are independent traces, each
 * bound by rd_trace_upload to its own workspace as for rd_check.  rd_check_many enqueues one pass
 * of the pipeline over their concatenation: every trace keeps its own blocks, threads and words
 * (blocks and global words are renumbered apart, trace indices shifted), so no pair and no
 * happens-before edge crosses traces and the merged report, sorted, is every member's report in a
 * run of its own.  Afterwards rd_races(ctx, traces[j], ...) returns exactly what rd_check followed
 * by rd_races would for traces[j], errors included: when the merged pass cannot answer for a member
 * (some member is invalid, a capacity of the merged pass overflowed, or the member has more pairs
 * than its own rd_limits.max_pairs) that rd_races checks the member on its own first.  Members with
 * different warp sizes, or more than 2^32 - 1 events or threads in all, are checked one by one.
 *
 * `workspace` (caller-owned device memory, 256-byte aligned, rd_batch_workspace_bytes() bytes) holds
 * the merged trace and its check; it and the members' workspaces and events must stay valid until
 * the members' reports have been read.  `limits` (may be NULL) applies to the merged pass; its
 * default max_pairs is the sum of the members' limits, at most the default of one trace of the
 * merged length.  Asynchronous on `stream`. */
/* *bytes = 0 when the members cannot share one pass (rd_check_many then needs no workspace). */
rd_status rd_batch_workspace_bytes(rd_ctx ctx, const rd_trace *traces, uint32_t n, const rd_limits *limits,
                                   uint64_t *bytes);
rd_status rd_check_many(rd_ctx ctx, const rd_trace *traces, uint32_t n, void *workspace, uint64_t workspace_bytes,
                        const rd_limits *limits, hipStream_t stream);

/* The batched pass captured once into a HIP graph (on a non-default `stream`), for members whose
 * event buffers are refilled in place and checked again: rd_graph_launch replays the whole pass
 * (table upload, merge, check, pair sort) with one launch, after which the members' reports are
 * read as after rd_check_many.  The members, their events and the workspace must stay valid until
 * rd_graph_free; the member set and sizes are those of the capture. */
typedef struct rd_graph_s *rd_graph;
rd_status rd_batch_capture(rd_ctx ctx, const rd_trace *traces, uint32_t n, void *workspace, uint64_t workspace_bytes,
                           const rd_limits *limits, hipStream_t stream, rd_graph *out);
rd_status rd_graph_launch(rd_ctx ctx, rd_graph graph, hipStream_t stream);
rd_status rd_graph_free(rd_ctx ctx, rd_graph graph);

/* Reports of n checked traces in one call: member j's pairs follow member j-1's in `out` (canonical
 * order inside each member), counts[j] = member j's total, statuses[j] = what rd_races would return
 * for it (RD_ETRUNC when its pairs did not all fit in what was left of `capacity`).  Members of one
 * batch are copied from the device in one transfer.  Returns RD_OK, or the first member status that
 * is not RD_OK. */
rd_status rd_races_many(rd_ctx ctx, const rd_trace *traces, uint32_t n, rd_pair *out, uint64_t capacity,
                        uint64_t *counts, rd_status *statuses);

rd_status rd_trace_free(rd_ctx ctx, rd_trace trace);

/* Figures of a trace's last check (diagnostics; waits for it).  The knowledge vectors are the
 * happens-before clocks of Algorithm 1 (Section 4.1) stored with the compression of Section 5.2:
 * one word per block (the block's barrier phase stands for every thread of the block) plus one word
 * per thread that releases (or takes part in a warp barrier), instead of one word per thread. */
typedef struct {
    uint64_t n_events;          /* records */
    uint64_t n_accesses;        /* reads, writes, atomics, lock acquires and releases */
    uint64_t kind_count[8];     /* records of each kind */
    uint32_t key_bits;          /* significant bits of the location key (sort passes follow from it) */
    uint32_t max_phase;         /* the most block barriers any thread passed */
    uint32_t engine;            /* 0: no knowledge vectors needed; 1: parallel engine; 2: interpreter */
    uint32_t packed;            /* where category and phase rode: 1 the location key word, 2 the
                                   thread word, 0 a word of their own */
    uint64_t clock_vectors;     /* knowledge vectors written (the empty one included) */
    uint64_t clock_words;       /* words per vector: blocks + threads with a column */
    uint64_t clock_bytes;       /* clock_vectors * clock_words * 4: pool bytes the check used */
    uint64_t dense_clock_bytes; /* the same vectors as one word per thread (no compression) */
    uint64_t engine_ops;        /* operations of the parallel engine (releases, acquires, barriers) */
    uint64_t engine_groups;     /* dependency-free groups they were evaluated in */
    uint64_t slow_chunks;       /* 64-access chunks the segment check sent to its exact slow path */
    uint64_t race_pairs;        /* pairs found (may exceed the pair buffer) */
    uint64_t workspace_bytes;   /* the workspace the trace needs (rd_workspace_bytes) */
} rd_stats;
rd_status rd_trace_stats(rd_ctx ctx, rd_trace trace, rd_stats *out);

/* Tuning of the location sort (the dominant kernel): built-in variants that differ in digit width
 * (7, 8 or 9 bits, hence passes), wavefronts per workgroup and items per lane (hence tile size).
 * Results never depend on the variant.  rd_set_tuning selects one for every later check on the
 * context (default 0); rd_autotune times every variant on the given traces -- one trace alone, or a
 * batch when batch_workspace is given -- with rd_check / rd_check_many (one warm-up and three timed
 * runs each, HIP events on `stream`), selects the fastest, returns its index in *best and the mean
 * milliseconds of each variant in ms[] (may be NULL; rd_tuning_count() entries), and leaves the
 * traces checked with the chosen variant.  Synchronous. */
typedef struct {
    uint32_t radix_bits, waves_per_block, items_per_lane, reserved;
} rd_tuning;
rd_status rd_tuning_count(uint32_t *n);
rd_status rd_tuning_get(uint32_t index, rd_tuning *out);
rd_status rd_set_tuning(rd_ctx ctx, uint32_t index);
rd_status rd_get_tuning(rd_ctx ctx, uint32_t *index);
rd_status rd_autotune(rd_ctx ctx, const rd_trace *traces, uint32_t n, void *batch_workspace, uint64_t batch_bytes,
                      hipStream_t stream, uint32_t *best, double *ms);

/* Served form: a request loop with continuous batching under an HBM budget.  The caller hands over
 * one device arena (its size is the budget for the requests' events and the passes' workspaces,
 * reused from pass to pass; the server allocates no other device memory).  Requests queue in
 * submission order; each of max_inflight workers (own thread, own HIP stream) takes, whenever it is
 * free, every waiting request that fits the arena and shares the first one's warp size (up to
 * max_batch) and checks them in one rd_check_many pass, so passes of different workers overlap on
 * the device and requests that arrive while others run are admitted as memory comes back.  Every
 * request's result is the one rd_check + rd_races gives for it alone (pairs, status, first offending
 * index).  A request larger than the whole arena fails with RD_ENOMEM. */
typedef struct {
    uint64_t device_bytes;  /* bytes of the arena (>= 4096) */
    uint32_t max_batch;     /* most requests in one pass (0: 256) */
    uint32_t max_inflight;  /* passes in flight at once (0: 2) */
} rd_server_config;
typedef struct {
    uint64_t n_races;    /* pairs of the request (RD_OK) */
    uint64_t bad_index;  /* first offending event (RD_ETRACE), else UINT64_MAX */
    double submit_s, start_s, done_s;  /* server clock (seconds since open): submitted, admitted, answered */
} rd_request_info;
typedef struct rd_server_s *rd_server;

/* device_arena: caller-owned device memory, 256-byte aligned, cfg->device_bytes long, valid until
 * rd_server_close returns. */
rd_status rd_server_open(rd_ctx ctx, void *device_arena, const rd_server_config *cfg, rd_server *out);
/* events: host memory, read until the request has been answered.  Thread safe. */
rd_status rd_server_submit(rd_server srv, const rd_grid *grid, const rd_event *events, uint64_t n_events,
                           uint64_t *ticket);
/* Blocks until the request is answered; copies min(capacity, n) pairs in canonical order, fills
 * *info (may be NULL) and forgets the ticket.  Returns the request's status (RD_ETRUNC when
 * capacity < n).  Thread safe. */
rd_status rd_server_wait(rd_server srv, uint64_t ticket, rd_pair *out, uint64_t capacity, rd_request_info *info);
rd_status rd_server_stats(rd_server srv, uint64_t *passes, uint64_t *requests_done);
/* Waits for every submitted request, stops the workers. */
rd_status rd_server_close(rd_server srv);

const char *rd_strerror(rd_status status);

/* Details of the last error on this context: for RD_ETRACE the first offending event index
 * (UINT64_MAX otherwise) and a message. */
rd_status rd_last_error(rd_ctx ctx, uint64_t *event_index, char *msg, uint64_t msg_len);

/* Per-kernel timing (diagnostics).  rd_profile_enable(ctx, name) brackets every later launch of the
 * named kernel ("prefix*" = every kernel whose name starts with prefix, "*" = every kernel, NULL =
 * off) made by rd_check/rd_races on this context with HIP events on the launch stream (inside the
 * captured graph for graph launches; a check collects the previous launch's times of that graph
 * before launching it again, waiting for it); rd_profile_read() waits for them and returns, per
 * kernel name, the number of launches and their summed duration since the last read or enable
 * (and resets the counters). */
typedef struct {
    char name[48];
    uint32_t launches;
    double total_ms;
} rd_kernel_time;
rd_status rd_profile_enable(rd_ctx ctx, const char *kernel);
rd_status rd_profile_read(rd_ctx ctx, rd_kernel_time *out, uint32_t capacity, uint32_t *n_out);

#ifdef __cplusplus
}
#endif
#endif /* RD_H */
