// rd_kernels.h -- host launchers of the pipeline stages (each defined in its own .hip file).
#pragma once
#include "rd_internal.h"

namespace rd {
void scan_exclusive(u32 *data, u64 n, u32 *part, hipStream_t s, const u32 *gate = nullptr,
                    const u32 *n_dev = nullptr);
void scan_exclusive_multi(u32 *data, u64 n, u32 regions, u32 *part, hipStream_t s);

// several fills in one launch
constexpr u32 MAX_FILL_JOBS = 10;
struct FillJob {
    void *p;
    const u32 *dyn_n;  // non-null: fill min(*dyn_n, n) entries (read on the device)
    u64 n, v;
    u32 esize;         // 1, 4 or 8 bytes
    u32 mode_mask;     // non-zero: only when DevParams::mode has one of these bits
    u32 eng;           // 1: only when the parallel knowledge engine is on; 2: only when it is not
};
struct FillJobs {
    FillJob j[MAX_FILL_JOBS];
    const DevParams *P;
    u32 count;
    void add(void *p, u64 n, u64 v, u32 esize, u32 mode_mask = 0, const u32 *dyn_n = nullptr, u32 eng = 0);
};
void fill_many(const FillJobs &jobs, const char *name, hipStream_t s);

void prep_init(const Bufs &b, u32 *rt_scan, hipStream_t s);
void prep_ingest(const Bufs &b, u64 *sync_mask, u64 *acc_mask, u64 *atom_mask, hipStream_t s);
void prep_sync_lists(const Bufs &b, const u64 *sync_mask, const u64 *atom_mask, hipStream_t s);
void prep_elements(const Bufs &b, const u64 *acc_mask, hipStream_t s);
void prep_thread_sync(const Bufs &b, u32 *rt_scan, hipStream_t s);
void prep_validate_wbar(const Bufs &b, hipStream_t s);

// knowledge vectors (releases, acquires, warp barriers)
void interp_run(const Bufs &b, const u32 *rt_scan, hipStream_t s);

// radix sort of the access elements by location key; the sorted elements end in buffer
// (passes % 2), passes = ceil(key_bits / 8) read on the device
void sort_elements(const Bufs &b, hipStream_t s);
// radix sort of the kept race pairs by (first, second), result in buffer 0; the count is *m_dev
// (launches sized for max_m) or m_host
void sort_pairs(const Bufs &b, const u32 *m_dev, u32 m_host, u64 max_m, hipStream_t s);
// The same sort over any two word arrays (ping-pong pairs f, s2), `half` 8-bit digits per word.
void sort_pairs_in(const Bufs &b, u32 *const f[2], u32 *const s2[2], const u32 *m_dev, u32 m_host, u64 max_m,
                   u32 half, const char *const names[3], hipStream_t s);
// Race kinds of the packed report (b.preport, m pairs): sorted unique (site_lo, site_hi, count)
// records in `rec` (3 words each) and their number in *n_out (device).  `scratch` holds
// 5 * m + 1 words plus ceil((m + 1) / 4096) + 16 scan partials.
void race_kinds(const Bufs &b, u32 m, u32 *scratch, u32 *rec, u32 *n_out, hipStream_t s);
// The sorted pairs (buffer 0) as (first, second) records in b.preport, *n_pairs_kept of them.
void pack_pairs(const Bufs &b, hipStream_t s);
// stable sort of (key, value) pairs by key (see rd_sort.hip)
void sort_kv(const Bufs &b, u32 *const k[2], u32 *const v[2], const u32 *n_dev, u64 max_n, u32 passes,
             const u32 *bits_dev, const char *name, hipStream_t s);
// parallel knowledge engine (traces without warp barriers); sets DevParams::eng
hipError_t engine_run(const Bufs &b, const u32 *rt_scan, hipStream_t s);

void segcheck_run(const Bufs &b, const u32 *rt_scan, hipStream_t s);

// The pair sort and the packing into (first, second) records over any buffers (count *m_dev, at
// most max_m); the sorted pairs end in f[0], s2[0].
void sort_pairs_to(const Bufs &b, u32 *const f[2], u32 *const s2[2], const u32 *m_dev, u64 max_m, hipStream_t s);
void pack_pairs_to(const u32 *first, const u32 *second, const u32 *m_dev, u64 max_m, u64 *out, hipStream_t s);

// lockset pass (rd_lockset.hip), after a check, in the knowledge-vector pool
struct LocksetBufs {
    u32 *pf[2], *ps[2];  // pair ping-pong buffers, `cap` each
    u64 *report;         // sorted pairs as (first, second) records, `cap`
    u32 *rows;           // lockset rows
    u32 row_cap;
    u64 cap;
};
bool lockset_layout(const Bufs &b, u64 cap, LocksetBufs &L);
void lockset_run(const Bufs &b, const LocksetBufs &L, hipStream_t s);

// GWCP pass (rd_gwcp.hip), after a check, in the knowledge-vector pool and the engine's per-entry
// scratch; dense clocks: at most GW_MAX_T threads
constexpr u32 GW_MAX_T = 4096;
struct GwcpBufs {
    u32 *pf[2], *ps[2];  // pair ping-pong buffers, `cap` each
    u64 *report;         // sorted pairs as (first, second) records, `cap`
    u64 cap;
    u32 *hdr;            // counters
    u32 *heap;           // clocks and tables (carved on the device)
    u64 heap_words;
    u32 *n_after, *depth, *snap;  // [sync entries] local time, sections open, copy of P after it
    u32 *evsnap, *evchk;          // [events at which P can change] copy of P after it, seen by its check
    u32 *barsnap;                 // [barrier instances] copy of P the instance leaves
};
bool gwcp_layout(const Bufs &b, u64 cap, GwcpBufs &G);
void gwcp_run(const Bufs &b, const GwcpBufs &G, hipStream_t s);

// batched form: merged trace from the members' events; each member's run of the merged report
void batch_merge(BatchTrace *tr, const u32 *off, u32 n_traces, u32 N, u32 tpb_merged, uint4 *out, u32 *bad,
                 hipStream_t s);
void batch_pair_ranges(BatchTrace *tr, const u32 *off, u32 n_traces, const Bufs &b, hipStream_t s);
}  // namespace rd
