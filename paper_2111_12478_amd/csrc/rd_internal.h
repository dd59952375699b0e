// rd_internal.h -- shared definitions of the gfx950 race checker (device state, workspace layout,
// wavefront helpers, kernel launchers).  Not part of the public interface (include/rd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd.h"

namespace rd {

typedef uint32_t u32;
typedef uint64_t u64;

constexpr u32 NONE = 0xffffffffu;

// Tiles: a workgroup of WG_THREADS threads (4 wavefronts of 64) owns TILE consecutive items; wave w
// of the workgroup owns the contiguous range [w*ITEMS*64, (w+1)*ITEMS*64) of the tile and walks it
// in ITEMS steps of 64 consecutive items, so "wave, step, lane" is the input order.
constexpr int WG_THREADS = 256;
constexpr int WAVES = WG_THREADS / 64;
constexpr int ITEMS = 16;
constexpr int TILE = WG_THREADS * ITEMS;  // 4096
constexpr int TILE_STATS = 16;            // per-tile ingest statistics (words)

// element categories (conflict classes of an access)
enum { CAT_R = 0, CAT_W = 1, CAT_AD = 2, CAT_AB = 3 };  // read, write, device/system atomic, block atomic

// element info word: category in bits 0-1, phase (block barriers passed) in bits 2-31
__host__ __device__ inline u32 info_make(u32 cat, u32 phase) { return cat | (phase << 2); }
__host__ __device__ inline u32 info_cat(u32 info) { return info & 3u; }
__host__ __device__ inline u32 info_phase(u32 info) { return info >> 2; }

// Packed elements: when the location key, the category and the largest phase fit in 32 bits
// together, an element's key word holds key | category << key_bits | phase << (key_bits + 2) and
// its info array is not written (the location sort then moves three arrays instead of four).
__host__ __device__ inline u32 bits_of(u32 x) {
    u32 n = 0;
    while (n < 32 && (x >> n)) n++;
    return n;
}
__host__ __device__ inline u32 key_mask(u32 key_bits) { return key_bits >= 32 ? ~0u : (1u << key_bits) - 1u; }
__host__ __device__ inline bool packed_elements(u32 key_bits, u32 max_phase) {
    return key_bits + 2 + bits_of(max_phase) <= 32;
}
__host__ __device__ inline u32 pack_element(u32 key, u32 key_bits, u32 cat, u32 phase) {
    return key | (cat << key_bits) | (key_bits + 2 >= 32 ? 0u : phase << (key_bits + 2));
}
__host__ __device__ inline u32 packed_info(u32 word, u32 key_bits) {
    return info_make((word >> key_bits) & 3u, key_bits + 2 >= 32 ? 0u : word >> (key_bits + 2));
}
// Otherwise, when the thread id, the category and the largest phase fit in 32 bits together, the
// thread word holds tid | category << tid_bits | phase << (tid_bits + 2) and the info array is not
// written either (three arrays move in the sort).
__host__ __device__ inline u32 tid_bits(u32 T) { return T > 1 ? bits_of(T - 1) : 1u; }
__host__ __device__ inline bool tinfo_elements(u32 key_bits, u32 max_phase, u32 T) {
    return !packed_elements(key_bits, max_phase) && tid_bits(T) + 2 + bits_of(max_phase) <= 32;
}
__host__ __device__ inline u32 tinfo_word(u32 tid, u32 tb, u32 cat, u32 phase) {
    return tid | (cat << tb) | (tb + 2 >= 32 ? 0u : phase << (tb + 2));
}

// sync-entry flags (per entry of the per-thread sync lists)
enum : uint8_t {
    SF_REL = 1,       // release (explicit, or an atomic right after a fence)
    SF_ACQ = 2,       // acquire (explicit, or an atomic right before a fence)
    SF_BAD_ARRIVAL = 4,  // warp-barrier arrival with a bad mask
    SF_NOMAT = 8,     // acquire whose knowledge only its thread's next barrier reads (no access or
                      // other sync entry but fences in between): a barrier evaluated after it may
                      // join the acquire's inputs instead of its vector
};

// error flags (DevParams::err)
enum : u32 {
    ERR_POOL = 1,       // knowledge-vector pool exhausted
    ERR_KEYSPAN = 2,    // address span does not fit a 32-bit location key
    ERR_PAIRS = 4,      // internal pair buffer overflowed
    ERR_TABLE = 8,      // sync-variable or warp-barrier table overflowed
    ERR_PHASE = 16,     // a thread passed more than 2^30 barriers
    ERR_SORT = 32,      // a radix-sort look-back wait hit its spin limit
    ERR_ENGINE = 64,    // a grid barrier of the knowledge engine hit its spin limit
    ERR_LOCKSET = 128,  // lockset pass: a thread held more than LS_MAX locks, or the row table is full
    ERR_LSPAIRS = 256,  // lockset pass: more pairs than its buffer holds
    ERR_RESPEC = 512,   // the trace needs a stage the launched pass was built without (SPEC_*)
    ERR_GWCP = 1024,    // GWCP pass: a thread held more than 64 locks, or its clocks exceed the pool
    ERR_GWPAIRS = 2048, // GWCP pass: more pairs than its buffer holds
};

// Stages a pass can be built without (Bufs::spec), for the kinds of trace its last check saw; the
// plan flags ERR_RESPEC when the trace needs one of them, and the check is then run again whole.
enum : u32 {
    SPEC_NO_SYNC = 1,  // no releases, acquires or warp barriers: no knowledge vectors
    SPEC_NO_WBAR = 2,  // no warp barriers
};

// Radix sort: the pair and key-value sorts use 8-bit digits (at most 8 passes: two 32-bit halves);
// the location sort uses 7-, 8- or 9-bit digits (a tuning choice), at most ELEM_MAX_PASSES passes.
constexpr u32 SORT_RB = 8, SORT_ND = 1u << SORT_RB;
constexpr u32 SORT_NDS = 512;        // digit stride of the count rows and totals (9-bit digits)
constexpr u32 MAX_SORT_PASSES = 8;
constexpr u32 ELEM_MAX_PASSES = 5;   // ceil(32 / 7)
// the largest location-sort tile (16 wavefronts x 16 items): the element arrays are padded to a
// whole number of such tiles, so the sort loads full tiles without a bounds test
constexpr u32 SORT_MAX_TILE = 16384;
// Digit counts: every tile writes one row of partial counts ([pass][digit], ELEM_MAX_PASSES passes
// for the location sort, MAX_SORT_PASSES for the pair sort); a reduction adds the rows into
// per-pass totals.

// Location-sort variants (the tuner picks one per context): digit bits, wavefronts per
// workgroup, items per lane.
struct SortVariant {
    u32 rb, waves, items;
};
constexpr u32 N_SORT_VARIANTS = 11;
constexpr SortVariant kSortVariants[N_SORT_VARIANTS] = {
    {8, 4, 16}, {8, 8, 8}, {8, 8, 16}, {7, 4, 16}, {7, 8, 16}, {9, 8, 16},
    {9, 8, 8},  {8, 4, 8}, {7, 8, 8},  {7, 16, 16}, {8, 16, 16}};

// Device-side state of one check.  Zeroed (and the "min" fields set to NONE) by k_init.
struct DevParams {
    u32 first_bad_record;  // smallest index breaking a record rule
    u32 first_bad_sync;    // smallest index breaking a barrier rule
    u32 err;
    u32 n_sync;            // events in the sync lists (everything but plain reads and writes)
    u32 kind_count[8];
    u32 gmin, gmax, smin, smax;  // address ranges of global / shared accesses
    u32 n_acc;             // accesses (= elements)
    u32 key_bits;          // significant bits of the location key
    u32 g_span, s_span;    // key = addr - gmin (global) | g_span + block * s_span + addr - smin
    u32 gbase, sbase;      // gmin, smin used for keys
    u32 mode;              // MODE_* bits
    u32 n_rt;              // threads with a column in knowledge vectors (releasers, warp-barrier lanes)
    u32 D;                 // knowledge vector width = n_blocks + n_rt
    u32 pool_next;         // next free knowledge vector (0 is the empty vector)
    u32 pool_cap;          // vectors in the pool
    u32 n_pairs;           // pairs found (may exceed the buffer)
    u32 n_pairs_kept;      // min(n_pairs, capacity)
    u32 n_winst;           // warp-barrier instances
    u32 eng;               // ENG_* bits: which knowledge engine runs
    u32 n_ral;             // release/acquire accesses (engine)
    u32 n_bl;              // block-scoped ones among them
    u32 n_ops;             // engine operations
    u32 n_handles;         // knowledge vectors the engine writes (+1 for the empty one)
    u32 n_groups;          // dependency-free groups of operations
    u32 gbar;              // grid-barrier arrivals of the engine kernel
    u32 gprog;             // progress of the engine's sequential phases (bounds barrier waits)
    u32 wlist;             // entries of the engine's window input list
    u32 max_phase;         // the largest barrier phase of any thread
    u32 ls_pairs;          // lockset pass: pairs found (may exceed its buffer)
    u32 ls_kept;           // ... min(ls_pairs, its buffer)
    u32 gw_pairs;          // GWCP pass: pairs found (may exceed its buffer)
    u32 gw_kept;           // ... min(gw_pairs, its buffer)
    u32 n_long;            // slow-path accesses of the segment check queued whole (chunk queue full)
    unsigned long long n_chunks;  // queued slow-path chunks of the segment check (8-byte aligned)
};

// Errors after which later stages must not read what the failed stage should have written (sorted
// elements, operation tables, knowledge handles): the check's answer is the error, so they skip.
constexpr u32 ERR_ABANDON = ERR_POOL | ERR_TABLE | ERR_SORT | ERR_ENGINE | ERR_RESPEC;
__host__ __device__ inline bool check_abandoned(const DevParams *P) { return (P->err & ERR_ABANDON) != 0; }

// The engine evaluates runs of small dependent groups in windows of ENG_WIN operations; each
// operation of a window has ENG_JOB_WORDS words of job description.
constexpr u32 ENG_WIN = 4096;
constexpr u32 ENG_JOB_WORDS = 16;

// knowledge engine selection (DevParams::eng)
enum : u32 {
    ENG_PARALLEL = 1,  // the parallel engine computes the knowledge vectors
    ENG_FALLBACK = 2,  // too large for its buffers: the sequential interpreter does
};

enum : u32 {
    MODE_BAR = 1,    // block barriers present
    MODE_SYNC = 2,   // releases/acquires/warp barriers possible: knowledge vectors needed
    MODE_WBAR = 4,
};

// Device buffers of one trace (carved out of the caller's workspace).
struct Bufs {
    const uint4 *ev;        // events
    DevParams *prm;
    uint8_t *act;           // [T] thread has >= 1 event
    u32 *s_cnt;             // [T+1] sync entries per thread -> exclusive offsets
    u32 *s_fill;            // [T]
    u32 *a_cnt;             // [T] atomics per thread
    u32 *tile_s;            // [n_tiles+1] sync events per ingest tile -> offsets
    u32 *tile_stats;        // [n_tiles * TILE_STATS] ingest statistics per tile
    u32 *s_tidx;            // [N] sync events in trace order (event index)
    u32 *s_pidx;            // [N] per-thread sync lists (event index), trace order inside a thread
    u32 *s_pq;              // [N] trace-order position of each list entry
    u32 *s_inv;             // [N] list position of each trace-order sync event
    u32 *s_phase;           // [N] barriers passed up to and including the entry
    uint8_t *s_kind;        // [N]
    uint8_t *s_flags;       // [N]
    uint8_t *s_scope;       // [N] release scope (bits 0-1), acquire scope (bits 2-3)
    u32 *s_imin;            // [N] smallest access index between the entry and the thread's next entry
    u32 *s_know;            // [N] knowledge vector after the entry
    u32 *s_khandle;         // [N] knowledge vector created at the entry (interpreter output)
    u32 *s_winst;           // [N] warp-barrier instance of the entry
    // parallel knowledge engine (per sync entry p)
    u32 *e_prev0, *e_prev1; // release: previous release of its chains (entry ids)
    u32 *e_src0, *e_src1;   // acquire: latest release of the chains it reads; barrier: contribution
    u32 *e_cur;             // knowledge before the entry: acquire entry id, or BK_MARK | phase
    u32 *e_relh;            // first knowledge vector a release writes
    u32 *e_op;              // operation index of the entry
    u32 *e_scan0, *e_scan1; // [N+1] scan scratch
    u32 *inst_opo;          // [N] barrier instance -> operation index (or NONE)
    u32 *inst_bko;          // [N] operation that wrote the block knowledge after the instance
    u32 *inst_coff;         // [N+1] contributions per instance -> offsets
    u32 *eng_jobs;          // [ENG_WIN * ENG_JOB_WORDS + ENG_WIN] window job table and list (engine)
    u32 *ral_p, *ral_key;   // [ECAP] release/acquire accesses in (location, trace) order
    u32 *op_p;              // [ECAP] operation -> entry
    u32 *op_dep;            // [ECAP] largest operation index it depends on (NONE: none)
    u32 *grp;               // [ECAP+1] group starts
    u32 ecap;
    u32 *blk_maxbar;        // [B]
    u32 *inst_off;          // [B+1]
    u32 *inst_cnt;          // [N]
    u32 *inst_last;         // [N]
    u32 *inst_handle;       // [N]
    u32 *n_active;          // [B]
    u32 *rt;                // [T] knowledge column of a thread, or NONE
    u32 *priv;              // [T] private knowledge vector of a thread (since its last barrier)
    u32 *priv_next;         // [T]
    u32 *t_kfirst;          // [T] trace index of the thread's first sync entry with knowledge (NONE: none)
    u32 *t_acq;             // [T] 1 when the thread has an acquire that joins knowledge of its own
    u32 *bk;                // [B] knowledge vector of a block after its latest barrier
    u32 *priv_head;         // [B]
    // sync-variable table (open addressing)
    u64 *sv_key;            // [SV] location key | tag
    u32 *sv_tag;            // [SV]
    u32 *sv_handle;         // [SV]
    u32 sv_cap;
    // warp-barrier tables
    u64 *wo_key;            // [WO] (tid, id) -> occurrences so far
    u32 *wo_val;
    u32 wo_cap;
    u64 *wi_key;            // [WO] (warp lane-0 tid, id) hashed with occurrence -> instance
    u32 *wi_occ;
    u32 *wi_inst;
    u32 *winst_mask, *winst_arrived, *winst_last, *winst_nar;  // [WO]
    u32 *winst_arr;         // [WO*32] arrival list entries
    u32 *pool;              // knowledge vectors
    u64 pool_words;
    // elements (ping-pong)
    u32 *ekey[2], *eidx[2], *etid[2], *einfo[2];
    // radix sort
    u64 *sort_status;       // [2][words] look-back words (flag << 62 | count), [tile][digits of the variant]
    u64 sort_status_stride; // words per array
    u32 *sort_partial;      // [tiles][passes][SORT_ND] per-tile digit counts
    u32 *sort_tot;          // [MAX_SORT_PASSES][SORT_NDS] digit totals of each pass
    u32 *sort_ctr;          // [MAX_SORT_PASSES] tile tickets of each pass
    u32 *part;              // [scan partials]
    // segment check
    void *tile_agg;         // [n_tiles] aggregates -> exclusive prefixes
    // pairs (ping-pong)
    u32 *pfirst[2], *psecond[2];
    u64 *preport;           // [max_pairs] the sorted report as (first, second) records (over buffer 1)
    u64 max_pairs;
    // shape
    u32 N, T, B, tpb, ws;
    u32 div_m, div_s1, div_s2;  // tid / tpb as a multiply-high and shifts
    u32 n_tiles;            // ceil(N / TILE)
    u32 radix_bits;         // digit width of the location sort (its variant's)
    u32 sort_variant;       // index into kSortVariants
    u32 sorted_buf;         // which element buffer holds the sorted elements (set by the host plan)
    u32 pair_buf;
    u32 spec;               // SPEC_* stages this pass is built without
};

// One member of a batched check (device table): where its events are, its grid and its place in
// the merged trace; the global-word range and pair run are filled in on the device.
struct BatchTrace {
    const uint4 *ev;
    u32 n, n_blocks, tpb, blk_off;
    u32 gmin, gmax, goff;   // global words of its accesses: [gmin, gmax] -> [goff, goff + span)
    u32 pair_lo, pair_hi;   // its run in the merged, sorted report
};

// ---------------------------------------------------------------- wavefront helpers (wave64)

__device__ inline u32 lane_id() { return __lane_id(); }
__device__ inline u64 lanemask_lt() { return (u64(1) << lane_id()) - 1; }
__device__ inline u64 ballot(bool p) { return __ballot(p); }
__device__ inline u32 popc64(u64 x) { return (u32)__popcll(x); }

// Block of a thread: tid / tpb by multiplication (division by an invariant integer: with
// l = ceil(log2 tpb) and m = floor(2^32 (2^l - tpb) / tpb) + 1, q = (t1 + ((n - t1) >> s1)) >> s2
// where t1 = mulhi(m, n), s1 = min(l, 1), s2 = max(l - 1, 0); exact for every 32-bit n).
__device__ inline u32 block_of(const Bufs &b, u32 tid) {
    const u32 t1 = __umulhi(b.div_m, tid);
    return (t1 + ((tid - t1) >> b.div_s1)) >> b.div_s2;
}

// ---------------------------------------------------------------- host side

struct Layout {
    u64 total;
    u64 off_params, off_ev, off_act, off_s_cnt, off_s_fill, off_tile_s, off_s_tidx, off_s_pidx,
        off_s_pq, off_s_inv, off_s_phase, off_s_kind, off_s_flags, off_s_scope, off_s_imin,
        off_s_know, off_s_khandle, off_s_winst, off_e_prev0, off_e_prev1, off_e_src0, off_e_src1, off_e_cur,
        off_e_relh, off_e_op, off_e_scan0, off_e_scan1, off_inst_opo, off_inst_bko, off_inst_coff, off_eng_jobs, off_t_kfirst, off_t_acq,
        off_ral_p, off_ral_key, off_op_p, off_op_dep, off_grp, off_blk_maxbar, off_inst_off, off_inst_cnt,
        off_inst_last, off_inst_handle, off_n_active, off_rt, off_priv, off_priv_next, off_bk,
        off_priv_head, off_sv_key, off_sv_tag, off_sv_handle, off_wo_key, off_wo_val, off_wi_key,
        off_wi_occ, off_wi_inst, off_winst_mask, off_winst_arrived, off_winst_last, off_winst_nar,
        off_winst_arr, off_pool, off_ekey[2], off_eidx[2], off_etid[2], off_einfo[2], off_sort_status,
        off_sort_partial, off_sort_tot, off_part, off_tile_agg, off_pfirst[2], off_psecond[2];
    u32 sv_cap, wo_cap, pool_cap_bytes_hi, ecap;
    u64 pool_bytes, max_pairs;
};

size_t agg_bytes();

// Optional per-kernel timing: when a profiler is active on this host thread, every launch made
// through RD_LAUNCH whose name matches the profiler's filter is bracketed by two HIP events on the
// launch stream.
void prof_begin(const char *name, hipStream_t s);
void prof_end(hipStream_t s);
#define RD_LAUNCH(NAME, KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                       \
    do {                                                                               \
        ::rd::prof_begin(NAME, STREAM);                                                \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);            \
        ::rd::prof_end(STREAM);                                                        \
    } while (0)

}  // namespace rd

namespace rd {
// Last entry of thread t's sync list with event index < idx, or NONE.
__device__ inline u32 list_search(const Bufs &b, u32 t, u32 idx) {
    u32 lo = b.s_cnt[t], hi = b.s_cnt[t + 1];
    const u32 first = lo;
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (b.s_pidx[mid] < idx) lo = mid + 1;
        else hi = mid;
    }
    return lo == first ? NONE : lo - 1;
}

// The sorted elements after the location sort (and the sort's free buffers, the segment check's
// queue of slow-path chunks).
struct SegCtx {
    const u32 *k, *i, *t, *f;
    u32 *cpos, *clo, *chi;  // the queue of slow-path chunks (in the sort's free buffers)
    u32 *lpos;              // accesses queued whole when the chunk queue is full: sorted position,
                            // bit 31 set when only the access's block-and-phase run can race
    u32 n;
    bool packed;            // category and phase in the key word, above key_bits
    bool tinfo;             // category and phase in the thread word, above tbits
    u32 key_bits, kmask;
    u32 tbits, tmask;
};

__device__ inline SegCtx seg_ctx(const Bufs &b) {
    // the sort leaves the elements in buffer (passes % 2); passes = ceil(key_bits / radix_bits)
    const u32 bits = b.prm->key_bits, passes = (bits + b.radix_bits - 1) / b.radix_bits;
    const u32 c = passes & 1;
    SegCtx s; s.k = b.ekey[c]; s.i = b.eidx[c]; s.t = b.etid[c]; s.f = b.einfo[c]; s.n = b.prm->n_acc;
    s.cpos = b.ekey[c ^ 1]; s.clo = b.etid[c ^ 1]; s.chi = b.einfo[c ^ 1]; s.lpos = b.eidx[c ^ 1];
    s.packed = packed_elements(bits, b.prm->max_phase);
    s.tinfo = tinfo_elements(bits, b.prm->max_phase, b.T);
    s.key_bits = bits;
    s.kmask = s.packed ? key_mask(bits) : ~0u;
    s.tbits = tid_bits(b.T);
    s.tmask = s.tinfo ? key_mask(s.tbits) : ~0u;
    return s;
}

// the location key and the info (category | phase) of sorted element p
__device__ inline u32 seg_key(const SegCtx &s, u64 p) { return s.k[p] & s.kmask; }
__device__ inline u32 seg_info(const SegCtx &s, u64 p) {
    return s.packed ? packed_info(s.k[p], s.key_bits) : s.tinfo ? packed_info(s.t[p], s.tbits) : s.f[p];
}
// the thread of sorted element p
__device__ inline u32 seg_tid(const SegCtx &s, u64 p) { return s.t[p] & s.tmask; }

// The knowledge handle of thread t at its access with trace index idx and barrier phase ph (block
// blk), 0 for none.  A thread without acquires of its own knows, after its k-th barrier, what its
// block knows after that barrier instance (no search); others search their sync list.
__device__ inline u32 knowledge_at(const Bufs &b, u32 t, u32 idx, u32 blk, u32 ph) {
    if (!b.t_acq[t]) return ph ? b.inst_handle[b.inst_off[blk] + ph - 1] : 0u;
    const u32 j = list_search(b, t, idx);
    return j == NONE ? 0u : b.s_know[j];
}
}  // namespace rd
