// rd_host.hip -- workspace layout, pipeline orchestration and the C interface of include/rd.h.
#include <algorithm>
#include <memory>
#include <mutex>
#include <new>
#include <string.h>
#include <string>
#include <vector>

#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

static u64 align_up(u64 x, u64 a) { return (x + a - 1) / a * a; }
static u32 next_pow2(u64 x) {
    u64 p = 1;
    while (p < x) p <<= 1;
    return (u32)p;
}

struct Plan {
    Layout L;
    u64 off_masks, off_rt_scan, off_tile_stats, off_a_cnt;
    u64 off_kinds;  // rd_race_kinds' scratch, over memory the check no longer needs when it ends
    u32 n_tiles, T, B, radix_bits, pair_tiles, part_words;
    u64 partial_words, status_words;
};

static Plan make_plan(u64 n, u32 nb, u32 tpb, const rd_limits *lim, bool copy_events, bool kinds = true) {
    Plan P;
    memset(&P, 0, sizeof(P));
    Layout &L = P.L;
    const u64 T = (u64)nb * tpb, B = nb;
    const u32 n_tiles = (u32)((n + TILE - 1) / TILE);
    u64 max_pairs = lim && lim->max_pairs ? lim->max_pairs : (n / 4 > (1u << 20) ? n / 4 : (1u << 20));
    if (max_pairs > 0xfffffff0ull) max_pairs = 0xfffffff0ull;
    const u64 pool_bytes = lim && lim->clock_bytes ? lim->clock_bytes : (256ull << 20);
    const u64 N1 = n ? n : 1;
    P.n_tiles = n_tiles; P.T = (u32)T; P.B = nb; P.radix_bits = SORT_RB;
    P.pair_tiles = (u32)((max_pairs + TILE - 1) / TILE);
    const u64 ecap = N1 / 4 > (1u << 20) ? N1 / 4 : (N1 < (1u << 20) ? N1 : (1u << 20));
    {
        // look-back words per array: the largest tiles x digits over the sort variants, the pairs and
        // the knowledge engine's sort of its release/acquire list (at most ecap items)
        const u64 small_tiles = (P.pair_tiles > (ecap + TILE - 1) / TILE ? P.pair_tiles : (ecap + TILE - 1) / TILE);
        u64 w = small_tiles * SORT_ND;
        for (u32 v = 0; v < N_SORT_VARIANTS; v++) {
            const u64 ts = (u64)kSortVariants[v].waves * 64 * kSortVariants[v].items;
            const u64 x = ((N1 + ts - 1) / ts) << kSortVariants[v].rb;
            if (x > w) w = x;
        }
        P.status_words = w;
        const u64 e = (u64)n_tiles * ELEM_MAX_PASSES, q = small_tiles * MAX_SORT_PASSES;
        P.partial_words = (e > q ? e : q) * SORT_NDS;
    }
    u64 scan_max = N1 + 1;  // the knowledge engine scans per sync entry
    if (T + 1 > scan_max) scan_max = T + 1;
    if (B + 1 > scan_max) scan_max = B + 1;
    P.part_words = (u32)((scan_max + 4095) / 4096 + 16);
    L.sv_cap = next_pow2(2 * N1 < (1u << 22) ? 2 * N1 + 64 : (1u << 22));
    L.wo_cap = next_pow2(N1 / 4 < (1u << 18) ? N1 / 4 + 64 : (1u << 18));
    L.pool_bytes = pool_bytes;
    L.max_pairs = max_pairs;

    u64 o = 0;
    auto take = [&](u64 bytes) { const u64 r = o; o = align_up(o + (bytes ? bytes : 4), 256); return r; };
    L.off_params = take(sizeof(DevParams));
    L.off_ev = copy_events ? take(16 * N1) : 0;
    L.off_act = take(T);
    L.off_s_cnt = take(4 * (T + 1));
    L.off_s_fill = take(4 * T);
    L.off_tile_s = take(4 * 3 * ((u64)n_tiles + 1));
    P.off_a_cnt = take(4 * T);
    P.off_tile_stats = take(4ull * TILE_STATS * ((u64)n_tiles + 1));
    P.off_masks = take(8 * 3 * (u64)n_tiles * 64);
    L.off_s_tidx = take(4 * N1);
    L.off_s_pidx = take(4 * N1);
    L.off_s_pq = take(4 * N1);
    L.off_s_inv = take(4 * N1);
    L.off_s_phase = take(4 * N1);
    L.off_s_kind = take(N1);
    L.off_s_flags = take(N1);
    L.off_s_scope = take(N1);
    L.off_s_imin = take(4 * N1);
    L.off_s_know = take(4 * N1);
    L.off_s_khandle = take(4 * N1);
    L.off_s_winst = take(4 * N1);
    L.ecap = (u32)ecap;
    L.off_e_prev0 = take(4 * N1);
    L.off_e_prev1 = take(4 * N1);
    L.off_e_src0 = take(4 * N1);
    L.off_e_src1 = take(4 * N1);
    L.off_e_cur = take(4 * N1);
    L.off_e_relh = take(4 * N1);
    L.off_e_op = take(4 * N1);
    L.off_e_scan0 = take(4 * (N1 + 1));
    L.off_e_scan1 = take(4 * (N1 + 1));
    L.off_inst_opo = take(4 * N1);
    L.off_inst_bko = take(4 * N1);
    L.off_inst_coff = take(4 * (N1 + 1));
    L.off_eng_jobs = take(4ull * ENG_WIN * (ENG_JOB_WORDS + 1));
    L.off_ral_p = take(4ull * L.ecap);
    L.off_ral_key = take(4ull * L.ecap);
    L.off_op_p = take(4ull * L.ecap);
    L.off_op_dep = take(4ull * L.ecap);
    L.off_grp = take(4ull * (L.ecap + 1));
    L.off_blk_maxbar = take(4 * (B + 1));
    L.off_inst_cnt = take(4 * N1);
    L.off_inst_last = take(4 * N1);
    L.off_inst_handle = take(4 * N1);
    L.off_n_active = take(4 * B);
    P.off_rt_scan = take(4 * (T + 1));
    L.off_priv = take(4 * T);
    L.off_priv_next = take(4 * T);
    L.off_t_kfirst = take(4 * T);
    L.off_t_acq = take(4 * T);
    L.off_bk = take(4 * B);
    L.off_priv_head = take(4 * B);
    L.off_sv_key = take(8ull * L.sv_cap);
    L.off_sv_tag = take(4ull * L.sv_cap);
    L.off_sv_handle = take(4ull * L.sv_cap);
    L.off_wo_key = take(8ull * L.wo_cap);
    L.off_wo_val = take(4ull * L.wo_cap);
    L.off_wi_key = take(8ull * L.wo_cap);
    L.off_wi_occ = take(4ull * L.wo_cap);
    L.off_wi_inst = take(4ull * L.wo_cap);
    L.off_winst_mask = take(4ull * L.wo_cap);
    L.off_winst_arrived = take(4ull * L.wo_cap);
    L.off_winst_last = take(4ull * L.wo_cap);
    L.off_winst_nar = take(4ull * L.wo_cap);
    L.off_winst_arr = take(4ull * 32 * L.wo_cap);
    L.off_pool = take(pool_bytes);
    const u64 NE = (N1 + SORT_MAX_TILE - 1) / SORT_MAX_TILE * SORT_MAX_TILE;
    for (int c = 0; c < 2; c++) {
        L.off_ekey[c] = take(4 * NE);
        L.off_eidx[c] = take(4 * NE);
        L.off_etid[c] = take(4 * NE);
        L.off_einfo[c] = take(4 * NE);
    }
    // rd_race_kinds (after a check) needs 8 words per race pair plus scan partials: the knowledge
    // pool when it is large enough, else the element buffers, extended when they are too small
    // (neither is read once the check has ended)
    {
        const u64 kparts = (max_pairs + 1 + 4095) / 4096 + 16;
        const u64 kbytes = 4 * (8 * max_pairs + kparts + 2);
        if (!kinds) {
            P.off_kinds = 0;  // a workspace that rd_race_kinds never uses
        } else if (pool_bytes >= kbytes) {
            P.off_kinds = L.off_pool;
        } else {
            P.off_kinds = L.off_ekey[0];
            const u64 have = o - L.off_ekey[0];
            if (kbytes > have) take(kbytes - have);
        }
    }
    L.off_sort_status = take(2 * 8ull * P.status_words);
    L.off_sort_partial = take(4ull * P.partial_words);
    L.off_sort_tot = take(4ull * (MAX_SORT_PASSES * SORT_NDS + MAX_SORT_PASSES));
    L.off_part = take(4ull * P.part_words);
    // the tile summaries, then the chunk totals of their scan (4,096 tiles a chunk)
    L.off_tile_agg = take(agg_bytes() * ((u64)n_tiles + 1 + ((u64)n_tiles + 4095) / 4096 + 1));
    L.off_pfirst[0] = take(4 * max_pairs);
    L.off_psecond[0] = take(4 * max_pairs);
    // the second pair buffer is one block: after the sort it holds the report as rd_pair records
    L.off_pfirst[1] = take(8 * max_pairs);
    L.off_psecond[1] = L.off_pfirst[1] + 4 * max_pairs;
    L.total = o;
    return P;
}

static Bufs make_bufs(const Plan &P, char *ws, const void *events_dev, u64 n, u32 nb, u32 tpb, u32 warp_size) {
    const Layout &L = P.L;
    Bufs b;
    memset(&b, 0, sizeof(b));
    b.ev = (const uint4 *)(events_dev ? events_dev : ws + L.off_ev);
    b.prm = (DevParams *)(ws + L.off_params);
    b.act = (uint8_t *)(ws + L.off_act);
    b.s_cnt = (u32 *)(ws + L.off_s_cnt);
    b.s_fill = (u32 *)(ws + L.off_s_fill);
    b.a_cnt = (u32 *)(ws + P.off_a_cnt);
    b.tile_s = (u32 *)(ws + L.off_tile_s);
    b.tile_stats = (u32 *)(ws + P.off_tile_stats);
    b.s_tidx = (u32 *)(ws + L.off_s_tidx);
    b.s_pidx = (u32 *)(ws + L.off_s_pidx);
    b.s_pq = (u32 *)(ws + L.off_s_pq);
    b.s_inv = (u32 *)(ws + L.off_s_inv);
    b.s_phase = (u32 *)(ws + L.off_s_phase);
    b.s_kind = (uint8_t *)(ws + L.off_s_kind);
    b.s_flags = (uint8_t *)(ws + L.off_s_flags);
    b.s_scope = (uint8_t *)(ws + L.off_s_scope);
    b.s_imin = (u32 *)(ws + L.off_s_imin);
    b.s_know = (u32 *)(ws + L.off_s_know);
    b.s_khandle = (u32 *)(ws + L.off_s_khandle);
    b.s_winst = (u32 *)(ws + L.off_s_winst);
    b.e_prev0 = (u32 *)(ws + L.off_e_prev0);
    b.e_prev1 = (u32 *)(ws + L.off_e_prev1);
    b.e_src0 = (u32 *)(ws + L.off_e_src0);
    b.e_src1 = (u32 *)(ws + L.off_e_src1);
    b.e_cur = (u32 *)(ws + L.off_e_cur);
    b.e_relh = (u32 *)(ws + L.off_e_relh);
    b.e_op = (u32 *)(ws + L.off_e_op);
    b.e_scan0 = (u32 *)(ws + L.off_e_scan0);
    b.e_scan1 = (u32 *)(ws + L.off_e_scan1);
    b.inst_opo = (u32 *)(ws + L.off_inst_opo);
    b.inst_bko = (u32 *)(ws + L.off_inst_bko);
    b.inst_coff = (u32 *)(ws + L.off_inst_coff);
    b.eng_jobs = (u32 *)(ws + L.off_eng_jobs);
    b.ral_p = (u32 *)(ws + L.off_ral_p);
    b.ral_key = (u32 *)(ws + L.off_ral_key);
    b.op_p = (u32 *)(ws + L.off_op_p);
    b.op_dep = (u32 *)(ws + L.off_op_dep);
    b.grp = (u32 *)(ws + L.off_grp);
    b.ecap = L.ecap;
    b.blk_maxbar = (u32 *)(ws + L.off_blk_maxbar);
    b.inst_off = b.blk_maxbar;  // scanned in place
    b.inst_cnt = (u32 *)(ws + L.off_inst_cnt);
    b.inst_last = (u32 *)(ws + L.off_inst_last);
    b.inst_handle = (u32 *)(ws + L.off_inst_handle);
    b.n_active = (u32 *)(ws + L.off_n_active);
    b.priv = (u32 *)(ws + L.off_priv);
    b.priv_next = (u32 *)(ws + L.off_priv_next);
    b.t_kfirst = (u32 *)(ws + L.off_t_kfirst);
    b.t_acq = (u32 *)(ws + L.off_t_acq);
    b.bk = (u32 *)(ws + L.off_bk);
    b.priv_head = (u32 *)(ws + L.off_priv_head);
    b.sv_key = (u64 *)(ws + L.off_sv_key);
    b.sv_tag = (u32 *)(ws + L.off_sv_tag);
    b.sv_handle = (u32 *)(ws + L.off_sv_handle);
    b.sv_cap = L.sv_cap;
    b.wo_key = (u64 *)(ws + L.off_wo_key);
    b.wo_val = (u32 *)(ws + L.off_wo_val);
    b.wo_cap = L.wo_cap;
    b.wi_key = (u64 *)(ws + L.off_wi_key);
    b.wi_occ = (u32 *)(ws + L.off_wi_occ);
    b.wi_inst = (u32 *)(ws + L.off_wi_inst);
    b.winst_mask = (u32 *)(ws + L.off_winst_mask);
    b.winst_arrived = (u32 *)(ws + L.off_winst_arrived);
    b.winst_last = (u32 *)(ws + L.off_winst_last);
    b.winst_nar = (u32 *)(ws + L.off_winst_nar);
    b.winst_arr = (u32 *)(ws + L.off_winst_arr);
    b.pool = (u32 *)(ws + L.off_pool);
    b.pool_words = L.pool_bytes / 4;
    for (int c = 0; c < 2; c++) {
        b.ekey[c] = (u32 *)(ws + L.off_ekey[c]);
        b.eidx[c] = (u32 *)(ws + L.off_eidx[c]);
        b.etid[c] = (u32 *)(ws + L.off_etid[c]);
        b.einfo[c] = (u32 *)(ws + L.off_einfo[c]);
        b.pfirst[c] = (u32 *)(ws + L.off_pfirst[c]);
        b.psecond[c] = (u32 *)(ws + L.off_psecond[c]);
    }
    b.preport = (u64 *)(ws + L.off_pfirst[1]);
    b.sort_status = (u64 *)(ws + L.off_sort_status);
    b.sort_status_stride = P.status_words;
    b.sort_partial = (u32 *)(ws + L.off_sort_partial);
    b.sort_tot = (u32 *)(ws + L.off_sort_tot);
    b.sort_ctr = b.sort_tot + MAX_SORT_PASSES * SORT_NDS;
    b.part = (u32 *)(ws + L.off_part);
    b.tile_agg = ws + L.off_tile_agg;
    b.max_pairs = L.max_pairs;
    b.N = (u32)n;
    b.T = nb * tpb;
    b.B = nb;
    b.tpb = tpb;
    b.ws = warp_size;
    b.n_tiles = P.n_tiles;
    b.radix_bits = P.radix_bits;
    b.sort_variant = 0;
    u32 l = 0;
    while (((u64)1 << l) < tpb) l++;
    b.div_m = (u32)((((u64)1 << 32) * (((u64)1 << l) - tpb)) / tpb + 1);
    b.div_s1 = l < 1 ? l : 1;
    b.div_s2 = l > 1 ? l - 1 : 0;
    return b;
}

// ---------------------------------------------------------------- per-kernel timing

struct ProfRec {
    const char *name;
    hipEvent_t a, b;
    uint32_t launches;  // kernels between the two events
};

// A piece of a captured check.  Without profiling the whole check is one piece; with it, each
// profiled kernel is a piece of its own (`name` set), so that a check brackets its launch with HIP
// events on the launch stream.
struct GraphSeg {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const char *name = nullptr;  // first profiled kernel of the piece
    uint32_t launches = 0;       // profiled kernels in it (consecutive launches share a piece)
};

struct Profiler {
    std::string filter;  // "" off, "*" every kernel, else one kernel name
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    const char *open_name = nullptr;
    hipEvent_t open_ev = nullptr;
    std::vector<GraphSeg> *capture = nullptr;  // during a capture: where the pieces go
    hipError_t cap_err = hipSuccess;
    const char *group_name = nullptr;  // during a capture: the open piece of profiled kernels
    uint32_t group_n = 0;
    struct Acc { const char *name; uint32_t launches; double total_ms; };
    std::vector<Acc> acc;  // collected times
    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void add(const char *name, double ms, uint32_t launches) {
        size_t k = 0;
        while (k < acc.size() && strcmp(acc[k].name, name) != 0) k++;
        if (k == acc.size()) acc.push_back({name, 0, 0.0});
        acc[k].launches += launches;
        acc[k].total_ms += ms;
    }
    // times of the records (waits for them)
    bool collect() {
        for (auto &r : recs) {
            if (hipEventSynchronize(r.b) != hipSuccess) return false;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return false;
            add(r.name, ms, r.launches);
        }
        recs.clear();
        used = 0;
        return true;
    }
    // during a capture: close the piece so far and open the next one (`name`, `n`: the profiled
    // kernels of the closed piece)
    void cut(hipStream_t s, const char *name, uint32_t n) {
        GraphSeg g;
        hipError_t e = hipStreamEndCapture(s, &g.graph);
        if (e == hipSuccess) {
            g.name = name;
            g.launches = n;
            capture->push_back(g);
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        }
        if (e != hipSuccess && cap_err == hipSuccess) cap_err = e;
    }
};
static thread_local Profiler *g_prof = nullptr;

void prof_begin(const char *name, hipStream_t s) {
    Profiler *p = g_prof;
    if (!p || p->filter.empty()) return;
    const std::string &f = p->filter;
    bool match;
    if (f.back() == '*') match = strncmp(name, f.c_str(), f.size() - 1) == 0;  // prefix ("*": every kernel)
    else match = f == name;
    if (p->capture) {
        // consecutive profiled kernels form one piece, bracketed by one pair of events at launch
        // (with "*", every kernel is a piece of its own)
        if (match && p->group_name && f == "*") {
            p->cut(s, p->group_name, p->group_n);
            p->group_name = nullptr;
        }
        if (match && !p->group_name) {
            p->cut(s, nullptr, 0);
            p->group_name = name;
            p->group_n = 0;
        } else if (!match && p->group_name) {
            p->cut(s, p->group_name, p->group_n);
            p->group_name = nullptr;
        }
        if (match) p->group_n++;
        return;
    }
    if (!match) return;
    hipEvent_t e = p->get();
    if (!e) return;
    (void)hipEventRecord(e, s);
    p->open_name = name;
    p->open_ev = e;
}
void prof_end(hipStream_t s) {
    Profiler *p = g_prof;
    if (!p || p->capture || !p->open_name) return;
    hipEvent_t e = p->get();
    if (e) {
        (void)hipEventRecord(e, s);
        p->recs.push_back({p->open_name, p->open_ev, e, 1u});
    }
    p->open_name = nullptr;
}

hipError_t enqueue_check(const Bufs &b, u64 *masks, u32 *rt_scan, hipStream_t s) {
    u64 *sync_mask = masks, *acc_mask = masks + (u64)b.n_tiles * 64, *atom_mask = masks + 2 * (u64)b.n_tiles * 64;
    prep_init(b, rt_scan, s);
    prep_ingest(b, sync_mask, acc_mask, atom_mask, s);
    prep_sync_lists(b, sync_mask, atom_mask, s);
    prep_elements(b, acc_mask, s);
    prep_thread_sync(b, rt_scan, s);
    sort_elements(b, s);
    if (!(b.spec & SPEC_NO_SYNC)) {
        const hipError_t e = engine_run(b, rt_scan, s);
        if (e != hipSuccess) return e;
        interp_run(b, rt_scan, s);
    }
    if (!(b.spec & (SPEC_NO_SYNC | SPEC_NO_WBAR))) prep_validate_wbar(b, s);
    segcheck_run(b, rt_scan, s);
    return hipGetLastError();
}

// A check of one trace with its report sorted on the device (count read on the device too), so the
// whole pass needs no host decision and can be captured.
hipError_t enqueue_plain(const Bufs &b, u64 *masks, u32 *rt_scan, hipStream_t s) {
    const hipError_t e = enqueue_check(b, masks, rt_scan, s);
    if (e != hipSuccess) return e;
    sort_pairs(b, &b.prm->n_pairs_kept, 0, b.max_pairs, s);
    pack_pairs(b, s);
    return hipGetLastError();
}

}  // namespace rd

// ================================================================ C interface

using namespace rd;

struct rd_ctx_s {
    int device;
    u32 sort_variant = 0;  // location-sort variant (rd_set_tuning / rd_autotune)
    std::mutex mu;
    uint64_t last_index;
    char last_msg[192];  // fixed: recording an error allocates nothing
    Profiler prof;
    hipStream_t cap_stream = nullptr;  // where checks are captured into graphs
};

// A batched check: the merged trace's workspace and the member table.  Shared by the member traces
// (each keeps its index); the first rd_races of a member reads the batch's state once.
struct Batch {
    Plan plan;
    Bufs bufs;
    char *ws;
    u64 *masks;
    u32 *rt_scan;
    BatchTrace *tr_dev;
    u32 *off_dev, *bad_dev;
    std::vector<BatchTrace> tr_init;  // uploaded table (never changes: a captured graph reads it again)
    std::vector<BatchTrace> tr_host;  // the table as read back after the pass
    std::vector<u32> off_host;
    u32 zero = 0;
    u64 ws_bytes;
    hipStream_t stream;
    std::mutex mu, ws_mu;  // ws_mu: members checked alone in this workspace, one at a time
    bool read = false, failed = false;
};

// Page-locked host memory a report is copied into by DMA (no staging by the runtime), then to the
// caller's buffer; grown on demand, released with its trace.
struct HostStage {
    char *p = nullptr;
    u64 bytes = 0;
    bool ensure(u64 n) {
        if (n <= bytes) return true;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        if (hipHostMalloc((void **)&p, n, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return false;
        }
        bytes = n;
        return true;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
};

struct rd_trace_s {
    Plan plan;
    Bufs bufs;
    char *ws;
    u64 *masks;
    u32 *rt_scan;
    hipStream_t stream;
    int checked;
    rd_grid grid;
    uint64_t n;
    std::shared_ptr<Batch> batch;  // set by rd_check_many until the next rd_check
    u32 batch_idx;
    rd_limits lim;
    // a member without a workspace of its own whose batch could not answer for it is checked alone
    // in the batch's workspace once; its report is kept here
    int cached;
    rd_status cache_st;
    uint64_t cache_idx, cache_n;
    std::string cache_msg;
    std::vector<rd_pair> cache;
    // the plain check captured into a graph (replayed by later checks of the same trace)
    std::vector<GraphSeg> segs;
    u32 graph_variant = 0;
    u32 graph_spec = 0;      // stages the captured pass is built without
    u32 last_mode = ~0u;     // the trace kinds (MODE_*) its last check found; all until one is read
    std::string graph_filter;
    bool graph_off = false;  // capture failed once: checks are enqueued kernel by kernel
    uint64_t n_checks = 0;
    u64 last_pairs = 0;  // the previous report's length: copied together with the check state
    HostStage stage;     // where rd_races copies the state and the report to
};

// A captured batched pass: replayed by rd_graph_launch for the same members and workspace.
struct rd_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::shared_ptr<Batch> batch;
    std::vector<rd_trace> traces;
};

// Shape of the merged trace of a batch; false when the members cannot be merged (different warp
// sizes, or more than 2^32 - 1 events or threads in all).
struct BatchShape {
    u64 N, B;
    u32 tpb, ws;
    rd_limits lim;
    u64 table_off, off_off, bad_off, total;
    Plan plan;
};
static bool batch_shape(const rd_trace *traces, uint32_t n, const rd_limits *limits, BatchShape &S) {
    S.N = 0;
    S.B = 0;
    S.tpb = 1;
    S.ws = 0;
    u64 pairs = 0;
    for (uint32_t j = 0; j < n; j++) {
        const rd_trace t = traces[j];
        const u32 ws = t->grid.warp_size ? t->grid.warp_size : 32;
        if (j == 0) S.ws = ws;
        else if (ws != S.ws) return false;
        S.N += t->n;
        S.B += t->grid.n_blocks;
        if (t->grid.threads_per_block > S.tpb) S.tpb = t->grid.threads_per_block;
        pairs += t->bufs.max_pairs;
    }
    if (S.N >= (1ull << 32) || S.B * S.tpb >= (1ull << 32)) return false;
    const u64 dflt = S.N / 4 > (1u << 20) ? S.N / 4 : (1u << 20);  // as for one trace of N events
    S.lim.max_pairs = limits && limits->max_pairs ? limits->max_pairs : (pairs < dflt ? pairs : dflt);
    S.lim.clock_bytes = limits && limits->clock_bytes ? limits->clock_bytes : 0;
    S.plan = make_plan(S.N, (u32)S.B, S.tpb, &S.lim, true);
    S.table_off = align_up(S.plan.L.total, 256);
    S.off_off = align_up(S.table_off + sizeof(BatchTrace) * (u64)n, 256);
    S.bad_off = align_up(S.off_off + 4ull * (n + 1), 256);
    S.total = S.bad_off + 256;
    return true;
}

namespace rd {
int ctx_device(rd_ctx c) { return c->device; }
}  // namespace rd

static rd_status set_err(rd_ctx ctx, rd_status st, uint64_t index, const char *msg) {
    if (ctx) {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->last_index = index;
        strncpy(ctx->last_msg, msg ? msg : "", sizeof(ctx->last_msg) - 1);
        ctx->last_msg[sizeof(ctx->last_msg) - 1] = 0;
    }
    return st;
}

// ---------------------------------------------------------------- checks that allocate nothing
//
// rd_check_static's workspace: one fixed array per GPU, reached through the device address that
// rd_init looks up once per device (the array's name is a host-side stand-in, not that address).
static_assert(RD_STATIC_SCRATCH_BYTES % 256 == 0, "whole 256-byte units");
static __device__ __align__(256) unsigned char scratch[RD_STATIC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static char *g_scratch[MAX_DEVICES];  // device address of `scratch` on each device, once looked up

// Looks up the array's address on `dev` (with `dev` current) the first time a context is made
// there; the calling thread's current device is restored.
static bool static_scratch_setup(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return true;  // no static path on such a device
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch[dev]) return true;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return false;
    bool ok = hipSetDevice(dev) == hipSuccess;
    void *ptr = nullptr;
    if (ok && hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr) g_scratch[dev] = (char *)ptr;
    else ok = false;
    (void)hipGetLastError();
    (void)hipSetDevice(prev);
    return ok;
}

static char *static_scratch(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch[dev];
}

static bool grid_ok(const rd_grid *g, uint64_t n) {
    if (!g || g->n_blocks == 0 || g->threads_per_block == 0 || g->threads_per_block > 1024) return false;
    if (g->warp_size > 32 || g->reserved != 0) return false;
    if ((uint64_t)g->n_blocks * g->threads_per_block >= (1ull << 32)) return false;
    if (n >= (1ull << 32)) return false;
    return true;
}

extern "C" {

rd_status rd_init(int hip_device, rd_ctx *out) {
    if (!out) return RD_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return RD_EINVAL;
    if (!static_scratch_setup(hip_device)) return RD_EHIP;
    rd_ctx c = new (std::nothrow) rd_ctx_s;
    if (!c) return RD_ENOMEM;
    c->device = hip_device;
    c->last_index = UINT64_MAX;
    c->last_msg[0] = 0;
    *out = c;
    return RD_OK;
}

rd_status rd_shutdown(rd_ctx ctx) {
    if (!ctx) return RD_EINVAL;
    for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return RD_OK;
}

rd_status rd_workspace_bytes(rd_ctx ctx, const rd_grid *grid, uint64_t n_events, const rd_limits *limits,
                             uint64_t *bytes) {
    if (!ctx || !bytes) return RD_EINVAL;
    if (!grid_ok(grid, n_events)) return set_err(ctx, RD_EINVAL, UINT64_MAX, "bad grid or event count");
    const Plan P = make_plan(n_events, grid->n_blocks, grid->threads_per_block, limits, true);
    *bytes = P.L.total;
    return RD_OK;
}

rd_status rd_trace_upload(rd_ctx ctx, const rd_grid *grid, const rd_event *events, uint64_t n_events,
                          int events_on_device, void *workspace, uint64_t workspace_bytes, const rd_limits *limits,
                          hipStream_t stream, rd_trace *out) {
    if (!ctx || !out) return RD_EINVAL;
    *out = nullptr;
    if (!grid_ok(grid, n_events)) return set_err(ctx, RD_EINVAL, UINT64_MAX, "bad grid or event count");
    if (n_events && !events) return set_err(ctx, RD_EINVAL, UINT64_MAX, "null events");
    const u32 ws = grid->warp_size ? grid->warp_size : 32;
    if (!workspace && events_on_device) {
        // a batch member only: its events stay where they are, no workspace of its own
        rd_trace t = new (std::nothrow) rd_trace_s;
        if (!t) return RD_ENOMEM;
        t->plan = make_plan(n_events, grid->n_blocks, grid->threads_per_block, limits, false);
        memset(&t->bufs, 0, sizeof(t->bufs));
        t->bufs.ev = (const uint4 *)events;
        t->bufs.max_pairs = t->plan.L.max_pairs;
        t->bufs.N = (u32)n_events;
        t->ws = nullptr;
        t->masks = nullptr;
        t->rt_scan = nullptr;
        t->grid = *grid;
        t->n = n_events;
        t->stream = stream;
        t->checked = 0;
        t->cached = 0;
        t->lim = limits ? *limits : rd_limits{0, 0};
        *out = t;
        return RD_OK;
    }
    if (!workspace || ((uintptr_t)workspace & 255)) return set_err(ctx, RD_EINVAL, UINT64_MAX, "workspace null or not 256-byte aligned");
    const Plan P = make_plan(n_events, grid->n_blocks, grid->threads_per_block, limits, true);
    if (workspace_bytes < P.L.total) return set_err(ctx, RD_ENOMEM, UINT64_MAX, "workspace too small");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    rd_trace t = new (std::nothrow) rd_trace_s;
    if (!t) return RD_ENOMEM;
    t->plan = P;
    t->ws = (char *)workspace;
    t->grid = *grid;
    t->n = n_events;
    t->stream = stream;
    t->checked = 0;
    t->cached = 0;
    t->lim = limits ? *limits : rd_limits{0, 0};
    const void *dev_events = nullptr;
    if (events_on_device) dev_events = events;
    else if (n_events) {
        if (hipMemcpyAsync(t->ws + P.L.off_ev, events, 16 * n_events, hipMemcpyHostToDevice, stream) != hipSuccess) {
            delete t;
            return set_err(ctx, RD_EHIP, UINT64_MAX, "hipMemcpyAsync of the events failed");
        }
    }
    t->bufs = make_bufs(P, t->ws, dev_events, n_events, grid->n_blocks, grid->threads_per_block, ws);
    t->masks = (u64 *)(t->ws + P.off_masks);
    t->rt_scan = (u32 *)(t->ws + P.off_rt_scan);
    *out = t;
    return RD_OK;
}

// Releases a trace's captured check.
static void graph_drop(rd_trace t) {
    for (GraphSeg &g : t->segs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    t->segs.clear();
}

// Captures the trace's plain check into graph pieces (cut around the profiled kernels).
static bool graph_capture(rd_ctx ctx, rd_trace t, u32 spec) {
    if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        ctx->cap_stream = nullptr;
        return false;
    }
    hipStream_t cs = ctx->cap_stream;
    Profiler &p = ctx->prof;
    Profiler *saved = g_prof;
    g_prof = p.filter.empty() ? nullptr : &p;
    p.capture = &t->segs;
    p.cap_err = hipSuccess;
    p.open_name = nullptr;
    p.group_name = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    hipError_t e2 = hipSuccess;
    if (e == hipSuccess) {
        Bufs gb = t->bufs;
        gb.spec = spec;
        e2 = enqueue_plain(gb, t->masks, t->rt_scan, cs);
        GraphSeg last;
        e = hipStreamEndCapture(cs, &last.graph);
        last.name = p.group_name;
        last.launches = p.group_name ? p.group_n : 0;
        if (e == hipSuccess) t->segs.push_back(last);
    }
    p.group_name = nullptr;
    if (e2 == hipSuccess) e2 = p.cap_err;
    p.capture = nullptr;
    p.open_name = nullptr;
    g_prof = saved;
    // pieces without a node (between two profiled kernels) are left out
    std::vector<GraphSeg> kept;
    for (GraphSeg &g : t->segs) {
        size_t nodes = 0;
        if (e == hipSuccess && e2 == hipSuccess && hipGraphGetNodes(g.graph, nullptr, &nodes) == hipSuccess && !nodes) {
            (void)hipGraphDestroy(g.graph);
            continue;
        }
        kept.push_back(g);
    }
    t->segs.swap(kept);
    for (GraphSeg &g : t->segs) {
        if (e != hipSuccess || e2 != hipSuccess) break;
        e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    }
    if (e != hipSuccess || e2 != hipSuccess) {
        (void)hipGetLastError();
        graph_drop(t);
        return false;
    }
    t->graph_variant = ctx->sort_variant;
    t->graph_filter = p.filter;
    t->graph_spec = spec;
    return true;
}

// One check as launches of the captured pieces; a profiled kernel's piece is bracketed by events.
static hipError_t graph_launch(rd_ctx ctx, rd_trace t, hipStream_t stream) {
    Profiler &p = ctx->prof;
    for (GraphSeg &g : t->segs) {
        hipEvent_t a = nullptr, b = nullptr;
        if (g.name && !p.filter.empty()) {
            a = p.get();
            if (a && hipEventRecord(a, stream) != hipSuccess) a = nullptr;
        }
        const hipError_t e = hipGraphLaunch(g.exec, stream);
        if (e != hipSuccess) return e;
        if (a) {
            b = p.get();
            if (b && hipEventRecord(b, stream) == hipSuccess) p.recs.push_back({g.name, a, b, g.launches});
        }
    }
    return hipSuccess;
}

rd_status rd_check(rd_ctx ctx, rd_trace trace, hipStream_t stream) {
    if (!ctx || !trace) return RD_EINVAL;
    if (!trace->ws) return set_err(ctx, RD_ESTATE, UINT64_MAX, "the trace has no workspace: check it with rd_check_many");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    trace->stream = stream;
    trace->batch.reset();
    trace->cached = 0;
    trace->bufs.sort_variant = ctx->sort_variant;
    trace->bufs.radix_bits = kSortVariants[ctx->sort_variant].rb;
    // from the second check of a trace on, the pass is one graph launch (captured again when the
    // sort variant or the profiled kernels change)
    if (trace->n_checks++ > 0 && !trace->graph_off) {
        // the pass is built without the stages the trace's last check did not need (checked on the
        // device: a trace that needs one after all is checked again whole by rd_races)
        u32 spec = 0;
        if (!(trace->last_mode & MODE_SYNC)) spec |= SPEC_NO_SYNC;
        if (!(trace->last_mode & MODE_WBAR)) spec |= SPEC_NO_WBAR;
        if (trace->segs.empty() || trace->graph_variant != ctx->sort_variant || trace->graph_filter != ctx->prof.filter ||
            trace->graph_spec != spec) {
            graph_drop(trace);
            if (!graph_capture(ctx, trace, spec)) trace->graph_off = true;
        }
        if (!trace->segs.empty()) {
            const hipError_t e = graph_launch(ctx, trace, stream);
            if (e != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, hipGetErrorString(e));
            trace->checked = 1;
            return RD_OK;
        }
    }
    Profiler *saved = g_prof;
    g_prof = ctx->prof.filter.empty() ? nullptr : &ctx->prof;
    const hipError_t e = enqueue_plain(trace->bufs, trace->masks, trace->rt_scan, stream);
    g_prof = saved;
    if (e != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, hipGetErrorString(e));
    trace->checked = 1;
    return RD_OK;
}

// Report of a member of a batched check.  Returns false when the batch cannot answer for the trace
// (some member was invalid, a capacity of the merged check overflowed, or the trace has more pairs
// than its own limit): the caller then checks the trace on its own, which gives the plain result,
// errors included.
// Waits for the batch and reads its state once; false when that fails (HIP error, status set).
static bool batch_read_state(rd_ctx ctx, Batch &B, rd_status *st) {
    std::lock_guard<std::mutex> g(B.mu);
    if (B.read) return true;
    DevParams prm;
    u32 bad = 0;
    if (hipMemcpyAsync(&prm, B.bufs.prm, sizeof(prm), hipMemcpyDeviceToHost, B.stream) != hipSuccess ||
        hipMemcpyAsync(&bad, B.bad_dev, 4, hipMemcpyDeviceToHost, B.stream) != hipSuccess ||
        hipMemcpyAsync(B.tr_host.data(), B.tr_dev, sizeof(BatchTrace) * B.tr_host.size(), hipMemcpyDeviceToHost,
                       B.stream) != hipSuccess ||
        hipStreamSynchronize(B.stream) != hipSuccess) {
        *st = set_err(ctx, RD_EHIP, UINT64_MAX, "reading the batch state failed");
        return false;
    }
    B.failed = bad || prm.err || prm.first_bad_record != NONE || prm.first_bad_sync != NONE;
    B.read = true;
    return true;
}

static bool batch_races(rd_ctx ctx, rd_trace trace, rd_pair *out, uint64_t capacity, uint64_t *n_races,
                        rd_status *st) {
    Batch &B = *trace->batch;
    if (!batch_read_state(ctx, B, st)) return true;
    if (B.failed) return false;
    const BatchTrace &t = B.tr_host[trace->batch_idx];
    const u64 m = t.pair_hi - t.pair_lo;
    *n_races = m;
    if (m > trace->bufs.max_pairs) {  // what the member's own check reports
        *st = set_err(ctx, RD_ENOMEM, UINT64_MAX, "race pairs exceed rd_limits.max_pairs");
        return true;
    }
    *st = RD_OK;
    if (!out || !capacity || !m) {
        if (m > capacity) *st = set_err(ctx, RD_ETRUNC, UINT64_MAX, "capacity");
        return true;
    }
    const u64 k = capacity < m ? capacity : m;
    std::vector<u32> f(k), sec(k);
    if (hipMemcpyAsync(f.data(), B.bufs.pfirst[0] + t.pair_lo, 4 * k, hipMemcpyDeviceToHost, B.stream) != hipSuccess ||
        hipMemcpyAsync(sec.data(), B.bufs.psecond[0] + t.pair_lo, 4 * k, hipMemcpyDeviceToHost, B.stream) !=
            hipSuccess ||
        hipStreamSynchronize(B.stream) != hipSuccess) {
        *st = set_err(ctx, RD_EHIP, UINT64_MAX, "copying the pairs failed");
        return true;
    }
    const u32 base = B.off_host[trace->batch_idx];
    for (u64 q = 0; q < k; q++) { out[q].first = f[q] - base; out[q].second = sec[q] - base; }
    if (capacity < m) *st = set_err(ctx, RD_ETRUNC, UINT64_MAX, "more races than capacity");
    return true;
}

// The check's own errors (the trace, its capacities, a wait that gave up), the pair buffer aside.
static rd_status state_error(rd_ctx ctx, const DevParams &prm) {
    if (prm.first_bad_record != NONE) return set_err(ctx, RD_ETRACE, prm.first_bad_record, "malformed record");
    if (prm.err & ERR_PHASE) return set_err(ctx, RD_EINVAL, UINT64_MAX, "a thread passed more than 2^30 barriers");
    if (prm.first_bad_sync != NONE)
        return set_err(ctx, RD_ETRACE, prm.first_bad_sync, "event runs ahead of an unfinished barrier");
    if (prm.err & ERR_SORT) return set_err(ctx, RD_EHIP, UINT64_MAX, "location sort look-back did not finish");
    if (prm.err & ERR_ENGINE) return set_err(ctx, RD_EHIP, UINT64_MAX, "knowledge engine barrier did not finish");
    if (prm.err & ERR_KEYSPAN)
        return set_err(ctx, RD_EINVAL, UINT64_MAX, "address span too large for a 32-bit location key");
    if (prm.err & ERR_POOL) return set_err(ctx, RD_ENOMEM, UINT64_MAX, "knowledge-vector pool exhausted (rd_limits.clock_bytes)");
    if (prm.err & ERR_TABLE) return set_err(ctx, RD_ENOMEM, UINT64_MAX, "sync-variable or warp-barrier table full");
    return RD_OK;
}

// The report of a check enqueued on `s` over buffers `b` (waits for it).
static rd_status plain_races(rd_ctx ctx, const Bufs &b, hipStream_t s, rd_pair *out, uint64_t capacity,
                             uint64_t *n_races, u64 *hint, HostStage *stage = nullptr, u32 *mode = nullptr,
                             bool *respec = nullptr) {
    // the check left the sorted report as rd_pair records (pack_pairs); as many as the previous
    // report of these buffers held are copied together with the state, so a report no longer than
    // the last one takes a single wait.  With a stage, both go by DMA to page-locked memory and only
    // the returned records are copied on to `out`.
    constexpr u64 HDR = 256;
    static_assert(sizeof(DevParams) <= HDR, "the state fits the stage's header");
    DevParams prm;
    const u64 lim = capacity < b.max_pairs ? capacity : b.max_pairs;
    const u64 early = out && hint ? (*hint < lim ? *hint : lim) : 0;
    const bool staged = stage && stage->ensure(HDR + 8 * early);
    rd_pair *early_dst = staged ? (rd_pair *)(stage->p + HDR) : out;
    if (hipMemcpyAsync(staged ? (void *)stage->p : (void *)&prm, b.prm, sizeof(prm), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        (early && hipMemcpyAsync(early_dst, b.preport, 8 * early, hipMemcpyDeviceToHost, s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_err(ctx, RD_EHIP, UINT64_MAX, "reading the check state failed");
    if (staged) memcpy(&prm, stage->p, sizeof(prm));
    if (mode) *mode = prm.mode;
    if (prm.err & ERR_RESPEC) {
        if (respec) {
            *respec = true;
            return RD_OK;
        }
        return set_err(ctx, RD_ESTATE, UINT64_MAX, "the pass was built without a stage the trace needs");
    }
    const rd_status se = state_error(ctx, prm);
    if (se != RD_OK) return se;
    if (prm.err & ERR_PAIRS) {
        *n_races = prm.n_pairs;
        return set_err(ctx, RD_ENOMEM, UINT64_MAX, "race pairs exceed rd_limits.max_pairs");
    }
    const u32 m = prm.n_pairs_kept;
    *n_races = m;
    if (hint) *hint = m;
    if (!out || !capacity || !m) return m > capacity ? set_err(ctx, RD_ETRUNC, UINT64_MAX, "capacity") : RD_OK;
    const u64 k = capacity < m ? capacity : m;
    if (staged) memcpy(out, stage->p + HDR, 8 * (k < early ? k : early));
    if (k > early && (hipMemcpyAsync(out + early, b.preport + early, 8 * (k - early), hipMemcpyDeviceToHost, s) !=
                          hipSuccess ||
                      hipStreamSynchronize(s) != hipSuccess))
        return set_err(ctx, RD_EHIP, UINT64_MAX, "copying the pairs failed");
    if (capacity < m) return set_err(ctx, RD_ETRUNC, UINT64_MAX, "more races than capacity");
    return RD_OK;
}

// A member without a workspace whose batch cannot answer for it: checked alone in the batch's
// workspace (which is at least as large as the member's own would be), once; the report is kept.
static rd_status member_alone(rd_ctx ctx, rd_trace trace, rd_pair *out, uint64_t capacity, uint64_t *n_races) {
    Batch &B = *trace->batch;
    if (!trace->cached) {
        std::lock_guard<std::mutex> g(B.ws_mu);
        const u32 ws = trace->grid.warp_size ? trace->grid.warp_size : 32;
        const Plan P = make_plan(trace->n, trace->grid.n_blocks, trace->grid.threads_per_block, &trace->lim, false);
        if (P.L.total > B.ws_bytes)
            return set_err(ctx, RD_ENOMEM, UINT64_MAX, "the batch workspace cannot hold this member's own check");
        Bufs b = make_bufs(P, B.ws, trace->bufs.ev, trace->n, trace->grid.n_blocks,
                           trace->grid.threads_per_block, ws);
        b.sort_variant = ctx->sort_variant;
        b.radix_bits = kSortVariants[ctx->sort_variant].rb;
        Profiler *saved = g_prof;
        g_prof = ctx->prof.filter.empty() ? nullptr : &ctx->prof;
        const hipError_t e = enqueue_plain(b, (u64 *)(B.ws + P.off_masks), (u32 *)(B.ws + P.off_rt_scan), B.stream);
        g_prof = saved;
        if (e != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, hipGetErrorString(e));
        uint64_t n = 0;
        rd_status st = plain_races(ctx, b, B.stream, nullptr, 0, &n, nullptr);
        trace->cache.clear();
        if (st == RD_OK || st == RD_ETRUNC) {
            trace->cache.resize(n);
            st = plain_races(ctx, b, B.stream, trace->cache.data(), n, &n, nullptr);
        }
        if (st == RD_EHIP) return st;
        trace->cache_st = st;
        trace->cache_n = n;
        {
            std::lock_guard<std::mutex> g2(ctx->mu);
            trace->cache_idx = ctx->last_index;
            trace->cache_msg = ctx->last_msg;
        }
        trace->cached = 1;
    }
    *n_races = trace->cache_n;
    if (trace->cache_st != RD_OK) return set_err(ctx, trace->cache_st, trace->cache_idx, trace->cache_msg.c_str());
    const u64 k = out ? (capacity < trace->cache_n ? capacity : trace->cache_n) : 0;
    for (u64 q = 0; q < k; q++) out[q] = trace->cache[q];
    if (capacity < trace->cache_n) return set_err(ctx, RD_ETRUNC, UINT64_MAX, "more races than capacity");
    return RD_OK;
}

// The trace's last check was a pass built without a stage that the trace turned out to need (its
// events were rewritten in place): the check again, whole and kernel by kernel, and no graph until
// the next rd_check captures one for the kinds now seen.
static rd_status recheck_whole(rd_ctx ctx, rd_trace t) {
    graph_drop(t);
    t->last_mode = ~0u;
    Bufs b = t->bufs;
    b.spec = 0;
    Profiler *saved = g_prof;
    g_prof = ctx->prof.filter.empty() ? nullptr : &ctx->prof;
    const hipError_t e = enqueue_plain(b, t->masks, t->rt_scan, t->stream);
    g_prof = saved;
    if (e != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, hipGetErrorString(e));
    return RD_OK;
}

rd_status rd_races(rd_ctx ctx, rd_trace trace, rd_pair *out, uint64_t capacity, uint64_t *n_races) {
    if (!ctx || !trace || !n_races) return RD_EINVAL;
    *n_races = 0;
    if (!trace->checked) return set_err(ctx, RD_ESTATE, UINT64_MAX, "rd_races before rd_check");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    if (trace->batch) {
        rd_status st = RD_OK;
        if (batch_races(ctx, trace, out, capacity, n_races, &st)) return st;
        if (!trace->ws) return member_alone(ctx, trace, out, capacity, n_races);
        const rd_status c = rd_check(ctx, trace, trace->batch->stream);  // on its own; drops the batch
        if (c != RD_OK) return c;
    }
    bool respec = false;
    rd_status st = plain_races(ctx, trace->bufs, trace->stream, out, capacity, n_races, &trace->last_pairs,
                               &trace->stage, &trace->last_mode, &respec);
    if (respec) {
        st = recheck_whole(ctx, trace);
        if (st != RD_OK) return st;
        st = plain_races(ctx, trace->bufs, trace->stream, out, capacity, n_races, &trace->last_pairs, &trace->stage,
                         &trace->last_mode, nullptr);
    }
    return st;
}

rd_status rd_check_static(rd_ctx ctx, const rd_grid *grid, const rd_event *events, uint64_t n_events,
                          const rd_limits *limits, rd_pair *out, uint64_t capacity, uint64_t *n_races,
                          hipStream_t stream) {
    if (!ctx || !n_races || (capacity && !out)) return RD_EINVAL;
    *n_races = 0;
    if (!grid_ok(grid, n_events)) return set_err(ctx, RD_EINVAL, UINT64_MAX, "bad grid or event count");
    if (n_events && !events) return set_err(ctx, RD_EINVAL, UINT64_MAX, "null events");
    char *ws = static_scratch(ctx->device);
    if (!ws) return set_err(ctx, RD_EHIP, UINT64_MAX, "no device address for the static scratch array");
    rd_limits lim = limits ? *limits : rd_limits{0, 0};
    if (!lim.clock_bytes) lim.clock_bytes = RD_STATIC_CLOCK_BYTES;
    const Plan P = make_plan(n_events, grid->n_blocks, grid->threads_per_block, &lim, false, false);
    if (P.L.total > RD_STATIC_SCRATCH_BYTES)
        return set_err(ctx, RD_ENOMEM, UINT64_MAX, "the trace needs more than the static scratch array");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    const u32 wsz = grid->warp_size ? grid->warp_size : 32;
    Bufs b = make_bufs(P, ws, n_events ? (const void *)events : (const void *)ws, n_events, grid->n_blocks,
                       grid->threads_per_block, wsz);
    b.sort_variant = ctx->sort_variant;
    b.radix_bits = kSortVariants[ctx->sort_variant].rb;
    // launched kernel by kernel on the caller's stream: no graph, no profiling events
    Profiler *saved = g_prof;
    g_prof = nullptr;
    const hipError_t e = enqueue_plain(b, (u64 *)(ws + P.off_masks), (u32 *)(ws + P.off_rt_scan), stream);
    g_prof = saved;
    if (e != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, hipGetErrorString(e));
    return plain_races(ctx, b, stream, out, capacity, n_races, nullptr, nullptr);
}

rd_status rd_lockset(rd_ctx ctx, rd_trace trace, rd_pair *out, uint64_t capacity, uint64_t *n_pairs) {
    if (!ctx || !trace || !n_pairs || (capacity && !out)) return RD_EINVAL;
    *n_pairs = 0;
    if (!trace->ws) return set_err(ctx, RD_ESTATE, UINT64_MAX, "the lockset pass needs the trace's own workspace");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    LocksetBufs L;
    if (!lockset_layout(trace->bufs, trace->bufs.max_pairs, L))
        return set_err(ctx, RD_ENOMEM, UINT64_MAX, "the knowledge-vector pool cannot hold the lockset pass's pairs");
    // a check of its own (the pass reads its sync lists and sorted accesses), then the pass, on the
    // trace's stream; the trace's report afterwards is that check's
    trace->batch.reset();
    trace->cached = 0;
    trace->bufs.sort_variant = ctx->sort_variant;
    trace->bufs.radix_bits = kSortVariants[ctx->sort_variant].rb;
    Profiler *saved = g_prof;
    g_prof = ctx->prof.filter.empty() ? nullptr : &ctx->prof;
    hipError_t e = enqueue_plain(trace->bufs, trace->masks, trace->rt_scan, trace->stream);
    if (e == hipSuccess) {
        lockset_run(trace->bufs, L, trace->stream);
        e = hipGetLastError();
    }
    g_prof = saved;
    if (e != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, hipGetErrorString(e));
    trace->checked = 1;
    DevParams prm;
    if (hipMemcpyAsync(&prm, trace->bufs.prm, sizeof(prm), hipMemcpyDeviceToHost, trace->stream) != hipSuccess ||
        hipStreamSynchronize(trace->stream) != hipSuccess)
        return set_err(ctx, RD_EHIP, UINT64_MAX, "reading the check state failed");
    const rd_status se = state_error(ctx, prm);
    if (se != RD_OK) return se;
    if (prm.err & ERR_LOCKSET)
        return set_err(ctx, RD_ENOMEM, UINT64_MAX, "a thread holds more than 64 locks at once, or the lockset rows exceed the pool");
    *n_pairs = prm.ls_pairs;
    if (prm.err & ERR_LSPAIRS) return set_err(ctx, RD_ENOMEM, UINT64_MAX, "lockset pairs exceed rd_limits.max_pairs");
    const u64 m = prm.ls_kept, k = capacity < m ? capacity : m;
    if (k && (hipMemcpyAsync(out, L.report, 8 * k, hipMemcpyDeviceToHost, trace->stream) != hipSuccess ||
              hipStreamSynchronize(trace->stream) != hipSuccess))
        return set_err(ctx, RD_EHIP, UINT64_MAX, "copying the lockset pairs failed");
    if (capacity < m) return set_err(ctx, RD_ETRUNC, UINT64_MAX, "more lockset pairs than capacity");
    return RD_OK;
}

rd_status rd_gwcp(rd_ctx ctx, rd_trace trace, rd_pair *out, uint64_t capacity, uint64_t *n_pairs) {
    if (!ctx || !trace || !n_pairs || (capacity && !out)) return RD_EINVAL;
    *n_pairs = 0;
    if (!trace->ws) return set_err(ctx, RD_ESTATE, UINT64_MAX, "the GWCP pass needs the trace's own workspace");
    if (trace->bufs.T > GW_MAX_T)
        return set_err(ctx, RD_EINVAL, UINT64_MAX, "the GWCP pass keeps dense clocks: at most 4096 threads");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    GwcpBufs G;
    if (!gwcp_layout(trace->bufs, trace->bufs.max_pairs, G))
        return set_err(ctx, RD_ENOMEM, UINT64_MAX, "the knowledge-vector pool cannot hold the GWCP pass's pairs and clocks");
    // a check of its own (the pass reads its sync lists, barrier instances and sorted accesses), then
    // the pass, on the trace's stream; the trace's report afterwards is that check's
    trace->batch.reset();
    trace->cached = 0;
    trace->bufs.sort_variant = ctx->sort_variant;
    trace->bufs.radix_bits = kSortVariants[ctx->sort_variant].rb;
    Profiler *saved = g_prof;
    g_prof = ctx->prof.filter.empty() ? nullptr : &ctx->prof;
    hipError_t e = enqueue_plain(trace->bufs, trace->masks, trace->rt_scan, trace->stream);
    if (e == hipSuccess) {
        gwcp_run(trace->bufs, G, trace->stream);
        e = hipGetLastError();
    }
    g_prof = saved;
    if (e != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, hipGetErrorString(e));
    trace->checked = 1;
    DevParams prm;
    if (hipMemcpyAsync(&prm, trace->bufs.prm, sizeof(prm), hipMemcpyDeviceToHost, trace->stream) != hipSuccess ||
        hipStreamSynchronize(trace->stream) != hipSuccess)
        return set_err(ctx, RD_EHIP, UINT64_MAX, "reading the check state failed");
    const rd_status se = state_error(ctx, prm);
    if (se != RD_OK) return se;
    if (prm.err & ERR_GWCP)
        return set_err(ctx, RD_ENOMEM, UINT64_MAX,
                       "a thread holds more than 64 locks at once, or the GWCP clocks exceed the knowledge-vector pool");
    *n_pairs = prm.gw_pairs;
    if (prm.err & ERR_GWPAIRS) return set_err(ctx, RD_ENOMEM, UINT64_MAX, "GWCP pairs exceed rd_limits.max_pairs");
    const u64 m = prm.gw_kept, k = capacity < m ? capacity : m;
    if (k && (hipMemcpyAsync(out, G.report, 8 * k, hipMemcpyDeviceToHost, trace->stream) != hipSuccess ||
              hipStreamSynchronize(trace->stream) != hipSuccess))
        return set_err(ctx, RD_EHIP, UINT64_MAX, "copying the GWCP pairs failed");
    if (capacity < m) return set_err(ctx, RD_ETRUNC, UINT64_MAX, "more GWCP pairs than capacity");
    return RD_OK;
}

rd_status rd_race_kinds(rd_ctx ctx, rd_trace trace, rd_race_kind *out, uint64_t capacity, uint64_t *n_kinds) {
    if (!ctx || !trace || !n_kinds || (capacity && !out)) return RD_EINVAL;
    *n_kinds = 0;
    if (!trace->checked) return set_err(ctx, RD_ESTATE, UINT64_MAX, "rd_race_kinds before rd_check");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    if (trace->batch) {
        // the kinds are built from the trace's own report
        if (!trace->ws) return set_err(ctx, RD_ESTATE, UINT64_MAX, "race kinds of a batch member need its own workspace");
        const rd_status c = rd_check(ctx, trace, trace->batch->stream);
        if (c != RD_OK) return c;
    }
    uint64_t m = 0;
    bool respec = false;
    rd_status st = plain_races(ctx, trace->bufs, trace->stream, nullptr, 0, &m, nullptr, nullptr, &trace->last_mode,
                               &respec);
    if (respec) {
        st = recheck_whole(ctx, trace);
        if (st != RD_OK) return st;
        st = plain_races(ctx, trace->bufs, trace->stream, nullptr, 0, &m, nullptr, nullptr, &trace->last_mode);
    }
    if (st != RD_OK && st != RD_ETRUNC) return st;
    if (!m) return RD_OK;
    // scratch in the trace's workspace (sized for max_pairs): 5m + 1 words, scan partials, 3m
    // record words, the count
    const u64 parts = (m + 1 + 4095) / 4096 + 16;
    u32 *scratch = (u32 *)(trace->ws + trace->plan.off_kinds), *rec = scratch + 5 * m + 1 + parts, *n_out = rec + 3 * m;
    Profiler *saved = g_prof;
    g_prof = ctx->prof.filter.empty() ? nullptr : &ctx->prof;
    race_kinds(trace->bufs, (u32)m, scratch, rec, n_out, trace->stream);
    g_prof = saved;
    u32 nk = 0;
    DevParams prm;
    if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&nk, n_out, 4, hipMemcpyDeviceToHost, trace->stream) != hipSuccess ||
        hipMemcpyAsync(&prm, trace->bufs.prm, sizeof(prm), hipMemcpyDeviceToHost, trace->stream) != hipSuccess ||
        hipStreamSynchronize(trace->stream) != hipSuccess)
        return set_err(ctx, RD_EHIP, UINT64_MAX, "building the race kinds failed");
    if (prm.err & ERR_SORT) return set_err(ctx, RD_EHIP, UINT64_MAX, "race-kind sort look-back did not finish");
    *n_kinds = nk;
    const u64 k = capacity < nk ? capacity : nk;
    if (k && (hipMemcpyAsync(out, rec, 12 * k, hipMemcpyDeviceToHost, trace->stream) != hipSuccess ||
              hipStreamSynchronize(trace->stream) != hipSuccess))
        return set_err(ctx, RD_EHIP, UINT64_MAX, "copying the race kinds failed");
    if (capacity < nk) return set_err(ctx, RD_ETRUNC, UINT64_MAX, "more race kinds than capacity");
    return RD_OK;
}

// The merged pass's buffers and member table (host side) for members that can share one pass.
static rd_status batch_prepare(rd_ctx ctx, const rd_trace *traces, uint32_t n, void *workspace,
                               uint64_t workspace_bytes, const BatchShape &S, hipStream_t stream,
                               std::shared_ptr<Batch> &out) {
    if (!workspace || ((uintptr_t)workspace & 255))
        return set_err(ctx, RD_EINVAL, UINT64_MAX, "workspace null or not 256-byte aligned");
    if (workspace_bytes < S.total) return set_err(ctx, RD_ENOMEM, UINT64_MAX, "batch workspace too small");
    std::shared_ptr<Batch> B(new (std::nothrow) Batch);
    if (!B) return RD_ENOMEM;
    char *ws = (char *)workspace;
    B->plan = S.plan;
    B->ws = ws;
    B->ws_bytes = workspace_bytes;
    B->bufs = make_bufs(S.plan, ws, nullptr, S.N, (u32)S.B, S.tpb, S.ws);
    B->bufs.sort_variant = ctx->sort_variant;
    B->bufs.radix_bits = kSortVariants[ctx->sort_variant].rb;
    B->masks = (u64 *)(ws + S.plan.off_masks);
    B->rt_scan = (u32 *)(ws + S.plan.off_rt_scan);
    B->tr_dev = (BatchTrace *)(ws + S.table_off);
    B->off_dev = (u32 *)(ws + S.off_off);
    B->bad_dev = (u32 *)(ws + S.bad_off);
    B->stream = stream;
    B->tr_init.resize(n);
    B->tr_host.resize(n);
    B->off_host.resize(n + 1);
    u32 off = 0, blk = 0;
    for (uint32_t j = 0; j < n; j++) {
        const rd_trace t = traces[j];
        BatchTrace &d = B->tr_init[j];
        memset(&d, 0, sizeof(d));
        d.ev = t->bufs.ev;
        d.n = (u32)t->n;
        d.n_blocks = t->grid.n_blocks;
        d.tpb = t->grid.threads_per_block;
        d.blk_off = blk;
        d.gmin = NONE;
        d.gmax = 0;
        B->off_host[j] = off;
        off += (u32)t->n;
        blk += t->grid.n_blocks;
    }
    B->off_host[n] = off;
    out = B;
    return RD_OK;
}

// The merged pass, enqueued on `stream` (also what a captured graph holds).
static hipError_t batch_enqueue(Batch &B, uint32_t n, const BatchShape &S, hipStream_t stream) {
    hipError_t e = hipMemcpyAsync(B.tr_dev, B.tr_init.data(), sizeof(BatchTrace) * n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(B.off_dev, B.off_host.data(), 4ull * (n + 1), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(B.bad_dev, &B.zero, 4, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) {
        batch_merge(B.tr_dev, B.off_dev, n, (u32)S.N, S.tpb, (uint4 *)B.bufs.ev, B.bad_dev, stream);
        e = enqueue_check(B.bufs, B.masks, B.rt_scan, stream);
    }
    if (e == hipSuccess) {
        sort_pairs(B.bufs, &B.bufs.prm->n_pairs_kept, 0, B.bufs.max_pairs, stream);
        batch_pair_ranges(B.tr_dev, B.off_dev, n, B.bufs, stream);
        e = hipGetLastError();
    }
    return e;
}

static void batch_attach(const std::shared_ptr<Batch> &B, const rd_trace *traces, uint32_t n, hipStream_t stream) {
    {
        std::lock_guard<std::mutex> g(B->mu);
        B->read = false;
        B->failed = false;
        B->stream = stream;
    }
    for (uint32_t j = 0; j < n; j++) {
        traces[j]->batch = B;
        traces[j]->batch_idx = j;
        traces[j]->checked = 1;
        traces[j]->cached = 0;
        traces[j]->stream = stream;
    }
}

rd_status rd_batch_workspace_bytes(rd_ctx ctx, const rd_trace *traces, uint32_t n, const rd_limits *limits,
                                   uint64_t *bytes) {
    if (!ctx || !bytes || (n && !traces)) return RD_EINVAL;
    for (uint32_t j = 0; j < n; j++)
        if (!traces[j]) return set_err(ctx, RD_EINVAL, UINT64_MAX, "null trace in the batch");
    BatchShape S;
    *bytes = !n ? 256 : batch_shape(traces, n, limits, S) ? S.total : 0;
    return RD_OK;
}

rd_status rd_check_many(rd_ctx ctx, const rd_trace *traces, uint32_t n, void *workspace, uint64_t workspace_bytes,
                        const rd_limits *limits, hipStream_t stream) {
    if (!ctx || (n && !traces)) return RD_EINVAL;
    for (uint32_t j = 0; j < n; j++)
        if (!traces[j]) return set_err(ctx, RD_EINVAL, UINT64_MAX, "null trace in the batch");
    if (!n) return RD_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    BatchShape S;
    if (!batch_shape(traces, n, limits, S)) {
        // members that cannot share one merged trace are checked one by one, in order
        for (uint32_t j = 0; j < n; j++)
            if (!traces[j]->ws)
                return set_err(ctx, RD_EINVAL, UINT64_MAX,
                               "members cannot share one pass (warp sizes or sizes) and one has no workspace");
        for (uint32_t j = 0; j < n; j++) {
            const rd_status st = rd_check(ctx, traces[j], stream);
            if (st != RD_OK) return st;
        }
        return RD_OK;
    }
    if (!workspace || ((uintptr_t)workspace & 255))
        return set_err(ctx, RD_EINVAL, UINT64_MAX, "workspace null or not 256-byte aligned");
    if (workspace_bytes < S.total) return set_err(ctx, RD_ENOMEM, UINT64_MAX, "batch workspace too small");
    std::shared_ptr<Batch> B;
    const rd_status st = batch_prepare(ctx, traces, n, workspace, workspace_bytes, S, stream, B);
    if (st != RD_OK) return st;
    Profiler *saved = g_prof;
    g_prof = ctx->prof.filter.empty() ? nullptr : &ctx->prof;
    const hipError_t e = batch_enqueue(*B, n, S, stream);
    g_prof = saved;
    if (e != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, hipGetErrorString(e));
    batch_attach(B, traces, n, stream);
    return RD_OK;
}

rd_status rd_races_many(rd_ctx ctx, const rd_trace *traces, uint32_t n, rd_pair *out, uint64_t capacity,
                        uint64_t *counts, rd_status *statuses) {
    if (!ctx || (n && (!traces || !counts || !statuses))) return RD_EINVAL;
    for (uint32_t j = 0; j < n; j++)
        if (!traces[j]) return set_err(ctx, RD_EINVAL, UINT64_MAX, "null trace");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    // one copy of the merged report when every member comes from the same healthy batch
    std::shared_ptr<Batch> B = n ? traces[0]->batch : nullptr;
    for (uint32_t j = 0; j < n && B; j++)
        if (traces[j]->batch != B) B = nullptr;
    std::vector<u32> f, sec;
    if (B) {
        rd_status st = RD_OK;
        if (!batch_read_state(ctx, *B, &st)) return st;
        if (B->failed) {
            B = nullptr;  // members answer one by one below
        } else {
            u64 total = 0;
            for (uint32_t j = 0; j < n; j++) {
                const BatchTrace &t = B->tr_host[traces[j]->batch_idx];
                if (t.pair_hi > total) total = t.pair_hi;
            }
            f.resize(total);
            sec.resize(total);
            if (total && (hipMemcpyAsync(f.data(), B->bufs.pfirst[0], 4 * total, hipMemcpyDeviceToHost, B->stream) !=
                              hipSuccess ||
                          hipMemcpyAsync(sec.data(), B->bufs.psecond[0], 4 * total, hipMemcpyDeviceToHost,
                                         B->stream) != hipSuccess ||
                          hipStreamSynchronize(B->stream) != hipSuccess))
                return set_err(ctx, RD_EHIP, UINT64_MAX, "copying the pairs failed");
        }
    }
    rd_status worst = RD_OK;
    u64 used = 0;
    for (uint32_t j = 0; j < n; j++) {
        const rd_trace tr = traces[j];
        rd_pair *dst = out ? out + used : nullptr;
        const u64 room = out && capacity > used ? capacity - used : 0;
        rd_status st;
        uint64_t m = 0;
        if (B) {
            const BatchTrace &t = B->tr_host[tr->batch_idx];
            m = t.pair_hi - t.pair_lo;
            if (m > tr->bufs.max_pairs) {
                st = RD_ENOMEM;  // what the member's own check reports: more pairs than its limit
            } else {
                const u64 k = room < m ? room : m;
                const u32 base = B->off_host[tr->batch_idx];
                for (u64 q = 0; q < k; q++) {
                    dst[q].first = f[t.pair_lo + q] - base;
                    dst[q].second = sec[t.pair_lo + q] - base;
                }
                st = k < m ? RD_ETRUNC : RD_OK;
            }
        } else {
            st = rd_races(ctx, tr, dst, room, &m);
        }
        counts[j] = m;
        statuses[j] = st;
        if (st == RD_OK || st == RD_ETRUNC) used += m < room ? m : room;
        if (st != RD_OK && worst == RD_OK) worst = st;
    }
    return worst;
}

rd_status rd_batch_capture(rd_ctx ctx, const rd_trace *traces, uint32_t n, void *workspace, uint64_t workspace_bytes,
                           const rd_limits *limits, hipStream_t stream, rd_graph *out) {
    if (!ctx || !out || !n || !traces || !stream) return RD_EINVAL;
    *out = nullptr;
    for (uint32_t j = 0; j < n; j++)
        if (!traces[j]) return set_err(ctx, RD_EINVAL, UINT64_MAX, "null trace in the batch");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    BatchShape S;
    if (!batch_shape(traces, n, limits, S))
        return set_err(ctx, RD_EINVAL, UINT64_MAX, "members cannot share one pass (warp sizes or sizes)");
    std::shared_ptr<Batch> B;
    const rd_status st = batch_prepare(ctx, traces, n, workspace, workspace_bytes, S, stream, B);
    if (st != RD_OK) return st;
    rd_graph g = new (std::nothrow) rd_graph_s;
    if (!g) return RD_ENOMEM;
    g->batch = B;
    g->traces.assign(traces, traces + n);
    Profiler *saved = g_prof;
    g_prof = nullptr;  // no event records inside a captured graph
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    hipError_t e2 = hipSuccess;
    if (e == hipSuccess) {
        e2 = batch_enqueue(*B, n, S, stream);
        e = hipStreamEndCapture(stream, &g->graph);
    }
    g_prof = saved;
    if (e == hipSuccess && e2 == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess || e2 != hipSuccess) {
        (void)hipGetLastError();
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return set_err(ctx, RD_EHIP, UINT64_MAX, hipGetErrorString(e != hipSuccess ? e : e2));
    }
    *out = g;
    return RD_OK;
}

rd_status rd_graph_launch(rd_ctx ctx, rd_graph g, hipStream_t stream) {
    if (!ctx || !g) return RD_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    if (hipGraphLaunch(g->exec, stream) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipGraphLaunch failed");
    batch_attach(g->batch, g->traces.data(), (uint32_t)g->traces.size(), stream);
    return RD_OK;
}

rd_status rd_graph_free(rd_ctx ctx, rd_graph g) {
    if (!ctx || !g) return RD_EINVAL;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return RD_OK;
}

rd_status rd_tuning_count(uint32_t *n) {
    if (!n) return RD_EINVAL;
    *n = N_SORT_VARIANTS;
    return RD_OK;
}

rd_status rd_tuning_get(uint32_t index, rd_tuning *out) {
    if (!out || index >= N_SORT_VARIANTS) return RD_EINVAL;
    out->radix_bits = kSortVariants[index].rb;
    out->waves_per_block = kSortVariants[index].waves;
    out->items_per_lane = kSortVariants[index].items;
    out->reserved = 0;
    return RD_OK;
}

rd_status rd_set_tuning(rd_ctx ctx, uint32_t index) {
    if (!ctx || index >= N_SORT_VARIANTS) return RD_EINVAL;
    ctx->sort_variant = index;
    return RD_OK;
}

rd_status rd_get_tuning(rd_ctx ctx, uint32_t *index) {
    if (!ctx || !index) return RD_EINVAL;
    *index = ctx->sort_variant;
    return RD_OK;
}

rd_status rd_autotune(rd_ctx ctx, const rd_trace *traces, uint32_t n, void *batch_workspace, uint64_t batch_bytes,
                      hipStream_t stream, uint32_t *best, double *ms) {
    if (!ctx || !n || !traces) return RD_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return RD_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return RD_EHIP; }
    const u32 saved = ctx->sort_variant;
    u32 arg = saved;
    double tbest = 1e300;
    rd_status st = RD_OK;
    for (u32 v = 0; v < N_SORT_VARIANTS && st == RD_OK; v++) {
        ctx->sort_variant = v;
        auto run = [&]() -> rd_status {
            return batch_workspace ? rd_check_many(ctx, traces, n, batch_workspace, batch_bytes, nullptr, stream)
                                   : rd_check(ctx, traces[0], stream);
        };
        st = run();  // warm-up
        float total = 0.f;
        for (int r = 0; r < 3 && st == RD_OK; r++) {
            if (hipEventRecord(e0, stream) != hipSuccess) { st = RD_EHIP; break; }
            st = run();
            if (st != RD_OK) break;
            float msr = 0.f;
            if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&msr, e0, e1) != hipSuccess) {
                st = RD_EHIP;
                break;
            }
            total += msr;
        }
        if (st != RD_OK) break;
        const double avg = total / 3.0;
        if (ms) ms[v] = avg;
        if (avg < tbest) { tbest = avg; arg = v; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->sort_variant = st == RD_OK ? arg : saved;
    if (best) *best = ctx->sort_variant;
    // leave the traces checked with the chosen variant
    if (st == RD_OK)
        st = batch_workspace ? rd_check_many(ctx, traces, n, batch_workspace, batch_bytes, nullptr, stream)
                             : rd_check(ctx, traces[0], stream);
    return st;
}

rd_status rd_trace_stats(rd_ctx ctx, rd_trace trace, rd_stats *out) {
    if (!ctx || !trace || !out) return RD_EINVAL;
    if (!trace->checked) return set_err(ctx, RD_ESTATE, UINT64_MAX, "rd_trace_stats before rd_check");
    if (!trace->ws) return set_err(ctx, RD_ESTATE, UINT64_MAX, "the trace has no workspace of its own");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RD_EHIP, UINT64_MAX, "hipSetDevice failed");
    if (trace->batch) {
        const rd_status c = rd_check(ctx, trace, trace->batch->stream);  // its own figures
        if (c != RD_OK) return c;
    }
    DevParams prm;
    for (int round = 0; round < 2; round++) {
        if (hipMemcpyAsync(&prm, trace->bufs.prm, sizeof(prm), hipMemcpyDeviceToHost, trace->stream) != hipSuccess ||
            hipStreamSynchronize(trace->stream) != hipSuccess)
            return set_err(ctx, RD_EHIP, UINT64_MAX, "reading the check state failed");
        if (!(prm.err & ERR_RESPEC)) break;
        const rd_status st = recheck_whole(ctx, trace);
        if (st != RD_OK) return st;
    }
    memset(out, 0, sizeof(*out));
    out->n_events = trace->n;
    out->n_accesses = prm.n_acc;
    for (int k = 0; k < 8; k++) out->kind_count[k] = prm.kind_count[k];
    out->key_bits = prm.key_bits;
    out->max_phase = prm.max_phase;
    out->packed = packed_elements(prm.key_bits, prm.max_phase) ? 1u : tinfo_elements(prm.key_bits, prm.max_phase, trace->bufs.T) ? 2u : 0u;
    const bool sync = (prm.mode & MODE_SYNC) != 0;
    const bool par = sync && (prm.eng & ENG_PARALLEL) && !(prm.eng & ENG_FALLBACK);
    out->engine = !sync ? 0u : (par ? 1u : 2u);
    if (sync) {
        out->clock_vectors = par ? prm.n_handles : prm.pool_next;
        out->clock_words = prm.D;
        out->clock_bytes = out->clock_vectors * out->clock_words * 4;
        out->dense_clock_bytes = out->clock_vectors * (u64)trace->bufs.T * 4;
    }
    out->engine_ops = par ? prm.n_ops : 0;
    out->engine_groups = par ? prm.n_groups : 0;
    out->slow_chunks = prm.n_chunks;
    out->race_pairs = prm.n_pairs;
    out->workspace_bytes = trace->plan.L.total;
    return RD_OK;
}

rd_status rd_trace_free(rd_ctx ctx, rd_trace trace) {
    if (!ctx || !trace) return RD_EINVAL;
    graph_drop(trace);
    trace->stage.release();
    delete trace;
    return RD_OK;
}

rd_status rd_profile_enable(rd_ctx ctx, const char *kernel) {
    if (!ctx) return RD_EINVAL;
    Profiler &p = ctx->prof;
    p.filter = kernel ? kernel : "";
    p.recs.clear();
    p.used = 0;
    p.acc.clear();
    return RD_OK;
}

rd_status rd_profile_read(rd_ctx ctx, rd_kernel_time *out, uint32_t capacity, uint32_t *n_out) {
    if (!ctx || !n_out) return RD_EINVAL;
    Profiler &p = ctx->prof;
    if (!p.collect()) return RD_EHIP;
    *n_out = (uint32_t)p.acc.size();
    for (uint32_t k = 0; k < p.acc.size() && k < capacity && out; k++) {
        rd_kernel_time z;
        memset(&z, 0, sizeof(z));
        strncpy(z.name, p.acc[k].name, sizeof(z.name) - 1);
        z.launches = p.acc[k].launches;
        z.total_ms = p.acc[k].total_ms;
        out[k] = z;
    }
    p.acc.clear();
    return RD_OK;
}

const char *rd_strerror(rd_status s) {
    switch (s) {
    case RD_OK: return "ok";
    case RD_EINVAL: return "invalid argument";
    case RD_ENOMEM: return "capacity exceeded";
    case RD_ETRACE: return "invalid trace";
    case RD_ETRUNC: return "output truncated";
    case RD_EHIP: return "HIP runtime error";
    case RD_ESTATE: return "call out of order";
    default: return "unknown status";
    }
}

rd_status rd_last_error(rd_ctx ctx, uint64_t *event_index, char *msg, uint64_t msg_len) {
    if (!ctx) return RD_EINVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    if (event_index) *event_index = ctx->last_index;
    if (msg && msg_len) {
        strncpy(msg, ctx->last_msg, msg_len - 1);
        msg[msg_len - 1] = 0;
    }
    return RD_OK;
}

}  // extern "C"
