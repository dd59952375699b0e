// rd_segcheck.hip -- the race check over the accesses sorted by location (gfx950).
//
// After the stable sort, the accesses of one location form a segment in trace order.  An earlier
// access a and a later access b of a segment race iff they conflict (different threads, at least one
// writes, not two atomics with overlapping scopes: Section 1, Section 4, Section 5.1) and a does not
// happen before b (scoped HB, Section 2.2).  Happens-before between two accesses is decided by:
//   same thread                                   -> ordered (rule i)
//   same block and phase(a) < phase(b)            -> ordered (rule iii: a block barrier separates)
//   knowledge of b's thread at b (releases, acquires, warp barriers; rd_interp.hip) covers a
//                                                 -> ordered (rule iv, composed with i and iii)
//   otherwise                                     -> race.
//
// Most accesses cannot race at all, and a prefix summary decides that in O(1): for the part of the
// segment before b it keeps, per conflict category (read, write, device atomic, block atomic), up to
// two distinct blocks, and for the trailing run of accesses with b's block and phase, up to two
// distinct threads.  If every earlier access of the segment is in b's block, only accesses of b's
// run (same block and phase) can race with b, and they can only if a conflicting category has a
// thread other than b's.  Otherwise b is checked against the earlier accesses one by one.
// The summaries are a segmented scan: per-tile totals, one scan over tiles, then the tile pass.
#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

struct Agg {
    u32 nonempty;
    u32 head_inside;     // a location change between two elements of the range
    u32 first_key, last_key;
    u32 run_blk, run_ph;
    u32 run_whole;       // every element of the range has the same location, block and phase
    u32 cb[4][2];        // per category: up to two distinct blocks in the last segment of the range
    u32 rt[4][2];        // per category: up to two distinct threads in the trailing run
};

size_t agg_bytes() { return sizeof(Agg); }

__device__ inline void set2_add(u32 s[2], u32 v) {
    if (v == NONE) return;
    if (s[0] == NONE) s[0] = v;
    else if (s[0] != v && s[1] == NONE) s[1] = v;
}
__device__ inline bool set2_has_other(const u32 s[2], u32 v) {
    return (s[0] != NONE && s[0] != v) || (s[1] != NONE && s[1] != v);
}
__device__ inline bool set2_empty(const u32 s[2]) { return s[0] == NONE; }

__device__ inline void agg_empty(Agg &a) {
    a.nonempty = 0; a.head_inside = 0; a.first_key = a.last_key = 0;
    a.run_blk = a.run_ph = 0; a.run_whole = 1;
#pragma unroll
    for (int c = 0; c < 4; c++) { a.cb[c][0] = a.cb[c][1] = NONE; a.rt[c][0] = a.rt[c][1] = NONE; }
}
__device__ inline void agg_one(Agg &a, u32 key, u32 blk, u32 ph, u32 tid, u32 cat) {
    agg_empty(a);
    a.nonempty = 1; a.first_key = a.last_key = key; a.run_blk = blk; a.run_ph = ph;
    a.cb[cat][0] = blk; a.rt[cat][0] = tid;
}
// r := l (+) r, l before r
__device__ inline void agg_combine(const Agg &l, Agg &r) {
    if (!l.nonempty) return;
    if (!r.nonempty) { r = l; return; }
    const bool boundary = r.head_inside || r.first_key != l.last_key;
    const bool extend = !boundary && r.run_whole && r.run_blk == l.run_blk && r.run_ph == l.run_ph;
    if (!boundary) {
#pragma unroll
        for (int c = 0; c < 4; c++) {
            u32 s[2] = {l.cb[c][0], l.cb[c][1]};
            set2_add(s, r.cb[c][0]); set2_add(s, r.cb[c][1]);
            r.cb[c][0] = s[0]; r.cb[c][1] = s[1];
        }
    }
    if (extend) {
#pragma unroll
        for (int c = 0; c < 4; c++) {
            u32 s[2] = {l.rt[c][0], l.rt[c][1]};
            set2_add(s, r.rt[c][0]); set2_add(s, r.rt[c][1]);
            r.rt[c][0] = s[0]; r.rt[c][1] = s[1];
        }
    }
    r.run_whole = l.run_whole && extend;
    r.head_inside = l.head_inside || r.head_inside || (r.first_key != l.last_key);
    r.first_key = l.first_key;
}

struct Elem { u32 key, idx, tid, info; };

__device__ inline Elem load_elem(const u32 *k, const u32 *i, const u32 *t, const u32 *f, u32 pos) {
    Elem e; e.key = k[pos]; e.idx = i[pos]; e.tid = t[pos]; e.info = f[pos];
    return e;
}

// ---------------------------------------------------------------- shared pieces

struct SegCtx {
    const u32 *k, *i, *t, *f;
    u32 n;
};

__device__ inline SegCtx seg_ctx(const Bufs &b) {
    // the sort leaves the elements in buffer (passes % 2); passes = ceil(key_bits / radix_bits)
    const u32 bits = b.prm->key_bits, passes = (bits + b.radix_bits - 1) / b.radix_bits;
    const u32 c = passes & 1;
    SegCtx s; s.k = b.ekey[c]; s.i = b.eidx[c]; s.t = b.etid[c]; s.f = b.einfo[c]; s.n = b.prm->n_acc;
    return s;
}

// Per-thread contiguous run of items: thread x of tile owns [tile*TILE + x*ITEMS, +ITEMS).
__device__ inline void thread_agg(const SegCtx &s, const Bufs &b, u64 base, Agg &acc) {
    agg_empty(acc);
    for (int q = 0; q < ITEMS; q++) {
        const u64 pos = base + q;
        if (pos >= s.n) break;
        const u32 info = s.f[pos], tid = s.t[pos];
        Agg one;
        agg_one(one, s.k[pos], tid / b.tpb, info_phase(info), tid, info_cat(info));
        agg_combine(acc, one);
        acc = one;
    }
}

// Block-wide (256 threads) exclusive scan of Aggs in LDS; returns this thread's exclusive prefix
// and writes the block total into *total (when non-null).
__device__ inline void block_exscan_agg(Agg &mine, Agg *buf /* 2*256 */, Agg *total) {
    const u32 x = threadIdx.x;
    buf[x] = mine;
    __syncthreads();
    u32 src = 0;
    for (u32 d = 1; d < WG_THREADS; d <<= 1) {
        Agg v = buf[src * WG_THREADS + x];
        if (x >= d) agg_combine(buf[src * WG_THREADS + x - d], v);
        buf[(src ^ 1) * WG_THREADS + x] = v;
        __syncthreads();
        src ^= 1;
    }
    if (total) *total = buf[src * WG_THREADS + WG_THREADS - 1];
    Agg ex;
    if (x == 0) agg_empty(ex);
    else ex = buf[src * WG_THREADS + x - 1];
    __syncthreads();
    mine = ex;
}

__global__ __launch_bounds__(WG_THREADS) void k_seg_reduce(Bufs b) {
    __shared__ Agg buf[2 * WG_THREADS];
    const SegCtx s = seg_ctx(b);
    Agg *tile_agg = (Agg *)b.tile_agg;
    const u64 tile0 = (u64)blockIdx.x * TILE;
    if (tile0 >= s.n) return;
    Agg mine;
    thread_agg(s, b, tile0 + (u64)threadIdx.x * ITEMS, mine);
    Agg total;
    block_exscan_agg(mine, buf, &total);
    if (threadIdx.x == 0) tile_agg[blockIdx.x] = total;
}

// exclusive scan over the tile totals (one workgroup)
__global__ __launch_bounds__(WG_THREADS) void k_seg_scan(Bufs b) {
    __shared__ Agg buf[2 * WG_THREADS];
    const SegCtx s = seg_ctx(b);
    Agg *tile_agg = (Agg *)b.tile_agg;
    const u32 nt = (u32)((s.n + TILE - 1) / TILE);
    const u32 per = (nt + WG_THREADS - 1) / WG_THREADS;
    const u32 lo = threadIdx.x * per, hi = min(lo + per, nt);
    Agg acc;
    agg_empty(acc);
    for (u32 q = lo; q < hi; q++) { Agg v = tile_agg[q]; agg_combine(acc, v); acc = v; }
    block_exscan_agg(acc, buf, nullptr);
    for (u32 q = lo; q < hi; q++) { Agg v = tile_agg[q]; tile_agg[q] = acc; agg_combine(acc, v); acc = v; }
}

// ---------------------------------------------------------------- the check

__device__ inline bool cat_write(u32 c) { return c != CAT_R; }
__device__ inline bool cat_atomic(u32 c) { return c >= CAT_AD; }

__device__ inline bool conflicts(u32 ca, u32 ba, u32 cb, u32 bb) {
    if (!cat_write(ca) && !cat_write(cb)) return false;
    if (cat_atomic(ca) && cat_atomic(cb) && (ca == CAT_AD || cb == CAT_AD || ba == bb)) return false;
    return true;
}

struct BCtx {
    u32 idx, tid, blk, ph, cat;
    u32 h;        // knowledge vector of b's thread at b (NONE until looked up)
};

__device__ inline bool happens_before(const Bufs &b, const u32 *rt_scan, BCtx &bc, u32 ta, u32 ba, u32 pha, u32 ia) {
    if (ba == bc.blk && pha < bc.ph) return true;
    if (!(b.prm->mode & MODE_SYNC)) return false;
    if (bc.h == NONE) {
        const u32 j = list_search(b, bc.tid, bc.idx);
        bc.h = j == NONE ? 0u : b.s_know[j];
    }
    if (!bc.h) return false;
    const u32 *V = b.pool + (u64)bc.h * b.prm->D;
    if (V[ba] > pha) return true;
    if (rt_scan[ta + 1] > rt_scan[ta]) {
        const u32 col = b.B + rt_scan[ta];
        if (V[col] >= ia + 1) return true;
    }
    return false;
}

__device__ inline void emit(const Bufs &b, u32 first, u32 second) {
    const u32 slot = atomicAdd(&b.prm->n_pairs, 1u);
    if (slot < b.max_pairs) { b.pfirst[0][slot] = first; b.psecond[0][slot] = second; }
    else atomicOr(&b.prm->err, ERR_PAIRS);
}

// Checks b against earlier accesses of its segment, walking back from pos-1.
// group_only: stop at the first access outside b's (block, phase) run.
__device__ inline void slow_check(const Bufs &b, const SegCtx &s, const u32 *rt_scan, u32 pos, u32 key, BCtx &bc,
                                  bool group_only) {
    for (u32 q = pos; q-- > 0;) {
        if (s.k[q] != key) break;
        const u32 ta = s.t[q], info = s.f[q];
        const u32 ba = ta / b.tpb, pha = info_phase(info), ca = info_cat(info);
        if (group_only && (ba != bc.blk || pha != bc.ph)) break;
        if (ta == bc.tid) continue;
        if (!conflicts(ca, ba, bc.cat, bc.blk)) continue;
        const u32 ia = s.i[q];
        if (happens_before(b, rt_scan, bc, ta, ba, pha, ia)) continue;
        emit(b, ia, bc.idx);
    }
}

__global__ __launch_bounds__(WG_THREADS) void k_seg_check(Bufs b, const u32 *rt_scan) {
    __shared__ Agg buf[2 * WG_THREADS];
    const SegCtx s = seg_ctx(b);
    const Agg *tile_agg = (const Agg *)b.tile_agg;
    const u64 tile0 = (u64)blockIdx.x * TILE;
    if (tile0 >= s.n) return;
    const u64 base = tile0 + (u64)threadIdx.x * ITEMS;
    Agg mine;
    thread_agg(s, b, base, mine);
    block_exscan_agg(mine, buf, nullptr);
    // prefix of everything before this thread's first item
    Agg P = tile_agg[blockIdx.x];
    agg_combine(P, mine);
    P = mine;
    for (int q = 0; q < ITEMS; q++) {
        const u64 pos = base + q;
        if (pos >= s.n) break;
        const Elem e = load_elem(s.k, s.i, s.t, s.f, (u32)pos);
        const u32 cat = info_cat(e.info), ph = info_phase(e.info), blk = e.tid / b.tpb;
        if (P.nonempty && P.last_key == e.key) {
            // conflicting categories of b
            const bool cR = cat != CAT_R && true;   // a read conflicts with b unless b is a read
            const bool cW = true;                   // a write always conflicts
            const bool cAD = !cat_atomic(cat);      // device atomics conflict with plain accesses only
            const bool cAB_same = !cat_atomic(cat); // block atomics of b's block: with plain accesses
            bool single = true;
#pragma unroll
            for (int c = 0; c < 4; c++) single = single && !set2_has_other(P.cb[c], blk);
            bool slow = false, group_only = false;
            if (single) {
                if (P.run_blk == blk && P.run_ph == ph) {
                    slow = (cR && set2_has_other(P.rt[CAT_R], e.tid)) || (cW && set2_has_other(P.rt[CAT_W], e.tid)) ||
                           (cAD && set2_has_other(P.rt[CAT_AD], e.tid)) ||
                           (cAB_same && set2_has_other(P.rt[CAT_AB], e.tid));
                    group_only = true;
                }
            } else {
                // some earlier access of the segment is in another block
                const bool cAB_other = cat != CAT_AD;  // block atomics of other blocks: all but device atomics
                slow = (cR && !set2_empty(P.cb[CAT_R])) || (cW && !set2_empty(P.cb[CAT_W])) ||
                       (cAD && !set2_empty(P.cb[CAT_AD])) ||
                       (cAB_same && !set2_empty(P.cb[CAT_AB])) ||
                       (cAB_other && set2_has_other(P.cb[CAT_AB], blk));
            }
            if (slow) {
                BCtx bc;
                bc.idx = e.idx; bc.tid = e.tid; bc.blk = blk; bc.ph = ph; bc.cat = cat; bc.h = NONE;
                slow_check(b, s, rt_scan, (u32)pos, e.key, bc, group_only);
            }
        }
        Agg one;
        agg_one(one, e.key, blk, ph, e.tid, cat);
        agg_combine(P, one);
        P = one;
    }
}

__global__ void k_pairs_kept(Bufs b) {
    if (threadIdx.x == 0) {
        const u32 n = b.prm->n_pairs;
        b.prm->n_pairs_kept = n < b.max_pairs ? n : (u32)b.max_pairs;
    }
}

void segcheck_run(const Bufs &b, const u32 *rt_scan, hipStream_t s) {
    if (!b.N) { RD_LAUNCH("k_pairs_kept", k_pairs_kept, dim3(1), dim3(64), 0, s, b); return; }
    RD_LAUNCH("k_seg_reduce", k_seg_reduce, dim3(b.n_tiles), dim3(WG_THREADS), 0, s, b);
    RD_LAUNCH("k_seg_scan", k_seg_scan, dim3(1), dim3(WG_THREADS), 0, s, b);
    RD_LAUNCH("k_seg_check", k_seg_check, dim3(b.n_tiles), dim3(WG_THREADS), 0, s, b, rt_scan);
    RD_LAUNCH("k_pairs_kept", k_pairs_kept, dim3(1), dim3(64), 0, s, b);
}

}  // namespace rd
