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
// Most accesses cannot race at all, and a prefix summary decides that in O(1).  For the part of the
// segment before b it keeps the categories present (read, write, device atomic, block atomic) and
// whether more than one block appears; for the trailing run of accesses with b's block and phase it
// keeps, for write-ish, plain and all accesses, one thread and whether a second one appears.  If
// every earlier access of the segment is in b's block, only b's run can race with b (earlier phases
// of a block happen before later ones), and only if a conflicting class there has another thread.
// Otherwise b is checked against the earlier accesses one by one (the exact predicate above): by a
// backward walk that stops early when the prefix holds at most two blocks (see lane_walks), else
// by queued chunks of 64 positions, one wavefront each.
// The summaries form a segmented scan: per-tile totals, one scan over tiles, then the tile pass.
#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

enum : u32 {
    F_NONEMPTY = 1u,
    F_HEAD = 2u,        // a location change between two elements of the range
    F_RUNWHOLE = 4u,    // every element of the range is in one run (location, block, phase)
    F_BLKMULTI = 8u,    // two or more blocks in the last segment of the range
    F_CAT0 = 16u,       // bit (4 + category): category present in the last segment
    F_TWA_MULTI = 256u, // two or more threads among the write-ish accesses of the trailing run
    F_TNA_MULTI = 512u, // ... among the plain (non-atomic) accesses
    F_TALL_MULTI = 1024u,
    F_BLK3 = 2048u,     // three or more blocks in the last segment of the range
    F_CATS = 0xf0u,
};

struct Agg {
    u32 first_key, last_key;
    u32 run_blk, run_ph;
    u32 blk, blk2;       // up to two blocks of the last segment (blk2: a second one, or NONE)
    u32 pw1, pa1;        // blk's latest phase + 1 of a write-ish access, of any access (0: none)
    u32 pw2, pa2;        // ... of blk2
    u32 twa, tna, tall;  // a thread of the trailing run: write-ish, plain, any (NONE if none)
    u32 fl;
    u32 first_pos;       // sorted position of the first element of the range
    u32 seg_pos;         // ... of the first element of the last segment
    u32 run_pos;         // ... of the first element of the trailing run
};

size_t agg_bytes() { return sizeof(Agg); }

// a set summarised by one member and a "more than one member" flag
__device__ inline void set1_merge(u32 &v, u32 &fl, u32 multi_bit, u32 ov, u32 ofl) {
    if ((ofl & multi_bit) || (ov != NONE && v != NONE && ov != v)) fl |= multi_bit;
    if (v == NONE) v = ov;
}
// up to two blocks with their latest phases (+1) of write-ish and of any accesses, and a "more
// than two" flag: block x with phases (w, a) joins the set
__device__ inline void blk_add(u32 &b1, u32 &b2, u32 &w1, u32 &a1, u32 &w2, u32 &a2, u32 &fl, u32 x, u32 w, u32 a) {
    if (x == NONE) return;
    if (x == b1) { w1 = max(w1, w); a1 = max(a1, a); }
    else if (x == b2) { w2 = max(w2, w); a2 = max(a2, a); }
    else if (b1 == NONE) { b1 = x; w1 = w; a1 = a; }
    else if (b2 == NONE) { b2 = x; w2 = w; a2 = a; }
    else fl |= F_BLK3;
}
__device__ inline bool set1_has_other(u32 v, u32 fl, u32 multi_bit, u32 x) {
    return (fl & multi_bit) || (v != NONE && v != x);
}

__device__ inline void agg_empty(Agg &a) {
    a.first_key = a.last_key = 0;
    a.run_blk = a.run_ph = 0;
    a.blk = a.blk2 = a.twa = a.tna = a.tall = NONE;
    a.pw1 = a.pa1 = a.pw2 = a.pa2 = 0;
    a.fl = F_RUNWHOLE;
    a.first_pos = a.seg_pos = a.run_pos = 0;
}
__device__ inline void agg_one(Agg &a, u32 key, u32 blk, u32 ph, u32 tid, u32 cat, u32 pos) {
    a.first_pos = a.seg_pos = a.run_pos = pos;
    a.first_key = a.last_key = key;
    a.run_blk = blk; a.run_ph = ph; a.blk = blk; a.blk2 = NONE;
    a.pw1 = cat != CAT_R ? ph + 1 : 0u;
    a.pa1 = ph + 1;
    a.pw2 = a.pa2 = 0;
    a.tall = tid;
    a.twa = cat != CAT_R ? tid : NONE;
    a.tna = cat <= CAT_W ? tid : NONE;
    a.fl = F_NONEMPTY | F_RUNWHOLE | (F_CAT0 << cat);
}
// r := l (+) r, l before r
__device__ inline void agg_combine(const Agg &l, Agg &r) {
    if (!(l.fl & F_NONEMPTY)) return;
    if (!(r.fl & F_NONEMPTY)) { r = l; return; }
    const bool keychange = r.first_key != l.last_key;
    const bool boundary = (r.fl & F_HEAD) || keychange;
    const bool extend = !boundary && (r.fl & F_RUNWHOLE) && r.run_blk == l.run_blk && r.run_ph == l.run_ph;
    u32 fl = F_NONEMPTY | ((l.fl | r.fl) & F_HEAD) | (keychange ? F_HEAD : 0u);
    if (!boundary) {
        // the blocks of the segment (up to two tracked) with their latest phases: phases of one
        // block at one location never decrease in trace order, so the latest is the largest
        u32 bfl = (l.fl | r.fl) & (F_BLKMULTI | F_BLK3);
        u32 bv = l.blk, bv2 = l.blk2, w1 = l.pw1, a1 = l.pa1, w2 = l.pw2, a2 = l.pa2;
        blk_add(bv, bv2, w1, a1, w2, a2, bfl, r.blk, r.pw1, r.pa1);
        blk_add(bv, bv2, w1, a1, w2, a2, bfl, r.blk2, r.pw2, r.pa2);
        if (bv2 != NONE) bfl |= F_BLKMULTI;
        fl |= bfl | ((l.fl | r.fl) & F_CATS);
        r.blk = bv;
        r.blk2 = bv2;
        r.pw1 = w1; r.pa1 = a1; r.pw2 = w2; r.pa2 = a2;
    } else {
        fl |= r.fl & (F_BLKMULTI | F_BLK3 | F_CATS);
    }
    if (extend) {
        u32 tfl = (l.fl | r.fl) & (F_TWA_MULTI | F_TNA_MULTI | F_TALL_MULTI);
        u32 a = l.twa, b = l.tna, c = l.tall;
        set1_merge(a, tfl, F_TWA_MULTI, r.twa, 0);
        set1_merge(b, tfl, F_TNA_MULTI, r.tna, 0);
        set1_merge(c, tfl, F_TALL_MULTI, r.tall, 0);
        r.twa = a; r.tna = b; r.tall = c;
        fl |= tfl | (l.fl & F_RUNWHOLE);
    } else {
        fl |= r.fl & (F_TWA_MULTI | F_TNA_MULTI | F_TALL_MULTI);
    }
    r.fl = fl;
    r.first_key = l.first_key;
    if (!boundary) r.seg_pos = l.seg_pos;
    if (extend) r.run_pos = l.run_pos;
    r.first_pos = l.first_pos;
}

// ---------------------------------------------------------------- shared pieces

// Thread x of a tile owns the ITEMS consecutive elements [tile*TILE + x*ITEMS, +ITEMS).
struct Items {
    u32 key[ITEMS], tid[ITEMS], info[ITEMS];
};

__device__ inline void load_items(const SegCtx &s, u64 base, Items &it) {
    if (base + ITEMS <= s.n) {
#pragma unroll
        for (int q = 0; q < ITEMS; q += 4) {
            const uint4 k4 = *(const uint4 *)(s.k + base + q);
            const uint4 t4 = *(const uint4 *)(s.t + base + q);
            it.key[q] = k4.x; it.key[q + 1] = k4.y; it.key[q + 2] = k4.z; it.key[q + 3] = k4.w;
            it.tid[q] = t4.x; it.tid[q + 1] = t4.y; it.tid[q + 2] = t4.z; it.tid[q + 3] = t4.w;
            if (!s.packed && !s.tinfo) {
                const uint4 f4 = *(const uint4 *)(s.f + base + q);
                it.info[q] = f4.x; it.info[q + 1] = f4.y; it.info[q + 2] = f4.z; it.info[q + 3] = f4.w;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < ITEMS; q++) {
            const u64 pos = base + q;
            const bool in = pos < s.n;
            it.key[q] = in ? s.k[pos] : 0;
            it.tid[q] = in ? s.t[pos] : 0;
            it.info[q] = in && !s.packed && !s.tinfo ? s.f[pos] : 0;
        }
    }
    if (s.packed) {
#pragma unroll
        for (int q = 0; q < ITEMS; q++) {
            it.info[q] = packed_info(it.key[q], s.key_bits);
            it.key[q] &= s.kmask;
        }
    } else if (s.tinfo) {
#pragma unroll
        for (int q = 0; q < ITEMS; q++) {
            it.info[q] = packed_info(it.tid[q], s.tbits);
            it.tid[q] &= s.tmask;
        }
    }
}

__device__ inline void items_agg(const Bufs &b, const Items &it, u32 cnt, u32 base, Agg &acc) {
    agg_empty(acc);
#pragma unroll
    for (int q = 0; q < ITEMS; q++) {
        if ((u32)q < cnt) {
            Agg one;
            agg_one(one, it.key[q], block_of(b, it.tid[q]), info_phase(it.info[q]), it.tid[q], info_cat(it.info[q]),
                    base + q);
            agg_combine(acc, one);
            acc = one;
        }
    }
}

__device__ inline Agg shfl_up_agg(const Agg &a, u32 d) {
    Agg r;
    r.first_key = __shfl_up(a.first_key, d, 64);
    r.last_key = __shfl_up(a.last_key, d, 64);
    r.run_blk = __shfl_up(a.run_blk, d, 64);
    r.run_ph = __shfl_up(a.run_ph, d, 64);
    r.blk = __shfl_up(a.blk, d, 64);
    r.blk2 = __shfl_up(a.blk2, d, 64);
    r.pw1 = __shfl_up(a.pw1, d, 64);
    r.pa1 = __shfl_up(a.pa1, d, 64);
    r.pw2 = __shfl_up(a.pw2, d, 64);
    r.pa2 = __shfl_up(a.pa2, d, 64);
    r.twa = __shfl_up(a.twa, d, 64);
    r.tna = __shfl_up(a.tna, d, 64);
    r.tall = __shfl_up(a.tall, d, 64);
    r.fl = __shfl_up(a.fl, d, 64);
    r.first_pos = __shfl_up(a.first_pos, d, 64);
    r.seg_pos = __shfl_up(a.seg_pos, d, 64);
    r.run_pos = __shfl_up(a.run_pos, d, 64);
    return r;
}

// Inclusive scan over the lanes of a wavefront: lane i gets a_0 (+) ... (+) a_i.
__device__ inline void wave_inscan_agg(Agg &v) {
    const u32 lane = lane_id();
#pragma unroll
    for (u32 d = 1; d < 64; d <<= 1) {
        const Agg o = shfl_up_agg(v, d);
        if (lane >= d) agg_combine(o, v);
    }
}

// Block-wide (NT threads) exclusive scan of Aggs: each wavefront scans its lanes with shuffles,
// one wavefront scans the wavefront totals (wtot, NT / 64 entries of LDS).  `mine` becomes this
// thread's exclusive prefix, *total (when non-null) the block total.
template <u32 NT = WG_THREADS>
__device__ inline void block_exscan_agg(Agg &mine, Agg *wtot /* NT / 64 */, Agg *total) {
    constexpr u32 W = NT / 64;
    static_assert(W >= 1 && W <= 64, "one wavefront scans the wavefront totals");
    const u32 lane = lane_id(), w = threadIdx.x >> 6;
    Agg inc = mine;
    wave_inscan_agg(inc);
    if (lane == 63) wtot[w] = inc;
    __syncthreads();
    if (w == 0) {
        Agg t;
        if (lane < W) t = wtot[lane];
        else agg_empty(t);
        wave_inscan_agg(t);
        if (lane < W) wtot[lane] = t;
    }
    __syncthreads();
    Agg ex = shfl_up_agg(inc, 1);
    if (lane == 0) agg_empty(ex);
    if (w > 0) {
        const Agg pw = wtot[w - 1];
        agg_combine(pw, ex);
    }
    if (total) *total = wtot[W - 1];
    __syncthreads();  // wtot is free for the caller again
    mine = ex;
}

__device__ inline u32 items_in(const SegCtx &s, u64 base) {
    return base >= s.n ? 0u : (u32)min((u64)ITEMS, s.n - base);
}

__global__ __launch_bounds__(WG_THREADS) void k_seg_reduce(Bufs b) {
    __shared__ Agg buf[WAVES];
    const SegCtx s = seg_ctx(b);
    if (check_abandoned(b.prm)) return;  // the answer is that error: nothing here is read
    Agg *tile_agg = (Agg *)b.tile_agg;
    const u64 tile0 = (u64)blockIdx.x * TILE;
    if (tile0 >= s.n) return;
    const u64 base = tile0 + (u64)threadIdx.x * ITEMS;
    Items it;
    load_items(s, base, it);
    Agg mine;
    items_agg(b, it, items_in(s, base), (u32)base, mine);
    Agg own = mine;
    block_exscan_agg(mine, buf, nullptr);
    if (threadIdx.x == WG_THREADS - 1) {  // tile total = last thread's prefix (+) its own items
        agg_combine(mine, own);
        tile_agg[blockIdx.x] = own;
    }
}

// exclusive scan over the tile totals (workgroups of SCAN_THREADS)
constexpr u32 SCAN_THREADS = 1024;

// Four consecutive summaries (a range starting at a multiple of four tiles) are AGG_WORDS aligned
// 16-byte vectors: loaded and stored as such.
constexpr int AGG_WORDS = (int)(sizeof(Agg) / 4);
static_assert(sizeof(Agg) % 4 == 0, "a summary is whole words");
__device__ inline void agg_load4(const Agg *src, Agg v[4]) {
    u32 w[4 * AGG_WORDS];
    const uint4 *p = (const uint4 *)src;
#pragma unroll
    for (int k = 0; k < AGG_WORDS; k++) {
        const uint4 x = p[k];
        w[4 * k] = x.x; w[4 * k + 1] = x.y; w[4 * k + 2] = x.z; w[4 * k + 3] = x.w;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) __builtin_memcpy(&v[j], &w[AGG_WORDS * j], sizeof(Agg));
}
__device__ inline void agg_store4(Agg *dst, const Agg v[4]) {
    u32 w[4 * AGG_WORDS];
#pragma unroll
    for (int j = 0; j < 4; j++) __builtin_memcpy(&w[AGG_WORDS * j], &v[j], sizeof(Agg));
    uint4 *p = (uint4 *)dst;
#pragma unroll
    for (int k = 0; k < AGG_WORDS; k++) p[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
}

// The tiles' exclusive prefixes in three launches: every workgroup scans a chunk of SCAN_CHUNK
// tiles (four per thread) for its total, one workgroup scans the chunk totals, and every workgroup
// scans its chunk again from its chunk's prefix and stores the tiles' prefixes.  The chunk totals
// live after the tile summaries.
constexpr u32 SCAN_PER = 4;
constexpr u32 SCAN_CHUNK = SCAN_THREADS * SCAN_PER;

__device__ inline u32 scan_tiles(const SegCtx &s) { return (u32)((s.n + TILE - 1) / TILE); }

// This thread's (up to) four tiles of chunk blockIdx.x, loaded; the number in range.
__device__ inline u32 chunk_load(const Agg *tile_agg, u32 nt, Agg v[4]) {
    const u32 q = blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_PER;
    if (q >= nt) return 0;
    if (q + 4 <= nt) {
        agg_load4(tile_agg + q, v);
        return 4;
    }
#pragma unroll
    for (u32 j = 0; j < 4; j++)
        if (q + j < nt) v[j] = tile_agg[q + j];
    return nt - q;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_seg_scan_up(Bufs b) {
    __shared__ Agg buf[SCAN_THREADS / 64];
    const SegCtx s = seg_ctx(b);
    if (check_abandoned(b.prm)) return;  // the answer is that error: nothing here is read
    const u32 nt = scan_tiles(s);
    if (blockIdx.x * SCAN_CHUNK >= nt) return;
    Agg *tile_agg = (Agg *)b.tile_agg, *chunk_tot = tile_agg + b.n_tiles + 1;
    Agg v[4], acc;
    agg_empty(acc);
    const u32 m = chunk_load(tile_agg, nt, v);
#pragma unroll
    for (u32 j = 0; j < 4; j++)
        if (j < m) { agg_combine(acc, v[j]); acc = v[j]; }
    Agg total;
    block_exscan_agg<SCAN_THREADS>(acc, buf, &total);
    if (threadIdx.x == 0) chunk_tot[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_seg_scan_top(Bufs b) {
    __shared__ Agg buf[SCAN_THREADS / 64];
    const SegCtx s = seg_ctx(b);
    if (check_abandoned(b.prm)) return;
    const u32 nc = (scan_tiles(s) + SCAN_CHUNK - 1) / SCAN_CHUNK;
    Agg *chunk_tot = (Agg *)b.tile_agg + b.n_tiles + 1;
    // each thread a contiguous range of chunks
    const u32 per = (nc + SCAN_THREADS - 1) / SCAN_THREADS;
    const u32 lo = min(threadIdx.x * per, nc), hi = min(lo + per, nc);
    Agg acc;
    agg_empty(acc);
    for (u32 c = lo; c < hi; c++) {
        Agg v = chunk_tot[c];
        agg_combine(acc, v);
        acc = v;
    }
    block_exscan_agg<SCAN_THREADS>(acc, buf, nullptr);
    for (u32 c = lo; c < hi; c++) {
        Agg t = chunk_tot[c];
        chunk_tot[c] = acc;
        agg_combine(acc, t);
        acc = t;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_seg_scan_down(Bufs b) {
    __shared__ Agg buf[SCAN_THREADS / 64];
    const SegCtx s = seg_ctx(b);
    if (check_abandoned(b.prm)) return;
    const u32 nt = scan_tiles(s);
    if (blockIdx.x * SCAN_CHUNK >= nt) return;
    Agg *tile_agg = (Agg *)b.tile_agg;
    const Agg *chunk_tot = tile_agg + b.n_tiles + 1;
    Agg acc;
    agg_empty(acc);
    u32 m;
    {
        Agg v[4];
        m = chunk_load(tile_agg, nt, v);
#pragma unroll
        for (u32 j = 0; j < 4; j++)
            if (j < m) { agg_combine(acc, v[j]); acc = v[j]; }
    }
    block_exscan_agg<SCAN_THREADS>(acc, buf, nullptr);  // everything of the chunk before this thread
    {
        Agg pc = chunk_tot[blockIdx.x];                 // everything before the chunk
        agg_combine(pc, acc);
    }
    // the totals in (read again, one at a time), the exclusive prefixes out
    const u32 q = blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_PER;
    for (u32 j = 0; j < m; j++) {
        Agg t = tile_agg[q + j];
        tile_agg[q + j] = acc;
        agg_combine(acc, t);
        acc = t;
    }
}

// ---------------------------------------------------------------- the check

__device__ inline bool cat_write(u32 c) { return c != CAT_R; }
__device__ inline bool cat_atomic(u32 c) { return c >= CAT_AD; }

__device__ inline bool conflicts(u32 ca, u32 ba, u32 cb, u32 bb) {
    if (!cat_write(ca) && !cat_write(cb)) return false;
    if (cat_atomic(ca) && cat_atomic(cb) && (ca == CAT_AD || cb == CAT_AD || ba == bb)) return false;
    return true;
}

// categories of earlier accesses that can conflict with an access of category c
__device__ inline u32 conflict_cats(u32 c) {
    // R: W AD AB ; W: all ; AD: R W ; AB: R W AB (block atomics of other blocks)
    const u32 R = F_CAT0 << CAT_R, W = F_CAT0 << CAT_W, AD = F_CAT0 << CAT_AD, AB = F_CAT0 << CAT_AB;
    return c == CAT_R ? (W | AD | AB) : c == CAT_W ? (R | W | AD | AB) : c == CAT_AD ? (R | W) : (R | W | AB);
}

// Does a (thread ta, block ba, phase pha, index ia) happen before b?  h: knowledge vector of b's
// thread at b, looked up on first use (NONE until then).
__device__ inline bool happens_before(const Bufs &b, const u32 *rt_scan, u32 bidx, u32 btid, u32 bblk, u32 bph,
                                      u32 &h, u32 ta, u32 ba, u32 pha, u32 ia) {
    if (ba == bblk && pha < bph) return true;
    if (!(b.prm->mode & MODE_SYNC)) return false;
    if (h == NONE) h = knowledge_at(b, btid, bidx, bblk, bph);
    if (!h) return false;
    const u32 *V = b.pool + (u64)h * b.prm->D;
    if (V[ba] > pha) return true;
    if (rt_scan[ta + 1] > rt_scan[ta]) {
        const u32 col = b.B + rt_scan[ta];
        if (V[col] >= ia + 1) return true;
    }
    return false;
}

// Appends (first, second) for every lane with `want`; one atomic per wavefront.  All lanes of the
// wavefront must call it.
__device__ inline void emit_wave(const Bufs &b, bool want, u32 first, u32 second) {
    const u64 m = ballot(want);
    if (!m) return;
    const u32 leader = (u32)__builtin_ctzll(m);
    u32 base = 0;
    if (lane_id() == leader) base = atomicAdd(&b.prm->n_pairs, popc64(m));
    base = __shfl(base, leader, 64);
    if (want) {
        const u32 slot = base + popc64(m & lanemask_lt());
        if (slot < b.max_pairs) { b.pfirst[0][slot] = first; b.psecond[0][slot] = second; }
        else atomicOr(&b.prm->err, ERR_PAIRS);
    }
}

// Checks b (at sorted position pos) against the earlier accesses of its segment, with the whole
// wavefront: each step examines the 64 positions below `top` at once, a ballot finds the first
// position that leaves the segment (or b's block-and-phase run when group_only), and the lanes
// before it apply the exact predicate.  Every lane calls this with the same arguments.
__device__ inline void wave_slow_check(const Bufs &b, const SegCtx &s, const u32 *rt_scan, u32 pos, u32 key,
                                       u32 btid, u32 bblk, u32 bph, u32 bcat, bool group_only) {
    const u32 lane = lane_id();
    const u32 bidx = s.i[pos];
    u32 h = NONE;
    for (u32 top = pos; top > 0; top = top > 64 ? top - 64 : 0) {
        const bool valid = lane < top;
        const u32 q = valid ? top - 1 - lane : 0;
        bool stop = !valid;
        u32 ta = 0, info = 0, ba = 0, pha = 0;
        if (valid) {
            stop = seg_key(s, q) != key;
            if (!stop) {
                ta = seg_tid(s, q);
                info = seg_info(s, q);
                ba = block_of(b, ta);
                pha = info_phase(info);
                if (group_only && (ba != bblk || pha != bph)) stop = true;
            }
        }
        const u64 sm = ballot(stop);
        const u32 first_stop = sm ? (u32)__builtin_ctzll(sm) : 64u;
        bool want = false;
        u32 ia = 0;
        if (lane < first_stop && ta != btid && conflicts(info_cat(info), ba, bcat, bblk)) {
            ia = s.i[q];
            want = !happens_before(b, rt_scan, bidx, btid, bblk, bph, h, ta, ba, pha, ia);
        }
        emit_wave(b, want, ia, bidx);
        if (sm) break;
    }
}

// How an access b is checked against the earlier accesses of its segment.
enum : u32 {
    SLOW_NONE = 0,  // no earlier access can race with b
    SLOW_RUN = 1,   // only b's run (same block and phase) can: chunks over the run
    SLOW_SEG = 2,   // three or more blocks before b: chunks over the whole segment prefix
    SLOW_WALK = 3,  // one or two blocks before b: a backward walk that stops early
    SLOW_KNOW = 4,  // one or two other blocks have conflicting accesses, b's own block none in b's
                    // phase: none races if b's thread knows each such block's latest conflicting
                    // phase (bits 8 and 9: which of the summary's two blocks), else SLOW_WALK
};

// Does b's thread have knowledge at b (at sorted position pos)?  Without it no other block can be
// settled, and a walk would only be a slower way to scan the whole prefix.
__device__ inline bool knows_at(const Bufs &b, const SegCtx &s, u32 tid, u32 pos) {
    return (b.prm->mode & MODE_SYNC) && b.t_kfirst[tid] != NONE && b.t_kfirst[tid] < s.i[pos];
}

// P: summary of everything before b (b's own segment when P.last_key == key).
__device__ inline u32 decide(const Agg &P, u32 key, u32 tid, u32 blk, u32 ph, u32 cat) {
    if (!(P.fl & F_NONEMPTY) || P.last_key != key) return SLOW_NONE;
    if (!(P.fl & F_BLKMULTI) && P.blk == blk) {
        // every earlier access is in b's block: only b's run is unordered with b
        if (P.run_blk != blk || P.run_ph != ph) return SLOW_NONE;
        bool slow;
        if (cat == CAT_R) slow = set1_has_other(P.twa, P.fl, F_TWA_MULTI, tid);
        else if (cat == CAT_W) slow = set1_has_other(P.tall, P.fl, F_TALL_MULTI, tid);
        else slow = set1_has_other(P.tna, P.fl, F_TNA_MULTI, tid);
        return slow ? SLOW_RUN : SLOW_NONE;
    }
    if (!(P.fl & conflict_cats(cat))) return SLOW_NONE;
    if (P.fl & F_BLK3) return SLOW_SEG;
    // one or two blocks: the latest phase (+1) of each one's accesses that can conflict with b
    // (write-ish ones for a read, any for the others: a superset for atomics)
    const u32 l1 = cat == CAT_R ? P.pw1 : P.pa1, l2 = cat == CAT_R ? P.pw2 : P.pa2;
    u32 need = 0;
    if (l1) {
        if (P.blk != blk) need |= 1u << 8;
        else if (l1 - 1 >= ph) return SLOW_WALK;  // b's block in b's phase: threads decide
    }
    if (l2 && P.blk2 != NONE) {
        if (P.blk2 != blk) need |= 1u << 9;
        else if (l2 - 1 >= ph) return SLOW_WALK;
    }
    return need ? (SLOW_KNOW | need) : SLOW_NONE;
}

// SLOW_KNOW: each other block with conflicting accesses is ordered before b when b's thread knows a
// later phase of it than its latest conflicting access (the accesses of one block to one location
// have non-decreasing phase); otherwise the walk decides.
__device__ inline u32 settle_known(const Bufs &b, const SegCtx &s, const Agg &P, u32 mode, u32 tid, u32 blk, u32 ph,
                                   u32 cat, u32 pos) {
    if (!(b.prm->mode & MODE_SYNC)) return SLOW_WALK;
    const u32 h = knowledge_at(b, tid, s.i[pos], blk, ph);
    if (!h) return SLOW_WALK;
    const u32 *V = b.pool + (u64)h * b.prm->D;
    if (mode & (1u << 8)) {
        const u32 l = cat == CAT_R ? P.pw1 : P.pa1;
        if (V[P.blk] < l) return SLOW_WALK;  // V[X] > latest phase, i.e. V[X] >= l
    }
    if (mode & (1u << 9)) {
        const u32 l = cat == CAT_R ? P.pw2 : P.pa2;
        if (V[P.blk2] < l) return SLOW_WALK;
    }
    return SLOW_NONE;
}

// Queue entries, one wavefront each: chunk (pos, lo, hi) = check b at pos against positions [lo, hi).
constexpr u32 LANE_WALK_CAP = 16;  // positions a lane walks before the rest is queued as chunks
constexpr u32 LANE_STEP = 4;       // positions a lane loads at once

// Pairs found by one wavefront, gathered in LDS and appended with one device atomic per flush.
constexpr u32 WAVE_PAIRS = 512;

struct WavePairs {
    u32 *pf, *ps;
    u32 fill;  // the same in every lane
};

__device__ inline void wp_flush(const Bufs &b, WavePairs &w) {
    if (!w.fill) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    u32 g = 0;
    if (lane_id() == 0) g = atomicAdd(&b.prm->n_pairs, w.fill);
    g = __shfl(g, 0, 64);
    for (u32 k = lane_id(); k < w.fill; k += 64) {
        const u32 slot = g + k;
        if (slot < b.max_pairs) { b.pfirst[0][slot] = w.pf[k]; b.psecond[0][slot] = w.ps[k]; }
        else atomicOr(&b.prm->err, ERR_PAIRS);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    w.fill = 0;
}

// Every lane of the wavefront calls this.
__device__ inline void wp_add(const Bufs &b, WavePairs &w, bool want, u32 first, u32 second) {
    const u64 m = ballot(want);
    if (!m) return;
    if (w.fill + popc64(m) > WAVE_PAIRS) wp_flush(b, w);
    if (want) {
        const u32 o = w.fill + popc64(m & lanemask_lt());
        w.pf[o] = first;
        w.ps[o] = second;
    }
    w.fill += popc64(m);
}

// The access b at sorted position pos, for the walks.
struct Walker {
    u32 pos, key, btid, bidx, bblk, bph, bcat;
    u32 h;          // knowledge handle of b's thread at b (0: none)
    const u32 *V;   // its vector, or null
};

__device__ inline Walker walker_at(const Bufs &b, const SegCtx &s, u32 pos) {
    Walker w;
    w.pos = pos;
    w.key = seg_key(s, pos);
    w.btid = seg_tid(s, pos);
    w.bidx = s.i[pos];
    const u32 info = seg_info(s, pos);
    w.bblk = block_of(b, w.btid);
    w.bph = info_phase(info);
    w.bcat = info_cat(info);
    w.h = 0;
    if (b.prm->mode & MODE_SYNC) w.h = knowledge_at(b, w.btid, w.bidx, w.bblk, w.bph);
    w.V = w.h ? b.pool + (u64)w.h * b.prm->D : nullptr;
    return w;
}

// The walks rest on one fact: the accesses of one block to one location appear in trace order with
// non-decreasing phase, because a valid trace completes every arrival at a barrier instance before
// any event after that instance (Section 5).  So once a backward walk meets an access of block X
// that happens before b through a barrier or through b's block knowledge -- X is b's block and
// the phase is lower, or b's thread knows a later phase of X -- every earlier access of X happens
// before b as well: X is settled.  The walk ends when all nb blocks of the prefix are settled.
__device__ inline bool settles(const Walker &w, u32 ba, u32 pha) {
    return ba == w.bblk ? pha < w.bph : (w.V != nullptr && w.V[ba] > pha);
}

// Is a (thread ta, block ba, phase pha, category ca, sorted position q) a race with b?
__device__ inline bool walk_race(const Bufs &b, const SegCtx &s, const u32 *rt_scan, const Walker &w, u32 q,
                                 u32 ta, u32 ba, u32 pha, u32 ca, u32 &ia) {
    if (ta == w.btid || !conflicts(ca, ba, w.bcat, w.bblk)) return false;
    ia = s.i[q];
    u32 h = w.h;
    return !happens_before(b, rt_scan, w.bidx, w.btid, w.bblk, w.bph, h, ta, ba, pha, ia);
}

// Block-wide (256 threads) exclusive scan of one u64 per thread; *total gets the sum.
__device__ inline u64 block_exscan_u64(u64 v, u64 *wsum /* WAVES */, u64 &total) {
    const u32 lane = lane_id(), w = threadIdx.x >> 6;
    u64 incl = v;
    for (u32 d = 1; d < 64; d <<= 1) {
        const u64 o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    u64 off = 0;
    total = 0;
    for (u32 k = 0; k < (u32)WAVES; k++) {
        const u64 x = wsum[k];
        if (k < w) off += x;
        total += x;
    }
    return off + incl - v;
}

// Queues the rest of a walk -- b against positions [segment start, top) -- as chunks; false when the
// queue is full (the walk then goes on).  The segment start is found by a binary search.
__device__ inline bool walk_spill(const Bufs &b, const SegCtx &s, const Walker &w, u32 top) {
    u32 lo = 0, hi = top;
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (seg_key(s, mid) < w.key) lo = mid + 1;
        else hi = mid;
    }
    const u32 cnt = (top - lo + 63) / 64;
    if (!cnt) return true;
    const u64 c0 = atomicAdd(&b.prm->n_chunks, (unsigned long long)cnt);
    if (c0 + cnt > s.n) {
        // neutralise the reserved slots below the capacity (the chunk kernel reads them)
        for (u64 c = c0; c < c0 + cnt && c < s.n; c++) { s.cpos[c] = 0; s.clo[c] = 0; s.chi[c] = 0; }
        return false;
    }
    for (u32 k = 0; k < cnt; k++) {
        const u32 c_lo = lo + 64 * k;
        s.cpos[c0 + k] = w.pos; s.clo[c0 + k] = c_lo; s.chi[c0 + k] = min(c_lo + 64, top);
    }
    return true;
}

// The walks of a lane's items (walk_bits; two_bits: the prefix has two blocks), one at a time: a
// lane takes its next item when its walk ends, and loads LANE_STEP positions at once.  All lanes
// of the wavefront call it.
__device__ void lane_walks(const Bufs &b, const SegCtx &s, const u32 *rt_scan, u64 base, u32 walk_bits,
                           u32 two_bits, WavePairs &wp) {
    bool act = false, d1 = false, d2 = false;
    Walker w = {};
    u32 nb = 1, x1 = NONE, top = 0, steps = 0;
    while (true) {
        if (!act && walk_bits) {
            const u32 q = (u32)__builtin_ctz(walk_bits);
            walk_bits &= walk_bits - 1;
            w = walker_at(b, s, (u32)(base + q));
            nb = (two_bits >> q) & 1u ? 2u : 1u;
            x1 = NONE;
            d1 = d2 = false;
            top = w.pos;
            steps = 0;
            act = true;
        }
        if (!ballot(act)) break;
        u32 kq[LANE_STEP], tq[LANE_STEP], fq[LANE_STEP];
#pragma unroll
        for (u32 j = 0; j < LANE_STEP; j++) {
            const bool ok = act && top > j;
            const u32 q = ok ? top - 1 - j : 0u;
            kq[j] = ok ? seg_key(s, q) : w.key ^ 1u;
            tq[j] = ok ? seg_tid(s, q) : 0u;
            fq[j] = ok ? seg_info(s, q) : 0u;
        }
#pragma unroll
        for (u32 j = 0; j < LANE_STEP; j++) {
            bool want = false;
            u32 ia = 0;
            if (act) {
                if (kq[j] != w.key) {
                    act = false;
                } else {
                    const u32 q = top - 1, ta = tq[j], info = fq[j];
                    const u32 ba = block_of(b, ta), pha = info_phase(info);
                    if (x1 == NONE) x1 = ba;
                    want = walk_race(b, s, rt_scan, w, q, ta, ba, pha, info_cat(info), ia);
                    if (settles(w, ba, pha)) {
                        if (ba == x1) d1 = true;
                        else d2 = true;
                    }
                    top = q;
                    if ((d1 && (nb < 2 || d2)) || top == 0) act = false;
                    else if (++steps == LANE_WALK_CAP && walk_spill(b, s, w, top)) act = false;
                }
            }
            wp_add(b, wp, want, ia, w.bidx);
        }
    }
}

constexpr u64 LOW48 = (1ull << 48) - 1;

union CheckLds {
    Agg buf[WAVES];
    struct { u32 pf[WAVES][WAVE_PAIRS], ps[WAVES][WAVE_PAIRS]; } pairs;
};

__global__ __launch_bounds__(WG_THREADS) void k_seg_check(Bufs b, const u32 *rt_scan) {
    __shared__ CheckLds L;
    __shared__ u64 wsum[WAVES];
    __shared__ u64 qbase;
    __shared__ u32 lbase;
    const SegCtx s = seg_ctx(b);
    if (check_abandoned(b.prm)) return;  // the answer is that error: nothing here is read
    const Agg *tile_agg = (const Agg *)b.tile_agg;
    const u64 tile0 = (u64)blockIdx.x * TILE;
    if (tile0 >= s.n) return;
    const u64 base = tile0 + (u64)threadIdx.x * ITEMS;
    const u32 lane = lane_id(), wv = threadIdx.x >> 6;
    Items it;
    load_items(s, base, it);
    const u32 cnt = items_in(s, base);
    Agg P0;
    items_agg(b, it, cnt, (u32)base, P0);
    block_exscan_agg(P0, L.buf, nullptr);
    {
        Agg T = tile_agg[blockIdx.x];  // everything before this tile
        agg_combine(T, P0);            // P0 := T (+) P0: everything before this thread's items
    }
    // pass 1: decisions in O(1) per item; the chunks that run, many-block and unsettleable items need
    u64 need = 0;
    u32 chunk_bits = 0, run_bits = 0, walk_bits = 0, two_bits = 0;
    {
        Agg P = P0;
#pragma unroll
        for (int q = 0; q < ITEMS; q++) {
            if ((u32)q >= cnt) continue;
            const u32 key = it.key[q], tid = it.tid[q], info = it.info[q];
            const u32 cat = info_cat(info), ph = info_phase(info), blk = block_of(b, tid);
            const u32 pos = (u32)(base + q);
            u32 mode = decide(P, key, tid, blk, ph, cat);
            if ((mode & 0xffu) == SLOW_KNOW) mode = settle_known(b, s, P, mode, tid, blk, ph, cat, pos);
            if (mode == SLOW_WALK && knows_at(b, s, tid, pos)) {
                walk_bits |= 1u << q;
                if (P.fl & F_BLKMULTI) two_bits |= 1u << q;
            } else if (mode != SLOW_NONE) {
                need += (pos - (mode == SLOW_RUN ? P.run_pos : P.seg_pos) + 63) / 64;
                chunk_bits |= 1u << q;
                if (mode == SLOW_RUN) run_bits |= 1u << q;
            }
            Agg one;
            agg_one(one, key, blk, ph, tid, cat, pos);
            agg_combine(P, one);
            P = one;
        }
    }
    // chunks (low 48 bits: at most 4,096 items of fewer than 2^26 chunks each) and chunk items
    u64 total;
    const u64 packed_off = block_exscan_u64(need | ((u64)__builtin_popcount(chunk_bits) << 48), wsum, total);
    const u64 off = packed_off & LOW48, item_off = packed_off >> 48;
    const u64 total_items = total >> 48;
    total &= LOW48;
    const bool any_walk = __syncthreads_or(walk_bits != 0);  // (also ends the use of L.buf)
    if (!total && !any_walk) return;
    if (threadIdx.x == 0) {
        qbase = ~0ull;
        lbase = NONE;
        if (total) {
            const u64 c0 = atomicAdd(&b.prm->n_chunks, (unsigned long long)total);
            if (c0 + total <= s.n) qbase = c0;
            else {
                // no room: neutralise the reserved slots below the capacity (the chunk kernel reads
                // min(counter, capacity) slots) and queue the tile's chunk items whole; an access is
                // queued whole at most once, so that queue (as long as the elements) has room
                for (u64 c = c0; c < c0 + total && c < s.n; c++) { s.cpos[c] = 0; s.clo[c] = 0; s.chi[c] = 0; }
                if (s.n <= 0x80000000u) {
                    const u32 l0 = atomicAdd(&b.prm->n_long, (u32)total_items);
                    if ((u64)l0 + total_items <= s.n) lbase = l0;
                }
            }
        }
    }
    __syncthreads();
    if (lbase != NONE) {
        u32 e = lbase + (u32)item_off;
#pragma unroll
        for (int q = 0; q < ITEMS; q++)
            if (chunk_bits & (1u << q)) s.lpos[e++] = (u32)(base + q) | ((run_bits >> q) & 1u) << 31;
        chunk_bits = 0;
    } else if (qbase != ~0ull) {
        // pass 2: the same decisions, chunks written to the queue at this thread's offset
        u64 e = qbase + off;
        Agg P = P0;
#pragma unroll
        for (int q = 0; q < ITEMS; q++) {
            if ((u32)q >= cnt) continue;
            const u32 key = it.key[q], tid = it.tid[q], info = it.info[q];
            const u32 cat = info_cat(info), ph = info_phase(info), blk = block_of(b, tid);
            const u32 pos = (u32)(base + q);
            if (chunk_bits & (1u << q)) {
                const u32 start = (run_bits & (1u << q)) ? P.run_pos : P.seg_pos;
                for (u32 lo = start; lo < pos; lo += 64, e++) {
                    s.cpos[e] = pos; s.clo[e] = lo; s.chi[e] = min(lo + 64, pos);
                }
            }
            Agg one;
            agg_one(one, key, blk, ph, tid, cat, pos);
            agg_combine(P, one);
            P = one;
        }
        chunk_bits = 0;
    }
    WavePairs wp;
    wp.pf = L.pairs.pf[wv];
    wp.ps = L.pairs.ps[wv];
    wp.fill = 0;
    // both queues full: each wavefront checks its lanes' chunk items by exact scans, of the run or
    // of the whole segment prefix
    for (u32 q = 0; q < (u32)ITEMS; q++) {
        u64 m = ballot((chunk_bits >> q) & 1u);
        const u64 mr = ballot((run_bits >> q) & 1u);
        while (m) {
            const u32 l = (u32)__builtin_ctzll(m);
            m &= m - 1;
            const u32 pos = (u32)(tile0 + (u64)(wv * 64 + l) * ITEMS + q);
            const u32 tid = seg_tid(s, pos), info = seg_info(s, pos);
            wave_slow_check(b, s, rt_scan, pos, seg_key(s, pos), tid, block_of(b, tid), info_phase(info),
                            info_cat(info), (mr >> l) & 1u);
        }
    }
    // the walks
    lane_walks(b, s, rt_scan, base, walk_bits, two_bits, wp);
    wp_flush(b, wp);
}

// One wavefront per queued chunk (lane l checks position lo + l against b), the four wavefronts of
// a workgroup in step; pairs are gathered in LDS and appended with one device atomic per flush of
// the workgroup.  Then one wavefront per access queued whole: an exact backward scan of its segment
// (or of its run), each wavefront on its own.
constexpr u32 PAIR_LDS = 2048;
constexpr u32 SLOW_GRID = 1024;

__global__ __launch_bounds__(WG_THREADS) void k_seg_slow(Bufs b, const u32 *rt_scan) {
    __shared__ u32 pf[PAIR_LDS], ps[PAIR_LDS];
    __shared__ u32 fill, gbase;
    const SegCtx s = seg_ctx(b);
    if (check_abandoned(b.prm)) return;  // the answer is that error: nothing here is read
    const u32 n_chunks = (u32)min(b.prm->n_chunks, (unsigned long long)s.n);
    const u32 lane = lane_id(), w = threadIdx.x >> 6;
    if (threadIdx.x == 0) fill = 0;
    __syncthreads();
    const u32 stride = gridDim.x * WAVES;
    for (u32 c0 = blockIdx.x * WAVES; c0 < n_chunks; c0 += stride) {
        const u32 c = c0 + w;
        bool want = false;
        u32 ia = 0, bidx = 0;
        if (c < n_chunks) {
            const u32 pos = s.cpos[c], lo = s.clo[c], hi = s.chi[c];
            const u32 q = lo + lane;
            if (q < hi) {
                const u32 btid = seg_tid(s, pos), binfo = seg_info(s, pos);
                const u32 bblk = block_of(b, btid), bph = info_phase(binfo), bcat = info_cat(binfo);
                const u32 ta = seg_tid(s, q), info = seg_info(s, q);
                const u32 ba = block_of(b, ta), pha = info_phase(info);
                if (ta != btid && conflicts(info_cat(info), ba, bcat, bblk)) {
                    u32 h = NONE;
                    ia = s.i[q];
                    bidx = s.i[pos];
                    want = !happens_before(b, rt_scan, bidx, btid, bblk, bph, h, ta, ba, pha, ia);
                }
            }
        }
        const u64 m = ballot(want);
        if (m) {
            u32 off = 0;
            const u32 leader = (u32)__builtin_ctzll(m);
            if (lane == leader) off = atomicAdd(&fill, popc64(m));
            off = __shfl(off, leader, 64) + popc64(m & lanemask_lt());
            if (want) { pf[off] = ia; ps[off] = bidx; }
        }
        __syncthreads();
        if (fill > PAIR_LDS - WG_THREADS || c0 + stride >= n_chunks) {
            if (threadIdx.x == 0) gbase = fill ? atomicAdd(&b.prm->n_pairs, fill) : 0;
            __syncthreads();
            for (u32 k = threadIdx.x; k < fill; k += WG_THREADS) {
                const u32 slot = gbase + k;
                if (slot < b.max_pairs) { b.pfirst[0][slot] = pf[k]; b.psecond[0][slot] = ps[k]; }
                else atomicOr(&b.prm->err, ERR_PAIRS);
            }
            __syncthreads();
            if (threadIdx.x == 0) fill = 0;
            __syncthreads();
        }
    }
    const u32 n_long = min(b.prm->n_long, s.n);
    for (u32 c = blockIdx.x * WAVES + w; c < n_long; c += stride) {
        const u32 e = s.lpos[c], pos = e & 0x7fffffffu;
        const u32 tid = seg_tid(s, pos), info = seg_info(s, pos);
        wave_slow_check(b, s, rt_scan, pos, seg_key(s, pos), tid, block_of(b, tid), info_phase(info),
                        info_cat(info), (e >> 31) != 0u);
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
    const unsigned nch = (unsigned)((b.n_tiles + SCAN_CHUNK - 1) / SCAN_CHUNK);
    RD_LAUNCH("k_seg_scan_up", k_seg_scan_up, dim3(nch ? nch : 1), dim3(SCAN_THREADS), 0, s, b);
    RD_LAUNCH("k_seg_scan_top", k_seg_scan_top, dim3(1), dim3(SCAN_THREADS), 0, s, b);
    RD_LAUNCH("k_seg_scan_down", k_seg_scan_down, dim3(nch ? nch : 1), dim3(SCAN_THREADS), 0, s, b);
    RD_LAUNCH("k_seg_check", k_seg_check, dim3(b.n_tiles), dim3(WG_THREADS), 0, s, b, rt_scan);
    RD_LAUNCH("k_seg_slow", k_seg_slow, dim3(SLOW_GRID), dim3(WG_THREADS), 0, s, b, rt_scan);
    RD_LAUNCH("k_pairs_kept", k_pairs_kept, dim3(1), dim3(64), 0, s, b);
}

}  // namespace rd
