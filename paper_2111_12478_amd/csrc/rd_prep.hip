// rd_prep.hip -- trace ingest, per-thread sync lists, barrier instances, access elements,
// release/acquire inference and barrier validation (gfx950).
//
// Everything here streams the 16-byte records once or twice with coalesced dwordx4 loads, or
// walks the short per-thread lists of synchronisation events (one lane per program thread).
#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

// ---------------------------------------------------------------- fills and scans


static inline unsigned grid_for(u64 n, unsigned per = 256, unsigned cap = 4096) {
    u64 g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Several fills in one launch: blockIdx.y picks the job.  A job with a mode mask runs only when the
// trace's mode (DevParams::mode, set by k_plan) has one of its bits; a job with dyn_n fills
// min(*dyn_n, n) entries.
__global__ void k_fill_many(FillJobs L) {
    const FillJob f = L.j[blockIdx.y];
    if (f.mode_mask && !(L.P->mode & f.mode_mask)) return;
    if (f.eng == 1 && !((L.P->eng & ENG_PARALLEL) && !(L.P->eng & ENG_FALLBACK))) return;  // engine only
    if (f.eng == 2 && ((L.P->eng & ENG_PARALLEL) && !(L.P->eng & ENG_FALLBACK))) return;   // interpreter only
    u64 n = f.n;
    if (f.dyn_n && (u64)*f.dyn_n < n) n = *f.dyn_n;
    const u64 step = (u64)gridDim.x * blockDim.x;
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (f.esize == 1)
        for (; i < n; i += step) ((uint8_t *)f.p)[i] = (uint8_t)f.v;
    else if (f.esize == 4)
        for (; i < n; i += step) ((u32 *)f.p)[i] = (u32)f.v;
    else
        for (; i < n; i += step) ((u64 *)f.p)[i] = f.v;
}

void fill_many(const FillJobs &jobs, const char *name, hipStream_t s) {
    u64 mx = 1;
    for (u32 k = 0; k < jobs.count; k++) mx = jobs.j[k].n > mx ? jobs.j[k].n : mx;
    if (jobs.count) RD_LAUNCH(name, k_fill_many, dim3(grid_for(mx, 256, 1024), jobs.count), dim3(256), 0, s, jobs);
}

void FillJobs::add(void *p, u64 n, u64 v, u32 esize, u32 mode_mask, const u32 *dyn_n, u32 eng) {
    if (count < MAX_FILL_JOBS && n) j[count++] = FillJob{p, dyn_n, n, v, esize, mode_mask, eng};
}


// Block-wide exclusive scan of one value per thread (256 threads).  Returns the exclusive prefix;
// *total gets the block total.
__device__ inline u32 block_exscan_256(u32 v, u32 *total, u32 *lds /* >= 8 words */) {
    const u32 lane = lane_id(), w = threadIdx.x >> 6;
    u32 x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        u32 y = __shfl_up(x, d, 64);
        if (lane >= (u32)d) x += y;
    }
    if (lane == 63) lds[w] = x;
    __syncthreads();
    u32 wbase = 0, tot = 0;
    for (u32 q = 0; q < WAVES; q++) {
        u32 s = lds[q];
        if (q < w) wbase += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wbase + x - v;
}

constexpr u32 SCAN_CHUNK = 4096;  // 256 threads x 16

// partial sums of SCAN_CHUNK-sized chunks
// gate (optional): the scan runs only while the knowledge engine is on (see eng_gate_open)
__device__ inline bool eng_gate_open(const u32 *gate) {
    return !gate || ((*gate & ENG_PARALLEL) && !(*gate & ENG_FALLBACK));
}

// the length of a scan: n, or with n_dev the first *n_dev + 1 words (at most n)
__device__ inline u64 scan_len(u64 n, const u32 *n_dev) {
    if (!n_dev) return n;
    const u64 m = (u64)*n_dev + 1;
    return m < n ? m : n;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const u32 *in, u64 n, u32 *part, const u32 *gate,
                                                      const u32 *n_dev) {
    __shared__ u32 lds[8];
    if (!eng_gate_open(gate)) return;
    n = scan_len(n, n_dev);
    u64 base = (u64)blockIdx.x * SCAN_CHUNK;
    if (base >= n) return;
    u32 s = 0;
    for (u32 k = 0; k < 16; k++) {
        u64 i = base + k * 256 + threadIdx.x;
        if (i < n) s += in[i];
    }
    u32 tot;
    block_exscan_256(s, &tot, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}
// exclusive scan of the partials in one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void k_scan_top(u32 *part, u32 np, const u32 *gate, u64 n, const u32 *n_dev) {
    __shared__ u32 lds[1024];
    if (!eng_gate_open(gate)) return;
    {
        const u64 npe = (scan_len(n, n_dev) + SCAN_CHUNK - 1) / SCAN_CHUNK;
        if (npe < np) np = (u32)npe;
    }
    u32 per = (np + 1023) / 1024;
    u32 lo = threadIdx.x * per, hi = lo + per < np ? lo + per : np;
    u32 s = 0;
    for (u32 i = lo; i < hi; i++) s += part[i];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (u32 d = 1; d < 1024; d <<= 1) {
        u32 y = threadIdx.x >= d ? lds[threadIdx.x - d] : 0;
        __syncthreads();
        lds[threadIdx.x] += y;
        __syncthreads();
    }
    u32 run = lds[threadIdx.x] - s;
    for (u32 i = lo; i < hi; i++) { u32 v = part[i]; part[i] = run; run += v; }
}
// in-place exclusive scan of each chunk plus its carry: part[blockIdx.x] after k_scan_top, or with
// `direct` (at most SCAN_DIRECT chunks) the sum of the earlier chunks' totals, read by every
// workgroup from L2 instead of a separate scan of the totals
constexpr u32 SCAN_DIRECT = 8192;  // up to 33.5M words: at most 8192 totals summed per workgroup
__global__ __launch_bounds__(256) void k_scan_apply(u32 *data, u64 n, const u32 *part, const u32 *gate,
                                                     const u32 *n_dev, bool direct) {
    __shared__ u32 lds[8];
    if (!eng_gate_open(gate)) return;
    n = scan_len(n, n_dev);
    if ((u64)blockIdx.x * SCAN_CHUNK >= n) return;
    u32 carry;
    if (direct) {
        u32 c = 0;
        for (u32 j = threadIdx.x; j < blockIdx.x; j += 256) c += part[j];
        (void)block_exscan_256(c, &carry, lds);
    } else {
        carry = part[blockIdx.x];
    }
    u64 base = (u64)blockIdx.x * SCAN_CHUNK + (u64)threadIdx.x * 16;
    u32 v[16], s = 0;
    for (u32 k = 0; k < 16; k++) { u64 i = base + k; v[k] = i < n ? data[i] : 0; s += v[k]; }
    u32 tot;
    u32 run = block_exscan_256(s, &tot, lds) + carry;
    for (u32 k = 0; k < 16; k++) { u64 i = base + k; if (i < n) data[i] = run; run += v[k]; }
}

// Small arrays in one workgroup each: region blockIdx.x of `regions` consecutive arrays of n words,
// n <= SCAN_SMALL; every thread scans a run of up to 16 consecutive words.
constexpr u32 SCAN_SMALL = 1024 * 16;
__global__ __launch_bounds__(1024) void k_scan_small(u32 *data, u32 n, const u32 *gate, const u32 *n_dev) {
    __shared__ u32 wsum[16];
    if (!eng_gate_open(gate)) return;
    n = (u32)scan_len(n, n_dev);
    u32 *d = data + (u64)blockIdx.x * n;
    const u32 per = (n + 1023) / 1024, lo = threadIdx.x * per, hi = lo + per < n ? lo + per : n;
    const u32 lane = lane_id(), w = threadIdx.x >> 6;
    u32 v[16], sum = 0;
#pragma unroll
    for (u32 k = 0; k < 16; k++) {
        v[k] = lo + k < hi ? d[lo + k] : 0;
        sum += v[k];
    }
    u32 x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const u32 y = __shfl_up(x, o, 64);
        if (lane >= (u32)o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    u32 run = x - sum;
    for (u32 q = 0; q < w; q++) run += wsum[q];
#pragma unroll
    for (u32 k = 0; k < 16; k++) {
        if (lo + k < hi) d[lo + k] = run;
        run += v[k];
    }
}

// Exclusive scans of `regions` consecutive arrays of n words each, in place.
void scan_exclusive_multi(u32 *data, u64 n, u32 regions, u32 *part, hipStream_t s) {
    if (!n || !regions) return;
    if (n <= SCAN_SMALL) {
        RD_LAUNCH("k_scan_small", k_scan_small, dim3(regions), dim3(1024), 0, s, data, (u32)n, (const u32 *)nullptr,
                  (const u32 *)nullptr);
        return;
    }
    for (u32 r = 0; r < regions; r++) scan_exclusive(data + (u64)r * n, n, part, s);
}

// Exclusive scan of data[0..n) in place; `part` needs ceil(n / 4096) words (<= 2^20).  With a gate,
// nothing happens unless the knowledge engine is on.  With n_dev, only the first *n_dev + 1 words
// (at most n) are scanned: launches are sized for n, the workgroups past the length exit at once.
void scan_exclusive(u32 *data, u64 n, u32 *part, hipStream_t s, const u32 *gate, const u32 *n_dev) {
    if (!n) return;
    if (n <= SCAN_SMALL) {
        RD_LAUNCH("k_scan_small", k_scan_small, dim3(1), dim3(1024), 0, s, data, (u32)n, gate, n_dev);
        return;
    }
    u32 np = (u32)((n + SCAN_CHUNK - 1) / SCAN_CHUNK);
    const bool direct = np <= SCAN_DIRECT;
    RD_LAUNCH("k_scan_reduce", k_scan_reduce, dim3(np), dim3(256), 0, s, data, n, part, gate, n_dev);
    if (!direct) RD_LAUNCH("k_scan_top", k_scan_top, dim3(1), dim3(1024), 0, s, part, np, gate, n, n_dev);
    RD_LAUNCH("k_scan_apply", k_scan_apply, dim3(np), dim3(256), 0, s, data, n, part, gate, n_dev, direct);
}

// ---------------------------------------------------------------- init

__global__ void k_init_params(DevParams *p, u32 *sort_tot) {
    for (u32 i = threadIdx.x; i < MAX_SORT_PASSES * (SORT_NDS + 1); i += blockDim.x) sort_tot[i] = 0;  // + tickets
    if (threadIdx.x == 0) {
        DevParams z = {};
        z.first_bad_record = NONE;
        z.first_bad_sync = NONE;
        z.gmin = NONE;
        z.smin = NONE;
        *p = z;
    }
}

// ---------------------------------------------------------------- ingest

__device__ inline bool is_access_kind(u32 k) { return k <= 2u || k == 6u || k == 7u; }

// Record checks, kind histogram, address ranges, activity, sync counts per thread, and two
// bitmasks (sync events, accesses) with per-tile counts for the compactions that follow.
__global__ __launch_bounds__(WG_THREADS) void k_ingest(Bufs b, u64 *sync_mask, u64 *acc_mask, u64 *atom_mask) {
    __shared__ u32 lds_cnt[8][WAVES];
    __shared__ u32 lds_misc[WAVES][8];
    const u32 w = threadIdx.x >> 6, lane = lane_id();
    const u64 base = (u64)blockIdx.x * TILE + (u64)w * ITEMS * 64;
    u32 bad = NONE, ns = 0, na = 0, nt = 0;
    u32 kc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    u32 gmin = NONE, gmax = 0, smin = NONE, smax = 0;
#pragma unroll 4
    for (int k = 0; k < ITEMS; k++) {
        const u64 i = base + (u64)k * 64 + lane;
        const bool in = i < b.N;
        uint4 e = in ? b.ev[i] : make_uint4(0, 0, 0, 0);
        const u32 kind = e.z & 15u, scope = (e.z >> 4) & 3u, space = (e.z >> 6) & 1u;
        bool ok = in && (e.z >> 7) == 0 && kind <= 7u && scope <= 2u && e.y < b.T &&
                  !((kind == 3u || kind == 4u || kind == 5u) && space);
        if (in && !ok && (u32)i < bad) bad = (u32)i;
        if (in && e.y < b.T) b.act[e.y] = 1;
        // sync lists hold fences, barriers, warp barriers and locks; atomics join them only when the
        // trace has something that can make an atomic a release or an acquire (decided in k_plan)
        const bool is_sync = ok && kind >= 3u;
        const bool is_atom = ok && kind == 2u;
        const bool is_acc = ok && is_access_kind(kind);
        if (ok) {
#pragma unroll
            for (u32 q = 0; q < 8; q++) kc[q] += (kind == q);
        }
        if (is_acc) {
            if (space) { smin = min(smin, e.x); smax = max(smax, e.x); }
            else { gmin = min(gmin, e.x); gmax = max(gmax, e.x); }
        }
        if (is_sync) atomicAdd(&b.s_cnt[e.y], 1u);
        if (is_atom) atomicAdd(&b.a_cnt[e.y], 1u);
        const u64 ms = ballot(is_sync), ma = ballot(is_acc), mt = ballot(is_atom);
        if (lane == 0) {
            const u64 word = (base + (u64)k * 64) >> 6;
            sync_mask[word] = ms;
            acc_mask[word] = ma;
            atom_mask[word] = mt;
        }
        ns += popc64(ms);
        na += popc64(ma);
        nt += popc64(mt);
    }
    // wave reductions
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        bad = min(bad, (u32)__shfl_xor((int)bad, d, 64));
        gmin = min(gmin, (u32)__shfl_xor((int)gmin, d, 64));
        gmax = max(gmax, (u32)__shfl_xor((int)gmax, d, 64));
        smin = min(smin, (u32)__shfl_xor((int)smin, d, 64));
        smax = max(smax, (u32)__shfl_xor((int)smax, d, 64));
#pragma unroll
        for (int q = 0; q < 8; q++) kc[q] += __shfl_xor((int)kc[q], d, 64);
    }
    if (lane == 0) {
        for (int q = 0; q < 8; q++) lds_cnt[q][w] = kc[q];
        lds_misc[w][0] = bad; lds_misc[w][1] = gmin; lds_misc[w][2] = gmax;
        lds_misc[w][3] = smin; lds_misc[w][4] = smax; lds_misc[w][5] = ns; lds_misc[w][6] = na;
        lds_misc[w][7] = nt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 tb = NONE, tg0 = NONE, tg1 = 0, ts0 = NONE, ts1 = 0, tns = 0, tna = 0, tnt = 0;
        for (int q = 0; q < WAVES; q++) {
            tb = min(tb, lds_misc[q][0]); tg0 = min(tg0, lds_misc[q][1]); tg1 = max(tg1, lds_misc[q][2]);
            ts0 = min(ts0, lds_misc[q][3]); ts1 = max(ts1, lds_misc[q][4]);
            tns += lds_misc[q][5]; tna += lds_misc[q][6]; tnt += lds_misc[q][7];
        }
        // per-tile statistics, reduced by k_plan (no same-address atomics across tiles)
        u32 *st = b.tile_stats + (u64)blockIdx.x * TILE_STATS;
        st[0] = tb; st[1] = tg0; st[2] = tg1; st[3] = ts0; st[4] = ts1;
        for (int q = 0; q < 8; q++) {
            u32 c = 0;
            for (int ww = 0; ww < WAVES; ww++) c += lds_cnt[q][ww];
            st[5 + q] = c;
        }
        // three regions of n_tiles + 1 words: sync events, accesses, atomics
        b.tile_s[blockIdx.x] = tns;
        b.tile_s[(b.n_tiles + 1) + blockIdx.x] = tna;
        b.tile_s[2 * (b.n_tiles + 1) + blockIdx.x] = tnt;
    }
}

// Reduces the per-tile ingest statistics, then plans the location key and the mode of the check.
// fields 0..4 of a tile's statistics: min, min, max, min, max; 5..12: sums
__device__ inline void plan_fold(u32 *acc, const u32 *v) {
    acc[0] = min(acc[0], v[0]); acc[1] = min(acc[1], v[1]); acc[2] = max(acc[2], v[2]);
    acc[3] = min(acc[3], v[3]); acc[4] = max(acc[4], v[4]);
#pragma unroll
    for (int q = 5; q < 13; q++) acc[q] += v[q];
}

constexpr u32 PLAN_THREADS = 1024;

__global__ __launch_bounds__(PLAN_THREADS) void k_plan(Bufs b) {
    constexpr int F = 13;  // the statistics of a row (rows are TILE_STATS words apart)
    static_assert(TILE_STATS == 16, "rows of four 16-byte vectors");
    __shared__ u32 red[PLAN_THREADS / 64][F];
    const u32 lane = lane_id(), w = threadIdx.x >> 6;
    u32 acc[F];
    acc[0] = NONE; acc[1] = NONE; acc[2] = 0; acc[3] = NONE; acc[4] = 0;
    for (int q = 5; q < F; q++) acc[q] = 0;
    // four tiles' rows in flight per thread
    for (u32 t0 = threadIdx.x; t0 < b.n_tiles; t0 += 4 * PLAN_THREADS) {
        u32 v[4][F];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const u32 t = t0 + j * PLAN_THREADS;
            if (t < b.n_tiles) {
                // a row is 64 aligned bytes: four 16-byte loads
                const uint4 *st = (const uint4 *)(b.tile_stats + (u64)t * TILE_STATS);
                const uint4 r0 = st[0], r1 = st[1], r2 = st[2], r3 = st[3];
                const u32 row[16] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w,
                                     r2.x, r2.y, r2.z, r2.w, r3.x, r3.y, r3.z, r3.w};
#pragma unroll
                for (int q = 0; q < F; q++) v[j][q] = row[q];
            } else {
#pragma unroll
                for (int q = 0; q < F; q++) v[j][q] = q == 0 || q == 1 || q == 3 ? NONE : 0u;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; j++) plan_fold(acc, v[j]);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        u32 o[F];
#pragma unroll
        for (int q = 0; q < F; q++) o[q] = (u32)__shfl_xor((int)acc[q], d, 64);
        plan_fold(acc, o);
    }
    if (lane == 0)
        for (int q = 0; q < F; q++) red[w][q] = acc[q];
    __syncthreads();
    if (threadIdx.x) return;
    for (u32 x = 1; x < PLAN_THREADS / 64; x++) plan_fold(acc, red[x]);
    DevParams *p = b.prm;
    p->first_bad_record = acc[0];
    p->gmin = acc[1]; p->gmax = acc[2]; p->smin = acc[3]; p->smax = acc[4];
    for (int q = 0; q < 8; q++) p->kind_count[q] = acc[5 + q];
    const u32 n_other = b.tile_s[b.n_tiles], n_atom = b.tile_s[3 * b.n_tiles + 2];
    p->n_acc = b.tile_s[2 * b.n_tiles + 1];
    u64 gs = p->gmin != NONE ? (u64)p->gmax - p->gmin + 1 : 0;
    u64 ss = p->smin != NONE ? (u64)p->smax - p->smin + 1 : 0;
    u64 total = gs + (u64)b.B * ss;
    if (total > 0xffffffffull) { p->err |= ERR_KEYSPAN; total = 0xffffffffull; }
    u32 bits = 0;
    while (bits < 32 && ((u64)1 << bits) < total) bits++;
    p->key_bits = bits;
    p->g_span = (u32)gs;
    p->s_span = (u32)ss;
    p->gbase = p->gmin != NONE ? p->gmin : 0;
    p->sbase = p->smin != NONE ? p->smin : 0;
    u32 mode = 0;
    if (p->kind_count[4]) mode |= MODE_BAR;
    if (p->kind_count[3] || p->kind_count[5] || p->kind_count[6] || p->kind_count[7]) mode |= MODE_SYNC;
    if (p->kind_count[5]) mode |= MODE_WBAR;
    p->mode = mode;
    if (((mode & MODE_SYNC) && (b.spec & SPEC_NO_SYNC)) || ((mode & MODE_WBAR) && (b.spec & SPEC_NO_WBAR)))
        p->err |= ERR_RESPEC;
    p->n_sync = n_other + ((mode & MODE_SYNC) ? n_atom : 0u);
}

// Position of item (lane, step) among the set bits of a tile's bitmask, in input order.
// masks: the tile's ITEMS words of this wave are read by every lane.
__device__ inline void wave_mask_prefix(const u64 *mask, const u64 *mask2, u64 tile_word0, u32 w, u32 *wave_base_lds,
                                        u32 tile_off, u64 m_items[ITEMS], u32 pre[ITEMS]) {
    const u32 lane = lane_id();
    u32 run = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; k++) {
        const u64 wi = tile_word0 + (u64)w * ITEMS + k;
        const u64 m = mask[wi] | (mask2 ? mask2[wi] : 0ull);
        m_items[k] = m;
        pre[k] = run + popc64(m & lanemask_lt());
        run += popc64(m);
    }
    if (lane == 0) wave_base_lds[w] = run;
    __syncthreads();
    u32 wb = tile_off;
    for (u32 q = 0; q < w; q++) wb += wave_base_lds[q];
#pragma unroll
    for (int k = 0; k < ITEMS; k++) pre[k] += wb;
}

// Sync events in trace order: s_tidx[q] = event index.
__global__ __launch_bounds__(WG_THREADS) void k_sync_compact(Bufs b, const u64 *sync_mask, const u64 *atom_mask) {
    __shared__ u32 wbase[WAVES];
    const u32 w = threadIdx.x >> 6, lane = lane_id();
    const u64 word0 = (u64)blockIdx.x * (TILE / 64);
    const bool with_atomics = (b.prm->mode & MODE_SYNC) != 0;
    const u32 off = b.tile_s[blockIdx.x] + (with_atomics ? b.tile_s[2 * (b.n_tiles + 1) + blockIdx.x] : 0u);
    u64 m[ITEMS];
    u32 pre[ITEMS];
    wave_mask_prefix(sync_mask, with_atomics ? atom_mask : nullptr, word0, w, wbase, off, m, pre);
    const u64 base = (u64)blockIdx.x * TILE + (u64)w * ITEMS * 64;
#pragma unroll
    for (int k = 0; k < ITEMS; k++)
        if ((m[k] >> lane) & 1) b.s_tidx[pre[k]] = (u32)(base + (u64)k * 64 + lane);
}

// The sync events in trace order keyed by their thread, for the stable sort into per-thread lists
// (key[q] = tid, val[q] = q, kindq[q] = kind).
__global__ void k_sync_keys(Bufs b, u32 *key, u32 *val, u32 *kindq) {
    const u32 n = b.prm->n_sync;
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const uint4 e = b.ev[b.s_tidx[q]];
        key[q] = e.y;
        val[q] = q;
        kindq[q] = e.z & 15u;
    }
}

// After the sort by thread: list position p holds the thread's entries in trace order.  Each entry
// gets its event, kind and trace-order position, its per-entry fields cleared, and a barrier flag
// for the phase scan.  The sort's totals and tickets are cleared for the location sort.
__global__ void k_sync_place(Bufs b, const u32 *val, const u32 *kindq, u32 *barflag) {
    const u32 n = b.prm->n_sync;
    if (blockIdx.x == 0)
        for (u32 i = threadIdx.x; i < MAX_SORT_PASSES * (SORT_NDS + 1); i += blockDim.x) b.sort_tot[i] = 0;
    for (u32 p = blockIdx.x * blockDim.x + threadIdx.x; p <= n; p += gridDim.x * blockDim.x) {
        if (p == n) {
            barflag[p] = 0;
            continue;
        }
        const u32 q = val[p], kind = kindq[q];
        b.s_pidx[p] = b.s_tidx[q];
        b.s_pq[p] = q;
        b.s_inv[q] = p;
        b.s_kind[p] = (uint8_t)kind;
        b.s_imin[p] = NONE;
        b.s_flags[p] = 0;
        b.s_scope[p] = 0;
        barflag[p] = kind == 4u ? 1u : 0u;
    }
}

// Phase of each entry: the barriers of its thread's list up to and including it (barscan: exclusive
// prefix of the barrier flags over all lists).
__global__ void k_sync_phase(Bufs b, const u32 *key, const u32 *barscan) {
    const u32 n = b.prm->n_sync;
    for (u32 p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x)
        b.s_phase[p] = barscan[p + 1] - barscan[b.s_cnt[key[p]]];
}

// One lane per program thread: its barrier count (phase bound), the block's largest (one atomic per
// block present in the wavefront) and the trace's largest.
__global__ __launch_bounds__(64) void k_thread_maxbar(Bufs b, const u32 *barscan) {
    u32 top = 0;
    const u32 lane = lane_id();
    for (u32 base = blockIdx.x * 64; base < b.T; base += gridDim.x * 64) {
        const u32 t = base + lane;
        const bool valid = t < b.T;
        const u32 ph = valid ? barscan[b.s_cnt[t + 1]] - barscan[b.s_cnt[t]] : 0u;
        if (ph >= (1u << 30)) atomicOr(&b.prm->err, ERR_PHASE);
        top = max(top, ph);
        const u32 blk = valid ? t / b.tpb : NONE;
        u64 pending = ballot(ph != 0);
        while (pending) {
            const u32 leader = (u32)__builtin_ctzll(pending);
            const u32 lb = __shfl(blk, leader, 64);
            const bool mine = ph != 0 && blk == lb;
            u32 mx = mine ? ph : 0u;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (u32)__shfl_xor((int)mx, d, 64));
            if (lane == leader) atomicMax(&b.blk_maxbar[lb], mx);
            pending &= ~ballot(mine);
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) top = max(top, (u32)__shfl_xor((int)top, d, 64));
    if (lane == 0 && top) atomicMax(&b.prm->max_phase, top);
}


// Barrier arrivals per (block, instance) and active threads per block.  Lanes of a wavefront are
// consecutive threads, mostly of one block, so arrivals are aggregated per (instance) across the
// wave before the device atomics.
__global__ void k_bar_register(Bufs b) {
    const u32 lane = lane_id();
    for (u32 t0 = blockIdx.x * blockDim.x; t0 < b.T; t0 += gridDim.x * blockDim.x) {
        const u32 t = t0 + threadIdx.x;
        const bool in = t < b.T;
        const u32 blk = in ? block_of(b, t) : 0;
        // active threads per block
        {
            bool a = in && b.act[t];
            u64 pending = ballot(a);
            while (pending) {
                const u32 leader = __builtin_ctzll(pending);
                const u32 lb = __shfl(blk, leader, 64);
                const u64 m = ballot(a && blk == lb);
                if (lane == leader) atomicAdd(&b.n_active[lb], popc64(m));
                if (blk == lb) a = false;
                pending &= ~m;
            }
        }
        u32 p = in ? b.s_cnt[t] : 0;
        const u32 hi = in ? b.s_cnt[t + 1] : 0;
        for (u32 k = 0;; k++) {
            // this lane's k-th barrier arrival, if any
            while (p < hi && b.s_kind[p] != 4) p++;
            bool has = p < hi;
            if (!__any(has)) break;
            const u32 slot = has ? b.inst_off[blk] + k : 0;
            const u32 idx = has ? b.s_pidx[p] : 0;
            u64 pending = ballot(has);
            while (pending) {
                const u32 leader = __builtin_ctzll(pending);
                const u32 ls = __shfl(slot, leader, 64);
                const bool mine = has && slot == ls;
                const u64 m = ballot(mine);
                u32 mx = mine ? idx : 0;
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (u32)__shfl_xor((int)mx, d, 64));
                if (lane == leader) { atomicAdd(&b.inst_cnt[ls], popc64(m)); atomicMax(&b.inst_last[ls], mx); }
                if (mine) has = false;
                pending &= ~m;
            }
            if (p < hi) p++;
        }
    }
}

// Access elements (location key, index, tid, category | phase), compacted in trace order; packed
// (category and phase above the key bits of the key word, no info array) when they fit.  Plain
// reads and writes also record, per list entry, the first access that follows it.
// Also counts the digits of every location-sort pass (one row of per-tile counts; digits of the
// context's sort variant, radix_bits wide).
__global__ __launch_bounds__(WG_THREADS) void k_elements(Bufs b, const u64 *acc_mask) {
    __shared__ u32 wbase[WAVES];
    __shared__ u32 dcnt[ELEM_MAX_PASSES][SORT_NDS];
    const u32 w = threadIdx.x >> 6, lane = lane_id();
    const u32 rb = b.radix_bits, nd = 1u << rb;
    for (u32 x = threadIdx.x; x < ELEM_MAX_PASSES * SORT_NDS; x += WG_THREADS) (&dcnt[0][0])[x] = 0;
    const u64 word0 = (u64)blockIdx.x * (TILE / 64);
    // each item's output slot, NONE where the lane's event is not an access
    u32 slot[ITEMS];
    {
        u64 m[ITEMS];
        u32 pre[ITEMS];
        wave_mask_prefix(acc_mask, nullptr, word0, w, wbase, b.tile_s[b.n_tiles + 1 + blockIdx.x], m, pre);
#pragma unroll
        for (int k = 0; k < ITEMS; k++) slot[k] = (m[k] >> lane) & 1 ? pre[k] : NONE;
    }
    const DevParams *p = b.prm;
    const u32 gbase = p->gbase, sbase = p->sbase, g_span = p->g_span, s_span = p->s_span;
    const u32 mode = p->mode;
    const u32 np = (p->key_bits + rb - 1) / rb;
    const bool packed = packed_elements(p->key_bits, p->max_phase);
    const bool tinfo = tinfo_elements(p->key_bits, p->max_phase, b.T);
    const u32 tb = tid_bits(b.T);
    const bool lists = (mode & (MODE_SYNC | MODE_BAR)) != 0;
    u32 *ekey = b.ekey[0], *eidx = b.eidx[0], *etid = b.etid[0], *einfo = b.einfo[0];
    const u64 base = (u64)blockIdx.x * TILE + (u64)w * ITEMS * 64;
    // items in groups of GI: the loads of a group's items are issued together (events, list bounds,
    // one binary-search step for every item of the group at a time, entries, barrier instances),
    // so a lane has GI dependent chains in flight instead of one
    constexpr int GI = 4;
    static_assert(ITEMS % GI == 0, "whole groups");
    for (int k0 = 0; k0 < ITEMS; k0 += GI) {
        u32 idx[GI], t[GI], meta[GI], addr[GI], lo[GI], hi[GI], j[GI];
#pragma unroll
        for (int i = 0; i < GI; i++) {
            idx[i] = (u32)(base + (u64)(k0 + i) * 64 + lane);
            t[i] = meta[i] = addr[i] = 0;
            if (slot[k0 + i] != NONE) {
                const uint4 e = b.ev[idx[i]];
                addr[i] = e.x;
                t[i] = e.y;
                meta[i] = e.z;
            }
        }
        // the last list entry of the thread before the access (a binary search in lockstep)
#pragma unroll
        for (int i = 0; i < GI; i++) {
            lo[i] = hi[i] = 0;
            if (lists && slot[k0 + i] != NONE) { lo[i] = b.s_cnt[t[i]]; hi[i] = b.s_cnt[t[i] + 1]; }
            j[i] = lo[i];  // the list's first entry, for now
        }
        for (;;) {
            u32 mid[GI], v[GI];
            bool any = false;
#pragma unroll
            for (int i = 0; i < GI; i++) {
                mid[i] = (lo[i] + hi[i]) >> 1;
                v[i] = 0;
                if (lo[i] < hi[i]) { v[i] = b.s_pidx[mid[i]]; any = true; }
            }
            if (!any) break;
#pragma unroll
            for (int i = 0; i < GI; i++) {
                if (lo[i] < hi[i]) {
                    if (v[i] < idx[i]) lo[i] = mid[i] + 1;
                    else hi[i] = mid[i];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < GI; i++) j[i] = lo[i] == j[i] ? NONE : lo[i] - 1;
        // phases and the checks that need the entry
        u32 ph[GI], blk[GI];
#pragma unroll
        for (int i = 0; i < GI; i++) {
            blk[i] = block_of(b, t[i]);
            ph[i] = 0;
            if (slot[k0 + i] == NONE || j[i] == NONE) continue;
            if (mode & MODE_SYNC) {
                ph[i] = b.s_phase[j[i]];
                // the first plain access after an atomic, a fence, a warp barrier or a lock acquire
                // (release/acquire inference, warp-barrier rule, acquires only a barrier reads)
                const u32 kj = b.s_kind[j[i]], kind = meta[i] & 15u;
                if (kind <= 1 && (kj == 2 || kj == 3 || kj == 5 || kj == 6) && b.s_imin[j[i]] > idx[i])
                    atomicMin(&b.s_imin[j[i]], idx[i]);
            } else {
                // the thread's list holds only its barriers: the phase is the number of entries
                // before idx
                ph[i] = j[i] - b.s_cnt[t[i]] + 1;
            }
        }
        // after a block barrier the access checks the barrier rule itself
#pragma unroll
        for (int i = 0; i < GI; i++) {
            if (ph[i] == 0) continue;
            const u32 sl = b.inst_off[blk[i]] + ph[i] - 1;
            if (b.inst_cnt[sl] != b.n_active[blk[i]] || b.inst_last[sl] > idx[i])
                atomicMin(&b.prm->first_bad_sync, idx[i]);
        }
#pragma unroll
        for (int i = 0; i < GI; i++) {
            const bool mine = slot[k0 + i] != NONE;
            const u64 act = ballot(mine);
            if (!act) continue;
            u32 key = 0;
            if (mine) {
                const u32 kind = meta[i] & 15u, scope = (meta[i] >> 4) & 3u, space = (meta[i] >> 6) & 1u;
                key = space ? g_span + blk[i] * s_span + (addr[i] - sbase) : addr[i] - gbase;
                u32 cat;
                if (kind == 0) cat = CAT_R;
                else if (kind == 1) cat = CAT_W;
                else cat = scope == 0 ? CAT_AB : CAT_AD;
                const u32 o = slot[k0 + i];
                if (packed) {
                    ekey[o] = pack_element(key, p->key_bits, cat, ph[i]);
                    etid[o] = t[i];
                } else if (tinfo) {
                    ekey[o] = key;
                    etid[o] = tinfo_word(t[i], tb, cat, ph[i]);
                } else {
                    ekey[o] = key;
                    einfo[o] = info_make(cat, ph[i]);
                    etid[o] = t[i];
                }
                eidx[o] = idx[i];
            }
            // digit counts: where every active lane has the wavefront's first digit (high digits of
            // clustered addresses), one lane adds them all instead of 64 atomics on one LDS word
            const u32 first = (u32)__builtin_ctzll(act);
            for (u32 q = 0; q < np; q++) {
                const u32 d = (key >> (q * rb)) & (nd - 1);
                const u32 d0 = __shfl(d, first, 64);
                if (ballot(mine && d == d0) == act) {
                    if (lane == first) atomicAdd(&dcnt[q][d0], popc64(act));
                } else if (mine) {
                    atomicAdd(&dcnt[q][d], 1u);
                }
            }
        }
    }
    __syncthreads();
    u32 *row = b.sort_partial + (u64)blockIdx.x * ELEM_MAX_PASSES * SORT_NDS;
    for (u32 q = 0; q < np; q++)
        for (u32 d = threadIdx.x; d < nd; d += WG_THREADS) row[q * SORT_NDS + d] = dcnt[q][d];
}

// One lane per program thread: releases/acquires (explicit, or atomics next to a fence with no
// access in between), knowledge-column flags, and the block-barrier rule for the first event after
// each of the thread's barriers.
__global__ void k_thread_sync(Bufs b, u32 *rt_flag) {
    const u32 mode = b.prm->mode;
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < b.T; t += gridDim.x * blockDim.x) {
        const u32 lo = b.s_cnt[t], hi = b.s_cnt[t + 1], blk = t / b.tpb;
        u32 has_rt = 0, k = 0;
        for (u32 p = lo; p < hi; p++) {
            const u32 kind = b.s_kind[p];
            if (mode & MODE_SYNC) {
                uint8_t f = 0, sc = 0;
                if (kind == 7) { f |= SF_REL; sc |= (uint8_t)((b.ev[b.s_pidx[p]].z >> 4) & 3u); }
                if (kind == 6) { f |= SF_ACQ; sc |= (uint8_t)(((b.ev[b.s_pidx[p]].z >> 4) & 3u) << 2); }
                if (kind == 2) {
                    if (p > lo && b.s_kind[p - 1] == 3 && b.s_imin[p - 1] == NONE) {
                        f |= SF_REL;
                        sc |= (uint8_t)((b.ev[b.s_pidx[p - 1]].z >> 4) & 3u);
                    }
                    if (p + 1 < hi && b.s_kind[p + 1] == 3 && b.s_imin[p] == NONE) {
                        f |= SF_ACQ;
                        sc |= (uint8_t)(((b.ev[b.s_pidx[p + 1]].z >> 4) & 3u) << 2);
                    }
                }
                if (kind == 5) has_rt = 1;
                if (f & SF_REL) has_rt = 1;
                b.s_flags[p] = f;
                b.s_scope[p] = sc;
            }
            if (kind == 4) {
                // the first event of t after its k-th barrier must follow the instance's last arrival
                // (for the sync entries here; every access after a barrier checks this itself)
                const u32 slot = b.inst_off[blk] + k;
                k++;
                u32 next = b.s_imin[p];
                if (p + 1 < hi) next = min(next, b.s_pidx[p + 1]);
                if (next != NONE) {
                    const bool complete = b.inst_cnt[slot] == b.n_active[blk];
                    if (!complete || next < b.inst_last[slot]) atomicMin(&b.prm->first_bad_sync, next);
                }
            }
        }
        if (rt_flag) rt_flag[t] = has_rt;
    }
}

// The warp-barrier rule, once the instances are known (interpreter output): a bad arrival, or the
// first event after an arrival at an instance that is incomplete or completes later.
__global__ void k_validate_wbar(Bufs b) {
    if (!(b.prm->mode & MODE_WBAR)) return;
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < b.T; t += gridDim.x * blockDim.x) {
        const u32 lo = b.s_cnt[t], hi = b.s_cnt[t + 1];
        for (u32 p = lo; p < hi; p++) {
            if (b.s_kind[p] != 5) continue;
            const u32 idx = b.s_pidx[p];
            if (b.s_flags[p] & SF_BAD_ARRIVAL) { atomicMin(&b.prm->first_bad_sync, idx); continue; }
            const u32 inst = b.s_winst[p];
            u32 next = b.s_imin[p];
            if (p + 1 < hi) next = min(next, b.s_pidx[p + 1]);
            if (next == NONE) continue;
            if (inst == NONE) { atomicMin(&b.prm->first_bad_sync, next); continue; }
            const bool complete = b.winst_arrived[inst] == b.winst_mask[inst];
            if (!complete || next < b.winst_last[inst]) atomicMin(&b.prm->first_bad_sync, next);
        }
    }
}

// With releases/acquires possible, atomics join the sync lists: add their per-thread counts.
__global__ void k_merge_counts(Bufs b) {
    if (!(b.prm->mode & MODE_SYNC)) return;
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < b.T; t += gridDim.x * blockDim.x) b.s_cnt[t] += b.a_cnt[t];
}

// ---------------------------------------------------------------- launchers

void prep_init(const Bufs &b, u32 *rt_scan, hipStream_t s) {
    RD_LAUNCH("k_init_params", k_init_params, dim3(1), dim3(256), 0, s, b.prm, b.sort_tot);
    FillJobs f = {};
    f.P = b.prm;
    f.add(b.act, b.T, 0, 1);
    f.add(b.s_cnt, (u64)b.T + 1, 0, 4);
    f.add(b.s_fill, b.T, 0, 4);
    f.add(b.blk_maxbar, (u64)b.B + 1, 0, 4);
    f.add(b.n_active, b.B, 0, 4);
    f.add(b.tile_s, 3 * ((u64)b.n_tiles + 1), 0, 4);
    f.add(b.a_cnt, b.T, 0, 4);
    f.add(rt_scan, (u64)b.T + 1, 0, 4);
    fill_many(f, "k_fill_init", s);
}

// ingest + tile scans + plan
void prep_ingest(const Bufs &b, u64 *sync_mask, u64 *acc_mask, u64 *atom_mask, hipStream_t s) {
    if (b.N) RD_LAUNCH("k_ingest", k_ingest, dim3(b.n_tiles), dim3(WG_THREADS), 0, s, b, sync_mask, acc_mask, atom_mask);
    scan_exclusive_multi(b.tile_s, (u64)b.n_tiles + 1, 3, b.part, s);
    RD_LAUNCH("k_plan", k_plan, dim3(1), dim3(PLAN_THREADS), 0, s, b);
}

// per-thread sync lists and block-barrier instances
void prep_sync_lists(const Bufs &b, const u64 *sync_mask, const u64 *atom_mask, hipStream_t s) {
    RD_LAUNCH("k_merge_counts", k_merge_counts, dim3(grid_for(b.T)), dim3(256), 0, s, b);
    if (b.N) RD_LAUNCH("k_sync_compact", k_sync_compact, dim3(b.n_tiles), dim3(WG_THREADS), 0, s, b, sync_mask, atom_mask);
    scan_exclusive(b.s_cnt, (u64)b.T + 1, b.part, s);
    // per-thread lists in trace order: a stable sort of the trace-ordered sync events by thread
    // (the element buffers are free until the elements are written), then the entries placed and
    // numbered with coalesced passes over the list positions
    u32 tbits = 0;
    while (tbits < 32 && ((u64)1 << tbits) < (u64)b.T) tbits++;
    const u32 tpasses = (tbits + SORT_RB - 1) / SORT_RB;
    u32 *const k2[2] = {b.ekey[0], b.ekey[1]}, *const v2[2] = {b.eidx[0], b.eidx[1]};
    RD_LAUNCH("k_sync_keys", k_sync_keys, dim3(grid_for(b.N)), dim3(256), 0, s, b, k2[0], v2[0], b.e_scan1);
    sort_kv(b, k2, v2, &b.prm->n_sync, b.N, tpasses, nullptr, "k_sync_sort", s);
    const u32 c = tpasses & 1u;
    RD_LAUNCH("k_sync_place", k_sync_place, dim3(grid_for(b.N + 1)), dim3(256), 0, s, b, (const u32 *)v2[c],
              (const u32 *)b.e_scan1, b.e_scan0);
    scan_exclusive(b.e_scan0, (u64)b.N + 1, b.part, s, nullptr, &b.prm->n_sync);
    RD_LAUNCH("k_sync_phase", k_sync_phase, dim3(grid_for(b.N)), dim3(256), 0, s, b, (const u32 *)k2[c],
              (const u32 *)b.e_scan0);
    RD_LAUNCH("k_thread_maxbar", k_thread_maxbar, dim3(grid_for(b.T, 64)), dim3(64), 0, s, b, (const u32 *)b.e_scan0);
    scan_exclusive(b.blk_maxbar, (u64)b.B + 1, b.part, s);  // -> instance offsets (inst_off)
    FillJobs f = {};
    f.P = b.prm;
    f.add(b.inst_cnt, b.N, 0, 4, 0, b.inst_off + b.B);
    f.add(b.inst_last, b.N, 0, 4, 0, b.inst_off + b.B);
    fill_many(f, "k_fill_inst", s);
    RD_LAUNCH("k_bar_register", k_bar_register, dim3(grid_for(b.T, 64)), dim3(64), 0, s, b);
}

void prep_elements(const Bufs &b, const u64 *acc_mask, hipStream_t s) {
    if (b.N) RD_LAUNCH("k_elements", k_elements, dim3(b.n_tiles), dim3(WG_THREADS), 0, s, b, acc_mask);
}

// releases/acquires, knowledge columns (rt_scan gets T+1 words), block-barrier validation
void prep_thread_sync(const Bufs &b, u32 *rt_scan, hipStream_t s) {
    RD_LAUNCH("k_thread_sync", k_thread_sync, dim3(grid_for(b.T, 64)), dim3(64), 0, s, b, rt_scan);
    scan_exclusive(rt_scan, (u64)b.T + 1, b.part, s);
}

void prep_validate_wbar(const Bufs &b, hipStream_t s) {
    RD_LAUNCH("k_validate_wbar", k_validate_wbar, dim3(grid_for(b.T, 64)), dim3(64), 0, s, b);
}

}  // namespace rd
