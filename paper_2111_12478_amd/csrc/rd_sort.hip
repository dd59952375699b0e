// rd_sort.hip -- stable LSD radix sort (8-bit digits) of u32 keys with one or three u32 payload
// arrays (gfx950), one sweep kernel per pass.
//
// Digit totals come first: every tile writes one row of per-tile digit counts for all passes (the
// location sort counts in k_elements, which produces the keys; the pair sort in k_pair_count), and
// k_sort_reduce adds the rows into per-pass totals.  Each pass is then a single kernel: a workgroup
// takes the next tile ticket from a counter (so every earlier tile is already being worked on),
// ranks its keys stably -- wavefront ballots find the lanes that share a digit, per-wave running
// counts in LDS order the steps, per-digit wave prefixes order the waves -- publishes its per-digit
// counts and looks back over the earlier tiles' published counts for its output offsets (decoupled
// look-back, four predecessor words per round).  Keys and payloads go through LDS in sorted order and
// out as contiguous runs per digit.  The look-back words carry all the information exchanged between
// workgroups (no other data is published through them), so they are relaxed device-scope atomics:
// coherent across the XCDs without the L2 write-back / invalidate an acquire or release would add
// to every access.  Every wait is bounded: a look-back that does not finish within its spin limit
// sets ERR_SORT and goes on, so the kernel always ends.  Two arrays of look-back words alternate
// between passes; each pass clears its tiles' words in the other array for the next pass.
// Stability keeps trace order inside a location, which the segment check relies on.
#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

constexpr u64 ST_AGG = 1ull << 62, ST_PRE = 2ull << 62, ST_FLAGS = 3ull << 62, ST_VAL = (1ull << 62) - 1;
constexpr u32 SPIN_LIMIT = 1u << 20;

static_assert(WG_THREADS == SORT_ND, "one digit per thread in the 8-bit counting kernels");

// Pair sort digit counts (8-bit digits): tile t writes row t ([pass][digit]) of the per-tile
// counts and clears its look-back words of the first pass; workgroup 0 clears the totals (added up
// by the next kernel).  Pass p < half takes digit p of `second`, pass p >= half digit p - half of
// `first`; np passes in all (a single-key sort passes first == second and half == np).  The count
// is *m_dev when m_dev is set (workgroups past the last tile only exit), else m_host.
__global__ __launch_bounds__(WG_THREADS) void k_pair_count(const u32 *first, const u32 *second, const u32 *m_dev,
                                                           u32 m_host, u32 half, u32 np, u32 *partial,
                                                           u64 *status0, u32 *tot) {
    __shared__ u32 h[MAX_SORT_PASSES][SORT_ND];
    const u32 m = m_dev ? *m_dev : m_host;
    if (blockIdx.x == 0)  // totals and the tile tickets that follow them
        for (u32 q = threadIdx.x; q < MAX_SORT_PASSES * SORT_NDS + MAX_SORT_PASSES; q += WG_THREADS) tot[q] = 0;
    for (u32 tile = blockIdx.x; (u64)tile * TILE < m; tile += gridDim.x) {
    const u64 base = (u64)tile * TILE;
#pragma unroll
    for (u32 q = 0; q < MAX_SORT_PASSES; q++) h[q][threadIdx.x] = 0;
    status0[(u64)tile * SORT_ND + threadIdx.x] = 0;
    __syncthreads();
    u32 f[ITEMS], sc[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; k++) {
        const u64 i = base + (u64)k * WG_THREADS + threadIdx.x;
        f[k] = i < m ? first[i] : 0;
        sc[k] = i < m ? second[i] : 0;
    }
#pragma unroll
    for (int k = 0; k < ITEMS; k++) {
        if (base + (u64)k * WG_THREADS + threadIdx.x >= m) continue;
        for (u32 q = 0; q < np; q++) {
            const u32 key = q < half ? sc[k] : f[k];
            const u32 sh = SORT_RB * (q < half ? q : q - half);
            atomicAdd(&h[q][(key >> sh) & (SORT_ND - 1)], 1u);
        }
    }
    __syncthreads();
    u32 *row = partial + (u64)tile * MAX_SORT_PASSES * SORT_NDS;
    for (u32 q = 0; q < np; q++) row[q * SORT_NDS + threadIdx.x] = h[q][threadIdx.x];
    __syncthreads();
    }
}

// Adds the rows of per-tile counts into the pass totals: workgroup (p, c) sums rows
// [64c, 64c + 64) of pass p for the 2^rb digits.  Passes past the key width (bits_dev) are skipped.
// The number of rows is n_rows, or ceil(*items_dev / TILE) when items_dev is set.  With clear_words,
// the workgroups also clear the first look-back array (clear_words words).
__global__ __launch_bounds__(WG_THREADS) void k_sort_reduce(const u32 *partial, u32 row_passes, u32 n_rows,
                                                            const u32 *items_dev, const u32 *bits_dev, u32 rb,
                                                            u32 *tot, u64 *status0, u64 clear_words) {
    if (status0) {
        const u64 nthreads = (u64)gridDim.x * gridDim.y * WG_THREADS;
        const u64 me = ((u64)blockIdx.y * gridDim.x + blockIdx.x) * WG_THREADS + threadIdx.x;
        for (u64 i = me; i < clear_words; i += nthreads) status0[i] = 0;
    }
    const u32 p = blockIdx.x, nd = 1u << rb;
    if (bits_dev && p >= (*bits_dev + rb - 1) / rb) return;
    if (items_dev) n_rows = (u32)(((u64)*items_dev + TILE - 1) / TILE);
    const u32 r0 = blockIdx.y * 64, r1 = r0 + 64 < n_rows ? r0 + 64 : n_rows;
    if (r0 >= r1) return;
    const u64 stride = (u64)row_passes * SORT_NDS;
    for (u32 d = threadIdx.x; d < nd; d += WG_THREADS) {
        const u32 *src = partial + (u64)p * SORT_NDS + d;
        u32 acc = 0, r = r0;
        for (; r + 16 <= r1; r += 16) {
            u32 v[16];
#pragma unroll
            for (int j = 0; j < 16; j++) v[j] = src[(u64)(r + j) * stride];
#pragma unroll
            for (int j = 0; j < 16; j++) acc += v[j];
        }
        for (; r < r1; r++) acc += src[(u64)r * stride];
        if (acc) atomicAdd(&tot[p * SORT_NDS + d], acc);
    }
}

template <int RB, int NW, int NI>
struct SweepLds {
    u32 wcnt[NW][1 << RB];  // per-wave digit counts -> tile-local start of (wave, digit)
    u32 dg[1 << RB];        // global output position minus tile-local position, per digit
    u32 stage[NW * 64 * NI];
    u32 wtot[2][NW];
    u32 tile;
};

struct SweepArgs {
    const u32 *kin, *pin[3];
    u32 *kout, *pout[3];
    const u32 *n_dev;
    u32 n_host, shift, pass;
    const u32 *bits_dev;  // non-null: skip the pass when shift >= *bits_dev
    u64 *status_cur, *status_next;
    const u32 *tot;       // digit totals of the pass ([pass][SORT_NDS])
    u32 *ctr, *err;
    const DevParams *prm;  // the element sort: packed elements move their first two payloads only
    u32 T;                 // ... (threads of the trace: whether the thread word is packed)
};

constexpr int LOOKBACK = 4;  // predecessor words read at once per digit

// One pass: 2^RB digits, NW wavefronts per workgroup, NI items per lane (tile NW * 64 * NI).
// Look-back words of a tile: 2^RB, consecutive.
template <int NP, int RB, int NW, int NI, bool LOOP = false>
__global__ __launch_bounds__(NW * 64) void k_sort_sweep(SweepArgs a) {
    constexpr u32 ND = 1u << RB, DM = ND - 1, THREADS = NW * 64, TS = THREADS * NI;
    static_assert(ND <= THREADS, "one digit per thread");
    __shared__ SweepLds<RB, NW, NI> L;
    if (a.bits_dev && a.shift >= *a.bits_dev) return;  // past the key width: the pass is not needed
    // digits come from the key bits only (packed elements carry more above them)
    const u32 kmask = a.bits_dev ? key_mask(*a.bits_dev) : ~0u;
    const u32 np_run = NP == 3 && a.prm &&
                               (packed_elements(a.prm->key_bits, a.prm->max_phase) ||
                                tinfo_elements(a.prm->key_bits, a.prm->max_phase, a.T))
                           ? 2u
                           : (u32)NP;
    const u32 n = a.n_dev ? *a.n_dev : a.n_host;
    const u32 n_tiles = (u32)(((u64)n + TS - 1) / TS);
    const u32 w = threadIdx.x >> 6, lane = lane_id(), dme = threadIdx.x;  // digit dme when dme < ND
    const bool has_d = dme < ND;
    // tiles by ticket, in order; with LOOP, until none is left (a grid smaller than the tile count)
    do {
    if (threadIdx.x == 0) {
        // looping grids outnumber the tiles of small sorts: the ticket counter only grows, so once
        // it is past the tiles a workgroup leaves without taking one
        const u32 seen = LOOP ? __hip_atomic_load(&a.ctr[a.pass], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        L.tile = seen >= n_tiles && LOOP ? seen : atomicAdd(&a.ctr[a.pass], 1u);
    }
    if (has_d) {
#pragma unroll
        for (u32 q = 0; q < NW; q++) L.wcnt[q][dme] = 0;
    }
    __syncthreads();
    const u32 tile = L.tile;
    if (tile >= n_tiles) return;  // no tile for this workgroup; no later tile waits on it
    const u64 tile0 = (u64)tile * TS;
    const u64 wbase = tile0 + (u64)w * NI * 64;
    const u32 shift = a.shift;
    const u32 total = has_d ? a.tot[a.pass * SORT_NDS + dme] : 0u;
    // the element arrays are padded to whole tiles: their loads need no bounds test (items past n
    // are loaded and never used)
    constexpr bool PADDED = NP == 3;
    static_assert(!PADDED || TS <= SORT_MAX_TILE, "element tiles fit the padding");
    // keys now; each payload array is read when it goes through the LDS (fewer live registers)
    u32 key[NI], off[NI];
#pragma unroll
    for (int k = 0; k < NI; k++) {
        const u64 i = wbase + (u64)k * 64 + lane;
        key[k] = PADDED || i < n ? a.kin[i] : 0;
    }
    // rank: position of each key among the equal digits of its wave, in input order
#pragma unroll
    for (int k = 0; k < NI; k++) {
        const bool valid = wbase + (u64)k * 64 + lane < n;
        const u32 d = ((key[k] & kmask) >> shift) & DM;
        // lanes with the same digit: the intersection over the digit bits of the lanes that agree
        // with this lane on the bit, in 32-bit halves: with s = 0 or ~0 the lane's bit, the lanes
        // that agree are ~(ballot ^ s)
        const u64 vm = ballot(valid);
        u32 mlo = (u32)vm, mhi = (u32)(vm >> 32);
#pragma unroll
        for (int bit = 0; bit < RB; bit++) {
            const u32 sb = (u32)((int)(d << (31 - bit)) >> 31);
            const u64 bb = ballot(sb != 0u);
            mlo &= ~((u32)bb ^ sb);
            mhi &= ~((u32)(bb >> 32) ^ sb);
        }
        const u32 rank = __builtin_amdgcn_mbcnt_hi(mhi, __builtin_amdgcn_mbcnt_lo(mlo, 0u));
        u32 old = 0;
        if (valid) old = L.wcnt[w][d];
        // wave-synchronous: every lane of the group has read the old count before the leader writes
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) L.wcnt[w][d] = old + __builtin_popcount(mlo) + __builtin_popcount(mhi);
        __builtin_amdgcn_wave_barrier();
        // tile-local rank below 2^14, the digit above bit 16 (one register per item)
        off[k] = valid ? (old + rank) | (d << 16) : NONE;
        // computed here: left to the compiler, the ballot masks of all items stay live until the
        // ranks are used after the barrier (four registers per item instead of one)
        __asm__ volatile("" : "+v"(off[k]));
    }
    __syncthreads();
    // digit dme: exclusive wave prefixes and the tile's count
    u32 cnt = 0;
    if (has_d) {
#pragma unroll
        for (u32 q = 0; q < NW; q++) {
            const u32 c = L.wcnt[q][dme];
            L.wcnt[q][dme] = cnt;
            cnt += c;
        }
    }
    u64 *my = a.status_cur + (u64)tile * ND + dme;
    if (has_d) {
        __hip_atomic_store(my, (tile == 0 ? ST_PRE : ST_AGG) | (u64)cnt, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        // the next pass's look-back words of this tile start cleared
        if (a.status_next) a.status_next[(u64)tile * ND + dme] = 0;
    }
    // exclusive scans over the digits: tile-local starts (cnt) and global digit bases (total)
    u32 x = cnt, y = total;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const u32 xs = __shfl_up(x, o, 64), ys = __shfl_up(y, o, 64);
        if (lane >= (u32)o) { x += xs; y += ys; }
    }
    if (lane == 63) { L.wtot[0][w] = x; L.wtot[1][w] = y; }
    __syncthreads();
    // tile-local start (pre) and global base (gb) of digit dme; (wave, digit) starts in the tile
    u32 pre = 0, gb = 0;
    if (has_d) {
        pre = x - cnt;
        gb = y - total;
        for (u32 q = 0; q < w; q++) { pre += L.wtot[0][q]; gb += L.wtot[1][q]; }
#pragma unroll
        for (u32 q = 0; q < NW; q++) L.wcnt[q][dme] += pre;
    }
    __syncthreads();
    // local sorted positions, and the keys into the LDS: the key registers are free from here
#pragma unroll
    for (int k = 0; k < NI; k++) {
        if (off[k] != NONE) {
            off[k] = (off[k] & 0xffffu) + L.wcnt[w][off[k] >> 16];
            L.stage[off[k]] = key[k];
        }
    }
    // the first payload's loads are in flight during the look-back
    u32 pay[NI];
#pragma unroll
    for (int k = 0; k < NI; k++) pay[k] = PADDED || off[k] != NONE ? a.pin[0][wbase + (u64)k * 64 + lane] : 0u;
    // look back: digit dme's count in all earlier tiles, LOOKBACK predecessor words per round
    u64 excl = 0;
    if (has_d && tile > 0) {
        int i = (int)tile - 1;
        u32 spins = 0;
        for (;;) {
            u64 v[LOOKBACK];
#pragma unroll
            for (int j = 0; j < LOOKBACK; j++)
                v[j] = i - j >= 0 ? __hip_atomic_load(a.status_cur + (u64)(i - j) * ND + dme, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT)
                                  : ST_PRE;  // before tile 0: nothing
            bool done = false, stall = false;
#pragma unroll
            for (int j = 0; j < LOOKBACK; j++) {
                if (done || stall) continue;
                const u64 f = v[j] & ST_FLAGS;
                if (f != ST_AGG && f != ST_PRE) { stall = true; continue; }
                excl += v[j] & ST_VAL;
                i--;
                if (f == ST_PRE) done = true;
            }
            if (done) break;
            if (stall) {
                if (++spins > SPIN_LIMIT) {
                    atomicOr(a.err, ERR_SORT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __hip_atomic_store(my, ST_PRE | (excl + cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (has_d) L.dg[dme] = gb + (u32)excl - pre;  // global position minus tile-local position
    __syncthreads();
    const u32 cnt_tile = (u32)((n - tile0) < (u64)TS ? (n - tile0) : (u64)TS);
    // keys out, in runs per digit; each sorted position's digit is kept (packed) for the payloads
    constexpr int DW = RB <= 8 ? 8 : 16, DPW = 32 / DW;
    u32 dgt[(NI + DPW - 1) / DPW];
#pragma unroll
    for (int r = 0; r < (NI + DPW - 1) / DPW; r++) dgt[r] = 0;
#pragma unroll
    for (int r = 0; r < NI; r++) {
        const u32 j = r * THREADS + threadIdx.x;
        if (j < cnt_tile) {
            const u32 kk = L.stage[j];
            const u32 d = ((kk & kmask) >> shift) & DM;
            dgt[r / DPW] |= d << (DW * (r % DPW));
            a.kout[L.dg[d] + j] = kk;
        }
    }
    // payloads through the LDS; the next one's loads are issued before this one is written out
#pragma unroll
    for (int q = 0; q < NP; q++) {
        if ((u32)q >= np_run) break;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NI; k++)
            if (off[k] != NONE) L.stage[off[k]] = pay[k];
        if ((u32)q + 1 < np_run) {
#pragma unroll
            for (int k = 0; k < NI; k++)
                pay[k] = PADDED || off[k] != NONE ? a.pin[q + 1][wbase + (u64)k * 64 + lane] : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NI; r++) {
            const u32 j = r * THREADS + threadIdx.x;
            if (j < cnt_tile) {
                const u32 d = (dgt[r / DPW] >> (DW * (r % DPW))) & ((1u << DW) - 1);
                a.pout[q][L.dg[d] + j] = L.stage[j];
            }
        }
    }
    if (LOOP) __syncthreads();  // the LDS is reused for the next tile
    } while (LOOP);
}

static const char *const kSweepName[ELEM_MAX_PASSES] = {"k_sort_sweep_p0", "k_sort_sweep_p1", "k_sort_sweep_p2",
                                                        "k_sort_sweep_p3", "k_sort_sweep_p4"};

static SweepArgs sweep_args(const Bufs &b, u32 pass, u32 n_passes, u32 shift, const u32 *n_dev, u32 n_host,
                            const u32 *bits_dev) {
    SweepArgs a = {};
    a.n_dev = n_dev;
    a.n_host = n_host;
    a.shift = shift;
    a.pass = pass;
    a.bits_dev = bits_dev;
    a.status_cur = b.sort_status + (pass & 1) * b.sort_status_stride;
    a.status_next = pass + 1 < n_passes ? b.sort_status + ((pass + 1) & 1) * b.sort_status_stride : nullptr;
    a.tot = b.sort_tot;
    a.ctr = b.sort_ctr;
    a.err = &b.prm->err;
    return a;
}

template <int RB, int NW, int NI>
static void elem_passes(const Bufs &b, const u32 *n_dev, const u32 *bits, hipStream_t s) {
    constexpr u32 TS = NW * 64 * NI;
    constexpr u32 PASSES = (32 + RB - 1) / RB;
    const u32 tiles = (u32)(((u64)b.N + TS - 1) / TS);
    for (u32 pass = 0; pass < PASSES; pass++) {
        const u32 c = pass & 1, o = c ^ 1;
        SweepArgs a = sweep_args(b, pass, PASSES, pass * RB, n_dev, 0, bits);
        a.kin = b.ekey[c];
        a.pin[0] = b.eidx[c];
        a.pin[1] = b.etid[c];
        a.pin[2] = b.einfo[c];
        a.kout = b.ekey[o];
        a.pout[0] = b.eidx[o];
        a.pout[1] = b.etid[o];
        a.pout[2] = b.einfo[o];
        a.prm = b.prm;
        a.T = b.T;
        RD_LAUNCH(kSweepName[pass], (k_sort_sweep<3, RB, NW, NI>), dim3(tiles), dim3(NW * 64), 0, s, a);
    }
}

// Elements: key = location, payloads = index, tid, info, with the context's variant.  The digit
// counts (per-tile rows), the zeroed totals and tickets come from earlier kernels (k_elements,
// k_init_params); k_sort_reduce clears the first look-back array.  Passes past the key width found
// on the device do nothing, so the result is in buffer (passes % 2), passes = ceil(key_bits / rb).
void sort_elements(const Bufs &b, hipStream_t s) {
    if (!b.N) return;
    const SortVariant v = kSortVariants[b.sort_variant < N_SORT_VARIANTS ? b.sort_variant : 0];
    const u32 *n_dev = &b.prm->n_acc, *bits = &b.prm->key_bits;
    const u32 passes = (32 + v.rb - 1) / v.rb, ts = v.waves * 64 * v.items;
    const u64 clear = (((u64)b.N + ts - 1) / ts) << v.rb;
    RD_LAUNCH("k_sort_reduce", k_sort_reduce, dim3(passes, (b.n_tiles + 63) / 64), dim3(WG_THREADS), 0, s,
              b.sort_partial, ELEM_MAX_PASSES, b.n_tiles, (const u32 *)nullptr, bits, v.rb, b.sort_tot,
              b.sort_status, clear);
    switch (b.sort_variant) {
    case 1: elem_passes<8, 8, 8>(b, n_dev, bits, s); break;
    case 2: elem_passes<8, 8, 16>(b, n_dev, bits, s); break;
    case 3: elem_passes<7, 4, 16>(b, n_dev, bits, s); break;
    case 4: elem_passes<7, 8, 16>(b, n_dev, bits, s); break;
    case 5: elem_passes<9, 8, 16>(b, n_dev, bits, s); break;
    case 6: elem_passes<9, 8, 8>(b, n_dev, bits, s); break;
    case 7: elem_passes<8, 4, 8>(b, n_dev, bits, s); break;
    case 8: elem_passes<7, 8, 8>(b, n_dev, bits, s); break;
    case 9: elem_passes<7, 16, 16>(b, n_dev, bits, s); break;
    case 10: elem_passes<8, 16, 16>(b, n_dev, bits, s); break;
    default: elem_passes<8, 4, 16>(b, n_dev, bits, s); break;
    }
}

// Pairs: sort by (first, second) -- LSD over second, then over first.  The pair count is *m_dev
// (device-driven launches sized for max_m pairs) or m_host.  An even number of passes leaves the
// result in buffer 0.
// Sorts whose item count is read on the device are launched with at most this many workgroups;
// their kernels loop over the tiles.
constexpr u32 SMALL_SORT_GRID = 256;

// Shape of the sweeps of the device-counted sorts (pairs, release/acquire entries): the tile is the
// counting kernels' TILE, spread over 16 wavefronts of 4 items (a small sort's time is one tile's
// latency, which more wavefronts per tile shorten).
constexpr int SMALL_NW = 16, SMALL_NI = 4;
static_assert(SMALL_NW * 64 * SMALL_NI == TILE, "the sweep's tiles are the counted tiles");

// Stable sort of (f[0][i], s2[0][i]) pairs by (first, second), `half` 8-bit digits per word (2 * half
// passes: the result is back in buffer 0).  The count is *m_dev when set, else m_host; launches
// are sized for max_m.  Uses the sort state of the workspace (sized for max_m <= max(elements,
// max_pairs)).
void sort_pairs_in(const Bufs &b, u32 *const f[2], u32 *const s2[2], const u32 *m_dev, u32 m_host, u64 max_m,
                   u32 half, const char *const names[3], hipStream_t s) {
    const u32 passes = 2 * half;
    if (!max_m || !passes) return;
    const u32 n_tiles = (u32)((max_m + TILE - 1) / TILE), grid = n_tiles < SMALL_SORT_GRID ? n_tiles : SMALL_SORT_GRID;
    RD_LAUNCH(names[0], k_pair_count, dim3(grid), dim3(WG_THREADS), 0, s, f[0], s2[0], m_dev, m_host, half, passes,
              b.sort_partial, b.sort_status, b.sort_tot);
    RD_LAUNCH(names[1], k_sort_reduce, dim3(passes, (n_tiles + 63) / 64), dim3(WG_THREADS), 0, s, b.sort_partial,
              MAX_SORT_PASSES, n_tiles, m_dev, (const u32 *)nullptr, SORT_RB, b.sort_tot, (u64 *)nullptr, (u64)0);
    u32 cur = 0;
    for (u32 pass = 0; pass < passes; pass++) {
        const u32 o = cur ^ 1;
        const bool lo = pass < half;
        SweepArgs a = sweep_args(b, pass, passes, (lo ? pass : pass - half) * SORT_RB, m_dev, m_host, nullptr);
        a.kin = lo ? s2[cur] : f[cur];
        a.pin[0] = lo ? f[cur] : s2[cur];
        a.kout = lo ? s2[o] : f[o];
        a.pout[0] = lo ? f[o] : s2[o];
        RD_LAUNCH(names[2], (k_sort_sweep<1, 8, SMALL_NW, SMALL_NI, true>), dim3(grid), dim3(SMALL_NW * 64), 0, s, a);
        cur = o;
    }
}

void sort_pairs(const Bufs &b, const u32 *m_dev, u32 m_host, u64 max_m, hipStream_t s) {
    u32 bits = 0;
    while (bits < 32 && ((u64)1 << bits) < (u64)b.N) bits++;
    const u32 half = (bits + SORT_RB - 1) / SORT_RB;
    u32 *const f[2] = {b.pfirst[0], b.pfirst[1]}, *const s2[2] = {b.psecond[0], b.psecond[1]};
    static const char *const names[3] = {"k_pair_count", "k_pair_reduce", "k_pair_sweep"};
    sort_pairs_in(b, f, s2, m_dev, m_host, max_m, half, names, s);
}

void sort_pairs_to(const Bufs &b, u32 *const f[2], u32 *const s2[2], const u32 *m_dev, u64 max_m, hipStream_t s) {
    u32 bits = 0;
    while (bits < 32 && ((u64)1 << bits) < (u64)b.N) bits++;
    const u32 half = (bits + SORT_RB - 1) / SORT_RB;
    static const char *const names[3] = {"k_ls_pair_count", "k_ls_pair_reduce", "k_ls_pair_sweep"};
    sort_pairs_in(b, f, s2, m_dev, 0, max_m, half, names, s);
}

// Interleaves the sorted pairs into (first, second) records, the report's host layout.
__global__ __launch_bounds__(WG_THREADS) void k_pair_pack(const u32 *first, const u32 *second, const u32 *m_dev,
                                                          u64 max_m, u64 *out) {
    const u64 m = *m_dev < max_m ? *m_dev : max_m;
    for (u64 i = (u64)blockIdx.x * WG_THREADS + threadIdx.x; i < m; i += (u64)gridDim.x * WG_THREADS)
        out[i] = (u64)first[i] | ((u64)second[i] << 32);
}

void pack_pairs(const Bufs &b, hipStream_t s) {
    if (!b.max_pairs) return;
    const u64 tiles = (b.max_pairs + WG_THREADS - 1) / WG_THREADS;
    const u32 grid = tiles < 1024 ? (u32)tiles : 1024u;
    RD_LAUNCH("k_pair_pack", k_pair_pack, dim3(grid), dim3(WG_THREADS), 0, s, b.pfirst[0], b.psecond[0],
              &b.prm->n_pairs_kept, b.max_pairs, b.preport);
}

void pack_pairs_to(const u32 *first, const u32 *second, const u32 *m_dev, u64 max_m, u64 *out, hipStream_t s) {
    if (!max_m) return;
    const u64 tiles = (max_m + WG_THREADS - 1) / WG_THREADS;
    const u32 grid = tiles < 1024 ? (u32)tiles : 1024u;
    RD_LAUNCH("k_ls_pair_pack", k_pair_pack, dim3(grid), dim3(WG_THREADS), 0, s, first, second, m_dev, max_m, out);
}

// Stable sort of (key, value) pairs in k[0], v[0] by key: n = *n_dev items (launches sized for max_n),
// at most `passes` 8-bit passes; with bits_dev the passes past *bits_dev bits do nothing (the result
// is then in buffer ceil(*bits_dev / 8) % 2, else in buffer passes % 2).  Uses the sort state and
// the digit-count rows of the workspace, sized for max_n <= max(elements, max_pairs).
void sort_kv(const Bufs &b, u32 *const k[2], u32 *const v[2], const u32 *n_dev, u64 max_n, u32 passes,
             const u32 *bits_dev, const char *name, hipStream_t s) {
    if (!max_n || !passes) return;
    const u32 n_tiles = (u32)((max_n + TILE - 1) / TILE), grid = n_tiles < SMALL_SORT_GRID ? n_tiles : SMALL_SORT_GRID;
    RD_LAUNCH(name, k_pair_count, dim3(grid), dim3(WG_THREADS), 0, s, k[0], k[0], n_dev, 0u, passes, passes,
              b.sort_partial, b.sort_status, b.sort_tot);
    RD_LAUNCH(name, k_sort_reduce, dim3(passes, (n_tiles + 63) / 64), dim3(WG_THREADS), 0, s, b.sort_partial,
              MAX_SORT_PASSES, n_tiles, n_dev, bits_dev, SORT_RB, b.sort_tot, (u64 *)nullptr, (u64)0);
    for (u32 pass = 0; pass < passes; pass++) {
        const u32 c = pass & 1, o = c ^ 1;
        SweepArgs a = sweep_args(b, pass, passes, pass * SORT_RB, n_dev, 0, bits_dev);
        a.kin = k[c];
        a.pin[0] = v[c];
        a.kout = k[o];
        a.pout[0] = v[o];
        RD_LAUNCH(name, (k_sort_sweep<1, 8, SMALL_NW, SMALL_NI, true>), dim3(grid), dim3(SMALL_NW * 64), 0, s, a);
    }
}

}  // namespace rd
