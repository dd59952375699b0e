// rd_sort.hip -- stable LSD radix sort of u32 keys with up to three u32 payload arrays (gfx950).
//
// Each pass: (1) every tile of TILE keys writes its digit histogram, digit-major, (2) one exclusive
// scan over the (digit, tile) matrix gives every (digit, tile) its output base, (3) every tile ranks
// its keys stably -- wavefront ballots find the lanes that share a digit, per-wave running counts in
// LDS order the steps, per-digit wave prefixes order the waves -- stages keys and payloads through
// LDS in sorted order and writes them out as contiguous runs per digit.
// Stability across passes keeps trace order inside a location, which the segment check relies on.
#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

template <int R>
__global__ __launch_bounds__(WG_THREADS) void k_radix_hist(const u32 *keys, const u32 *n_dev, u32 n_host,
                                                          u32 shift, const u32 *bits_dev, u32 *hist, u32 n_tiles) {
    constexpr u32 ND = 1u << R;
    __shared__ u32 h[ND];
    const u32 n = n_dev ? *n_dev : n_host;
    if (bits_dev && shift >= *bits_dev) return;  // pass not needed
    for (u32 d = threadIdx.x; d < ND; d += WG_THREADS) h[d] = 0;
    __syncthreads();
    const u64 base = (u64)blockIdx.x * TILE;
    for (u32 k = 0; k < ITEMS; k++) {
        const u64 i = base + (u64)k * WG_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (ND - 1)], 1u);
    }
    __syncthreads();
    for (u32 d = threadIdx.x; d < ND; d += WG_THREADS) hist[(u64)d * n_tiles + blockIdx.x] = h[d];
}

template <int R>
struct ScatterLds {
    u32 wcnt[WAVES][1u << R];  // per-wave counts -> tile-local start of (wave, digit)
    u32 dg[1u << R];           // global output base minus tile-local start, per digit
    u32 stage[TILE];
    u32 wtot[WAVES];
};

template <int R>
__global__ __launch_bounds__(WG_THREADS) void k_radix_scatter(
    const u32 *kin, const u32 *p0in, const u32 *p1in, const u32 *p2in, u32 *kout, u32 *p0out, u32 *p1out,
    u32 *p2out, const u32 *n_dev, u32 n_host, u32 shift, const u32 *bits_dev, const u32 *hist, u32 n_tiles) {
    constexpr u32 ND = 1u << R, MASK = ND - 1;
    __shared__ ScatterLds<R> L;
    const u32 n = n_dev ? *n_dev : n_host;
    if (bits_dev && shift >= *bits_dev) return;
    const u64 tile0 = (u64)blockIdx.x * TILE;
    if (tile0 >= n) return;
    const u32 w = threadIdx.x >> 6, lane = lane_id();
    for (u32 d = threadIdx.x; d < ND; d += WG_THREADS)
        for (u32 q = 0; q < WAVES; q++) L.wcnt[q][d] = 0;
    __syncthreads();
    const u64 wbase = tile0 + (u64)w * ITEMS * 64;
    u32 key[ITEMS], off[ITEMS];
    // ---- rank: position of each key among the equal digits of its wave, in input order
#pragma unroll
    for (int k = 0; k < ITEMS; k++) {
        const u64 i = wbase + (u64)k * 64 + lane;
        const bool valid = i < n;
        key[k] = valid ? kin[i] : 0;
        const u32 d = (key[k] >> shift) & MASK;
        u64 m = ballot(valid);
#pragma unroll
        for (int bit = 0; bit < R; bit++) {
            const u64 bb = ballot((d >> bit) & 1u);
            m &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const u32 rank = popc64(m & lanemask_lt());
        u32 old = 0;
        if (valid) old = L.wcnt[w][d];
        // wave-synchronous: every lane of the group has read the old count before the leader writes
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) L.wcnt[w][d] = old + popc64(m);
        __builtin_amdgcn_wave_barrier();
        off[k] = old + rank;
    }
    __syncthreads();
    // ---- per digit: wave prefixes and tile totals; tile-local digit starts
    constexpr u32 DPT = ND / WG_THREADS > 0 ? ND / WG_THREADS : 1;  // digits per thread
    u32 tot[DPT];
    u32 mysum = 0;
#pragma unroll
    for (u32 j = 0; j < DPT; j++) {
        const u32 d = threadIdx.x * DPT + j;
        u32 run = 0;
        if (d < ND) {
            for (u32 q = 0; q < WAVES; q++) { const u32 c = L.wcnt[q][d]; L.wcnt[q][d] = run; run += c; }
        }
        tot[j] = run;
        mysum += run;
    }
    // exclusive scan of mysum over the 256 threads
    u32 x = mysum;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
        const u32 y = __shfl_up(x, dd, 64);
        if (lane >= (u32)dd) x += y;
    }
    if (lane == 63) L.wtot[w] = x;
    __syncthreads();
    u32 pre = x - mysum;
    for (u32 q = 0; q < w; q++) pre += L.wtot[q];
#pragma unroll
    for (u32 j = 0; j < DPT; j++) {
        const u32 d = threadIdx.x * DPT + j;
        if (d < ND) {
            for (u32 q = 0; q < WAVES; q++) L.wcnt[q][d] += pre;
            L.dg[d] = hist[(u64)d * n_tiles + blockIdx.x] - pre;
        }
        pre += tot[j];
    }
    __syncthreads();
    const u32 cnt_tile = (u32)((n - tile0) < (u64)TILE ? (n - tile0) : (u64)TILE);
    // ---- local sorted positions
    u32 lpos[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; k++) {
        const u64 i = wbase + (u64)k * 64 + lane;
        const u32 d = (key[k] >> shift) & MASK;
        lpos[k] = i < n ? L.wcnt[w][d] + off[k] : NONE;
    }
    // ---- keys through LDS, then each payload array
    u32 gpos[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; k++) if (lpos[k] != NONE) L.stage[lpos[k]] = key[k];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; r++) {
        const u32 j = r * WG_THREADS + threadIdx.x;
        gpos[r] = NONE;
        if (j < cnt_tile) {
            const u32 kk = L.stage[j], d = (kk >> shift) & MASK;
            gpos[r] = L.dg[d] + j;
            kout[gpos[r]] = kk;
        }
    }
    const u32 *pin[3] = {p0in, p1in, p2in};
    u32 *pout[3] = {p0out, p1out, p2out};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (!pin[a]) continue;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ITEMS; k++) {
            const u64 i = wbase + (u64)k * 64 + lane;
            if (lpos[k] != NONE) L.stage[lpos[k]] = pin[a][i];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ITEMS; r++) {
            const u32 j = r * WG_THREADS + threadIdx.x;
            if (gpos[r] != NONE) pout[a][gpos[r]] = L.stage[j];
        }
    }
}

static const char *const kScatterName[2][4] = {
    {"k_sort_scatter_p0", "k_sort_scatter_p1", "k_sort_scatter_p2", "k_sort_scatter_p3"},
    {"k_pair_scatter", "k_pair_scatter", "k_pair_scatter", "k_pair_scatter"}};

template <int R>
static void radix_pass(const u32 *kin, const u32 *p0, const u32 *p1, const u32 *p2, u32 *kout, u32 *q0, u32 *q1,
                       u32 *q2, const u32 *n_dev, u32 n_host, u32 shift, const u32 *bits_dev, u32 *hist, u32 *part,
                       u32 n_tiles, hipStream_t s, int pairs, int pass) {
    RD_LAUNCH(pairs ? "k_pair_hist" : "k_sort_hist", k_radix_hist<R>, dim3(n_tiles), dim3(WG_THREADS), 0, s, kin, n_dev, n_host, shift, bits_dev,
                       hist, n_tiles);
    scan_exclusive(hist, (u64)n_tiles << R, part, s);
    RD_LAUNCH(kScatterName[pairs][pass & 3], k_radix_scatter<R>, dim3(n_tiles), dim3(WG_THREADS), 0, s, kin, p0, p1, p2, kout, q0, q1, q2,
                       n_dev, n_host, shift, bits_dev, hist, n_tiles);
}

// Elements: key = location, payloads = index, tid, info.  The number of passes follows the key width
// found on the device; passes past it do nothing, so the result is in buffer (passes % 2).
void sort_elements(const Bufs &b, hipStream_t s) {
    if (!b.N) return;
    const u32 *n_dev = &b.prm->n_acc, *bits = &b.prm->key_bits;
    const u32 R = b.radix_bits;
    const u32 max_passes = (32 + R - 1) / R;
    for (u32 pass = 0; pass < max_passes; pass++) {
        const u32 c = pass & 1, o = c ^ 1;
        if (R == 11)
            radix_pass<11>(b.ekey[c], b.eidx[c], b.etid[c], b.einfo[c], b.ekey[o], b.eidx[o], b.etid[o], b.einfo[o],
                           n_dev, 0, pass * R, bits, b.hist, b.part, b.n_tiles, s, 0, pass);
        else
            radix_pass<8>(b.ekey[c], b.eidx[c], b.etid[c], b.einfo[c], b.ekey[o], b.eidx[o], b.etid[o], b.einfo[o],
                          n_dev, 0, pass * R, bits, b.hist, b.part, b.n_tiles, s, 0, pass);
    }
}

// Pairs: sort by (first, second) -- LSD over second, then over first.  m is known on the host.
u32 sort_pairs_host(const Bufs &b, u32 m, hipStream_t s) {
    u32 bits = 0;
    while (bits < 32 && ((u64)1 << bits) < (u64)b.N) bits++;
    const u32 R = 8, per_half = (bits + R - 1) / R;
    const u32 n_tiles = (m + TILE - 1) / TILE;
    u32 cur = 0;
    for (u32 half = 0; half < 2; half++) {
        for (u32 pass = 0; pass < per_half; pass++) {
            const u32 o = cur ^ 1;
            if (half == 0)
                radix_pass<8>(b.psecond[cur], b.pfirst[cur], nullptr, nullptr, b.psecond[o], b.pfirst[o], nullptr,
                              nullptr, nullptr, m, pass * R, nullptr, b.hist, b.part, n_tiles, s, 1, pass);
            else
                radix_pass<8>(b.pfirst[cur], b.psecond[cur], nullptr, nullptr, b.pfirst[o], b.psecond[o], nullptr,
                              nullptr, nullptr, m, pass * R, nullptr, b.hist, b.part, n_tiles, s, 1, pass);
            cur = o;
        }
    }
    return cur;
}

}  // namespace rd
