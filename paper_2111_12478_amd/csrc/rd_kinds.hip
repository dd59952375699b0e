// Unique race kinds (the "unique kinds" of races counted in Table 2, Section 6): a kind is the
// unordered pair of the two racing accesses' site ids (the records' aux words).  From the sorted
// report the kinds are built on the device: site pairs gathered per race pair, sorted by
// (site_lo, site_hi) with the pair sort, heads of equal runs flagged and scanned, one record per
// run with the run's length as the count.
#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

__global__ __launch_bounds__(WG_THREADS) void k_kind_keys(const u64 *report, const uint4 *ev, u32 m, u32 *lo,
                                                          u32 *hi) {
    for (u32 i = blockIdx.x * WG_THREADS + threadIdx.x; i < m; i += gridDim.x * WG_THREADS) {
        const u64 r = report[i];
        const u32 sa = ev[(u32)r].w, sb = ev[(u32)(r >> 32)].w;
        lo[i] = sa < sb ? sa : sb;
        hi[i] = sa < sb ? sb : sa;
    }
}

__device__ inline bool kind_head(const u32 *lo, const u32 *hi, u32 i) {
    return i == 0 || lo[i] != lo[i - 1] || hi[i] != hi[i - 1];
}

// flag[i] = 1 where a run of equal site pairs starts (i < m), flag[m] = 0 (the scan's total slot)
__global__ __launch_bounds__(WG_THREADS) void k_kind_heads(const u32 *lo, const u32 *hi, u32 m, u32 *flag) {
    for (u32 i = blockIdx.x * WG_THREADS + threadIdx.x; i <= m; i += gridDim.x * WG_THREADS)
        flag[i] = i < m && kind_head(lo, hi, i) ? 1u : 0u;
}

// ex = exclusive scan of the flags: a run starting at i is kind ex[i]; its start goes to start[]
__global__ __launch_bounds__(WG_THREADS) void k_kind_write(const u32 *lo, const u32 *hi, const u32 *ex, u32 m,
                                                           u32 *rec, u32 *start) {
    for (u32 i = blockIdx.x * WG_THREADS + threadIdx.x; i < m; i += gridDim.x * WG_THREADS) {
        if (!kind_head(lo, hi, i)) continue;
        const u32 k = ex[i];
        rec[3 * k] = lo[i];
        rec[3 * k + 1] = hi[i];
        start[k] = i;
    }
}

__global__ __launch_bounds__(WG_THREADS) void k_kind_count(const u32 *ex, u32 m, const u32 *start, u32 *rec,
                                                           u32 *n_out) {
    const u32 nk = ex[m];
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = nk;
    for (u32 k = blockIdx.x * WG_THREADS + threadIdx.x; k < nk; k += gridDim.x * WG_THREADS)
        rec[3 * k + 2] = (k + 1 < nk ? start[k + 1] : m) - start[k];
}

void race_kinds(const Bufs &b, u32 m, u32 *scratch, u32 *rec, u32 *n_out, hipStream_t s) {
    u32 *lo0 = scratch, *hi0 = scratch + (u64)m, *lo1 = scratch + 2ull * m, *hi1 = scratch + 3ull * m;
    u32 *flag = scratch + 4ull * m, *part = scratch + 5ull * m + 1;
    const u64 blocks = ((u64)m + WG_THREADS) / WG_THREADS;
    const u32 grid = blocks < 4096 ? (u32)blocks : 4096u;
    RD_LAUNCH("k_kind_keys", k_kind_keys, dim3(grid), dim3(WG_THREADS), 0, s, b.preport, b.ev, m, lo0, hi0);
    u32 *const f[2] = {lo0, lo1}, *const s2[2] = {hi0, hi1};
    static const char *const names[3] = {"k_kind_count_digits", "k_kind_reduce", "k_kind_sweep"};
    sort_pairs_in(b, f, s2, nullptr, m, m, 4, names, s);  // 2 x 4 passes: the result is in lo0 / hi0
    RD_LAUNCH("k_kind_heads", k_kind_heads, dim3(grid), dim3(WG_THREADS), 0, s, lo0, hi0, m, flag);
    scan_exclusive(flag, (u64)m + 1, part, s);
    RD_LAUNCH("k_kind_write", k_kind_write, dim3(grid), dim3(WG_THREADS), 0, s, lo0, hi0, flag, m, rec, lo1);
    RD_LAUNCH("k_kind_count", k_kind_count, dim3(grid), dim3(WG_THREADS), 0, s, flag, m, lo1, rec, n_out);
}

}  // namespace rd
