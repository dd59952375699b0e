// rd_batch.hip -- batched form: many independent traces checked in one pass of the pipeline over
// their concatenation (gfx950).
//
// Traces never interact, so their union is one trace whose race set is the union of theirs, once
// every trace has its own threads, blocks and global words: trace j's blocks become merged blocks
// [blk_off_j, blk_off_j + n_blocks_j) (threads keep their index inside the block; a smaller block
// is padded with threads that have no events, which count as inactive), and its global words are
// shifted into a range of their own, [goff_j, goff_j + span_j).  Shared words, warp barriers and
// block barriers are per block already.  Trace indices are shifted by off_j, so the merged report,
// sorted by (first, second), holds each trace's pairs as one contiguous run, in the trace's own
// canonical order.
#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

// merged index -> trace: the last j with off[j] <= i, searched in [lo, hi]
__device__ inline u32 trace_of(const u32 *off, u32 lo, u32 hi, u32 i) {
    while (lo < hi) {
        const u32 mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline bool is_global_access(u32 meta) {
    const u32 kind = meta & 15u, scope = (meta >> 4) & 3u, space = (meta >> 6) & 1u;
    return (meta >> 7) == 0 && scope <= 2u && space == 0 && (kind <= 2u || kind == 6u || kind == 7u);
}

constexpr u32 RANGE_SLOTS = 16;

// Global-word range of every trace's well-formed accesses.  A tile's traces share LDS slots when
// the tile meets at most RANGE_SLOTS of them, else every element updates its trace directly.
__global__ __launch_bounds__(WG_THREADS) void k_batch_range(BatchTrace *tr, const u32 *off, u32 n_traces, u32 N) {
    __shared__ u32 smin[RANGE_SLOTS], smax[RANGE_SLOTS];
    const u64 tile0 = (u64)blockIdx.x * TILE;
    const u32 last = (u32)((tile0 + TILE < N ? tile0 + TILE : N) - 1);
    const u32 j0 = trace_of(off, 0, n_traces - 1, (u32)tile0);
    const u32 j1 = trace_of(off, j0, n_traces - 1, last);
    const bool slots = j1 - j0 < RANGE_SLOTS;
    if (threadIdx.x < RANGE_SLOTS) { smin[threadIdx.x] = NONE; smax[threadIdx.x] = 0; }
    __syncthreads();
    for (u32 k = 0; k < ITEMS; k++) {
        const u64 i = tile0 + (u64)k * WG_THREADS + threadIdx.x;
        if (i >= N) break;
        const u32 j = j0 == j1 ? j0 : trace_of(off, j0, j1, (u32)i);
        const BatchTrace &t = tr[j];
        const uint4 e = t.ev[i - off[j]];
        if (!is_global_access(e.z) || e.y >= t.n_blocks * t.tpb) continue;
        if (slots) {
            atomicMin(&smin[j - j0], e.x);
            atomicMax(&smax[j - j0], e.x);
        } else {
            atomicMin(&tr[j].gmin, e.x);
            atomicMax(&tr[j].gmax, e.x);
        }
    }
    __syncthreads();
    if (slots && threadIdx.x <= j1 - j0 && smin[threadIdx.x] != NONE) {
        atomicMin(&tr[j0 + threadIdx.x].gmin, smin[threadIdx.x]);
        atomicMax(&tr[j0 + threadIdx.x].gmax, smax[threadIdx.x]);
    }
}

// goff_j = sum of the spans of the traces before j; a total above 2^32 words sets *bad.
__global__ __launch_bounds__(1024) void k_batch_offsets(BatchTrace *tr, u32 n_traces, u32 *bad) {
    __shared__ u64 part[1024];
    const u32 per = (n_traces + 1023) / 1024, lo = threadIdx.x * per;
    const u32 hi = lo + per < n_traces ? lo + per : n_traces;
    u64 s = 0;
    for (u32 j = lo; j < hi; j++) s += tr[j].gmin != NONE ? (u64)tr[j].gmax - tr[j].gmin + 1 : 0;
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 run = 0;
        for (u32 q = 0; q < 1024; q++) { const u64 v = part[q]; part[q] = run; run += v; }
        if (run > 0xffffffffull) atomicOr(bad, 1u);
    }
    __syncthreads();
    u64 run = part[threadIdx.x];
    for (u32 j = lo; j < hi; j++) {
        tr[j].goff = (u32)run;
        run += tr[j].gmin != NONE ? (u64)tr[j].gmax - tr[j].gmin + 1 : 0;
    }
}

// Writes the merged trace: thread ids moved to the trace's merged blocks (an id outside the trace's
// grid becomes NONE, which the checker rejects as a record error), global words of accesses moved
// into the trace's range.
__global__ __launch_bounds__(WG_THREADS) void k_batch_merge(const BatchTrace *tr, const u32 *off, u32 n_traces,
                                                            u32 N, u32 tpb_merged, uint4 *out) {
    const u64 tile0 = (u64)blockIdx.x * TILE;
    const u32 last = (u32)((tile0 + TILE < N ? tile0 + TILE : N) - 1);
    const u32 j0 = trace_of(off, 0, n_traces - 1, (u32)tile0);
    const u32 j1 = trace_of(off, j0, n_traces - 1, last);
    for (u32 k = 0; k < ITEMS; k++) {
        const u64 i = tile0 + (u64)k * WG_THREADS + threadIdx.x;
        if (i >= N) break;
        const u32 j = j0 == j1 ? j0 : trace_of(off, j0, j1, (u32)i);
        const BatchTrace &t = tr[j];
        uint4 e = t.ev[i - off[j]];
        if (e.y < t.n_blocks * t.tpb) {
            const u32 blk = e.y / t.tpb, th = e.y - blk * t.tpb;
            if (is_global_access(e.z)) e.x = e.x - t.gmin + t.goff;
            e.y = (t.blk_off + blk) * tpb_merged + th;
        } else {
            e.y = NONE;
        }
        out[i] = e;
    }
}

// Each trace's run of pairs in the merged report (sorted by first): [pair_lo, pair_hi).
__global__ void k_batch_pairs(BatchTrace *tr, const u32 *off, u32 n_traces, const u32 *first, const u32 *m_dev) {
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_traces) return;
    const u32 m = *m_dev;
    auto lower = [&](u32 x) {
        u32 lo = 0, hi = m;
        while (lo < hi) {
            const u32 mid = (lo + hi) >> 1;
            if (first[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    tr[j].pair_lo = lower(off[j]);
    tr[j].pair_hi = lower(off[j + 1]);
}

void batch_merge(BatchTrace *tr, const u32 *off, u32 n_traces, u32 N, u32 tpb_merged, uint4 *out, u32 *bad,
                 hipStream_t s) {
    if (!N) return;
    const u32 tiles = (N + TILE - 1) / TILE;
    RD_LAUNCH("k_batch_range", k_batch_range, dim3(tiles), dim3(WG_THREADS), 0, s, tr, off, n_traces, N);
    RD_LAUNCH("k_batch_offsets", k_batch_offsets, dim3(1), dim3(1024), 0, s, tr, n_traces, bad);
    RD_LAUNCH("k_batch_merge", k_batch_merge, dim3(tiles), dim3(WG_THREADS), 0, s, tr, off, n_traces, N, tpb_merged,
              out);
}

void batch_pair_ranges(BatchTrace *tr, const u32 *off, u32 n_traces, const Bufs &b, hipStream_t s) {
    RD_LAUNCH("k_batch_pairs", k_batch_pairs, dim3((n_traces + 255) / 256), dim3(256), 0, s, tr, off, n_traces,
              b.pfirst[0], &b.prm->n_pairs_kept);
}

}  // namespace rd
