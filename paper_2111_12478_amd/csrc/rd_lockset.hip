// rd_lockset.hip -- the lockset pass the paper describes for ScoRD (Section 2.2, Section 3; after
// Eraser), over a checked trace on gfx950.
//
// Every access carries the set of locks its thread holds: the critical sections open at it (an
// acquire of a lock word the thread does not hold opens one, with the acquire's scope; the thread's
// next release of that word closes it; a flag publication closes nothing).  Each access is compared
// with the previous access of its location in trace order, lock operations aside, and the pair is
// reported when they conflict, at least one of the two holds a lock (the analysis is skipped for two
// unprotected accesses), and no lock word is held by both with overlapping scopes (either device
// scoped, or both of one block).
//
// The pass reads what the check leaves in the workspace: the per-thread sync lists with their
// release / acquire flags and scopes, and the accesses sorted by location (trace order inside a
// location).  Its own tables and pairs live in the knowledge-vector pool, which the check no longer
// reads once it has ended:
//   k_ls_flag    one flag per sync entry: is it a lock operation (scanned: row of the entry);
//   k_ls_thread  one lane per program thread walks its list, keeping its open sections (at most
//                LS_MAX), and writes
//                the lockset after each lock operation (a row) and, per entry, the row in force;
//   k_ls_check   one lane per sorted access: the previous access of its location that is not a
//                lock operation, the conflict test, both locksets (a binary search of each
//                thread's list), and the pair;
// then the pair sort of the report, into the pool.
#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

constexpr u32 LS_MAX = 64;                // locks a thread may hold at once
constexpr u32 LS_ROW = 1 + 2 * LS_MAX;    // words of a lockset row: count, words, scope keys
constexpr u32 LS_DEV = 0xffffffffu;       // scope key of a device / system scoped lock

__device__ inline bool ls_lockop(const Bufs &b, u32 p) { return (b.s_flags[p] & (SF_REL | SF_ACQ)) != 0; }

// The location key of a sync entry's word, as the elements carry it.
__device__ inline u32 ls_word(const Bufs &b, const DevParams *P, u32 p) {
    const uint4 e = b.ev[b.s_pidx[p]];
    return ((e.z >> 6) & 1u) ? P->g_span + block_of(b, e.y) * P->s_span + (e.x - P->sbase) : e.x - P->gbase;
}

__device__ inline bool ls_active(const DevParams *P) {
    return (P->mode & MODE_SYNC) && P->first_bad_record == NONE && P->first_bad_sync == NONE && !check_abandoned(P);
}

__global__ void k_ls_flag(Bufs b, u32 *flag) {
    DevParams *P = b.prm;
    const u32 n = P->n_sync;
    if (blockIdx.x == 0 && threadIdx.x == 0) P->ls_pairs = 0;
    for (u32 p = blockIdx.x * blockDim.x + threadIdx.x; p <= n; p += gridDim.x * blockDim.x)
        flag[p] = p < n && ls_active(P) && ls_lockop(b, p) ? 1u : 0u;
}

// rows: LS_ROW words per lock operation (at its scanned flag), `cap` rows; row_of[p]: the row in
// force after entry p (NONE: no lock held).
__global__ void k_ls_thread(Bufs b, const u32 *rowid, u32 *row_of, u32 *rows, u32 cap) {
    DevParams *P = b.prm;
    if (!ls_active(P)) return;
    if (rowid[P->n_sync] > cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&P->err, ERR_LOCKSET);
        return;
    }
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < b.T; t += gridDim.x * blockDim.x) {
        const u32 lo = b.s_cnt[t], hi = b.s_cnt[t + 1], blk = block_of(b, t);
        u32 w[LS_MAX], k[LS_MAX], n = 0, cur = NONE;
        for (u32 p = lo; p < hi; p++) {
            if (ls_lockop(b, p)) {
                const uint8_t f = b.s_flags[p];
                const u32 x = ls_word(b, P, p);
                // a release closes the section on its word (if one is open), then an acquire opens
                // one unless the word is already held
                if (f & SF_REL) {
                    for (u32 q = 0; q < n; q++)
                        if (w[q] == x) {
                            for (u32 r = q + 1; r < n; r++) { w[r - 1] = w[r]; k[r - 1] = k[r]; }
                            n--;
                            break;
                        }
                }
                if (f & SF_ACQ) {
                    bool held = false;
                    for (u32 q = 0; q < n; q++) held |= w[q] == x;
                    if (!held) {
                        if (n == LS_MAX) {
                            atomicOr(&P->err, ERR_LOCKSET);
                            return;
                        }
                        w[n] = x;
                        k[n] = ((b.s_scope[p] >> 2) & 3u) == 0 ? blk : LS_DEV;
                        n++;
                    }
                }
                const u32 r = rowid[p];
                u32 *row = rows + (u64)r * LS_ROW;
                row[0] = n;
                for (u32 q = 0; q < n; q++) { row[1 + q] = w[q]; row[1 + LS_MAX + q] = k[q]; }
                cur = n ? r : NONE;
            }
            row_of[p] = cur;
        }
    }
}

// The lockset row of thread t at its access with trace index idx (the entries before it; NONE: no
// lock held).
__device__ inline u32 ls_row_at(const Bufs &b, const u32 *row_of, u32 t, u32 idx) {
    const u32 j = list_search(b, t, idx);
    return j == NONE ? NONE : row_of[j];
}

__device__ inline bool ls_share(const u32 *rows, u32 ra, u32 rb) {
    const u32 *A = rows + (u64)ra * LS_ROW, *B = rows + (u64)rb * LS_ROW;
    const u32 na = A[0], nb = B[0];
    for (u32 i = 0; i < na; i++)
        for (u32 j = 0; j < nb; j++)
            if (A[1 + i] == B[1 + j] &&
                (A[1 + LS_MAX + i] == LS_DEV || B[1 + LS_MAX + j] == LS_DEV || A[1 + LS_MAX + i] == B[1 + LS_MAX + j]))
                return true;
    return false;
}

// Is the access with trace index idx of thread t a lock operation?  (Lock operations are atomics,
// which are sync entries of their thread.)
__device__ inline bool ls_access_is_lockop(const Bufs &b, u32 t, u32 idx, u32 cat) {
    if (cat < CAT_AD) return false;
    const u32 j = list_search(b, t, idx + 1);  // the entry of the access itself
    return j != NONE && b.s_pidx[j] == idx && ls_lockop(b, j);
}

__global__ __launch_bounds__(256) void k_ls_check(Bufs b, const u32 *row_of, const u32 *rows, u32 *pf, u32 *ps,
                                                  u64 cap) {
    DevParams *P = b.prm;
    if (!ls_active(P) || (P->err & ERR_LOCKSET)) return;
    const SegCtx s = seg_ctx(b);
    for (u64 pos = (u64)blockIdx.x * blockDim.x + threadIdx.x; pos < s.n; pos += (u64)gridDim.x * blockDim.x) {
        if (pos == 0) continue;
        const u32 kb = seg_key(s, pos), ib = s.i[pos], tb = seg_tid(s, pos), cb = info_cat(seg_info(s, pos));
        if (ls_access_is_lockop(b, tb, ib, cb)) continue;
        // the previous access of the location that is not a lock operation
        u64 q = pos;
        bool found = false;
        u32 ia = 0, ta = 0, ca = 0;
        while (q > 0) {
            q--;
            if (seg_key(s, q) != kb) break;
            ia = s.i[q];
            ta = seg_tid(s, q);
            ca = info_cat(seg_info(s, q));
            if (!ls_access_is_lockop(b, ta, ia, ca)) { found = true; break; }
        }
        if (!found || ta == tb) continue;
        if (ca == CAT_R && cb == CAT_R) continue;
        const u32 ba = block_of(b, ta), bb = block_of(b, tb);
        if (ca >= CAT_AD && cb >= CAT_AD && (ca == CAT_AD || cb == CAT_AD || ba == bb)) continue;
        const u32 ra = ls_row_at(b, row_of, ta, ia), rb = ls_row_at(b, row_of, tb, ib);
        if (ra == NONE && rb == NONE) continue;
        if (ra != NONE && rb != NONE && ls_share(rows, ra, rb)) continue;
        const u32 slot = atomicAdd(&P->ls_pairs, 1u);
        if (slot < cap) { pf[slot] = ia; ps[slot] = ib; }
        else atomicOr(&P->err, ERR_LSPAIRS);
    }
}

__global__ void k_ls_kept(DevParams *P, u64 cap) {
    if (threadIdx.x == 0) P->ls_kept = P->ls_pairs < cap ? P->ls_pairs : (u32)cap;
}

// Lays out the pass's tables in the pool: four pair arrays and the report (6 words per pair of
// `cap`), then the rows.  False when the pool cannot hold `cap` pairs and one row.
bool lockset_layout(const Bufs &b, u64 cap, LocksetBufs &L) {
    const u64 need = 6 * cap + LS_ROW;
    if (b.pool_words < need) return false;
    u32 *p = b.pool;
    L.pf[0] = p; L.ps[0] = p + cap; L.pf[1] = p + 2 * cap; L.ps[1] = p + 3 * cap;
    L.report = (u64 *)(p + 4 * cap);  // 8-byte aligned: cap words from a 256-byte aligned start, times 4
    L.rows = p + 6 * cap;
    L.row_cap = (u32)((b.pool_words - 6 * cap) / LS_ROW > 0xffffffffull ? 0xffffffffull : (b.pool_words - 6 * cap) / LS_ROW);
    L.cap = cap;
    return true;
}

void lockset_run(const Bufs &b, const LocksetBufs &L, hipStream_t s) {
    const u32 *n_sync = &b.prm->n_sync;
    const unsigned g = (unsigned)((b.N + 256) / 256 > 4096 ? 4096 : (b.N + 256) / 256);
    RD_LAUNCH("k_ls_flag", k_ls_flag, dim3(g), dim3(256), 0, s, b, b.e_scan0);
    scan_exclusive(b.e_scan0, (u64)b.N + 1, b.part, s, nullptr, n_sync);
    const unsigned gt = (unsigned)((b.T + 255) / 256 > 2048 ? 2048 : (b.T + 255) / 256);
    RD_LAUNCH("k_ls_thread", k_ls_thread, dim3(gt), dim3(256), 0, s, b, (const u32 *)b.e_scan0, b.e_scan1, L.rows,
              L.row_cap);
    const unsigned gc = (unsigned)((b.N + 255) / 256 > 8192 ? 8192 : ((b.N + 255) / 256 ? (b.N + 255) / 256 : 1));
    RD_LAUNCH("k_ls_check", k_ls_check, dim3(gc), dim3(256), 0, s, b, (const u32 *)b.e_scan1, (const u32 *)L.rows,
              L.pf[0], L.ps[0], L.cap);
    RD_LAUNCH("k_ls_kept", k_ls_kept, dim3(1), dim3(64), 0, s, b.prm, L.cap);
    u32 *const f[2] = {L.pf[0], L.pf[1]}, *const s2[2] = {L.ps[0], L.ps[1]};
    sort_pairs_to(b, f, s2, &b.prm->ls_kept, L.cap, s);
    pack_pairs_to(L.pf[0], L.ps[0], &b.prm->ls_kept, L.cap, L.report, s);
}

}  // namespace rd
