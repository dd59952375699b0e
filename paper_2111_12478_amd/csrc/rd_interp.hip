// rd_interp.hip -- happens-before knowledge carried by releases, acquires and warp barriers.
//
// Knowledge of a thread is a vector of D = n_blocks + n_rt words:
//   KB[blk]  = k : every event of block blk that passed fewer than k block barriers happens before;
//   KT[col]  = i+1 : every event of the thread owning column col with trace index <= i happens before.
// Columns exist for threads that release or take part in warp barriers.  This is Algorithm 1's
// H clock with the block's barrier phase standing for the clocks of all its threads (the forced
// compression of Section 5.2: after a barrier every participant's entry is the same).
//
// The interpreter walks the sync events in trace order, as the paper's analysis does, in one
// workgroup: lane 0 does the table bookkeeping and all 1024 lanes do the vector joins.
//   RELEASE(t, l, s):  H_<l,s> := H_<l,s> join H_t join {KB[blk] = phase, KT[t] = idx + 1}
//   ACQUIRE(t, l, s):  H_t := H_t join H_<l,DEVICE> join (s = BLOCK ? H_<l,blk> : every H_<l,b>)
//   block barrier:     at the last arrival, the block's vector := join of its participants
//   warp barrier:      at the last lane's arrival, every lane := join of the lanes + their KT
// Block-barrier phases themselves need no vector: "same block and fewer barriers" is checked
// directly from the phases of the two events.
#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

constexpr u32 TAG_DEV = 0xffffffffu;  // device/system-scope releases of a location
constexpr u32 TAG_ALL = 0xfffffffeu;  // block-scope releases of a location, all blocks joined
constexpr int IT = 1024;              // interpreter workgroup

__device__ inline u64 mix64(u64 x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdull; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ull; x ^= x >> 33;
    return x;
}

__device__ inline u64 loc_key64(uint4 e, u32 tpb) {
    const u32 space = (e.z >> 6) & 1u;
    return space ? ((u64)1 << 63) | ((u64)(e.y / tpb) << 32) | e.x : (u64)e.x;
}

// sync-variable table: (location, tag) -> knowledge vector (0 = empty slot)
__device__ inline u32 sv_find(const Bufs &b, u64 key, u32 tag, bool create, u32 *slot_out) {
    const u32 m = b.sv_cap - 1;
    u32 s = (u32)(mix64(key ^ ((u64)tag * 0x9e3779b97f4a7c15ull)) & m);
    for (u32 probe = 0; probe < b.sv_cap; probe++, s = (s + 1) & m) {
        if (b.sv_handle[s] == 0) {
            if (!create) return 0;
            *slot_out = s;
            return NONE;  // free slot for insertion
        }
        if (b.sv_key[s] == key && b.sv_tag[s] == tag) { *slot_out = s; return b.sv_handle[s]; }
    }
    *slot_out = NONE;
    return 0;
}

// warp-barrier occurrence table: (tid, id) -> occurrences so far; returns the old count
__device__ inline u32 wo_next(const Bufs &b, u32 t, u32 id, bool *ok) {
    const u64 key = ((u64)t << 32) | id;
    const u32 m = b.wo_cap - 1;
    u32 s = (u32)(mix64(key) & m);
    for (u32 probe = 0; probe < b.wo_cap; probe++, s = (s + 1) & m) {
        if (b.wo_key[s] == ~0ull) { b.wo_key[s] = key; b.wo_val[s] = 1; *ok = true; return 0; }
        if (b.wo_key[s] == key) { *ok = true; return b.wo_val[s]++; }
    }
    *ok = false;
    return 0;
}

// warp-barrier instance table: (lane-0 tid, id, occurrence) -> instance
__device__ inline u32 wi_get(const Bufs &b, u32 warp0, u32 id, u32 occ, u32 mask, bool *ok) {
    const u64 key = ((u64)warp0 << 32) | id;
    const u32 m = b.wo_cap - 1;
    u32 s = (u32)(mix64(key ^ ((u64)occ * 0xd1b54a32d192ed03ull)) & m);
    for (u32 probe = 0; probe < b.wo_cap; probe++, s = (s + 1) & m) {
        if (b.wi_inst[s] == NONE) {
            const u32 inst = b.prm->n_winst++;
            b.wi_key[s] = key; b.wi_occ[s] = occ; b.wi_inst[s] = inst;
            b.winst_mask[inst] = mask; b.winst_arrived[inst] = 0; b.winst_last[inst] = 0; b.winst_nar[inst] = 0;
            *ok = true;
            return inst;
        }
        if (b.wi_key[s] == key && b.wi_occ[s] == occ) { *ok = true; return b.wi_inst[s]; }
    }
    *ok = false;
    return NONE;
}

struct Shared {
    u32 list[IT];
    u32 cnt[IT / 64];
    u32 n;
    u32 abort;
    // work order for the current entry
    u32 op;          // 1 release, 2 acquire, 3 barrier completion, 4 warp completion
    u32 dst, src[3], nsrc;
    u32 kb_col, kb_val, kt_col, kt_val;
    u32 zero_dst;
};

__device__ inline u32 *vec(const Bufs &b, u32 D, u32 h) { return b.pool + (u64)h * D; }

__device__ inline void vjoin(u32 *dst, const u32 *src, u32 D) {
    for (u32 i = threadIdx.x; i < D; i += IT) { const u32 v = src[i]; if (v > dst[i]) dst[i] = v; }
}
__device__ inline void vzero(u32 *dst, u32 D) {
    for (u32 i = threadIdx.x; i < D; i += IT) dst[i] = 0;
}

__device__ inline u32 alloc_vec(const Bufs &b, Shared &sh) {
    DevParams *P = b.prm;
    const u32 h = P->pool_next;
    if (h >= P->pool_cap) { atomicOr(&P->err, ERR_POOL); sh.abort = 1; return 0; }
    P->pool_next = h + 1;
    return h;
}

__global__ __launch_bounds__(IT) void k_interp(Bufs b, const u32 *rt_scan) {
    __shared__ Shared sh;
    DevParams *P = b.prm;
    if (!(P->mode & MODE_SYNC) || P->first_bad_record != NONE || (P->err & ERR_PHASE)) return;
    if ((P->eng & ENG_PARALLEL) && !(P->eng & ENG_FALLBACK)) return;  // the parallel engine did it
    const u32 n_rt = rt_scan[b.T], D = b.B + n_rt, n_sync = P->n_sync;
    if (threadIdx.x == 0) {
        P->n_rt = n_rt;
        P->D = D;
        P->pool_next = 1;
        u64 cap = (u64)b.pool_words / D;
        P->pool_cap = cap > 0xffffffffull ? 0xffffffffu : (u32)cap;
        if (P->pool_cap < 1) atomicOr(&P->err, ERR_POOL);
        sh.abort = P->pool_cap < 1;
        P->n_winst = 0;
    }
    __syncthreads();
    if (sh.abort) return;
    vzero(b.pool, D);  // vector 0: the empty knowledge
    __syncthreads();

    for (u32 c0 = 0; c0 < n_sync; c0 += IT) {
        // ---- relevant entries of this chunk, in trace order
        const u32 q = c0 + threadIdx.x;
        bool rel = false;
        if (q < n_sync) {
            const u32 p = b.s_inv[q];
            const u32 kind = b.s_kind[p];
            if (b.s_flags[p] & (SF_REL | SF_ACQ)) rel = true;
            else if (kind == 5) rel = true;
            else if (kind == 4) {
                const u32 idx = b.s_pidx[p], t = b.ev[idx].y, blk = t / b.tpb;
                const u32 slot = b.inst_off[blk] + b.s_phase[p] - 1;
                rel = b.inst_last[slot] == idx && b.inst_cnt[slot] == b.n_active[blk];
            }
        }
        const u64 m = ballot(rel);
        const u32 w = threadIdx.x >> 6;
        if (lane_id() == 0) sh.cnt[w] = popc64(m);
        __syncthreads();
        u32 off = 0, tot = 0;
        for (u32 x = 0; x < IT / 64; x++) { if (x < w) off += sh.cnt[x]; tot += sh.cnt[x]; }
        if (rel) sh.list[off + popc64(m & lanemask_lt())] = q;
        if (threadIdx.x == 0) sh.n = tot;
        __syncthreads();
        const u32 nl = sh.n;

        for (u32 r = 0; r < nl; r++) {
            const u32 p = b.s_inv[sh.list[r]];
            const u32 idx = b.s_pidx[p];
            const uint4 e = b.ev[idx];
            const u32 t = e.y, blk = t / b.tpb, kind = e.z & 15u;
            const uint8_t fl = b.s_flags[p], sc = b.s_scope[p];

            // ---------------- release
            if (fl & SF_REL) {
                const u32 rs = sc & 3u;
                const u64 X = loc_key64(e, b.tpb);
                const u32 tags[2] = {rs == 0 ? blk : TAG_DEV, TAG_ALL};
                const u32 ntag = rs == 0 ? 2 : 1;
                for (u32 g = 0; g < ntag; g++) {
                    if (threadIdx.x == 0) {
                        u32 slot;
                        u32 h = sv_find(b, X, tags[g], true, &slot);
                        sh.zero_dst = 0;
                        if (slot == NONE) { atomicOr(&P->err, ERR_TABLE); sh.abort = 1; }
                        else if (h == NONE) {
                            h = alloc_vec(b, sh);
                            if (!sh.abort) { b.sv_key[slot] = X; b.sv_tag[slot] = tags[g]; b.sv_handle[slot] = h; sh.zero_dst = 1; }
                        }
                        sh.dst = h;
                        sh.src[0] = b.priv[t] ? b.priv[t] : b.bk[blk];
                        sh.kb_col = blk; sh.kb_val = b.s_phase[p];
                        sh.kt_col = b.B + rt_scan[t]; sh.kt_val = idx + 1;
                    }
                    __syncthreads();
                    if (sh.abort) return;
                    u32 *d = vec(b, D, sh.dst);
                    if (sh.zero_dst) vzero(d, D);
                    __syncthreads();
                    vjoin(d, vec(b, D, sh.src[0]), D);
                    __syncthreads();
                    if (threadIdx.x == 0) {
                        if (d[sh.kb_col] < sh.kb_val) d[sh.kb_col] = sh.kb_val;
                        if (d[sh.kt_col] < sh.kt_val) d[sh.kt_col] = sh.kt_val;
                    }
                    __syncthreads();
                }
            }

            // ---------------- acquire
            if (fl & SF_ACQ) {
                const u32 as = (sc >> 2) & 3u;
                const u64 X = loc_key64(e, b.tpb);
                if (threadIdx.x == 0) {
                    u32 slot, ns = 0;
                    const u32 hd = sv_find(b, X, TAG_DEV, false, &slot);
                    const u32 hb = sv_find(b, X, as == 0 ? blk : TAG_ALL, false, &slot);
                    if (hd && hd != NONE) sh.src[ns++] = hd;
                    if (hb && hb != NONE) sh.src[ns++] = hb;
                    sh.nsrc = ns;
                    sh.dst = 0;
                    if (ns) {
                        const u32 h = alloc_vec(b, sh);
                        sh.dst = h;
                        sh.src[ns] = b.priv[t] ? b.priv[t] : b.bk[blk];
                        if (!sh.abort) {
                            if (b.priv[t] == 0) { b.priv_next[t] = b.priv_head[blk]; b.priv_head[blk] = t; }
                            b.priv[t] = h;
                            b.s_khandle[p] = h;
                        }
                    }
                }
                __syncthreads();
                if (sh.abort) return;
                if (sh.dst) {
                    u32 *d = vec(b, D, sh.dst);
                    const u32 *s0 = vec(b, D, sh.src[sh.nsrc]);
                    for (u32 i = threadIdx.x; i < D; i += IT) d[i] = s0[i];
                    __syncthreads();
                    for (u32 g = 0; g < sh.nsrc; g++) { vjoin(d, vec(b, D, sh.src[g]), D); __syncthreads(); }
                }
            }

            // ---------------- last arrival at a block barrier
            if (kind == 4) {
                const u32 slot = b.inst_off[blk] + b.s_phase[p] - 1;
                if (threadIdx.x == 0) {
                    sh.dst = 0;
                    if (b.priv_head[blk] == NONE) b.inst_handle[slot] = b.bk[blk];
                    else {
                        const u32 h = alloc_vec(b, sh);
                        sh.dst = h;
                        sh.src[0] = b.bk[blk];
                    }
                }
                __syncthreads();
                if (sh.abort) return;
                if (sh.dst) {
                    u32 *d = vec(b, D, sh.dst);
                    const u32 *s0 = vec(b, D, sh.src[0]);
                    for (u32 i = threadIdx.x; i < D; i += IT) d[i] = s0[i];
                    __syncthreads();
                    // join every participant that holds private knowledge, then clear it
                    for (;;) {
                        if (threadIdx.x == 0) {
                            const u32 u = b.priv_head[blk];
                            sh.src[1] = NONE;
                            if (u != NONE) { sh.src[1] = b.priv[u]; b.priv_head[blk] = b.priv_next[u]; b.priv[u] = 0; }
                        }
                        __syncthreads();
                        const u32 hs = sh.src[1];
                        if (hs == NONE) break;
                        vjoin(d, vec(b, D, hs), D);
                        __syncthreads();
                    }
                    if (threadIdx.x == 0) { b.bk[blk] = sh.dst; b.inst_handle[slot] = sh.dst; }
                    __syncthreads();
                }
            }

            // ---------------- warp barrier arrival
            if (kind == 5) {
                if (threadIdx.x == 0) {
                    sh.dst = 0;
                    const u32 id = e.x, mask = e.w, local = t % b.tpb, lane = local % b.ws, warp0 = t - lane;
                    bool ok1, ok2 = false;
                    const u32 occ = wo_next(b, t, id, &ok1);
                    const u32 inst = ok1 ? wi_get(b, warp0, id, occ, mask, &ok2) : NONE;
                    if (!ok1 || !ok2) { atomicOr(&P->err, ERR_TABLE); sh.abort = 1; }
                    else {
                        b.s_winst[p] = inst;
                        if (!((mask >> lane) & 1u) || mask != b.winst_mask[inst]) b.s_flags[p] |= SF_BAD_ARRIVAL;
                        b.winst_arrived[inst] |= 1u << lane;
                        b.winst_last[inst] = idx;
                        const u32 nar = b.winst_nar[inst];
                        if (nar < 32) { b.winst_arr[(u64)inst * 32 + nar] = p; b.winst_nar[inst] = nar + 1; }
                        if (b.winst_arrived[inst] == b.winst_mask[inst]) {
                            const u32 h = alloc_vec(b, sh);
                            sh.dst = h;
                            sh.src[0] = inst;
                        }
                    }
                }
                __syncthreads();
                if (sh.abort) return;
                if (sh.dst) {
                    const u32 inst = sh.src[0], nar = b.winst_nar[inst];
                    u32 *d = vec(b, D, sh.dst);
                    vzero(d, D);
                    __syncthreads();
                    for (u32 a = 0; a < nar; a++) {
                        const u32 pa = b.winst_arr[(u64)inst * 32 + a];
                        const u32 ta = b.ev[b.s_pidx[pa]].y, ba = ta / b.tpb;
                        const u32 ha = b.priv[ta] ? b.priv[ta] : b.bk[ba];
                        vjoin(d, vec(b, D, ha), D);
                        __syncthreads();
                    }
                    if (threadIdx.x == 0) {
                        for (u32 a = 0; a < nar; a++) {
                            const u32 pa = b.winst_arr[(u64)inst * 32 + a];
                            const u32 ia = b.s_pidx[pa], ta = b.ev[ia].y, ba = ta / b.tpb;
                            const u32 col = b.B + rt_scan[ta];
                            if (d[col] < ia + 1) d[col] = ia + 1;
                            if (b.priv[ta] == 0) { b.priv_next[ta] = b.priv_head[ba]; b.priv_head[ba] = ta; }
                            b.priv[ta] = sh.dst;
                            b.s_khandle[pa] = sh.dst;
                        }
                    }
                    __syncthreads();
                }
            }
        }
        __syncthreads();
    }
}

// One lane per program thread: knowledge after each of its sync entries.
__global__ void k_know(Bufs b) {
    const DevParams *P = b.prm;
    if (!(P->mode & MODE_SYNC) || check_abandoned(P)) return;
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < b.T; t += gridDim.x * blockDim.x) {
        const u32 lo = b.s_cnt[t], hi = b.s_cnt[t + 1], blk = t / b.tpb;
        u32 cur = 0, first = NONE, acq = 0;
        for (u32 p = lo; p < hi; p++) {
            if (b.s_kind[p] == 4) cur = b.inst_handle[b.inst_off[blk] + b.s_phase[p] - 1];
            else if (b.s_khandle[p]) { cur = b.s_khandle[p]; acq = 1; }
            b.s_know[p] = cur;
            if (cur && first == NONE) first = b.s_pidx[p];
        }
        // knowledge only grows along a thread's program order: accesses after `first` have some
        b.t_kfirst[t] = first;
        b.t_acq[t] = acq;
    }
}

static inline unsigned grid_n(u64 n) {
    u64 g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

void interp_run(const Bufs &b, const u32 *rt_scan, hipStream_t s) {
    const DevParams *P = b.prm;
    // tables, only in traces with releases/acquires/warp barriers
    FillJobs f = {};
    f.P = P;
    f.add(b.priv, b.T, 0, 4, MODE_SYNC, nullptr, 2);
    f.add(b.bk, b.B, 0, 4, MODE_SYNC, nullptr, 2);
    f.add(b.priv_head, b.B, NONE, 4, MODE_SYNC, nullptr, 2);
    f.add(b.sv_handle, b.sv_cap, 0, 4, MODE_SYNC, nullptr, 2);
    f.add(b.wo_key, b.wo_cap, ~0ull, 8, MODE_WBAR, nullptr, 2);
    f.add(b.wi_inst, b.wo_cap, NONE, 4, MODE_WBAR, nullptr, 2);
    f.add(b.s_khandle, b.N, 0, 4, MODE_SYNC, &P->n_sync, 2);
    f.add(b.s_winst, b.N, NONE, 4, MODE_WBAR, &P->n_sync, 2);
    f.add(b.inst_handle, b.N, 0, 4, MODE_SYNC, b.inst_off + b.B, 2);
    fill_many(f, "k_fill_tables", s);
    RD_LAUNCH("k_interp", k_interp, dim3(1), dim3(IT), 0, s, b, rt_scan);
    RD_LAUNCH("k_know", k_know, dim3(grid_n(b.T)), dim3(256), 0, s, b);
}

}  // namespace rd
