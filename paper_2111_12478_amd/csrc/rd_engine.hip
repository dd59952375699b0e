// rd_engine.hip -- parallel computation of the happens-before knowledge carried by releases,
// acquires and block barriers (traces without warp barriers), on gfx950.
//
// The knowledge vectors are the sequential interpreter's (rd_interp.hip): Algorithm 1's H clock
// with block floors KB[blk] and per-releaser columns KT[col], rule (iv) of Section 2.2 with the
// scoped tags of a sync variable -- device scope, block scope of one block, every block.  Instead
// of walking the sync events one by one, every operation's inputs are resolved up front:
//   * a release on location X extends the chain (X, DEV), or the chains (X, its block) and
//     (X, ALL); its input is the previous release of each chain.  Segmented scans over the
//     release/acquire accesses in (location, trace) order -- the location sort's order -- find
//     them; for the per-block chains a wavefront scans back over the location's run;
//   * an acquire reads the latest release of (X, DEV) and of (X, its block) or (X, ALL);
//   * a thread's knowledge before an entry is its last acquire since its last barrier, else its
//     block's knowledge after that barrier (one lane per thread walks its own list);
//   * a completed block barrier joins the block's knowledge with its participants' acquires.
// Every input precedes its operation in trace order, so the operations split greedily, in trace
// order, into groups without a dependency inside a group.  One cooperative kernel evaluates the
// groups in order: a group with many operations is spread over every workgroup, a run of small
// groups (a lock handed from block to block) is evaluated by one workgroup in order; grid barriers
// with bounded waits separate them.  An operation joins a few vectors of D words.
#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

constexpr u32 BK_MARK = 0x80000000u;  // e_cur: the block's knowledge after (value & ~BK_MARK) barriers
constexpr u32 OP_SKIPPED = 0xfffffffeu;  // op_dep during evaluation: the operation wrote no vector
constexpr u32 ENG_WIDE = 16;          // groups with at least this many operations run on every workgroup
constexpr u32 ENG_THREADS = 512;
constexpr u32 CH_BLK = 128;                  // operations whose jobs a window replay stages at once
constexpr u32 CH_BLK_JOBS = 3 * CH_BLK;      // three job slots per operation
constexpr u32 ENG_SPIN = 1u << 19;  // ~1 s of polling: far above any legitimate wait

__device__ inline bool eng_active(const DevParams *P) {
    return (P->mode & MODE_SYNC) && !(P->mode & MODE_WBAR) && P->first_bad_record == NONE &&
           !(P->err & ERR_PHASE) && !check_abandoned(P);
}
__device__ inline bool eng_on(const DevParams *P) { return eng_active(P) && !(P->eng & ENG_FALLBACK); }

// buffer of the location sort's result (digits of the context's variant), and of a key-value
// sort by location key (8-bit digits)

// ---------------------------------------------------------------- release/acquire accesses

// e_scan0[q] = 1 when the trace-ordered sync entry q is a release/acquire access (an atomic, a lock
// acquire or a lock release with a release or acquire role); q <= n_sync (scanned next).
__global__ void k_eng_flag(Bufs b) {
    const DevParams *P = b.prm;
    if (!eng_active(P)) return;
    const u32 n = P->n_sync;
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q <= n; q += gridDim.x * blockDim.x) {
        u32 f = 0;
        if (q < n) {
            const u32 p = b.s_inv[q], kind = b.s_kind[p];
            if ((kind == 2u || kind == 6u || kind == 7u) && (b.s_flags[p] & (SF_REL | SF_ACQ))) f = 1;
        }
        b.e_scan0[q] = f;
    }
}

// ral_p / ral_key: the release/acquire accesses in trace order with their location keys (sorted by
// location next, stably, which gives (location, trace) order); fallback if too many.
__global__ void k_eng_compact(Bufs b) {
    DevParams *P = b.prm;
    if (!eng_active(P)) return;
    const u32 n = P->n_sync, total = b.e_scan0[n];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P->n_ral = total > b.ecap ? 0u : total;
        if (total > b.ecap) atomicOr(&P->eng, ENG_FALLBACK);
    }
    if (total > b.ecap) return;
    const u32 gbase = P->gbase, sbase = P->sbase, g_span = P->g_span, s_span = P->s_span;
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const u32 r = b.e_scan0[q];
        if (b.e_scan0[q + 1] == r) continue;
        const u32 p = b.s_inv[q];
        const uint4 e = b.ev[b.s_pidx[p]];
        const u32 space = (e.z >> 6) & 1u;
        b.ral_key[r] = space ? g_span + block_of(b, e.y) * s_span + (e.x - sbase) : e.x - gbase;
        b.ral_p[r] = p;
    }
}

// The location sort of the list leaves it in the second buffers when its passes are odd in number:
// copy it back.
__global__ void k_eng_ral_back(Bufs b) {
    const DevParams *P = b.prm;
    if (!eng_active(P) || !(((P->key_bits + SORT_RB - 1) / SORT_RB) & 1u)) return;
    for (u32 r = blockIdx.x * blockDim.x + threadIdx.x; r < P->n_ral; r += gridDim.x * blockDim.x) {
        b.ral_key[r] = b.op_dep[r];
        b.ral_p[r] = b.op_p[r];
    }
}

// One workgroup scans a list in chunks of 1024 lanes for "the latest marked item before this one in
// the same run" (segmented by run heads).  The carry holds the latest marked item of the run that
// is still open at the end of the previous chunk.  Every lane of the workgroup calls it.
struct SegLds {
    u32 v[1024];
    uint8_t h[1024];
    u32 carry;
};

__device__ inline u32 seg_scan_chunk(SegLds &L, bool head, u32 val, u32 nin) {
    const u32 i = threadIdx.x;
    L.v[i] = val;
    L.h[i] = head ? 1 : 0;
    __syncthreads();
    for (u32 off = 1; off < 1024; off <<= 1) {
        u32 pv = NONE;
        uint8_t ph = 0;
        if (i >= off) { pv = L.v[i - off]; ph = L.h[i - off]; }
        __syncthreads();
        if (i >= off) {
            // left segment (pv, ph) then this one: the left value survives unless this one has a
            // head or a value of its own
            if (!L.h[i] && L.v[i] == NONE) L.v[i] = pv;
            L.h[i] |= ph;
        }
        __syncthreads();
    }
    u32 ex = NONE;
    if (!head) {
        if (i > 0) {
            ex = L.v[i - 1];
            if (ex == NONE && !L.h[i - 1]) ex = L.carry;  // the run started before this chunk
        } else {
            ex = L.carry;
        }
    }
    __syncthreads();
    if (i == 0) {
        const u32 last = nin - 1;
        const u32 vl = L.v[last];
        L.carry = vl != NONE ? vl : (L.h[last] ? NONE : L.carry);
    }
    __syncthreads();
    return ex;
}

// Chains (X, DEV) and (X, ALL) over ral (runs: equal locations), in chunks of 1024 items, one
// workgroup per chunk.  A chunk's scan starts from the latest release of the run still open at its
// start (its carry): k_eng_chain_sums summarises each chunk (the latest release of its last run,
// whether a run starts in it), k_eng_chain_carry composes the summaries in order.  The summaries
// and carries live in op_dep and op_p (free until the operations are numbered).
constexpr u32 CHAIN_CHUNK = 1024;

__device__ inline void chain_item(const Bufs &b, u32 n, u32 k, u32 &p, uint8_t &f, uint8_t &sc, bool &head) {
    p = NONE;
    f = 0;
    sc = 0;
    head = true;
    if (k < n) {
        p = b.ral_p[k];
        f = b.s_flags[p];
        sc = b.s_scope[p];
        head = k == 0 || b.ral_key[k - 1] != b.ral_key[k];
    }
}

__global__ __launch_bounds__(1024) void k_eng_chain_sums(Bufs b) {
    DevParams *P = b.prm;
    if (!eng_on(P)) return;
    const u32 n = P->n_ral, nch = (n + CHAIN_CHUNK - 1) / CHAIN_CHUNK;
    __shared__ int mh, md, ma;
    for (u32 c = blockIdx.x; c < nch; c += gridDim.x) {
        if (threadIdx.x == 0) { mh = -1; md = -1; ma = -1; }
        __syncthreads();
        const u32 k = c * CHAIN_CHUNK + threadIdx.x;
        u32 p;
        uint8_t f, sc;
        bool head;
        chain_item(b, n, k, p, f, sc, head);
        if (k < n) {
            if (head) atomicMax(&mh, (int)threadIdx.x);
            if ((f & SF_REL) && (sc & 3u) != 0) atomicMax(&md, (int)threadIdx.x);
            if ((f & SF_REL) && (sc & 3u) == 0) atomicMax(&ma, (int)threadIdx.x);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // the latest release at or after the last run head (a head's own release counts)
            b.op_dep[3 * c] = md >= 0 && md >= mh ? b.ral_p[c * CHAIN_CHUNK + md] : NONE;
            b.op_dep[3 * c + 1] = ma >= 0 && ma >= mh ? b.ral_p[c * CHAIN_CHUNK + ma] : NONE;
            b.op_dep[3 * c + 2] = mh >= 0 ? 1u : 0u;
        }
        __syncthreads();
    }
}

// Summary composition (earlier, later): the later one's release, else nothing if a run starts in
// the later one, else the earlier one's.
__device__ inline uint4 chain_compose(uint4 l, uint4 r) {
    return make_uint4(r.x != NONE ? r.x : (r.z ? NONE : l.x), r.y != NONE ? r.y : (r.z ? NONE : l.y), l.z | r.z, 0u);
}

// One workgroup: carry of every chunk = composition of the summaries of the chunks before it
// (op_p[2c], op_p[2c + 1]), 1024 chunks per round of an inclusive scan in LDS.
__global__ __launch_bounds__(1024) void k_eng_chain_carry(Bufs b) {
    DevParams *P = b.prm;
    if (!eng_on(P)) return;
    const u32 n = P->n_ral, nch = (n + CHAIN_CHUNK - 1) / CHAIN_CHUNK, i = threadIdx.x;
    __shared__ uint4 S[1024];
    uint4 run = make_uint4(NONE, NONE, 0u, 0u);  // the summaries of the rounds before
    for (u32 base = 0; base < nch; base += 1024) {
        const u32 c = base + i;
        uint4 v = c < nch ? make_uint4(b.op_dep[3 * c], b.op_dep[3 * c + 1], b.op_dep[3 * c + 2], 0u)
                          : make_uint4(NONE, NONE, 0u, 0u);
        S[i] = v;
        __syncthreads();
        for (u32 off = 1; off < 1024; off <<= 1) {
            const uint4 l = i >= off ? S[i - off] : make_uint4(NONE, NONE, 0u, 0u);
            __syncthreads();
            if (i >= off) S[i] = chain_compose(l, S[i]);
            __syncthreads();
        }
        const uint4 ex = i == 0 ? run : chain_compose(run, S[i - 1]);
        if (c < nch) {
            b.op_p[2 * c] = ex.x;
            b.op_p[2 * c + 1] = ex.y;
        }
        run = chain_compose(run, S[1023]);
        __syncthreads();
    }
}

// The chains themselves: each chunk's segmented scans from its carry.  Packs each item's block and
// block-scope bits into e_scan1 for the per-block chains.
__global__ __launch_bounds__(1024) void k_eng_chains(Bufs b) {
    DevParams *P = b.prm;
    if (!eng_on(P)) return;
    const u32 n = P->n_ral, nch = (n + CHAIN_CHUNK - 1) / CHAIN_CHUNK;
    __shared__ SegLds Ld, La;
    for (u32 c = blockIdx.x; c < nch; c += gridDim.x) {
        if (threadIdx.x == 0) { Ld.carry = b.op_p[2 * c]; La.carry = b.op_p[2 * c + 1]; }
        __syncthreads();
        const u32 c0 = c * CHAIN_CHUNK;
        const u32 k = c0 + threadIdx.x, nin = n - c0 < CHAIN_CHUNK ? n - c0 : CHAIN_CHUNK;
        u32 p;
        uint8_t f, sc;
        bool head;
        chain_item(b, n, k, p, f, sc, head);
        const bool acq = f & SF_ACQ;
        const bool rel_dev = (f & SF_REL) && (sc & 3u) != 0, rel_blk = (f & SF_REL) && (sc & 3u) == 0;
        const u32 ex_dev = seg_scan_chunk(Ld, head, rel_dev ? p : NONE, nin);
        const u32 ex_all = seg_scan_chunk(La, head, rel_blk ? p : NONE, nin);
        if (k < n) {
            if (rel_dev) { b.e_prev0[p] = ex_dev; b.e_prev1[p] = NONE; }
            if (rel_blk) { b.e_prev0[p] = NONE; b.e_prev1[p] = ex_all; }  // e_prev0: block chain, later
            if (acq) {
                // an entry that is both releases first: its own release counts for its chains
                b.e_src0[p] = rel_dev ? p : ex_dev;
                b.e_src1[p] = ((sc >> 2) & 3u) != 0 ? (rel_blk ? p : ex_all) : NONE;  // block scope: later
            }
            // per-block chains, below: bit 31 block-scoped release, bit 30 needs its chain, low bits block
            const u32 blk = block_of(b, b.ev[b.s_pidx[p]].y);
            b.e_scan1[k] = (rel_blk ? 0x80000000u : 0u) |
                           ((rel_blk || (acq && ((sc >> 2) & 3u) == 0)) ? 0x40000000u : 0u) | blk;
        }
        __syncthreads();
    }
}

// Per-block chains (X, block): for every item that needs one, a whole wavefront scans backwards
// over its location's run in the (location, trace)-ordered list, 64 positions per step, for the
// latest block-scoped release of the same block.  Runs of one shared word belong to one block and
// end at once; a global word that many blocks take with block scope may take longer: past WALK_MAX
// steps the engine gives way to the sequential interpreter.
constexpr u32 WALK_MAX = 1u << 14;

__global__ __launch_bounds__(256) void k_eng_blk_walk(Bufs b) {
    DevParams *P = b.prm;
    if (!eng_on(P)) return;
    const u32 n = P->n_ral, lane = lane_id();
    const u32 wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, n_waves = (gridDim.x * blockDim.x) >> 6;
    for (u32 c0 = wave * 64; c0 < n; c0 += n_waves * 64) {
        const u32 k = c0 + lane;
        const u32 pk = k < n ? b.e_scan1[k] : 0u;
        u64 todo = ballot((pk & 0x40000000u) != 0);
        while (todo) {
            const u32 src = (u32)__builtin_ctzll(todo);
            todo &= todo - 1;
            const u32 kk = c0 + src;
            const u32 key = b.ral_key[kk], blk = b.e_scan1[kk] & 0x3fffffffu;
            u32 found = NONE, steps = 0;
            bool over = false;
            for (u32 top = kk; top > 0; top = top > 64 ? top - 64 : 0) {
                // lanes look at top-1-lane
                const bool in = lane < top;
                const u32 j = in ? top - 1 - lane : 0;
                const bool same = in && b.ral_key[j] == key;
                const u32 w = same ? b.e_scan1[j] : 0u;
                const u64 hit = ballot(same && (w & 0x80000000u) && (w & 0x3fffffffu) == blk);
                const u64 stop = ballot(in && !same);
                if (hit) {
                    const u32 first = (u32)__builtin_ctzll(hit);  // nearest position below
                    if (!stop || first < (u32)__builtin_ctzll(stop)) found = top - 1 - first;
                    break;
                }
                if (stop || top <= 64) break;
                if (++steps > WALK_MAX) { over = true; break; }
            }
            if (lane == 0) {
                if (over) {
                    atomicOr(&P->eng, ENG_FALLBACK);
                } else {
                    const u32 p = b.ral_p[kk];
                    const uint8_t f = b.s_flags[p], sc = b.s_scope[p];
                    const bool rel_blk = (f & SF_REL) && (sc & 3u) == 0;
                    const u32 prev = found == NONE ? NONE : b.ral_p[found];
                    if (rel_blk) b.e_prev0[p] = prev;
                    if ((f & SF_ACQ) && ((sc >> 2) & 3u) == 0) b.e_src1[p] = rel_blk ? p : prev;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- engine state

// Decides whether the parallel engine runs (sets ENG_PARALLEL), and its vector width.
__global__ void k_eng_init(Bufs b, const u32 *rt_scan) {
    DevParams *P = b.prm;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (!eng_active(P)) return;
    P->eng |= ENG_PARALLEL;
    // vectors padded to whole 16-byte words (the padding stays zero)
    const u32 n_rt = rt_scan[b.T], D = (b.B + n_rt + 3u) & ~3u;
    P->n_rt = n_rt;
    P->D = D;
    const u64 cap = (u64)b.pool_words / D;
    P->pool_cap = cap > 0xffffffffull ? 0xffffffffu : (u32)cap;
}

// ---------------------------------------------------------------- per-thread walk

// One lane per program thread, over its sync list in program order: the knowledge an entry starts
// from (e_cur), and for each barrier arrival the thread's latest acquire of the phase it ends
// (e_src0 of the arrival); a barrier instance records its latest such acquire (trace index + 1)
// in inst_coff.  An acquire that nothing but that barrier reads (no access, and no sync entry but
// fences, before it) is marked SF_NOMAT.
__global__ void k_eng_walk(Bufs b) {
    const DevParams *P = b.prm;
    if (!eng_on(P)) return;
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < b.T; t += gridDim.x * blockDim.x) {
        const u32 lo = b.s_cnt[t], hi = b.s_cnt[t + 1];
        if (lo == hi) continue;
        const u32 blk = block_of(b, t);
        u32 last = NONE;
        for (u32 p = lo; p < hi; p++) {
            const u32 kind = b.s_kind[p];
            uint8_t f = b.s_flags[p];
            if (kind == 4u) {
                b.e_src0[p] = last;
                if (last != NONE) atomicMax(&b.inst_coff[b.inst_off[blk] + b.s_phase[p] - 1], b.s_pidx[last] + 1);
                last = NONE;
            } else if (f & (SF_REL | SF_ACQ)) {
                b.e_cur[p] = last != NONE ? last : (BK_MARK | b.s_phase[p]);
                if ((f & SF_ACQ) && (b.e_src0[p] != NONE || b.e_src1[p] != NONE)) {
                    last = p;
                    if (!(f & SF_REL) && b.s_imin[p] == NONE) {
                        u32 q = p + 1;
                        while (q < hi && b.s_kind[q] == 3u && b.s_imin[q] == NONE) q++;
                        if (q < hi && b.s_kind[q] == 4u) b.s_flags[p] = f | SF_NOMAT;
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- operations

__device__ inline bool inst_complete(const Bufs &b, u32 blk, u32 slot) {
    return b.inst_cnt[slot] == b.n_active[blk];
}

// Per trace-ordered sync entry q <= n_sync: is it an operation, and how many vectors does it
// write.  e_scan0 / e_scan1 get 0/1 and the count (scanned next).
__global__ void k_eng_mark(Bufs b) {
    const DevParams *P = b.prm;
    if (!eng_on(P)) return;
    const u32 n_sync = P->n_sync;
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q <= n_sync; q += gridDim.x * blockDim.x) {
        u32 nout = 0;
        if (q < n_sync) {
            const u32 p = b.s_inv[q];
            const uint8_t f = b.s_flags[p];
            const u32 kind = b.s_kind[p];
            if (f & SF_REL) nout += (b.s_scope[p] & 3u) == 0 ? 2u : 1u;
            if ((f & SF_ACQ) && (b.e_src0[p] != NONE || b.e_src1[p] != NONE)) nout += 1;
            if (kind == 4u) {
                const u32 idx = b.s_pidx[p], blk = block_of(b, b.ev[idx].y);
                const u32 slot = b.inst_off[blk] + b.s_phase[p] - 1;
                if (b.inst_last[slot] == idx && inst_complete(b, blk, slot) && b.inst_coff[slot] != 0) nout += 1;
            }
        }
        b.e_scan0[q] = nout ? 1u : 0u;
        b.e_scan1[q] = nout;
    }
}

// Operation indices and vector handles (handle 0 is the empty knowledge).
__global__ void k_eng_assign(Bufs b) {
    DevParams *P = b.prm;
    if (!eng_on(P)) return;
    const u32 n_sync = P->n_sync, n_ops = b.e_scan0[n_sync], n_vec = b.e_scan1[n_sync];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P->n_ops = n_ops;
        P->n_handles = n_vec + 1;
        if (n_ops > b.ecap) atomicOr(&P->eng, ENG_FALLBACK);
        else if ((u64)n_vec + 1 > P->pool_cap) atomicOr(&P->err, ERR_POOL);
    }
    if (n_ops > b.ecap || (u64)n_vec + 1 > P->pool_cap) return;
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < n_sync; q += gridDim.x * blockDim.x) {
        const u32 o = b.e_scan0[q];
        if (b.e_scan0[q + 1] == o) continue;
        const u32 p = b.s_inv[q], h = 1 + b.e_scan1[q];
        const uint8_t f = b.s_flags[p];
        u32 used = 0;
        b.op_p[o] = p;
        b.e_op[p] = o;
        if (f & SF_REL) {
            b.e_relh[p] = h;
            used = (b.s_scope[p] & 3u) == 0 ? 2u : 1u;
        }
        if ((f & SF_ACQ) && (b.e_src0[p] != NONE || b.e_src1[p] != NONE)) {
            b.s_khandle[p] = h + used;
            used++;
        }
        if (b.s_kind[p] == 4u) {
            const u32 blk = block_of(b, b.ev[b.s_pidx[p]].y), slot = b.inst_off[blk] + b.s_phase[p] - 1;
            b.inst_opo[slot] = o;
            b.inst_handle[slot] = h + used;
        }
    }
}

// One lane per block: the block's knowledge after each of its barrier instances (handle and the
// operation that wrote it), inheriting through instances that add nothing.
__global__ void k_eng_bk(Bufs b) {
    const DevParams *P = b.prm;
    if (!eng_on(P) || P->n_ops > b.ecap) return;  // also when the pool ran out: k_eng_assign numbered nothing
    for (u32 blk = blockIdx.x * blockDim.x + threadIdx.x; blk < b.B; blk += gridDim.x * blockDim.x) {
        u32 h = 0, o = NONE;
        for (u32 slot = b.inst_off[blk]; slot < b.inst_off[blk + 1]; slot++) {
            if (b.inst_opo[slot] != NONE) { h = b.inst_handle[slot]; o = b.inst_opo[slot]; }
            b.inst_handle[slot] = h;
            b.inst_bko[slot] = o;
        }
    }
}

// The operation of the sync entry with trace index x (it exists).
__device__ inline u32 op_at_index(const Bufs &b, u32 n_ops, u32 x) {
    u32 lo = 0, hi = n_ops;
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (b.s_pidx[b.op_p[mid]] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ inline u32 dmax(u32 a, u32 c) { return a == NONE ? c : (c == NONE ? a : (a > c ? a : c)); }

// The latest operation each operation reads from (NONE: none).
__global__ void k_eng_deps(Bufs b) {
    const DevParams *P = b.prm;
    if (!eng_on(P) || P->n_ops > b.ecap) return;  // also when the pool ran out: k_eng_assign numbered nothing
    const u32 n_ops = P->n_ops;
    for (u32 o = blockIdx.x * blockDim.x + threadIdx.x; o < n_ops; o += gridDim.x * blockDim.x) {
        const u32 p = b.op_p[o], idx = b.s_pidx[p], blk = block_of(b, b.ev[idx].y);
        u32 d = NONE;
        if (b.s_kind[p] == 4u) {
            const u32 k = b.s_phase[p], slot = b.inst_off[blk] + k - 1;
            if (k > 1) d = dmax(d, b.inst_bko[slot - 1]);
            d = dmax(d, op_at_index(b, n_ops, b.inst_coff[slot] - 1));
        } else {
            const u32 cur = b.e_cur[p];
            if (cur & BK_MARK) {
                const u32 ph = cur & ~BK_MARK;
                if (ph > 0) d = dmax(d, b.inst_bko[b.inst_off[blk] + ph - 1]);
            } else {
                d = dmax(d, b.e_op[cur]);
            }
            const uint8_t f = b.s_flags[p];
            if (f & SF_REL) {
                if (b.e_prev0[p] != NONE) d = dmax(d, b.e_op[b.e_prev0[p]]);
                if (b.e_prev1[p] != NONE) d = dmax(d, b.e_op[b.e_prev1[p]]);
            }
            if (f & SF_ACQ) {
                if (b.e_src0[p] != NONE && b.e_src0[p] != p) d = dmax(d, b.e_op[b.e_src0[p]]);
                if (b.e_src1[p] != NONE && b.e_src1[p] != p) d = dmax(d, b.e_op[b.e_src1[p]]);
            }
        }
        b.op_dep[o] = d;
    }
}

// Greedy groups in trace order: a new group starts at the first operation that reads from the
// current group.  One wavefront takes the decisions over the dependencies staged in LDS, 4,096 at a
// time, while the workgroup's other wavefronts load the next 4,096.  grp[0..n_groups] are the group
// starts and the end.
constexpr u32 GRP_BLK = 4096;
__global__ __launch_bounds__(1024) void k_eng_groups(Bufs b) {
    DevParams *P = b.prm;
    if (!eng_on(P) || P->n_ops > b.ecap) return;  // also when the pool ran out: k_eng_assign numbered nothing
    __shared__ u32 deps[2][GRP_BLK];
    const u32 n = P->n_ops, lane = lane_id(), wave = threadIdx.x >> 6;
    for (u32 i = threadIdx.x; i < GRP_BLK; i += blockDim.x) deps[0][i] = i < n ? b.op_dep[i] : NONE;
    __syncthreads();
    u32 start = 0, ng = 0;  // wave 0's
    if (threadIdx.x == 0) b.grp[0] = 0;
    u32 cur = 0;
    for (u32 blk = 0; blk < n; blk += GRP_BLK, cur ^= 1u) {
        if (wave != 0) {
            const u32 nxt = blk + GRP_BLK;
            for (u32 i = threadIdx.x - 64; i < GRP_BLK; i += blockDim.x - 64) {
                const u32 o = nxt + i;
                deps[cur ^ 1u][i] = o < n ? b.op_dep[o] : NONE;
            }
        } else {
            const u32 lim = n - blk < GRP_BLK ? n - blk : GRP_BLK;
            for (u32 c0 = 0; c0 < lim; c0 += 64) {
                const u32 o = blk + c0 + lane;
                const u32 d = deps[cur][c0 + lane];
                u32 from = 0;  // lanes below `from` are settled
                for (;;) {
                    const bool cut = lane >= from && o < n && d != NONE && d >= start;
                    const u64 m = ballot(cut);
                    if (!m) break;
                    const u32 first = (u32)__builtin_ctzll(m);
                    start = blk + c0 + first;
                    ng++;
                    if (lane == 0) b.grp[ng] = start;
                    from = first + 1;
                }
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        b.grp[ng + 1] = n;
        P->n_groups = n ? ng + 1 : 0;
    }
}

// ---------------------------------------------------------------- evaluation

__device__ inline const u32 *vecp(const Bufs &b, u32 D, u32 h) { return b.pool + (u64)h * D; }

// Vectors are D words, D a multiple of 4: every lane joins 16-byte words, 4 at a time, with all
// of a step's loads issued before its stores.
__device__ inline uint4 max4(uint4 a, uint4 c) {
    return make_uint4(max(a.x, c.x), max(a.y, c.y), max(a.z, c.z), max(a.w, c.w));
}
__device__ inline void bump4(uint4 &v, u32 w4, u32 col, u32 val) {
    if ((col >> 2) != w4) return;
    switch (col & 3u) {
    case 0: v.x = max(v.x, val); break;
    case 1: v.y = max(v.y, val); break;
    case 2: v.z = max(v.z, val); break;
    default: v.w = max(v.w, val); break;
    }
}
constexpr u32 EV = 4;  // 16-byte words per lane per step

// Inside a window of operations (a run of small dependent groups), inputs with handles at or
// above `hint` are written by earlier operations of the same window.  The first phase joins the
// other inputs into the outputs (partial results) and describes the rest in the operation's job:
// three output slots (out, in0, in1, in2) and, for a barrier, a range of the window input list.
// The second phase joins those.  Wide groups pass hint = NONE and no job.
struct JobSink {
    u32 *job;     // ENG_JOB_WORDS words, or null
    u32 *list;    // ENG_WIN words
    u32 *list_n;  // entries used
};

__device__ inline u32 ext(u32 h, u32 hint) { return h >= hint ? 0u : h; }
__device__ inline u32 inn(u32 h, u32 hint) { return h >= hint ? h : 0u; }

// Block barrier operation: the block's previous knowledge joined with every participant's latest
// acquire of the phase the barrier ends.
__device__ void eval_bar(const Bufs &b, u32 p, u32 D, u32 *lds_list, u32 *lds_n, u32 hint, JobSink js) {
    const u32 idx = b.s_pidx[p], blk = block_of(b, b.ev[idx].y), k = b.s_phase[p];
    const u32 slot = b.inst_off[blk] + k - 1;
    if (threadIdx.x == 0) *lds_n = 0;
    __syncthreads();
    for (u32 u = threadIdx.x; u < b.tpb; u += ENG_THREADS) {
        const u32 t = blk * b.tpb + u;
        u32 lo = b.s_cnt[t], hi = b.s_cnt[t + 1];
        // first entry whose phase reaches k: the thread's k-th barrier arrival (if it has one)
        while (lo < hi) {
            const u32 mid = (lo + hi) >> 1;
            if (b.s_phase[mid] < k) lo = mid + 1;
            else hi = mid;
        }
        if (lo < b.s_cnt[t + 1] && b.s_kind[lo] == 4u && b.s_phase[lo] == k) {
            const u32 c = b.e_src0[lo];
            if (c != NONE) {
                if (b.op_dep[b.e_op[c]] == OP_SKIPPED) {
                    // the acquire wrote no vector: its inputs instead (its block knowledge before
                    // it is this barrier's previous one, joined below)
                    const u32 s0 = b.e_src0[c], s1 = b.e_src1[c], cur = b.e_cur[c];
                    const bool blk_acq = ((b.s_scope[c] >> 2) & 3u) == 0;
                    if (!(cur & BK_MARK)) lds_list[atomicAdd(lds_n, 1u)] = b.s_khandle[cur];
                    if (s0 != NONE) lds_list[atomicAdd(lds_n, 1u)] = b.e_relh[s0];
                    if (s1 != NONE) lds_list[atomicAdd(lds_n, 1u)] = b.e_relh[s1] + (blk_acq ? 0u : 1u);
                } else {
                    lds_list[atomicAdd(lds_n, 1u)] = b.s_khandle[c];
                }
            }
        }
    }
    __syncthreads();
    const u32 nc = *lds_n, D4 = D / 4;
    const u32 hout = b.inst_handle[slot], hprev = k > 1 ? b.inst_handle[slot - 1] : 0u;
    uint4 *out = (uint4 *)(b.pool + (u64)hout * D);
    const uint4 *prev = (const uint4 *)vecp(b, D, ext(hprev, hint));
    const bool lprev = ext(hprev, hint) != 0;  // the empty vector is not read
    for (u32 base = 0; base < D4; base += ENG_THREADS * EV) {
        uint4 v[EV];
#pragma unroll
        for (u32 e = 0; e < EV; e++) {
            const u32 i = base + e * ENG_THREADS + threadIdx.x;
            v[e] = lprev && i < D4 ? prev[i] : make_uint4(0, 0, 0, 0);
        }
        // the inputs four at a time, all their loads issued before the joins
        for (u32 c0 = 0; c0 < nc; c0 += 4) {
            uint4 w[4][EV];
#pragma unroll
            for (u32 j = 0; j < 4; j++) {
                const u32 h = c0 + j < nc ? lds_list[c0 + j] : 0u;
                const bool use = h != 0 && h < hint;  // (the empty vector, handle 0, is not read)
                const uint4 *src = (const uint4 *)vecp(b, D, use ? h : 0u);
#pragma unroll
                for (u32 e = 0; e < EV; e++) {
                    const u32 i = base + e * ENG_THREADS + threadIdx.x;
                    w[j][e] = use && i < D4 ? src[i] : make_uint4(0, 0, 0, 0);
                }
            }
#pragma unroll
            for (u32 j = 0; j < 4; j++)
#pragma unroll
                for (u32 e = 0; e < EV; e++) v[e] = max4(v[e], w[j][e]);
        }
#pragma unroll
        for (u32 e = 0; e < EV; e++) {
            const u32 i = base + e * ENG_THREADS + threadIdx.x;
            if (i < D4) out[i] = v[e];
        }
    }
    if (js.job && threadIdx.x == 0) {
        u32 n_in = 0;
        for (u32 c = 0; c < nc; c++) n_in += lds_list[c] >= hint;
        // each acquire of the window feeds at most one barrier: the list never holds more than
        // the window's operations
        const u32 off = n_in ? atomicAdd(js.list_n, n_in) : 0u;
        if (off + n_in > ENG_WIN) atomicOr(&b.prm->err, ERR_ENGINE);
        else
            for (u32 c = 0, m = 0; c < nc; c++)
                if (lds_list[c] >= hint) js.list[off + m++] = lds_list[c];
        uint4 *J = (uint4 *)js.job;
        J[0] = make_uint4(hout, inn(hprev, hint), 0, 0);
        J[1] = make_uint4(0, 0, 0, 0);
        J[2] = make_uint4(0, 0, 0, 0);
        J[3] = make_uint4(off, off + n_in > ENG_WIN ? 0u : n_in, 0, 0);
    }
}

// Release and / or acquire of one sync entry (release first).  In a wide group (no window) an
// acquire marked SF_NOMAT writes no vector: its operation is marked OP_SKIPPED and the barrier
// that reads it joins its inputs.
__device__ void eval_ra(const Bufs &b, const u32 *rt_scan, u32 o, u32 p, u32 D, u32 hint, JobSink js) {
    const u32 idx = b.s_pidx[p], t = b.ev[idx].y, blk = block_of(b, t);
    const uint8_t f = b.s_flags[p], sc = b.s_scope[p];
    const u32 cur = b.e_cur[p], D4 = D / 4;
    u32 hc;
    if (cur & BK_MARK) {
        const u32 ph = cur & ~BK_MARK;
        hc = ph > 0 ? b.inst_handle[b.inst_off[blk] + ph - 1] : 0u;
    } else {
        hc = b.s_khandle[cur];
    }
    const uint4 *vc = (const uint4 *)vecp(b, D, ext(hc, hint));
    const bool lc = ext(hc, hint) != 0;  // (the empty vector, handle 0, is never read)
    uint4 j0 = make_uint4(0, 0, 0, 0), j1 = j0, j2 = j0;
    if (f & SF_REL) {
        const u32 kb = blk, kbv = b.s_phase[p], kt = b.B + rt_scan[t], ktv = idx + 1;
        const u32 h0 = b.e_relh[p];
        const bool two = (sc & 3u) == 0;
        const u32 hv0 = b.e_prev0[p] != NONE ? b.e_relh[b.e_prev0[p]] : 0u;
        const u32 hv1 = two && b.e_prev1[p] != NONE ? b.e_relh[b.e_prev1[p]] + 1 : 0u;
        const uint4 *v0 = (const uint4 *)vecp(b, D, ext(hv0, hint));
        const uint4 *v1 = (const uint4 *)vecp(b, D, ext(hv1, hint));
        const bool l0 = ext(hv0, hint) != 0, l1 = two && ext(hv1, hint) != 0;
        uint4 *o0 = (uint4 *)(b.pool + (u64)h0 * D), *o1 = (uint4 *)(b.pool + (u64)(h0 + 1) * D);
        for (u32 base = 0; base < D4; base += ENG_THREADS * EV) {
            uint4 c[EV], x0[EV], x1[EV];
#pragma unroll
            for (u32 e = 0; e < EV; e++) {
                const u32 i = base + e * ENG_THREADS + threadIdx.x;
                const bool in = i < D4;
                c[e] = in && lc ? vc[i] : make_uint4(0, 0, 0, 0);
                x0[e] = in && l0 ? v0[i] : make_uint4(0, 0, 0, 0);
                x1[e] = in && l1 ? v1[i] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (u32 e = 0; e < EV; e++) {
                const u32 i = base + e * ENG_THREADS + threadIdx.x;
                if (i >= D4) continue;
                bump4(c[e], i, kb, kbv);
                bump4(c[e], i, kt, ktv);
                o0[i] = max4(c[e], x0[e]);
                if (two) o1[i] = max4(c[e], x1[e]);
            }
        }
        j0 = make_uint4(h0, inn(hc, hint), inn(hv0, hint), 0);
        if (two) j1 = make_uint4(h0 + 1, inn(hc, hint), inn(hv1, hint), 0);
        __syncthreads();  // an atomic's acquire may read its own release
    }
    const u32 ha = (f & SF_ACQ) ? b.s_khandle[p] : 0u;
    if (ha && (f & SF_NOMAT) && !(f & SF_REL) && hint == NONE) {
        if (threadIdx.x == 0) b.op_dep[o] = OP_SKIPPED;
    } else if (ha) {
        const u32 s0 = b.e_src0[p], s1 = b.e_src1[p];
        const bool blk_acq = ((sc >> 2) & 3u) == 0;
        const u32 ha0 = s0 != NONE ? b.e_relh[s0] : 0u;
        const u32 ha1 = s1 != NONE ? b.e_relh[s1] + (blk_acq ? 0u : 1u) : 0u;
        const uint4 *a0 = (const uint4 *)vecp(b, D, ext(ha0, hint));
        const uint4 *a1 = (const uint4 *)vecp(b, D, ext(ha1, hint));
        const bool la0 = ext(ha0, hint) != 0, la1 = ext(ha1, hint) != 0;
        uint4 *oa = (uint4 *)(b.pool + (u64)ha * D);
        for (u32 base = 0; base < D4; base += ENG_THREADS * EV) {
            uint4 c[EV], x0[EV], x1[EV];
#pragma unroll
            for (u32 e = 0; e < EV; e++) {
                const u32 i = base + e * ENG_THREADS + threadIdx.x;
                const bool in = i < D4;
                c[e] = in && lc ? vc[i] : make_uint4(0, 0, 0, 0);
                x0[e] = in && la0 ? a0[i] : make_uint4(0, 0, 0, 0);
                x1[e] = in && la1 ? a1[i] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (u32 e = 0; e < EV; e++) {
                const u32 i = base + e * ENG_THREADS + threadIdx.x;
                if (i < D4) oa[i] = max4(c[e], max4(x0[e], x1[e]));
            }
        }
        j2 = make_uint4(ha, inn(hc, hint), inn(ha0, hint), inn(ha1, hint));
    }
    if (js.job && threadIdx.x == 0) {
        uint4 *J = (uint4 *)js.job;
        J[0] = j0;
        J[1] = j1;
        J[2] = j2;
        J[3] = make_uint4(0, 0, 0, 0);
    }
}

__device__ inline void eval_op(const Bufs &b, const u32 *rt_scan, u32 o, u32 D, u32 *lds_list, u32 *lds_n, u32 hint,
                               JobSink js) {
    const u32 p = b.op_p[o];
    if (b.s_kind[p] == 4u) eval_bar(b, p, D, lds_list, lds_n, hint, js);
    else eval_ra(b, rt_scan, o, p, D, hint, js);
    __syncthreads();
}

// The smallest handle an operation writes (handles grow with the operation index).
__device__ inline u32 first_handle(const Bufs &b, u32 o) {
    const u32 p = b.op_p[o];
    if (b.s_kind[p] == 4u) {
        const u32 blk = block_of(b, b.ev[b.s_pidx[p]].y);
        return b.inst_handle[b.inst_off[blk] + b.s_phase[p] - 1];
    }
    return (b.s_flags[p] & SF_REL) ? b.e_relh[p] : b.s_khandle[p];
}

// Second phase of a window.  Every output column of every operation depends only on the same
// column of its inputs, so a workgroup owns a slice of 64 columns and its first wavefront replays
// the window's jobs in order over them, one column per lane: no barrier between operations.  For
// each block of CH_BLK operations the workgroup stages their jobs in LDS (one coalesced read),
// compacts the ones with inputs from the window, in order, and builds a table of values for the
// slice in LDS with every lane: each job's partial result (replaced by its output as the replay
// goes), the outputs of earlier blocks that the block's jobs read, and a row of zeros.  Each input
// of a job is then one of the replay's last three outputs (held in registers), or a row of the
// table: the replay itself reads no global memory.  Jobs with list inputs (barriers), or whose rows
// do not fit, take a general step that reads other outputs from the pool.

__device__ inline u32 uni(u32 x) { return __builtin_amdgcn_readfirstlane(x); }

// A load that waits for itself inside the same statement: the replay's join point then carries no
// vector-memory wait, which on this target would also wait for the previous operations' stores.
__device__ __attribute__((always_inline)) inline u32 load_now(const u32 *p) {
    u32 x;
    asm volatile("global_load_dword %0, %1, off\n\ts_waitcnt vmcnt(0)" : "=v"(x) : "v"(p) : "memory");
    return x;
}

constexpr u32 CH_HASH = 1024;                 // open-addressed map of a block's output handles
constexpr u32 CH_JOB_PER_THREAD = CH_BLK * ENG_JOB_WORDS / ENG_THREADS;
static_assert(CH_JOB_PER_THREAD * ENG_THREADS == CH_BLK * ENG_JOB_WORDS, "a block's job words split evenly");
constexpr u32 CH_ZROW = CH_BLK_JOBS;          // the table's row of zeros
constexpr u32 CH_ROWS_NONE = CH_ZROW | CH_ZROW << 10 | CH_ZROW << 20;
constexpr u32 CH_TABLE_WORDS = (CH_BLK_JOBS + 1) * 64;
static_assert(CH_ZROW < 1024, "rows are 10-bit fields");

// One job with inputs from the window: output handle, up to three input handles, and for a
// barrier a range of the window input list.
struct ChainLds {
    uint4 q[CH_BLK_JOBS + 2];          // (two more entries: the replay reads a job ahead)
    uint2 l[CH_BLK_JOBS];
    u32 wave_n[ENG_THREADS / 64];
    u32 n, nf;
    u32 ch[3];                         // handles of the replay's three latest outputs before the block
    u32 code[CH_BLK_JOBS + 2];         // per job: which of the three latest outputs it joins (bits
                                       // 0-2), or NONE when it takes the general step
    u32 rows[CH_BLK_JOBS + 2];         // per job: three rows of the table it joins (10 bits each)
    u32 farh[CH_BLK_JOBS];             // handle of each prefetched row
    u32 hkey[CH_HASH], hval[CH_HASH];  // output handle -> job index within the block
};

__device__ inline u32 ch_slot(u32 h) { return (h * 0x9E3779B1u) >> 22; }

// The general step's view of one input: a register when it is one of the three latest outputs,
// else the pool (every output is stored there as soon as it is computed).
__device__ __attribute__((always_inline)) inline u32 gen_join(u32 h, u32 h1, u32 h2, u32 h3, u32 a, u32 b2,
                                                              u32 c, const u32 *pool, u32 D, u32 col, u32 v) {
    if (h == h1) return max(v, a);
    if (h == h2) return max(v, b2);
    if (h == h3) return max(v, c);
    return max(v, load_now(pool + (u64)h * D + col));
}

__device__ void chain_window(const Bufs &b, u32 w0, u32 w1, u32 D, u32 *lj /* CH_BLK * ENG_JOB_WORDS */,
                             ChainLds &A, u32 *val /* CH_TABLE_WORDS */) {
    const u32 *jobs = b.eng_jobs, *list = b.eng_jobs + ENG_WIN * ENG_JOB_WORDS;
    u32 *pool = b.pool;
    const bool reporter = blockIdx.x == 0 && threadIdx.x == 0;
    const u32 lane = lane_id(), wave = threadIdx.x >> 6, nsl = (D + 63) / 64;
    if (threadIdx.x < 64) val[CH_ZROW * 64 + threadIdx.x] = 0;
    for (u32 sl = blockIdx.x; sl < nsl; sl += gridDim.x) {
        const u32 col = sl * 64 + lane;
        const bool mine = col < D;
        const u32 cc = mine ? col : 0u;
        // the ring of the latest outputs: r2 the newest, r1 and r0 before it (r3 is written next)
        u32 r0 = 0, r1 = 0, r2 = 0, r3 = 0;
        if (threadIdx.x < 3) A.ch[threadIdx.x] = 0;
        // each thread's words of the next block's jobs, loaded one block ahead (the window's jobs
        // are all written before the grid barrier that starts this phase)
        u32 nxt[CH_JOB_PER_THREAD];
#pragma unroll
        for (u32 i = 0; i < CH_JOB_PER_THREAD; i++) {
            const u32 x = threadIdx.x + i * ENG_THREADS;
            nxt[i] = x < (min(w0 + CH_BLK, w1) - w0) * ENG_JOB_WORDS ? jobs[x] : 0u;
        }
        for (u32 cb = w0; cb < w1; cb += CH_BLK) {
            const u32 ce = min(cb + CH_BLK, w1);
            __syncthreads();
#pragma unroll
            for (u32 i = 0; i < CH_JOB_PER_THREAD; i++) {
                const u32 x = threadIdx.x + i * ENG_THREADS;
                if (x < (ce - cb) * ENG_JOB_WORDS) lj[x] = nxt[i];
            }
            if (ce < w1) {
                const u32 ne = min(ce + CH_BLK, w1);
#pragma unroll
                for (u32 i = 0; i < CH_JOB_PER_THREAD; i++) {
                    const u32 x = threadIdx.x + i * ENG_THREADS;
                    nxt[i] = x < (ne - ce) * ENG_JOB_WORDS ? jobs[(u64)(ce - w0) * ENG_JOB_WORDS + x] : 0u;
                }
            }
            for (u32 x = threadIdx.x; x < CH_HASH; x += ENG_THREADS) A.hkey[x] = 0;
            if (threadIdx.x == 0) A.nf = 0;
            __syncthreads();
            // jobs with inputs from the window, in (operation, slot) order
            const u32 x = threadIdx.x;  // job x = operation cb + x / 3, slot x % 3
            bool act = false;
            uint4 q = make_uint4(0, 0, 0, 0);
            uint2 l = make_uint2(0, 0);
            if (x < (ce - cb) * 3) {
                const u32 *jo = lj + (x / 3) * ENG_JOB_WORDS;
                q = ((const uint4 *)jo)[x % 3];
                if (x % 3 == 0) l = make_uint2(jo[12], jo[13]);
                act = q.x && (q.y | q.z | q.w | l.y);
            }
            const u64 m = ballot(act);
            if (lane == 0) A.wave_n[wave] = (u32)__builtin_popcountll(m);
            __syncthreads();
            u32 off = 0;
            for (u32 w = 0; w < wave; w++) off += A.wave_n[w];
            if (act) {
                const u32 r = off + (u32)__builtin_popcountll(m & lanemask_lt());
                A.q[r] = q;
                A.l[r] = l;
                // output handles are written once each (handle 0, the empty vector, is never one)
                for (u32 s = ch_slot(q.x);; s = (s + 1) & (CH_HASH - 1))
                    if (atomicCAS(&A.hkey[s], 0u, q.x) == 0u) {
                        A.hval[s] = r;
                        break;
                    }
            }
            if (threadIdx.x == ENG_THREADS - 1) A.n = off + (u32)__builtin_popcountll(m);
            __syncthreads();
            const u32 n = A.n;
            // each job's inputs: registers (code), rows of this block (an earlier job's output) and
            // outputs of earlier blocks (prefetched rows, counted here and placed below)
            u32 code = NONE, rows = CH_ROWS_NONE, nfar = 0, far = 0;
            bool lean = false;
            if (threadIdx.x < n) {
                const u32 k = threadIdx.x;
                const uint4 jq = A.q[k];
                const u32 o1 = k >= 1 ? A.q[k - 1].x : A.ch[0];
                const u32 o2 = k >= 2 ? A.q[k - 2].x : A.ch[1 - k];
                const u32 o3 = k >= 3 ? A.q[k - 3].x : A.ch[2 - k];
                const u32 in[3] = {jq.y, jq.z, jq.w};
                lean = A.l[k].y == 0;
                code = 0;
#pragma unroll
                for (u32 j = 0; j < 3; j++) {
                    const u32 h = in[j];
                    if (!h) continue;
                    if (h == o1) { code |= 1u; continue; }
                    if (h == o2) { code |= 2u; continue; }
                    if (h == o3) { code |= 4u; continue; }
                    u32 r = NONE;
                    for (u32 s = ch_slot(h);; s = (s + 1) & (CH_HASH - 1)) {
                        const u32 key = A.hkey[s];
                        if (key == h) { r = A.hval[s]; break; }
                        if (key == 0u) break;
                    }
                    if (r == NONE) {
                        far |= 1u << j;
                        nfar++;
                    } else if (r < k) {
                        rows = (rows & ~(0x3FFu << (10 * j))) | (r << (10 * j));
                    } else {
                        lean = false;
                    }
                }
                if (!lean) nfar = 0;
            }
            // prefetched rows: an exclusive prefix of nfar over the block's jobs
            u32 incl = nfar;
#pragma unroll
            for (u32 d = 1; d < 64; d <<= 1) {
                const u32 y = __shfl_up(incl, d, 64);
                if (lane >= d) incl += y;
            }
            if (lane == 63) A.wave_n[wave] = incl;
            __syncthreads();
            u32 foff = incl - nfar;
            for (u32 w = 0; w < wave; w++) foff += A.wave_n[w];
            if (threadIdx.x < n) {
                const u32 k = threadIdx.x;
                if (nfar && n + foff + nfar <= CH_BLK_JOBS) {
                    const uint4 jq = A.q[k];
                    const u32 in[3] = {jq.y, jq.z, jq.w};
                    u32 f = foff;
#pragma unroll
                    for (u32 j = 0; j < 3; j++)
                        if (far & (1u << j)) {
                            A.farh[f] = in[j];
                            rows = (rows & ~(0x3FFu << (10 * j))) | ((n + f) << (10 * j));
                            f++;
                        }
                    // the rows in use end with the last job that fits (offsets grow with the job)
                    atomicMax(&A.nf, f);
                } else if (nfar) {
                    lean = false;
                }
                A.code[k] = lean ? code : NONE;
                A.rows[k] = lean ? rows : CH_ROWS_NONE;
            } else if (threadIdx.x < n + 2) {
                A.code[threadIdx.x] = NONE;
                A.rows[threadIdx.x] = CH_ROWS_NONE;
            }
            __syncthreads();
            // the table: the jobs' partial results, then the outputs of earlier blocks (stored by
            // this workgroup's first wavefront before the barriers above)
            // (each wavefront loads every eighth row, eight rows in flight)
            const u32 nr = n + A.nf;
            constexpr u32 NW = ENG_THREADS / 64, RF = 8;
            for (u32 r0 = wave; r0 < nr; r0 += NW * RF) {
                u32 x[RF];
#pragma unroll
                for (u32 j = 0; j < RF; j++) {
                    const u32 r = r0 + j * NW;
                    x[j] = 0;
                    if (r < nr && mine) x[j] = pool[(u64)(r < n ? A.q[r].x : A.farh[r - n]) * D + col];
                }
#pragma unroll
                for (u32 j = 0; j < RF; j++)
                    if (r0 + j * NW < nr) val[(r0 + j * NW) * 64 + lane] = x[j];
            }
            __syncthreads();
            if (wave == 0 && n) {
                // The replay.  A job's rows were written at least four jobs before it (nearer
                // outputs are registers), so its words and rows are read a job ahead.
                // (the next job's four values are joined only when it runs, so the reads have the
                // current job's time to arrive)
                u32 code_n = A.code[0], h_n = A.q[0].x, rows_nn = A.rows[1];
                u32 x0, x1, x2, x3;
                {
                    const u32 rr = uni(A.rows[0]);
                    x0 = val[lane];
                    x1 = val[(rr & 0x3FFu) * 64 + lane];
                    x2 = val[((rr >> 10) & 0x3FFu) * 64 + lane];
                    x3 = val[(rr >> 20) * 64 + lane];
                }
                auto step = [&](u32 k, u32 a, u32 b2, u32 c, u32 &dst) {
                    const u32 cd = uni(code_n), h = uni(h_n), rr = uni(rows_nn);
                    u32 v = max(max(x0, x1), max(x2, x3));
                    // the next job's words and values (after the last job: the padding, unused)
                    code_n = A.code[k + 1];
                    h_n = A.q[k + 1].x;
                    rows_nn = A.rows[k + 2];
                    x0 = val[(k + 1) * 64 + lane];
                    x1 = val[(rr & 0x3FFu) * 64 + lane];
                    x2 = val[((rr >> 10) & 0x3FFu) * 64 + lane];
                    x3 = val[(rr >> 20) * 64 + lane];
                    if (cd != NONE) {
                        // (the selected registers, by masks: no branch)
                        const u32 m0 = 0u - (cd & 1u), m1 = 0u - ((cd >> 1) & 1u), m2 = 0u - ((cd >> 2) & 1u);
                        v = max(max(v, a & m0), max(b2 & m1, c & m2));
                    } else {
                        const uint4 jq = make_uint4(0, uni(A.q[k].y), uni(A.q[k].z), uni(A.q[k].w));
                        const u32 h1 = uni(k >= 1 ? A.q[k - 1].x : A.ch[0]);
                        const u32 h2 = uni(k >= 2 ? A.q[k - 2].x : A.ch[k < 2 ? 1 - k : 0]);
                        const u32 h3 = uni(k >= 3 ? A.q[k - 3].x : A.ch[k < 3 ? 2 - k : 0]);
                        if (jq.y) v = gen_join(jq.y, h1, h2, h3, a, b2, c, pool, D, cc, v);
                        if (jq.z) v = gen_join(jq.z, h1, h2, h3, a, b2, c, pool, D, cc, v);
                        if (jq.w) v = gen_join(jq.w, h1, h2, h3, a, b2, c, pool, D, cc, v);
                        const u32 lo = uni(A.l[k].x), ln = uni(A.l[k].y);
                        for (u32 i = 0; i < ln; i++)
                            v = gen_join(uni(list[lo + i]), h1, h2, h3, a, b2, c, pool, D, cc, v);
                    }
                    if (mine) pool[(u64)h * D + cc] = v;
                    val[k * 64 + lane] = v;
                    dst = v;
                };
                u32 k = 0;
                for (; k + 4 <= n; k += 4) {
                    step(k, r2, r1, r0, r3);
                    step(k + 1, r3, r2, r1, r0);
                    step(k + 2, r0, r3, r2, r1);
                    step(k + 3, r1, r0, r3, r2);
                }
                const u32 rem = n - k;
                if (rem == 1) {
                    step(k, r2, r1, r0, r3);
                    r0 = r1; r1 = r2; r2 = r3;
                } else if (rem == 2) {
                    step(k, r2, r1, r0, r3);
                    step(k + 1, r3, r2, r1, r0);
                    const u32 t0 = r0;
                    r0 = r2; r1 = r3; r2 = t0;
                } else if (rem == 3) {
                    step(k, r2, r1, r0, r3);
                    step(k + 1, r3, r2, r1, r0);
                    step(k + 2, r0, r3, r2, r1);
                    const u32 t0 = r0, t1 = r1;
                    r0 = r3; r1 = t0; r2 = t1;
                }
                // the three latest handles for the next block
                if (lane == 0) {
                    const u32 c0 = A.ch[0], c1 = A.ch[1];
                    A.ch[0] = A.q[n - 1].x;
                    A.ch[1] = n >= 2 ? A.q[n - 2].x : c0;
                    A.ch[2] = n >= 3 ? A.q[n - 3].x : (n == 2 ? c0 : c1);
                }
            }
            if (reporter) atomicAdd(&b.prm->gprog, 1u);
        }
    }
}

// All workgroups meet; writes before are visible to every workgroup after.  The wait is bounded by
// time without progress: workgroup 0 advances P->gprog during the sequential phase of a window,
// which restarts the others' count.
__device__ inline void grid_barrier(DevParams *P, u32 round) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(&P->gbar, 1u);
        const u32 target = round * gridDim.x;
        u32 spins = 0, seen = __hip_atomic_load(&P->gprog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (__hip_atomic_load(&P->gbar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            const u32 now = __hip_atomic_load(&P->gprog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (now != seen) { seen = now; spins = 0; }
            if (++spins > ENG_SPIN) { atomicOr(&P->err, ERR_ENGINE); break; }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
    }
    __syncthreads();
}

// The end of the run of small groups that starts at group g: the first later group with at least
// ENG_WIDE operations, or ng.  The workgroup looks at ENG_THREADS groups at a time (a lock handed
// through thousands of critical sections is one run of thousands of groups).
__device__ inline u32 small_run_end(const Bufs &b, u32 g, u32 ng, u32 *lds) {
    for (u32 base = g + 1; base < ng; base += ENG_THREADS) {
        const u32 x = base + threadIdx.x;
        const bool wide = x < ng && b.grp[x + 1] - b.grp[x] >= ENG_WIDE;
        if (threadIdx.x == 0) *lds = NONE;
        __syncthreads();
        if (wide) atomicMin(lds, x);
        __syncthreads();
        const u32 f = *lds;
        __syncthreads();
        if (f != NONE) return f;
    }
    return ng;
}

// Cooperative: every workgroup runs the same group loop.  A wide group spreads its operations over
// the workgroups; a run of small groups is evaluated in windows of two phases (above).
__global__ __launch_bounds__(ENG_THREADS) void k_eng_eval(Bufs b, const u32 *rt_scan) {
    DevParams *P = b.prm;
    if (!eng_on(P) || P->n_ops > b.ecap) return;
    __shared__ u32 lds_list[3 * 1024];  // a barrier's inputs: up to three per participant
    __shared__ u32 lds_n;
    __shared__ u32 lds_jobs[CH_BLK * ENG_JOB_WORDS];
    __shared__ ChainLds lds_chain;
    __shared__ u32 lds_part[CH_TABLE_WORDS];
    __shared__ u32 lds_ops[ENG_THREADS];
    __shared__ u32 lds_nops;
    const u32 D = P->D, ng = P->n_groups;
    u32 round = 0;
    if (blockIdx.x == 0) {
        for (u32 i = threadIdx.x; i < D; i += ENG_THREADS) b.pool[i] = 0;  // the empty knowledge
        if (threadIdx.x == 0) P->wlist = 0;
    }
    // vectors written by the engine: their padding words must read as zero too (joins keep them 0)
    grid_barrier(P, ++round);
    JobSink none = {nullptr, nullptr, nullptr};
    u32 g = 0;
    while (g < ng) {
        const u32 g0 = b.grp[g], g1 = b.grp[g + 1];
        if (g1 - g0 >= ENG_WIDE) {
            // the workgroup's operations g0 + blockIdx.x + k * gridDim.x, ENG_THREADS at a time: an
            // acquire that only its thread's next barrier reads writes no vector and is marked by
            // one lane (no loads beyond its entry); the others are evaluated one by one
            for (u64 first = (u64)g0 + blockIdx.x; first < g1; first += (u64)ENG_THREADS * gridDim.x) {
                const u64 o = first + (u64)threadIdx.x * gridDim.x;
                bool keep = false;
                if (o < g1) {
                    const u32 p = b.op_p[o];
                    const uint8_t f = b.s_flags[p];
                    if (b.s_kind[p] != 4u && (f & SF_ACQ) && (f & SF_NOMAT) && !(f & SF_REL))
                        b.op_dep[o] = OP_SKIPPED;
                    else
                        keep = true;
                }
                if (threadIdx.x == 0) lds_nops = 0;
                __syncthreads();
                if (keep) lds_ops[atomicAdd(&lds_nops, 1u)] = (u32)o;
                __syncthreads();
                const u32 nk = lds_nops;
                for (u32 k = 0; k < nk; k++) eval_op(b, rt_scan, lds_ops[k], D, lds_list, &lds_n, NONE, none);
                __syncthreads();
            }
            g++;
            grid_barrier(P, ++round);
            continue;
        }
        const u32 g2 = small_run_end(b, g, ng, &lds_n);
        const u32 end = b.grp[g2];
        for (u32 w0 = g0; w0 < end; w0 += ENG_WIN) {
            const u32 w1 = min(w0 + ENG_WIN, end);
            if (w1 - w0 == 1) {  // one operation: all its inputs are ready
                if (blockIdx.x == 0) eval_op(b, rt_scan, w0, D, lds_list, &lds_n, NONE, none);
                grid_barrier(P, ++round);
                continue;
            }
            const u32 hint = first_handle(b, w0);
            for (u32 o = w0 + blockIdx.x; o < w1; o += gridDim.x) {
                JobSink js = {b.eng_jobs + (u64)(o - w0) * ENG_JOB_WORDS, b.eng_jobs + ENG_WIN * ENG_JOB_WORDS,
                              &P->wlist};
                eval_op(b, rt_scan, o, D, lds_list, &lds_n, hint, js);
            }
            grid_barrier(P, ++round);
            chain_window(b, w0, w1, D, lds_jobs, lds_chain, lds_part);
            if (blockIdx.x == 0 && threadIdx.x == 0) P->wlist = 0;  // the next window's list starts empty
            grid_barrier(P, ++round);
        }
        g = g2;
    }
}

static unsigned grid_over(u64 n, unsigned cap = 4096) {
    u64 g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

static int eng_grid(int device) {
    static int cus[64] = {0};
    if (device < 0 || device >= 64) return 64;
    if (!cus[device]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || v <= 0) v = 64;
        cus[device] = v;
    }
    return cus[device];
}

hipError_t engine_run(const Bufs &b, const u32 *rt_scan, hipStream_t s) {
    const u32 *gate = &b.prm->eng;
    RD_LAUNCH("k_eng_init", k_eng_init, dim3(1), dim3(64), 0, s, b, rt_scan);
    FillJobs f = {};
    f.P = b.prm;
    f.add(b.s_khandle, b.N, 0, 4, MODE_SYNC, &b.prm->n_sync, 1);
    f.add(b.inst_coff, b.N, 0, 4, MODE_SYNC, b.inst_off + b.B, 1);
    f.add(b.inst_opo, b.N, NONE, 4, MODE_SYNC, b.inst_off + b.B, 1);
    fill_many(f, "k_fill_engine", s);
    // chains of releases, over the release/acquire accesses in (location, trace) order: taken from
    // the sync entries in trace order, then sorted by location (op_dep and op_p, free until the
    // operations are numbered, are the sort's second buffers)
    const u32 *n_sync = &b.prm->n_sync;
    RD_LAUNCH("k_eng_flag", k_eng_flag, dim3(grid_over(b.N + 1)), dim3(256), 0, s, b);
    scan_exclusive(b.e_scan0, (u64)b.N + 1, b.part, s, gate, n_sync);
    RD_LAUNCH("k_eng_compact", k_eng_compact, dim3(grid_over(b.N)), dim3(256), 0, s, b);
    {
        u32 *const k2[2] = {b.ral_key, b.op_dep}, *const v2[2] = {b.ral_p, b.op_p};
        sort_kv(b, k2, v2, &b.prm->n_ral, b.ecap, 4, &b.prm->key_bits, "k_eng_ral_sort", s);
    }
    RD_LAUNCH("k_eng_ral_back", k_eng_ral_back, dim3(grid_over(b.ecap)), dim3(256), 0, s, b);
    {
        const u64 nch = (b.ecap + CHAIN_CHUNK - 1) / CHAIN_CHUNK;
        const unsigned g = (unsigned)(nch < 1 ? 1 : (nch > 2048 ? 2048 : nch));
        RD_LAUNCH("k_eng_chain_sums", k_eng_chain_sums, dim3(g), dim3(1024), 0, s, b);
        RD_LAUNCH("k_eng_chain_carry", k_eng_chain_carry, dim3(1), dim3(1024), 0, s, b);
        RD_LAUNCH("k_eng_chains", k_eng_chains, dim3(g), dim3(1024), 0, s, b);
    }
    RD_LAUNCH("k_eng_blk_walk", k_eng_blk_walk, dim3(grid_over(b.ecap, 1024)), dim3(256), 0, s, b);
    // operations and their inputs
    RD_LAUNCH("k_eng_walk", k_eng_walk, dim3(grid_over(b.T)), dim3(256), 0, s, b);
    RD_LAUNCH("k_eng_mark", k_eng_mark, dim3(grid_over(b.N + 1)), dim3(256), 0, s, b);
    scan_exclusive(b.e_scan0, (u64)b.N + 1, b.part, s, gate, n_sync);
    scan_exclusive(b.e_scan1, (u64)b.N + 1, b.part, s, gate, n_sync);
    RD_LAUNCH("k_eng_assign", k_eng_assign, dim3(grid_over(b.N)), dim3(256), 0, s, b);
    RD_LAUNCH("k_eng_bk", k_eng_bk, dim3(grid_over(b.B)), dim3(256), 0, s, b);
    RD_LAUNCH("k_eng_deps", k_eng_deps, dim3(grid_over(b.ecap)), dim3(256), 0, s, b);
    RD_LAUNCH("k_eng_groups", k_eng_groups, dim3(1), dim3(1024), 0, s, b);
    // evaluation: one cooperative launch
    int dev = 0;
    (void)hipGetDevice(&dev);
    Bufs bb = b;
    const u32 *rs = rt_scan;
    void *args[] = {&bb, &rs};
    prof_begin("k_eng_eval", s);
    const hipError_t e =
        hipLaunchCooperativeKernel((const void *)k_eng_eval, dim3(eng_grid(dev)), dim3(ENG_THREADS), args, 0, s);
    prof_end(s);
    return e;
}

}  // namespace rd
