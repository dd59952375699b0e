// rd_gwcp.hip -- the predictive relation GWCP (Section 4) over a checked trace, on gfx950.
//
// A pair (a, b) of conflicting accesses of different threads, a before b in the trace, is a GWCP race
// when a's local time is above b's thread's clock at b, C_t[u] = P_t[u] for u != t, where P is the
// clock Algorithms 1 and 2 keep.  P changes only at lock operations (releases and acquires, explicit
// or inferred from fences), at barrier completions and at reads or writes inside critical sections;
// every other access sees the P its thread had after the last such event.  The pass:
//   k_gw_thread   one lane per program thread walks its sync list: the thread's local time after
//                 each entry (releases and barrier arrivals increment it) and the critical sections
//                 open after it (reading G1: an acquire of a word the thread does not hold opens one,
//                 its next release of that word closes it);
//   k_gw_mark     one lane per event flags the events at which P can change (a lock operation, the
//                 last arrival of a barrier instance, a read or write inside a critical section) and
//                 counts what the tables need; a scan numbers them in trace order, k_gw_list lists
//                 them;
//   k_gw_clear    the clocks' initial values (N_t = 1, H_t = the unit vector of t, P_t = 0);
//   k_gw_interp   one workgroup walks that list in trace order over dense per-thread clocks P_t, H_t
//                 (one word per thread, as the algorithms keep them): ACQUIRE joins the lock clocks
//                 of overlapping scope; RELEASE joins, by rule (ii), the release time of other
//                 threads' released critical sections of the word whose acquire time is below C_t,
//                 until nothing joins, then publishes L^r / L^w for the section's reads and writes and
//                 the lock clocks (joined) and increments; SYNC gives every participant the join of
//                 their clocks; a read or write joins L^w (a write also L^r) of every held lock.  Lane
//                 0 takes the decisions and keeps the tables, all lanes join the clocks.  After each
//                 event whose thread's P changed, a copy of P is kept (barrier participants share
//                 one);
//   k_gw_post     one lane per thread carries those copies along its sync list;
//   k_gw_check    one lane per sorted access b: every earlier access of its location that conflicts
//                 with b, of another thread, with a local time above the copy's word for its thread,
//                 makes a pair;
// then the pair sort of the report.  Dense clocks limit the pass to GW_MAX_T threads.  Its clocks
// and tables live in the knowledge-vector pool, which the check no longer reads once it has ended;
// its per-entry arrays in the knowledge engine's per-entry scratch.
#include "rd_internal.h"
#include "rd_kernels.h"

namespace rd {

constexpr u32 GW_HELD = 64;          // critical sections a thread may hold at once
constexpr u32 GW_THREADS = 1024;     // the interpreter's workgroup
constexpr u32 GW_BATCH = 32;         // words per lane read at once by a full comparison
constexpr u32 GW_WPT = 4;            // clock words per lane of the workgroup (GW_MAX_T / GW_THREADS)
static_assert(GW_WPT * GW_THREADS >= GW_MAX_T, "every clock word has a lane");
constexpr u32 GW_DEV = 0xffffffffu;  // scope key of a device / system scoped lock
constexpr u32 GW_CSW = 8;            // words of a critical-section row (see k_gw_interp)
constexpr u32 GW_NW = 5;             // words of a lock-clock row (see GwHeap::nodes)

// counters at the head of the pass's pool area
enum : u32 { GH_LOCKOPS = 0, GH_CSREC = 1, GH_NWORDS = 2, GH_WORDS = 16 };

__device__ inline bool gw_lockop(const Bufs &b, u32 p) { return (b.s_flags[p] & (SF_REL | SF_ACQ)) != 0; }
__device__ inline bool gw_overlap(u32 a, u32 c) { return a == GW_DEV || c == GW_DEV || a == c; }

// The location key of event e, as the elements carry it.
__device__ inline u32 gw_loc(const Bufs &b, const DevParams *P, uint4 e) {
    return ((e.z >> 6) & 1u) ? P->g_span + block_of(b, e.y) * P->s_span + (e.x - P->sbase) : e.x - P->gbase;
}

__device__ inline bool gw_active(const DevParams *P) {
    return P->first_bad_record == NONE && P->first_bad_sync == NONE && !check_abandoned(P) && !(P->err & ERR_GWCP);
}

// The sync entry of event i of thread t (lock operations and barrier arrivals are entries), or NONE.
__device__ inline u32 gw_entry(const Bufs &b, u32 t, u32 i) {
    const u32 q = list_search(b, t, i + 1);
    return q != NONE && b.s_pidx[q] == i ? q : NONE;
}

// ---------------------------------------------------------------- the pass's heap

// Carved from the pool after the counters, the same way by every kernel: the dense clocks, the
// per-thread state, the tables (sized by the counts k_gw_thread and k_gw_mark leave), then clock
// vectors of T words to the end.
struct GwHeap {
    u32 *P, *H;        // [T][T]
    u32 *J;            // [T][T] row t: the join of the sections' release times that rule (ii) has
                       // found below P_t (joined, or already covered).  A release time is H_u when
                       // u published it, and H clocks are happens-before clocks: J[t][u] >= a
                       // release time's own word of u means row t, hence P_t, is above that whole
                       // release time, so the section adds nothing and is passed over
    u32 *N;            // [T] local times
    u32 *held_n;       // [T] critical sections held
    u32 *held;         // [T][GW_HELD] their rows
    u32 *lastsnap;     // [T] the copy of P_t in force (NONE: P_t = 0)
    u32 *JH;           // [T] scratch of a barrier join
    u32 *wsnap;        // [wo_cap] the copy a warp-barrier instance leaves
    u64 *wkey; u32 *wval; u32 cw;   // lock word -> word row
    u64 *lkey; u32 *lval; u32 cl;   // (lock clock, location, read / write) -> vector
    u32 *words;        // [n_lock][4] word, its queue's offset in warr, sections queued, first lock clock
    u32 *wcnt;         // [n_lock] sections each word will queue (counted before the walk)
    u32 *warr;         // [n_lock] the words' queues: their sections in acquire order
    u32 *nodes;        // [n_lock][GW_NW] scope key, H vector, P vector, next lock clock of the word,
                       // L^r / L^w vectors made under it (0: none, no lookup needed)
    u32 *cs;           // [n_lock][GW_CSW] critical sections
    u32 *rec;          // [n_rec][3] location, write, next record of the section
    u32 *wit;          // [n_lock] a thread whose word of section c's acquire time was above the
                       // clock of the last thread that compared them (NONE: none yet): checked
                       // first, it rejects most sections without a full comparison
    u32 n_lock, n_rec;
    u32 *vec;          // clock vectors
    u32 cap_vec;
    bool ok;
};

__device__ inline u32 gw_pow2(u64 n) {
    u64 c = 16;
    while (c < n && c < (1ull << 31)) c <<= 1;
    return (u32)c;
}

__device__ inline GwHeap gw_carve(const GwcpBufs &G, u32 T, u32 wo_cap) {
    GwHeap m;
    const u64 nl = G.hdr[GH_LOCKOPS], nr = G.hdr[GH_CSREC];
    u64 o = 0;
    // every array starts on an even word (8-byte aligned for the u64 keys)
    auto take = [&](u64 words) -> u32 * {
        u32 *p = G.heap + o;
        o += (words + 1) & ~1ull;
        return p;
    };
    const u64 TT = (u64)T * T;
    m.P = take(TT);
    m.H = take(TT);
    m.J = take(TT);
    m.N = take(T);
    m.held_n = take(T);
    m.held = take((u64)T * GW_HELD);
    m.lastsnap = take(T);
    m.JH = take(T);
    m.wsnap = take(wo_cap);
    m.cw = gw_pow2(2 * nl + 1);
    m.wkey = (u64 *)take(2ull * m.cw);
    m.wval = take(m.cw);
    m.cl = gw_pow2(2 * nr + 1);
    m.lkey = (u64 *)take(2ull * m.cl);
    m.lval = take(m.cl);
    m.n_lock = (u32)nl;
    m.n_rec = (u32)nr;
    m.words = take(4 * nl);
    m.wcnt = take(nl);
    m.warr = take(nl);
    m.nodes = take(GW_NW * nl);
    m.cs = take(GW_CSW * nl);
    m.rec = take(3 * nr);
    m.wit = take(nl);
    m.ok = o <= G.heap_words && nl < (1u << 30) && nr < (1u << 30);
    const u64 rest = m.ok ? (G.heap_words - o) / (T ? T : 1) : 0;
    m.vec = G.heap + o;
    m.cap_vec = (u32)(rest > 0x7fffffffull ? 0x7fffffffull : rest);
    return m;
}

__device__ inline u32 gw_hash(u64 key, u32 cap) { return (u32)((key * 0x9E3779B97F4A7C15ull) >> 32) & (cap - 1); }

// Lookup (any lane; the tables change only between barriers): the value of key, NONE when absent.
__device__ inline u32 gw_find(const u64 *keys, const u32 *vals, u32 cap, u64 key) {
    u32 s = gw_hash(key, cap);
    for (u32 probe = 0; probe < cap; probe++, s = (s + 1) & (cap - 1)) {
        const u64 k = keys[s];
        if (k == key) return vals[s];
        if (k == ~0ull) return NONE;
    }
    return NONE;
}

// Lane 0: the value slot of key, inserted with value NONE when absent (the tables are sized at
// twice the keys they can receive, so a free slot is always found).
__device__ inline u32 *gw_insert(u64 *keys, u32 *vals, u32 cap, u64 key) {
    u32 s = gw_hash(key, cap);
    for (u32 probe = 0; probe < cap; probe++, s = (s + 1) & (cap - 1)) {
        const u64 k = keys[s];
        if (k == key) return &vals[s];
        if (k == ~0ull) {
            keys[s] = key;
            vals[s] = NONE;
            return &vals[s];
        }
    }
    return nullptr;
}

__device__ inline u64 gw_lkey(u32 node, u32 x, u32 rw) { return ((u64)node << 33) | ((u64)x << 1) | rw; }

// ---------------------------------------------------------------- per-thread walk

__global__ void k_gw_init(DevParams *P, u32 *hdr) {
    if (threadIdx.x < GH_WORDS) hdr[threadIdx.x] = 0;
    if (threadIdx.x == 0) P->gw_pairs = 0;
}

__global__ void k_gw_thread(Bufs b, GwcpBufs G) {
    DevParams *P = b.prm;
    if (!gw_active(P)) return;
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < b.T; t += gridDim.x * blockDim.x) {
        const u32 lo = b.s_cnt[t], hi = b.s_cnt[t + 1];
        u32 n = 1, depth = 0, lockops = 0;
        u32 held[GW_HELD];
        for (u32 p = lo; p < hi; p++) {
            u32 opens = 0;
            if ((P->mode & MODE_SYNC) && gw_lockop(b, p)) {
                const uint8_t f = b.s_flags[p];
                const u32 x = gw_loc(b, P, b.ev[b.s_pidx[p]]);
                lockops++;
                if (f & SF_REL) {
                    for (u32 q = 0; q < depth; q++)
                        if (held[q] == x) {
                            for (u32 r = q + 1; r < depth; r++) held[r - 1] = held[r];
                            depth--;
                            break;
                        }
                    n++;
                }
                if (f & SF_ACQ) {
                    bool h = false;
                    for (u32 q = 0; q < depth; q++) h |= held[q] == x;
                    if (!h) {
                        if (depth == GW_HELD) {
                            atomicOr(&P->err, ERR_GWCP);
                            return;
                        }
                        held[depth++] = x;
                        opens = 1;
                    }
                }
            }
            // a barrier arrival: the local time after the instance completes (a valid trace has no
            // event of the thread before that)
            const u32 kind = b.s_kind[p];
            if (kind == 4u || kind == 5u) n++;
            G.n_after[p] = n;
            G.depth[p] = depth;
            G.snap[p] = opens;  // (snap is written again by k_gw_post, after the walk)
        }
        if (lockops) atomicAdd(&G.hdr[GH_LOCKOPS], lockops);
    }
}

// ---------------------------------------------------------------- relevant events

__device__ inline bool gw_bar_complete(const Bufs &b, u32 p, u32 i, u32 blk, u32 *slot) {
    *slot = b.inst_off[blk] + b.s_phase[p] - 1;
    return b.inst_last[*slot] == i && b.inst_cnt[*slot] == b.n_active[blk];
}
__device__ inline bool gw_wbar_complete(const Bufs &b, u32 p, u32 i) {
    const u32 inst = b.s_winst[p];
    return inst != NONE && b.winst_last[inst] == i && b.winst_arrived[inst] == b.winst_mask[inst];
}

// flag[i]: P can change at event i; flag[N] = 0.
__global__ void k_gw_mark(Bufs b, GwcpBufs G, u32 *flag) {
    DevParams *P = b.prm;
    const bool on = gw_active(P);
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i <= b.N; i += gridDim.x * blockDim.x) {
        u32 f = 0;
        if (on && i < b.N) {
            const uint4 e = b.ev[i];
            const u32 kind = e.z & 15u, t = e.y;
            if (kind == 4u) {
                const u32 p = gw_entry(b, t, i);
                u32 slot;
                f = p != NONE && gw_bar_complete(b, p, i, block_of(b, t), &slot);
            } else if (kind == 5u) {
                const u32 p = gw_entry(b, t, i);
                f = p != NONE && (P->mode & MODE_WBAR) && gw_wbar_complete(b, p, i);
            } else if (kind != 3u) {
                const u32 p = kind == 2u || kind >= 6u ? gw_entry(b, t, i) : NONE;
                if (p != NONE && (P->mode & MODE_SYNC) && gw_lockop(b, p)) {
                    f = 1;
                } else {
                    // a read or write (an atomic that is no lock operation is a write) inside the
                    // critical sections open after the thread's previous entry
                    const u32 j = list_search(b, t, i);
                    const u32 d = j == NONE ? 0u : G.depth[j];
                    if (d) {
                        f = 1;
                        atomicAdd(&G.hdr[GH_CSREC], d);
                    }
                }
            }
        }
        flag[i] = f;
    }
}

__global__ void k_gw_list(Bufs b, const u32 *scan, u32 *list) {
    if (!gw_active(b.prm)) return;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < b.N; i += gridDim.x * blockDim.x)
        if (scan[i + 1] != scan[i]) list[scan[i]] = i;
}

__global__ void k_gw_clear(Bufs b, GwcpBufs G) {
    DevParams *P = b.prm;
    if (!gw_active(P)) return;
    const u32 T = b.T;
    const GwHeap m = gw_carve(G, T, b.wo_cap);
    if (!m.ok) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&P->err, ERR_GWCP);
        return;
    }
    const u64 g = (u64)blockIdx.x * blockDim.x + threadIdx.x, stride = (u64)gridDim.x * blockDim.x;
    const u64 TT = (u64)T * T;
    for (u64 k = g; k < TT; k += stride) {
        m.P[k] = 0;
        m.J[k] = 0;
        m.H[k] = k % ((u64)T + 1) == 0 ? 1u : 0u;  // the diagonal
    }
    for (u64 t = g; t < T; t += stride) {
        m.N[t] = 1;
        m.held_n[t] = 0;
        m.lastsnap[t] = NONE;
    }
    for (u64 s = g; s < m.cw; s += stride) m.wkey[s] = ~0ull;
    for (u64 c = g; c < m.n_lock; c += stride) m.wit[c] = NONE;
    for (u64 s = g; s < m.cl; s += stride) m.lkey[s] = ~0ull;
}

// ---------------------------------------------------------------- lock words and their queues

// Every lock operation's word joins the word table (lock-free inserts).
__global__ void k_gw_words_insert(Bufs b, GwcpBufs G) {
    const DevParams *P = b.prm;
    if (!gw_active(P) || !(P->mode & MODE_SYNC)) return;
    const GwHeap m = gw_carve(G, b.T, b.wo_cap);
    if (!m.ok) return;
    for (u32 p = blockIdx.x * blockDim.x + threadIdx.x; p < P->n_sync; p += gridDim.x * blockDim.x) {
        if (!gw_lockop(b, p)) continue;
        const u64 key = gw_loc(b, P, b.ev[b.s_pidx[p]]);
        u32 sl = gw_hash(key, m.cw);
        for (u32 probe = 0; probe < m.cw; probe++, sl = (sl + 1) & (m.cw - 1)) {
            const u64 prev = atomicCAS((unsigned long long *)&m.wkey[sl], ~0ull, (unsigned long long)key);
            if (prev == ~0ull || prev == key) break;
        }
    }
}

// A row per word of the table, its queue empty.
__global__ void k_gw_words_rows(Bufs b, GwcpBufs G) {
    DevParams *P = b.prm;
    if (!gw_active(P) || !(P->mode & MODE_SYNC)) return;
    const GwHeap m = gw_carve(G, b.T, b.wo_cap);
    if (!m.ok) return;
    for (u32 sl = blockIdx.x * blockDim.x + threadIdx.x; sl < m.cw; sl += gridDim.x * blockDim.x) {
        const u64 key = m.wkey[sl];
        if (key == ~0ull) continue;
        const u32 w = atomicAdd(&G.hdr[GH_NWORDS], 1u);
        m.wval[sl] = w;
        m.words[(u64)w * 4] = (u32)key;
        m.words[(u64)w * 4 + 1] = 0;
        m.words[(u64)w * 4 + 2] = 0;
        m.words[(u64)w * 4 + 3] = NONE;
        m.wcnt[w] = 0;
    }
}

// Sections each word will queue: one per acquire that opens one (k_gw_thread flagged them).
__global__ void k_gw_words_count(Bufs b, GwcpBufs G) {
    const DevParams *P = b.prm;
    if (!gw_active(P) || !(P->mode & MODE_SYNC)) return;
    const GwHeap m = gw_carve(G, b.T, b.wo_cap);
    if (!m.ok) return;
    for (u32 p = blockIdx.x * blockDim.x + threadIdx.x; p < P->n_sync; p += gridDim.x * blockDim.x) {
        if (!G.snap[p]) continue;
        const u32 w = gw_find(m.wkey, m.wval, m.cw, gw_loc(b, P, b.ev[b.s_pidx[p]]));
        atomicAdd(&m.wcnt[w], 1u);
    }
}

// The queues' offsets: an exclusive scan of the counts (one workgroup).
__global__ __launch_bounds__(1024) void k_gw_words_off(Bufs b, GwcpBufs G) {
    __shared__ u32 tot[1024];
    const DevParams *P = b.prm;
    if (!gw_active(P) || !(P->mode & MODE_SYNC)) return;
    const GwHeap m = gw_carve(G, b.T, b.wo_cap);
    if (!m.ok) return;
    const u32 nw = G.hdr[GH_NWORDS], per = (nw + 1023) / 1024;
    const u32 lo = min(threadIdx.x * per, nw), hi = min(lo + per, nw);
    u32 sum = 0;
    for (u32 w = lo; w < hi; w++) sum += m.wcnt[w];
    tot[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 run = 0;
        for (u32 k = 0; k < 1024; k++) {
            const u32 v = tot[k];
            tot[k] = run;
            run += v;
        }
    }
    __syncthreads();
    u32 off = tot[threadIdx.x];
    for (u32 w = lo; w < hi; w++) {
        m.words[(u64)w * 4 + 1] = off;
        off += m.wcnt[w];
    }
}

// ---------------------------------------------------------------- the interpreter

// All lanes: dst = max(dst, src) over T words; true (in every lane) when a word grew.
__device__ inline bool gw_join(u32 *dst, const u32 *src, u32 T) {
    bool ch = false;
    for (u32 w = threadIdx.x; w < T; w += GW_THREADS) {
        const u32 v = src[w];
        if (v > dst[w]) {
            dst[w] = v;
            ch = true;
        }
    }
    return __syncthreads_or(ch);
}

// Lane 0's value to every lane.
__device__ inline u32 gw_bcast(u32 v, u32 *slot) {
    if (threadIdx.x == 0) *slot = v;
    __syncthreads();
    const u32 r = *slot;
    __syncthreads();
    return r;
}

// Critical-section row: [0] thread, [1] word row, [2] acquire key, [3] release key, [4] release
// event (NONE while open), [5] vector of C_t at the acquire, [6] vector of H_t at the release,
// [7] first read / write record.
__global__ __launch_bounds__(GW_THREADS) void k_gw_interp(Bufs b, GwcpBufs G, const u32 *scan, const u32 *list) {
    DevParams *P = b.prm;
    if (!gw_active(P)) return;
    const u32 T = b.T, n_rel = scan[b.N];
    const GwHeap m = gw_carve(G, T, b.wo_cap);
    __shared__ u32 s_b;                                    // broadcast slot
    __shared__ u32 s_vec, s_cs, s_nodes, s_rec;  // lane 0's allocation counters
    __shared__ u32 s_full;
    __shared__ u32 s_cand[GW_THREADS], s_ncand, s_more;   // rule (ii)'s candidates
    __shared__ u32 s_pt[GW_MAX_T];                         // ... and P_t meanwhile
    __shared__ u32 s_g[GW_MAX_T];                          // ... and the releaser's row of J
    if (threadIdx.x == 0) {
        s_vec = s_cs = s_nodes = s_rec = 0;
        s_full = 0;
    }
    __syncthreads();
    // lane 0: a fresh clock vector, NONE when the pool is spent
    auto new_vec = [&]() -> u32 {
        if (s_vec >= m.cap_vec) {
            s_full = 1;
            return NONE;
        }
        return s_vec++;
    };
    auto vec = [&](u32 h) -> u32 * { return m.vec + (u64)h * T; };
    for (u32 r = 0; r < n_rel; r++) {
        const u32 i = list[r];
        const uint4 e = b.ev[i];
        const u32 t = e.y, kind = e.z & 15u, blk = block_of(b, t);
        u32 *Pt = m.P + (u64)t * T, *Ht = m.H + (u64)t * T;
        const u32 pre = m.lastsnap[t];
        bool pch = false;

        if (kind == 4u || kind == 5u) {
            // SYNC at the last arrival: every participant takes the join J of their C (P with its
            // own local time) and of their H, then increments; J is their shared copy of P
            const u32 p = gw_entry(b, t, i);
            u32 ulo, uhi, wbase = 0, mask = 0, slot = NONE, inst = NONE;
            if (kind == 4u) {
                gw_bar_complete(b, p, i, blk, &slot);
                ulo = blk * b.tpb;
                uhi = ulo + b.tpb;
            } else {
                inst = b.s_winst[p];
                mask = b.winst_mask[inst];
                wbase = t - t % b.tpb % b.ws;
                ulo = wbase;
                uhi = wbase + 32;
            }
            const u32 hj = gw_bcast(threadIdx.x == 0 ? new_vec() : 0u, &s_b);
            if (hj == NONE) break;
            u32 *J = vec(hj);
            for (u32 w = threadIdx.x; w < T; w += GW_THREADS) {
                u32 mj = 0, mh = 0;
#pragma unroll 8
                for (u32 u = ulo; u < uhi; u++) {
                    const bool part = kind == 4u ? b.act[u] != 0 : ((mask >> (u - wbase)) & 1u) != 0;
                    if (!part) continue;
                    mj = max(mj, w == u ? m.N[u] : m.P[(u64)u * T + w]);
                    mh = max(mh, m.H[(u64)u * T + w]);
                }
                J[w] = mj;
                m.JH[w] = mh;
            }
            __syncthreads();
            for (u32 u = ulo; u < uhi; u++) {
                const bool part = kind == 4u ? b.act[u] != 0 : ((mask >> (u - wbase)) & 1u) != 0;
                if (!part) continue;
                u32 *Pu = m.P + (u64)u * T, *Hu = m.H + (u64)u * T;
                for (u32 w = threadIdx.x; w < T; w += GW_THREADS) {
                    Pu[w] = J[w];
                    Hu[w] = m.JH[w] + (w == u ? 1u : 0u);
                }
            }
            for (u32 u = ulo + threadIdx.x; u < uhi; u += GW_THREADS) {
                const bool part = kind == 4u ? b.act[u] != 0 : ((mask >> (u - wbase)) & 1u) != 0;
                if (!part) continue;
                m.N[u] += 1;
                m.lastsnap[u] = hj;
            }
            if (threadIdx.x == 0) {
                if (kind == 4u) G.barsnap[slot] = hj;
                else m.wsnap[inst] = hj;
            }
            __syncthreads();
            continue;
        }

        const u32 p = kind == 2u || kind >= 6u ? gw_entry(b, t, i) : NONE;
        const bool lockop = p != NONE && (P->mode & MODE_SYNC) && gw_lockop(b, p);
        const u32 x = gw_loc(b, P, e);
        if (!lockop) {
            // Algorithm 2 (a read, or a write: a plain write or an atomic): join L^w, for a write also
            // L^r, of x under every lock clock of a held section's word whose scope overlaps the
            // section's; then x joins the section's reads or writes
            // (every vector found is joined into registers, P_t written once)
            const bool write = kind != 0u;
            const u32 nh = m.held_n[t];
            u32 acc[GW_WPT];
#pragma unroll
            for (u32 k = 0; k < GW_WPT; k++) acc[k] = 0;
            bool any = false;
            for (u32 q = 0; q < nh; q++) {
                const u32 *C = m.cs + (u64)m.held[(u64)t * GW_HELD + q] * GW_CSW;
                for (u32 nd = m.words[(u64)C[1] * 4 + 3]; nd != NONE; nd = m.nodes[(u64)nd * GW_NW + 3]) {
                    if (!gw_overlap(m.nodes[(u64)nd * GW_NW], C[2]) || !m.nodes[(u64)nd * GW_NW + 4]) continue;
                    for (u32 rw = write ? 0u : 1u; rw < 2u; rw++) {
                        const u32 h = gw_find(m.lkey, m.lval, m.cl, gw_lkey(nd, x, rw));
                        if (h == NONE) continue;
                        any = true;
                        const u32 *V = vec(h);
#pragma unroll
                        for (u32 k = 0; k < GW_WPT; k++) {
                            const u32 w = threadIdx.x + k * GW_THREADS;
                            if (w < T) acc[k] = max(acc[k], V[w]);
                        }
                    }
                }
            }
            if (any) {
                bool ch = false;
#pragma unroll
                for (u32 k = 0; k < GW_WPT; k++) {
                    const u32 w = threadIdx.x + k * GW_THREADS;
                    if (w < T && acc[k] > Pt[w]) {
                        Pt[w] = acc[k];
                        ch = true;
                    }
                }
                pch |= __syncthreads_or(ch);
            }
            if (threadIdx.x == 0)
                for (u32 q = 0; q < nh; q++) {
                    u32 *C = m.cs + (u64)m.held[(u64)t * GW_HELD + q] * GW_CSW;
                    const u32 rc = s_rec++;  // counted by k_gw_mark: always below n_rec
                    m.rec[(u64)rc * 3] = x;
                    m.rec[(u64)rc * 3 + 1] = write ? 1u : 0u;
                    m.rec[(u64)rc * 3 + 2] = C[7];
                    C[7] = rc;
                }
            __syncthreads();
        } else {
            const uint8_t fl = b.s_flags[p], sc = b.s_scope[p];
            // the word's row (every lock word has one: k_gw_words_rows)
            const u32 wrow = gw_find(m.wkey, m.wval, m.cw, x);
            u32 *W = m.words + (u64)wrow * 4;
            if (fl & SF_REL) {
                // RELEASE (Algorithm 1)
                const u32 key = (sc & 3u) == 0 ? blk : GW_DEV;
                u32 ci = NONE;
                if (threadIdx.x == 0) {
                    // the section it closes: the thread's open one on the word, if any
                    const u32 nh = m.held_n[t];
                    u32 *hl = m.held + (u64)t * GW_HELD;
                    for (u32 q = 0; q < nh; q++)
                        if (m.cs[(u64)hl[q] * GW_CSW + 1] == wrow) {
                            ci = hl[q];
                            for (u32 q2 = q + 1; q2 < nh; q2++) hl[q2 - 1] = hl[q2];
                            m.held_n[t] = nh - 1;
                            break;
                        }
                }
                ci = gw_bcast(ci, &s_b);
                if (ci != NONE) {
                    // rule (ii): another thread's released section of the word, released with an
                    // overlapping scope, whose acquire time is below C_t: its release time joins
                    // P_t; again until a pass joins nothing new.  P_t lives in LDS meanwhile.  Every
                    // lane screens one section of the word's queue at a time (most fail on their own
                    // thread's word of the acquire time, or on a witness word); every wavefront then
                    // compares one survivor at a time in full and joins it with LDS atomics.  Joins
                    // only raise P_t, so a comparison that reads words another wavefront is raising
                    // still decides against a clock P_t reaches, and the passes end at the same
                    // least fixpoint as joins taken one by one.  A survivor whose release time is
                    // already below P_t is passed over without the comparison, and that release time
                    // joins the releaser's row of J, which screens later sections
                    for (u32 w = threadIdx.x; w < T; w += GW_THREADS) {
                        s_pt[w] = Pt[w];
                        s_g[w] = m.J[(u64)t * T + w];
                    }
                    __syncthreads();
                    const u32 qoff = W[1], qn = W[2], Nt = m.N[t];
                    const u32 lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
                    bool grew = false;
                    for (bool more = true; more;) {
                        if (threadIdx.x == 0) s_more = 0;
                        __syncthreads();
                        for (u32 c0 = 0; c0 < qn; c0 += GW_THREADS) {
                            bool cand = false;
                            u32 c = 0;
                            if (c0 + threadIdx.x < qn) {
                                c = m.warr[qoff + c0 + threadIdx.x];
                                const u32 *F = m.cs + (u64)c * GW_CSW;
                                if (F[0] != t && F[4] != NONE && gw_overlap(F[3], key)) {
                                    // (covered when the row of release times found below P_t
                                    // holds its own word of this one)
                                    const bool done = vec(F[6])[F[0]] <= s_g[F[0]];
                                    const u32 *A = vec(F[5]);
                                    const u32 wv = m.wit[c];
                                    cand = !done && A[F[0]] <= s_pt[F[0]] &&
                                           (wv == NONE || A[wv] <= (wv == t ? Nt : s_pt[wv]));
                                }
                            }
                            if (threadIdx.x == 0) s_ncand = 0;
                            __syncthreads();
                            if (cand) s_cand[atomicAdd(&s_ncand, 1u)] = c;
                            __syncthreads();
                            const u32 nc = s_ncand;
                            for (u32 k = wave; k < nc; k += GW_THREADS / 64) {
                                const u32 cc = s_cand[k];
                                const u32 *F = m.cs + (u64)cc * GW_CSW;
                                const u32 *A = vec(F[5]), *RH = vec(F[6]);
                                // (32 words per lane in flight: a comparison waits for memory once
                                // per 2,048 words)
                                // A release time already below P_t adds nothing, whatever the
                                // acquire time: the section is passed over without comparing that,
                                // and t covers its thread's sections up to it from now on (P_t only
                                // grows, and H_u is monotone)
                                bool adds = false;
                                for (u32 w0 = lane; w0 < T; w0 += 64 * GW_BATCH) {
                                    u32 x[GW_BATCH];
#pragma unroll
                                    for (u32 j = 0; j < GW_BATCH; j++) {
                                        const u32 w = w0 + j * 64;
                                        x[j] = w < T ? RH[w] : 0u;
                                    }
#pragma unroll
                                    for (u32 j = 0; j < GW_BATCH; j++) {
                                        const u32 w = w0 + j * 64;
                                        if (w < T && x[j] > s_pt[w]) adds = true;
                                    }
                                }
                                if (!ballot(adds)) {
                                    // (read again: the words are in the cache)
                                    for (u32 w0 = lane; w0 < T; w0 += 64 * GW_BATCH) {
                                        u32 x[GW_BATCH];
#pragma unroll
                                        for (u32 j = 0; j < GW_BATCH; j++) {
                                            const u32 w = w0 + j * 64;
                                            x[j] = w < T ? RH[w] : 0u;
                                        }
#pragma unroll
                                        for (u32 j = 0; j < GW_BATCH; j++) {
                                            const u32 w = w0 + j * 64;
                                            if (w < T && x[j] > s_g[w]) atomicMax(&s_g[w], x[j]);
                                        }
                                    }
                                    continue;
                                }
                                u32 wfail = NONE;
                                for (u32 w0 = lane; w0 < T; w0 += 64 * GW_BATCH) {
                                    u32 x[GW_BATCH];
#pragma unroll
                                    for (u32 j = 0; j < GW_BATCH; j++) {
                                        const u32 w = w0 + j * 64;
                                        x[j] = w < T ? A[w] : 0u;
                                    }
#pragma unroll
                                    for (u32 j = 0; j < GW_BATCH; j++) {
                                        const u32 w = w0 + j * 64;
                                        if (w < T && x[j] > (w == t ? Nt : s_pt[w])) wfail = w;
                                    }
                                }
                                const u64 am = ballot(wfail != NONE);
                                if (am) {
                                    // a witness for the next comparisons
                                    const u32 src = (u32)__builtin_ctzll(am);
                                    const u32 wf = __shfl(wfail, (int)src, 64);
                                    if (lane == 0) m.wit[cc] = wf;
                                    continue;
                                }
                                bool ch = false;
                                for (u32 w0 = lane; w0 < T; w0 += 64 * GW_BATCH) {
                                    u32 x[GW_BATCH];
#pragma unroll
                                    for (u32 j = 0; j < GW_BATCH; j++) {
                                        const u32 w = w0 + j * 64;
                                        x[j] = w < T ? RH[w] : 0u;
                                    }
#pragma unroll
                                    for (u32 j = 0; j < GW_BATCH; j++) {
                                        const u32 w = w0 + j * 64;
                                        if (w < T && x[j] > s_pt[w]) {
                                            atomicMax(&s_pt[w], x[j]);
                                            ch = true;
                                        }
                                        if (w < T && x[j] > s_g[w]) atomicMax(&s_g[w], x[j]);
                                    }
                                }
                                if (ballot(ch) && lane == 0) s_more = 1;
                            }
                            __syncthreads();  // s_cand and s_ncand are reused; the joins are done
                        }
                        __syncthreads();
                        more = s_more != 0;
                        grew |= more;
                        __syncthreads();  // s_more is reset next
                    }
                    for (u32 w = threadIdx.x; w < T; w += GW_THREADS) {
                        if (grew) Pt[w] = s_pt[w];
                        m.J[(u64)t * T + w] = s_g[w];
                    }
                    __syncthreads();
                    if (grew) pch = true;
                }
                // the lock clock of (word, key), created on first use
                u32 nd = NONE, fresh = 0;
                if (threadIdx.x == 0) {
                    nd = W[3];
                    while (nd != NONE && m.nodes[(u64)nd * GW_NW] != key) nd = m.nodes[(u64)nd * GW_NW + 3];
                    if (nd == NONE) {
                        const u32 hv = new_vec(), pv = new_vec();
                        if (hv != NONE && pv != NONE) {
                            nd = s_nodes++;  // at most one per release
                            m.nodes[(u64)nd * GW_NW] = key;
                            m.nodes[(u64)nd * GW_NW + 1] = hv;
                            m.nodes[(u64)nd * GW_NW + 2] = pv;
                            m.nodes[(u64)nd * GW_NW + 3] = W[3];
                            m.nodes[(u64)nd * GW_NW + 4] = 0;
                            W[3] = nd;
                            fresh = 1;
                        }
                    }
                }
                nd = gw_bcast(nd, &s_b);
                if (nd == NONE) break;
                fresh = gw_bcast(fresh, &s_b);
                u32 *HL = vec(m.nodes[(u64)nd * GW_NW + 1]), *PL = vec(m.nodes[(u64)nd * GW_NW + 2]);
                if (fresh) {
                    for (u32 w = threadIdx.x; w < T; w += GW_THREADS) HL[w] = PL[w] = 0;
                    __syncthreads();
                }
                if (ci != NONE) {
                    // L^r / L^w of (lock clock, x) join H_t for the section's reads / writes x
                    const u32 head = m.cs[(u64)ci * GW_CSW + 7];
                    for (u32 rc = head; rc != NONE; rc = m.rec[(u64)rc * 3 + 2]) {
                        u32 h = NONE, nw = 0;
                        if (threadIdx.x == 0) {
                            u32 *v = gw_insert(m.lkey, m.lval, m.cl, gw_lkey(nd, m.rec[(u64)rc * 3], m.rec[(u64)rc * 3 + 1]));
                            if (*v == NONE) {
                                *v = new_vec();
                                nw = 1;
                                m.nodes[(u64)nd * GW_NW + 4] += 1;
                            }
                            h = *v;
                        }
                        h = gw_bcast(h, &s_b);
                        nw = gw_bcast(nw, &s_b);
                        if (h == NONE) break;
                        u32 *L = vec(h);
                        for (u32 w = threadIdx.x; w < T; w += GW_THREADS) L[w] = nw ? Ht[w] : max(L[w], Ht[w]);
                        __syncthreads();
                    }
                    // the section's release time (Rel_l for the other threads)
                    u32 h = NONE;
                    if (threadIdx.x == 0) {
                        h = new_vec();
                        u32 *C = m.cs + (u64)ci * GW_CSW;
                        C[3] = key;
                        C[4] = i;
                        C[6] = h;
                    }
                    h = gw_bcast(h, &s_b);
                    if (h == NONE) break;
                    u32 *RH = vec(h);
                    for (u32 w = threadIdx.x; w < T; w += GW_THREADS) RH[w] = Ht[w];
                    __syncthreads();
                }
                // H_<l,s> and P_<l,s> publish the thread's clocks (joined), then its local time moves
                gw_join(HL, Ht, T);
                gw_join(PL, Pt, T);
                if (threadIdx.x == 0) {
                    m.N[t] += 1;
                    Ht[t] += 1;
                }
                __syncthreads();
            }
            if (fl & SF_ACQ) {
                // ACQUIRE (Algorithm 1): P and H of every lock clock of the word whose scope overlaps
                const u32 key = ((sc >> 2) & 3u) == 0 ? blk : GW_DEV;
                // (all of them joined into registers, P_t and H_t written once)
                {
                    u32 ap[GW_WPT], ah[GW_WPT];
#pragma unroll
                    for (u32 k = 0; k < GW_WPT; k++) ap[k] = ah[k] = 0;
                    for (u32 nd = W[3]; nd != NONE; nd = m.nodes[(u64)nd * GW_NW + 3]) {
                        if (!gw_overlap(m.nodes[(u64)nd * GW_NW], key)) continue;
                        const u32 *PL = vec(m.nodes[(u64)nd * GW_NW + 2]), *HL = vec(m.nodes[(u64)nd * GW_NW + 1]);
#pragma unroll
                        for (u32 k = 0; k < GW_WPT; k++) {
                            const u32 w = threadIdx.x + k * GW_THREADS;
                            if (w < T) {
                                ap[k] = max(ap[k], PL[w]);
                                ah[k] = max(ah[k], HL[w]);
                            }
                        }
                    }
                    bool ch = false;
#pragma unroll
                    for (u32 k = 0; k < GW_WPT; k++) {
                        const u32 w = threadIdx.x + k * GW_THREADS;
                        if (w < T) {
                            if (ap[k] > Pt[w]) {
                                Pt[w] = ap[k];
                                ch = true;
                            }
                            if (ah[k] > Ht[w]) Ht[w] = ah[k];
                        }
                    }
                    pch |= __syncthreads_or(ch);
                }
                // a section opens unless the thread holds the word (Acq_l for the other threads)
                u32 h = NONE;
                if (threadIdx.x == 0) {
                    const u32 nh = m.held_n[t];
                    bool holding = false;
                    for (u32 q = 0; q < nh; q++) holding |= m.cs[(u64)m.held[(u64)t * GW_HELD + q] * GW_CSW + 1] == wrow;
                    if (!holding) {
                        h = new_vec();
                        if (h != NONE) {
                            const u32 ci = s_cs++;  // at most one per acquire
                            u32 *C = m.cs + (u64)ci * GW_CSW;
                            C[0] = t; C[1] = wrow; C[2] = key; C[3] = key; C[4] = NONE; C[5] = h; C[6] = NONE;
                            C[7] = NONE;
                            m.warr[W[1] + W[2]] = ci;  // the word's queue (counted: k_gw_words_count)
                            W[2] += 1;
                            m.held[(u64)t * GW_HELD + nh] = ci;  // below GW_HELD: k_gw_thread checked
                            m.held_n[t] = nh + 1;
                        }
                    }
                }
                h = gw_bcast(h, &s_b);
                if (h != NONE) {
                    u32 *A = vec(h);
                    for (u32 w = threadIdx.x; w < T; w += GW_THREADS) A[w] = w == t ? m.N[t] : Pt[w];
                    __syncthreads();
                }
            }
        }
        if (s_full) break;
        // the copy of P_t after the event: a new one when it changed
        u32 post = pre;
        if (pch) {
            post = gw_bcast(threadIdx.x == 0 ? new_vec() : 0u, &s_b);
            if (post == NONE) break;
            u32 *S = vec(post);
            for (u32 w = threadIdx.x; w < T; w += GW_THREADS) S[w] = Pt[w];
        }
        if (threadIdx.x == 0) {
            m.lastsnap[t] = post;
            G.evsnap[r] = post;
            // the race check of an access sees P_t after Algorithm 2's joins, of a lock operation
            // before its own effect
            G.evchk[r] = lockop ? pre : post;
        }
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_full) atomicOr(&P->err, ERR_GWCP);
}

// The copy of P in force after each sync entry, carried along every thread's list.
__global__ void k_gw_post(Bufs b, GwcpBufs G, const u32 *scan) {
    if (!gw_active(b.prm)) return;
    const GwHeap m = gw_carve(G, b.T, b.wo_cap);
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < b.T; t += gridDim.x * blockDim.x) {
        const u32 lo = b.s_cnt[t], hi = b.s_cnt[t + 1], blk = block_of(b, t);
        u32 cur = NONE;
        for (u32 p = lo; p < hi; p++) {
            const u32 kind = b.s_kind[p];
            if (kind == 4u) {
                const u32 slot = b.inst_off[blk] + b.s_phase[p] - 1;
                if (b.inst_cnt[slot] == b.n_active[blk]) cur = G.barsnap[slot];
            } else if (kind == 5u) {
                const u32 inst = (b.prm->mode & MODE_WBAR) ? b.s_winst[p] : NONE;
                if (inst != NONE && b.winst_arrived[inst] == b.winst_mask[inst]) cur = m.wsnap[inst];
            } else {
                const u32 i = b.s_pidx[p];
                if (scan[i + 1] != scan[i]) cur = G.evsnap[scan[i]];
            }
            G.snap[p] = cur;
        }
    }
}

// The local time of thread t at its event with trace index i.
__device__ inline u32 gw_epoch(const Bufs &b, const GwcpBufs &G, u32 t, u32 i) {
    const u32 j = list_search(b, t, i);
    return j == NONE ? 1u : G.n_after[j];
}

__global__ __launch_bounds__(256) void k_gw_check(Bufs b, GwcpBufs G, const u32 *scan) {
    DevParams *P = b.prm;
    if (!gw_active(P)) return;
    const GwHeap m = gw_carve(G, b.T, b.wo_cap);
    const SegCtx s = seg_ctx(b);
    for (u64 pos = (u64)blockIdx.x * blockDim.x + threadIdx.x; pos < s.n; pos += (u64)gridDim.x * blockDim.x) {
        const u32 kb = seg_key(s, pos), ib = s.i[pos], tb = seg_tid(s, pos), cb = info_cat(seg_info(s, pos));
        const u32 bb = block_of(b, tb);
        // b's clock: its own when P can change at b, else the one after its thread's previous entry
        u32 h;
        if (scan[ib + 1] != scan[ib]) {
            h = G.evchk[scan[ib]];
        } else {
            const u32 j = list_search(b, tb, ib);
            h = j == NONE ? NONE : G.snap[j];
        }
        const u32 *V = h == NONE ? nullptr : m.vec + (u64)h * b.T;
        for (u64 q = pos; q > 0;) {
            q--;
            if (seg_key(s, q) != kb) break;
            const u32 ta = seg_tid(s, q);
            if (ta == tb) continue;
            const u32 ca = info_cat(seg_info(s, q));
            if (ca == CAT_R && cb == CAT_R) continue;
            if (ca >= CAT_AD && cb >= CAT_AD && (ca == CAT_AD || cb == CAT_AD || block_of(b, ta) == bb)) continue;
            const u32 ia = s.i[q];
            if (gw_epoch(b, G, ta, ia) <= (V ? V[ta] : 0u)) continue;
            const u32 slot = atomicAdd(&P->gw_pairs, 1u);
            if (slot < G.cap) {
                G.pf[0][slot] = ia;
                G.ps[0][slot] = ib;
            } else {
                atomicOr(&P->err, ERR_GWPAIRS);
            }
        }
    }
}

__global__ void k_gw_kept(DevParams *P, u64 cap) {
    if (threadIdx.x == 0) P->gw_kept = P->gw_pairs < cap ? P->gw_pairs : (u32)cap;
}

// Pool layout: four pair arrays and the report (6 words per pair of `cap`), the counters, then the
// heap.  False when the pool cannot hold the pairs, the counters and the dense clocks.
bool gwcp_layout(const Bufs &b, u64 cap, GwcpBufs &G) {
    const u64 fixed = 6 * cap + GH_WORDS;
    const u64 clocks = 3ull * b.T * b.T + (u64)b.T * (GW_HELD + 8) + b.wo_cap;
    if (b.T > GW_MAX_T || b.pool_words < fixed + clocks) return false;
    u32 *p = b.pool;
    G.pf[0] = p; G.ps[0] = p + cap; G.pf[1] = p + 2 * cap; G.ps[1] = p + 3 * cap;
    G.report = (u64 *)(p + 4 * cap);  // 8-byte aligned: the pool starts 256-byte aligned
    G.cap = cap;
    G.hdr = p + 6 * cap;
    G.heap = G.hdr + GH_WORDS;
    G.heap_words = b.pool_words - fixed;
    G.n_after = b.e_prev0;
    G.depth = b.e_prev1;
    G.snap = b.e_src0;
    G.evsnap = b.e_src1;
    G.evchk = b.e_cur;
    G.barsnap = b.inst_opo;
    return true;
}

void gwcp_run(const Bufs &b, const GwcpBufs &G, hipStream_t s) {
    const unsigned gn = (unsigned)((b.N + 256) / 256 > 8192 ? 8192 : (b.N + 256) / 256);
    const unsigned gt = (unsigned)((b.T + 255) / 256 > 2048 ? 2048 : ((b.T + 255) / 256 ? (b.T + 255) / 256 : 1));
    RD_LAUNCH("k_gw_init", k_gw_init, dim3(1), dim3(64), 0, s, b.prm, G.hdr);
    RD_LAUNCH("k_gw_thread", k_gw_thread, dim3(gt), dim3(256), 0, s, b, G);
    RD_LAUNCH("k_gw_mark", k_gw_mark, dim3(gn), dim3(256), 0, s, b, G, b.e_scan0);
    scan_exclusive(b.e_scan0, (u64)b.N + 1, b.part, s);
    RD_LAUNCH("k_gw_list", k_gw_list, dim3(gn), dim3(256), 0, s, b, (const u32 *)b.e_scan0, b.e_scan1);
    RD_LAUNCH("k_gw_clear", k_gw_clear, dim3(1024), dim3(256), 0, s, b, G);
    RD_LAUNCH("k_gw_words_insert", k_gw_words_insert, dim3(gn), dim3(256), 0, s, b, G);
    RD_LAUNCH("k_gw_words_rows", k_gw_words_rows, dim3(1024), dim3(256), 0, s, b, G);
    RD_LAUNCH("k_gw_words_count", k_gw_words_count, dim3(gn), dim3(256), 0, s, b, G);
    RD_LAUNCH("k_gw_words_off", k_gw_words_off, dim3(1), dim3(1024), 0, s, b, G);
    RD_LAUNCH("k_gw_interp", k_gw_interp, dim3(1), dim3(GW_THREADS), 0, s, b, G, (const u32 *)b.e_scan0,
              (const u32 *)b.e_scan1);
    RD_LAUNCH("k_gw_post", k_gw_post, dim3(gt), dim3(256), 0, s, b, G, (const u32 *)b.e_scan0);
    RD_LAUNCH("k_gw_check", k_gw_check, dim3(gn), dim3(256), 0, s, b, G, (const u32 *)b.e_scan0);
    RD_LAUNCH("k_gw_kept", k_gw_kept, dim3(1), dim3(64), 0, s, b.prm, G.cap);
    u32 *const f[2] = {G.pf[0], G.pf[1]}, *const s2[2] = {G.ps[0], G.ps[1]};
    sort_pairs_to(b, f, s2, &b.prm->gw_kept, G.cap, s);
    pack_pairs_to(G.pf[0], G.ps[0], &b.prm->gw_kept, G.cap, G.report, s);
}

}  // namespace rd
