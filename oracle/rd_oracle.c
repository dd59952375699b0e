/*
 * rd_oracle.c -- CPU oracle for scoped happens-before race checking over a recorded GPU trace.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product path (the HIP checker) never calls it, and the two
 * share no code: this file has its own record decoder, its own validation and its own analysis.
 *
 * It computes the same report two independent ways:
 *
 *   orc_bruteforce  The declarative definition.  It builds the happens-before graph of the trace
 *                   (program order; block and warp barriers; release -> acquire on one sync
 *                   variable subject to the scope rule) and takes its transitive closure with
 *                   bitsets in trace order, then reports every conflicting pair the closure does not
 *                   order.  Scoped HB: paper Section 2.2, rules (i), (iii), (iv); race definition:
 *                   Section 1 and Section 2.2; scoped atomics and scoped locks: Section 4 and
 *                   Section 5.1.
 *
 *   orc_check       The paper's per-event vector-clock detector.  Thread clocks H_t are updated as
 *                   in Algorithm 1 (SYNC joins all participants and increments; ACQUIRE joins the
 *                   sync-variable clocks of the scopes that cover the thread; RELEASE publishes H_t
 *                   and increments), and every access is checked, FastTrack style, against the
 *                   location's access history (metadata R_x / W_x of Section 4.1): an earlier access
 *                   a of thread u is ordered before the current access of thread t iff
 *                   epoch(a) <= H_t[u].  Two clock stores are offered:
 *                     mode 1: dense per-thread vector clocks (n_threads entries each);
 *                     mode 0: block-floor + per-thread-exception clocks shared between threads,
 *                             with the forced compression at block barriers of Section 5.2.
 *
 * Readings of the paper that this file fixes (each is also listed in the design notes):
 *   - atomics (ATOMIC, ACQ, REL) are read-modify-writes and count as writes;
 *   - two atomics do not race iff their scopes overlap: one is device/system scoped, or both come
 *     from the same block (Section 4 "scoped locks", Section 5.1 "scoped atomics");
 *   - release -> acquire orders unless both sides are block scoped in different blocks
 *     (rule (iv), Algorithm 1 ACQUIRE);
 *   - a sync-variable clock is joined on release, not overwritten;
 *   - every barrier participant increments its own clock;
 *   - rule (ii) "interwarp order" is not used (independent thread scheduling, Section 2.1);
 *   - a fence orders nothing by itself; an atomic directly preceded in program order by a fence is
 *     a release, one directly followed by a fence is an acquire, both with the fence's scope
 *     (Section 2.1 lock idiom; Section 5.1 "scoped atomics");
 *   - block-barrier participants are the block's active threads (threads with >= 1 event);
 *   - system scope behaves as device scope (one GPU).
 * The alternative "inclusive" reading of the atomic/lock scope rule (a pair is unsynchronised when
 * the blocks differ and at least one side is block scoped) is available through `inclusive` for
 * documentation only.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- record format (own decoder) */

typedef struct {
    uint32_t addr; /* 4-byte word; WBAR: barrier id; FENCE/BAR: unused */
    uint32_t tid;  /* block * threads_per_block + thread_in_block */
    uint32_t meta; /* kind bits 0-3, scope bits 4-5, space bit 6, bits 7-31 zero */
    uint32_t aux;  /* WBAR: lane mask; otherwise opaque */
} orc_event;

enum { K_READ = 0, K_WRITE = 1, K_ATOMIC = 2, K_FENCE = 3, K_BAR = 4, K_WBAR = 5, K_ACQ = 6, K_REL = 7 };
enum { S_BLOCK = 0, S_DEVICE = 1, S_SYSTEM = 2 };

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ETRACE = -3 };

static inline unsigned kind_of(const orc_event *e) { return e->meta & 15u; }
static inline unsigned scope_of(const orc_event *e) { return (e->meta >> 4) & 3u; }
static inline unsigned space_of(const orc_event *e) { return (e->meta >> 6) & 1u; }

static inline int is_access(unsigned k) { return k == K_READ || k == K_WRITE || k == K_ATOMIC || k == K_ACQ || k == K_REL; }
static inline int is_writeish(unsigned k) { return k == K_WRITE || k == K_ATOMIC || k == K_ACQ || k == K_REL; }
static inline int is_atomic(unsigned k) { return k == K_ATOMIC || k == K_ACQ || k == K_REL; }

/* ---------------------------------------------------------------- output pairs */

typedef struct {
    uint64_t n, cap;
    uint32_t *data; /* 2*n entries: first, second */
} orc_pairs;

static int pairs_push(orc_pairs *p, uint32_t a, uint32_t b) {
    if (p->n == p->cap) {
        uint64_t nc = p->cap ? p->cap * 2 : 1024;
        uint32_t *d = (uint32_t *)realloc(p->data, nc * 2 * sizeof(uint32_t));
        if (!d) return ORC_ENOMEM;
        p->data = d;
        p->cap = nc;
    }
    p->data[2 * p->n] = a;
    p->data[2 * p->n + 1] = b;
    p->n++;
    return ORC_OK;
}

static int cmp_pair(const void *x, const void *y) {
    const uint32_t *a = (const uint32_t *)x, *b = (const uint32_t *)y;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    return 0;
}

void orc_pairs_free(orc_pairs *p) {
    free(p->data);
    p->data = NULL;
    p->n = p->cap = 0;
}

/* ---------------------------------------------------------------- common pre-pass */

typedef struct {
    uint32_t n_blocks, tpb, warp_size, n_threads;
    uint64_t n;
    const orc_event *ev;
    /* program order: events of thread t are po_idx[po_start[t] .. po_start[t+1]) */
    uint32_t *po_start, *po_idx;
    uint32_t *po_pos;    /* position of event i inside its thread's list */
    uint32_t *phase;     /* number of BARs of the thread strictly before event i */
    uint8_t *rel_scope;  /* 0xff: not a release; else scope of the release */
    uint8_t *acq_scope;  /* 0xff: not an acquire; else scope of the acquire */
    uint32_t *n_active;  /* active threads per block */
    /* block-barrier instances: instance k (1-based) of block b is bar_inst[bar_off[b] + k - 1] */
    uint32_t *bar_off, *bar_cnt, *bar_last;
    /* warp barriers: per WBAR event, its instance id; instances hold mask and completion */
    uint32_t *wbar_inst;  /* per event: instance index, or UINT32_MAX */
    uint32_t n_winst;
    uint32_t *winst_mask, *winst_arrived, *winst_last, *winst_block;
} prep_t;

static void prep_free(prep_t *p) {
    free(p->po_start); free(p->po_idx); free(p->po_pos); free(p->phase);
    free(p->rel_scope); free(p->acq_scope); free(p->n_active);
    free(p->bar_off); free(p->bar_cnt); free(p->bar_last);
    free(p->wbar_inst); free(p->winst_mask); free(p->winst_arrived); free(p->winst_last);
    free(p->winst_block);
    memset(p, 0, sizeof(*p));
}

static inline uint32_t block_of(const prep_t *p, uint32_t tid) { return tid / p->tpb; }

/* Grid checks (argument errors, not trace errors). */
static int grid_ok(uint32_t n_blocks, uint32_t tpb, uint32_t *warp_size, uint64_t n) {
    if (*warp_size == 0) *warp_size = 32;
    if (n_blocks == 0 || tpb == 0 || tpb > 1024 || *warp_size > 32) return 0;
    if ((uint64_t)n_blocks * tpb >= ((uint64_t)1 << 32)) return 0;
    if (n >= ((uint64_t)1 << 32)) return 0;
    return 1;
}

/* Record-level checks: kind/scope/reserved bits, tid range, sync events in global space. */
static uint64_t first_record_error(const prep_t *p) {
    for (uint64_t i = 0; i < p->n; i++) {
        const orc_event *e = &p->ev[i];
        unsigned k = kind_of(e);
        if ((e->meta >> 7) != 0 || k > 7 || scope_of(e) > 2) return i;
        if (e->tid >= p->n_threads) return i;
        if ((k == K_FENCE || k == K_BAR || k == K_WBAR) && space_of(e) != 0) return i;
    }
    return UINT64_MAX;
}

/* Hash map from a 64-bit key to a dense index (linear probing). */
typedef struct {
    uint64_t cap, n;
    uint64_t *keys;
    uint32_t *vals; /* 0 = empty, else index + 1 */
} hmap;

static int hmap_init(hmap *h, uint64_t expect) {
    uint64_t c = 16;
    while (c < 2 * expect + 16) c <<= 1;
    h->cap = c;
    h->n = 0;
    h->keys = (uint64_t *)malloc(c * sizeof(uint64_t));
    h->vals = (uint32_t *)calloc(c, sizeof(uint32_t));
    return (h->keys && h->vals) ? ORC_OK : ORC_ENOMEM;
}
static void hmap_free(hmap *h) { free(h->keys); free(h->vals); memset(h, 0, sizeof(*h)); }
static inline uint64_t mix64(uint64_t x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL; x ^= x >> 33;
    return x;
}
/* Returns the index for key, inserting next_index if absent (and setting *inserted). */
static uint32_t hmap_get(hmap *h, uint64_t key, uint32_t next_index, int *inserted) {
    uint64_t m = h->cap - 1, s = mix64(key) & m;
    for (;;) {
        if (h->vals[s] == 0) {
            h->keys[s] = key;
            h->vals[s] = next_index + 1;
            h->n++;
            *inserted = 1;
            return next_index;
        }
        if (h->keys[s] == key) { *inserted = 0; return h->vals[s] - 1; }
        s = (s + 1) & m;
    }
}

/* Location of an access: global word, or (block, word) of shared memory (Section 4.1, "shared
 * memory": shared memory of each block is a distinct location). */
static inline uint64_t loc_key(const prep_t *p, const orc_event *e) {
    if (space_of(e) == 1) return ((uint64_t)1 << 63) | ((uint64_t)block_of(p, e->tid) << 32) | e->addr;
    return e->addr;
}

/*
 * Builds program order, barrier phases, inferred releases/acquires and barrier instances, and
 * validates the barrier discipline.  Returns ORC_OK, ORC_ENOMEM, or ORC_ETRACE with *bad set to
 * the first offending event index (record errors first; otherwise the smallest event that breaks
 * the block- or warp-barrier discipline).
 */
static int prepare(prep_t *p, uint32_t n_blocks, uint32_t tpb, uint32_t warp_size,
                   const orc_event *ev, uint64_t n, uint64_t *bad) {
    memset(p, 0, sizeof(*p));
    p->n_blocks = n_blocks; p->tpb = tpb; p->warp_size = warp_size;
    p->n_threads = n_blocks * tpb; p->n = n; p->ev = ev;
    uint64_t rec = first_record_error(p);
    if (rec != UINT64_MAX) { *bad = rec; return ORC_ETRACE; }

    uint32_t T = p->n_threads;
    p->po_start = (uint32_t *)calloc((size_t)T + 1, sizeof(uint32_t));
    p->po_idx = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    p->po_pos = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    p->phase = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    p->rel_scope = (uint8_t *)malloc(n ? n : 1);
    p->acq_scope = (uint8_t *)malloc(n ? n : 1);
    p->n_active = (uint32_t *)calloc(n_blocks, sizeof(uint32_t));
    p->wbar_inst = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    if (!p->po_start || !p->po_idx || !p->po_pos || !p->phase || !p->rel_scope || !p->acq_scope ||
        !p->n_active || !p->wbar_inst)
        return ORC_ENOMEM;

    /* program order: counting sort of event indices by thread (stable => trace order) */
    for (uint64_t i = 0; i < n; i++) p->po_start[ev[i].tid + 1]++;
    for (uint32_t t = 0; t < T; t++) p->po_start[t + 1] += p->po_start[t];
    {
        uint32_t *fill = (uint32_t *)malloc(((size_t)T + 1) * sizeof(uint32_t));
        if (!fill) return ORC_ENOMEM;
        memcpy(fill, p->po_start, ((size_t)T + 1) * sizeof(uint32_t));
        for (uint64_t i = 0; i < n; i++) {
            uint32_t t = ev[i].tid;
            p->po_pos[i] = fill[t] - p->po_start[t];
            p->po_idx[fill[t]++] = (uint32_t)i;
        }
        free(fill);
    }
    for (uint32_t t = 0; t < T; t++)
        if (p->po_start[t + 1] > p->po_start[t]) p->n_active[t / tpb]++;

    /* phases, and releases/acquires: explicit ones, and atomics next to a fence in program order */
    uint32_t *nbar = (uint32_t *)calloc(T ? T : 1, sizeof(uint32_t));
    if (!nbar) return ORC_ENOMEM;
    for (uint32_t t = 0; t < T; t++) {
        uint32_t s = p->po_start[t], e = p->po_start[t + 1], ph = 0;
        for (uint32_t j = s; j < e; j++) {
            uint32_t i = p->po_idx[j];
            unsigned k = kind_of(&ev[i]);
            p->phase[i] = ph;
            p->rel_scope[i] = 0xff;
            p->acq_scope[i] = 0xff;
            if (k == K_REL) p->rel_scope[i] = (uint8_t)scope_of(&ev[i]);
            if (k == K_ACQ) p->acq_scope[i] = (uint8_t)scope_of(&ev[i]);
            if (k == K_ATOMIC) {
                if (j > s && kind_of(&ev[p->po_idx[j - 1]]) == K_FENCE)
                    p->rel_scope[i] = (uint8_t)scope_of(&ev[p->po_idx[j - 1]]);
                if (j + 1 < e && kind_of(&ev[p->po_idx[j + 1]]) == K_FENCE)
                    p->acq_scope[i] = (uint8_t)scope_of(&ev[p->po_idx[j + 1]]);
            }
            if (k == K_BAR) ph++;
        }
        nbar[t] = ph;
    }

    /* block-barrier instances: per block, instance k holds its arrival count and last arrival */
    p->bar_off = (uint32_t *)calloc((size_t)n_blocks + 1, sizeof(uint32_t));
    if (!p->bar_off) { free(nbar); return ORC_ENOMEM; }
    for (uint32_t b = 0; b < n_blocks; b++) {
        uint32_t mx = 0;
        for (uint32_t t = b * tpb; t < (b + 1) * tpb; t++) if (nbar[t] > mx) mx = nbar[t];
        p->bar_off[b + 1] = p->bar_off[b] + mx;
    }
    uint32_t n_inst = p->bar_off[n_blocks];
    p->bar_cnt = (uint32_t *)calloc(n_inst ? n_inst : 1, sizeof(uint32_t));
    p->bar_last = (uint32_t *)calloc(n_inst ? n_inst : 1, sizeof(uint32_t));
    if (!p->bar_cnt || !p->bar_last) { free(nbar); return ORC_ENOMEM; }
    for (uint64_t i = 0; i < n; i++) {
        if (kind_of(&ev[i]) != K_BAR) continue;
        uint32_t b = block_of(p, ev[i].tid);
        uint32_t slot = p->bar_off[b] + p->phase[i]; /* the (phase+1)-th BAR -> instance phase+1 */
        p->bar_cnt[slot]++;
        p->bar_last[slot] = (uint32_t)i; /* trace order: the latest arrival so far */
    }
    free(nbar);

    /* warp-barrier instances: (block, warp, id, occurrence of that id in the lane's program order) */
    hmap wmap;
    uint64_t n_wbar = 0;
    for (uint64_t i = 0; i < n; i++) if (kind_of(&ev[i]) == K_WBAR) n_wbar++;
    if (hmap_init(&wmap, n_wbar) != ORC_OK) return ORC_ENOMEM;
    p->winst_mask = (uint32_t *)malloc((n_wbar ? n_wbar : 1) * sizeof(uint32_t));
    p->winst_arrived = (uint32_t *)calloc(n_wbar ? n_wbar : 1, sizeof(uint32_t));
    p->winst_last = (uint32_t *)calloc(n_wbar ? n_wbar : 1, sizeof(uint32_t));
    p->winst_block = (uint32_t *)calloc(n_wbar ? n_wbar : 1, sizeof(uint32_t));
    uint64_t *winst_first = (uint64_t *)malloc((n_wbar ? n_wbar : 1) * sizeof(uint64_t));
    uint8_t *bad_arrival = (uint8_t *)calloc(n ? n : 1, 1);
    if (!p->winst_mask || !p->winst_arrived || !p->winst_last || !p->winst_block || !winst_first ||
        !bad_arrival) {
        hmap_free(&wmap); free(winst_first); free(bad_arrival);
        return ORC_ENOMEM;
    }
    p->n_winst = 0;
    uint32_t *winst_id = (uint32_t *)malloc((n_wbar ? n_wbar : 1) * sizeof(uint32_t));
    uint32_t *winst_occ = (uint32_t *)malloc((n_wbar ? n_wbar : 1) * sizeof(uint32_t));
    if (!winst_id || !winst_occ) {
        hmap_free(&wmap); free(winst_first); free(bad_arrival); free(winst_id); free(winst_occ);
        return ORC_ENOMEM;
    }
    for (uint32_t t = 0; t < T; t++) {
        uint32_t s = p->po_start[t], e = p->po_start[t + 1];
        for (uint32_t j = s; j < e; j++) {
            uint32_t i = p->po_idx[j];
            p->wbar_inst[i] = UINT32_MAX;
            if (kind_of(&ev[i]) != K_WBAR) continue;
            uint32_t occ = 0; /* earlier WBARs of this thread with the same id */
            for (uint32_t jj = s; jj < j; jj++) {
                const orc_event *o = &ev[p->po_idx[jj]];
                if (kind_of(o) == K_WBAR && o->addr == ev[i].addr) occ++;
            }
            /* instance = (block, warp, id, occurrence); the warp is identified by the tid of its
             * lane 0, so (warp0, id, occ) names the instance exactly */
            uint32_t warp0 = t - ((t % tpb) % warp_size);
            uint64_t key = mix64(mix64(((uint64_t)warp0 << 32) | ev[i].addr) + 0x9e3779b97f4a7c15ULL * (occ + 1));
            int ins;
            uint32_t inst = hmap_get(&wmap, key, p->n_winst, &ins);
            if (ins) {
                p->winst_block[inst] = block_of(p, t);
                winst_first[inst] = warp0;
                winst_id[inst] = ev[i].addr;
                winst_occ[inst] = occ;
                p->n_winst++;
            } else if (winst_first[inst] != warp0 || winst_id[inst] != ev[i].addr || winst_occ[inst] != occ) {
                /* 64-bit hash collision between two different instances: not expected */
                hmap_free(&wmap); free(winst_first); free(bad_arrival); free(winst_id); free(winst_occ);
                return ORC_ENOMEM;
            }
            p->wbar_inst[i] = inst;
        }
    }
    free(winst_id);
    free(winst_occ);
    hmap_free(&wmap);
    free(winst_first);
    /* instance mask = mask of its earliest arrival; arrivals are processed in trace order */
    {
        uint8_t *seen = (uint8_t *)calloc(p->n_winst ? p->n_winst : 1, 1);
        if (!seen) { free(bad_arrival); return ORC_ENOMEM; }
        for (uint64_t i = 0; i < n; i++) {
            if (kind_of(&ev[i]) != K_WBAR) continue;
            uint32_t inst = p->wbar_inst[i], lane = (ev[i].tid % tpb) % warp_size;
            if (!seen[inst]) { seen[inst] = 1; p->winst_mask[inst] = ev[i].aux; }
            if (!((ev[i].aux >> lane) & 1u) || ev[i].aux != p->winst_mask[inst]) bad_arrival[i] = 1;
            p->winst_arrived[inst] |= 1u << lane;
            p->winst_last[inst] = (uint32_t)i;
        }
        free(seen);
    }

    /* barrier discipline: smallest event that runs ahead of an unfinished barrier */
    uint64_t first_bad = UINT64_MAX;
    for (uint32_t t = 0; t < T; t++) {
        uint32_t s = p->po_start[t], e = p->po_start[t + 1];
        uint32_t b = t / tpb, last_w = UINT32_MAX;
        for (uint32_t j = s; j < e; j++) {
            uint32_t i = p->po_idx[j];
            int off = bad_arrival[i];
            uint32_t ph = p->phase[i];
            if (ph >= 1) { /* block instance ph must be complete before i */
                uint32_t slot = p->bar_off[b] + ph - 1;
                if (p->bar_cnt[slot] != p->n_active[b] || p->bar_last[slot] > i) off = 1;
            }
            if (last_w != UINT32_MAX) { /* the thread's latest warp barrier must be complete */
                uint32_t inst = p->wbar_inst[last_w];
                if (p->winst_arrived[inst] != p->winst_mask[inst] || p->winst_last[inst] > i) off = 1;
            }
            if (off && i < first_bad) first_bad = i;
            if (kind_of(&ev[i]) == K_WBAR) last_w = i;
        }
    }
    free(bad_arrival);
    if (first_bad != UINT64_MAX) { *bad = first_bad; return ORC_ETRACE; }
    return ORC_OK;
}

/* Scope rules.  overlap(): two atomics do not race (Section 4, Section 5.1).  sync_edge(): a
 * release in block br with scope sr reaches an acquire in block bq with scope sq (rule (iv)). */
static int g_inclusive = 0;

static inline int scopes_cover(unsigned sa, uint32_t ba, unsigned sb, uint32_t bb) {
    if (g_inclusive) return (sa != S_BLOCK && sb != S_BLOCK) || ba == bb;
    return sa != S_BLOCK || sb != S_BLOCK || ba == bb;
}

static inline int conflict(const prep_t *p, uint32_t i, uint32_t j) {
    const orc_event *a = &p->ev[i], *b = &p->ev[j];
    unsigned ka = kind_of(a), kb = kind_of(b);
    if (!is_access(ka) || !is_access(kb)) return 0;
    if (a->tid == b->tid) return 0;
    if (loc_key(p, a) != loc_key(p, b)) return 0;
    if (!is_writeish(ka) && !is_writeish(kb)) return 0;
    if (is_atomic(ka) && is_atomic(kb) &&
        scopes_cover(scope_of(a), block_of(p, a->tid), scope_of(b), block_of(p, b->tid)))
        return 0;
    return 1;
}

/* ================================================================ brute-force closure */

int orc_bruteforce(uint32_t n_blocks, uint32_t tpb, uint32_t warp_size, const orc_event *ev,
                   uint64_t n, int inclusive, uint64_t *bad, orc_pairs *out) {
    memset(out, 0, sizeof(*out));
    *bad = UINT64_MAX;
    if (!grid_ok(n_blocks, tpb, &warp_size, n)) return ORC_EINVAL;
    if (n > 16384) return ORC_EINVAL; /* quadratic memory: tiny traces only */
    g_inclusive = inclusive;
    prep_t p;
    int rc = prepare(&p, n_blocks, tpb, warp_size, ev, n, bad);
    if (rc != ORC_OK) { prep_free(&p); return rc; }

    uint64_t W = (n + 63) / 64;
    uint64_t *reach = (uint64_t *)calloc(n * W + 1, sizeof(uint64_t)); /* reach[j]: events i ->* j */
    if (!reach) { prep_free(&p); return ORC_ENOMEM; }

#define SETBIT(row, i) (reach[(uint64_t)(row) * W + ((i) >> 6)] |= (uint64_t)1 << ((i) & 63))
#define OR_ROW(dst, src)                                                                         \
    do {                                                                                         \
        for (uint64_t w_ = 0; w_ < W; w_++) reach[(uint64_t)(dst) * W + w_] |= reach[(uint64_t)(src) * W + w_]; \
        SETBIT(dst, src);                                                                        \
    } while (0)

    for (uint64_t jj = 0; jj < n; jj++) {
        uint32_t j = (uint32_t)jj, t = ev[j].tid, pos = p.po_pos[j];
        if (pos == 0) continue;
        uint32_t pr = p.po_idx[p.po_start[t] + pos - 1]; /* program-order predecessor */
        OR_ROW(j, pr);                                      /* (i) program order */
        unsigned kp = kind_of(&ev[pr]);
        if (kp == K_BAR) { /* (iii) every participant's matching BAR reaches j */
            uint32_t b = t / tpb, ph = p.phase[pr];
            for (uint32_t u = b * tpb; u < (b + 1) * tpb; u++) {
                for (uint32_t q = p.po_start[u]; q < p.po_start[u + 1]; q++) {
                    uint32_t i = p.po_idx[q];
                    if (kind_of(&ev[i]) == K_BAR && p.phase[i] == ph && i != pr) OR_ROW(j, i);
                }
            }
        }
        if (kp == K_WBAR) { /* (iii) warp barrier: every participant's WBAR of the instance */
            uint32_t inst = p.wbar_inst[pr];
            for (uint64_t i = 0; i < j; i++)
                if (kind_of(&ev[i]) == K_WBAR && p.wbar_inst[i] == inst && i != pr) OR_ROW(j, i);
        }
        if (p.acq_scope[pr] != 0xff) { /* (iv) earlier releases on the same variable */
            uint64_t lq = loc_key(&p, &ev[pr]);
            for (uint64_t i = 0; i < pr; i++) {
                if (p.rel_scope[i] == 0xff || loc_key(&p, &ev[i]) != lq) continue;
                if (!scopes_cover(p.rel_scope[i], block_of(&p, ev[i].tid), p.acq_scope[pr],
                                  block_of(&p, ev[pr].tid)))
                    continue;
                OR_ROW(j, i);
            }
        }
    }
#undef OR_ROW
    for (uint64_t jj = 0; jj < n; jj++) {
        uint32_t j = (uint32_t)jj;
        if (!is_access(kind_of(&ev[j]))) continue;
        for (uint32_t i = 0; i < j; i++) {
            if (!conflict(&p, i, j)) continue;
            if ((reach[(uint64_t)j * W + (i >> 6)] >> (i & 63)) & 1) continue;
            if (pairs_push(out, i, j) != ORC_OK) { free(reach); prep_free(&p); return ORC_ENOMEM; }
        }
    }
#undef SETBIT
    free(reach);
    prep_free(&p);
    /* pairs were produced in (second, first) order; put them in canonical (first, second) order */
    qsort(out->data, out->n, 2 * sizeof(uint32_t), cmp_pair);
    return ORC_OK;
}

/* ================================================================ vector-clock detector */

/* ---- clock store, mode 0: block floors + per-thread exceptions (immutable, shared) ---- */
typedef struct {
    uint32_t nb, nt;
    uint32_t *b_id, *b_val; /* sorted by block: every thread of the block has at least b_val */
    uint32_t *t_id, *t_val; /* sorted by tid: per-thread values above the block's floor */
} cvc;

typedef struct arena_blk { struct arena_blk *next; size_t used, cap; } arena_blk;
typedef struct { arena_blk *head; } arena;

static void *arena_alloc(arena *a, size_t bytes) {
    bytes = (bytes + 15) & ~(size_t)15;
    if (!a->head || a->head->used + bytes > a->head->cap) {
        size_t cap = bytes > ((size_t)1 << 24) ? bytes : ((size_t)1 << 24);
        arena_blk *b = (arena_blk *)malloc(sizeof(arena_blk) + cap + 16);
        if (!b) return NULL;
        b->next = a->head; b->used = 0; b->cap = cap;
        a->head = b;
    }
    void *r = (char *)(a->head + 1) + a->head->used;
    a->head->used += bytes;
    return r;
}
static void arena_free(arena *a) {
    while (a->head) { arena_blk *n = a->head->next; free(a->head); a->head = n; }
}

static cvc *cvc_new(arena *a, uint32_t nb, uint32_t nt) {
    cvc *c = (cvc *)arena_alloc(a, sizeof(cvc) + (size_t)(2 * nb + 2 * nt) * sizeof(uint32_t));
    if (!c) return NULL;
    uint32_t *d = (uint32_t *)(c + 1);
    c->nb = nb; c->nt = nt;
    c->b_id = d; c->b_val = d + nb; c->t_id = d + 2 * nb; c->t_val = d + 2 * nb + nt;
    return c;
}

static uint32_t cvc_floor(const cvc *c, uint32_t blk) {
    uint32_t lo = 0, hi = c->nb;
    while (lo < hi) { uint32_t m = (lo + hi) / 2; if (c->b_id[m] < blk) lo = m + 1; else hi = m; }
    return (lo < c->nb && c->b_id[lo] == blk) ? c->b_val[lo] : 0;
}
static uint32_t cvc_get(const cvc *c, uint32_t tid, uint32_t tpb) {
    uint32_t f = cvc_floor(c, tid / tpb);
    uint32_t lo = 0, hi = c->nt;
    while (lo < hi) { uint32_t m = (lo + hi) / 2; if (c->t_id[m] < tid) lo = m + 1; else hi = m; }
    uint32_t e = (lo < c->nt && c->t_id[lo] == tid) ? c->t_val[lo] : 0;
    return e > f ? e : f;
}

/* join of x and y; extra_t/extra_v: one more exception (or UINT32_MAX); fb/fv: one more floor. */
static cvc *cvc_join(arena *a, const cvc *x, const cvc *y, uint32_t extra_t, uint32_t extra_v,
                     uint32_t fb, uint32_t fv, uint32_t tpb) {
    static const cvc empty = {0, 0, NULL, NULL, NULL, NULL};
    if (!x) x = &empty;
    if (!y) y = &empty;
    uint32_t nb = x->nb + y->nb + 1, nt = x->nt + y->nt + 1;
    cvc *r = cvc_new(a, nb, nt);
    if (!r) return NULL;
    /* floors: merge */
    uint32_t i = 0, j = 0, k = 0;
    while (i < x->nb || j < y->nb) {
        uint32_t bi = i < x->nb ? x->b_id[i] : UINT32_MAX, bj = j < y->nb ? y->b_id[j] : UINT32_MAX;
        uint32_t id = bi < bj ? bi : bj, v = 0;
        if (bi == id) { v = x->b_val[i]; i++; }
        if (bj == id && y->b_val[j] > v) v = y->b_val[j];
        if (bj == id) j++;
        r->b_id[k] = id; r->b_val[k] = v; k++;
    }
    if (fb != UINT32_MAX) { /* insert / raise one floor */
        uint32_t pos = 0;
        while (pos < k && r->b_id[pos] < fb) pos++;
        if (pos < k && r->b_id[pos] == fb) { if (fv > r->b_val[pos]) r->b_val[pos] = fv; }
        else {
            memmove(&r->b_id[pos + 1], &r->b_id[pos], (k - pos) * sizeof(uint32_t));
            memmove(&r->b_val[pos + 1], &r->b_val[pos], (k - pos) * sizeof(uint32_t));
            r->b_id[pos] = fb; r->b_val[pos] = fv; k++;
        }
    }
    r->nb = k;
    /* exceptions: merge, keeping only values above the (new) floor of the thread's block */
    i = j = 0;
    uint32_t m = 0;
    int extra_done = (extra_t == UINT32_MAX);
    while (i < x->nt || j < y->nt || !extra_done) {
        uint32_t ti = i < x->nt ? x->t_id[i] : UINT32_MAX, tj = j < y->nt ? y->t_id[j] : UINT32_MAX;
        uint32_t te = extra_done ? UINT32_MAX : extra_t;
        uint32_t id = ti < tj ? ti : tj;
        if (te < id) id = te;
        uint32_t v = 0;
        if (ti == id) { v = x->t_val[i]; i++; }
        if (tj == id) { if (y->t_val[j] > v) v = y->t_val[j]; j++; }
        if (te == id) { if (extra_v > v) v = extra_v; extra_done = 1; }
        if (v > cvc_floor(r, id / tpb)) { r->t_id[m] = id; r->t_val[m] = v; m++; }
    }
    r->nt = m;
    return r;
}

/* ---- detector state ---- */

typedef struct { uint32_t idx, tid, epoch, flags; } hist_t; /* flags: bit0 write, bit1 atomic, bits2-3 scope */

enum { L_READ = 0, L_WRITE = 1, L_ADEV = 2, L_ABLK = 3, NLISTS = 4 };

static inline int list_of(unsigned k, unsigned scope) {
    if (k == K_READ) return L_READ;
    if (k == K_WRITE) return L_WRITE;
    return scope == S_BLOCK ? L_ABLK : L_ADEV;
}

typedef struct {
    int dense;
    uint32_t T, tpb;
    arena ar;
    /* per-thread clocks */
    uint32_t *c;       /* own clock c_t (mode 0) */
    const cvc **vc;    /* H_t without the own entry (mode 0) */
    uint32_t *dvc;     /* dense H_t, T x T, own entry included (mode 1) */
} clocks_t;

static inline uint32_t H_get(const clocks_t *C, uint32_t t, uint32_t u) {
    if (C->dense) return C->dvc[(uint64_t)t * C->T + u];
    if (t == u) return C->c[t];
    return C->vc[t] ? cvc_get(C->vc[t], u, C->tpb) : 0;
}

/* A sync-variable clock H_<l,s>: per location, one for its device/system-scoped releases
 * (Algorithm 1's H_<l,DEVICE>) and one per block for block-scoped releases (H_<l,b>).  Under the
 * inclusive reading the device-scoped ones are kept per releasing block as well, since there an
 * acquire is reached only by releases whose scope covers its block. */
typedef struct {
    uint32_t blk;       /* block of the releasing threads; UINT32_MAX: device-scoped releases of
                         * every block (default reading) */
    uint32_t blk_scope; /* 1: block-scoped releases, 0: device/system-scoped releases */
    const cvc *v;       /* mode 0 */
    uint32_t *d;        /* mode 1 */
} syncvar;

int orc_check(uint32_t n_blocks, uint32_t tpb, uint32_t warp_size, const orc_event *ev, uint64_t n,
              int dense, int inclusive, uint64_t *bad, orc_pairs *out) {
    memset(out, 0, sizeof(*out));
    *bad = UINT64_MAX;
    if (!grid_ok(n_blocks, tpb, &warp_size, n)) return ORC_EINVAL;
    uint64_t T64 = (uint64_t)n_blocks * tpb;
    if (dense && T64 * T64 > ((uint64_t)1 << 28)) return ORC_EINVAL; /* dense clocks: <= 16K threads */
    g_inclusive = inclusive;
    prep_t p;
    int rc = prepare(&p, n_blocks, tpb, warp_size, ev, n, bad);
    if (rc != ORC_OK) { prep_free(&p); return rc; }
    uint32_t T = p.n_threads;

    /* ---- locations and their access histories (count first, then fill in trace order) ---- */
    uint64_t n_acc = 0;
    for (uint64_t i = 0; i < n; i++) if (is_access(kind_of(&ev[i]))) n_acc++;
    hmap lmap;
    uint32_t *loc = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    if (hmap_init(&lmap, n_acc) != ORC_OK || !loc) { prep_free(&p); free(loc); return ORC_ENOMEM; }
    uint32_t L = 0;
    for (uint64_t i = 0; i < n; i++) {
        loc[i] = UINT32_MAX;
        if (!is_access(kind_of(&ev[i]))) continue;
        int ins;
        loc[i] = hmap_get(&lmap, loc_key(&p, &ev[i]), L, &ins);
        if (ins) L++;
    }
    uint64_t *hoff = (uint64_t *)calloc((uint64_t)L * NLISTS + 1, sizeof(uint64_t));
    uint64_t *hfill = (uint64_t *)malloc(((uint64_t)L * NLISTS + 1) * sizeof(uint64_t));
    hist_t *hist = (hist_t *)malloc((n_acc ? n_acc : 1) * sizeof(hist_t));
    uint64_t *loc_keys = (uint64_t *)malloc((L ? L : 1) * sizeof(uint64_t));
    if (!hoff || !hfill || !hist || !loc_keys) rc = ORC_ENOMEM;
    if (rc == ORC_OK) {
        for (uint64_t i = 0; i < n; i++) {
            if (loc[i] == UINT32_MAX) continue;
            hoff[(uint64_t)loc[i] * NLISTS + list_of(kind_of(&ev[i]), scope_of(&ev[i])) + 1]++;
            loc_keys[loc[i]] = loc_key(&p, &ev[i]);
        }
        for (uint64_t s = 0; s < (uint64_t)L * NLISTS; s++) hoff[s + 1] += hoff[s];
        memcpy(hfill, hoff, ((uint64_t)L * NLISTS + 1) * sizeof(uint64_t));
    }

    /* ---- clocks ---- */
    clocks_t C;
    memset(&C, 0, sizeof(C));
    C.dense = dense; C.T = T; C.tpb = tpb;
    if (rc == ORC_OK) {
        if (dense) {
            C.dvc = (uint32_t *)calloc((size_t)T * T + 1, sizeof(uint32_t));
            if (!C.dvc) rc = ORC_ENOMEM;
            else for (uint32_t t = 0; t < T; t++) C.dvc[(uint64_t)t * T + t] = 1;
        } else {
            C.c = (uint32_t *)malloc((T ? T : 1) * sizeof(uint32_t));
            C.vc = (const cvc **)calloc(T ? T : 1, sizeof(cvc *));
            if (!C.c || !C.vc) rc = ORC_ENOMEM;
            else for (uint32_t t = 0; t < T; t++) C.c[t] = 1;
        }
    }

    /* sync-variable clocks: per location, a small list of syncvars */
    syncvar **loc_sv = NULL;
    uint32_t *loc_nsv = NULL, *loc_svcap = NULL;
    if (rc == ORC_OK) {
        loc_sv = (syncvar **)calloc(L ? L : 1, sizeof(syncvar *));
        loc_nsv = (uint32_t *)calloc(L ? L : 1, sizeof(uint32_t));
        loc_svcap = (uint32_t *)calloc(L ? L : 1, sizeof(uint32_t));
        if (!loc_sv || !loc_nsv || !loc_svcap) rc = ORC_ENOMEM;
    }

    /* barrier bookkeeping: per block instance, per warp instance, the arrived participants */
    uint32_t *bar_arr = NULL; /* participants of instances, by arrival; CSR by instance */
    uint32_t *bar_arr_n = NULL;
    uint32_t *bar_arr_off = NULL;
    uint32_t *wbar_arr_n = NULL;
    uint32_t *wbar_arr = NULL; /* up to 32 per instance */
    if (rc == ORC_OK) {
        uint32_t n_inst = p.bar_off[n_blocks];
        bar_arr_off = (uint32_t *)calloc((size_t)n_inst + 1, sizeof(uint32_t));
        bar_arr_n = (uint32_t *)calloc(n_inst ? n_inst : 1, sizeof(uint32_t));
        if (!bar_arr_off || !bar_arr_n) rc = ORC_ENOMEM;
        else {
            for (uint32_t s = 0; s < n_inst; s++) bar_arr_off[s + 1] = bar_arr_off[s] + p.bar_cnt[s];
            bar_arr = (uint32_t *)malloc(((size_t)bar_arr_off[n_inst] + 1) * sizeof(uint32_t));
            wbar_arr_n = (uint32_t *)calloc(p.n_winst ? p.n_winst : 1, sizeof(uint32_t));
            wbar_arr = (uint32_t *)malloc(((size_t)p.n_winst * 32 + 1) * sizeof(uint32_t));
            if (!bar_arr || !wbar_arr_n || !wbar_arr) rc = ORC_ENOMEM;
        }
    }

    /* ---- the per-event pass, in trace order ---- */
    for (uint64_t ii = 0; ii < n && rc == ORC_OK; ii++) {
        uint32_t i = (uint32_t)ii, t = ev[i].tid, bt = t / tpb;
        unsigned k = kind_of(&ev[i]);

        if (is_access(k)) {
            /* check against earlier accesses of the location that may conflict with this one */
            uint32_t X = loc[i];
            unsigned sc = scope_of(&ev[i]);
            for (int li = 0; li < NLISTS; li++) {
                if (k == K_READ && li == L_READ) continue; /* read/read never conflicts */
                uint64_t s = hoff[(uint64_t)X * NLISTS + li], e = hfill[(uint64_t)X * NLISTS + li];
                for (uint64_t q = s; q < e; q++) {
                    const hist_t *a = &hist[q];
                    if (a->tid == t) continue;
                    if (!conflict(&p, a->idx, i)) continue;
                    if (a->epoch <= H_get(&C, t, a->tid)) continue; /* a happens before i */
                    if (pairs_push(out, a->idx, i) != ORC_OK) { rc = ORC_ENOMEM; break; }
                }
            }
            /* record this access */
            int li = list_of(k, sc);
            hist_t *h = &hist[hfill[(uint64_t)X * NLISTS + li]++];
            h->idx = i; h->tid = t; h->epoch = H_get(&C, t, t);
            h->flags = (is_writeish(k) ? 1u : 0u) | (is_atomic(k) ? 2u : 0u) | (sc << 2);
        }
        if (rc != ORC_OK) break;

        if (p.rel_scope[i] != 0xff) {
            /* RELEASE(t, l, s): H_<l,s> := H_<l,s> join H_t; then increment t's own entry */
            uint32_t X = loc[i];
            uint32_t bs = p.rel_scope[i] == S_BLOCK ? 1u : 0u;
            /* Algorithm 1 keeps one clock H_<l,DEVICE> that the device-scoped releases of every
             * block join, and one H_<l,b> per block b for block-scoped releases; the inclusive
             * reading also needs the releasing block of a device-scoped release */
            uint32_t key_blk = (bs || g_inclusive) ? bt : UINT32_MAX;
            syncvar *s = NULL;
            for (uint32_t q = 0; q < loc_nsv[X]; q++)
                if (loc_sv[X][q].blk == key_blk && loc_sv[X][q].blk_scope == bs) s = &loc_sv[X][q];
            if (!s) {
                if (loc_nsv[X] == loc_svcap[X]) {
                    uint32_t nc = loc_svcap[X] ? loc_svcap[X] * 2 : 4;
                    syncvar *nl = (syncvar *)realloc(loc_sv[X], nc * sizeof(syncvar));
                    if (!nl) { rc = ORC_ENOMEM; break; }
                    loc_sv[X] = nl; loc_svcap[X] = nc;
                }
                s = &loc_sv[X][loc_nsv[X]++];
                memset(s, 0, sizeof(*s));
                s->blk = key_blk; s->blk_scope = bs;
                if (dense) {
                    s->d = (uint32_t *)calloc(T, sizeof(uint32_t));
                    if (!s->d) { rc = ORC_ENOMEM; break; }
                }
            }
            if (dense) {
                uint32_t *h = &C.dvc[(uint64_t)t * T];
                for (uint32_t u = 0; u < T; u++) if (h[u] > s->d[u]) s->d[u] = h[u];
                h[t] += 1;
            } else {
                const cvc *nv = cvc_join(&C.ar, s->v, C.vc[t], t, C.c[t], UINT32_MAX, 0, tpb);
                if (!nv) { rc = ORC_ENOMEM; break; }
                s->v = nv;
                C.c[t] += 1;
            }
        }

        if (p.acq_scope[i] != 0xff) {
            /* ACQUIRE(t, l, s): join every clock of l whose releases reach this acquire: device-
             * scoped ones always; block-scoped ones of t's own block; and, for a device-scoped
             * acquire, block-scoped ones of every block (rule (iv) with the default scope reading) */
            uint32_t X = loc[i];
            unsigned s = p.acq_scope[i];
            for (uint32_t q = 0; q < loc_nsv[X]; q++) {
                syncvar *v = &loc_sv[X][q];
                if (!scopes_cover(v->blk_scope ? S_BLOCK : S_DEVICE, v->blk, s, bt)) continue;
                if (dense) {
                    uint32_t *h = &C.dvc[(uint64_t)t * T];
                    for (uint32_t u = 0; u < T; u++) if (v->d[u] > h[u]) h[u] = v->d[u];
                } else {
                    const cvc *nv = cvc_join(&C.ar, C.vc[t], v->v, UINT32_MAX, 0, UINT32_MAX, 0, tpb);
                    if (!nv) { rc = ORC_ENOMEM; break; }
                    C.vc[t] = nv;
                }
            }
            if (rc != ORC_OK) break;
        }

        if (k == K_BAR) {
            /* SYNC(scope = the block's active threads), applied when the last participant arrives */
            uint32_t slot = p.bar_off[bt] + p.phase[i];
            bar_arr[bar_arr_off[slot] + bar_arr_n[slot]++] = t;
            if (bar_arr_n[slot] == p.n_active[bt]) {
                uint32_t *parts = &bar_arr[bar_arr_off[slot]], np = bar_arr_n[slot];
                if (dense) {
                    uint32_t *J = (uint32_t *)calloc(T, sizeof(uint32_t));
                    if (!J) { rc = ORC_ENOMEM; break; }
                    for (uint32_t q = 0; q < np; q++) {
                        uint32_t *h = &C.dvc[(uint64_t)parts[q] * T];
                        for (uint32_t u = 0; u < T; u++) if (h[u] > J[u]) J[u] = h[u];
                    }
                    for (uint32_t q = 0; q < np; q++) {
                        uint32_t *h = &C.dvc[(uint64_t)parts[q] * T];
                        memcpy(h, J, (size_t)T * sizeof(uint32_t));
                        h[parts[q]] += 1; /* each participant increments its own entry */
                    }
                    free(J);
                } else {
                    /* join, then forced compression: every participant's entry becomes the largest
                     * participant clock M (the block floor) and each own clock becomes M + 1 */
                    const cvc *J = NULL;
                    uint32_t M = 0;
                    for (uint32_t q = 0; q < np; q++) {
                        uint32_t u = parts[q];
                        if (C.c[u] > M) M = C.c[u];
                        J = cvc_join(&C.ar, J, C.vc[u], UINT32_MAX, 0, UINT32_MAX, 0, tpb);
                        if (!J) break;
                    }
                    if (!J) { rc = ORC_ENOMEM; break; }
                    J = cvc_join(&C.ar, J, NULL, UINT32_MAX, 0, bt, M, tpb);
                    if (!J) { rc = ORC_ENOMEM; break; }
                    for (uint32_t q = 0; q < np; q++) { C.vc[parts[q]] = J; C.c[parts[q]] = M + 1; }
                }
            }
        }

        if (k == K_WBAR) {
            /* SYNC(scope = the lanes of the mask), applied when the last lane arrives */
            uint32_t inst = p.wbar_inst[i];
            wbar_arr[(uint64_t)inst * 32 + wbar_arr_n[inst]++] = t;
            uint32_t need = (uint32_t)__builtin_popcount(p.winst_mask[inst]);
            if (wbar_arr_n[inst] == need) {
                uint32_t *parts = &wbar_arr[(uint64_t)inst * 32], np = need;
                if (dense) {
                    uint32_t *J = (uint32_t *)calloc(T, sizeof(uint32_t));
                    if (!J) { rc = ORC_ENOMEM; break; }
                    for (uint32_t q = 0; q < np; q++) {
                        uint32_t *h = &C.dvc[(uint64_t)parts[q] * T];
                        for (uint32_t u = 0; u < T; u++) if (h[u] > J[u]) J[u] = h[u];
                    }
                    for (uint32_t q = 0; q < np; q++) {
                        uint32_t *h = &C.dvc[(uint64_t)parts[q] * T];
                        memcpy(h, J, (size_t)T * sizeof(uint32_t));
                        h[parts[q]] += 1;
                    }
                    free(J);
                } else {
                    const cvc *J = NULL;
                    for (uint32_t q = 0; q < np; q++) {
                        uint32_t u = parts[q];
                        J = cvc_join(&C.ar, J, C.vc[u], u, C.c[u], UINT32_MAX, 0, tpb);
                        if (!J) break;
                    }
                    if (!J) { rc = ORC_ENOMEM; break; }
                    for (uint32_t q = 0; q < np; q++) { C.vc[parts[q]] = J; C.c[parts[q]] += 1; }
                }
            }
        }
        /* FENCE: no effect of its own; it only marks neighbouring atomics (see prepare) */
    }

    /* ---- cleanup ---- */
    if (loc_sv) {
        for (uint32_t x = 0; x < L; x++) {
            if (dense) for (uint32_t q = 0; q < loc_nsv[x]; q++) free(loc_sv[x][q].d);
            free(loc_sv[x]);
        }
    }
    free(loc_sv); free(loc_nsv); free(loc_svcap);
    free(bar_arr); free(bar_arr_n); free(bar_arr_off); free(wbar_arr_n); free(wbar_arr);
    free(C.dvc); free(C.c); free((void *)C.vc);
    arena_free(&C.ar);
    free(hoff); free(hfill); free(hist); free(loc_keys); free(loc);
    hmap_free(&lmap);
    prep_free(&p);
    if (rc != ORC_OK) { orc_pairs_free(out); return rc; }
    qsort(out->data, out->n, 2 * sizeof(uint32_t), cmp_pair);
    return ORC_OK;
}

/* Validation only: returns ORC_OK, ORC_EINVAL, or ORC_ETRACE with the first offending index. */
int orc_validate(uint32_t n_blocks, uint32_t tpb, uint32_t warp_size, const orc_event *ev,
                 uint64_t n, uint64_t *bad) {
    *bad = UINT64_MAX;
    if (!grid_ok(n_blocks, tpb, &warp_size, n)) return ORC_EINVAL;
    prep_t p;
    int rc = prepare(&p, n_blocks, tpb, warp_size, ev, n, bad);
    prep_free(&p);
    return rc;
}
