/*
 * rd_oracle.c -- CPU oracle for scoped happens-before race checking over a recorded GPU trace.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product path (the HIP checker) never calls it, and the two
 * share no code: this file has its own record decoder, its own validation and its own analysis.
 *
 * It computes the scoped happens-before report two independent ways, and the GWCP report of
 * Section 4 two ways (at the end of this file):
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
/* Doubles the table when it is half full (keys keep their values). */
static void hmap_grow(hmap *h) {
    if (2 * (h->n + 1) + 16 <= h->cap) return;
    uint64_t nc = h->cap * 2;
    uint64_t *nk = (uint64_t *)malloc(nc * sizeof(uint64_t));
    uint32_t *nv = (uint32_t *)calloc(nc, sizeof(uint32_t));
    if (!nk || !nv) { free(nk); free(nv); return; } /* stays full: callers size generously */
    for (uint64_t j = 0; j < h->cap; j++) {
        if (!h->vals[j]) continue;
        uint64_t q = mix64(h->keys[j]) & (nc - 1);
        while (nv[q]) q = (q + 1) & (nc - 1);
        nk[q] = h->keys[j];
        nv[q] = h->vals[j];
    }
    free(h->keys); free(h->vals);
    h->keys = nk; h->vals = nv; h->cap = nc;
}

/* Returns the index for key, inserting next_index if absent (and setting *inserted). */
static uint32_t hmap_get(hmap *h, uint64_t key, uint32_t next_index, int *inserted) {
    hmap_grow(h);
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

/* Whether key is in the map. */
static int hmap_has(const hmap *h, uint64_t key) {
    uint64_t m = h->cap - 1, s = mix64(key) & m;
    while (h->vals[s]) {
        if (h->keys[s] == key) return 1;
        s = (s + 1) & m;
    }
    return 0;
}
/* Removes key (linear probing: the rest of its cluster is inserted again). */
static void hmap_unget(hmap *h, uint64_t key) {
    uint64_t m = h->cap - 1, s = mix64(key) & m;
    while (h->vals[s] && h->keys[s] != key) s = (s + 1) & m;
    if (!h->vals[s]) return;
    h->vals[s] = 0;
    h->n--;
    for (uint64_t j = (s + 1) & m; h->vals[j]; j = (j + 1) & m) {
        uint64_t k = h->keys[j];
        uint32_t v = h->vals[j];
        h->vals[j] = 0;
        h->n--;
        uint64_t q = mix64(k) & m;
        while (h->vals[q]) q = (q + 1) & m;
        h->keys[q] = k;
        h->vals[q] = v;
        h->n++;
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

/* The scoped happens-before graph of a prepared trace closed transitively, as bitsets:
 * reach[j * W + ...] holds every event i with a path i ->+ j (W = ceil(n / 64) words per row).
 * Edges: program order (rule (i)); every participant's barrier arrival to each participant's next
 * event (rule (iii)); a release to the event after an acquire of the same variable that its scope
 * reaches (rule (iv)).  Trace order is a topological order, so one pass suffices. */
static uint64_t *hb_reach(const prep_t *p0) {
    uint64_t n = p0->n, W = (n + 63) / 64;
    const orc_event *ev = p0->ev;
    const prep_t p = *p0;
    uint32_t tpb = p.tpb;
    uint64_t *reach = (uint64_t *)calloc(n * W + 1, sizeof(uint64_t)); /* reach[j]: events i ->* j */
    if (!reach) return NULL;

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
#undef SETBIT
    return reach;
}


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
    uint64_t *reach = hb_reach(&p);
    if (!reach) { prep_free(&p); return ORC_ENOMEM; }
    for (uint64_t jj = 0; jj < n; jj++) {
        uint32_t j = (uint32_t)jj;
        if (!is_access(kind_of(&ev[j]))) continue;
        for (uint32_t i = 0; i < j; i++) {
            if (!conflict(&p, i, j)) continue;
            if ((reach[(uint64_t)j * W + (i >> 6)] >> (i & 63)) & 1) continue;
            if (pairs_push(out, i, j) != ORC_OK) { free(reach); prep_free(&p); return ORC_ENOMEM; }
        }
    }
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

/* ================================================================ GWCP (Section 4)
 *
 * The predictive relation of Section 4: weak causal precedence for GPUs.  Two computations:
 *
 *   orc_gwcp             Algorithms 1 and 2 (Section 4.1) step by step, with dense vector clocks:
 *                        per-thread local time N_t and clocks P_t (GWCP) and H_t (scoped HB), the
 *                        logical time C_t = P_t{t := N_t}; per-lock clocks P_<l,s>, H_<l,s>;
 *                        per-(lock, location) clocks L^r and L^w; per-thread locksets with the read
 *                        and write sets of each held critical section; Acq_l / Rel_l queues.  An
 *                        access by t of an earlier access a of thread u != t races when they
 *                        conflict and a's local time is above C_t[u] (= P_t[u]).
 *
 *   orc_gwcp_bruteforce  The definition: rules (i)-(iv) as a least fixpoint over event pairs with
 *                        bitsets (tiny traces only), every conflicting pair it leaves unordered.
 *
 * Readings (each also listed in the design notes):
 *   G1 critical sections: a thread's acquire of a lock word it does not hold opens one (held with
 *      the acquire's scope); the thread's next release of that word closes it.  An acquire of a
 *      word already held opens nothing; a release of a word not held (a flag publication) closes
 *      nothing; both keep their happens-before role (rule (iv)), and the P clock flows along every
 *      release -> acquire edge as Algorithm 1 publishes and joins P_<l,s> for every release and
 *      acquire.
 *   G2 acquires and releases are lock operations, not reads or writes of critical sections
 *      (Algorithm 2 runs for reads and writes); the race report still checks them as atomic
 *      accesses of their word.  Atomics that are not lock operations are writes.
 *   G3 rule (i)'s "conflicting" is the memory conflict of two accesses (same location, at least one
 *      write), whatever their threads, as Algorithm 2 joins every earlier critical section's
 *      L^r / L^w; the race report is over pairs of different threads.
 *   G4 scopes: a lock held or released with device/system scope has key DEVICE, with block scope
 *      the key of the thread's block; two keys overlap when either is DEVICE or they are equal
 *      (Section 4, "scoped locks").  The queue join of Algorithm 1's RELEASE uses that overlap
 *      between the dequeued release and the current one; Algorithm 2's joins and ACQUIRE's joins
 *      are those printed (which are the same overlap).
 *   G5 queues hold other threads' critical sections (Algorithm 1 enqueues for t' != t), paired
 *      acquire with release of the same critical section; one whose release has not happened yet
 *      stays at the front.  Rule (ii) is read for critical sections of different threads.
 *   G6 lock clocks are joined, not overwritten, on release (as H_<l,s> in the detector above).
 * The definition and the algorithm agree on traces whose synchronisation is locks (the WCP
 * setting); with barriers the algorithm's SYNC joins only C_t, so it orders less than rule (iii)
 * composed with happens-before (rule (iv)) on the left: its report contains the definition's.
 */

#define KEY_DEV UINT32_MAX
static inline uint32_t scope_key(unsigned scope, uint32_t blk) { return scope == S_BLOCK ? blk : KEY_DEV; }
static inline int keys_overlap(uint32_t a, uint32_t b) { return a == KEY_DEV || b == KEY_DEV || a == b; }
static inline int is_lockop(const prep_t *p, uint32_t i) { return p->rel_scope[i] != 0xff || p->acq_scope[i] != 0xff; }

typedef struct {
    uint32_t tid, acq, rel;    /* events; rel = UINT32_MAX while open */
    uint64_t word;             /* the lock word */
    uint32_t acq_key, rel_key; /* scope keys */
} orc_cs;

typedef struct {
    uint32_t n_cs;
    orc_cs *cs;                /* in order of their acquires (trace order) */
    uint32_t *open_cs;         /* per event: the critical section an acquire opens, or UINT32_MAX */
    uint32_t *close_cs;        /* per event: the critical section a release closes, or UINT32_MAX */
} cs_info;

static void cs_free(cs_info *c) { free(c->cs); free(c->open_cs); free(c->close_cs); memset(c, 0, sizeof(*c)); }

/* Critical sections (reading G1), numbered in trace order of their acquires. */
static int cs_build(const prep_t *p, cs_info *c) {
    memset(c, 0, sizeof(*c));
    uint64_t n = p->n;
    c->open_cs = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    c->close_cs = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t n_acq = 0;
    for (uint64_t i = 0; i < n; i++) n_acq += p->acq_scope[i] != 0xff;
    c->cs = (orc_cs *)malloc((n_acq ? n_acq : 1) * sizeof(orc_cs));
    uint32_t *held = (uint32_t *)malloc((n_acq ? n_acq : 1) * sizeof(uint32_t)); /* open ones, per thread */
    uint32_t *held_n = (uint32_t *)calloc(p->n_threads ? p->n_threads : 1, sizeof(uint32_t));
    uint32_t *held_off = (uint32_t *)malloc(((size_t)p->n_threads + 1) * sizeof(uint32_t));
    if (!c->open_cs || !c->close_cs || !c->cs || !held || !held_n || !held_off) {
        free(held); free(held_n); free(held_off); cs_free(c);
        return ORC_ENOMEM;
    }
    /* room for each thread's open sections: at most its acquires */
    held_off[0] = 0;
    for (uint32_t t = 0; t < p->n_threads; t++) {
        uint32_t a = 0;
        for (uint32_t q = p->po_start[t]; q < p->po_start[t + 1]; q++) a += p->acq_scope[p->po_idx[q]] != 0xff;
        held_off[t + 1] = held_off[t] + a;
    }
    for (uint64_t ii = 0; ii < n; ii++) {
        uint32_t i = (uint32_t)ii, t = p->ev[i].tid, b = block_of(p, t);
        c->open_cs[i] = c->close_cs[i] = UINT32_MAX;
        uint64_t w = loc_key(p, &p->ev[i]);
        uint32_t *h = &held[held_off[t]];
        if (p->rel_scope[i] != 0xff) {
            for (uint32_t q = held_n[t]; q-- > 0;) {
                orc_cs *x = &c->cs[h[q]];
                if (x->word != w) continue;
                x->rel = i;
                x->rel_key = scope_key(p->rel_scope[i], b);
                c->close_cs[i] = h[q];
                memmove(&h[q], &h[q + 1], (held_n[t] - q - 1) * sizeof(uint32_t));
                held_n[t]--;
                break;
            }
        }
        if (p->acq_scope[i] != 0xff) {
            int holding = 0;
            for (uint32_t q = 0; q < held_n[t]; q++) holding |= c->cs[h[q]].word == w;
            if (!holding) {
                orc_cs *x = &c->cs[c->n_cs];
                x->tid = t; x->acq = i; x->rel = UINT32_MAX; x->word = w;
                x->acq_key = scope_key(p->acq_scope[i], b); x->rel_key = x->acq_key;
                c->open_cs[i] = c->n_cs;
                h[held_n[t]++] = c->n_cs++;
            }
        }
    }
    free(held); free(held_n); free(held_off);
    return ORC_OK;
}

/* ---- growable arrays of dense clocks ---- */
typedef struct { uint32_t **v; uint64_t n, cap; uint32_t T; } vecs;
static uint32_t vecs_new(vecs *a) {
    if (a->n == a->cap) {
        uint64_t nc = a->cap ? 2 * a->cap : 64;
        uint32_t **nv = (uint32_t **)realloc(a->v, nc * sizeof(uint32_t *));
        if (!nv) return UINT32_MAX;
        a->v = nv; a->cap = nc;
    }
    a->v[a->n] = (uint32_t *)calloc(a->T ? a->T : 1, sizeof(uint32_t));
    if (!a->v[a->n]) return UINT32_MAX;
    return (uint32_t)a->n++;
}
static void vecs_free(vecs *a) { for (uint64_t i = 0; i < a->n; i++) free(a->v[i]); free(a->v); memset(a, 0, sizeof(*a)); }
static inline void vjoin(uint32_t *d, const uint32_t *s, uint32_t T) { for (uint32_t u = 0; u < T; u++) if (s[u] > d[u]) d[u] = s[u]; }

/* growable u32 list */
typedef struct { uint32_t *v; uint32_t n, cap; } ulist;
static int ulist_push(ulist *l, uint32_t x) {
    if (l->n == l->cap) {
        uint32_t nc = l->cap ? 2 * l->cap : 8;
        uint32_t *nv = (uint32_t *)realloc(l->v, nc * sizeof(uint32_t));
        if (!nv) return ORC_ENOMEM;
        l->v = nv; l->cap = nc;
    }
    l->v[l->n++] = x;
    return ORC_OK;
}

int orc_gwcp(uint32_t n_blocks, uint32_t tpb, uint32_t warp_size, const orc_event *ev, uint64_t n,
             uint64_t *bad, orc_pairs *out) {
    memset(out, 0, sizeof(*out));
    *bad = UINT64_MAX;
    if (!grid_ok(n_blocks, tpb, &warp_size, n)) return ORC_EINVAL;
    uint64_t T64 = (uint64_t)n_blocks * tpb;
    if (T64 > 8192) return ORC_EINVAL; /* dense clocks */
    g_inclusive = 0;
    prep_t p;
    int rc = prepare(&p, n_blocks, tpb, warp_size, ev, n, bad);
    if (rc != ORC_OK) { prep_free(&p); return rc; }
    cs_info C;
    rc = cs_build(&p, &C);
    if (rc != ORC_OK) { prep_free(&p); return rc; }
    const uint32_t T = p.n_threads;

    /* locations (dense ids) and their access histories in trace order */
    hmap lmap = {0}, lkmap = {0}, wmap = {0}, lwmap = {0}, curmap = {0}, joinmap = {0};
    uint32_t *loc = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *epoch = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    if (hmap_init(&lmap, n) != ORC_OK || !loc || !epoch) { rc = ORC_ENOMEM; }
    uint32_t L = 0;
    for (uint64_t i = 0; i < n && rc == ORC_OK; i++) {
        int ins;
        loc[i] = is_access(kind_of(&ev[i])) ? hmap_get(&lmap, loc_key(&p, &ev[i]), L, &ins) : UINT32_MAX;
        if (loc[i] != UINT32_MAX && ins) L++;
    }
    ulist *hist = (ulist *)calloc(L ? L : 1, sizeof(ulist));

    /* clocks */
    uint32_t *N = (uint32_t *)malloc((T ? T : 1) * sizeof(uint32_t));
    uint32_t *P = (uint32_t *)calloc((size_t)T * T + 1, sizeof(uint32_t));
    uint32_t *H = (uint32_t *)calloc((size_t)T * T + 1, sizeof(uint32_t));
    uint32_t *J = (uint32_t *)malloc(((size_t)T + 1) * sizeof(uint32_t));
    uint32_t *JH = (uint32_t *)malloc(((size_t)T + 1) * sizeof(uint32_t));
    if (!hist || !N || !P || !H || !J || !JH) rc = ORC_ENOMEM;
    for (uint32_t t = 0; t < T && rc == ORC_OK; t++) { N[t] = 1; H[(uint64_t)t * T + t] = 1; }

    /* lock clocks H_<l,s>, P_<l,s>: (word, key) -> index into hl/pl; each word's keys listed */
    vecs hl = {0}, pl = {0}, lrw = {0}, csv = {0};
    hl.T = pl.T = lrw.T = csv.T = T;
    /* map sizes: lock words and lock clocks are at most the lock operations (two keys each), the
     * queue cursors the closing releases, the L^r / L^w clocks the (access, held section) pairs */
    uint64_t n_lockops = 0, inside = 0;
    for (uint64_t i = 0; i < n; i++) n_lockops += is_lockop(&p, (uint32_t)i);
    for (uint32_t t = 0; t < T; t++) {
        uint64_t depth = 0;
        for (uint32_t q = p.po_start[t]; q < p.po_start[t + 1]; q++) {
            uint32_t i = p.po_idx[q];
            if (is_access(kind_of(&ev[i])) && !is_lockop(&p, i)) inside += depth;
            depth -= C.close_cs[i] != UINT32_MAX;
            depth += C.open_cs[i] != UINT32_MAX;
        }
    }
    if (rc == ORC_OK && (hmap_init(&lkmap, 2 * n_lockops + 1) != ORC_OK || hmap_init(&wmap, n_lockops + 1) != ORC_OK ||
                         hmap_init(&lwmap, inside + 1) != ORC_OK))
        rc = ORC_ENOMEM;
    ulist *word_keys = NULL;   /* per lock word index: lock-clock indices present */
    uint32_t n_words = 0, n_lk = 0, n_lw = 0, wcap = 0;
    uint32_t *lk_key = NULL;   /* per lock-clock index: its scope key */
    uint32_t lkcap = 0;
    /* per critical section: C_t at its acquire, H_t at its release; read/write sets while open */
    uint32_t *cs_acqC = (uint32_t *)malloc(((size_t)C.n_cs + 1) * sizeof(uint32_t));
    uint32_t *cs_relH = (uint32_t *)malloc(((size_t)C.n_cs + 1) * sizeof(uint32_t));
    ulist *cs_R = (ulist *)calloc((size_t)C.n_cs + 1, sizeof(ulist));
    ulist *cs_W = (ulist *)calloc((size_t)C.n_cs + 1, sizeof(ulist));
    /* per lock word: its critical sections in acquire order; per (thread, word): queue cursor */
    ulist *word_cs = NULL;
    ulist cursor = {0};
    ulist *held = (ulist *)calloc(T ? T : 1, sizeof(ulist)); /* open critical sections per thread */
    /* (thread, critical section) pairs joined by rule (ii): at most one per thread and section */
    if (rc == ORC_OK && (!cs_acqC || !cs_relH || !cs_R || !cs_W || !held || hmap_init(&curmap, n_lockops + 1) != ORC_OK ||
                         hmap_init(&joinmap, 1024) != ORC_OK))
        rc = ORC_ENOMEM;

#define WORD_INDEX(w, out_idx)                                                                   \
    do {                                                                                         \
        int ins_;                                                                                \
        out_idx = hmap_get(&wmap, (w), n_words, &ins_);                                          \
        if (ins_) {                                                                              \
            if (n_words == wcap) {                                                               \
                uint32_t nc_ = wcap ? 2 * wcap : 64;                                             \
                ulist *a_ = (ulist *)realloc(word_keys, nc_ * sizeof(ulist));                    \
                ulist *b_ = (ulist *)realloc(word_cs, nc_ * sizeof(ulist));                      \
                if (!a_ || !b_) { if (a_) word_keys = a_; if (b_) word_cs = b_; rc = ORC_ENOMEM; break; } \
                word_keys = a_; word_cs = b_;                                                    \
                memset(&word_keys[wcap], 0, (nc_ - wcap) * sizeof(ulist));                       \
                memset(&word_cs[wcap], 0, (nc_ - wcap) * sizeof(ulist));                         \
                wcap = nc_;                                                                      \
            }                                                                                    \
            n_words++;                                                                           \
        }                                                                                        \
    } while (0)

    /* the lock clock of (word index wi, key k), created on first use */
#define LOCK_CLOCK(wi, k, out_idx)                                                               \
    do {                                                                                         \
        int ins_;                                                                                \
        out_idx = hmap_get(&lkmap, ((uint64_t)(wi) << 32) | (k), n_lk, &ins_);                    \
        if (ins_) {                                                                              \
            if (vecs_new(&hl) == UINT32_MAX || vecs_new(&pl) == UINT32_MAX) { rc = ORC_ENOMEM; break; } \
            if (n_lk == lkcap) {                                                                 \
                uint32_t nc_ = lkcap ? 2 * lkcap : 64;                                           \
                uint32_t *a_ = (uint32_t *)realloc(lk_key, nc_ * sizeof(uint32_t));             \
                if (!a_) { rc = ORC_ENOMEM; break; }                                             \
                lk_key = a_; lkcap = nc_;                                                        \
            }                                                                                    \
            lk_key[n_lk] = (k);                                                                  \
            n_lk++;                                                                              \
            if (ulist_push(&word_keys[wi], out_idx) != ORC_OK) { rc = ORC_ENOMEM; break; }       \
        }                                                                                        \
    } while (0)

    /* L^r (rw = 0) / L^w (rw = 1) of lock clock lk and location x, created on first use when
     * create is set; UINT32_MAX when absent */
#define LRW(lk, x, rw, create, out_idx)                                                          \
    do {                                                                                         \
        uint64_t key_ = ((uint64_t)(lk) << 33) | ((uint64_t)(x) << 1) | (rw);                     \
        int ins_;                                                                                \
        if (!(create)) {                                                                         \
            uint64_t m_ = lwmap.cap - 1, s_ = mix64(key_) & m_;                                  \
            out_idx = UINT32_MAX;                                                                \
            while (lwmap.vals[s_]) {                                                             \
                if (lwmap.keys[s_] == key_) { out_idx = lwmap.vals[s_] - 1; break; }             \
                s_ = (s_ + 1) & m_;                                                              \
            }                                                                                    \
        } else {                                                                                 \
            out_idx = hmap_get(&lwmap, key_, n_lw, &ins_);                                       \
            if (ins_) { if (vecs_new(&lrw) == UINT32_MAX) { rc = ORC_ENOMEM; break; } n_lw++; }  \
        }                                                                                        \
    } while (0)

    /* barrier bookkeeping */
    uint32_t n_inst = p.bar_off[n_blocks];
    uint32_t *bar_n = (uint32_t *)calloc(n_inst ? n_inst : 1, sizeof(uint32_t));
    uint32_t *bar_list_off = (uint32_t *)calloc((size_t)n_inst + 1, sizeof(uint32_t));
    uint32_t *bar_list = NULL;
    uint32_t *wbar_n = (uint32_t *)calloc(p.n_winst ? p.n_winst : 1, sizeof(uint32_t));
    uint32_t *wbar_list = (uint32_t *)malloc(((size_t)p.n_winst * 32 + 1) * sizeof(uint32_t));
    if (!bar_n || !bar_list_off || !wbar_n || !wbar_list) rc = ORC_ENOMEM;
    if (rc == ORC_OK) {
        for (uint32_t s = 0; s < n_inst; s++) bar_list_off[s + 1] = bar_list_off[s] + p.bar_cnt[s];
        bar_list = (uint32_t *)malloc(((size_t)bar_list_off[n_inst] + 1) * sizeof(uint32_t));
        if (!bar_list) rc = ORC_ENOMEM;
    }

    for (uint64_t ii = 0; ii < n && rc == ORC_OK; ii++) {
        const uint32_t i = (uint32_t)ii, t = ev[i].tid, bt = t / tpb;
        const unsigned k = kind_of(&ev[i]);
        uint32_t *Pt = &P[(uint64_t)t * T], *Ht = &H[(uint64_t)t * T];

        if (is_access(k)) {
            const uint32_t x = loc[i];
            const int lockop = is_lockop(&p, i);
            /* Algorithm 2 READ / WRITE (reads and writes only, reading G2): for every held
             * <l, s>, join L^w (and L^r for a write) of the lock clocks whose scope overlaps s */
            if (!lockop) {
                for (uint32_t q = 0; q < held[t].n && rc == ORC_OK; q++) {
                    const orc_cs *c = &C.cs[held[t].v[q]];
                    uint32_t wi;
                    WORD_INDEX(c->word, wi);
                    if (rc != ORC_OK) break;
                    for (uint32_t kk = 0; kk < word_keys[wi].n; kk++) {
                        uint32_t lk = word_keys[wi].v[kk], idx;
                        if (!keys_overlap(lk_key[lk], c->acq_key)) continue;
                        LRW(lk, x, 1, 0, idx);
                        if (idx != UINT32_MAX) vjoin(Pt, lrw.v[idx], T);
                        if (k != K_READ) {
                            LRW(lk, x, 0, 0, idx);
                            if (idx != UINT32_MAX) vjoin(Pt, lrw.v[idx], T);
                        }
                    }
                }
                if (rc != ORC_OK) break;
            }
            /* the check: an earlier conflicting access a of thread u races unless
             * epoch(a) <= C_t[u] = P_t[u] */
            for (uint32_t q = 0; q < hist[x].n; q++) {
                uint32_t a = hist[x].v[q];
                if (!conflict(&p, a, i)) continue;
                if (epoch[a] <= Pt[ev[a].tid]) continue;
                if (pairs_push(out, a, i) != ORC_OK) { rc = ORC_ENOMEM; break; }
            }
            if (rc != ORC_OK) break;
            epoch[i] = N[t];
            if (ulist_push(&hist[x], i) != ORC_OK) { rc = ORC_ENOMEM; break; }
            /* the read and write sets of every held critical section */
            if (!lockop)
                for (uint32_t q = 0; q < held[t].n; q++) {
                    uint32_t ci = held[t].v[q];
                    if (ulist_push(k == K_READ ? &cs_R[ci] : &cs_W[ci], x) != ORC_OK) { rc = ORC_ENOMEM; break; }
                }
            if (rc != ORC_OK) break;
        }

        if (p.rel_scope[i] != 0xff) {
            /* RELEASE(t, l, R, W, s) */
            const uint32_t key = scope_key(p.rel_scope[i], bt), ci = C.close_cs[i];
            uint32_t wi, lk;
            WORD_INDEX(loc_key(&p, &ev[i]), wi);
            if (rc != ORC_OK) break;
            if (ci != UINT32_MAX) {
                /* rule (ii): other threads' critical sections on l released before this one, in
                 * acquire order, whose acquire time is below C_t: join the release's H when the
                 * scopes overlap (G4).  Every queued entry is examined, not only the front (G5),
                 * until a pass joins nothing more; entries joined, or of t itself, before the first
                 * pending one are dropped from the queue. */
                uint32_t cur;
                {
                    int ins;
                    cur = hmap_get(&curmap, ((uint64_t)t << 32) | wi, cursor.n, &ins);
                    if (ins && ulist_push(&cursor, 0) != ORC_OK) { rc = ORC_ENOMEM; break; }
                }
                const uint32_t Nt = N[t];
                for (int more = 1; more && rc == ORC_OK;) {
                    more = 0;
                    for (uint32_t pos = cursor.v[cur]; pos < word_cs[wi].n; pos++) {
                        const uint32_t fi = word_cs[wi].v[pos];
                        const orc_cs *f = &C.cs[fi];
                        if (f->tid == t || f->rel == UINT32_MAX || f->rel > i || !keys_overlap(f->rel_key, key)) continue;
                        int ins;
                        (void)hmap_get(&joinmap, ((uint64_t)t << 32) | fi, 0, &ins);
                        if (!ins) continue; /* joined at an earlier release of t */
                        const uint32_t *ac = csv.v[cs_acqC[fi]];
                        int below = 1;
                        for (uint32_t u = 0; u < T && below; u++) below = ac[u] <= (u == t ? Nt : Pt[u]);
                        if (!below) { hmap_unget(&joinmap, ((uint64_t)t << 32) | fi); continue; }
                        vjoin(Pt, csv.v[cs_relH[fi]], T);
                        more = 1;
                    }
                }
                {
                    uint32_t pos = cursor.v[cur];
                    while (pos < word_cs[wi].n) {
                        const uint32_t fi = word_cs[wi].v[pos];
                        if (C.cs[fi].tid != t && !hmap_has(&joinmap, ((uint64_t)t << 32) | fi)) break;
                        pos++;
                    }
                    cursor.v[cur] = pos;
                }
                /* L^r_<l,s>,x and L^w_<l,s>,x join H_t for the section's reads and writes */
                LOCK_CLOCK(wi, key, lk);
                if (rc != ORC_OK) break;
                for (int rw = 0; rw < 2 && rc == ORC_OK; rw++) {
                    const ulist *S = rw ? &cs_W[ci] : &cs_R[ci];
                    for (uint32_t q = 0; q < S->n; q++) {
                        uint32_t idx;
                        LRW(lk, S->v[q], rw, 1, idx);
                        if (rc != ORC_OK) break;
                        vjoin(lrw.v[idx], Ht, T);
                    }
                }
                if (rc != ORC_OK) break;
                /* Rel_l(t').enque(<H_t, s>) for t' != t: the section's release time */
                uint32_t v = vecs_new(&csv);
                if (v == UINT32_MAX) { rc = ORC_ENOMEM; break; }
                memcpy(csv.v[v], Ht, (size_t)T * sizeof(uint32_t));
                cs_relH[ci] = v;
                /* the lockset loses the section */
                for (uint32_t q = 0; q < held[t].n; q++)
                    if (held[t].v[q] == ci) {
                        memmove(&held[t].v[q], &held[t].v[q + 1], (held[t].n - q - 1) * sizeof(uint32_t));
                        held[t].n--;
                        break;
                    }
            } else {
                LOCK_CLOCK(wi, key, lk);
                if (rc != ORC_OK) break;
            }
            /* H_<l,s> and P_<l,s> publish t's clocks (joined, G6) */
            vjoin(hl.v[lk], Ht, T);
            vjoin(pl.v[lk], Pt, T);
            N[t] += 1;
            Ht[t] += 1;
        }

        if (p.acq_scope[i] != 0xff) {
            /* ACQUIRE(t, l, s): join P and H of every lock clock of l whose scope reaches s */
            const uint32_t key = scope_key(p.acq_scope[i], bt);
            uint32_t wi;
            WORD_INDEX(loc_key(&p, &ev[i]), wi);
            if (rc != ORC_OK) break;
            for (uint32_t kk = 0; kk < word_keys[wi].n; kk++) {
                uint32_t lk = word_keys[wi].v[kk];
                if (!keys_overlap(lk_key[lk], key)) continue;
                vjoin(Pt, pl.v[lk], T);
                vjoin(Ht, hl.v[lk], T);
            }
            const uint32_t ci = C.open_cs[i];
            if (ci != UINT32_MAX) {
                /* Acq_l(t').enque(<C_t, s>) for t' != t */
                uint32_t v = vecs_new(&csv);
                if (v == UINT32_MAX) { rc = ORC_ENOMEM; break; }
                memcpy(csv.v[v], Pt, (size_t)T * sizeof(uint32_t));
                csv.v[v][t] = N[t];
                cs_acqC[ci] = v;
                if (ulist_push(&word_cs[wi], ci) != ORC_OK || ulist_push(&held[t], ci) != ORC_OK) { rc = ORC_ENOMEM; break; }
            }
        }

        /* SYNC(scope): at the last arrival of a block or warp barrier instance */
        uint32_t *parts = NULL, np = 0;
        if (k == K_BAR) {
            uint32_t slot = p.bar_off[bt] + p.phase[i];
            bar_list[bar_list_off[slot] + bar_n[slot]++] = t;
            if (bar_n[slot] == p.n_active[bt]) { parts = &bar_list[bar_list_off[slot]]; np = bar_n[slot]; }
        }
        if (k == K_WBAR) {
            uint32_t inst = p.wbar_inst[i];
            wbar_list[(uint64_t)inst * 32 + wbar_n[inst]++] = t;
            if (wbar_n[inst] == (uint32_t)__builtin_popcount(p.winst_mask[inst])) { parts = &wbar_list[(uint64_t)inst * 32]; np = wbar_n[inst]; }
        }
        if (parts) {
            memset(J, 0, (size_t)T * sizeof(uint32_t));
            memset(JH, 0, (size_t)T * sizeof(uint32_t));
            for (uint32_t q = 0; q < np; q++) {
                uint32_t u = parts[q];
                uint32_t *Pu = &P[(uint64_t)u * T];
                for (uint32_t w = 0; w < T; w++) {
                    uint32_t cu = w == u ? N[u] : Pu[w]; /* C_u = P_u{u := N_u} */
                    if (cu > J[w]) J[w] = cu;
                }
                vjoin(JH, &H[(uint64_t)u * T], T);
            }
            for (uint32_t q = 0; q < np; q++) {
                uint32_t u = parts[q];
                memcpy(&P[(uint64_t)u * T], J, (size_t)T * sizeof(uint32_t));
                memcpy(&H[(uint64_t)u * T], JH, (size_t)T * sizeof(uint32_t));
                N[u] += 1;
                H[(uint64_t)u * T + u] += 1;
            }
        }
    }
#undef WORD_INDEX
#undef LOCK_CLOCK
#undef LRW

    if (hist) for (uint32_t x = 0; x < L; x++) free(hist[x].v);
    free(hist); free(loc); free(epoch); free(N); free(P); free(H); free(J); free(JH);
    vecs_free(&hl); vecs_free(&pl); vecs_free(&lrw); vecs_free(&csv);
    if (word_keys) for (uint32_t w = 0; w < n_words; w++) { free(word_keys[w].v); free(word_cs[w].v); }
    free(word_keys); free(word_cs); free(lk_key); free(cursor.v);
    if (cs_R) for (uint32_t c = 0; c < C.n_cs; c++) { free(cs_R[c].v); free(cs_W[c].v); }
    if (held) for (uint32_t t = 0; t < T; t++) free(held[t].v);
    free(cs_R); free(cs_W); free(cs_acqC); free(cs_relH); free(held);
    free(bar_n); free(bar_list_off); free(bar_list); free(wbar_n); free(wbar_list);
    hmap_free(&lmap); hmap_free(&lkmap); hmap_free(&wmap); hmap_free(&lwmap); hmap_free(&curmap);
    hmap_free(&joinmap);
    cs_free(&C);
    prep_free(&p);
    if (rc != ORC_OK) { orc_pairs_free(out); return rc; }
    qsort(out->data, out->n, 2 * sizeof(uint32_t), cmp_pair);
    return ORC_OK;
}

/* The definition (rules (i)-(iv)) on a tiny trace: base edges from rule (i) (a release r and a
 * later read or write e inside a critical section of the same lock word, the sections' scopes
 * overlapping, r's section holding an access of e's location with a write on either side), rule
 * (iii) (every event before a participant's barrier arrival to every event after another
 * participant's arrival) and rule (ii) (two releases of one lock word by different threads whose
 * critical sections, acquire and release included, hold GWCP-ordered events, the releases' scopes
 * overlapping); rule (iv) composes each base edge with happens-before on both sides; the relation
 * is closed transitively, and rule (ii) is applied again until nothing changes.  The report is
 * every conflicting pair of different threads left unordered. */
int orc_gwcp_bruteforce(uint32_t n_blocks, uint32_t tpb, uint32_t warp_size, const orc_event *ev, uint64_t n,
                        uint64_t *bad, orc_pairs *out) {
    memset(out, 0, sizeof(*out));
    *bad = UINT64_MAX;
    if (!grid_ok(n_blocks, tpb, &warp_size, n)) return ORC_EINVAL;
    if (n > 4096) return ORC_EINVAL; /* cubic work: tiny traces only */
    g_inclusive = 0;
    prep_t p;
    int rc = prepare(&p, n_blocks, tpb, warp_size, ev, n, bad);
    if (rc != ORC_OK) { prep_free(&p); return rc; }
    cs_info C;
    rc = cs_build(&p, &C);
    if (rc != ORC_OK) { prep_free(&p); return rc; }
    const uint64_t W = (n + 63) / 64;
    uint64_t *hb = hb_reach(&p);                                         /* hb[j]: i ->+ j */
    uint64_t *gw = (uint64_t *)calloc(n * W + 1, sizeof(uint64_t));     /* gw[j]: i <GWCP j */
    uint32_t *esrc = NULL, *edst = NULL;                                 /* base edges */
    uint64_t n_edges = 0, cap_edges = 0;
    uint8_t *have_ii = (uint8_t *)calloc((size_t)C.n_cs * C.n_cs + 1, 1); /* rule (ii) edge added */
    if (!hb || !gw || !have_ii) rc = ORC_ENOMEM;
#define BIT(m, row, i) (((m)[(uint64_t)(row) * W + ((i) >> 6)] >> ((i) & 63)) & 1)
#define HB(i, j) ((i) == (j) || BIT(hb, j, i))
#define ADD_EDGE(a, b)                                                                           \
    do {                                                                                         \
        if (n_edges == cap_edges) {                                                              \
            uint64_t nc_ = cap_edges ? 2 * cap_edges : 256;                                      \
            uint32_t *s_ = (uint32_t *)realloc(esrc, nc_ * sizeof(uint32_t));                    \
            uint32_t *d_ = (uint32_t *)realloc(edst, nc_ * sizeof(uint32_t));                    \
            if (s_) esrc = s_;                                                                   \
            if (d_) edst = d_;                                                                   \
            if (!s_ || !d_) { rc = ORC_ENOMEM; break; }                                          \
            cap_edges = nc_;                                                                     \
        }                                                                                        \
        esrc[n_edges] = (a); edst[n_edges] = (b); n_edges++;                                     \
    } while (0)

    /* po range of a critical section: [po_pos(acq), po_pos(rel)] of its thread (rel: to the end) */
#define CS_LO(c) (p.po_start[(c)->tid] + p.po_pos[(c)->acq])
#define CS_HI(c) ((c)->rel == UINT32_MAX ? p.po_start[(c)->tid + 1] - 1 : p.po_start[(c)->tid] + p.po_pos[(c)->rel])

    /* rule (i) */
    for (uint32_t c1i = 0; c1i < C.n_cs && rc == ORC_OK; c1i++) {
        const orc_cs *c1 = &C.cs[c1i];
        if (c1->rel == UINT32_MAX) continue;
        for (uint64_t jj = c1->rel + 1; jj < n && rc == ORC_OK; jj++) {
            uint32_t e = (uint32_t)jj;
            if (!is_access(kind_of(&ev[e])) || is_lockop(&p, e)) continue;
            /* e inside a critical section of its thread on c1's word, scopes overlapping */
            int inside = 0;
            for (uint32_t c2i = 0; c2i < C.n_cs && !inside; c2i++) {
                const orc_cs *c2 = &C.cs[c2i];
                if (c2->tid != ev[e].tid || c2->word != c1->word || c2i == c1i) continue;
                uint32_t pe = p.po_start[c2->tid] + p.po_pos[e];
                if (pe > CS_LO(c2) && pe < CS_HI(c2) + (c2->rel == UINT32_MAX)) inside = keys_overlap(c1->rel_key, c2->acq_key);
            }
            if (!inside) continue;
            int hit = 0;
            for (uint32_t q = CS_LO(c1) + 1; q < CS_HI(c1) && !hit; q++) {
                uint32_t a = p.po_idx[q];
                if (!is_access(kind_of(&ev[a])) || is_lockop(&p, a)) continue;
                if (loc_key(&p, &ev[a]) != loc_key(&p, &ev[e])) continue;
                hit = is_writeish(kind_of(&ev[a])) || is_writeish(kind_of(&ev[e]));
            }
            if (hit) ADD_EDGE(c1->rel, e);
        }
    }
    /* rule (iii): block barriers (participants' k-th BAR) and warp barriers (an instance's WBARs) */
    for (uint64_t jj = 0; jj < n && rc == ORC_OK; jj++) {
        uint32_t bu = (uint32_t)jj;
        unsigned kb = kind_of(&ev[bu]);
        if (kb != K_BAR && kb != K_WBAR) continue;
        uint32_t u = ev[bu].tid;
        if (p.po_pos[bu] == 0) continue;
        uint32_t before = p.po_idx[p.po_start[u] + p.po_pos[bu] - 1];
        for (uint64_t kk = 0; kk < n && rc == ORC_OK; kk++) {
            uint32_t bv = (uint32_t)kk, v = ev[bv].tid;
            if (kind_of(&ev[bv]) != kb) continue;
            if (kb == K_BAR && (block_of(&p, v) != block_of(&p, u) || p.phase[bv] != p.phase[bu])) continue;
            if (kb == K_WBAR && p.wbar_inst[bv] != p.wbar_inst[bu]) continue;
            if (p.po_start[v] + p.po_pos[bv] + 1 >= p.po_start[v + 1]) continue;
            ADD_EDGE(before, p.po_idx[p.po_start[v] + p.po_pos[bv] + 1]);
        }
    }
    /* fixpoint with rule (ii) */
    int changed = 1;
    while (changed && rc == ORC_OK) {
        changed = 0;
        memset(gw, 0, n * W * sizeof(uint64_t));
        /* rule (iv): x ->HB* x0 -> y0 ->HB* y */
        for (uint64_t q = 0; q < n_edges; q++) {
            uint32_t x0 = esrc[q], y0 = edst[q];
            for (uint64_t yy = y0; yy < n; yy++) {
                uint32_t y = (uint32_t)yy;
                if (!HB(y0, y)) continue;
                for (uint64_t w = 0; w < W; w++) gw[(uint64_t)y * W + w] |= hb[(uint64_t)x0 * W + w];
                gw[(uint64_t)y * W + (x0 >> 6)] |= (uint64_t)1 << (x0 & 63);
            }
        }
        /* transitive closure in trace order (every edge points forward) */
        for (uint64_t yy = 0; yy < n; yy++)
            for (uint64_t xx = 0; xx < yy; xx++)
                if (BIT(gw, yy, xx))
                    for (uint64_t w = 0; w < W; w++) gw[yy * W + w] |= gw[xx * W + w];
        /* rule (ii) */
        for (uint32_t c1i = 0; c1i < C.n_cs && rc == ORC_OK; c1i++) {
            const orc_cs *c1 = &C.cs[c1i];
            if (c1->rel == UINT32_MAX) continue;
            for (uint32_t c2i = 0; c2i < C.n_cs; c2i++) {
                const orc_cs *c2 = &C.cs[c2i];
                if (c2->rel == UINT32_MAX || c2->tid == c1->tid || c2->word != c1->word || c2->rel <= c1->rel) continue;
                if (!keys_overlap(c1->rel_key, c2->rel_key) || have_ii[(uint64_t)c1i * C.n_cs + c2i]) continue;
                int ordered = 0;
                for (uint32_t q1 = CS_LO(c1); q1 <= CS_HI(c1) && !ordered; q1++)
                    for (uint32_t q2 = CS_LO(c2); q2 <= CS_HI(c2) && !ordered; q2++)
                        ordered = BIT(gw, p.po_idx[q2], p.po_idx[q1]);
                if (!ordered) continue;
                have_ii[(uint64_t)c1i * C.n_cs + c2i] = 1;
                ADD_EDGE(c1->rel, c2->rel);
                changed = 1;
            }
        }
    }
    for (uint64_t jj = 0; jj < n && rc == ORC_OK; jj++) {
        uint32_t j = (uint32_t)jj;
        if (!is_access(kind_of(&ev[j]))) continue;
        for (uint32_t i = 0; i < j; i++) {
            if (!conflict(&p, i, j) || BIT(gw, j, i)) continue;
            if (pairs_push(out, i, j) != ORC_OK) { rc = ORC_ENOMEM; break; }
        }
    }
#undef BIT
#undef HB
#undef ADD_EDGE
#undef CS_LO
#undef CS_HI
    free(hb); free(gw); free(esrc); free(edst); free(have_ii);
    cs_free(&C);
    prep_free(&p);
    if (rc != ORC_OK) { orc_pairs_free(out); return rc; }
    qsort(out->data, out->n, 2 * sizeof(uint32_t), cmp_pair);
    return ORC_OK;
}

/* ================================================================ lockset pass (Section 2.2, Section 3)
 *
 * The lockset analysis the paper describes for ScoRD (after Eraser): every access carries the set
 * of locks its thread holds at it; the shadow of a location keeps its previous access, and each
 * access is compared with that one.  The paper states when ScoRD reports: a pair whose locksets
 * share no lock (Figure 3: the lockset at e6 holds l, the one at e1 is empty, so the race is
 * reported), except that the analysis is skipped when neither access holds a lock (Figure 4 and
 * Figure 5: both accesses unprotected, nothing reported).
 *
 *   orc_lockset  walks the trace in order with per-thread locksets and per-location previous
 *                accesses, and reports (previous, current) for every access that
 *                  - conflicts with the location's previous access (conflict() above),
 *                  - where at least one of the two holds a lock,
 *                  - and no lock word is held by both with overlapping scope keys.
 *
 * Readings (each also listed in the design notes):
 *   L1 a lock held is a critical section of reading G1 that is open at the access, with the scope
 *      key of its acquire (G4); lock operations (explicit or inferred acquires and releases) are not
 *      compared and do not become a location's previous access: they are the locks;
 *   L2 the previous access is the location's latest earlier access other than a lock operation,
 *      whatever its thread (one shadow entry per location; a pair of one thread is never reported);
 *   L3 two locksets share a lock when one word is held in both with keys that overlap (either is
 *      device scoped, or both in one block).
 */
#define LS_NEST 64 /* nesting kept per access (a deeper trace is refused with ORC_ENOMEM) */
typedef struct { uint32_t n; uint64_t word[LS_NEST]; uint32_t key[LS_NEST]; } lockset_t;

static int locksets_share(const lockset_t *a, const lockset_t *b) {
    for (uint32_t i = 0; i < a->n; i++)
        for (uint32_t j = 0; j < b->n; j++)
            if (a->word[i] == b->word[j] && keys_overlap(a->key[i], b->key[j])) return 1;
    return 0;
}

int orc_lockset(uint32_t n_blocks, uint32_t tpb, uint32_t warp_size, const orc_event *ev, uint64_t n,
                uint64_t *bad, orc_pairs *out) {
    memset(out, 0, sizeof(*out));
    *bad = UINT64_MAX;
    if (!grid_ok(n_blocks, tpb, &warp_size, n)) return ORC_EINVAL;
    prep_t p;
    int rc = prepare(&p, n_blocks, tpb, warp_size, ev, n, bad);
    if (rc != ORC_OK) { prep_free(&p); return rc; }
    cs_info C;
    rc = cs_build(&p, &C);
    if (rc != ORC_OK) { prep_free(&p); return rc; }
    const uint32_t T = p.n_threads;
    lockset_t *held = (lockset_t *)calloc(T ? T : 1, sizeof(lockset_t));  /* per thread, open sections */
    hmap lmap = {0};
    uint32_t L = 0;
    uint32_t *prev = NULL;       /* per location: previous access (UINT32_MAX: none) */
    lockset_t *prev_ls = NULL;   /* ... and its lockset */
    if (!held || hmap_init(&lmap, n) != ORC_OK) rc = ORC_ENOMEM;
    uint64_t n_loc = 0;
    for (uint64_t i = 0; i < n && rc == ORC_OK; i++) n_loc += is_access(kind_of(&ev[i])) && !is_lockop(&p, (uint32_t)i);
    if (rc == ORC_OK) {
        prev = (uint32_t *)malloc((n_loc ? n_loc : 1) * sizeof(uint32_t));
        prev_ls = (lockset_t *)malloc((n_loc ? n_loc : 1) * sizeof(lockset_t));
        if (!prev || !prev_ls) rc = ORC_ENOMEM;
    }
    for (uint64_t ii = 0; ii < n && rc == ORC_OK; ii++) {
        const uint32_t i = (uint32_t)ii, t = ev[i].tid;
        if (is_lockop(&p, i)) {
            /* a release closes the section it closes (reading G1), then an acquire opens one */
            lockset_t *h = &held[t];
            const uint32_t cc = C.close_cs[i], oc = C.open_cs[i];
            if (cc != UINT32_MAX) {
                for (uint32_t q = 0; q < h->n; q++)
                    if (h->word[q] == C.cs[cc].word) {
                        memmove(&h->word[q], &h->word[q + 1], (h->n - q - 1) * sizeof(uint64_t));
                        memmove(&h->key[q], &h->key[q + 1], (h->n - q - 1) * sizeof(uint32_t));
                        h->n--;
                        break;
                    }
            }
            if (oc != UINT32_MAX) {
                if (h->n == LS_NEST) { rc = ORC_ENOMEM; break; }
                h->word[h->n] = C.cs[oc].word;
                h->key[h->n] = C.cs[oc].acq_key;
                h->n++;
            }
            continue;
        }
        if (!is_access(kind_of(&ev[i]))) continue;
        int ins;
        const uint32_t x = hmap_get(&lmap, loc_key(&p, &ev[i]), L, &ins);
        if (ins) { prev[x] = UINT32_MAX; L++; }
        const uint32_t a = prev[x];
        if (a != UINT32_MAX && conflict(&p, a, i) && (prev_ls[x].n || held[t].n) &&
            !locksets_share(&prev_ls[x], &held[t])) {
            if (pairs_push(out, a, i) != ORC_OK) { rc = ORC_ENOMEM; break; }
        }
        prev[x] = i;
        prev_ls[x] = held[t];
    }
    free(held); free(prev); free(prev_ls);
    hmap_free(&lmap);
    cs_free(&C);
    prep_free(&p);
    if (rc != ORC_OK) { orc_pairs_free(out); return rc; }
    qsort(out->data, out->n, 2 * sizeof(uint32_t), cmp_pair);
    return ORC_OK;
}
