/*
 * stencil.c -- seeded synthetic trace of a halo-exchange stencil with a lock-guarded global
 * reduction (input generator only; no race analysis).
 *
 * The modelled kernel: a grid of RB x CB blocks of tpb threads; block (rb, cb) owns rows
 * [rb*R, rb*R + R) of a H x W matrix (H = RB*R, W = CB*tpb) and thread t its column cb*tpb + t.
 * Two buffers, rows `pitch` words apart (row-major, so a column walk is strided).  Each of S sweeps
 * reads the 5-point neighbourhood of every owned cell from one buffer and writes the cell in the
 * other (Jacobi), then
 *   BAR;  thread 0: FENCE(dev), ATOMIC flag[b]                    (release: publishes sweep s)
 *         thread k (k = 0..3 for the N, S, W, E neighbour that exists): ATOMIC flag[nb], FENCE(dev)
 *                                                                 (acquire of the neighbour)
 *   BAR.
 * After the last sweep thread 0 of every block, in a seeded order, takes a device lock:
 *   ACQ(lock, dev); READ acc; WRITE acc; REL(lock, dev).
 * Halo cells read from a neighbour block are ordered by the neighbour's release and this block's
 * acquire of the same flag; everything else by barriers and program order; the accumulator by the
 * lock.  The only races are planted scope downgrades, taken in pairs so that an edge disappears:
 * a neighbour's release fence and this block's acquire fence of the same sweep and flag become
 * block scoped (an edge is lost only when both sides are block scoped in different blocks), or the
 * release of one critical section and the acquire of the next one.
 *
 * Trace order: sweep by sweep; the cell accesses of a sweep at warp-instruction granularity over
 * groups of `group` blocks (a group's blocks take turns instruction by instruction), then the
 * first barrier of every block, every release, every acquire, the second barrier of every block.
 * Every acquire therefore follows the release it reads, and every barrier is valid.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { K_READ = 0, K_WRITE = 1, K_ATOMIC = 2, K_FENCE = 3, K_BAR = 4, K_ACQ = 6, K_REL = 7 };
enum { SC_BLOCK = 0, SC_DEVICE = 1 };

typedef struct {
    uint32_t rb, cb, tpb, warp_size;
    uint32_t rows;       /* R: rows per block */
    uint32_t sweeps;     /* S */
    uint32_t pitch;      /* words between rows (>= W) */
    uint32_t group;      /* blocks interleaved in the cell phase */
    double plant_rate;   /* fraction of fences (and of lock operations) downgraded, in pairs */
    uint64_t seed;
} tg_stencil_cfg;

typedef struct {
    uint64_t n_events;
    uint64_t n_fence_plants, n_lock_plants;
    uint32_t buf0, buf1, flags, acc, lock; /* word addresses */
} tg_stencil_stats;

static inline uint64_t smix(uint64_t *s) {
    uint64_t z = (*s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
static inline double hunif(uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
    uint64_t s = a * 0x9e3779b97f4a7c15ULL ^ (b + 1) * 0xd1b54a32d192ed03ULL ^ (c + 7) * 0xabc98388fb8fac03ULL ^
                 (d + 3) * 0x8cb92ba72f3d8dd7ULL;
    return (smix(&s) >> 11) * (1.0 / 9007199254740992.0);
}

static inline uint32_t meta(uint32_t kind, uint32_t scope) { return kind | (scope << 4); }

typedef struct {
    uint32_t *out;
    uint64_t pos, cap;
    int overflow;
} sink;

static inline void put(sink *k, uint32_t addr, uint32_t tid, uint32_t m, uint32_t aux) {
    if (k->out) {
        if (k->pos >= k->cap) { k->overflow = 1; return; }
        uint32_t *o = k->out + 4 * k->pos;
        o[0] = addr; o[1] = tid; o[2] = m; o[3] = aux;
    }
    k->pos++;
}

/* neighbour of block (r, c) in direction d (0 N, 1 S, 2 W, 3 E), or -1 */
static inline int64_t nbr(const tg_stencil_cfg *g, uint32_t r, uint32_t c, int d) {
    if (d == 0) return r > 0 ? (int64_t)(r - 1) * g->cb + c : -1;
    if (d == 1) return r + 1 < g->rb ? (int64_t)(r + 1) * g->cb + c : -1;
    if (d == 2) return c > 0 ? (int64_t)r * g->cb + c - 1 : -1;
    return c + 1 < g->cb ? (int64_t)r * g->cb + c + 1 : -1;
}

/* Is the acquire of block b, direction d, in sweep s downgraded (with the neighbour's release)? */
static inline int fence_plant(const tg_stencil_cfg *g, uint32_t b, uint32_t s, int d) {
    return g->plant_rate > 0 && s + 1 < g->sweeps && hunif(g->seed, b, s, (uint64_t)d) < g->plant_rate;
}

/* out == NULL: count only.  Returns 0, or -1 on bad configuration / too small a buffer. */
int tg_stencil(const tg_stencil_cfg *g, uint32_t *out, uint64_t cap, tg_stencil_stats *st,
               uint32_t *plants, uint64_t plant_cap) {
    if (!g || !st || !g->rb || !g->cb || !g->tpb || !g->rows || !g->sweeps || g->tpb > 1024) return -1;
    const uint64_t nb = (uint64_t)g->rb * g->cb, W = (uint64_t)g->cb * g->tpb, H = (uint64_t)g->rb * g->rows;
    if (g->pitch < W || 2 * H * g->pitch + nb + 2 >= (1ull << 32) || nb * g->tpb >= (1ull << 32)) return -1;
    const uint32_t buf0 = 0, buf1 = (uint32_t)(H * g->pitch), flags = (uint32_t)(2 * H * g->pitch);
    const uint32_t acc = flags + (uint32_t)nb, lock = acc + 1;
    const uint32_t ws = g->warp_size ? g->warp_size : 32, grp = g->group ? g->group : 64;
    memset(st, 0, sizeof(*st));
    st->buf0 = buf0; st->buf1 = buf1; st->flags = flags; st->acc = acc; st->lock = lock;
    sink k = {out, 0, cap, 0};
    uint64_t np = 0;

    for (uint32_t s = 0; s < g->sweeps; s++) {
        const uint32_t src = (s & 1) ? buf1 : buf0, dst = (s & 1) ? buf0 : buf1;
        /* cells: per group of blocks, per owned row, per access slot, per block, per warp, per lane */
        for (uint64_t b0 = 0; b0 < nb; b0 += grp) {
            const uint64_t b1 = b0 + grp < nb ? b0 + grp : nb;
            for (uint32_t i = 0; i < g->rows; i++)
                for (int slot = 0; slot < 6; slot++)
                    for (uint64_t b = b0; b < b1; b++) {
                        const uint32_t br = (uint32_t)(b / g->cb), bc = (uint32_t)(b % g->cb);
                        const uint64_t r = (uint64_t)br * g->rows + i;
                        for (uint32_t w0 = 0; w0 < g->tpb; w0 += ws)
                            for (uint32_t t = w0; t < w0 + ws && t < g->tpb; t++) {
                                const uint64_t c = (uint64_t)bc * g->tpb + t;
                                const uint32_t tid = (uint32_t)(b * g->tpb + t);
                                switch (slot) {
                                case 0: if (r > 0) put(&k, (uint32_t)(src + (r - 1) * g->pitch + c), tid, meta(K_READ, 0), 0); break;
                                case 1: if (c > 0) put(&k, (uint32_t)(src + r * g->pitch + c - 1), tid, meta(K_READ, 0), 0); break;
                                case 2: put(&k, (uint32_t)(src + r * g->pitch + c), tid, meta(K_READ, 0), 0); break;
                                case 3: if (c + 1 < W) put(&k, (uint32_t)(src + r * g->pitch + c + 1), tid, meta(K_READ, 0), 0); break;
                                case 4: if (r + 1 < H) put(&k, (uint32_t)(src + (r + 1) * g->pitch + c), tid, meta(K_READ, 0), 0); break;
                                default: put(&k, (uint32_t)(dst + r * g->pitch + c), tid, meta(K_WRITE, 0), 0); break;
                                }
                            }
                    }
        }
        /* first barrier */
        for (uint64_t b = 0; b < nb; b++)
            for (uint32_t t = 0; t < g->tpb; t++) put(&k, 0, (uint32_t)(b * g->tpb + t), meta(K_BAR, 0), 0);
        /* releases: thread 0 of every block; the fence is downgraded when an acquirer's pair is planted */
        for (uint64_t b = 0; b < nb; b++) {
            const uint32_t br = (uint32_t)(b / g->cb), bc = (uint32_t)(b % g->cb);
            int down = 0;
            for (int d = 0; d < 4; d++) {
                const int64_t a = nbr(g, br, bc, d);  /* a acquires b's flag from direction d^1 */
                if (a >= 0 && fence_plant(g, (uint32_t)a, s, d ^ 1)) down = 1;
            }
            const uint32_t tid = (uint32_t)(b * g->tpb);
            put(&k, 0, tid, meta(K_FENCE, down ? SC_BLOCK : SC_DEVICE), 0);
            put(&k, flags + (uint32_t)b, tid, meta(K_ATOMIC, SC_DEVICE), 0);
        }
        /* acquires: thread d of block b reads the flag of its neighbour in direction d */
        for (uint64_t b = 0; b < nb; b++) {
            const uint32_t br = (uint32_t)(b / g->cb), bc = (uint32_t)(b % g->cb);
            for (int d = 0; d < 4; d++) {
                const int64_t a = nbr(g, br, bc, d);
                if (a < 0 || (uint32_t)d >= g->tpb) continue;
                const int down = fence_plant(g, (uint32_t)b, s, d);
                const uint32_t tid = (uint32_t)(b * g->tpb + (uint32_t)d);
                put(&k, flags + (uint32_t)a, tid, meta(K_ATOMIC, SC_DEVICE), 0);
                put(&k, 0, tid, meta(K_FENCE, down ? SC_BLOCK : SC_DEVICE), 0);
                if (down) {
                    if (plants && np < plant_cap) {
                        plants[4 * np] = 0; plants[4 * np + 1] = (uint32_t)b;
                        plants[4 * np + 2] = s; plants[4 * np + 3] = (uint32_t)d;
                    }
                    np++;
                    st->n_fence_plants++;
                }
            }
        }
        /* second barrier */
        for (uint64_t b = 0; b < nb; b++)
            for (uint32_t t = 0; t < g->tpb; t++) put(&k, 0, (uint32_t)(b * g->tpb + t), meta(K_BAR, 0), 0);
    }
    /* lock-guarded reduction in a seeded order (Fisher-Yates over the blocks) */
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * nb);
    if (!order) return -1;
    for (uint64_t b = 0; b < nb; b++) order[b] = (uint32_t)b;
    uint64_t rs = g->seed ^ 0x10c4ULL;
    for (uint64_t i = nb; i > 1; i--) {
        const uint64_t j = smix(&rs) % i;
        const uint32_t x = order[i - 1]; order[i - 1] = order[j]; order[j] = x;
    }
    for (uint64_t q = 0; q < nb; q++) {
        const uint32_t b = order[q], tid = b * g->tpb;
        /* section q's acquire is downgraded together with section q-1's release */
        const int down_acq = q > 0 && g->plant_rate > 0 && hunif(g->seed, 0x10c4, q, 9) < g->plant_rate;
        const int down_rel = q + 1 < nb && g->plant_rate > 0 && hunif(g->seed, 0x10c4, q + 1, 9) < g->plant_rate;
        put(&k, lock, tid, meta(K_ACQ, down_acq ? SC_BLOCK : SC_DEVICE), 0);
        put(&k, acc, tid, meta(K_READ, 0), 0);
        put(&k, acc, tid, meta(K_WRITE, 0), 0);
        put(&k, lock, tid, meta(K_REL, down_rel ? SC_BLOCK : SC_DEVICE), 0);
        if (down_acq) {
            if (plants && np < plant_cap) {
                plants[4 * np] = 1; plants[4 * np + 1] = b; plants[4 * np + 2] = (uint32_t)q; plants[4 * np + 3] = 0;
            }
            np++;
            st->n_lock_plants++;
        }
    }
    free(order);
    st->n_events = k.pos;
    return k.overflow ? -1 : 0;
}
