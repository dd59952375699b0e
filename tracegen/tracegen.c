/*
 * tracegen.c -- seeded synthetic GPU event traces (input generator only; no race analysis).
 *
 * A trace is a list of 16-byte records (addr, tid, meta, aux), meta = kind | scope<<4 | space<<6.
 * The generator follows a synchronisation discipline so that the only unsynchronised conflicting
 * accesses are the ones it plants on purpose:
 *
 *   global words are READ-ONLY, DEVICE-ATOMIC (only device-scoped atomics), or OWNED by one block;
 *   shared words belong to their block.  Inside the owning block, in each barrier phase, an owned
 *   word is PRIVATE to one thread (read and written by it alone), PHASE-READ-ONLY, or
 *   BLOCK-ATOMIC (only block-scoped atomics of that block).
 *
 * Each thread draws an access kind from the configured mix and then a word that the discipline
 * allows for that kind, with Zipf-distributed reuse over the candidate list (continuous inverse-CDF
 * approximation of Zipf(s); s = 0 is uniform).  Block barriers and device fences sit at fixed
 * per-thread positions.  Plants turn an access into a write of a word that another thread uses
 * where the discipline forbids it: a word owned by another block, or a word another thread of the
 * same block uses in the same phase.  Threads are interleaved phase by phase at warp-instruction
 * granularity with a seeded shuffle, which keeps every barrier valid.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { K_READ = 0, K_WRITE = 1, K_ATOMIC = 2, K_FENCE = 3, K_BAR = 4 };
enum { SC_BLOCK = 0, SC_DEVICE = 1 };

typedef struct {
    uint32_t n_blocks, tpb, warp_size;
    uint32_t n_global;    /* global words */
    uint32_t n_shared;    /* shared words per block */
    uint64_t n_events;
    double zipf_s;        /* 0: uniform */
    double p_write, p_atomic_block, p_atomic_device;
    uint32_t bar_period;  /* 0: none */
    uint32_t fence_period;/* 0: none */
    double plant_rate;    /* per access */
    uint32_t plant_count; /* if nonzero: exactly this many plants (overrides plant_rate) */
    uint32_t plant_ww;    /* plants hit a write of another block (write-write races) */
    double p_plant_same_block; /* fraction of plants aimed at the same block and phase */
    uint32_t plant_victim_cap; /* victims only among words with at most this many accesses */
    double frac_ro, frac_da;   /* global word classes (rest: owned) */
    double frac_priv, frac_pro;/* owned word classes per phase (rest: block-atomic) */
    double p_read_ro;          /* a read goes to a read-only global word with this probability */
    uint32_t addr_base;
    uint64_t seed, trace_index;
} tg_config;

typedef struct {
    uint64_t n_planted;
    uint64_t n_degraded; /* accesses whose drawn kind had no legal word and became reads */
    uint64_t n_bar, n_fence, n_write, n_read, n_atomic;
} tg_stats;

/* ---------------------------------------------------------------- random numbers */

static inline uint64_t splitmix64(uint64_t *s) {
    uint64_t z = (*s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
typedef struct { uint64_t s[4]; } rng_t;
static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static inline uint64_t rng_next(rng_t *r) { /* xoshiro256** */
    uint64_t *s = r->s, res = rotl(s[1] * 5, 7) * 9, t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3]; s[2] ^= t; s[3] = rotl(s[3], 45);
    return res;
}
static void rng_seed(rng_t *r, uint64_t a, uint64_t b, uint64_t c) {
    uint64_t s = a * 0x9e3779b97f4a7c15ULL ^ (b + 0x632be59bd9b4e019ULL) * 0xbf58476d1ce4e5b9ULL ^ c;
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&s);
}
static inline double rng_unif(rng_t *r) { return (rng_next(r) >> 11) * (1.0 / 9007199254740992.0); }
static inline uint64_t rng_below(rng_t *r, uint64_t n) { return n ? rng_next(r) % n : 0; }
static inline uint64_t hash3(uint64_t a, uint64_t b, uint64_t c) {
    uint64_t s = a ^ (b * 0xd1b54a32d192ed03ULL) ^ (c * 0xabc98388fb8fac03ULL);
    return splitmix64(&s);
}
static inline double hash_unif(uint64_t a, uint64_t b, uint64_t c) {
    return (hash3(a, b, c) >> 11) * (1.0 / 9007199254740992.0);
}

/* Zipf(s)-distributed rank in [0, n): continuous inverse CDF of x^-s on [1, n+1). */
static inline uint32_t zipf_rank(rng_t *r, uint32_t n, double s) {
    if (n <= 1) return 0;
    double u = rng_unif(r), x;
    if (s == 0.0) return (uint32_t)rng_below(r, n);
    if (fabs(s - 1.0) < 1e-9) x = exp(u * log((double)n + 1.0));
    else {
        double a = 1.0 - s, hi = pow((double)n + 1.0, a);
        x = pow(1.0 + u * (hi - 1.0), 1.0 / a);
    }
    uint32_t k = (uint32_t)(x - 1.0);
    return k >= n ? n - 1 : k;
}

/* ---------------------------------------------------------------- generation */

/* word ids: global words are 0..G-1, shared word s of block b is G + b*S + s */
typedef struct {
    uint32_t word, kind, scope, space;
} slot_t;

static inline void emit(uint32_t *out, uint64_t pos, uint32_t addr, uint32_t tid, uint32_t meta,
                        uint32_t aux) {
    out[4 * pos + 0] = addr; out[4 * pos + 1] = tid; out[4 * pos + 2] = meta; out[4 * pos + 3] = aux;
}

int tg_generate(const tg_config *cfg, uint32_t *out, tg_stats *st, uint64_t *plant_idx,
                uint64_t plant_cap) {
    memset(st, 0, sizeof(*st));
    const uint32_t NB = cfg->n_blocks, TPB = cfg->tpb, WS = cfg->warp_size ? cfg->warp_size : 32;
    const uint64_t T = (uint64_t)NB * TPB, N = cfg->n_events;
    const uint32_t G = cfg->n_global, S = cfg->n_shared;
    const uint64_t seed = cfg->seed, tix = cfg->trace_index;
    if (NB == 0 || TPB == 0 || (G == 0 && S == 0)) return -1;

    /* per-thread event counts */
    uint64_t base = N / T, rem = N % T;
    /* all threads of a block share barrier and fence positions: use the block's minimum length */
    /* (threads t < rem get one extra event; the smallest count in block b is base unless every
     * thread of the block gets the extra event) */

    /* ---- global word classes and rank order ---- */
    uint8_t *gclass = (uint8_t *)malloc(G ? G : 1);  /* 0 owned, 1 read-only, 2 device-atomic */
    uint32_t *gowner = (uint32_t *)malloc((G ? G : 1) * sizeof(uint32_t));
    uint32_t *gperm = (uint32_t *)malloc((G ? G : 1) * sizeof(uint32_t)); /* rank -> word */
    uint32_t *gaddr = (uint32_t *)malloc((G ? G : 1) * sizeof(uint32_t)); /* word -> address */
    if (!gclass || !gowner || !gperm || !gaddr) return -2;
    rng_t rg;
    rng_seed(&rg, seed, tix, 0x51);
    for (uint32_t x = 0; x < G; x++) {
        double u = hash_unif(seed ^ (tix << 40), x, 1);
        gclass[x] = u < cfg->frac_ro ? 1 : (u < cfg->frac_ro + cfg->frac_da ? 2 : 0);
        gowner[x] = (uint32_t)(hash3(seed ^ (tix << 40), x, 2) % NB);
        gperm[x] = x;
        gaddr[x] = x;
    }
    for (uint32_t i = G; i > 1; i--) { uint32_t j = (uint32_t)rng_below(&rg, i); uint32_t t = gperm[i - 1]; gperm[i - 1] = gperm[j]; gperm[j] = t; }
    for (uint32_t i = G; i > 1; i--) { uint32_t j = (uint32_t)rng_below(&rg, i); uint32_t t = gaddr[i - 1]; gaddr[i - 1] = gaddr[j]; gaddr[j] = t; }
    /* rank-ordered lists: read-only, device-atomic, and owned words per block */
    uint32_t n_ro = 0, n_da = 0;
    uint32_t *ro = (uint32_t *)malloc((G ? G : 1) * sizeof(uint32_t));
    uint32_t *da = (uint32_t *)malloc((G ? G : 1) * sizeof(uint32_t));
    uint32_t *own_off = (uint32_t *)calloc((size_t)NB + 1, sizeof(uint32_t));
    uint32_t *own = (uint32_t *)malloc((G ? G : 1) * sizeof(uint32_t));
    if (!ro || !da || !own_off || !own) return -2;
    for (uint32_t r = 0; r < G; r++) {
        uint32_t x = gperm[r];
        if (gclass[x] == 1) ro[n_ro++] = x;
        else if (gclass[x] == 2) da[n_da++] = x;
        else own_off[gowner[x] + 1]++;
    }
    for (uint32_t b = 0; b < NB; b++) own_off[b + 1] += own_off[b];
    {
        uint32_t *fill = (uint32_t *)malloc(((size_t)NB + 1) * sizeof(uint32_t));
        if (!fill) return -2;
        memcpy(fill, own_off, ((size_t)NB + 1) * sizeof(uint32_t));
        for (uint32_t r = 0; r < G; r++) {
            uint32_t x = gperm[r];
            if (gclass[x] == 0) own[fill[gowner[x]]++] = x;
        }
        free(fill);
    }

    /* ---- per-thread streams ---- */
    uint64_t *tstart = (uint64_t *)malloc((T + 1) * sizeof(uint64_t));
    slot_t *slots = (slot_t *)malloc((N ? N : 1) * sizeof(slot_t));
    uint32_t *cnt = (uint32_t *)calloc((size_t)G + (size_t)NB * S + 1, sizeof(uint32_t));
    if (!tstart || !slots || !cnt) return -2;
    tstart[0] = 0;
    for (uint64_t t = 0; t < T; t++) tstart[t + 1] = tstart[t] + base + (t < rem ? 1 : 0);

    /* per block, per phase candidate lists (owned globals + the block's shared words) */
    uint32_t max_blk_words = 0;
    for (uint32_t b = 0; b < NB; b++) {
        uint32_t m = own_off[b + 1] - own_off[b] + S;
        if (m > max_blk_words) max_blk_words = m;
    }
    uint32_t *bw = (uint32_t *)malloc(((size_t)max_blk_words + 1) * sizeof(uint32_t));   /* block words by rank */
    uint32_t *priv_off = (uint32_t *)malloc(((size_t)TPB + 2) * sizeof(uint32_t));
    uint32_t *priv = (uint32_t *)malloc(((size_t)max_blk_words + 1) * sizeof(uint32_t));
    uint32_t *pro = (uint32_t *)malloc(((size_t)max_blk_words + 1) * sizeof(uint32_t));
    uint32_t *bat = (uint32_t *)malloc(((size_t)max_blk_words + 1) * sizeof(uint32_t));
    uint32_t *wowner = (uint32_t *)malloc(((size_t)max_blk_words + 1) * sizeof(uint32_t));
    uint8_t *wcls = (uint8_t *)malloc((size_t)max_blk_words + 1);
    uint32_t *sperm = (uint32_t *)malloc(((size_t)S + 1) * sizeof(uint32_t));
    if (!bw || !priv_off || !priv || !pro || !bat || !wowner || !wcls || !sperm) return -2;

    const uint32_t barp = cfg->bar_period, fencep = cfg->fence_period;
    for (uint32_t b = 0; b < NB; b++) {
        uint64_t t0 = (uint64_t)b * TPB;
        uint64_t emin = UINT64_MAX;
        for (uint32_t l = 0; l < TPB; l++) {
            uint64_t e = tstart[t0 + l + 1] - tstart[t0 + l];
            if (e < emin) emin = e;
        }
        /* the block's words in rank order: owned globals, then its shared words (own shuffle) */
        uint32_t nbw = 0;
        for (uint32_t q = own_off[b]; q < own_off[b + 1]; q++) bw[nbw++] = own[q];
        rng_t rs;
        rng_seed(&rs, seed, tix, 0x1000000ULL + b);
        for (uint32_t s = 0; s < S; s++) sperm[s] = s;
        for (uint32_t i = S; i > 1; i--) { uint32_t j = (uint32_t)rng_below(&rs, i); uint32_t tt = sperm[i - 1]; sperm[i - 1] = sperm[j]; sperm[j] = tt; }
        /* interleave shared words into the rank order (alternating) for a mixed hot set */
        {
            uint32_t ng = nbw, k = 0, gi = 0, si = 0;
            uint32_t *tmp = wowner; /* scratch */
            for (uint32_t q = 0; q < ng; q++) tmp[q] = bw[q];
            while (gi < ng || si < S) {
                if (gi < ng && (si >= S || (k & 1) == 0)) bw[k++] = tmp[gi++];
                else bw[k++] = G + b * S + sperm[si++];
            }
            nbw = k;
        }
        /* phases: phase ph covers per-thread positions between barriers */
        uint32_t ph = 0;
        uint64_t pos_lo = 0;
        for (;;) {
            /* next barrier position (exclusive end of this phase's accesses) */
            uint64_t bar_pos = UINT64_MAX;
            if (barp) {
                /* barriers at positions p with (p + 1) % barp == barp / 2, p < emin */
                uint64_t first = barp / 2 ? barp / 2 - 1 : barp - 1;
                uint64_t k = pos_lo <= first ? 0 : (pos_lo - first + barp - 1) / barp;
                uint64_t p = first + k * barp;
                if (p < emin) bar_pos = p;
            }
            /* classes of the block's words in this phase */
            for (uint32_t l = 0; l <= TPB; l++) priv_off[l] = 0;
            uint32_t npro = 0, nbat = 0, n_priv_dealt = 0;
            uint32_t rot = (uint32_t)(hash3(seed ^ (tix << 40), b, 0x100 + ph) % TPB);
            for (uint32_t q = 0; q < nbw; q++) {
                double u = hash_unif(seed ^ (tix << 40), ((uint64_t)bw[q] << 16) ^ ph, 3);
                if (u < cfg->frac_priv) {
                    /* private words are dealt to the block's threads round robin (with a
                     * per-phase rotation), so every thread gets its share */
                    wcls[q] = 0;
                    wowner[q] = (uint32_t)((n_priv_dealt++ + rot) % TPB);
                    priv_off[wowner[q] + 1]++;
                } else if (u < cfg->frac_priv + cfg->frac_pro) {
                    wcls[q] = 1; pro[npro++] = bw[q];
                } else {
                    wcls[q] = 2; bat[nbat++] = bw[q];
                }
            }
            for (uint32_t l = 0; l < TPB; l++) priv_off[l + 1] += priv_off[l];
            {
                uint32_t *fill = priv_off + 0;
                /* counting-sort private words by owner thread (rank order kept) */
                uint32_t *f2 = (uint32_t *)malloc(((size_t)TPB + 1) * sizeof(uint32_t));
                if (!f2) return -2;
                memcpy(f2, fill, ((size_t)TPB + 1) * sizeof(uint32_t));
                for (uint32_t q = 0; q < nbw; q++) if (wcls[q] == 0) priv[f2[wowner[q]]++] = bw[q];
                free(f2);
            }
            /* fill this phase's slots of every thread of the block */
            for (uint32_t l = 0; l < TPB; l++) {
                uint64_t t = t0 + l, len = tstart[t + 1] - tstart[t];
                uint64_t hi = bar_pos == UINT64_MAX ? len : bar_pos;
                rng_t r;
                rng_seed(&r, seed, tix, 0x2000000000ULL + t * 4096 + ph);
                uint32_t *mypriv = &priv[priv_off[l]];
                uint32_t nmy = priv_off[l + 1] - priv_off[l];
                for (uint64_t p = pos_lo; p < hi && p < len; p++) {
                    slot_t *sl = &slots[tstart[t] + p];
                    if (fencep && (p + 1) % fencep == fencep / 2) {
                        sl->kind = K_FENCE; sl->scope = SC_DEVICE; sl->word = 0; sl->space = 0;
                        continue;
                    }
                    double u = rng_unif(&r);
                    uint32_t kind = K_READ, scope = 0, word = UINT32_MAX;
                    if (u < cfg->p_write) {
                        if (nmy) { kind = K_WRITE; word = mypriv[zipf_rank(&r, nmy, cfg->zipf_s)]; }
                    } else if (u < cfg->p_write + cfg->p_atomic_block) {
                        if (nbat) { kind = K_ATOMIC; scope = SC_BLOCK; word = bat[zipf_rank(&r, nbat, cfg->zipf_s)]; }
                    } else if (u < cfg->p_write + cfg->p_atomic_block + cfg->p_atomic_device) {
                        if (n_da) { kind = K_ATOMIC; scope = SC_DEVICE; word = da[zipf_rank(&r, n_da, cfg->zipf_s)]; }
                    } else {
                        kind = K_READ;
                    }
                    if (word == UINT32_MAX) {
                        if (u < cfg->p_write + cfg->p_atomic_block + cfg->p_atomic_device)
                            st->n_degraded++; /* no legal word for the drawn kind */
                        kind = K_READ;
                        double v = rng_unif(&r);
                        if (n_ro && (v < cfg->p_read_ro || (nmy == 0 && npro == 0)))
                            word = ro[zipf_rank(&r, n_ro, cfg->zipf_s)];
                        else if (npro && (nmy == 0 || rng_unif(&r) < 0.5))
                            word = pro[zipf_rank(&r, npro, cfg->zipf_s)];
                        else if (nmy)
                            word = mypriv[zipf_rank(&r, nmy, cfg->zipf_s)];
                        else if (n_ro)
                            word = ro[zipf_rank(&r, n_ro, cfg->zipf_s)];
                        else
                            return -4; /* no legal word at all for this thread */
                    }
                    sl->kind = kind; sl->scope = scope; sl->word = word;
                    sl->space = word >= G ? 1 : 0;
                    cnt[word]++;
                }
                if (bar_pos != UINT64_MAX && bar_pos < len) {
                    slot_t *sl = &slots[tstart[t] + bar_pos];
                    sl->kind = K_BAR; sl->scope = 0; sl->word = 0; sl->space = 0;
                }
            }
            if (bar_pos == UINT64_MAX) break;
            pos_lo = bar_pos + 1;
            ph++;
        }
    }

    /* ---- plants ---- */
    uint64_t n_plants_target = 0;
    rng_t rp;
    rng_seed(&rp, seed, tix, 0x77);
    uint8_t *is_plant = (uint8_t *)calloc(N ? N : 1, 1);
    if (!is_plant) return -2;
    {
        /* choose planter slots */
        uint64_t want = cfg->plant_count;
        if (!want && cfg->plant_rate > 0) {
            for (uint64_t i = 0; i < N; i++) if (rng_unif(&rp) < cfg->plant_rate) { is_plant[i] = 1; n_plants_target++; }
        } else {
            for (uint64_t k = 0; k < want * 64 && n_plants_target < want; k++) {
                uint64_t i = rng_below(&rp, N);
                if (!is_plant[i]) { is_plant[i] = 1; n_plants_target++; }
            }
        }
    }
    /* thread of each slot, and phase per slot (barrier count before it) */
    uint64_t tcur = 0;
    for (uint64_t i = 0; i < N; i++) {
        while (i >= tstart[tcur + 1]) tcur++;
        if (!is_plant[i]) continue;
        is_plant[i] = 0;
        slot_t *sl = &slots[i];
        if (sl->kind == K_BAR || sl->kind == K_FENCE) continue;
        uint64_t t = tcur;
        uint32_t b = (uint32_t)(t / TPB);
        uint32_t ph_i = 0;
        for (uint64_t q = tstart[t]; q < i; q++) if (slots[q].kind == K_BAR) ph_i++;
        int same_block = !cfg->plant_ww && NB >= 1 && TPB > 1 && rng_unif(&rp) < cfg->p_plant_same_block;
        if (NB == 1 && !same_block) { if (TPB > 1 && !cfg->plant_ww) same_block = 1; else continue; }
        int done = 0;
        for (int tries = 0; tries < 256 && !done; tries++) {
            uint64_t u;
            if (same_block) u = (uint64_t)b * TPB + rng_below(&rp, TPB);
            else {
                uint32_t ob = (uint32_t)rng_below(&rp, NB - 1);
                if (ob >= b) ob++;
                u = (uint64_t)ob * TPB + rng_below(&rp, TPB);
            }
            if (u == t) continue;
            uint64_t ulen = tstart[u + 1] - tstart[u];
            if (!ulen) continue;
            uint64_t q = tstart[u] + rng_below(&rp, ulen);
            slot_t *v = &slots[q];
            if (is_plant[q]) continue; /* a planter (chosen or done) is never a victim */
            if (v->kind == K_BAR || v->kind == K_FENCE) continue;
            if (cfg->plant_ww && v->kind != K_WRITE) continue;
            if (cfg->plant_victim_cap && cnt[v->word] > cfg->plant_victim_cap) continue;
            if (same_block) {
                uint32_t ph_q = 0;
                for (uint64_t z = tstart[u]; z < q; z++) if (slots[z].kind == K_BAR) ph_q++;
                if (ph_q != ph_i) continue;
            } else {
                if (v->word >= G) continue;          /* shared words cannot be reached */
                if (gclass[v->word] != 0) continue;  /* a word owned by the other block */
            }
            cnt[sl->word]--;
            sl->kind = K_WRITE; sl->scope = 0; sl->word = v->word; sl->space = v->space;
            cnt[sl->word]++;
            is_plant[i] = 1;
            done = 1;
        }
    }

    /* ---- interleave: phase-synchronous rounds of warp instructions ---- */
    uint32_t n_warps_blk = (TPB + WS - 1) / WS;
    uint64_t n_warps = (uint64_t)NB * n_warps_blk;
    uint64_t *cur = (uint64_t *)malloc((T ? T : 1) * sizeof(uint64_t));   /* next slot per thread */
    uint32_t *wlist = (uint32_t *)malloc((N + n_warps + 1) * sizeof(uint32_t));
    if (!cur || !wlist) return -2;
    for (uint64_t t = 0; t < T; t++) cur[t] = tstart[t];
    rng_t ri;
    rng_seed(&ri, seed, tix, 0x99);
    uint64_t outp = 0, np = 0;
    for (;;) {
        /* the round ends at each thread's next barrier (inclusive) */
        uint64_t nl = 0;
        for (uint64_t w = 0; w < n_warps; w++) {
            uint32_t b = (uint32_t)(w / n_warps_blk), wi = (uint32_t)(w % n_warps_blk);
            uint64_t mx = 0;
            for (uint32_t l = 0; l < WS && wi * WS + l < TPB; l++) {
                uint64_t t = (uint64_t)b * TPB + wi * WS + l, c = cur[t], k = 0;
                while (c + k < tstart[t + 1]) {
                    k++;
                    if (slots[c + k - 1].kind == K_BAR) break;
                }
                if (k > mx) mx = k;
            }
            for (uint64_t k = 0; k < mx; k++) wlist[nl++] = (uint32_t)w;
        }
        if (nl == 0) break;
        for (uint64_t i = nl; i > 1; i--) { uint64_t j = rng_below(&ri, i); uint32_t tt = wlist[i - 1]; wlist[i - 1] = wlist[j]; wlist[j] = tt; }
        uint8_t *stopped = (uint8_t *)calloc(T ? T : 1, 1); /* thread reached its barrier */
        if (!stopped) return -2;
        for (uint64_t k = 0; k < nl; k++) {
            uint64_t w = wlist[k];
            uint32_t b = (uint32_t)(w / n_warps_blk), wi = (uint32_t)(w % n_warps_blk);
            for (uint32_t l = 0; l < WS && wi * WS + l < TPB; l++) {
                uint64_t t = (uint64_t)b * TPB + wi * WS + l;
                if (stopped[t] || cur[t] >= tstart[t + 1]) continue;
                uint64_t q = cur[t]++;
                const slot_t *sl = &slots[q];
                uint32_t addr, meta = sl->kind | (sl->scope << 4) | (sl->space << 6);
                if (sl->kind == K_BAR || sl->kind == K_FENCE) addr = 0;
                else if (sl->space) addr = sl->word - G - b * S; /* shared: word offset in the block */
                else addr = cfg->addr_base + gaddr[sl->word];
                emit(out, outp, addr, (uint32_t)t, meta, (uint32_t)((q - tstart[t]) & 0xffff));
                if (is_plant[q] && plant_idx && np < plant_cap) plant_idx[np] = outp;
                if (is_plant[q]) np++;
                switch (sl->kind) {
                case K_BAR: st->n_bar++; stopped[t] = 1; break;
                case K_FENCE: st->n_fence++; break;
                case K_WRITE: st->n_write++; break;
                case K_READ: st->n_read++; break;
                default: st->n_atomic++; break;
                }
                outp++;
            }
        }
        free(stopped);
    }
    st->n_planted = np;

    free(gclass); free(gowner); free(gperm); free(gaddr); free(ro); free(da); free(own_off); free(own);
    free(tstart); free(slots); free(cnt); free(bw); free(priv_off); free(priv); free(pro); free(bat);
    free(wowner); free(wcls); free(sperm); free(is_plant); free(cur); free(wlist);
    return outp == N ? 0 : -3;
}
