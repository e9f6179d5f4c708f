/*
 * Seeded synthetic edge-stream generators.
 *
 * These produce the dynamic graph streams that both the CPU oracle and the
 * GPU library consume.  They contain none of the sketching arithmetic: they
 * only emit (u, v, op) triples, op = 1 for an insertion and 0 for a deletion,
 * following the stream legality rules of the streaming connected-components
 * problem (Sec. 2.1: insert only absent edges, delete only present ones).
 *
 * Randomness: PCG32 (O'Neill, "PCG: A Family of Simple Fast Space-Efficient
 * Statistically Good Algorithms for Random Number Generation", 2014), the
 * 64-bit-state XSH-RR variant with its published seeding procedure.
 *
 * Stand-in for the paper's datasets (Sec. 6.1 builds Graph500 Kronecker
 * graphs): R-MAT draws with a per-level quadrant choice (a, b, c, d).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t state;
    uint64_t inc;
} pcg32_t;

static uint32_t pcg32_next(pcg32_t *g) {
    uint64_t old = g->state;
    g->state = old * 6364136223846793005ULL + g->inc;
    uint32_t xs = (uint32_t)(((old >> 18u) ^ old) >> 27u);
    uint32_t rot = (uint32_t)(old >> 59u);
    return (xs >> rot) | (xs << ((32u - rot) & 31u));
}

static void pcg32_seed(pcg32_t *g, uint64_t initstate, uint64_t initseq) {
    g->state = 0u;
    g->inc = (initseq << 1u) | 1u;
    pcg32_next(g);
    g->state += initstate;
    pcg32_next(g);
}

static uint64_t rng64(pcg32_t *g) {
    uint64_t hi = pcg32_next(g);
    uint64_t lo = pcg32_next(g);
    return (hi << 32) | lo;
}

/* uniform integer in [0, m), Lemire's multiply-high reduction (bias < m/2^64) */
static uint64_t rng_below(pcg32_t *g, uint64_t m) {
    return (uint64_t)(((unsigned __int128)rng64(g) * (unsigned __int128)m) >> 64);
}

/* uniform double in [0, 1) with 53 random bits */
static double rng_unit(pcg32_t *g) {
    return (double)(rng64(g) >> 11) * (1.0 / 9007199254740992.0);
}

/* ---------- live-edge bookkeeping: V*V bitmap + array of live keys ---------- */

typedef struct {
    uint32_t V;
    uint64_t *bits;   /* bit (u*V+v) set <=> edge {u<v} live */
    uint64_t *live;   /* keys of live edges, unordered */
    uint64_t nlive, cap;
} liveset_t;

static int live_init(liveset_t *L, uint32_t V, uint64_t cap) {
    L->V = V;
    uint64_t nbits = (uint64_t)V * (uint64_t)V;
    L->bits = (uint64_t *)calloc((nbits + 63) / 64, sizeof(uint64_t));
    L->live = (uint64_t *)malloc((cap ? cap : 1) * sizeof(uint64_t));
    L->nlive = 0;
    L->cap = cap;
    return (L->bits && L->live) ? 0 : -1;
}

static void live_free(liveset_t *L) {
    free(L->bits);
    free(L->live);
}

static uint64_t key_of(uint32_t V, uint32_t u, uint32_t v) {
    if (u > v) { uint32_t t = u; u = v; v = t; }
    return (uint64_t)u * V + v;
}

static int live_has(const liveset_t *L, uint64_t k) {
    return (int)((L->bits[k >> 6] >> (k & 63)) & 1u);
}

static int live_insert(liveset_t *L, uint64_t k) {
    if (L->nlive >= L->cap) return -1;
    L->bits[k >> 6] |= (1ULL << (k & 63));
    L->live[L->nlive++] = k;
    return 0;
}

/* remove a uniformly chosen live edge, return its key */
static uint64_t live_pop_random(liveset_t *L, pcg32_t *g) {
    uint64_t i = rng_below(g, L->nlive);
    uint64_t k = L->live[i];
    L->live[i] = L->live[L->nlive - 1];
    L->nlive--;
    L->bits[k >> 6] &= ~(1ULL << (k & 63));
    return k;
}

static void emit(uint32_t *src, uint32_t *dst, uint8_t *op, uint64_t at, uint32_t V, uint64_t k,
                 uint8_t o, pcg32_t *g) {
    uint32_t u = (uint32_t)(k / V), v = (uint32_t)(k % V);
    /* endpoint order inside an update is random: the stream does not promise u<v */
    if (g && (pcg32_next(g) & 1u)) { uint32_t t = u; u = v; v = t; }
    src[at] = u;
    dst[at] = v;
    if (op) op[at] = o;
}

static void shuffle_keys(uint64_t *a, uint64_t n, pcg32_t *g) {
    for (uint64_t i = n; i > 1; --i) {
        uint64_t j = rng_below(g, i);
        uint64_t t = a[i - 1]; a[i - 1] = a[j]; a[j] = t;
    }
}

/*
 * Uniform stream: n_ins insertions of uniformly random distinct pairs, then
 * n_del deletions of live edges chosen uniformly without replacement.
 * Output arrays hold n_ins + n_del entries.  Returns 0, or -1 on bad input.
 */
int gen_uniform(uint32_t V, uint64_t n_ins, uint64_t n_del, uint64_t seed,
                uint32_t *src, uint32_t *dst, uint8_t *op) {
    if (V < 2) return -1;
    uint64_t npairs = (uint64_t)V * (V - 1) / 2;
    if (n_ins > npairs || n_del > n_ins) return -1;
    pcg32_t g;
    pcg32_seed(&g, seed, 0x5eed0001ULL);
    liveset_t L;
    if (live_init(&L, V, n_ins)) return -1;
    uint64_t at = 0;
    while (L.nlive < n_ins) {
        uint32_t u = (uint32_t)rng_below(&g, V), v = (uint32_t)rng_below(&g, V);
        if (u == v) continue;
        uint64_t k = key_of(V, u, v);
        if (live_has(&L, k)) continue;
        live_insert(&L, k);
        emit(src, dst, op, at++, V, k, 1, &g);
    }
    for (uint64_t i = 0; i < n_del; ++i) {
        uint64_t k = live_pop_random(&L, &g);
        emit(src, dst, op, at++, V, k, 0, &g);
    }
    live_free(&L);
    return 0;
}

/* ---------------- R-MAT ---------------- */

static uint32_t log2_ceil(uint32_t V) {
    uint32_t L = 0;
    while ((1ULL << L) < V) ++L;
    return L;
}

/* one R-MAT draw over [0, 2^L)^2; returns 0 if it must be rejected */
static int rmat_draw(pcg32_t *g, uint32_t L, uint32_t V, double a, double b, double c,
                     uint32_t *pu, uint32_t *pv) {
    uint32_t u = 0, v = 0;
    for (uint32_t l = 0; l < L; ++l) {
        double x = rng_unit(g);
        uint32_t bu, bv;
        if (x < a) { bu = 0; bv = 0; }
        else if (x < a + b) { bu = 0; bv = 1; }
        else if (x < a + b + c) { bu = 1; bv = 0; }
        else { bu = 1; bv = 1; }
        u = (u << 1) | bu;
        v = (v << 1) | bv;
    }
    if (u == v || u >= V || v >= V) return 0;
    *pu = u;
    *pv = v;
    return 1;
}

static double lfact(int k) { return lgamma((double)k + 1.0); }

/*
 * Poissonised distinct-edge set of an R-MAT process on V = 2^L nodes: the set of
 * distinct pairs seen in Poisson(K) draws includes each unordered pair {u,v}
 * independently with probability 1 - exp(-K * (P(u,v) + P(v,u))), where P is
 * the R-MAT cell probability.  K is solved so the expected set size is
 * `target`.  Pair probabilities depend only on the per-level bit-pattern counts,
 * which makes the expectation a small sum over compositions of L.
 */
static double rmat_expected_edges(uint32_t L, double a, double b, double c, double d, double K) {
    double la = log(a), lb = log(b), lc = log(c), ld = log(d);
    double total = 0.0;
    for (int n01 = 0; n01 <= (int)L; ++n01)
        for (int n10 = 0; n10 + n01 <= (int)L; ++n10) {
            if (n01 + n10 == 0) continue; /* u == v */
            for (int n11 = 0; n11 + n10 + n01 <= (int)L; ++n11) {
                int n00 = (int)L - n01 - n10 - n11;
                double lmult = lfact((int)L) - lfact(n00) - lfact(n01) - lfact(n10) - lfact(n11);
                double p1 = exp(n00 * la + n01 * lb + n10 * lc + n11 * ld);
                double p2 = exp(n00 * la + n10 * lb + n01 * lc + n11 * ld);
                double q = -expm1(-K * (p1 + p2));
                total += 0.5 * exp(lmult) * q; /* ordered pairs -> unordered */
            }
        }
    return total;
}

static double rmat_solve_K(uint32_t L, double a, double b, double c, double d, double target) {
    double lo = 1.0, hi = 1.0;
    while (rmat_expected_edges(L, a, b, c, d, hi) < target) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (rmat_expected_edges(L, a, b, c, d, mid) < target) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

static int popc(uint32_t x) { return __builtin_popcount(x); }

/* fills keys[] with the sampled distinct pairs (u<v), returns count or -1 */
static int64_t rmat_edge_set(uint32_t V, double a, double b, double c, double d, double target,
                             pcg32_t *g, uint64_t *keys, uint64_t cap) {
    uint32_t L = log2_ceil(V);
    if ((1u << L) != V) return -1; /* calibration assumes a power-of-two node count */
    double K = rmat_solve_K(L, a, b, c, d, target);
    int S = (int)L + 1;
    double *q = (double *)malloc(sizeof(double) * S * S * S);
    if (!q) return -1;
    double la = log(a), lb = log(b), lc = log(c), ld = log(d);
    for (int n01 = 0; n01 < S; ++n01)
        for (int n10 = 0; n10 < S; ++n10)
            for (int n11 = 0; n11 < S; ++n11) {
                int n00 = (int)L - n01 - n10 - n11;
                double v = 0.0;
                if (n00 >= 0) {
                    double p1 = exp(n00 * la + n01 * lb + n10 * lc + n11 * ld);
                    double p2 = exp(n00 * la + n10 * lb + n01 * lc + n11 * ld);
                    v = -expm1(-K * (p1 + p2));
                }
                q[(n01 * S + n10) * S + n11] = v;
            }
    uint64_t cnt = 0;
    uint32_t mask = V - 1;
    for (uint32_t v = 1; v < V; ++v)
        for (uint32_t u = 0; u < v; ++u) {
            int n11 = popc(u & v), n01 = popc(~u & v & mask), n10 = popc(u & ~v & mask);
            double p = q[(n01 * S + n10) * S + n11];
            if (rng_unit(g) < p) {
                if (cnt >= cap) { free(q); return -1; }
                keys[cnt++] = (uint64_t)u * V + v;
            }
        }
    free(q);
    return (int64_t)cnt;
}

/*
 * Phased R-MAT stream: about `target_edges` distinct R-MAT edges inserted in
 * random order, then round(del_frac * E) of the live edges deleted, uniformly
 * without replacement, in random order.  `cap` bounds the output length.
 * Returns the number of updates written, or -1.
 */
int64_t gen_rmat_phased(uint32_t V, double a, double b, double c, double d, double target_edges,
                        double del_frac, uint64_t seed, uint32_t *src, uint32_t *dst, uint8_t *op,
                        uint64_t cap) {
    pcg32_t g;
    pcg32_seed(&g, seed, 0x5eed0002ULL);
    uint64_t kcap = (uint64_t)(target_edges * 1.01 + 64.0 * sqrt(target_edges) + 1024);
    uint64_t *keys = (uint64_t *)malloc(kcap * sizeof(uint64_t));
    if (!keys) return -1;
    int64_t E = rmat_edge_set(V, a, b, c, d, target_edges, &g, keys, kcap);
    if (E < 0) { free(keys); return -1; }
    shuffle_keys(keys, (uint64_t)E, &g);
    uint64_t ndel = (uint64_t)llround(del_frac * (double)E);
    if ((uint64_t)E + ndel > cap) { free(keys); return -1; }
    uint64_t at = 0;
    for (int64_t i = 0; i < E; ++i) emit(src, dst, op, at++, V, keys[i], 1, &g);
    /* partial Fisher-Yates: the first ndel keys of a fresh shuffle are a uniform sample */
    for (uint64_t i = 0; i < ndel; ++i) {
        uint64_t j = i + rng_below(&g, (uint64_t)E - i);
        uint64_t t = keys[i]; keys[i] = keys[j]; keys[j] = t;
        emit(src, dst, op, at++, V, keys[i], 0, &g);
    }
    free(keys);
    return (int64_t)at;
}

/*
 * Interleaved R-MAT stream: n_steps steps; at each step, with probability
 * del_prob (and if any edge is live) delete a uniformly chosen live edge,
 * otherwise insert the next edge of a shuffled Poissonised R-MAT edge set.
 * Stops early if the edge set runs out.  Returns updates written, or -1.
 */
int64_t gen_rmat_interleaved(uint32_t V, double a, double b, double c, double d, uint64_t n_steps,
                             double del_prob, uint64_t seed, uint32_t *src, uint32_t *dst,
                             uint8_t *op) {
    pcg32_t g;
    pcg32_seed(&g, seed, 0x5eed0003ULL);
    double target = (1.0 - del_prob) * (double)n_steps * 1.002 + 1024.0;
    uint64_t kcap = (uint64_t)(target * 1.01 + 64.0 * sqrt(target) + 1024);
    uint64_t *keys = (uint64_t *)malloc(kcap * sizeof(uint64_t));
    if (!keys) return -1;
    int64_t E = rmat_edge_set(V, a, b, c, d, target, &g, keys, kcap);
    if (E < 0) { free(keys); return -1; }
    shuffle_keys(keys, (uint64_t)E, &g);
    liveset_t L;
    if (live_init(&L, V, (uint64_t)E)) { free(keys); return -1; }
    uint64_t at = 0, next = 0;
    for (uint64_t s = 0; s < n_steps; ++s) {
        if (L.nlive > 0 && rng_unit(&g) < del_prob) {
            uint64_t k = live_pop_random(&L, &g);
            emit(src, dst, op, at++, V, k, 0, &g);
        } else {
            if (next >= (uint64_t)E) break;
            uint64_t k = keys[next++];
            live_insert(&L, k);
            emit(src, dst, op, at++, V, k, 1, &g);
        }
    }
    live_free(&L);
    free(keys);
    return (int64_t)at;
}

/*
 * G(n,p) stream: every pair included independently with probability p
 * (geometric skipping over the pair order), insertions shuffled, then
 * round(del_frac * E) uniform live deletions, shuffled.  Returns length or -1.
 */
int64_t gen_gnp(uint32_t V, double p, double del_frac, uint64_t seed, uint32_t *src,
                uint32_t *dst, uint8_t *op, uint64_t cap) {
    if (V < 2 || !(p > 0.0) || p >= 1.0) return -1;
    pcg32_t g;
    pcg32_seed(&g, seed, 0x5eed0004ULL);
    uint64_t npairs = (uint64_t)V * (V - 1) / 2;
    uint64_t kcap = cap + 1;
    uint64_t *keys = (uint64_t *)malloc(kcap * sizeof(uint64_t));
    if (!keys) return -1;
    uint64_t E = 0;
    double lq = log1p(-p);
    /* walk the upper triangle row by row: row u holds pairs (u, u+1 .. V-1) */
    uint64_t u = 0, off = 0; /* next candidate is (u, u + 1 + off) */
    (void)npairs;
    for (;;) {
        double r = rng_unit(&g);
        uint64_t skip = (uint64_t)floor(log1p(-r) / lq);
        off += skip;
        while (u + 1 < V && off >= (uint64_t)(V - 1 - u)) { off -= (V - 1 - u); ++u; }
        if (u + 1 >= V) break;
        if (E >= kcap) { free(keys); return -1; }
        keys[E++] = u * V + (u + 1 + off);
        ++off;
    }
    shuffle_keys(keys, E, &g);
    uint64_t ndel = (uint64_t)llround(del_frac * (double)E);
    if (E + ndel > cap) { free(keys); return -1; }
    uint64_t at = 0;
    for (uint64_t i = 0; i < E; ++i) emit(src, dst, op, at++, V, keys[i], 1, &g);
    for (uint64_t i = 0; i < ndel; ++i) {
        uint64_t j = i + rng_below(&g, E - i);
        uint64_t t = keys[i]; keys[i] = keys[j]; keys[j] = t;
        emit(src, dst, op, at++, V, keys[i], 0, &g);
    }
    free(keys);
    return (int64_t)at;
}

/*
 * Session stream for the serving workload: n_updates updates on V nodes; each
 * is a deletion of a uniform live edge with probability del_prob (if any is
 * live), otherwise the insertion of an R-MAT draw that is not live (after
 * max_tries rejected draws: a uniform non-live pair; the number of such
 * fallbacks is returned through *fallbacks).  Returns length or -1.
 */
int64_t gen_rmat_session(uint32_t V, double a, double b, double c, double d, uint64_t n_updates,
                         double del_prob, uint64_t seed, uint32_t *src, uint32_t *dst, uint8_t *op,
                         uint64_t *fallbacks) {
    if (V < 2) return -1;
    pcg32_t g;
    pcg32_seed(&g, seed, 0x5eed0005ULL);
    uint32_t L = log2_ceil(V);
    uint64_t npairs = (uint64_t)V * (V - 1) / 2;
    liveset_t LS;
    if (live_init(&LS, V, n_updates)) return -1;
    uint64_t fb = 0;
    for (uint64_t s = 0; s < n_updates; ++s) {
        if (LS.nlive > 0 && (rng_unit(&g) < del_prob || LS.nlive >= npairs)) {
            uint64_t k = live_pop_random(&LS, &g);
            emit(src, dst, op, s, V, k, 0, &g);
            continue;
        }
        uint64_t k = 0;
        int found = 0;
        for (int t = 0; t < 1024 && !found; ++t) {
            uint32_t u, v;
            if (!rmat_draw(&g, L, V, a, b, c, &u, &v)) continue;
            k = key_of(V, u, v);
            if (!live_has(&LS, k)) found = 1;
        }
        while (!found) {
            uint32_t u = (uint32_t)rng_below(&g, V), v = (uint32_t)rng_below(&g, V);
            if (u == v) continue;
            k = key_of(V, u, v);
            if (!live_has(&LS, k)) { found = 1; ++fb; }
        }
        live_insert(&LS, k);
        emit(src, dst, op, s, V, k, 1, &g);
    }
    live_free(&LS);
    if (fallbacks) *fallbacks = fb;
    return (int64_t)n_updates;
}

/* generic seeded draws the workload layer needs (sizes, batch lengths) */
void gen_uniform_u64(uint64_t seed, uint64_t n, uint64_t lo, uint64_t hi, uint64_t *out) {
    pcg32_t g;
    pcg32_seed(&g, seed, 0x5eed0006ULL);
    for (uint64_t i = 0; i < n; ++i) out[i] = lo + rng_below(&g, hi - lo + 1);
}

void gen_unit_f64(uint64_t seed, uint64_t stream, uint64_t n, double *out) {
    pcg32_t g;
    pcg32_seed(&g, seed, 0x5eed1000ULL + stream);
    for (uint64_t i = 0; i < n; ++i) out[i] = rng_unit(&g);
}

/*
 * Raw R-MAT draws on V = 2^L nodes, for large sparse-in-time streams where a
 * live-edge set would not fit: n updates, each an R-MAT draw with self-loops
 * redrawn; a pair drawn again toggles the edge (the draw is then a deletion
 * under the Z2 view of Sec. 3.1).  The quadrant of each level is chosen from
 * one 32-bit draw against the cumulative thresholds of (a, b, c).  Draws are
 * made in blocks of 2^20, block k from its own PCG32 sequence (seed, k), so
 * the output does not depend on `threads`.  Returns n, or -1.
 */
#include <pthread.h>

typedef struct {
    uint32_t V, L;
    uint32_t ta, tb, tc;
    uint64_t seed, n, block, next;
    uint32_t *src, *dst;
    pthread_mutex_t mu;
} draws_job_t;

static void *draws_worker(void *arg) {
    draws_job_t *J = (draws_job_t *)arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        uint64_t k = J->next++;
        pthread_mutex_unlock(&J->mu);
        uint64_t lo = k * J->block;
        if (lo >= J->n) break;
        uint64_t hi = lo + J->block < J->n ? lo + J->block : J->n;
        pcg32_t g;
        pcg32_seed(&g, J->seed, 0x5eed0007ULL + 2 * k);
        for (uint64_t i = lo; i < hi;) {
            uint32_t u = 0, v = 0;
            for (uint32_t l = 0; l < J->L; ++l) {
                uint32_t x = pcg32_next(&g);
                uint32_t bu = x >= J->tb, bv = (x >= J->ta && x < J->tb) || x >= J->tc;
                u = (u << 1) | bu;
                v = (v << 1) | bv;
            }
            if (u == v) continue;
            if (pcg32_next(&g) & 1u) { uint32_t t = u; u = v; v = t; }
            J->src[i] = u;
            J->dst[i] = v;
            ++i;
        }
    }
    return NULL;
}

int64_t gen_rmat_draws(uint32_t V, double a, double b, double c, uint64_t n, uint64_t seed,
                       uint32_t threads, uint32_t *src, uint32_t *dst) {
    uint32_t L = log2_ceil(V);
    if (V < 2 || (1u << L) != V || a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
    draws_job_t J;
    J.V = V; J.L = L;
    J.ta = (uint32_t)(a * 4294967296.0);
    J.tb = (uint32_t)((a + b) * 4294967296.0);
    J.tc = (uint32_t)((a + b + c) * 4294967296.0);
    J.seed = seed; J.n = n; J.block = 1u << 20; J.next = 0;
    J.src = src; J.dst = dst;
    pthread_mutex_init(&J.mu, NULL);
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    pthread_t tid[64];
    uint32_t started = 0;
    for (uint32_t t = 1; t < threads; ++t)
        if (pthread_create(&tid[started], NULL, draws_worker, &J) == 0) ++started;
    draws_worker(&J);
    for (uint32_t t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    pthread_mutex_destroy(&J.mu);
    return (int64_t)n;
}
