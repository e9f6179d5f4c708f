/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded reference for CubeSketch ingestion and the
 * Boruvka connected-components query of GraphZeppelin (Tench et al., SIGMOD
 * 2022).  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this code.  It shares nothing with the GPU library.
 *
 * Every step follows the paper directly:
 *   - edge index over node pairs: Sec. 2.2 (characteristic vectors);
 *   - CubeSketch update and query: Sec. 3.1, Fig. "cube_code", Eq. (1)-(2) and
 *     the per-bucket result rule that follows them;
 *   - one independent CubeSketch per Boruvka round per node: Sec. 2.2;
 *   - Boruvka rounds (recover an edge per component, merge, sum sketches):
 *     Sec. 2.2 and the three phases of Sec. 4.2.
 *
 * Readings where the paper leaves a choice open (all shared with the GPU side
 * only through this written contract, never through code):
 *   - shape: C = 8 columns, R = bitlen(V-1)+1 rounds, n = V(V-1)/2,
 *     B = bitlen(n-1)+1 rows (Lemma "goodset" needs a row i with
 *     2^(i-2) <= |cut| < 2^(i-1) for every cut up to n edges);
 *   - the row loop of the update stops at row B-1;
 *   - seeds: a SplitMix64 stream started at the graph seed yields, for every
 *     round r, column c and hash k in (h1, h2hi, h2lo), a multiplier then an
 *     increment;
 *   - hash (2-independent, multiply-add-shift): h(x) = ((a*x + b) mod 2^64) >> 32;
 *   - graphs with V > 2^16 ("wide": indices need more than 31 bits) hash the
 *     node pair instead of the index, with the vector form of the same family:
 *     h(u, v) = ((a*u + a2*v + b) mod 2^64) >> 32 for u < v, and their seed
 *     stream yields, per (round, column, hash), a, a2, then b, for four hashes:
 *     row (low word), checksum high, checksum low, row (high word); their row
 *     hash is 64 bits, row_hi * 2^32 + row_lo, since B exceeds 33 rows once
 *     n > 2^32;
 *   - checksum = h2hi(x) * 2^32 + h2lo(x);
 *   - bucket classes: EMPTY (alpha = gamma = 0), GOOD (not EMPTY, gamma equals
 *     the checksum of alpha, alpha < n), otherwise BAD; the query scans columns
 *     in order, rows ascending, returns the first GOOD bucket, else ZERO if all
 *     buckets are EMPTY, else FAIL;
 *   - Boruvka: a GOOD sample whose edge does not leave the component counts as
 *     FAIL; hooks form a functional graph in which every cycle loses the hook
 *     of its smallest component; component labels are the smallest node id.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_C 8

enum { OR_EMPTY = 0, OR_GOOD = 1, OR_BAD = 2 };
enum { OR_ZERO = 0, OR_SAMPLE = 1, OR_FAIL = 2 };
enum { OR_OK = 0, OR_SKETCH_FAIL = 1, OR_EINVAL = -1, OR_ENOMEM = -2 };

/* ---------------------------------------------------------------- shape --- */

static uint32_t bitlen(uint64_t x) {
    uint32_t n = 0;
    while (x) { ++n; x >>= 1; }
    return n;
}

#define ORACLE_MAX_NARROW 65536u
#define ORACLE_MAX_NODES (1u << 24)

int oracle_shape(uint32_t V, uint32_t *R, uint32_t *C, uint32_t *B, uint64_t *n) {
    if (V < 2 || V > ORACLE_MAX_NODES) return OR_EINVAL;
    uint64_t pairs = (uint64_t)V * (uint64_t)(V - 1) / 2;
    *n = pairs;
    *R = bitlen((uint64_t)V - 1) + 1;
    *C = ORACLE_C;
    *B = bitlen(pairs - 1) + 1;
    return OR_OK;
}

int oracle_is_wide(uint32_t V) { return V > ORACLE_MAX_NARROW; }

/* ----------------------------------------------------------- edge index --- */

/* position of pair {u, v}, u < v, in the characteristic vector (Sec. 2.2) */
uint64_t oracle_edge_index(uint32_t u, uint32_t v) {
    if (u > v) { uint32_t t = u; u = v; v = t; }
    return (uint64_t)v * (uint64_t)(v - 1) / 2 + u;
}

/* inverse: the largest v with v(v-1)/2 <= i, found by bisection over v <= 2^25
 * (node ids are below 2^24, and mid*(mid-1) stays far from 2^64) */
void oracle_edge_decode(uint64_t i, uint32_t *u, uint32_t *v) {
    uint64_t lo = 1, hi = (1ull << 25);
    while (lo < hi) {
        uint64_t mid = (lo + hi + 1) / 2;
        if (mid * (mid - 1) / 2 <= i) lo = mid; else hi = mid - 1;
    }
    *v = (uint32_t)lo;
    *u = (uint32_t)(i - lo * (lo - 1) / 2);
}

/* ---------------------------------------------------------------- seeds --- */

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) */
uint64_t oracle_splitmix64_next(uint64_t *state) {
    *state += 0x9E3779B97F4A7C15ull;
    uint64_t z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/*
 * tab[((r*C + c)*3 + k)*2 + 0] = multiplier, [... + 1] = increment,
 * k = 0: row hash h1, k = 1: checksum high word, k = 2: checksum low word.
 */
void oracle_seed_table(uint64_t seed, uint32_t R, uint64_t *tab) {
    uint64_t st = seed;
    for (uint32_t r = 0; r < R; ++r)
        for (uint32_t c = 0; c < ORACLE_C; ++c)
            for (uint32_t k = 0; k < 3; ++k) {
                uint64_t a = oracle_splitmix64_next(&st);
                uint64_t b = oracle_splitmix64_next(&st);
                tab[((r * ORACLE_C + c) * 3 + k) * 2 + 0] = a;
                tab[((r * ORACLE_C + c) * 3 + k) * 2 + 1] = b;
            }
}

/*
 * Wide graphs: tab3[((r*C + c)*4 + k)*3 + j], k = 0: row hash (low word),
 * 1: checksum high word, 2: checksum low word, 3: row hash (high word);
 * j = 0: a (multiplier of the smaller endpoint), 1: a2 (multiplier of the
 * larger endpoint), 2: b.
 */
#define WIDE_HASHES 4
void oracle_seed_table_wide(uint64_t seed, uint32_t R, uint64_t *tab3) {
    uint64_t st = seed;
    for (uint32_t r = 0; r < R; ++r)
        for (uint32_t c = 0; c < ORACLE_C; ++c)
            for (uint32_t k = 0; k < WIDE_HASHES; ++k)
                for (uint32_t j = 0; j < 3; ++j)
                    tab3[((r * ORACLE_C + c) * WIDE_HASHES + k) * 3 + j] = oracle_splitmix64_next(&st);
}

/* ----------------------------------------------------------------- hash --- */

/* multiply-add-shift (Dietzfelbinger 1996): strongly universal for x < 2^32 */
uint32_t oracle_hash32(uint64_t a, uint64_t b, uint64_t x) {
    uint64_t t = a * x + b; /* arithmetic modulo 2^64 */
    return (uint32_t)(t >> 32);
}

/*
 * Vector multiply-add-shift over the pair (u, v), u < v < 2^32: strongly
 * universal into 32 bits because 64 >= 32 + 32 - 1 (Dietzfelbinger 1996;
 * Thorup, High Speed Hashing for Integers and Strings, multiply-shift for
 * vectors).
 */
uint32_t oracle_hash32_pair(uint64_t a, uint64_t a2, uint64_t b, uint32_t u, uint32_t v) {
    uint64_t t = a * (uint64_t)u + a2 * (uint64_t)v + b; /* modulo 2^64 */
    return (uint32_t)(t >> 32);
}

static const uint64_t *seed3_of(const uint64_t *tab3, uint32_t r, uint32_t c, uint32_t k) {
    return tab3 + ((r * ORACLE_C + c) * WIDE_HASHES + k) * 3;
}

/* the 64-bit row hash of a wide graph's pair: row_hi * 2^32 + row_lo */
uint64_t oracle_row_hash_pair(const uint64_t *tab3, uint32_t r, uint32_t c, uint32_t u, uint32_t v) {
    const uint64_t *lo = seed3_of(tab3, r, c, 0);
    const uint64_t *hi = seed3_of(tab3, r, c, 3);
    return ((uint64_t)oracle_hash32_pair(hi[0], hi[1], hi[2], u, v) << 32) |
           (uint64_t)oracle_hash32_pair(lo[0], lo[1], lo[2], u, v);
}

uint64_t oracle_checksum_pair(const uint64_t *tab3, uint32_t r, uint32_t c, uint32_t u, uint32_t v) {
    const uint64_t *hi = seed3_of(tab3, r, c, 1);
    const uint64_t *lo = seed3_of(tab3, r, c, 2);
    return ((uint64_t)oracle_hash32_pair(hi[0], hi[1], hi[2], u, v) << 32) |
           (uint64_t)oracle_hash32_pair(lo[0], lo[1], lo[2], u, v);
}

static const uint64_t *seed_of(const uint64_t *tab, uint32_t r, uint32_t c, uint32_t k) {
    return tab + ((r * ORACLE_C + c) * 3 + k) * 2;
}

uint32_t oracle_row_hash(const uint64_t *tab, uint32_t r, uint32_t c, uint64_t idx) {
    const uint64_t *s = seed_of(tab, r, c, 0);
    return oracle_hash32(s[0], s[1], idx);
}

uint64_t oracle_checksum(const uint64_t *tab, uint32_t r, uint32_t c, uint64_t idx) {
    const uint64_t *hi = seed_of(tab, r, c, 1);
    const uint64_t *lo = seed_of(tab, r, c, 2);
    return ((uint64_t)oracle_hash32(hi[0], hi[1], idx) << 32) |
           (uint64_t)oracle_hash32(lo[0], lo[1], idx);
}

/* ---------------------------------------------------------------- state --- */

typedef struct {
    uint32_t V, R, C, B;
    uint64_t n;
    uint32_t wide;   /* V > 2^16: pair-keyed hashes (tab holds R*C*4*3 words) */
    uint64_t *tab;   /* R*C*3*2 */
    uint64_t *alpha; /* [V][R][C][B] */
    uint64_t *gamma; /* [V][R][C][B] */
} oracle_t;

static size_t slot(const oracle_t *O, uint32_t v, uint32_t r, uint32_t c, uint32_t b) {
    return (((size_t)v * O->R + r) * O->C + c) * O->B + b;
}

/* R_override = 0 keeps the shape rule (tests use a smaller R to force failures) */
oracle_t *oracle_new(uint32_t V, uint64_t seed, uint32_t R_override) {
    uint32_t R, C, B;
    uint64_t n;
    if (oracle_shape(V, &R, &C, &B, &n) != OR_OK) return NULL;
    if (R_override) R = R_override;
    oracle_t *O = (oracle_t *)calloc(1, sizeof(oracle_t));
    if (!O) return NULL;
    O->V = V; O->R = R; O->C = C; O->B = B; O->n = n;
    O->wide = (uint32_t)oracle_is_wide(V);
    O->tab = (uint64_t *)malloc(sizeof(uint64_t) * R * C * (O->wide ? 3 * WIDE_HASHES : 6));
    size_t cells = (size_t)V * R * C * B;
    O->alpha = (uint64_t *)calloc(cells, sizeof(uint64_t));
    O->gamma = (uint64_t *)calloc(cells, sizeof(uint64_t));
    if (!O->tab || !O->alpha || !O->gamma) {
        free(O->tab); free(O->alpha); free(O->gamma); free(O);
        return NULL;
    }
    if (O->wide) oracle_seed_table_wide(seed, R, O->tab);
    else oracle_seed_table(seed, R, O->tab);
    return O;
}

void oracle_free(oracle_t *O) {
    if (!O) return;
    free(O->tab); free(O->alpha); free(O->gamma); free(O);
}

void oracle_dims(const oracle_t *O, uint32_t *dims /* V R C B */, uint64_t *n) {
    dims[0] = O->V; dims[1] = O->R; dims[2] = O->C; dims[3] = O->B;
    *n = O->n;
}

const uint64_t *oracle_seed_ptr(const oracle_t *O) { return O->tab; }
int oracle_wide(const oracle_t *O) { return (int)O->wide; }

/* row hash and checksum of edge {u, v} (u < v, idx its index) under O's contract */
static uint64_t key_row_hash(const oracle_t *O, uint32_t r, uint32_t c, uint64_t idx, uint32_t u,
                             uint32_t v) {
    return O->wide ? oracle_row_hash_pair(O->tab, r, c, u, v) : oracle_row_hash(O->tab, r, c, idx);
}

static uint64_t key_checksum(const oracle_t *O, uint32_t r, uint32_t c, uint64_t idx, uint32_t u,
                             uint32_t v) {
    return O->wide ? oracle_checksum_pair(O->tab, r, c, u, v) : oracle_checksum(O->tab, r, c, idx);
}
uint64_t *oracle_alpha_ptr(oracle_t *O) { return O->alpha; }
uint64_t *oracle_gamma_ptr(oracle_t *O) { return O->gamma; }

/* a seed table whose checksum of index 0 vanishes would make edge 0 unsampleable */
int oracle_seeds_valid(const oracle_t *O) {
    for (uint32_t r = 0; r < O->R; ++r)
        for (uint32_t c = 0; c < O->C; ++c)
            if (key_checksum(O, r, c, 0, 0, 1) == 0) return 0;
    return 1;
}

/* ------------------------------------------------------------ update ------ */

/*
 * Toggle vector index idx in every CubeSketch of node w: for each round and
 * column, row 0 always takes the update and row k+1 takes it while bit k of
 * the row hash is zero (Fig. "cube_code"), here bounded by the B rows.
 */
static void toggle(oracle_t *O, uint32_t w, uint64_t idx, uint32_t u, uint32_t v) {
    for (uint32_t r = 0; r < O->R; ++r)
        for (uint32_t c = 0; c < O->C; ++c) {
            uint64_t col_hash = key_row_hash(O, r, c, idx, u, v);
            uint64_t checksum = key_checksum(O, r, c, idx, u, v);
            uint32_t row = 0;
            while (row < O->B && (row == 0 || ((col_hash >> (row - 1)) & 1u) == 0)) {
                O->alpha[slot(O, w, r, c, row)] ^= idx;
                O->gamma[slot(O, w, r, c, row)] ^= checksum;
                ++row;
            }
        }
}

/* one stream update: each endpoint's characteristic vector flips index (u,v) */
int oracle_update(oracle_t *O, uint32_t u, uint32_t v) {
    if (u == v || u >= O->V || v >= O->V) return OR_EINVAL;
    uint64_t idx = oracle_edge_index(u, v);
    uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
    toggle(O, u, idx, lo, hi);
    toggle(O, v, idx, lo, hi);
    return OR_OK;
}

/* whole stream, validated first so that a bad update applies nothing */
int oracle_ingest(oracle_t *O, const uint32_t *src, const uint32_t *dst, uint64_t N) {
    for (uint64_t i = 0; i < N; ++i)
        if (src[i] == dst[i] || src[i] >= O->V || dst[i] >= O->V) return OR_EINVAL;
    for (uint64_t i = 0; i < N; ++i) oracle_update(O, src[i], dst[i]);
    return OR_OK;
}

/* same, but only the endpoints w with keep[w] != 0 are updated */
int oracle_ingest_nodes(oracle_t *O, const uint32_t *src, const uint32_t *dst, uint64_t N,
                        const uint8_t *keep) {
    for (uint64_t i = 0; i < N; ++i)
        if (src[i] == dst[i] || src[i] >= O->V || dst[i] >= O->V) return OR_EINVAL;
    for (uint64_t i = 0; i < N; ++i) {
        uint64_t idx = oracle_edge_index(src[i], dst[i]);
        uint32_t lo = src[i] < dst[i] ? src[i] : dst[i], hi = src[i] < dst[i] ? dst[i] : src[i];
        if (keep[src[i]]) toggle(O, src[i], idx, lo, hi);
        if (keep[dst[i]]) toggle(O, dst[i], idx, lo, hi);
    }
    return OR_OK;
}

/* -------------------------------------------------------------- query ----- */

int oracle_bucket_class(const uint64_t *tab, uint32_t r, uint32_t c, uint64_t n, uint64_t alpha,
                        uint64_t gamma) {
    if (alpha == 0 && gamma == 0) return OR_EMPTY;
    if (alpha < n && gamma == oracle_checksum(tab, r, c, alpha)) return OR_GOOD;
    return OR_BAD;
}

/* wide graphs: the checksum of the pair alpha encodes */
int oracle_bucket_class_wide(const uint64_t *tab3, uint32_t r, uint32_t c, uint64_t n,
                             uint64_t alpha, uint64_t gamma) {
    if (alpha == 0 && gamma == 0) return OR_EMPTY;
    if (alpha < n) {
        uint32_t u, v;
        oracle_edge_decode(alpha, &u, &v);
        if (gamma == oracle_checksum_pair(tab3, r, c, u, v)) return OR_GOOD;
    }
    return OR_BAD;
}

/*
 * Query one CubeSketch given as alpha[C][B], gamma[C][B] (round r's seeds):
 * columns in order, rows ascending, first GOOD bucket wins.
 */
static int query_sketch(const uint64_t *tab, int wide, uint32_t r, uint32_t C, uint32_t B,
                        uint64_t n, const uint64_t *alpha, const uint64_t *gamma,
                        uint64_t *out_idx) {
    int all_empty = 1;
    for (uint32_t c = 0; c < C; ++c)
        for (uint32_t b = 0; b < B; ++b) {
            int k = wide ? oracle_bucket_class_wide(tab, r, c, n, alpha[c * B + b], gamma[c * B + b])
                         : oracle_bucket_class(tab, r, c, n, alpha[c * B + b], gamma[c * B + b]);
            if (k == OR_GOOD) { *out_idx = alpha[c * B + b]; return OR_SAMPLE; }
            if (k != OR_EMPTY) all_empty = 0;
        }
    return all_empty ? OR_ZERO : OR_FAIL;
}

int oracle_query(const uint64_t *tab, uint32_t r, uint32_t C, uint32_t B, uint64_t n,
                 const uint64_t *alpha, const uint64_t *gamma, uint64_t *out_idx) {
    return query_sketch(tab, 0, r, C, B, n, alpha, gamma, out_idx);
}

int oracle_query_wide(const uint64_t *tab3, uint32_t r, uint32_t C, uint32_t B, uint64_t n,
                      const uint64_t *alpha, const uint64_t *gamma, uint64_t *out_idx) {
    return query_sketch(tab3, 1, r, C, B, n, alpha, gamma, out_idx);
}

/* query node v's round-r CubeSketch */
int oracle_query_node(const oracle_t *O, uint32_t v, uint32_t r, uint64_t *out_idx) {
    return query_sketch(O->tab, (int)O->wide, r, O->C, O->B, O->n, O->alpha + slot(O, v, r, 0, 0),
                        O->gamma + slot(O, v, r, 0, 0), out_idx);
}

/* ------------------------------------------------------------ boruvka ----- */

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/*
 * Spanning forest and components.  labels[V] receives the smallest node id of
 * each node's component; forest[2*(V-1)] receives (u, v) pairs, u < v, sorted
 * by edge index; *nforest the number of pairs.  Returns OR_OK, or
 * OR_SKETCH_FAIL if some component was still active when the rounds ran out
 * (labels and forest are still written).  The sketches are not modified.
 */
int oracle_connected_components(const oracle_t *O, uint32_t *labels, uint32_t *forest,
                                 uint64_t *nforest, uint32_t *rounds_used) {
    uint32_t V = O->V, C = O->C, B = O->B;
    uint32_t *comp = (uint32_t *)malloc(sizeof(uint32_t) * V);
    uint8_t *done = (uint8_t *)calloc(V, 1);
    int64_t *hook = (int64_t *)malloc(sizeof(int64_t) * V);
    uint64_t *hedge = (uint64_t *)malloc(sizeof(uint64_t) * V);
    uint8_t *color = (uint8_t *)malloc(V);
    uint32_t *path = (uint32_t *)malloc(sizeof(uint32_t) * (V + 1));
    uint32_t *root = (uint32_t *)malloc(sizeof(uint32_t) * V);
    uint32_t *newlab = (uint32_t *)malloc(sizeof(uint32_t) * V);
    uint8_t *merged = (uint8_t *)malloc(V);
    uint64_t *acc_a = (uint64_t *)malloc(sizeof(uint64_t) * C * B);
    uint64_t *acc_g = (uint64_t *)malloc(sizeof(uint64_t) * C * B);
    uint64_t *fidx = (uint64_t *)malloc(sizeof(uint64_t) * (V ? V : 1));
    uint32_t *first = (uint32_t *)malloc(sizeof(uint32_t) * (V + 1)); /* members by label */
    uint32_t *members = (uint32_t *)malloc(sizeof(uint32_t) * V);
    if (!comp || !done || !hook || !hedge || !color || !path || !root || !newlab || !merged ||
        !acc_a || !acc_g || !fidx || !first || !members) {
        free(comp); free(done); free(hook); free(hedge); free(color); free(path); free(root);
        free(newlab); free(merged); free(acc_a); free(acc_g); free(fidx); free(first);
        free(members);
        return OR_ENOMEM;
    }
    for (uint32_t v = 0; v < V; ++v) comp[v] = v;
    uint64_t nf = 0;
    int status = OR_SKETCH_FAIL;
    uint32_t used = 0;

    for (uint32_t r = 0; r < O->R; ++r) {
        int active = 0;
        for (uint32_t X = 0; X < V; ++X)
            if (comp[X] == X && !done[X]) active = 1;
        if (!active) { status = OR_OK; break; }
        used = r + 1;

        /* members of every component, listed by label (a counting sort of node ids) */
        memset(first, 0, sizeof(uint32_t) * (V + 1));
        for (uint32_t v = 0; v < V; ++v) first[comp[v] + 1]++;
        for (uint32_t X = 0; X < V; ++X) first[X + 1] += first[X];
        for (uint32_t v = 0; v < V; ++v) members[first[comp[v]]++] = v;
        for (uint32_t X = V; X > 0; --X) first[X] = first[X - 1];
        first[0] = 0;

        /* phase 1: one sample per active component from the XOR of its members */
        for (uint32_t X = 0; X < V; ++X) hook[X] = -1;
        for (uint32_t X = 0; X < V; ++X) {
            if (comp[X] != X || done[X]) continue;
            memset(acc_a, 0, sizeof(uint64_t) * C * B);
            memset(acc_g, 0, sizeof(uint64_t) * C * B);
            for (uint32_t m = first[X]; m < first[X + 1]; ++m) {
                const uint32_t v = members[m];
                for (uint32_t c = 0; c < C; ++c)
                    for (uint32_t b = 0; b < B; ++b) {
                        acc_a[c * B + b] ^= O->alpha[slot(O, v, r, c, b)];
                        acc_g[c * B + b] ^= O->gamma[slot(O, v, r, c, b)];
                    }
            }
            uint64_t idx = 0;
            int q = query_sketch(O->tab, (int)O->wide, r, C, B, O->n, acc_a, acc_g, &idx);
            if (q == OR_ZERO) { done[X] = 1; continue; }
            if (q == OR_FAIL) continue;
            uint32_t a, b;
            oracle_edge_decode(idx, &a, &b);
            int ina = comp[a] == X, inb = comp[b] == X;
            if (ina == inb) continue; /* sampled edge does not leave X: treated as FAIL */
            hook[X] = ina ? comp[b] : comp[a];
            hedge[X] = idx;
        }

        /* phase 2: break every hook cycle at its smallest component, merge */
        memset(color, 0, V);
        for (uint32_t X = 0; X < V; ++X) {
            if (comp[X] != X || color[X]) continue;
            uint32_t len = 0;
            int64_t y = X;
            while (hook[y] >= 0 && color[y] == 0) {
                color[y] = 1;
                path[len++] = (uint32_t)y;
                y = hook[y];
            }
            if (hook[y] >= 0 && color[y] == 1) {
                /* y lies on a cycle made of the tail of this path */
                uint32_t start = 0;
                while (path[start] != (uint32_t)y) ++start;
                uint32_t m = path[start];
                for (uint32_t k = start; k < len; ++k)
                    if (path[k] < m) m = path[k];
                hook[m] = -1;
            }
            for (uint32_t k = 0; k < len; ++k) color[path[k]] = 2;
            color[y] = 2;
        }
        for (uint32_t X = 0; X < V; ++X) {
            if (comp[X] != X) continue;
            uint32_t y = X;
            while (hook[y] >= 0) y = (uint32_t)hook[y];
            root[X] = y;
        }
        for (uint32_t X = 0; X < V; ++X) { newlab[X] = UINT32_MAX; merged[X] = 0; }
        for (uint32_t X = 0; X < V; ++X) {
            if (comp[X] != X) continue;
            if (X < newlab[root[X]]) newlab[root[X]] = X;
            if (hook[X] >= 0) {
                merged[root[X]] = 1;
                fidx[nf++] = hedge[X];
            }
        }
        /* phase 3 is implicit: the next round XORs members by their new label */
        uint8_t *was_done = (uint8_t *)malloc(V);
        memcpy(was_done, done, V);
        for (uint32_t X = 0; X < V; ++X) done[X] = 0;
        for (uint32_t X = 0; X < V; ++X) {
            if (comp[X] != X) continue;
            uint32_t L = newlab[root[X]];
            if (!merged[root[X]] && was_done[X]) done[L] = 1;
        }
        free(was_done);
        for (uint32_t v = 0; v < V; ++v) comp[v] = newlab[root[comp[v]]];
    }
    if (status != OR_OK) {
        int active = 0;
        for (uint32_t X = 0; X < V; ++X)
            if (comp[X] == X && !done[X]) active = 1;
        if (!active) status = OR_OK;
    }

    qsort(fidx, nf, sizeof(uint64_t), cmp_u64);
    for (uint64_t k = 0; k < nf; ++k) {
        uint32_t a, b;
        oracle_edge_decode(fidx[k], &a, &b);
        forest[2 * k] = a;
        forest[2 * k + 1] = b;
    }
    *nforest = nf;
    if (rounds_used) *rounds_used = used;
    memcpy(labels, comp, sizeof(uint32_t) * V);
    free(comp); free(done); free(hook); free(hedge); free(color); free(path); free(root);
    free(newlab); free(merged); free(acc_a); free(acc_g); free(fidx); free(first); free(members);
    return status;
}
