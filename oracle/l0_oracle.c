/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * The standard l0-sampler that GraphZeppelin compares CubeSketch against
 * (Tench et al., SIGMOD 2022, Sec. 3, Fig. "agm_code"; the sampler of Cormode
 * and Firmani as used by Ahn, Guha and McGregor), applied to the node vectors
 * of a graph stream.  Plain and slow; only the test suite and the benchmark's
 * CPU leg may load it, and it shares nothing with the GPU library.
 *
 * What it computes, following Fig. "agm_code":
 *   - a sketch is a matrix of buckets, columns c = 0..C-1, rows 0..B-1; a
 *     bucket holds a (sum of index times Delta), b (sum of Delta) and a
 *     checksum c (sum of Delta * z^index modulo a prime p);
 *   - update (index, Delta): for every column, row 0 always takes it and row
 *     k+1 takes it while bit k of the column's hash of the index is zero;
 *   - query: scan columns, then rows; a bucket passes when b divides a, the
 *     quotient v is a valid index and c = b * z^v (mod p); the first passing
 *     bucket yields (v, b).  All buckets zero means the vector is zero.
 *
 * Readings (the figure leaves them open), written out here and nowhere else
 * shared with the GPU side:
 *   - shape as the CubeSketch oracle: C = 8 columns, R = bitlen(V-1)+1 rounds
 *     (one sampler per Boruvka round per node, Sec. 2.2), B = bitlen(n-1)+1
 *     rows, n = V(V-1)/2, 2 <= V <= 65536;
 *   - the column hash is the CubeSketch row hash of the same round and column
 *     (multiply-add-shift, seeds from the SplitMix64 table), and the row loop
 *     stops at row B-1;
 *   - p = 2^61 - 1 (prime); the column's base z = 1 + (m mod (p-1)), m the
 *     checksum-high multiplier of the round and column in the seed table;
 *   - node vectors: edge {u, v}, u < v, at index v(v-1)/2 + u carries +Delta
 *     in u's vector and -Delta in v's, so the vectors of a node set sum to its
 *     cut (edges inside cancel); Delta = +1 for an insertion, -1 for a
 *     deletion;
 *   - a passing bucket also needs b != 0; a bucket of b = 0 that is not all
 *     zero fails.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define L0_C 8
#define L0_P 2305843009213693951ull /* 2^61 - 1 */

enum { L0_ZERO = 0, L0_SAMPLE = 1, L0_FAIL = 2 };

static uint32_t l0_bitlen(uint64_t x) {
    uint32_t n = 0;
    while (x) { ++n; x >>= 1; }
    return n;
}

static uint64_t l0_splitmix64(uint64_t *s) {
    *s += 0x9E3779B97F4A7C15ull;
    uint64_t z = *s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* x * y mod p, x and y < p, through a 128-bit product */
uint64_t l0_mulmod(uint64_t x, uint64_t y) {
    unsigned __int128 t = (unsigned __int128)x * y;
    return (uint64_t)(t % L0_P);
}

/* z^e mod p by square and multiply */
uint64_t l0_powmod(uint64_t z, uint64_t e) {
    uint64_t r = 1, b = z % L0_P;
    while (e) {
        if (e & 1) r = l0_mulmod(r, b);
        b = l0_mulmod(b, b);
        e >>= 1;
    }
    return r;
}

typedef struct {
    uint32_t V, R, C, B;
    uint64_t n;
    uint64_t *hash;  /* [R][C][2]: row-hash multiplier, increment */
    uint64_t *z;     /* [R][C] */
    int64_t *a;      /* [V][R][C][B] */
    int64_t *b;
    uint64_t *c;
} l0_t;

static size_t l0_slot(const l0_t *S, uint32_t v, uint32_t r, uint32_t c, uint32_t row) {
    return (((size_t)v * S->R + r) * S->C + c) * S->B + row;
}

l0_t *l0_new(uint32_t V, uint64_t seed) {
    if (V < 2 || V > 65536) return NULL;
    l0_t *S = (l0_t *)calloc(1, sizeof(l0_t));
    if (!S) return NULL;
    S->V = V;
    S->n = (uint64_t)V * (V - 1) / 2;
    S->R = l0_bitlen(V - 1) + 1;
    S->C = L0_C;
    S->B = l0_bitlen(S->n - 1) + 1;
    S->hash = (uint64_t *)malloc(sizeof(uint64_t) * S->R * S->C * 2);
    S->z = (uint64_t *)malloc(sizeof(uint64_t) * S->R * S->C);
    size_t cells = (size_t)V * S->R * S->C * S->B;
    S->a = (int64_t *)calloc(cells, sizeof(int64_t));
    S->b = (int64_t *)calloc(cells, sizeof(int64_t));
    S->c = (uint64_t *)calloc(cells, sizeof(uint64_t));
    if (!S->hash || !S->z || !S->a || !S->b || !S->c) {
        free(S->hash); free(S->z); free(S->a); free(S->b); free(S->c); free(S);
        return NULL;
    }
    /* the CubeSketch seed stream: per (round, column), three hashes of
       (multiplier, increment): row hash, checksum high, checksum low */
    uint64_t st = seed;
    for (uint32_t r = 0; r < S->R; ++r)
        for (uint32_t c = 0; c < S->C; ++c) {
            uint64_t w[6];
            for (int k = 0; k < 6; ++k) w[k] = l0_splitmix64(&st);
            S->hash[(r * S->C + c) * 2 + 0] = w[0];
            S->hash[(r * S->C + c) * 2 + 1] = w[1];
            S->z[r * S->C + c] = 1 + w[2] % (L0_P - 1);
        }
    return S;
}

void l0_free(l0_t *S) {
    if (!S) return;
    free(S->hash); free(S->z); free(S->a); free(S->b); free(S->c); free(S);
}

void l0_dims(const l0_t *S, uint32_t *dims, uint64_t *n) {
    dims[0] = S->V; dims[1] = S->R; dims[2] = S->C; dims[3] = S->B;
    *n = S->n;
}
int64_t *l0_a_ptr(l0_t *S) { return S->a; }
int64_t *l0_b_ptr(l0_t *S) { return S->b; }
uint64_t *l0_c_ptr(l0_t *S) { return S->c; }
const uint64_t *l0_z_ptr(const l0_t *S) { return S->z; }

static uint32_t l0_col_hash(const l0_t *S, uint32_t r, uint32_t c, uint64_t idx) {
    const uint64_t *h = S->hash + (r * S->C + c) * 2;
    return (uint32_t)((h[0] * idx + h[1]) >> 32);
}

/* Fig. "agm_code" update of node w's samplers by (idx, delta) */
static void l0_apply(l0_t *S, uint32_t w, uint64_t idx, int64_t delta) {
    for (uint32_t r = 0; r < S->R; ++r)
        for (uint32_t c = 0; c < S->C; ++c) {
            uint32_t col_hash = l0_col_hash(S, r, c, idx);
            uint64_t chk = l0_powmod(S->z[r * S->C + c], idx);
            uint64_t dchk = delta > 0 ? chk : (chk ? L0_P - chk : 0);
            uint32_t row = 0;
            while (row < S->B && (row == 0 || ((col_hash >> (row - 1)) & 1u) == 0)) {
                size_t k = l0_slot(S, w, r, c, row);
                S->a[k] += (int64_t)idx * delta;
                S->b[k] += delta;
                S->c[k] = (S->c[k] + dchk) % L0_P;
                ++row;
            }
        }
}

int l0_update(l0_t *S, uint32_t u, uint32_t v, int delta) {
    if (u == v || u >= S->V || v >= S->V || (delta != 1 && delta != -1)) return -1;
    uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
    uint64_t idx = (uint64_t)hi * (hi - 1) / 2 + lo;
    l0_apply(S, lo, idx, delta);
    l0_apply(S, hi, idx, -delta);
    return 0;
}

/* op[k] = 1 inserts (Delta = +1), 0 deletes (Delta = -1); op NULL: all insertions */
int l0_ingest(l0_t *S, const uint32_t *src, const uint32_t *dst, const uint8_t *op, uint64_t N) {
    for (uint64_t i = 0; i < N; ++i)
        if (src[i] == dst[i] || src[i] >= S->V || dst[i] >= S->V) return -1;
    for (uint64_t i = 0; i < N; ++i) l0_update(S, src[i], dst[i], (!op || op[i]) ? 1 : -1);
    return 0;
}

/* only the endpoint halves whose node has keep[w] != 0 */
int l0_ingest_nodes(l0_t *S, const uint32_t *src, const uint32_t *dst, const uint8_t *op,
                    uint64_t N, const uint8_t *keep) {
    for (uint64_t i = 0; i < N; ++i)
        if (src[i] == dst[i] || src[i] >= S->V || dst[i] >= S->V) return -1;
    for (uint64_t i = 0; i < N; ++i) {
        uint32_t lo = src[i] < dst[i] ? src[i] : dst[i], hi = src[i] < dst[i] ? dst[i] : src[i];
        uint64_t idx = (uint64_t)hi * (hi - 1) / 2 + lo;
        int64_t delta = (!op || op[i]) ? 1 : -1;
        if (keep[lo]) l0_apply(S, lo, idx, delta);
        if (keep[hi]) l0_apply(S, hi, idx, -delta);
    }
    return 0;
}

/*
 * Query one sampler given as a[C][B], b[C][B], c[C][B] with round r's
 * seeds: columns in order, rows ascending, the first passing bucket wins.
 */
int l0_query(const l0_t *S, uint32_t r, const int64_t *a, const int64_t *b, const uint64_t *c,
             uint64_t *out_idx, int64_t *out_mult) {
    int all_zero = 1;
    for (uint32_t col = 0; col < S->C; ++col)
        for (uint32_t row = 0; row < S->B; ++row) {
            size_t k = (size_t)col * S->B + row;
            if (a[k] == 0 && b[k] == 0 && c[k] == 0) continue;
            all_zero = 0;
            if (b[k] == 0 || a[k] % b[k] != 0) continue;
            int64_t v = a[k] / b[k];
            if (v < 0 || (uint64_t)v >= S->n) continue;
            uint64_t bm = b[k] > 0 ? (uint64_t)b[k] % L0_P : L0_P - (uint64_t)(-b[k]) % L0_P;
            if (bm == L0_P) bm = 0;
            if (c[k] == l0_mulmod(bm, l0_powmod(S->z[r * S->C + col], (uint64_t)v))) {
                *out_idx = (uint64_t)v;
                *out_mult = b[k];
                return L0_SAMPLE;
            }
        }
    return all_zero ? L0_ZERO : L0_FAIL;
}

int l0_query_node(const l0_t *S, uint32_t v, uint32_t r, uint64_t *out_idx, int64_t *out_mult) {
    size_t k = l0_slot(S, v, r, 0, 0);
    return l0_query(S, r, S->a + k, S->b + k, S->c + k, out_idx, out_mult);
}
