"""Pins of the CPU oracle against facts fixed outside it (paper and mathematics).

Each test names the passage it relies on.  None of these needs a GPU.
"""
import itertools
import json
import math
import os
import random

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


# ----------------------------------------------------------------- shape ---

def test_shape_rule_closed_form(built):
    """R = ceil(log2 V) + 1, B = ceil(log2 n) + 1 with n = C(V, 2), C = 8.

    The small uniform workload states R = 11 and B = 20 for V = 1024 and the dense
    R-MAT workload states R = 15 for V = 2^14; the rest is the closed form.
    """
    assert oracle.shape(1024)[:3] == (11, 8, 20)
    assert oracle.shape(1 << 14)[0] == 15
    for V in [2, 3, 4, 5, 63, 64, 65, 1000, 1024, 1025, 2048, 1 << 14, 1 << 15, 1 << 16]:
        R, C, B, n = oracle.shape(V)
        assert n == V * (V - 1) // 2
        assert C == 8
        # smallest k with 2^k >= V, by exact integer search
        k = 0
        while (1 << k) < V:
            k += 1
        assert R == k + 1
        k = 0
        while (1 << k) < n:
            k += 1
        assert B == k + 1
        assert B <= 32  # row hash has 32 bits


def test_shape_rejects_out_of_range(built):
    for V in [0, 1, (1 << 24) + 1]:
        with pytest.raises(ValueError):
            oracle.shape(V)


# ------------------------------------------------------------ edge index ---

def test_edge_index_is_a_bijection_onto_pairs(built):
    """Sec. 2.2: characteristic vectors are indexed by the C(V,2) node pairs."""
    for V in [2, 3, 7, 64, 181]:
        n = V * (V - 1) // 2
        seen = np.zeros(n, bool)
        for v in range(V):
            for u in range(v):
                i = oracle.edge_index(u, v)
                assert oracle.edge_index(v, u) == i
                assert 0 <= i < n and not seen[i]
                seen[i] = True
                assert oracle.edge_decode(i) == (u, v)
        assert seen.all()


def test_edge_decode_extremes(built):
    V = 1 << 16
    n = V * (V - 1) // 2
    rng = random.Random(7)
    probes = [0, 1, 2, n - 1, n - 2] + [rng.randrange(n) for _ in range(2000)]
    for i in probes:
        u, v = oracle.edge_decode(i)
        # the row is fixed by the triangular numbers: v(v-1)/2 <= i < v(v+1)/2
        assert v * (v - 1) // 2 <= i < v * (v + 1) // 2
        assert 0 <= u < v < V
        assert oracle.edge_index(u, v) == i


# ----------------------------------------------------------------- seeds ---

def test_splitmix64_known_answer(built):
    kat = json.load(open(os.path.join(GOLDEN, "splitmix64_kat.json")))
    assert oracle.splitmix64(kat["seed"], len(kat["outputs"])) == kat["outputs"]


def test_seed_table_is_the_splitmix_stream_in_round_column_hash_order(built):
    R = 5
    tab = oracle.seed_table(1234567, R)
    stream = oracle.splitmix64(1234567, R * 8 * 6)
    assert tab.reshape(-1).tolist() == stream


def test_seed_table_prefix_independent_of_round_count(built):
    a = oracle.seed_table(99, 7)
    b = oracle.seed_table(99, 12)
    assert (a == b[:7]).all()


# ------------------------------------------------------------------ hash ---

def test_hash_depth_law(built):
    """Row membership: h1(e) = 0 mod 2^k with probability 2^-k (Sec. 3.1)."""
    O = oracle.Oracle(1 << 14, seed=2024)
    counts = np.zeros(12)
    rng = np.random.default_rng(1)
    xs = rng.integers(0, O.n, 20000)
    total = 0
    for r, c in [(0, 0), (3, 5), (14, 7)]:
        for x in xs.tolist():
            h = O.row_hash(r, c, x)
            tz = (h & -h).bit_length() - 1 if h else 32
            for k in range(12):
                if tz >= k:
                    counts[k] += 1
            total += 1
    for k in range(12):
        p = counts[k] / total
        expect = 2.0 ** -k
        sd = math.sqrt(expect * (1 - expect) / total)
        assert abs(p - expect) < 6 * sd + 1e-12, (k, p, expect)


@pytest.mark.parametrize("x,y", [(0, 1), (2, 6), (4, 12), (1 << 20, (1 << 20) + 2), (123456, 7654321)])
def test_hash_pairwise_uniform(built, x, y):
    """2-wise independence (Sec. 3.1): over random seeds, (h(x), h(y)) low bits are uniform."""
    rng = random.Random(x * 31 + y)
    cells = np.zeros(16)
    trials = 16000
    for _ in range(trials):
        a, b = rng.getrandbits(64), rng.getrandbits(64)
        hx, hy = oracle.hash32(a, b, x), oracle.hash32(a, b, y)
        cells[(hx & 3) * 4 + (hy & 3)] += 1
    exp = trials / 16
    chi2 = float(((cells - exp) ** 2 / exp).sum())
    assert chi2 < 45.0, chi2  # 15 dof; p ~ 1e-4


def test_checksum_of_zero_nonzero(built):
    """Edge index 0 must stay sampleable: its checksum may not vanish."""
    for seed in range(50):
        O = oracle.Oracle(64, seed)
        assert O.seeds_valid()


# ---------------------------------------------------------------- sketch ---

def _py_hash(a, b, x):
    return ((a * x + b) & M64) >> 32


def _closed_form(V, seed, edges):
    """Eq. (1)-(2): bucket (r, c, b) of node w XORs every final incident edge in it."""
    R, C, B, n = oracle.shape(V)
    tab = oracle.seed_table(seed, R)
    al = np.zeros((V, R, C, B), np.uint64)
    ga = np.zeros((V, R, C, B), np.uint64)
    for (u, v) in edges:
        i = v * (v - 1) // 2 + u
        for r in range(R):
            for c in range(C):
                (a1, b1), (ah, bh), (alo, blo) = [tuple(int(t) for t in tab[r, c, k]) for k in range(3)]
                h1 = _py_hash(a1, b1, i)
                chk = (_py_hash(ah, bh, i) << 32) | _py_hash(alo, blo, i)
                for b in range(B):
                    # e is in row b when h1(e) = 0 mod 2^b; the last row also keeps deeper ones
                    if h1 % (1 << b) == 0:
                        for w in (u, v):
                            al[w, r, c, b] ^= np.uint64(i)
                            ga[w, r, c, b] ^= np.uint64(chk)
    return al, ga


def _random_toggle_stream(V, n, rng):
    src, dst = [], []
    for _ in range(n):
        u, v = rng.sample(range(V), 2)
        src.append(u)
        dst.append(v)
    return np.array(src, np.uint32), np.array(dst, np.uint32)


def test_sketch_equals_closed_form_eq_1_2(built):
    rng = random.Random(3)
    for V, n, seed in [(2, 5, 1), (9, 60, 2), (23, 400, 3)]:
        src, dst = _random_toggle_stream(V, n, rng)
        O = oracle.Oracle(V, seed)
        O.ingest(src, dst)
        s = workloads.Stream(V, src, dst, np.ones(len(src), np.uint8))
        fu, fv = workloads.final_edges(s)
        al, ga = _closed_form(V, seed, list(zip(fu.tolist(), fv.tolist())))
        assert (O.alpha == al).all()
        assert (O.gamma == ga).all()


def test_sketch_independent_of_stream_order(built):
    rng = random.Random(5)
    src, dst = _random_toggle_stream(40, 3000, rng)
    perm = np.random.default_rng(0).permutation(len(src))
    A = oracle.Oracle(40, 77)
    A.ingest(src, dst)
    Bo = oracle.Oracle(40, 77)
    Bo.ingest(dst[perm], src[perm])  # endpoint order flipped as well
    assert (A.alpha == Bo.alpha).all() and (A.gamma == Bo.gamma).all()


def test_linearity_xor(built):
    """S(A) xor S(B) = S(A symmetric-difference B) (Sec. 3.1, linearity by XOR)."""
    rng = random.Random(11)
    V = 30
    sa, da = _random_toggle_stream(V, 500, rng)
    sb, db = _random_toggle_stream(V, 700, rng)
    A, Bo, AB = oracle.Oracle(V, 5), oracle.Oracle(V, 5), oracle.Oracle(V, 5)
    A.ingest(sa, da)
    Bo.ingest(sb, db)
    AB.ingest(np.concatenate([sa, sb]), np.concatenate([da, db]))
    assert ((A.alpha ^ Bo.alpha) == AB.alpha).all()
    assert ((A.gamma ^ Bo.gamma) == AB.gamma).all()


def test_support_one_exact_recovery(built):
    """Lemma goodcheck: a bucket holding one nonzero entry always passes."""
    V = 1 << 12
    rng = random.Random(2)
    for trial in range(20):
        u, v = rng.sample(range(V), 2)
        O = oracle.Oracle(V, 1000 + trial)
        O.update(u, v)
        i = oracle.edge_index(u, v)
        for w in (u, v):
            for r in range(O.R):
                kind, got = O.query_node(w, r)
                assert kind == oracle.SAMPLE and got == i
                for c in range(O.C):
                    h = O.row_hash(r, c, i)
                    depth = min(((h & -h).bit_length() - 1) if h else 32, O.B - 1)
                    chk = O.checksum(r, c, i)
                    for b in range(O.B):
                        if b <= depth:
                            assert O.alpha[w, r, c, b] == i and O.gamma[w, r, c, b] == chk
                        else:
                            assert O.alpha[w, r, c, b] == 0 and O.gamma[w, r, c, b] == 0
        # every other node is untouched: ZERO
        other = next(x for x in range(V) if x not in (u, v))
        assert O.query_node(other, 0)[0] == oracle.ZERO
    # edge index 0 (pair (0, 1)) has alpha = 0 but is still recovered
    O = oracle.Oracle(V, 3)
    O.update(0, 1)
    assert O.query_node(0, 0) == (oracle.SAMPLE, 0)


def test_sampled_index_in_support_and_goodset_bound(built):
    """Lemma goodcheck (sample is in the support) and Lemma goodset (per column > 1/8)."""
    V = 600
    rng = random.Random(9)
    fails = 0
    col_good = 0
    col_total = 0
    for trial in range(60):
        deg = rng.choice([1, 2, 3, 5, 9, 17, 40, 120, 400])
        nbrs = rng.sample(range(1, V), deg)
        O = oracle.Oracle(V, 5000 + trial)
        O.ingest(np.zeros(deg, np.uint32), np.array(nbrs, np.uint32))
        support = {oracle.edge_index(0, x) for x in nbrs}
        for r in range(O.R):
            kind, got = O.query_node(0, r)
            if kind == oracle.SAMPLE:
                assert got in support
            else:
                assert kind == oracle.FAIL
                fails += 1
            for c in range(O.C):
                col_total += 1
                good = False
                for b in range(O.B):
                    k = O.bucket_class(r, c, int(O.alpha[0, r, c, b]), int(O.gamma[0, r, c, b]))
                    if k == oracle.GOOD:
                        # a GOOD bucket holds exactly one member (collisions have p ~ 2^-64)
                        members = [i for i in support
                                   if O.row_hash(r, c, i) % (1 << b) == 0]
                        assert len(members) == 1 and members[0] == O.alpha[0, r, c, b]
                        good = True
                col_good += good
    assert col_good / col_total > 1 / 8
    assert fails <= 2


def _py_checksum(tab, r, c, x):
    (ah, bh), (alo, blo) = [tuple(int(t) for t in tab[r, c, k]) for k in (1, 2)]
    return (_py_hash(ah, bh, x) << 32) | _py_hash(alo, blo, x)


def _planted_sketch(V, seed, r, good, bad):
    """[C, B] alpha/gamma of round r with GOOD buckets planted at good[(c, b)] = index and BAD
    ones at the cells of `bad`; checksums in Python big integers from the seed table."""
    R, C, B, n = oracle.shape(V)
    tab = oracle.seed_table(seed, R)
    al = np.zeros((C, B), np.uint64)
    ga = np.zeros((C, B), np.uint64)
    for (c, b), i in good.items():
        al[c, b] = i
        ga[c, b] = _py_checksum(tab, r, c, i)
    for (c, b), i in bad.items():
        al[c, b] = i
        ga[c, b] = _py_checksum(tab, r, c, i) ^ 1  # checksum off by one bit
    return al, ga, n


def test_query_returns_first_good_bucket_columns_outer_rows_ascending(built):
    """Fig. cube_code query: columns in the outer loop, buckets of a column in the inner loop,
    the first bucket that passes the checksum test is returned."""
    V, seed, r = 1 << 12, 4242, 3
    O = oracle.Oracle(V, seed)
    rng = random.Random(8)
    i1, i2, i3, j1, j2 = (rng.randrange(1, O.n) for _ in range(5))
    # GOOD at (2, 5), (2, 1), (5, 0); BAD at (0, 3) and (1, 0).  Columns-then-rows gives (2, 1);
    # rows-then-columns would give (5, 0), deepest-first (2, 5), last-found (5, 0).
    al, ga, _ = _planted_sketch(V, seed, r, {(2, 5): i1, (2, 1): i2, (5, 0): i3},
                                {(0, 3): j1, (1, 0): j2})
    assert O.query(r, al, ga) == (oracle.SAMPLE, i2)
    # a GOOD bucket in a lower column beats every row of a higher column, even row 0
    al, ga, _ = _planted_sketch(V, seed, r, {(1, O.B - 1): i1, (3, 0): i3}, {(0, 0): j1})
    assert O.query(r, al, ga) == (oracle.SAMPLE, i1)
    # the checksum belongs to the round and column: the same pair placed in another column
    # (or queried as another round) is BAD, so the next GOOD bucket wins
    al, ga, _ = _planted_sketch(V, seed, r, {(4, 2): i2, (6, 0): i3}, {})
    al[0, 0], ga[0, 0] = al[4, 2], ga[4, 2]
    assert O.query(r, al, ga) == (oracle.SAMPLE, i2)
    assert O.query(r + 1, al, ga)[0] == oracle.FAIL or O.query(r + 1, al, ga)[1] != i2
    # classes of the result rule after Eq. (1)-(2): all EMPTY -> ZERO, BAD only -> FAIL
    al, ga, _ = _planted_sketch(V, seed, r, {}, {})
    assert O.query(r, al, ga)[0] == oracle.ZERO
    al, ga, _ = _planted_sketch(V, seed, r, {}, {(7, 4): j1})
    assert O.query(r, al, ga)[0] == oracle.FAIL
    # an alpha outside [0, n) is never a sample, even with a matching checksum
    tab = oracle.seed_table(seed, O.R)
    al, ga, _ = _planted_sketch(V, seed, r, {(3, 0): i3}, {})
    al[1, 0] = O.n + 5
    ga[1, 0] = _py_checksum(tab, r, 1, O.n + 5)
    assert O.query(r, al, ga) == (oracle.SAMPLE, i3)


def _round0_sample(V, seed, w, incident):
    """Round-0 query of node w's sketch, modelled in Python: the nested buckets of Eq. (1)-(2)
    from the incident edge set, scanned columns first, rows ascending."""
    R, C, B, n = oracle.shape(V)
    tab = oracle.seed_table(seed, R)
    for c in range(C):
        a1, b1 = (int(t) for t in tab[0, c, 0])
        for b in range(B):
            al, ga = 0, 0
            for (u, v) in incident:
                i = v * (v - 1) // 2 + u
                if _py_hash(a1, b1, i) % (1 << b) == 0:
                    al ^= i
                    ga ^= _py_checksum(tab, 0, c, i)
            if (al or ga) and al < n and ga == _py_checksum(tab, 0, c, al):
                return al
    return None


def _idx(u, v):
    return v * (v - 1) // 2 + u


def test_hook_cycle_loses_the_hook_of_its_smallest_component(built):
    """Sec. 2.2: Boruvka merges along one sampled edge per component and the paper leaves open
    which edges form the forest.  Reading taken: the sampled edges form a functional graph and
    every cycle drops the hook of its smallest component.  Graph: triangle {1, 2, 3} plus the
    pendant edge (0, 3).  Seeds are searched (in the Python model) for a round 0 whose hooks are
    0 -> 3 and a 3-cycle around the triangle, so that the smallest member of the cycle (1) is
    neither where the walk from 0 enters it (3) nor its largest member (3)."""
    V = 4
    edges = [(1, 2), (1, 3), (2, 3), (0, 3)]
    inc = {w: [e for e in edges if w in e] for w in range(V)}
    found = 0
    for seed in range(1, 4000):
        hook, hedge = {}, {}
        for w in range(V):
            i = _round0_sample(V, seed, w, inc[w])
            if i is None:  # no GOOD bucket in round 0 (possible with B = 4 rows): another seed
                break
            u, v = next((a, b) for a, b in edges if _idx(a, b) == i)
            hook[w], hedge[w] = (v if u == w else u), i
        if len(hook) < V or hook[0] != 3 or hook[3] == 0:
            continue
        if {hook[1], hook[2], hook[3]} != {1, 2, 3} or hook[1] == 1 or hook[2] == 2:
            continue
        # a 3-cycle through 1, 2, 3 and the tail 0 -> 3: every hook but node 1's is kept
        expect = sorted(hedge[w] for w in (0, 2, 3))
        O = oracle.Oracle(V, seed)
        O.ingest(np.array([e[0] for e in edges], np.uint32), np.array([e[1] for e in edges], np.uint32))
        for w in range(V):  # the oracle's own round-0 samples agree with the model
            assert O.query_node(w, 0) == (oracle.SAMPLE, hedge[w])
        st, labels, forest, used = O.connected_components()
        assert st == oracle.OK and labels.tolist() == [0, 0, 0, 0]
        assert [_idx(a, b) for a, b in forest.tolist()] == expect
        # the rules that drop the hook of the cycle's entry point or of its largest member
        # (node 3 in both cases) would keep hedge[1] instead
        assert hedge[1] not in expect
        found += 1
        if found == 3:
            break
    assert found == 3


# ------------------------------------------------------------- boruvka -----

def _check_forest(V, labels, forest, fu, fv):
    edges = set(zip(fu.tolist(), fv.tolist()))
    ncc = len(set(labels.tolist()))
    assert len(forest) == V - ncc
    parent = list(range(V))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in forest.tolist():
        assert a < b and (a, b) in edges
        ra, rb = find(a), find(b)
        assert ra != rb, "forest has a cycle"
        parent[ra] = rb
        assert labels[a] == labels[b]
    idx = [b * (b - 1) // 2 + a for a, b in forest.tolist()]
    assert idx == sorted(idx)


def test_components_match_union_find_many_tiny_streams(built):
    """Paper's own correctness method (Sec. 6): compare against an exact graph algorithm."""
    rng = random.Random(2022)
    for trial in range(600):
        V = rng.randint(2, 48)
        density = rng.random()
        n_upd = rng.randint(0, 3 * V)
        src, dst = [], []
        for _ in range(n_upd):
            if rng.random() < density:
                u, v = rng.sample(range(V), 2)
                src.append(u)
                dst.append(v)
        s = workloads.Stream(V, np.array(src, np.uint32), np.array(dst, np.uint32),
                             np.ones(len(src), np.uint8))
        O = oracle.Oracle(V, rng.getrandbits(64))
        O.ingest(s.src, s.dst)
        st, labels, forest, used = O.connected_components()
        fu, fv = workloads.final_edges(s)
        ref = workloads.union_find_labels(V, fu, fv)
        assert st == oracle.OK
        assert (labels == ref).all(), trial
        _check_forest(V, labels, forest, fu, fv)


def test_components_periodic_queries_mid_stream(built):
    """Queries interleaved with ingestion see the prefix graph and leave sketches intact."""
    s = workloads.uniform_stream(256, 900, 400, seed=17)
    O = oracle.Oracle(256, 99)
    step = 100
    for k in range(0, s.N, step):
        O.ingest(s.src[k:k + step], s.dst[k:k + step])
        before = O.alpha.copy()
        st, labels, forest, _ = O.connected_components()
        assert (O.alpha == before).all()
        pre = workloads.Stream(256, s.src[:k + step], s.dst[:k + step], s.op[:k + step])
        fu, fv = workloads.final_edges(pre)
        assert st == oracle.OK
        assert (labels == workloads.union_find_labels(256, fu, fv)).all()
        _check_forest(256, labels, forest, fu, fv)


def test_small_uniform_workload_components(built):
    s = workloads.config_uniform_small()
    O = oracle.Oracle(s.V, 1)
    O.ingest(s.src, s.dst)
    st, labels, forest, used = O.connected_components()
    fu, fv = workloads.final_edges(s)
    assert st == oracle.OK
    assert (labels == workloads.scipy_labels(s.V, fu, fv)).all()
    _check_forest(s.V, labels, forest, fu, fv)


def test_forced_sketch_failure_when_rounds_run_out(built):
    """With a single round a long path cannot finish: status SKETCH_FAIL, labels still a coarsening."""
    V = 64
    src = np.arange(V - 1, dtype=np.uint32)
    dst = np.arange(1, V, dtype=np.uint32)
    O = oracle.Oracle(V, 3, R=1)
    O.ingest(src, dst)
    st, labels, forest, used = O.connected_components()
    assert st == oracle.SKETCH_FAIL
    assert used == 1
    assert len(set(labels.tolist())) > 1
    # every label class is a set of consecutive path nodes joined by forest edges
    for a, b in forest.tolist():
        assert b == a + 1 and labels[a] == labels[b]


def test_invalid_updates_rejected_atomically(built):
    O = oracle.Oracle(10, 1)
    with pytest.raises(ValueError):
        O.ingest(np.array([1, 2], np.uint32), np.array([2, 2], np.uint32))
    assert not O.alpha.any()
    with pytest.raises(ValueError):
        O.ingest(np.array([1], np.uint32), np.array([10], np.uint32))


# ------------------------------------------------------- wide graphs (V > 2^16) ---

def test_wide_shape_keeps_log_n_rows(built):
    """B = ceil(log2 n) + 1 for every V (Lemma goodset needs a row i with
    2^(i-2) <= |cut| < 2^(i-1) for cuts of up to n edges): 33 rows at V = 2^16 + 1, 48 at 2^24."""
    assert not oracle.is_wide(1 << 16) and oracle.is_wide((1 << 16) + 1)
    assert oracle.shape(1 << 16)[2] == 32
    for V, R, B in [((1 << 16) + 1, 18, 33), (100000, 18, 34), (1 << 18, 19, 36),
                    (1 << 20, 21, 40), (1 << 24, 25, 48)]:
        r, c, b, n = oracle.shape(V)
        k = 0
        while (1 << k) < n:
            k += 1
        assert (r, c, b, n) == (R, 8, B, V * (V - 1) // 2) and b == k + 1


def test_wide_seed_table_is_the_splitmix_stream(built):
    """Per (round, column): row hash low word, checksum high, checksum low, row hash high word,
    each (a, a2, b), in SplitMix64 order."""
    R = 4
    tab = oracle.seed_table_wide(4242, R)
    assert tab.shape == (R, 8, 4, 3)
    assert tab.reshape(-1).tolist() == oracle.splitmix64(4242, R * 8 * 12)
    O = oracle.Oracle(70000, 4242, R=R)
    assert O.wide and (O.seeds == tab).all()


def test_wide_pair_hash_closed_form(built):
    rng = random.Random(17)
    for _ in range(3000):
        a, a2, b = rng.getrandbits(64), rng.getrandbits(64), rng.getrandbits(64)
        u = rng.randrange(1 << 24)
        v = rng.randrange(1 << 24)
        assert oracle.hash32_pair(a, a2, b, u, v) == ((a * u + a2 * v + b) & M64) >> 32


@pytest.mark.parametrize("p,q", [((0, 1), (0, 2)), ((5, 70000), (6, 70000)),
                                 ((65536, 65537), (65537, 65538)), ((1, 1 << 23), (2, 1 << 22))])
def test_wide_pair_hash_pairwise_uniform(built, p, q):
    """2-wise independence over random seeds for two distinct pairs (Sec. 3.1)."""
    rng = random.Random(p[1] * 7 + q[0])
    cells = np.zeros(16)
    trials = 16000
    for _ in range(trials):
        a, a2, b = rng.getrandbits(64), rng.getrandbits(64), rng.getrandbits(64)
        hx = oracle.hash32_pair(a, a2, b, *p)
        hy = oracle.hash32_pair(a, a2, b, *q)
        cells[(hx & 3) * 4 + (hy & 3)] += 1
    exp = trials / 16
    chi2 = float(((cells - exp) ** 2 / exp).sum())
    assert chi2 < 45.0, chi2


def _wide_edges(V, k, rng, hubs):
    edges = set()
    while len(edges) < k:
        u, v = rng.choice(hubs), rng.randrange(V)
        if u != v:
            edges.add((min(u, v), max(u, v)))
    return sorted(edges)


def test_wide_sketch_equals_closed_form_eq_1_2(built):
    """Eq. (1)-(2) with the pair-keyed hashes, for nodes far above 2^16."""
    V, seed, R = 90000, 31, 3
    rng = random.Random(31)
    hubs = [0, 1, 65535, 65536, 70001, 89999]
    edges = _wide_edges(V, 60, rng, hubs)
    O = oracle.Oracle(V, seed, R=R)
    src = np.array([e[1] for e in edges] + [edges[0][0]], np.uint32)
    dst = np.array([e[0] for e in edges] + [edges[0][1]], np.uint32)
    src = np.concatenate([src, dst[-1:]])  # the first edge three times: net present once
    dst = np.concatenate([dst, src[-2:-1]])
    O.ingest(src, dst)
    tab = oracle.seed_table_wide(seed, R)
    B = O.B
    for w in hubs:
        al = np.zeros((R, 8, B), np.uint64)
        ga = np.zeros((R, 8, B), np.uint64)
        for (u, v) in edges:
            if w not in (u, v):
                continue
            i = v * (v - 1) // 2 + u
            for r in range(R):
                for c in range(8):
                    (a1, a1b, b1), (ah, ahb, bh), (al_, alb, bl), (a4, a4b, b4) = [
                        tuple(int(t) for t in tab[r, c, k]) for k in range(4)]
                    h1 = ((((a4 * u + a4b * v + b4) & M64) >> 32) << 32) | \
                        (((a1 * u + a1b * v + b1) & M64) >> 32)
                    chk = ((((ah * u + ahb * v + bh) & M64) >> 32) << 32) | \
                        (((al_ * u + alb * v + bl) & M64) >> 32)
                    for b in range(B):
                        if h1 % (1 << b) == 0:
                            al[r, c, b] ^= np.uint64(i)
                            ga[r, c, b] ^= np.uint64(chk)
        assert (O.alpha[w] == al).all() and (O.gamma[w] == ga).all(), w


def test_wide_row_hash_high_word_sets_rows_past_32(built):
    """A pair whose 64-bit row hash has a zero low word reaches rows 32 + ctz(high word): rows
    past 32 exist once n > 2^32 (V = 2^20: B = 40) and take exactly such pairs."""
    import wide_pairs

    V, seed, R = 1 << 20, 99, 1
    tab = oracle.seed_table_wide(seed, R)
    c = 3
    a, a2, b = (int(t) for t in tab[0, c, 0])
    u, v = wide_pairs.zero_low_row_pair(a, a2, b, V)
    assert ((a * u + a2 * v + b) & M64) >> 32 == 0
    a4, a4b, b4 = (int(t) for t in tab[0, c, 3])
    hi = ((a4 * u + a4b * v + b4) & M64) >> 32
    depth = min(32 + ((hi & -hi).bit_length() - 1 if hi else 32), 39)
    O = oracle.Oracle(V, seed, R=R)
    assert O.B == 40
    O.update(u, v)
    i = oracle.edge_index(u, v)
    assert O.row_hash(0, c, i) == hi << 32
    for w in (u, v):
        rows = [bb for bb in range(O.B) if O.alpha[w, 0, c, bb] != 0]
        assert rows == list(range(depth + 1)) and all(O.alpha[w, 0, c, :depth + 1] == i)
        assert O.query_node(w, 0) == (oracle.SAMPLE, i)


def test_wide_support_one_is_recovered(built):
    """Lemma "goodcheck": a lone edge between nodes above 2^16 is sampled exactly."""
    V = 200000
    O = oracle.Oracle(V, 5)
    u, v = 123456, 199999
    O.update(u, v)
    i = oracle.edge_index(u, v)
    assert i >= 1 << 32
    for r in range(O.R):
        for w in (u, v):
            k, got = O.query_node(w, r)
            assert (k, got) == (1, i)


def test_wide_components_match_union_find(built):
    """Borůvka over pair-keyed sketches: labels equal union-find on the final graph."""
    V, R = 70000, 5
    rng = random.Random(77)
    edges = []
    # small stars and paths around nodes on both sides of 2^16; everything else isolated
    for k in range(300):
        c = rng.randrange(V)
        for _ in range(rng.randrange(1, 4)):
            x = rng.randrange(V)
            if x != c:
                edges.append((c, x))
    src = np.array([e[0] for e in edges], np.uint32)
    dst = np.array([e[1] for e in edges], np.uint32)
    O = oracle.Oracle(V, 12, R=R)
    O.ingest(src, dst)
    st, labels, forest, used = O.connected_components()
    s = workloads.Stream(V, src, dst, np.ones(len(src), np.uint8))
    fu, fv = workloads.final_edges(s)
    ref = workloads.union_find_labels(V, fu, fv)
    assert st == 0 and (labels == ref).all()
    assert len(forest) == V - len(np.unique(ref))
    keys = set(zip(fu.tolist(), fv.tolist()))
    assert all((int(a), int(b)) in keys for a, b in forest)
