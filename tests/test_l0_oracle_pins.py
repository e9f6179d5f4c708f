"""Pins of the standard l0-sampler oracle (Sec. 3, Fig. agm_code) against facts fixed outside it:
modular arithmetic recomputed with Python integers, the closed form of the bucket sums, linearity,
cancellation of edges inside a node set, and exact recovery of a single nonzero entry."""
import random

import numpy as np
import pytest

import oracle

M64 = (1 << 64) - 1
P = (1 << 61) - 1


def test_mulmod_and_powmod_match_python_integers(built):
    rng = random.Random(1)
    vals = [0, 1, 2, P - 1, P - 2, (1 << 60), (1 << 61) - 3] + [rng.randrange(P) for _ in range(200)]
    for x in vals:
        y = rng.randrange(P)
        assert oracle.l0_mulmod(x, y) == (x * y) % P
    for z in [1, 2, 3, P - 1] + [rng.randrange(1, P) for _ in range(100)]:
        for e in [0, 1, 2, 31, (1 << 31) - 1, 2147450879] + [rng.randrange(1 << 31) for _ in range(5)]:
            assert oracle.l0_powmod(z, e) == pow(z, e, P)


def _py_hash(a, b, x):
    return ((a * x + b) & M64) >> 32


def _stream(V, n, rng, del_frac=0.3):
    """Random inserts of pairs, then deletes of some of them (a pair may be inserted twice)."""
    src, dst, op = [], [], []
    live = []
    for _ in range(n):
        if live and rng.random() < del_frac:
            u, v = live.pop(rng.randrange(len(live)))
            src.append(v)
            dst.append(u)
            op.append(0)
        else:
            u, v = rng.sample(range(V), 2)
            live.append((u, v))
            src.append(u)
            dst.append(v)
            op.append(1)
    return np.array(src, np.uint32), np.array(dst, np.uint32), np.array(op, np.uint8)


def _closed_form(V, seed, src, dst, op):
    """Fig. agm_code applied to the final integer vectors: bucket (r, c, row) of node w holds
    sum x_w[e] * e, sum x_w[e] and sum x_w[e] * z^e (mod p) over the indices e in it."""
    R, C, B, n = oracle.shape(V)
    tab = oracle.seed_table(seed, R)
    x = {}
    for u, v, o in zip(src.tolist(), dst.tolist(), op.tolist()):
        lo, hi = min(u, v), max(u, v)
        e = hi * (hi - 1) // 2 + lo
        d = 1 if o else -1
        x[(lo, e)] = x.get((lo, e), 0) + d
        x[(hi, e)] = x.get((hi, e), 0) - d
    a = np.zeros((V, R, C, B), np.int64)
    b = np.zeros((V, R, C, B), np.int64)
    c = np.zeros((V, R, C, B), np.uint64)
    cc = {}
    for (w, e), m in x.items():
        if m == 0:
            continue
        for r in range(R):
            for col in range(C):
                h = _py_hash(int(tab[r, col, 0, 0]), int(tab[r, col, 0, 1]), e)
                z = 1 + int(tab[r, col, 1, 0]) % (P - 1)
                for row in range(B):
                    if h % (1 << row) == 0:
                        a[w, r, col, row] += m * e
                        b[w, r, col, row] += m
                        cc[(w, r, col, row)] = (cc.get((w, r, col, row), 0) + m * pow(z, e, P)) % P
    for k, val in cc.items():
        c[k] = val
    return a, b, c


def test_sketch_equals_closed_form(built):
    rng = random.Random(4)
    for V, n, seed in [(2, 6, 1), (9, 80, 2), (30, 500, 3)]:
        src, dst, op = _stream(V, n, rng)
        S = oracle.L0Oracle(V, seed)
        S.ingest(src, dst, op)
        a, b, c = _closed_form(V, seed, src, dst, op)
        assert (S.a == a).all() and (S.b == b).all() and (S.c == c).all()


def test_column_base_from_the_seed_table(built):
    S = oracle.L0Oracle(100, 77)
    tab = oracle.seed_table(77, S.R)
    for r in range(S.R):
        for col in range(S.C):
            assert S.z[r, col] == 1 + int(tab[r, col, 1, 0]) % (P - 1)


def test_linearity_and_edge_cancellation(built):
    """Sketches add (a, b as integers, c modulo p); the vectors of all nodes sum to zero, and
    those of a node set sum to the sketch of its cut."""
    rng = random.Random(8)
    V = 24
    s1 = _stream(V, 300, rng)
    s2 = _stream(V, 200, rng)
    A, Bs, AB = oracle.L0Oracle(V, 9), oracle.L0Oracle(V, 9), oracle.L0Oracle(V, 9)
    A.ingest(*s1)
    Bs.ingest(*s2)
    AB.ingest(*[np.concatenate([p, q]) for p, q in zip(s1, s2)])
    assert (A.a + Bs.a == AB.a).all() and (A.b + Bs.b == AB.b).all()
    assert ((A.c.astype(object) + Bs.c.astype(object)) % P == AB.c.astype(object)).all()
    # every edge is +x in one endpoint and -x in the other: the sum over all nodes is zero
    assert (AB.a.sum(axis=0) == 0).all() and (AB.b.sum(axis=0) == 0).all()
    assert (AB.c.astype(object).sum(axis=0) % P == 0).all()
    # edges only inside {0..11} and inside {12..23}: each half sums to zero
    H = oracle.L0Oracle(V, 9)
    src = rng.choices(range(12), k=200)
    dst = [(s + rng.randrange(1, 12)) % 12 for s in src]
    H.ingest(np.array(src + [u + 12 for u in src], np.uint32),
             np.array(dst + [v + 12 for v in dst], np.uint32))
    assert (H.a[:12].sum(axis=0) == 0).all() and (H.b[12:].sum(axis=0) == 0).all()


def test_single_entry_recovered_with_its_multiplicity(built):
    """Support 1: every bucket that holds the entry passes, in every round, with b = x[e]."""
    V = 1 << 12
    rng = random.Random(3)
    for trial in range(12):
        u, v = sorted(rng.sample(range(V), 2))
        m = rng.randint(1, 5)
        S = oracle.L0Oracle(V, 100 + trial)
        for _ in range(m):
            S.update(u, v, 1)
        e = v * (v - 1) // 2 + u
        for r in range(S.R):
            assert S.query_node(u, r) == (oracle.SAMPLE, e, m)
            assert S.query_node(v, r) == (oracle.SAMPLE, e, -m)
        other = next(x for x in range(V) if x not in (u, v))
        assert S.query_node(other, 0)[0] == oracle.ZERO
    S = oracle.L0Oracle(64, 5)
    S.update(3, 9, 1)
    S.update(9, 3, -1)  # inserted then deleted: the zero vector
    assert S.query_node(3, 0)[0] == oracle.ZERO and not S.a.any() and not S.c.any()


def test_sample_is_in_the_support_with_its_value(built):
    V = 400
    rng = random.Random(11)
    fails = 0
    for trial in range(40):
        deg = rng.choice([2, 3, 6, 20, 90, 300])
        nbrs = rng.sample(range(1, V), deg)
        mult = [rng.choice([1, 1, 1, 2, 3]) for _ in nbrs]
        S = oracle.L0Oracle(V, 900 + trial)
        src = np.repeat(np.zeros(deg, np.uint32), mult)
        dst = np.repeat(np.array(nbrs, np.uint32), mult)
        S.ingest(src, dst)
        x = {x * (x - 1) // 2: m for x, m in zip(nbrs, mult)}
        for r in range(S.R):
            kind, e, m = S.query_node(0, r)
            if kind == oracle.SAMPLE:
                assert e in x and m == x[e]
            else:
                assert kind == oracle.FAIL
                fails += 1
    assert fails <= 3


def test_query_scans_columns_then_rows(built):
    """Fig. agm_code query: first passing bucket in column order, rows ascending; zero buckets
    are skipped, a bucket with b = 0 but a != 0 fails."""
    V = 1000
    S = oracle.L0Oracle(V, 42)
    r = 2
    C, B = S.C, S.B
    a = np.zeros((C, B), np.int64)
    b = np.zeros((C, B), np.int64)
    c = np.zeros((C, B), np.uint64)

    def plant(col, row, e, m):
        z = int(S.z[r, col])
        a[col, row], b[col, row], c[col, row] = m * e, m, (m * pow(z, e, P)) % P

    assert S.query(r, a, b, c)[0] == oracle.ZERO
    a[0, 0] = 5  # b = 0: never a sample
    assert S.query(r, a, b, c)[0] == oracle.FAIL
    plant(3, 7, 1234, 2)
    plant(3, 2, 777, -1)
    plant(5, 0, 99, 1)
    assert S.query(r, a, b, c) == (oracle.SAMPLE, 777, -1)
    plant(1, B - 1, 4321, 3)
    assert S.query(r, a, b, c) == (oracle.SAMPLE, 4321, 3)
    c[1, B - 1] ^= 1  # wrong checksum: the next passing bucket wins
    assert S.query(r, a, b, c) == (oracle.SAMPLE, 777, -1)
