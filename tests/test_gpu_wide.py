"""Graphs with V > 2^16: pair-keyed hashes, 64-bit edge indices, four 32-bit planes.

The HIP path against the oracle bit for bit (sketch words, labels, forest,
status), at V just above 2^16, at the paper's largest Kronecker size (2^18) and
at the largest V the library takes (2^24).
"""
import numpy as np
import pytest

import oracle
import workloads
from helpers import (assert_query_equal, assert_sketch_equal, check_forest_valid, final_labels,
                     oracle_for, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gz(built):
    import torch

    assert torch.cuda.is_available()
    import paper_2203_14927_amd as gz

    gz.lib()
    return gz


def _trees_stream(V, used, max_size, noise, seed):
    """Random trees of 1..max_size nodes over `used` random nodes, plus `noise`
    random pairs that are inserted and later deleted; shuffled."""
    rng = np.random.default_rng(seed)
    nodes = rng.permutation(V)[:used]
    src, dst = [], []
    at = 0
    while at < used:
        k = int(rng.integers(1, max_size + 1))
        grp = nodes[at:at + k]
        for j in range(1, len(grp)):
            src.append(grp[j])
            dst.append(grp[int(rng.integers(0, j))])
        at += k
    a = rng.integers(0, V, noise)
    b = rng.integers(0, V, noise)
    keep = a != b
    a, b = a[keep], b[keep]
    src = np.concatenate([np.array(src, np.int64), a, b])
    dst = np.concatenate([np.array(dst, np.int64), b, a])
    order = rng.permutation(len(src))
    return workloads.Stream(V, src[order].astype(np.uint32), dst[order].astype(np.uint32),
                            np.ones(len(src), np.uint8))


def test_wide_shape_rule(gz):
    """B = bitlen(n - 1) + 1 as for narrow graphs (33 up to n = 2^32, 40 at V = 2^20, 48 at
    V = 2^24: the row hash has 64 bits); R follows the usual rule."""
    g = gz.Graph(70000, seed=3, rounds=2)
    assert (g.V, g.R, g.C, g.B) == (70000, 2, 8, 33)
    assert g.n == 70000 * 69999 // 2
    for V, B in [(92682, 33), (92683, 34), (1 << 20, 40), (1 << 24, 48)]:
        g = gz.Graph(V, seed=3, rounds=1)
        assert g.B == B == (V * (V - 1) // 2 - 1).bit_length() + 1, V
        g.close()
    g = gz.Graph(65537, seed=3, rounds=1)
    assert g.B == 33 and g.n == 65537 * 65536 // 2
    g = gz.Graph(65536, seed=3, rounds=1)
    assert g.B == 32  # the largest narrow graph keeps the index-keyed contract
    with pytest.raises(gz.GzError):
        gz.Graph((1 << 24) + 1, seed=3, rounds=1)


def test_wide_small_trees_full_parity(gz):
    """V=70000, R=4: every sketch word, labels, forest, status; host and device inputs."""
    V, seed = 70000, 77
    s = _trees_stream(V, 60000, 4, 120000, 5)
    g = gz.Graph(V, seed=seed, rounds=4)
    h = s.N // 3
    g.ingest(s.src[:h], s.dst[:h])  # host arrays
    g.ingest(to_dev(s.src[h:]), to_dev(s.dst[h:]))
    O = oracle_for(s, seed, R=4)
    assert_sketch_equal(g, O)
    st, labels, forest = assert_query_equal(g, O)
    assert st == gz.GZ_OK
    ref, fu, fv = final_labels(s)
    assert (labels == ref).all()
    check_forest_valid(V, labels, forest, fu, fv)


@pytest.mark.parametrize("tuning", [dict(lds_rows=5), dict(chunk=3, wg_size=512),
                                    dict(lds_rows=1, chunk=4096, wgs_per_cu=1)])
def test_wide_tuning_variants_are_bit_exact(gz, tuning):
    """Row tiles smaller than B (rows above them go to HBM) and other launch shapes."""
    V, seed = 65600, 101
    s = _trees_stream(V, 30000, 6, 60000, 6)
    g = gz.Graph(V, seed=seed, rounds=3)
    g.set_tuning(**tuning)
    g.ingest(to_dev(s.src), to_dev(s.dst))
    O = oracle_for(s, seed, R=3)
    assert_sketch_equal(g, O)
    assert_query_equal(g, O)


def test_wide_per_node_batches(gz):
    """The per-node call toggles only that node's sketch, as the oracle's node-filtered ingest."""
    V, seed = 90000, 11
    rng = np.random.default_rng(12)
    g = gz.Graph(V, seed=seed, rounds=3)
    O = oracle.Oracle(V, seed, R=3)
    for node, cnt in [(0, 5000), (V - 1, 20000), (45678, 1), (65536, 3000)]:
        nb = rng.integers(0, V, cnt).astype(np.uint32)
        nb = nb[nb != node]
        g.update_sketch_batch(node, to_dev(nb))
        g.update_sketch_batch(node, nb[: len(nb) // 3])  # host path, toggles a third back
        src = np.concatenate([np.full(len(nb), node, np.uint32),
                              np.full(len(nb) // 3, node, np.uint32)])
        dst = np.concatenate([nb, nb[: len(nb) // 3]])
        O.ingest_nodes(src, dst, [node])
    for node in (0, 1, V - 1, 45678, 65536, 89998):
        a, b = g.export(node, node + 1)
        assert (a[0] == O.alpha[node]).all() and (b[0] == O.gamma[node]).all(), f"node {node}"


def test_wide_kron18_sampled_nodes_and_labels(gz):
    """V=2^18 (the paper's largest Kronecker size), full R=19: an R-MAT session stream with
    interleaved deletes; sampled node sketches against the oracle, labels against
    union-find on the final graph, forest valid."""
    V, seed = 1 << 18, 2018
    s, _ = workloads.rmat_session(V, workloads.RMAT_GRAPH500, 3_000_000, 0.1, 18)
    g = gz.Graph(V, seed=seed)
    assert g.R == 19 and g.B == 36
    g.ingest(to_dev(s.src), to_dev(s.dst))
    deg = np.bincount(np.concatenate([s.src, s.dst]).astype(np.int64), minlength=V)
    rng = np.random.default_rng(3)
    nodes = sorted(set(rng.choice(V, 12, replace=False).tolist())
                   | {0, V - 1, int(np.argmax(deg)), int(s.src[0])})
    O = oracle.Oracle(V, seed)
    O.ingest_nodes(s.src, s.dst, nodes)
    for v in nodes:
        a, b = g.export(v, v + 1)
        assert (a[0] == O.alpha[v]).all() and (b[0] == O.gamma[v]).all(), f"node {v}"
    st, labels, ncc, forest = g.query()
    assert st == gz.GZ_OK
    ref, fu, fv = final_labels(s)
    assert (labels == ref).all()
    assert ncc == len(np.unique(ref))
    check_forest_valid(V, labels, forest, fu, fv)


def test_wide_host_tier_equals_hbm(gz):
    """Host-DRAM tier of a wide graph through several slabs, three calls with queries."""
    V, seed = 70000, 31
    s = _trees_stream(V, 50000, 4, 80000, 7)
    h = gz.Graph(V, seed=seed, rounds=3)
    node_bytes = 16 * h.B * h.R * h.C
    t = gz.Graph(V, seed=seed, rounds=3, host_tier=True, staging_bytes=2 * 9000 * node_bytes)
    for k in range(3):
        lo, hi = s.N * k // 3, s.N * (k + 1) // 3
        h.ingest(to_dev(s.src[lo:hi]), to_dev(s.dst[lo:hi]))
        t.ingest(s.src[lo:hi], s.dst[lo:hi])
        a, b = h.query(), t.query()
        assert a[0] == b[0] and (a[1] == b[1]).all() and a[2] == b[2] and (a[3] == b[3]).all()
    x1, y1 = h.export(0, 20000)
    x2, y2 = t.export(0, 20000)
    assert (x1 == x2).all() and (y1 == y2).all()
    O = oracle_for(s, seed, R=3)
    assert_sketch_equal(t, O)
    assert_query_equal(t, O)


def test_wide_multi_graph_ingest_and_plan(gz):
    """Several wide graphs in one fused call and in a captured plan equal separate calls;
    wide and narrow graphs do not share a call, and wide graphs are queried alone."""
    import torch

    Vs, seeds = [65537, 80000, 66000], [1, 2, 3]
    streams = [_trees_stream(V, 20000, 5, 30000, 50 + k) for k, V in enumerate(Vs)]
    sep = [gz.Graph(V, seed=sd, rounds=2) for V, sd in zip(Vs, seeds)]
    fused = [gz.Graph(V, seed=sd, rounds=2) for V, sd in zip(Vs, seeds)]
    planned = [gz.Graph(V, seed=sd, rounds=2) for V, sd in zip(Vs, seeds)]
    for g, s in zip(sep, streams):
        g.ingest(to_dev(s.src), to_dev(s.dst))
    offs = np.zeros(len(Vs) + 1, np.uint64)
    offs[1:] = np.cumsum([s.N for s in streams])
    src = np.concatenate([s.src for s in streams])
    dst = np.concatenate([s.dst for s in streams])
    gz.ingest_multi(fused, offs, to_dev(src), to_dev(dst))
    plan = gz.Plan(planned, [s.N for s in streams])
    plan.ingest(offs, to_dev(src), to_dev(dst))
    torch.cuda.synchronize()
    plan.close()
    for a, b, c in zip(sep, fused, planned):
        x1, y1 = a.export()
        x2, y2 = b.export()
        x3, y3 = c.export()
        assert (x1 == x2).all() and (y1 == y2).all()
        assert (x1 == x3).all() and (y1 == y3).all()
    O = oracle_for(streams[1], seeds[1], R=2)
    assert_sketch_equal(fused[1], O)
    assert_query_equal(fused[1], O)
    narrow = gz.Graph(1000, seed=9)
    with pytest.raises(gz.GzError):
        gz.ingest_multi([fused[0], narrow], np.array([0, 1, 2], np.uint64),
                        to_dev(np.array([0, 1], np.uint32)), to_dev(np.array([1, 2], np.uint32)))
    with pytest.raises(gz.GzError):
        gz.connected_components_multi(fused)


def test_wide_largest_graph(gz):
    """V=2^24, one round: edges among the highest and lowest ids (edge indices near 2^47);
    touched node sketches, labels, forest and status against the oracle."""
    V, seed = 1 << 24, 7
    rng = np.random.default_rng(1)
    src = rng.integers(V - 5000, V, 3000)
    dst = np.concatenate([rng.integers(0, V, 1500), rng.integers(V - 5000, V, 1500)])
    keep = src != dst
    s = workloads.Stream(V, src[keep].astype(np.uint32), dst[keep].astype(np.uint32),
                         np.ones(int(keep.sum()), np.uint8))
    g = gz.Graph(V, seed=seed, rounds=1)
    g.ingest(to_dev(s.src), to_dev(s.dst))
    O = oracle_for(s, seed, R=1)
    nodes = sorted(set(s.src[:20].tolist()) | set(s.dst[:20].tolist()) | {0, 1, V - 1, V // 2})
    assert_sketch_equal(g, O, nodes=nodes)
    assert_query_equal(g, O)


@pytest.mark.parametrize("V,R,n,seed", [(65537, 3, 1_000_000, 61), (1 << 20, 2, 6_000_000, 62)])
def test_wide_two_pass_grouping_edges(gz, V, R, n, seed):
    """The bucket-first grouping at its smallest (V = 2^16 + 1) and largest (V = 2^20) sizes,
    on hub-heavy R-MAT draws whose first bucket is cut into many pieces: sampled node
    sketches (the six largest hubs included) against the oracle."""
    s = workloads.rmat_draws(1 << (V - 1).bit_length(), workloads.RMAT_GRAPH500, n, seed)
    keep = (s.src < V) & (s.dst < V)
    s = workloads.Stream(V, s.src[keep], s.dst[keep], s.op[keep])
    g = gz.Graph(V, seed=seed, rounds=R)
    g.ingest(to_dev(s.src), to_dev(s.dst))
    deg = np.bincount(np.concatenate([s.src, s.dst]).astype(np.int64), minlength=V)
    rng = np.random.default_rng(seed)
    hubs = np.argsort(deg)[::-1][:6].tolist()
    nodes = sorted(set(rng.choice(V, 10, replace=False).tolist()) | set(hubs) | {0, V - 1})
    O = oracle.Oracle(V, seed, R=R)
    O.ingest_nodes(s.src, s.dst, nodes)
    for v in nodes:
        a, b = g.export(v, v + 1)
        assert (a[0] == O.alpha[v]).all() and (b[0] == O.gamma[v]).all(), f"node {v}"


@pytest.mark.parametrize("V", [70000, (1 << 20) + 3])
def test_wide_invalid_updates_rejected_and_nothing_applied(gz, V):
    """Self-loops and ids >= V are rejected by the bucket-first grouping (V <= 2^20) and by
    the one-pass grouping (larger V) alike, synchronously and at flush, applying nothing."""
    g = gz.Graph(V, seed=5, rounds=1)
    good = (np.array([1, V - 1, 70], np.uint32), np.array([V - 2, 3, 65536], np.uint32))
    g.ingest(to_dev(good[0]), to_dev(good[1]))
    nodes = [1, 3, 70, 65536, V - 2, V - 1]
    before = [g.export(v, v + 1) for v in nodes]
    for src, dst in [([1, 7], [1, 8]), ([1, 2], [3, V]), ([V + 5], [1])]:
        with pytest.raises(gz.GzError) as e:
            g.ingest(to_dev(np.array(src, np.uint32)), to_dev(np.array(dst, np.uint32)))
        assert e.value.status == gz.GZ_EINVAL
        with pytest.raises(gz.GzError):
            g.ingest(np.array(src, np.uint32), np.array(dst, np.uint32))
    g.ingest(to_dev(np.array([9, 9], np.uint32)), to_dev(np.array([9, 10], np.uint32)),
             flags=gz.GZ_ASYNC)
    with pytest.raises(gz.GzError):
        g.flush()
    g.flush()
    after = [g.export(v, v + 1) for v in nodes]
    for (a1, b1), (a2, b2), v in zip(before, after, nodes):
        assert (a1 == a2).all() and (b1 == b2).all(), f"node {v} changed"
    O = oracle.Oracle(V, 5, R=1)
    O.ingest_nodes(good[0], good[1], nodes)
    for v, (a, b) in zip(nodes, after):
        assert (a[0] == O.alpha[v]).all() and (b[0] == O.gamma[v]).all(), f"node {v}"


def test_wide_single_graph_plan_replays(gz):
    """A captured plan over one wide graph (bucket-first grouping, side split) replayed on
    new inputs equals eager ingest, with eager work between replays."""
    import torch

    V, seed = 200000, 44
    s = workloads.rmat_draws(1 << 18, workloads.RMAT_GRAPH500, 3_000_000, 45)
    keep = (s.src < V) & (s.dst < V)
    src, dst = s.src[keep], s.dst[keep]
    eager = gz.Graph(V, seed=seed, rounds=2)
    planned = gz.Graph(V, seed=seed, rounds=2)
    parts = 3
    cap = len(src) // parts + 1
    plan = gz.Plan([planned], [cap])
    for k in range(parts):
        lo, hi = len(src) * k // parts, len(src) * (k + 1) // parts
        eager.ingest(to_dev(src[lo:hi]), to_dev(dst[lo:hi]))
        plan.ingest(np.array([0, hi - lo], np.uint64), to_dev(src[lo:hi]), to_dev(dst[lo:hi]))
        torch.cuda.synchronize()
        for v in (0, 1, 2, 65536, V - 1):
            a1, b1 = eager.export(v, v + 1)
            a2, b2 = planned.export(v, v + 1)
            assert (a1 == a2).all() and (b1 == b2).all(), f"replay {k}, node {v}"
        planned.connected_components()
    plan.close()
    x1, y1 = eager.export(0, 4096)
    x2, y2 = planned.export(0, 4096)
    assert (x1 == x2).all() and (y1 == y2).all()


def _zero_low_pair(seed, c):
    """A pair u < v < 2^20 whose row hash in column c of round 0 has a zero low word."""
    import wide_pairs

    tab = oracle.seed_table_wide(seed, 1)
    a, a2, b = (int(t) for t in tab[0, c, 0])
    u, v = wide_pairs.zero_low_row_pair(a, a2, b, 1 << 20)
    assert ((a * u + a2 * v + b) % (1 << 64)) >> 32 == 0
    return u, v


@pytest.mark.parametrize("path", ["fused", "per_node"])
def test_wide_rows_past_32(gz, path):
    """V = 2^20 (B = 40), one round: an edge whose 64-bit row hash has a zero low word
    lands in a row past 32 (the hash's high word decides how far), among a few thousand
    other edges at both of its nodes, through the grouped path and the per-node path;
    those node sketches bit-exact with the oracle, and their queries sample it."""
    V, seed, c = 1 << 20, 99, 3
    u, v = _zero_low_pair(seed, c)
    rng = np.random.default_rng(8)
    others = rng.integers(0, V, 6000).astype(np.uint32)
    nu = others[:3000][(others[:3000] != u) & (others[:3000] != v)]
    nv = others[3000:][(others[3000:] != u) & (others[3000:] != v)]
    src = np.concatenate([np.full(len(nu), u, np.uint32), np.full(len(nv), v, np.uint32),
                          np.array([u], np.uint32)])
    dst = np.concatenate([nu, nv, np.array([v], np.uint32)])
    g = gz.Graph(V, seed=seed, rounds=1)
    assert g.B == 40
    if path == "fused":
        order = rng.permutation(len(src))
        g.ingest(to_dev(src[order]), to_dev(dst[order]))
        nodes = [u, v, int(nu[0]), int(nv[-1])]
    else:
        for node, nb in [(u, np.concatenate([nu, [v]])), (v, np.concatenate([[u], nv]))]:
            g.update_sketch_batch(node, to_dev(nb.astype(np.uint32)))
        nodes = [u, v]
    O = oracle.Oracle(V, seed, R=1)
    O.ingest_nodes(src, dst, nodes)
    deep = [bb for bb in range(O.B) if O.alpha[u, 0, c, bb] != 0]
    assert max(deep) >= 32  # the pair reaches past row 31 in u's sketch
    for w in nodes:
        a, b = g.export(w, w + 1)
        assert (a[0] == O.alpha[w]).all() and (b[0] == O.gamma[w]).all(), f"node {w}"
