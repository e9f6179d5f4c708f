"""Shared helpers of the GPU parity tests (inputs and comparisons only)."""
import numpy as np

import oracle
import workloads


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).cuda()


def oracle_for(stream, seed, R=None, nodes=None):
    O = oracle.Oracle(stream.V, seed, R=R)
    if nodes is None:
        O.ingest(stream.src, stream.dst)
    else:
        O.ingest_nodes(stream.src, stream.dst, nodes)
    return O


def assert_sketch_equal(graph, O, nodes=None):
    """GPU export (nested, canonical) == oracle state, bit for bit."""
    if nodes is None:
        a, g = graph.export()
        bad = np.argwhere((a != O.alpha) | (g != O.gamma))
        assert bad.size == 0, f"first mismatch at node/r/c/b {bad[0].tolist()} ({len(bad)} total)"
        return
    for v in nodes:
        a, g = graph.export(int(v), int(v) + 1)
        assert (a[0] == O.alpha[v]).all() and (g[0] == O.gamma[v]).all(), f"node {v} differs"


GZ_OK, GZ_ESKETCH_FAIL = 0, 4


def gz_status_of(oracle_status):
    """Oracle status (OK / SKETCH_FAIL) -> the library's status code."""
    return {oracle.OK: GZ_OK, oracle.SKETCH_FAIL: GZ_ESKETCH_FAIL}[oracle_status]


def assert_query_equal(graph, O):
    st, labels, ncc, forest = graph.query()
    ost, olabels, oforest, _ = O.connected_components()
    assert st == gz_status_of(ost)
    assert (labels == olabels).all()
    assert ncc == len(set(olabels.tolist()))
    assert forest.shape == oforest.shape and (forest == oforest).all(), (
        f"forest differs: gpu {forest.tolist()[:20]} oracle {oforest.tolist()[:20]}")
    return st, labels, forest


def check_forest_valid(V, labels, forest, fu, fv):
    edges = set(zip(fu.tolist(), fv.tolist()))
    ncc = len(np.unique(labels))
    assert len(forest) == V - ncc
    parent = np.arange(V)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in forest.tolist():
        assert a < b and (a, b) in edges
        ra, rb = find(a), find(b)
        assert ra != rb
        parent[ra] = rb
        assert labels[a] == labels[b]
    idx = [b * (b - 1) // 2 + a for a, b in forest.tolist()]
    assert idx == sorted(idx)


def final_labels(stream):
    fu, fv = workloads.final_edges(stream)
    return workloads.scipy_labels(stream.V, fu, fv), fu, fv
