"""Host-DRAM sketch tier: sketches in pinned host memory, streamed through HBM slabs.

Every result must be bit-identical to the HBM-resident graph and to the oracle.
Small staging budgets force many slabs, so slab boundaries, skipped slabs and
buffer reuse are all exercised.
"""
import numpy as np
import pytest

import oracle
import workloads
from helpers import assert_query_equal, assert_sketch_equal, oracle_for, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gz(built):
    import torch

    assert torch.cuda.is_available()
    import paper_2203_14927_amd as gz

    gz.lib()
    return gz


def _stream(V, n, seed):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, V, n, dtype=np.int64)
    dst = rng.integers(0, V, n, dtype=np.int64)
    keep = src != dst
    return workloads.Stream(V, src[keep].astype(np.uint32), dst[keep].astype(np.uint32),
                            np.ones(int(keep.sum()), np.uint8))


def _node_bytes(g):
    return 12 * g.B * g.R * g.C


def test_host_tier_equals_oracle(gz):
    """V=1024 small uniform workload through ten slabs: every sketch bit, labels, forest."""
    s = workloads.config_uniform_small()
    probe = gz.Graph(s.V, seed=1)
    g = gz.Graph(s.V, seed=1, host_tier=True, staging_bytes=2 * 103 * _node_bytes(probe))
    g.ingest(to_dev(s.src), to_dev(s.dst))
    O = oracle_for(s, 1)
    assert_sketch_equal(g, O)
    assert_query_equal(g, O)


def test_host_tier_matches_hbm_over_calls(gz):
    """V=6000 (two-pass grouping), five calls with queries between them."""
    s = _stream(6000, 150000, 41)
    h = gz.Graph(6000, seed=9)
    t = gz.Graph(6000, seed=9, host_tier=True, staging_bytes=2 * 777 * _node_bytes(h))
    for k in range(5):
        lo, hi = s.N * k // 5, s.N * (k + 1) // 5
        h.ingest(to_dev(s.src[lo:hi]), to_dev(s.dst[lo:hi]))
        t.ingest(s.src[lo:hi], s.dst[lo:hi])  # host arrays on the host-tier graph
        a = h.query()
        b = t.query()
        assert a[0] == b[0] and (a[1] == b[1]).all() and a[2] == b[2]
        assert (a[3] == b[3]).all()
    x1, y1 = h.export()
    x2, y2 = t.export()
    assert (x1 == x2).all() and (y1 == y2).all()
    x1, y1 = h.export(100, 2100)
    x2, y2 = t.export(100, 2100)
    assert (x1 == x2).all() and (y1 == y2).all()


def test_host_tier_sparse_batch_skips_slabs(gz):
    """A batch touching a few nodes: only their slabs move; the rest stay as they were."""
    V = 3000
    base = _stream(V, 40000, 42)
    h = gz.Graph(V, seed=5)
    t = gz.Graph(V, seed=5, host_tier=True, staging_bytes=2 * 100 * _node_bytes(h))
    for g in (h, t):
        g.ingest(to_dev(base.src), to_dev(base.dst))
    src = np.array([10, 10, 2500, 1999], np.uint32)
    dst = np.array([11, 2999, 7, 1998], np.uint32)
    for g in (h, t):
        g.ingest(to_dev(src), to_dev(dst))
    x1, y1 = h.export()
    x2, y2 = t.export()
    assert (x1 == x2).all() and (y1 == y2).all()


def test_host_tier_plain_path(gz):
    s = _stream(200, 6000, 43)
    probe = gz.Graph(200, seed=3)
    g = gz.Graph(200, seed=3, host_tier=True, staging_bytes=2 * 16 * _node_bytes(probe))
    u = np.concatenate([s.src, s.dst])
    v = np.concatenate([s.dst, s.src])
    order = np.argsort(u, kind="stable")
    u, v = u[order], v[order]
    starts = np.searchsorted(u, np.arange(201))
    for node in range(200):
        nb = v[starts[node]:starts[node + 1]]
        if len(nb):
            g.update_sketch_batch(node, to_dev(nb))
    O = oracle_for(s, 3)
    assert_sketch_equal(g, O)
    assert_query_equal(g, O)


def test_host_tier_reset_errors_and_single_graph_calls(gz):
    s = _stream(500, 5000, 44)
    g = gz.Graph(500, seed=8, host_tier=True, staging_bytes=1 << 20)
    g.ingest(to_dev(s.src), to_dev(s.dst))
    before = g.export()
    with pytest.raises(gz.GzError) as e:
        g.ingest(to_dev(np.array([1, 2], np.uint32)), to_dev(np.array([3, 500], np.uint32)))
    assert e.value.status == gz.GZ_EINVAL
    after = g.export()
    assert (before[0] == after[0]).all() and (before[1] == after[1]).all()
    other = gz.Graph(300, seed=2)
    with pytest.raises(gz.GzError):
        gz.ingest_multi([g, other], [0, 1, 2], to_dev(np.array([1, 1], np.uint32)),
                        to_dev(np.array([2, 2], np.uint32)))
    with pytest.raises(gz.GzError):
        gz.Plan([g], [100])
    with pytest.raises(gz.GzError):
        gz.connected_components_multi([g, other])
    g.reset()
    a, b = g.export()
    assert not a.any() and not b.any()
    st, labels, ncc, forest = g.query()
    assert st == gz.GZ_OK and ncc == 500 and (labels == np.arange(500)).all()
