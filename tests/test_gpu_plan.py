"""Captured ingest plans (HIP graph replays) against eager fused ingest and the oracle.

Every replay is checked against the eager result, with eager work and host
synchronisation between the replays.
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


def _chunks(streams, k, parts):
    """Part k of `parts` of every stream, flattened with per-graph offsets."""
    src, dst, offs = [], [], [0]
    for s in streams:
        lo = s.N * k // parts
        hi = s.N * (k + 1) // parts
        src.append(s.src[lo:hi])
        dst.append(s.dst[lo:hi])
        offs.append(offs[-1] + hi - lo)
    return np.concatenate(src), np.concatenate(dst), np.array(offs, np.uint64)


def test_plan_replays_match_eager_and_oracle(gz):
    import torch

    streams = workloads.config_many_gnp(seed=40, G=12, vlo=2, vhi=400)
    seeds = [workloads.many_graph_seed(40, k) for k in range(len(streams))]
    eager = [gz.Graph(s.V, seed=sd) for s, sd in zip(streams, seeds)]
    graphed = [gz.Graph(s.V, seed=sd) for s, sd in zip(streams, seeds)]
    parts = 3
    caps = [s.N // parts + 1 for s in streams]
    plan = gz.Plan(graphed, caps)
    for k in range(parts):
        src, dst, offs = _chunks(streams, k, parts)
        gz.ingest_multi(eager, offs, to_dev(src), to_dev(dst))
        plan.ingest(offs, to_dev(src), to_dev(dst))
        torch.cuda.synchronize()
        for ge, gg in zip(eager, graphed):
            a1, b1 = ge.export()
            a2, b2 = gg.export()
            assert (a1 == a2).all() and (b1 == b2).all(), f"replay {k} differs"
        # eager work between replays: a query on every graph
        for gg in graphed:
            gg.connected_components()
    for s, sd, gg in zip(streams, seeds, graphed):
        O = oracle_for(s, sd)
        assert_sketch_equal(gg, O)
        assert_query_equal(gg, O)
    plan.close()


def test_plan_rejects_calls_outside_its_capacities(gz):
    g1, g2 = gz.Graph(50, seed=1), gz.Graph(60, seed=2)
    plan = gz.Plan([g1, g2], [10, 10])
    src = to_dev(np.array([1, 2, 3], np.uint32))
    dst = to_dev(np.array([4, 5, 6], np.uint32))
    with pytest.raises(gz.GzError):
        plan.ingest([0, 3, 3], src, dst)  # fine ...
        plan.ingest([0, 11, 11], src, dst)  # ... but 11 > 10
    before = g2.export()
    with pytest.raises(gz.GzError) as e:
        plan.ingest([0, 1, 3], src, to_dev(np.array([4, 5, 60], np.uint32)))  # 60 >= V of g2
    assert e.value.status == gz.GZ_EINVAL
    after = g2.export()
    assert (before[0] == after[0]).all() and (before[1] == after[1]).all()
    plan.close()


def test_plan_with_empty_graphs_and_empty_calls(gz):
    s = workloads.uniform_stream(80, 300, 100, seed=3)
    g_full, g_empty = gz.Graph(80, seed=7), gz.Graph(30, seed=8)
    plan = gz.Plan([g_empty, g_full], [5, s.N])
    plan.ingest([0, 0, 0], to_dev(np.zeros(1, np.uint32)), to_dev(np.zeros(1, np.uint32)))
    plan.ingest([0, 0, s.N], to_dev(s.src), to_dev(s.dst))
    O = oracle_for(s, 7)
    assert_sketch_equal(g_full, O)
    a, b = g_empty.export()
    assert not a.any() and not b.any()
    plan.close()


def test_single_large_graph_plan_replays(gz):
    """A captured plan over one graph with V > 4096 (two-pass placement), replayed on
    three parts of a stream, equals one eager ingest of the whole stream."""
    import torch

    s = workloads.uniform_stream(6000, 120000, 30000, seed=31)
    g_eager, g_plan = gz.Graph(6000, seed=12), gz.Graph(6000, seed=12)
    g_eager.ingest(to_dev(s.src), to_dev(s.dst))
    parts = 3
    plan = gz.Plan([g_plan], [s.N // parts + 1])
    for k in range(parts):
        lo, hi = s.N * k // parts, s.N * (k + 1) // parts
        plan.ingest([0, hi - lo], to_dev(s.src[lo:hi]), to_dev(s.dst[lo:hi]))
        torch.cuda.synchronize()
        g_plan.connected_components()  # eager work between replays
    a1, b1 = g_eager.export()
    a2, b2 = g_plan.export()
    assert (a1 == a2).all() and (b1 == b2).all()
    plan.close()
