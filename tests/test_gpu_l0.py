"""GPU standard l0-sampler (Fig. agm_code) against its CPU oracle: every bucket word and every
node's sample per round, bit for bit, on signed streams with insertions, deletions and repeated
pairs; host and device inputs; items split across workgroups; the largest V."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gz(built):
    import torch

    assert torch.cuda.is_available()
    import paper_2203_14927_amd as gz

    gz.lib()
    return gz


def _dev(a, dtype=np.int32):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(dtype)).cuda()


def _signed_stream(V, n, seed, hub=False):
    """Inserts of random pairs (a pair may repeat: multiplicity > 1), deletes of live ones."""
    rng = np.random.default_rng(seed)
    src, dst, op, live = [], [], [], []
    for _ in range(n):
        if live and rng.random() < 0.25:
            u, v = live.pop(int(rng.integers(len(live))))
            src.append(v); dst.append(u); op.append(0)
        else:
            u = 0 if hub and rng.random() < 0.5 else int(rng.integers(V))
            v = int(rng.integers(V))
            if u == v:
                v = (v + 1) % V
            live.append((u, v))
            src.append(u); dst.append(v); op.append(1)
    return np.array(src, np.uint32), np.array(dst, np.uint32), np.array(op, np.uint8)


def _check(S, O, nodes=None):
    if nodes is None:
        a, b, c = S.export()
        assert (a == O.a).all() and (b == O.b).all() and (c == O.c).all()
    else:
        for v in nodes:
            a, b, c = S.export(int(v), int(v) + 1)
            assert (a[0] == O.a[v]).all() and (b[0] == O.b[v]).all() and (c[0] == O.c[v]).all(), v
    for r in range(S.R):
        kind, idx, mult = S.sample(r)
        for v in (range(S.V) if nodes is None else nodes):
            k, i, m = O.query_node(int(v), r)
            assert kind[v] == k, (v, r)
            if k == oracle.SAMPLE:
                assert idx[v] == i and mult[v] == m, (v, r)


@pytest.mark.parametrize("V,n,seed", [(2, 9, 1), (10, 120, 2), (200, 3000, 3), (1000, 6000, 4)])
def test_l0_small_streams_bit_exact(gz, V, n, seed):
    src, dst, op = _signed_stream(V, n, seed)
    O = oracle.L0Oracle(V, 50 + seed)
    O.ingest(src, dst, op)
    S = gz.L0Sketch(V, 50 + seed)
    S.ingest(_dev(src), _dev(dst), op=_dev(op, np.uint8))
    _check(S, O)
    # host arrays, and op left out (all insertions)
    S2 = gz.L0Sketch(V, 50 + seed)
    S2.ingest(src, dst)
    O2 = oracle.L0Oracle(V, 50 + seed)
    O2.ingest(src, dst)
    _check(S2, O2)


def test_l0_two_calls_and_split_items(gz):
    """A hub node with far more entries than one work item takes, over two ingest calls."""
    V = 3000
    src, dst, op = _signed_stream(V, 24000, 7, hub=True)
    hub = int((src == 0).sum() + (dst == 0).sum())
    print(f"[l0] hub entries {hub}", file=sys.stderr, flush=True)
    assert hub > 2 * 4096
    nodes = [0, 1, 2, 17, 1499, 2999]
    O = oracle.L0Oracle(V, 11)
    O.ingest_nodes(src, dst, op, nodes)
    S = gz.L0Sketch(V, 11)
    h = len(src) // 2
    S.ingest(_dev(src[:h]), _dev(dst[:h]), op=_dev(op[:h], np.uint8))
    S.ingest(_dev(src[h:]), _dev(dst[h:]), op=_dev(op[h:], np.uint8))
    _check(S, O, nodes=nodes)


def test_l0_largest_graph(gz):
    """V = 2^16: 17 rounds, 136 pairs (three-wave groups)."""
    V = 1 << 16
    src, dst, op = _signed_stream(V, 20000, 8, hub=True)
    nodes = sorted({0, 1, V - 1, int(src[5]), int(dst[9]), int(src[100])})
    O = oracle.L0Oracle(V, 12)
    O.ingest_nodes(src, dst, op, nodes)
    S = gz.L0Sketch(V, 12)
    S.ingest(_dev(src), _dev(dst), op=_dev(op, np.uint8))
    for v in nodes:
        a, b, c = S.export(v, v + 1)
        assert (a[0] == O.a[v]).all() and (b[0] == O.b[v]).all() and (c[0] == O.c[v]).all(), v
    for r in (0, 5, S.R - 1):
        kind, idx, mult = S.sample(r)
        for v in nodes:
            k, i, m = O.query_node(v, r)
            assert kind[v] == k and (k != oracle.SAMPLE or (idx[v] == i and mult[v] == m))


def test_l0_invalid_update_applies_nothing(gz):
    S = gz.L0Sketch(50, 3)
    S.ingest(np.array([1, 2], np.uint32), np.array([3, 4], np.uint32))
    before = S.export()
    for s, d in [([1, 5], [2, 5]), ([1], [50])]:
        with pytest.raises(gz.GzError) as e:
            S.ingest(_dev(np.array(s, np.uint32)), _dev(np.array(d, np.uint32)))
        assert e.value.status == gz.GZ_EINVAL
    after = S.export()
    assert all((x == y).all() for x, y in zip(before, after))
