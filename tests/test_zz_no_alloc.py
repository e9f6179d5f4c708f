"""gz_ingest_noalloc (buffers carved from the library's fixed per-device array) against
gz_ingest (allocating scratch) and the oracle: bit-exact sketches over two calls in a row,
the second smaller, so the second call runs on the first call's leftover scratch."""
import sys

import numpy as np
import pytest

from helpers import assert_query_equal, assert_sketch_equal, oracle_for, to_dev
import workloads

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


@pytest.mark.parametrize("V,n1,n2,seed", [(3000, 200000, 7000, 1),    # two-pass grouping
                                          (700, 60000, 900, 2),       # one-pass grouping
                                          (70000, 30000, 4000, 3)])   # pair-keyed (wide) graph
def test_noalloc_equals_ingest_on_two_calls(gz, V, n1, n2, seed):
    print(f"[no-alloc] V={V} n1={n1} n2={n2} seed={seed}", file=sys.stderr, flush=True)
    s1, s2 = _stream(V, n1, seed), _stream(V, n2, seed + 100)
    a = gz.Graph(V, seed=seed + 7, rounds=4 if V > 65536 else 0)
    b = gz.Graph(V, seed=seed + 7, rounds=4 if V > 65536 else 0)
    both = workloads.Stream(V, np.concatenate([s1.src, s2.src]), np.concatenate([s1.dst, s2.dst]),
                            np.ones(s1.N + s2.N, np.uint8))
    for k, s in enumerate((s1, s2)):
        a.ingest_noalloc(to_dev(s.src), to_dev(s.dst))
        b.ingest(to_dev(s.src), to_dev(s.dst))
        a.flush()
        ea, eb = a.export(), b.export()
        assert (ea[0] == eb[0]).all() and (ea[1] == eb[1]).all(), f"call {k} differs from gz_ingest"
    O = oracle_for(both, seed + 7, R=4 if V > 65536 else None)
    assert_sketch_equal(a, O)
    if V <= 65536:
        assert_query_equal(a, O)
    a.close()
    b.close()


def test_noalloc_rejects_what_it_cannot_hold(gz):
    import torch

    g = gz.Graph(1 << 16, seed=3)
    n = 6_000_000  # needs far more than the fixed scratch
    z = torch.zeros(n, dtype=torch.int32, device="cuda")
    o = torch.ones(n, dtype=torch.int32, device="cuda")
    with pytest.raises(gz.GzError) as e:
        g.ingest_noalloc(z, o)
    assert e.value.status == gz.GZ_EINVAL and "scratch" in str(e.value)
    with pytest.raises(ValueError):
        g.ingest_noalloc(np.zeros(4, np.uint32), np.ones(4, np.uint32))
    a, b = g.export(0, 4)
    assert not a.any() and not b.any()
    # an invalid update: nothing applied, reported at the next flush
    g.ingest_noalloc(to_dev(np.array([1, 5], np.uint32)), to_dev(np.array([2, 5], np.uint32)))
    with pytest.raises(gz.GzError):
        g.flush()
    a, b = g.export(0, 8)
    assert not a.any() and not b.any()
    g.close()
