"""Seeded stream generators: determinism and the R-MAT quadrant law (host only)."""
import numpy as np

import workloads


def test_rmat_draws_independent_of_thread_count():
    V = 1 << 12
    a = workloads.rmat_draws(V, workloads.RMAT_GRAPH500, 3_000_000, 7, threads=1)
    b = workloads.rmat_draws(V, workloads.RMAT_GRAPH500, 3_000_000, 7, threads=5)
    assert (a.src == b.src).all() and (a.dst == b.dst).all()
    c = workloads.rmat_draws(V, workloads.RMAT_GRAPH500, 3_000_000, 8, threads=5)
    assert (a.src != c.src).any()


def test_rmat_draws_ids_and_quadrant_frequencies():
    """Ids in range, no self-loops; the top level's quadrant shares follow (a, b, c, d)
    (b and c together: endpoints are swapped at random), within 5 standard errors."""
    V, n = 1 << 10, 2_000_000
    abcd = (0.57, 0.19, 0.19, 0.05)
    s = workloads.rmat_draws(V, abcd, n, 11)
    assert s.N == n
    assert (s.src < V).all() and (s.dst < V).all() and (s.src != s.dst).all()
    top = V >> 1
    hu = (s.src >= top).astype(int)
    hv = (s.dst >= top).astype(int)
    both0 = np.mean((hu == 0) & (hv == 0))
    both1 = np.mean((hu == 1) & (hv == 1))
    mixed = np.mean(hu != hv)
    # self-loops are redrawn: a draw is a self-loop exactly when every level picks
    # quadrant a or d, so conditioned on acceptance the top level's shares are
    # (p_q - p_q [q in {a, d}] (a+d)^(L-1)) / (1 - (a+d)^L)
    a, b, c, d = abcd
    L = 10
    loop = (a + d) ** (L - 1)
    acc = 1 - (a + d) ** L
    for got, want in [(both0, a * (1 - loop) / acc), (both1, d * (1 - loop) / acc),
                      (mixed, (b + c) / acc)]:
        se = np.sqrt(want * (1 - want) / n)
        assert abs(got - want) < 5 * se, (got, want)


def test_rmat_draws_rejects_non_power_of_two():
    import pytest

    with pytest.raises(ValueError):
        workloads.rmat_draws(1000, workloads.RMAT_GRAPH500, 10, 1)
