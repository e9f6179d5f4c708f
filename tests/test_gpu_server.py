"""Serving: many sessions through the server, each result equal to the session alone.

Exact equality (integer results): every query's labels must be the components of
exactly that session's prefix of updates, whatever else runs in the same ticks.
"""
import threading

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gz(built):
    import torch

    assert torch.cuda.is_available()
    import paper_2203_14927_amd as gz

    gz.lib()
    return gz


def _session_plan(seed, V, batches):
    s, _ = workloads.rmat_session(V, workloads.RMAT_GRAPH500, sum(batches), 0.1, seed)
    out, at = [], 0
    for b in batches:
        out.append((s.src[at:at + b], s.dst[at:at + b]))
        at += b
    return s, out


def _expected(V, stream, upto):
    pre = workloads.Stream(V, stream.src[:upto], stream.dst[:upto], stream.op[:upto])
    fu, fv = workloads.final_edges(pre)
    return workloads.union_find_labels(V, fu, fv)


def test_sessions_in_the_mix_equal_alone(gz):
    from paper_2203_14927_amd.server import Server

    srv = Server(hbm_budget=8 << 30, tick_updates=20000)
    specs = [(100 + k, int(V)) for k, V in enumerate([40, 300, 1000, 64, 2000, 513])]
    results = {}
    errors = []

    def client(seed, V):
        try:
            rng = np.random.default_rng(seed)
            batches = [int(x) for x in rng.integers(1, 4000, 12)]
            stream, plan = _session_plan(seed, V, batches)
            sess = srv.open(V, seed)
            tickets, done = [], 0
            for i, (src, dst) in enumerate(plan):
                tickets.append(("u", sess.submit_updates(src, dst), None))
                done += len(src)
                if i % 3 == 2:
                    tickets.append(("q", sess.submit_query(), done))
            tickets.append(("q", sess.submit_query(), done))
            out = []
            for kind, t, upto in tickets:
                r = t.wait()
                assert r["submit_ns"] <= r["start_ns"] <= r["done_ns"]
                if kind == "q":
                    out.append((upto, r["labels"].copy(), r["num_cc"], r["status"]))
            sess.close()
            results[seed] = (V, stream, out)
        except Exception as e:  # surfaced below
            errors.append(e)

    th = [threading.Thread(target=client, args=sp) for sp in specs]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for seed, (V, stream, out) in results.items():
        for upto, labels, ncc, status in out:
            ref = _expected(V, stream, upto)
            assert status == gz.GZ_OK
            assert (labels == ref).all(), (seed, upto)
            assert ncc == len(np.unique(ref))
    st = srv.stats()
    assert st["sessions_admitted"] == len(specs) and st["queries"] > 0
    srv.close()


def test_admission_by_budget(gz):
    from paper_2203_14927_amd.server import Server

    V = 2000
    # room for two sessions of this size, not three
    per = 12 * 22 * 12 * 8 * V + V * (3 * 22 * 8 * 4 + 96)
    srv = Server(hbm_budget=int(per * 2.5))
    sess = [srv.open(V, 7 + k) for k in range(3)]
    streams = [workloads.uniform_stream(V, 3000, 500, seed=50 + k) for k in range(3)]
    tick = [s.submit_updates(st.src, st.dst) for s, st in zip(sess, streams)]
    q = [s.submit_query() for s in sess]
    # the first two complete while the third waits for memory
    for k in range(2):
        tick[k].wait()
        r = q[k].wait()
        assert (r["labels"] == _expected(V, streams[k], streams[k].N)).all()
    st = srv.stats()
    assert st["sessions_active"] == 2 and st["sessions_waiting"] == 1
    sess[0].close()  # frees memory: the third is admitted and runs
    tick[2].wait()
    r = q[2].wait()
    assert (r["labels"] == _expected(V, streams[2], streams[2].N)).all()
    sess[1].close()
    sess[2].close()
    srv.close()


def test_invalid_submissions(gz):
    from paper_2203_14927_amd.server import Server

    srv = Server(hbm_budget=1 << 30)
    s = srv.open(10, 1)
    with pytest.raises(gz.GzError):
        s.submit_updates(np.array([1], np.uint32), np.array([1], np.uint32))
    with pytest.raises(gz.GzError):
        s.submit_updates(np.array([1], np.uint32), np.array([10], np.uint32))
    with pytest.raises(gz.GzError):
        srv.open(1, 1)
    with pytest.raises(gz.GzError):
        srv.open(65536, 1)  # larger than the whole budget
    r = s.submit_query().wait()
    assert r["num_cc"] == 10
    s.close()
    srv.close()
