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


@pytest.mark.parametrize("gutter", [None, 0])
def test_sessions_in_the_mix_equal_alone(gz, gutter):
    """With gutters (the default) and without: a query applies its session's gutter first."""
    from paper_2203_14927_amd.server import Server

    srv = Server(hbm_budget=8 << 30, tick_updates=20000, gutter_per_node=gutter)
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


def _drive_mixed(srv, plans, torch):
    """Submit each session's batches, cycling through the three submission forms (host
    copy, in-place device tensor, in-place pinned tensor at an offset), and wait for all."""
    tickets = []
    for k, (sess, batches) in enumerate(plans):
        for i, (src, dst) in enumerate(batches):
            form = (i + k) % 3
            if form == 0:
                tickets.append(sess.submit_updates(src, dst))
            elif form == 1:
                s = torch.from_numpy(src.astype(np.int32)).cuda()
                d = torch.from_numpy(dst.astype(np.int32)).cuda()
                torch.cuda.synchronize()
                tickets.append(sess.submit_updates(s, d))
            else:
                pad = 5  # a view that starts inside the pinned allocation
                s = torch.zeros(len(src) + pad, dtype=torch.int32).pin_memory()
                d = torch.zeros(len(dst) + pad, dtype=torch.int32).pin_memory()
                s[pad:] = torch.from_numpy(src.astype(np.int32))
                d[pad:] = torch.from_numpy(dst.astype(np.int32))
                tickets.append(sess.submit_updates(s[pad:], d[pad:]))
    for t in tickets:
        assert t.wait()["status"] == 0


@pytest.mark.parametrize("gutter", [None, 0])
def test_session_sketches_equal_oracle_and_solo(gz, gutter):
    """Sessions served together, through every submission form, end with the sketches
    the oracle computes for each session's stream alone, and the same as a solo graph
    (with gutters, the session's graph is handed out once its gutter is applied)."""
    import torch

    import oracle
    from paper_2203_14927_amd.server import Server

    srv = Server(hbm_budget=8 << 30, tick_updates=5000, gutter_per_node=gutter)
    plans, streams = [], []
    for k, V in enumerate([50, 700, 3000, 129]):
        rng = np.random.default_rng(70 + k)
        batches = [int(x) for x in rng.integers(1, 3000, 9)]
        stream, plan = _session_plan(300 + k, V, batches)
        plans.append((srv.open(V, 900 + k), plan))
        streams.append(stream)
    _drive_mixed(srv, plans, torch)
    for k, ((sess, _), stream) in enumerate(zip(plans, streams)):
        g = sess.graph()
        a, b = g.export()
        O = oracle.Oracle(stream.V, 900 + k)
        O.ingest(stream.src, stream.dst)
        assert (a == O.alpha).all() and (b == O.gamma).all(), f"session {k}"
        solo = gz.Graph(stream.V, seed=900 + k)
        solo.ingest(stream.src, stream.dst)
        a2, b2 = solo.export()
        assert (a == a2).all() and (b == b2).all()
        st, labels, ncc, forest = g.query()
        ost, olabels, oforest, _ = O.connected_components()
        assert (labels == olabels).all() and (forest == oforest).all()
        solo.close()
    st = srv.stats()
    assert st["batches_inplace"] > 0 and st["batches_copied"] > 0
    assert st["staged_bytes"] == 8 * st["updates"]
    assert st["ingested"] == st["updates"]  # every gutter was applied
    assert (st["flushes"] > 0) == (gutter is None)
    for sess, _ in plans:
        sess.close()
    srv.close()


def test_one_client_over_sessions_beyond_the_budget_finishes(gz):
    """One client drives four sessions closed-loop (one request outstanding each) with room
    for two: waiting on whichever ticket completes first, it never blocks on a session that
    is not admitted, so sessions finish, close, and let the others in."""
    from paper_2203_14927_amd.server import Server, wait_any

    V = 2000
    per = 12 * 22 * 12 * 8 * V + V * (3 * 22 * 8 * 4 + 96)
    srv = Server(hbm_budget=int(per * 2.5), tick_updates=4000)
    plans = []
    for k in range(4):
        rng = np.random.default_rng(40 + k)
        batches = [int(x) for x in rng.integers(100, 2000, 6)]
        plans.append(_session_plan(400 + k, V, batches))
    sess = [srv.open(V, 800 + k) for k in range(4)]
    nxt = [0] * 4
    labels = [None] * 4
    out = {}  # ticket index -> session

    def submit(k):
        stream, batches = plans[k]
        if nxt[k] < len(batches):
            t = sess[k].submit_updates(*batches[nxt[k]])
        elif nxt[k] == len(batches):
            t = sess[k].submit_query()
        else:
            sess[k].close()
            return None
        nxt[k] += 1
        return t

    live = [(submit(k), k) for k in range(4)]
    while live:
        i, r = wait_any([t for t, _ in live])
        _, k = live.pop(i)
        if r["kind"] == "query":
            labels[k] = r["labels"].copy()
        t = submit(k)
        if t is not None:
            live.append((t, k))
    for k in range(4):
        stream, _ = plans[k]
        assert (labels[k] == _expected(V, stream, stream.N)).all(), k
    assert srv.stats()["sessions_admitted"] == 4
    srv.close()


def test_wait_any_times_out_while_a_session_waits_for_memory(gz):
    from paper_2203_14927_amd.server import Server, wait_any

    V = 2000
    per = 12 * 22 * 12 * 8 * V + V * (3 * 22 * 8 * 4 + 96)
    srv = Server(hbm_budget=int(per * 1.5))
    a, b = srv.open(V, 1), srv.open(V, 2)
    ta = a.submit_updates(np.array([1, 2], np.uint32), np.array([3, 4], np.uint32))
    tb = b.submit_updates(np.array([5], np.uint32), np.array([6], np.uint32))
    assert ta.wait()["status"] == 0
    assert wait_any([tb], timeout_s=0.05) is None  # b is not admitted while a is open
    with pytest.raises(gz.GzError):
        b.graph()
    a.close()
    i, r = wait_any([tb], timeout_s=30)
    assert i == 0 and r["status"] == 0 and r["updates"] == 1
    g = b.graph()
    labels = g.query()[1]
    assert labels[6] == labels[5] and labels[1] != labels[3]
    b.close()
    srv.close()


def test_invalid_inplace_submissions(gz):
    import ctypes

    import torch

    from paper_2203_14927_amd.server import Server

    srv = Server(hbm_budget=1 << 30)
    s = srv.open(10, 1)
    bad = torch.tensor([1, 2], dtype=torch.int32)
    with pytest.raises(gz.GzError):  # device memory, id out of range
        s.submit_updates(bad.cuda(), torch.tensor([3, 10], dtype=torch.int32).cuda())
    with pytest.raises(gz.GzError):  # pinned memory, self-loop
        s.submit_updates(bad.pin_memory(), torch.tensor([3, 2], dtype=torch.int32).pin_memory())
    with pytest.raises(ValueError):  # pageable host tensors cannot be lent
        s.submit_updates(bad, torch.tensor([3, 4], dtype=torch.int32))
    host = np.array([1, 2], np.uint32)
    t = ctypes.c_void_p()
    st = gz.lib().gz_submit_updates_inplace(s._h, ctypes.c_void_p(host.ctypes.data),
                                             ctypes.c_void_p(host.ctypes.data), 2,
                                             ctypes.byref(t))
    assert st == gz.GZ_EINVAL
    r = s.submit_updates(torch.tensor([1], dtype=torch.int32).cuda(),
                         torch.tensor([2], dtype=torch.int32).cuda()).wait()
    assert r["status"] == 0
    assert s.submit_query().wait()["num_cc"] == 9
    s.close()
    srv.close()


@pytest.mark.parametrize("open_loop", [False, True])
def test_replay_drives_every_request(gz, open_loop):
    """The native replay clients submit every batch and query of every session, closed loop
    and with scheduled arrivals, under a budget that holds only some sessions at once."""
    from paper_2203_14927_amd.server import Server

    Vs = [300, 2000, 64, 2000, 1000, 2000, 513, 2000]
    rng = np.random.default_rng(9)
    sess, srcs, dsts, sizes = [], [], [], []
    at = 0
    for k, V in enumerate(Vs):
        nb = [int(x) for x in rng.integers(1, 1500, 7)]
        stream, _ = _session_plan(600 + k, V, nb)
        srcs.append(stream.src)
        dsts.append(stream.dst)
        sizes += nb
        sess.append([V, 700 + k, at, len(nb), 0])
        at += len(nb)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    arrival = None
    if open_loop:
        arrival = np.zeros(len(sizes), np.uint64)
        for k, s in enumerate(sess):
            s[4] = k * 2_000_000
            arrival[s[2]:s[2] + s[3]] = s[4] + 1_000_000 * np.arange(1, s[3] + 1)
    per = 12 * 22 * 12 * 8 * 2000 + 2000 * (3 * 22 * 8 * 4 + 96)
    srv = Server(hbm_budget=int(per * 2.5), tick_updates=3000)
    r = srv.replay(sess, offs, np.concatenate(srcs), np.concatenate(dsts), arrival,
                   query_every=3, client_threads=3)
    st = srv.stats()
    tl = srv.timeline()
    srv.close()
    assert len(tl) == st["ticks"] and int(tl["updates"].sum()) == int(offs[-1])
    assert (tl["device_ms"] > 0).all() and (tl["take_ns"] <= tl["launched_ns"]).all()
    assert (tl["launched_ns"] <= tl["done_ns"]).all() and int(tl["batches"].sum()) == len(sizes)
    assert 1 <= st["query_runs"] <= st["queries"]
    assert (r["batch_latency_ns"] > 0).all() and (r["batch_service_ns"] > 0).all()
    assert (r["batch_service_ns"] <= r["batch_latency_ns"]).all()
    n_q = sum((s[3] // 3) + (1 if s[3] % 3 else 0) for s in sess)
    assert (r["query_latency_ns"] > 0).sum() == n_q == st["queries"]
    assert st["updates"] == int(offs[-1]) and st["sessions_admitted"] == len(Vs)
    assert r["wall_ns"] > 0


def test_full_gutters_flush_between_queries(gz):
    """Sessions whose batches overflow their gutter (65536 updates) between queries, one
    batch larger than the gutter itself, and a tick budget smaller than one flush: every
    query equals union-find on its prefix and the final sketches equal the oracle's."""
    import oracle
    from paper_2203_14927_amd.server import Server

    srv = Server(hbm_budget=8 << 30, tick_updates=20000)
    specs = []
    for k, V in enumerate([300, 64, 1500]):
        batches = [9000] * 9 + ([70000] if k == 1 else []) + [9000] * 9
        stream, plan = _session_plan(800 + k, V, batches)
        specs.append((V, stream, plan, srv.open(V, 40 + k)))
    pending = []
    for V, stream, plan, sess in specs:
        done = 0
        for i, (src, dst) in enumerate(plan):
            pending.append(("u", sess.submit_updates(src, dst), None, None))
            done += len(src)
            if i in (8, len(plan) - 1):
                pending.append(("q", sess.submit_query(), (V, stream), done))
    for kind, t, vs, upto in pending:
        r = t.wait()
        assert r["status"] == 0
        if kind == "q":
            V, stream = vs
            assert (r["labels"] == _expected(V, stream, upto)).all(), (V, upto)
    st = srv.stats()
    # at least one flush per query interval (each holds more than a gutter; where a
    # batch that overflows the gutter shares a tick with the batches before the
    # query, that one flush serves the query too)
    assert st["flushes"] >= 6 and st["ingested"] == st["updates"] == sum(
        s[1].N for s in specs)
    for k, (V, stream, _, sess) in enumerate(specs):
        a, b = sess.graph().export()
        O = oracle.Oracle(V, 40 + k)
        O.ingest(stream.src, stream.dst)
        assert (a == O.alpha).all() and (b == O.gamma).all(), f"session {k}"
        sess.close()
    srv.close()


def test_graph_applies_the_gutter(gz):
    """Batches acknowledged into the gutter are in the sketches the session's graph hands
    out, and a later batch still goes to the (emptied) gutter."""
    import oracle
    from paper_2203_14927_amd.server import Server

    srv = Server(hbm_budget=1 << 30)
    V = 500
    stream, plan = _session_plan(21, V, [3000, 2000, 1000])
    sess = srv.open(V, 77)
    for src, dst in plan[:2]:
        assert sess.submit_updates(src, dst).wait()["status"] == 0
    st = srv.stats()
    assert st["updates"] == 5000 and st["ingested"] == 0  # still in the gutter
    a, b = sess.graph().export()
    O = oracle.Oracle(V, 77)
    O.ingest(stream.src[:5000], stream.dst[:5000])
    assert (a == O.alpha).all() and (b == O.gamma).all()
    assert srv.stats()["ingested"] == 5000
    assert sess.submit_updates(*plan[2]).wait()["status"] == 0
    r = sess.submit_query().wait()
    assert (r["labels"] == _expected(V, stream, 6000)).all()
    st = srv.stats()
    assert st["ingested"] == 6000 and st["flushes"] == 2
    sess.close()
    srv.close()
