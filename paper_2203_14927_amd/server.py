"""Binding of the serving entry points of libgz.so (sessions, tickets, latency stamps)."""
from __future__ import annotations

import ctypes

import numpy as np


class gz_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("num_cc", ctypes.c_uint32),
                ("kind", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("updates", ctypes.c_uint64), ("submit_ns", ctypes.c_uint64),
                ("start_ns", ctypes.c_uint64), ("done_ns", ctypes.c_uint64),
                ("admit_ns", ctypes.c_uint64)]


class gz_replay_session(ctypes.Structure):
    _fields_ = [("V", ctypes.c_uint32), ("n_batches", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("first_batch", ctypes.c_uint64), ("open_ns", ctypes.c_uint64)]


class gz_tick_record(ctypes.Structure):
    _fields_ = [("take_ns", ctypes.c_uint64), ("launched_ns", ctypes.c_uint64),
                ("done_ns", ctypes.c_uint64), ("updates", ctypes.c_uint64),
                ("ingested", ctypes.c_uint64),
                ("batches", ctypes.c_uint32), ("graphs", ctypes.c_uint32),
                ("device_ms", ctypes.c_float), ("reserved", ctypes.c_uint32)]


class gz_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("ticks", "updates", "queries", "sessions_admitted",
                                               "sessions_active", "sessions_waiting", "hbm_used",
                                               "hbm_budget", "batches_copied", "batches_inplace",
                                               "staged_bytes", "worker_wait_ns",
                                               "worker_launch_ns", "query_runs", "create_ns",
                                               "create_ns_max", "free_ns", "free_ns_max",
                                               "ingested", "flushes")]


def _declare(L):
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.gz_server_create.argtypes = [u64, u64, pp]
    L.gz_server_create.restype = i32
    L.gz_session_open.argtypes = [vp, u32, u64, pp]
    L.gz_session_open.restype = i32
    L.gz_submit_updates.argtypes = [vp, vp, vp, u64, pp]
    L.gz_submit_updates.restype = i32
    L.gz_submit_updates_inplace.argtypes = [vp, vp, vp, u64, pp]
    L.gz_submit_updates_inplace.restype = i32
    L.gz_submit_query.argtypes = [vp, vp, pp]
    L.gz_submit_query.restype = i32
    L.gz_wait.argtypes = [vp, ctypes.POINTER(gz_result)]
    L.gz_wait.restype = i32
    L.gz_wait_any.argtypes = [pp, u32, u64, ctypes.POINTER(u32), ctypes.POINTER(gz_result)]
    L.gz_wait_any.restype = i32
    L.gz_session_graph.argtypes = [vp, pp]
    L.gz_session_graph.restype = i32
    L.gz_server_set_gutter.argtypes = [vp, u32]
    L.gz_server_set_gutter.restype = i32
    L.gz_server_replay.argtypes = [vp, vp, u32, vp, u64, vp, vp, vp, u32, u32, vp, vp, vp,
                                   ctypes.POINTER(u64)]
    L.gz_server_replay.restype = i32
    L.gz_server_timeline.argtypes = [vp, vp, u64, ctypes.POINTER(u64)]
    L.gz_server_timeline.restype = i32
    L.gz_session_close.argtypes = [vp]
    L.gz_session_close.restype = i32
    L.gz_server_get_stats.argtypes = [vp, ctypes.POINTER(gz_server_stats)]
    L.gz_server_get_stats.restype = i32
    L.gz_server_destroy.argtypes = [vp]
    L.gz_server_destroy.restype = i32
    return L


def _res_dict(r: gz_result) -> dict:
    return {"status": r.status, "num_cc": r.num_cc, "kind": "query" if r.kind else "updates",
            "updates": r.updates, "submit_ns": r.submit_ns, "start_ns": r.start_ns,
            "done_ns": r.done_ns, "admit_ns": r.admit_ns,
            "latency_ms": (r.done_ns - r.submit_ns) / 1e6}


class Ticket:
    def __init__(self, handle, keep=None, lent=None):
        self._h = handle
        self._keep = keep  # buffers the library writes into
        self._lent = lent  # in-place batch buffers the library reads until completion

    def _finish(self, r: gz_result) -> dict:
        self._h = None
        self._lent = None
        d = _res_dict(r)
        if self._keep is not None:
            d["labels"] = self._keep
        return d

    def wait(self) -> dict:
        from . import check, lib

        r = gz_result()
        h = self._h
        st = lib().gz_wait(h, ctypes.byref(r))
        d = self._finish(r)
        check(st)
        return d


def wait_any(tickets, timeout_s: float | None = None):
    """Wait for the first of `tickets` (one server) to complete: (index, result), or None
    when none completed within timeout_s.  The completed ticket is released."""
    from . import GZ_ETIMEOUT, check, lib

    arr = (ctypes.c_void_p * len(tickets))(*[t._h for t in tickets])
    idx = ctypes.c_uint32()
    r = gz_result()
    ns = 0xFFFFFFFFFFFFFFFF if timeout_s is None else max(0, int(timeout_s * 1e9))
    st = lib().gz_wait_any(arr, len(tickets), ns, ctypes.byref(idx), ctypes.byref(r))
    if st == GZ_ETIMEOUT:
        return None
    i = idx.value
    d = tickets[i]._finish(r) if i < len(tickets) else None
    check(st)
    return i, d


def _inplace_arg(x):
    """(device-readable pointer, keepalive) of a torch tensor in device or pinned memory."""
    import torch

    if x.dtype not in (torch.int32, torch.uint32):
        raise TypeError("expected an int32/uint32 tensor")
    if not x.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if not (x.is_cuda or x.is_pinned()):
        raise ValueError("in-place batches must be device tensors or pinned host tensors")
    return ctypes.c_void_p(x.data_ptr()), x


class Session:
    def __init__(self, server: "Server", V: int, seed: int):
        from . import check, lib

        h = ctypes.c_void_p()
        check(lib().gz_session_open(server._h, V, seed & 0xFFFFFFFFFFFFFFFF, ctypes.byref(h)))
        self._h = h
        self.V = V
        self.seed = seed

    def submit_updates(self, src, dst) -> Ticket:
        """Host arrays are copied once (into pinned memory) before the call returns; torch
        tensors in device or pinned memory are read in place until the ticket completes."""
        from . import _is_torch, check, lib

        if _is_torch(src) or _is_torch(dst):
            ps, ks = _inplace_arg(src)
            pd, kd = _inplace_arg(dst)
            if ks.numel() != kd.numel():
                raise ValueError("src and dst lengths differ")
            t = ctypes.c_void_p()
            check(lib().gz_submit_updates_inplace(self._h, ps, pd, ks.numel(), ctypes.byref(t)))
            return Ticket(t, lent=(ks, kd))
        s = np.ascontiguousarray(src, np.uint32)
        d = np.ascontiguousarray(dst, np.uint32)
        if len(s) != len(d):
            raise ValueError("src and dst lengths differ")
        t = ctypes.c_void_p()
        check(lib().gz_submit_updates(self._h, ctypes.c_void_p(s.ctypes.data),
                                      ctypes.c_void_p(d.ctypes.data), len(s), ctypes.byref(t)))
        return Ticket(t)

    def submit_query(self) -> Ticket:
        from . import check, lib

        labels = np.zeros(self.V, np.uint32)
        t = ctypes.c_void_p()
        check(lib().gz_submit_query(self._h, ctypes.c_void_p(labels.ctypes.data), ctypes.byref(t)))
        return Ticket(t, keep=labels)

    def graph(self):
        """The session's graph (export, query) while none of its requests is in flight, once
        its gutter is applied; the server keeps ownership, so the object frees nothing."""
        from . import Graph, check, lib

        h = ctypes.c_void_p()
        check(lib().gz_session_graph(self._h, ctypes.byref(h)))
        return Graph.borrowed(h)

    def close(self):
        from . import lib

        if getattr(self, "_h", None):
            lib().gz_session_close(self._h)
            self._h = None


class Server:
    def __init__(self, hbm_budget: int, tick_updates: int = 0, gutter_per_node=None):
        """gutter_per_node: gutter updates per node of each session (None: the library's
        default; 0: no gutters)."""
        from . import check, lib

        h = ctypes.c_void_p()
        check(lib().gz_server_create(int(hbm_budget), int(tick_updates), ctypes.byref(h)))
        self._h = h
        from . import _track

        _track("server", self)
        if gutter_per_node is not None:
            check(lib().gz_server_set_gutter(h, int(gutter_per_node)))

    def open(self, V: int, seed: int) -> Session:
        return Session(self, V, seed)

    def replay(self, sessions, batch_offs, src, dst, arrival_ns=None, query_every=50,
               client_threads=16) -> dict:
        """Drive sessions [(V, seed, first_batch, n_batches, open_ns)] through the server from
        native client threads (closed loop when arrival_ns is None); per-batch latency,
        service latency and following-query latency in ns (0: no query), and the wall time."""
        from . import check, lib

        arr = (gz_replay_session * len(sessions))(
            *[gz_replay_session(int(V), int(nb), int(sd) & 0xFFFFFFFFFFFFFFFF, int(fb), int(op))
              for V, sd, fb, nb, op in sessions])
        offs = np.ascontiguousarray(batch_offs, np.uint64)
        s = np.ascontiguousarray(src, np.uint32)
        d = np.ascontiguousarray(dst, np.uint32)
        nb = len(offs) - 1
        arrival = None if arrival_ns is None else np.ascontiguousarray(arrival_ns, np.uint64)
        lat = np.zeros(nb, np.uint64)
        svc = np.zeros(nb, np.uint64)
        qlat = np.zeros(nb, np.uint64)
        wall = ctypes.c_uint64()
        vp = ctypes.c_void_p
        check(lib().gz_server_replay(
            self._h, ctypes.cast(arr, vp), len(sessions), vp(offs.ctypes.data), nb,
            vp(s.ctypes.data), vp(d.ctypes.data),
            None if arrival is None else vp(arrival.ctypes.data), query_every, client_threads,
            vp(lat.ctypes.data), vp(svc.ctypes.data), vp(qlat.ctypes.data), ctypes.byref(wall)))
        return {"batch_latency_ns": lat, "batch_service_ns": svc, "query_latency_ns": qlat,
                "wall_ns": wall.value}

    def timeline(self) -> np.ndarray:
        """Tick records (structured array: take/launched/done ns, new updates, updates ingested,
        batches, graphs, device_ms)."""
        from . import check, lib

        n = ctypes.c_uint64()
        check(lib().gz_server_timeline(self._h, None, 0, ctypes.byref(n)))
        arr = (gz_tick_record * n.value)()
        check(lib().gz_server_timeline(self._h, ctypes.cast(arr, ctypes.c_void_p), n.value,
                                       ctypes.byref(n)))
        dt = np.dtype([("take_ns", "u8"), ("launched_ns", "u8"), ("done_ns", "u8"),
                       ("updates", "u8"), ("ingested", "u8"), ("batches", "u4"), ("graphs", "u4"),
                       ("device_ms", "f4"), ("reserved", "u4")])
        return np.frombuffer(bytes(arr), dtype=dt).copy()

    def stats(self) -> dict:
        from . import lib

        st = gz_server_stats()
        lib().gz_server_get_stats(self._h, ctypes.byref(st))
        return {n: int(getattr(st, n)) for n, _ in st._fields_}

    def close(self):
        from . import lib

        if getattr(self, "_h", None):
            lib().gz_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
