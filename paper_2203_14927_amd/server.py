"""Binding of the serving entry points of libgz.so (sessions, tickets, latency stamps)."""
from __future__ import annotations

import ctypes

import numpy as np


class gz_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("num_cc", ctypes.c_uint32),
                ("kind", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("updates", ctypes.c_uint64), ("submit_ns", ctypes.c_uint64),
                ("start_ns", ctypes.c_uint64), ("done_ns", ctypes.c_uint64)]


class gz_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("ticks", "updates", "queries", "sessions_admitted",
                                               "sessions_active", "sessions_waiting", "hbm_used",
                                               "hbm_budget")]


def _declare(L):
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.gz_server_create.argtypes = [u64, u64, pp]
    L.gz_server_create.restype = i32
    L.gz_session_open.argtypes = [vp, u32, u64, pp]
    L.gz_session_open.restype = i32
    L.gz_submit_updates.argtypes = [vp, vp, vp, u64, pp]
    L.gz_submit_updates.restype = i32
    L.gz_submit_query.argtypes = [vp, vp, pp]
    L.gz_submit_query.restype = i32
    L.gz_wait.argtypes = [vp, ctypes.POINTER(gz_result)]
    L.gz_wait.restype = i32
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
            "done_ns": r.done_ns, "latency_ms": (r.done_ns - r.submit_ns) / 1e6}


class Ticket:
    def __init__(self, handle, keep=None):
        self._h = handle
        self._keep = keep  # buffers the library writes into

    def wait(self) -> dict:
        from . import check, lib

        r = gz_result()
        h, self._h = self._h, None
        check(lib().gz_wait(h, ctypes.byref(r)))
        d = _res_dict(r)
        if self._keep is not None:
            d["labels"] = self._keep
        return d


class Session:
    def __init__(self, server: "Server", V: int, seed: int):
        from . import check, lib

        h = ctypes.c_void_p()
        check(lib().gz_session_open(server._h, V, seed & 0xFFFFFFFFFFFFFFFF, ctypes.byref(h)))
        self._h = h
        self.V = V
        self.seed = seed

    def submit_updates(self, src, dst) -> Ticket:
        from . import check, lib

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

    def close(self):
        from . import lib

        if getattr(self, "_h", None):
            lib().gz_session_close(self._h)
            self._h = None


class Server:
    def __init__(self, hbm_budget: int, tick_updates: int = 0):
        from . import check, lib

        h = ctypes.c_void_p()
        check(lib().gz_server_create(int(hbm_budget), int(tick_updates), ctypes.byref(h)))
        self._h = h
        from . import _track

        _track("server", self)

    def open(self, V: int, seed: int) -> Session:
        return Session(self, V, seed)

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
