"""MI355X-native CubeSketch ingestion and Boruvka connectivity (GraphZeppelin's hot path).

This package is a thin ctypes binding over ``libgz.so`` (HIP, gfx950).  It only
marshals arguments: every step of ingestion and of the query runs in the
library's kernels.  PyTorch is used, when present, for device memory and
streams.  Importing fails loudly if the library has not been built.

The functions keep the C names of ``include/gz.h``; :class:`Graph` wraps a
handle for convenience.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgz.so")

GZ_OK, GZ_EINVAL, GZ_ENOMEM, GZ_EDEVICE, GZ_ESKETCH_FAIL, GZ_EBUSY, GZ_ESTATE, GZ_ETIMEOUT = range(8)
GZ_DEVICE_PTR = 0x1
GZ_ASYNC = 0x2
GZ_UNCHECKED = 0x4
GZ_COLUMNS = 8


class GzError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_status_name(status)}: {msg}")
        self.status = status


class gz_config(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint32), ("tier", ctypes.c_uint32),
                ("staging_bytes", ctypes.c_uint64), ("storage", ctypes.c_void_p),
                ("storage_bytes", ctypes.c_uint64)]


GZ_TIER_HBM = 0
GZ_TIER_HOST = 1


class gz_tuning(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_uint32), ("lds_rows", ctypes.c_uint32),
                ("chunk", ctypes.c_uint32), ("wgs_per_cu", ctypes.c_uint32),
                ("group_blocks", ctypes.c_uint32), ("node_chunk", ctypes.c_uint32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class gz_peaks(ctypes.Structure):
    _fields_ = [("copy_gbs", ctypes.c_double), ("mul_lo_u32_tops", ctypes.c_double),
                ("mad_u64_u32_tops", ctypes.c_double), ("xor_b32_tops", ctypes.c_double),
                ("mad_u32_u24_tops", ctypes.c_double), ("add_u32_tops", ctypes.c_double),
                ("ctz_b32_tops", ctypes.c_double), ("cus", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class gz_profile(ctypes.Structure):
    _fields_ = [("group_ms", ctypes.c_float), ("update_ms", ctypes.c_float),
                ("ingest_ms", ctypes.c_float), ("calls", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


_lib = None

_SIGS = {
    "gz_sketch_init": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32, ctypes.c_uint64,
                        ctypes.POINTER(gz_config)], ctypes.c_int32),
    "gz_free": ([ctypes.c_void_p], ctypes.c_int32),
    "gz_shape": ([ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_uint32)] * 4
                 + [ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
    "gz_reset": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int32),
    "gz_update_sketch_batch": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64,
                                ctypes.c_uint32, ctypes.c_void_p], ctypes.c_int32),
    "gz_ingest": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p], ctypes.c_int32),
    "gz_ingest_noalloc": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                           ctypes.c_uint32, ctypes.c_void_p], ctypes.c_int32),
    "gz_ingest_multi": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32,
                         ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.c_uint32, ctypes.c_void_p], ctypes.c_int32),
    "gz_flush": ([ctypes.c_void_p], ctypes.c_int32),
    "gz_connected_components": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                 ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int32),
    "gz_list_spanning_forest": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                 ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
    "gz_query": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                  ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
    "gz_connected_components_multi": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32,
                                       ctypes.POINTER(ctypes.c_uint32),
                                       ctypes.POINTER(ctypes.c_uint32),
                                       ctypes.POINTER(ctypes.c_int32)], ctypes.c_int32),
    "gz_export_sketches": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                            ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)],
                           ctypes.c_int32),
    "gz_sketch_storage": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                           ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
    "gz_get_tuning": ([ctypes.c_void_p, ctypes.POINTER(gz_tuning)], ctypes.c_int32),
    "gz_set_tuning": ([ctypes.c_void_p, ctypes.POINTER(gz_tuning)], ctypes.c_int32),
    "gz_autotune": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                     ctypes.c_uint32, ctypes.c_void_p, ctypes.POINTER(gz_tuning),
                     ctypes.POINTER(ctypes.c_float)], ctypes.c_int32),
    "gz_profile_enable": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int32),
    "gz_profile_last": ([ctypes.c_void_p, ctypes.POINTER(gz_profile)], ctypes.c_int32),
    "gz_plan_create": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32,
                        ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p,
                        ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int32),
    "gz_plan_ingest": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p,
                        ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p], ctypes.c_int32),
    "gz_plan_free": ([ctypes.c_void_p], ctypes.c_int32),
    "gz_measure_peaks": ([ctypes.POINTER(gz_peaks), ctypes.c_void_p], ctypes.c_int32),
    "gz_l0_init": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32, ctypes.c_uint64],
                   ctypes.c_int32),
    "gz_l0_free": ([ctypes.c_void_p], ctypes.c_int32),
    "gz_l0_reset": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int32),
    "gz_l0_shape": ([ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_uint32)] * 4
                    + [ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
    "gz_l0_ingest": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p], ctypes.c_int32),
    "gz_l0_last_update_ms": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)], ctypes.c_int32),
    "gz_l0_export": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                      ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
    "gz_l0_sample": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int32),
                      ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int64)],
                     ctypes.c_int32),
    "gz_status_str": ([ctypes.c_int32], ctypes.c_char_p),
    "gz_last_error": ([], ctypes.c_char_p),
}

# exported names declared in include/gz.h and the optional server/autotune headers
EXPORTED = list(_SIGS)


def lib():
    """Load libgz.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _extend_server(L)
    _lib = L
    return L


def _extend_server(L):
    from . import server as _srv  # noqa: F401  (declares the server entry points)
    _srv._declare(L)


# Handles still open when the interpreter exits are released by an exit hook,
# in dependency order (servers, then plans, then graphs), while the HIP runtime
# is still up: the library never frees device memory from static destructors.
_live = {"server": weakref.WeakSet(), "plan": weakref.WeakSet(), "graph": weakref.WeakSet()}


def _track(kind, obj):
    _live[kind].add(obj)


def close_all():
    """Release every server, plan and graph this process still holds."""
    for kind in ("server", "plan", "graph"):
        for obj in list(_live[kind]):
            try:
                obj.close()
            except Exception:
                pass


atexit.register(close_all)


def _status_name(s: int) -> str:
    try:
        return lib().gz_status_str(s).decode()
    except Exception:  # library not loaded yet
        return str(s)


def check(status: int, allow=()):
    if status != GZ_OK and status not in allow:
        raise GzError(status, lib().gz_last_error().decode())
    return status


# ------------------------------------------------------------- marshalling


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _stream_handle(stream):
    if stream is not None:
        return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    try:
        import torch

        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return ctypes.c_void_p(0)


def _u32_arg(x):
    """-> (pointer, flags, keepalive) for a uint32 array on the host or the device."""
    if _is_torch(x):
        import torch

        if x.dtype not in (torch.int32, torch.uint32):
            raise TypeError("expected an int32/uint32 tensor")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if x.is_cuda:
            return ctypes.c_void_p(x.data_ptr()), GZ_DEVICE_PTR, x
        x = x.numpy()
    a = np.ascontiguousarray(x, dtype=np.uint32)
    return ctypes.c_void_p(a.ctypes.data), 0, a


class Graph:
    """One graph's node sketches (in HBM, or in pinned host memory with host_tier=True)."""

    def __init__(self, V: int, seed: int, rounds: int = 0, host_tier: bool = False,
                 staging_bytes: int = 0, storage=None):
        """storage: optional device tensor that holds the sketches (kept alive by the graph)."""
        L = lib()
        h = ctypes.c_void_p()
        cfg = gz_config(rounds, GZ_TIER_HOST if host_tier else GZ_TIER_HBM, int(staging_bytes))
        if storage is not None:
            cfg.storage = storage.data_ptr()
            cfg.storage_bytes = storage.numel() * storage.element_size()
            self._storage = storage
        check(L.gz_sketch_init(ctypes.byref(h), V, seed & 0xFFFFFFFFFFFFFFFF, ctypes.byref(cfg)))
        self._h = h
        _track("graph", self)
        self.seed = seed
        dims = [ctypes.c_uint32() for _ in range(4)]
        n = ctypes.c_uint64()
        check(L.gz_shape(h, *[ctypes.byref(d) for d in dims], ctypes.byref(n)))
        self.V, self.R, self.C, self.B = (d.value for d in dims)
        self.n = n.value

    @classmethod
    def borrowed(cls, h):
        """A view of a graph owned elsewhere (a server session): close() frees nothing."""
        self = cls.__new__(cls)
        self._h = h
        self._borrowed = True
        self.seed = None
        L = lib()
        dims = [ctypes.c_uint32() for _ in range(4)]
        n = ctypes.c_uint64()
        check(L.gz_shape(h, *[ctypes.byref(d) for d in dims], ctypes.byref(n)))
        self.V, self.R, self.C, self.B = (d.value for d in dims)
        self.n = n.value
        return self

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            if not getattr(self, "_borrowed", False):
                lib().gz_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ingestion ---------------------------------------------------------
    def ingest(self, src, dst, flags: int = 0, stream=None, op=None):
        """op: optional per-update insert/delete flags (uint8, same memory as src); the
        library never reads them (insertions and deletions are the same toggle)."""
        ps, fs, ks = _u32_arg(src)
        pd, fd, kd = _u32_arg(dst)
        if fs != fd:
            raise ValueError("src and dst must both live on the host or both on the device")
        n = len(ks)
        if len(kd) != n:
            raise ValueError("src and dst lengths differ")
        pop, kop = None, None
        if op is not None:
            if len(op) != n:
                raise ValueError("op length differs from src")
            if _is_torch(op):
                kop = op
                pop = ctypes.c_void_p(op.data_ptr())
            else:
                kop = np.ascontiguousarray(op, np.uint8)
                pop = ctypes.c_void_p(kop.ctypes.data)
        return check(lib().gz_ingest(self._h, ps, pd, pop, n, fs | flags, _stream_handle(stream)))

    def ingest_noalloc(self, src, dst, flags: int = 0, stream=None):
        """gz_ingest_noalloc: device arrays only, always asynchronous, no device allocation."""
        ps, fs, ks = _u32_arg(src)
        pd, fd, kd = _u32_arg(dst)
        if not (fs & fd & GZ_DEVICE_PTR):
            raise ValueError("gz_ingest_noalloc takes device arrays")
        if len(kd) != len(ks):
            raise ValueError("src and dst lengths differ")
        return check(lib().gz_ingest_noalloc(self._h, ps, pd, len(ks), GZ_DEVICE_PTR | flags,
                                             _stream_handle(stream)))

    def update_sketch_batch(self, node: int, nbrs, flags: int = 0, stream=None):
        p, f, k = _u32_arg(nbrs)
        return check(lib().gz_update_sketch_batch(self._h, node, p, len(k), f | flags,
                                                  _stream_handle(stream)))

    def reset(self, stream=None):
        return check(lib().gz_reset(self._h, _stream_handle(stream)))

    def flush(self):
        return check(lib().gz_flush(self._h))

    # queries -----------------------------------------------------------
    def query(self, forest: bool = True):
        """-> (status, labels uint32[V], num_cc, forest uint32[F, 2] or None)."""
        labels = np.zeros(self.V, np.uint32)
        ncc = ctypes.c_uint32()
        edges = np.zeros(2 * max(self.V - 1, 1), np.uint32) if forest else None
        ne = ctypes.c_uint64()
        st = lib().gz_query(
            self._h, labels.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(ncc),
            edges.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)) if forest else None,
            ctypes.byref(ne) if forest else None)
        check(st, allow=(GZ_ESKETCH_FAIL,))
        f = edges[: 2 * ne.value].reshape(-1, 2).copy() if forest else None
        return st, labels, ncc.value, f

    def connected_components(self):
        labels = np.zeros(self.V, np.uint32)
        ncc = ctypes.c_uint32()
        st = lib().gz_connected_components(
            self._h, labels.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(ncc))
        check(st, allow=(GZ_ESKETCH_FAIL,))
        return st, labels, ncc.value

    def list_spanning_forest(self):
        edges = np.zeros(2 * max(self.V - 1, 1), np.uint32)
        ne = ctypes.c_uint64()
        st = lib().gz_list_spanning_forest(
            self._h, edges.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(ne))
        check(st, allow=(GZ_ESKETCH_FAIL,))
        return st, edges[: 2 * ne.value].reshape(-1, 2).copy()

    def export(self, lo: int = 0, hi: int | None = None):
        """Canonical nested sketches: (alpha, gamma) uint64[hi-lo, R, C, B]."""
        hi = self.V if hi is None else hi
        shape = (hi - lo, self.R, self.C, self.B)
        a = np.zeros(shape, np.uint64)
        g = np.zeros(shape, np.uint64)
        check(lib().gz_export_sketches(self._h, lo, hi,
                                       a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                       g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return a, g

    def storage(self):
        p = ctypes.c_void_p()
        n = ctypes.c_uint64()
        check(lib().gz_sketch_storage(self._h, ctypes.byref(p), ctypes.byref(n)))
        return p.value, n.value

    def autotune(self, src, dst, stream=None):
        """Time candidate launch configurations on a device-resident sample; keep the best."""
        ps, fs, ks = _u32_arg(src)
        pd, fd, kd = _u32_arg(dst)
        if not (fs & fd & GZ_DEVICE_PTR):
            raise ValueError("autotune needs the sample in device memory")
        best = gz_tuning()
        ms = ctypes.c_float()
        check(lib().gz_autotune(self._h, ps, pd, len(ks), GZ_DEVICE_PTR, _stream_handle(stream),
                                ctypes.byref(best), ctypes.byref(ms)))
        return best.as_dict(), float(ms.value)

    def profile(self, on: bool = True):
        check(lib().gz_profile_enable(self._h, int(on)))

    def last_profile(self) -> dict:
        p = gz_profile()
        check(lib().gz_profile_last(self._h, ctypes.byref(p)))
        return {"group_ms": p.group_ms, "update_ms": p.update_ms, "ingest_ms": p.ingest_ms,
                "calls": p.calls}

    @property
    def tuning(self) -> dict:
        t = gz_tuning()
        check(lib().gz_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = gz_tuning()
        check(lib().gz_get_tuning(self._h, ctypes.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        check(lib().gz_set_tuning(self._h, ctypes.byref(t)))


class L0Sketch:
    """Standard l0-sampler node sketches (Fig. agm_code) on the device, for comparison."""

    def __init__(self, V: int, seed: int):
        h = ctypes.c_void_p()
        check(lib().gz_l0_init(ctypes.byref(h), V, seed & 0xFFFFFFFFFFFFFFFF))
        self._h = h
        _track("graph", self)
        dims = [ctypes.c_uint32() for _ in range(4)]
        n = ctypes.c_uint64()
        check(lib().gz_l0_shape(h, *[ctypes.byref(d) for d in dims], ctypes.byref(n)))
        self.V, self.R, self.C, self.B = (d.value for d in dims)
        self.n = n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().gz_l0_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ingest(self, src, dst, op=None, stream=None):
        ps, fs, ks = _u32_arg(src)
        pd, fd, kd = _u32_arg(dst)
        if fs != fd:
            raise ValueError("src and dst must both live on the host or both on the device")
        pop, kop = None, None
        if op is not None:
            if _is_torch(op):
                if bool(op.is_cuda) != bool(fs & GZ_DEVICE_PTR):
                    raise ValueError("op must live where src and dst do")
                kop, pop = op, ctypes.c_void_p(op.data_ptr())
            else:
                if fs & GZ_DEVICE_PTR:
                    raise ValueError("op must live where src and dst do")
                kop = np.ascontiguousarray(op, np.uint8)
                pop = ctypes.c_void_p(kop.ctypes.data)
        return check(lib().gz_l0_ingest(self._h, ps, pd, pop, len(ks), fs, _stream_handle(stream)))

    def reset(self, stream=None):
        return check(lib().gz_l0_reset(self._h, _stream_handle(stream)))

    def last_update_ms(self) -> float:
        ms = ctypes.c_float()
        check(lib().gz_l0_last_update_ms(self._h, ctypes.byref(ms)))
        return float(ms.value)

    def export(self, lo: int = 0, hi: int | None = None):
        """(a, b, c): int64, int64, uint64 [hi-lo, R, C, B] in the figure's nested rows."""
        hi = self.V if hi is None else hi
        shape = (hi - lo, self.R, self.C, self.B)
        a = np.zeros(shape, np.int64)
        b = np.zeros(shape, np.int64)
        c = np.zeros(shape, np.uint64)
        check(lib().gz_l0_export(self._h, lo, hi, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 b.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return a, b, c

    def sample(self, r: int):
        """-> kind int32[V] (0 zero, 1 sample, 2 fail), idx uint64[V], mult int64[V]."""
        kind = np.zeros(self.V, np.int32)
        idx = np.zeros(self.V, np.uint64)
        mult = np.zeros(self.V, np.int64)
        check(lib().gz_l0_sample(self._h, r, kind.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                 mult.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return kind, idx, mult


def _handles(graphs):
    arr = (ctypes.c_void_p * len(graphs))(*[g.handle for g in graphs])
    return arr


def ingest_multi(graphs, offs, src, dst, flags: int = 0, stream=None):
    """Fused ingest over several graphs: updates offs[k]..offs[k+1]-1 go to graphs[k]."""
    ps, fs, ks = _u32_arg(src)
    pd, fd, kd = _u32_arg(dst)
    if fs != fd:
        raise ValueError("src and dst must both live on the host or both on the device")
    o = np.ascontiguousarray(offs, np.uint64)
    if len(o) != len(graphs) + 1:
        raise ValueError("offs needs len(graphs)+1 entries")
    return check(lib().gz_ingest_multi(_handles(graphs), len(graphs),
                                       o.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), ps, pd,
                                       fs | flags, _stream_handle(stream)))


def connected_components_multi(graphs, out=None):
    """-> (labels per graph (list of uint32 arrays), num_cc uint32[G], status int32[G]).

    out: optional caller-owned uint32 array of at least sum(V) labels (for example
    a view of pinned host memory, reused across calls); the per-graph label
    arrays are views of it.
    """
    G = len(graphs)
    total = sum(g.V for g in graphs)
    if out is None:
        labels = np.zeros(total, np.uint32)
    else:
        labels = out
        if labels.dtype != np.uint32 or labels.ndim != 1 or labels.size < total \
                or not labels.flags["C_CONTIGUOUS"]:
            raise ValueError(f"out must be a contiguous uint32 array of at least {total} labels")
    ncc = np.zeros(G, np.uint32)
    stt = np.zeros(G, np.int32)
    st = lib().gz_connected_components_multi(
        _handles(graphs), G, labels.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
        ncc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
        stt.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    check(st, allow=(GZ_ESKETCH_FAIL,))
    out, o = [], 0
    for g in graphs:
        out.append(labels[o:o + g.V])
        o += g.V
    return out, ncc, stt


class Plan:
    """A captured (HIP graph) ingest sequence over a fixed set of graphs."""

    def __init__(self, graphs, caps, stream=None):
        self.graphs = list(graphs)  # keep the graphs alive
        c = np.ascontiguousarray(caps, np.uint64)
        if len(c) != len(self.graphs):
            raise ValueError("one capacity per graph")
        h = ctypes.c_void_p()
        check(lib().gz_plan_create(_handles(self.graphs), len(self.graphs),
                                   c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                   _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        _track("plan", self)

    def ingest(self, offs, src, dst, flags: int = 0, stream=None):
        ps, fs, ks = _u32_arg(src)
        pd, fd, kd = _u32_arg(dst)
        if not (fs & fd & GZ_DEVICE_PTR):
            raise ValueError("plans take device arrays")
        o = np.ascontiguousarray(offs, np.uint64)
        return check(lib().gz_plan_ingest(self._h, o.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                          ps, pd, GZ_DEVICE_PTR | flags, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().gz_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def measure_peaks(stream=None) -> dict:
    """Device copy bandwidth and integer VALU issue rates (gz_measure_peaks)."""
    p = gz_peaks()
    check(lib().gz_measure_peaks(ctypes.byref(p), _stream_handle(stream)))
    return {f: (float(getattr(p, f)) if t is ctypes.c_double else int(getattr(p, f)))
            for f, t in p._fields_ if f != "reserved"}
