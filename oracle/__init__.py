"""CPU oracle for CubeSketch ingestion and Boruvka connectivity -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never loads it, and the two share no
code: the oracle is plain C (``cubesketch_oracle.c``) driven through ctypes.

Parity pins (see ``tests/test_oracle_pins.py``): edge-index bijection, the
SplitMix64 known-answer sequence, hash uniformity and pairwise independence,
sketch bits against the closed form of Eq. (1)-(2), order independence,
linearity under XOR, exact recovery for support size one, sampled index in
the support, the per-column success bound of Lemma "goodset", and component
labels against brute-force union-find.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cubesketch_oracle.c")
_SO = os.path.join(_HERE, "_oracle.so")
_lib = None

EMPTY, GOOD, BAD = 0, 1, 2
ZERO, SAMPLE, FAIL = 0, 1, 2
OK, SKETCH_FAIL = 0, 1
C_COLUMNS = 8


_SRC_L0 = os.path.join(_HERE, "l0_oracle.c")


def build() -> str:
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, _SRC_L0, "-o", tmp])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        raise RuntimeError(f"oracle not built: {_SO} (run __graft_entry__.build())")
    L = ctypes.CDLL(_SO)
    u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    u32p = ctypes.POINTER(u32)
    u64p = ctypes.POINTER(u64)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    vp = ctypes.c_void_p
    L.oracle_shape.argtypes = [u32, u32p, u32p, u32p, u64p]
    L.oracle_shape.restype = i32
    L.oracle_edge_index.argtypes = [u32, u32]
    L.oracle_edge_index.restype = u64
    L.oracle_edge_decode.argtypes = [u64, u32p, u32p]
    L.oracle_edge_decode.restype = None
    L.oracle_splitmix64_next.argtypes = [u64p]
    L.oracle_splitmix64_next.restype = u64
    L.oracle_seed_table.argtypes = [u64, u32, u64p]
    L.oracle_seed_table.restype = None
    L.oracle_hash32.argtypes = [u64, u64, u64]
    L.oracle_hash32.restype = u32
    L.oracle_row_hash.argtypes = [u64p, u32, u32, u64]
    L.oracle_row_hash.restype = u32
    L.oracle_checksum.argtypes = [u64p, u32, u32, u64]
    L.oracle_checksum.restype = u64
    L.oracle_new.argtypes = [u32, u64, u32]
    L.oracle_new.restype = vp
    L.oracle_free.argtypes = [vp]
    L.oracle_free.restype = None
    L.oracle_dims.argtypes = [vp, u32p, u64p]
    L.oracle_dims.restype = None
    L.oracle_seed_ptr.argtypes = [vp]
    L.oracle_seed_ptr.restype = u64p
    L.oracle_alpha_ptr.argtypes = [vp]
    L.oracle_alpha_ptr.restype = u64p
    L.oracle_gamma_ptr.argtypes = [vp]
    L.oracle_gamma_ptr.restype = u64p
    L.oracle_seeds_valid.argtypes = [vp]
    L.oracle_seeds_valid.restype = i32
    L.oracle_update.argtypes = [vp, u32, u32]
    L.oracle_update.restype = i32
    L.oracle_ingest.argtypes = [vp, u32p, u32p, u64]
    L.oracle_ingest.restype = i32
    L.oracle_ingest_nodes.argtypes = [vp, u32p, u32p, u64, u8p]
    L.oracle_ingest_nodes.restype = i32
    L.oracle_bucket_class.argtypes = [u64p, u32, u32, u64, u64, u64]
    L.oracle_bucket_class.restype = i32
    L.oracle_query.argtypes = [u64p, u32, u32, u32, u64, u64p, u64p, u64p]
    L.oracle_query.restype = i32
    L.oracle_query_node.argtypes = [vp, u32, u32, u64p]
    L.oracle_query_node.restype = i32
    L.oracle_connected_components.argtypes = [vp, u32p, u32p, u64p, u32p]
    L.oracle_connected_components.restype = i32
    L.oracle_is_wide.argtypes = [u32]
    L.oracle_is_wide.restype = i32
    L.oracle_wide.argtypes = [vp]
    L.oracle_wide.restype = i32
    L.oracle_seed_table_wide.argtypes = [u64, u32, u64p]
    L.oracle_seed_table_wide.restype = None
    L.oracle_hash32_pair.argtypes = [u64, u64, u64, u32, u32]
    L.oracle_hash32_pair.restype = u32
    L.oracle_row_hash_pair.argtypes = [u64p, u32, u32, u32, u32]
    L.oracle_row_hash_pair.restype = u64
    L.oracle_checksum_pair.argtypes = [u64p, u32, u32, u32, u32]
    L.oracle_checksum_pair.restype = u64
    L.oracle_bucket_class_wide.argtypes = [u64p, u32, u32, u64, u64, u64]
    L.oracle_bucket_class_wide.restype = i32
    L.oracle_query_wide.argtypes = [u64p, u32, u32, u32, u64, u64p, u64p, u64p]
    L.oracle_query_wide.restype = i32
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.l0_mulmod.argtypes = [u64, u64]
    L.l0_mulmod.restype = u64
    L.l0_powmod.argtypes = [u64, u64]
    L.l0_powmod.restype = u64
    L.l0_new.argtypes = [u32, u64]
    L.l0_new.restype = vp
    L.l0_free.argtypes = [vp]
    L.l0_free.restype = None
    L.l0_dims.argtypes = [vp, u32p, u64p]
    L.l0_dims.restype = None
    L.l0_a_ptr.argtypes = [vp]
    L.l0_a_ptr.restype = i64p
    L.l0_b_ptr.argtypes = [vp]
    L.l0_b_ptr.restype = i64p
    L.l0_c_ptr.argtypes = [vp]
    L.l0_c_ptr.restype = u64p
    L.l0_z_ptr.argtypes = [vp]
    L.l0_z_ptr.restype = u64p
    L.l0_update.argtypes = [vp, u32, u32, ctypes.c_int]
    L.l0_update.restype = i32
    L.l0_ingest.argtypes = [vp, u32p, u32p, u8p, u64]
    L.l0_ingest.restype = i32
    L.l0_ingest_nodes.argtypes = [vp, u32p, u32p, u8p, u64, u8p]
    L.l0_ingest_nodes.restype = i32
    L.l0_query.argtypes = [vp, u32, i64p, i64p, u64p, u64p, i64p]
    L.l0_query.restype = i32
    L.l0_query_node.argtypes = [vp, u32, u32, u64p, i64p]
    L.l0_query_node.restype = i32
    _lib = L
    return L


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def shape(V: int):
    """(R, C, B, n) of the shape rule for V nodes."""
    L = _load()
    R, C, B, n = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
    if L.oracle_shape(V, ctypes.byref(R), ctypes.byref(C), ctypes.byref(B), ctypes.byref(n)):
        raise ValueError(f"unsupported V={V}")
    return R.value, C.value, B.value, n.value


def edge_index(u: int, v: int) -> int:
    return int(_load().oracle_edge_index(u, v))


def edge_decode(i: int):
    u, v = ctypes.c_uint32(), ctypes.c_uint32()
    _load().oracle_edge_decode(i, ctypes.byref(u), ctypes.byref(v))
    return u.value, v.value


def splitmix64(seed: int, count: int):
    st = ctypes.c_uint64(seed)
    L = _load()
    return [int(L.oracle_splitmix64_next(ctypes.byref(st))) for _ in range(count)]


def seed_table(seed: int, R: int) -> np.ndarray:
    """uint64[R, C, 3, 2]: (multiplier, increment) of h1, checksum-high, checksum-low."""
    tab = np.zeros(R * C_COLUMNS * 6, np.uint64)
    _load().oracle_seed_table(seed, R, _p(tab, ctypes.c_uint64))
    return tab.reshape(R, C_COLUMNS, 3, 2)


def hash32_pair(a: int, a2: int, b: int, u: int, v: int) -> int:
    return int(_load().oracle_hash32_pair(a, a2, b, u, v))


def seed_table_wide(seed: int, R: int) -> np.ndarray:
    """uint64[R, C, 4, 3]: (a, a2, b) of the row hash's low word, checksum high, checksum low,
    row hash's high word."""
    tab = np.zeros(R * 8 * 12, np.uint64)
    _load().oracle_seed_table_wide(seed, R, _p(tab, ctypes.c_uint64))
    return tab.reshape(R, 8, 4, 3)


def is_wide(V: int) -> bool:
    return bool(_load().oracle_is_wide(V))


def hash32(a: int, b: int, x: int) -> int:
    return int(_load().oracle_hash32(a, b, x))


class Oracle:
    """Sketch state of one graph: alpha/gamma uint64[V, R, C, B], all zero at start."""

    def __init__(self, V: int, seed: int, R: int | None = None):
        L = _load()
        self._h = L.oracle_new(V, seed, R or 0)
        if not self._h:
            raise ValueError(f"oracle_new failed for V={V}")
        dims = (ctypes.c_uint32 * 4)()
        n = ctypes.c_uint64()
        L.oracle_dims(self._h, dims, ctypes.byref(n))
        self.V, self.R, self.C, self.B = (int(x) for x in dims)
        self.n = int(n.value)
        self.seed = seed
        cells = self.V * self.R * self.C * self.B
        self.alpha = np.ctypeslib.as_array(L.oracle_alpha_ptr(self._h), shape=(cells,)).reshape(
            self.V, self.R, self.C, self.B)
        self.gamma = np.ctypeslib.as_array(L.oracle_gamma_ptr(self._h), shape=(cells,)).reshape(
            self.V, self.R, self.C, self.B)
        self._tab = L.oracle_seed_ptr(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().oracle_free(h)
            self._h = None

    @property
    def wide(self) -> bool:
        """V > 2^16: hashes keyed by the node pair, seeds (a, a2, b) per hash."""
        return bool(_load().oracle_wide(self._h))

    @property
    def seeds(self) -> np.ndarray:
        """[R, C, 3, 2] (multiplier, increment) or, for wide graphs, [R, C, 4, 3] (a, a2, b)."""
        k, w = (4, 3) if self.wide else (3, 2)
        n = self.R * self.C * k * w
        return np.ctypeslib.as_array(self._tab, shape=(n,)).reshape(self.R, self.C, k, w).copy()

    def seeds_valid(self) -> bool:
        return bool(_load().oracle_seeds_valid(self._h))

    def update(self, u: int, v: int) -> None:
        if _load().oracle_update(self._h, u, v):
            raise ValueError("invalid update")

    def ingest(self, src: np.ndarray, dst: np.ndarray) -> None:
        src = np.ascontiguousarray(src, np.uint32)
        dst = np.ascontiguousarray(dst, np.uint32)
        if _load().oracle_ingest(self._h, _p(src, ctypes.c_uint32), _p(dst, ctypes.c_uint32),
                                 len(src)):
            raise ValueError("invalid update in stream")

    def ingest_nodes(self, src: np.ndarray, dst: np.ndarray, nodes) -> None:
        """Apply only the endpoint halves of updates whose endpoint is in `nodes`."""
        src = np.ascontiguousarray(src, np.uint32)
        dst = np.ascontiguousarray(dst, np.uint32)
        keep = np.zeros(self.V, np.uint8)
        keep[np.asarray(nodes, np.int64)] = 1
        if _load().oracle_ingest_nodes(self._h, _p(src, ctypes.c_uint32),
                                       _p(dst, ctypes.c_uint32), len(src),
                                       _p(keep, ctypes.c_uint8)):
            raise ValueError("invalid update in stream")

    def row_hash(self, r: int, c: int, idx: int) -> int:
        if self.wide:
            u, v = edge_decode(idx)
            return int(_load().oracle_row_hash_pair(self._tab, r, c, u, v))
        return int(_load().oracle_row_hash(self._tab, r, c, idx))

    def checksum(self, r: int, c: int, idx: int) -> int:
        if self.wide:
            u, v = edge_decode(idx)
            return int(_load().oracle_checksum_pair(self._tab, r, c, u, v))
        return int(_load().oracle_checksum(self._tab, r, c, idx))

    def bucket_class(self, r: int, c: int, alpha: int, gamma: int) -> int:
        f = _load().oracle_bucket_class_wide if self.wide else _load().oracle_bucket_class
        return int(f(self._tab, r, c, self.n, alpha, gamma))

    def query(self, r: int, alpha_cb: np.ndarray, gamma_cb: np.ndarray):
        """Query a round-r CubeSketch given as [C, B] arrays -> (ZERO|SAMPLE|FAIL, idx)."""
        a = np.ascontiguousarray(alpha_cb, np.uint64)
        g = np.ascontiguousarray(gamma_cb, np.uint64)
        out = ctypes.c_uint64(0)
        f = _load().oracle_query_wide if self.wide else _load().oracle_query
        k = f(self._tab, r, self.C, self.B, self.n, _p(a, ctypes.c_uint64), _p(g, ctypes.c_uint64),
              ctypes.byref(out))
        return int(k), int(out.value)

    def query_node(self, v: int, r: int):
        out = ctypes.c_uint64(0)
        k = _load().oracle_query_node(self._h, v, r, ctypes.byref(out))
        return int(k), int(out.value)

    def connected_components(self):
        """-> (status, labels uint32[V], forest uint32[F, 2], rounds_used)."""
        labels = np.zeros(self.V, np.uint32)
        forest = np.zeros(2 * max(self.V - 1, 1), np.uint32)
        nf = ctypes.c_uint64()
        used = ctypes.c_uint32()
        st = _load().oracle_connected_components(self._h, _p(labels, ctypes.c_uint32),
                                                 _p(forest, ctypes.c_uint32), ctypes.byref(nf),
                                                 ctypes.byref(used))
        if st < 0:
            raise MemoryError("oracle_connected_components")
        return int(st), labels, forest[: 2 * nf.value].reshape(-1, 2).copy(), int(used.value)


# ------------------------------------------------ standard l0 sampler (Fig. agm_code)

L0_P = (1 << 61) - 1


def l0_mulmod(x: int, y: int) -> int:
    return int(_load().l0_mulmod(x, y))


def l0_powmod(z: int, e: int) -> int:
    return int(_load().l0_powmod(z, e))


class L0Oracle:
    """Standard l0-sampler node sketches: a, b int64 and c uint64 [V, R, C, B], zero at start."""

    def __init__(self, V: int, seed: int):
        L = _load()
        self._h = L.l0_new(V, seed)
        if not self._h:
            raise ValueError(f"l0_new failed for V={V}")
        dims = (ctypes.c_uint32 * 4)()
        n = ctypes.c_uint64()
        L.l0_dims(self._h, dims, ctypes.byref(n))
        self.V, self.R, self.C, self.B = (int(x) for x in dims)
        self.n = int(n.value)
        cells = self.V * self.R * self.C * self.B
        shp = (self.V, self.R, self.C, self.B)
        self.a = np.ctypeslib.as_array(L.l0_a_ptr(self._h), shape=(cells,)).reshape(shp)
        self.b = np.ctypeslib.as_array(L.l0_b_ptr(self._h), shape=(cells,)).reshape(shp)
        self.c = np.ctypeslib.as_array(L.l0_c_ptr(self._h), shape=(cells,)).reshape(shp)
        self.z = np.ctypeslib.as_array(L.l0_z_ptr(self._h), shape=(self.R * self.C,)).reshape(
            self.R, self.C).copy()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().l0_free(h)
            self._h = None

    def update(self, u: int, v: int, delta: int = 1) -> None:
        if _load().l0_update(self._h, u, v, delta):
            raise ValueError("invalid update")

    def ingest(self, src, dst, op=None) -> None:
        src = np.ascontiguousarray(src, np.uint32)
        dst = np.ascontiguousarray(dst, np.uint32)
        o = None if op is None else np.ascontiguousarray(op, np.uint8)
        if _load().l0_ingest(self._h, _p(src, ctypes.c_uint32), _p(dst, ctypes.c_uint32),
                             None if o is None else _p(o, ctypes.c_uint8), len(src)):
            raise ValueError("invalid update in stream")

    def ingest_nodes(self, src, dst, op, nodes) -> None:
        src = np.ascontiguousarray(src, np.uint32)
        dst = np.ascontiguousarray(dst, np.uint32)
        o = None if op is None else np.ascontiguousarray(op, np.uint8)
        keep = np.zeros(self.V, np.uint8)
        keep[np.asarray(nodes, np.int64)] = 1
        if _load().l0_ingest_nodes(self._h, _p(src, ctypes.c_uint32), _p(dst, ctypes.c_uint32),
                                   None if o is None else _p(o, ctypes.c_uint8), len(src),
                                   _p(keep, ctypes.c_uint8)):
            raise ValueError("invalid update in stream")

    def query(self, r: int, a_cb, b_cb, c_cb):
        """Query a round-r sampler given as [C, B] arrays -> (ZERO|SAMPLE|FAIL, idx, mult)."""
        a = np.ascontiguousarray(a_cb, np.int64)
        b = np.ascontiguousarray(b_cb, np.int64)
        c = np.ascontiguousarray(c_cb, np.uint64)
        idx = ctypes.c_uint64(0)
        mult = ctypes.c_int64(0)
        k = _load().l0_query(self._h, r, _p(a, ctypes.c_int64), _p(b, ctypes.c_int64),
                             _p(c, ctypes.c_uint64), ctypes.byref(idx), ctypes.byref(mult))
        return int(k), int(idx.value), int(mult.value)

    def query_node(self, v: int, r: int):
        idx = ctypes.c_uint64(0)
        mult = ctypes.c_int64(0)
        k = _load().l0_query_node(self._h, v, r, ctypes.byref(idx), ctypes.byref(mult))
        return int(k), int(idx.value), int(mult.value)
