"""Seeded synthetic edge streams shared by the tests, the smoke check and the benchmark.

This module only produces inputs: arrays of (u, v) node pairs with an op code
(1 = insert, 0 = delete).  It holds none of the sketching arithmetic; the CPU
oracle and the GPU library each turn pairs into sketches on their own.

The generators live in ``gen.c`` (PCG32-driven, see its header) and are built
into ``_gen.so`` by :func:`build`.  The workload recipes below stand in for the
paper's Graph500 Kronecker streams (Sec. 6.1), which are not available here.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_SO = os.path.join(_HERE, "_gen.so")
_lib = None


def build() -> str:
    """Compile the generator library (gcc, host only)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp,
                           "-lm"])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        raise RuntimeError(f"workload generator not built: {_SO} (run __graft_entry__.build())")
    L = ctypes.CDLL(_SO)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    f64p = ctypes.POINTER(ctypes.c_double)
    c_u32, c_u64, c_f64, c_i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_int64
    L.gen_uniform.argtypes = [c_u32, c_u64, c_u64, c_u64, u32p, u32p, u8p]
    L.gen_uniform.restype = ctypes.c_int
    L.gen_rmat_phased.argtypes = [c_u32, c_f64, c_f64, c_f64, c_f64, c_f64, c_f64, c_u64,
                                  u32p, u32p, u8p, c_u64]
    L.gen_rmat_phased.restype = c_i64
    L.gen_rmat_interleaved.argtypes = [c_u32, c_f64, c_f64, c_f64, c_f64, c_u64, c_f64, c_u64,
                                       u32p, u32p, u8p]
    L.gen_rmat_interleaved.restype = c_i64
    L.gen_gnp.argtypes = [c_u32, c_f64, c_f64, c_u64, u32p, u32p, u8p, c_u64]
    L.gen_gnp.restype = c_i64
    L.gen_rmat_session.argtypes = [c_u32, c_f64, c_f64, c_f64, c_f64, c_u64, c_f64, c_u64,
                                   u32p, u32p, u8p, u64p]
    L.gen_rmat_session.restype = c_i64
    L.gen_rmat_draws.argtypes = [c_u32, c_f64, c_f64, c_f64, c_u64, c_u64, c_u32, u32p, u32p]
    L.gen_rmat_draws.restype = c_i64
    L.gen_uniform_u64.argtypes = [c_u64, c_u64, c_u64, c_u64, u64p]
    L.gen_uniform_u64.restype = None
    L.gen_unit_f64.argtypes = [c_u64, c_u64, c_u64, f64p]
    L.gen_unit_f64.restype = None
    _lib = L
    return L


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclass
class Stream:
    """An edge-update stream over nodes [0, V)."""

    V: int
    src: np.ndarray  # uint32[N]
    dst: np.ndarray  # uint32[N]
    op: np.ndarray   # uint8[N], 1 insert / 0 delete (the sketches ignore it)
    name: str = ""

    @property
    def N(self) -> int:
        return int(self.src.shape[0])


def uniform_stream(V: int, n_ins: int, n_del: int, seed: int) -> Stream:
    L = _load()
    N = n_ins + n_del
    src = np.empty(N, np.uint32)
    dst = np.empty(N, np.uint32)
    op = np.empty(N, np.uint8)
    rc = L.gen_uniform(V, n_ins, n_del, seed, _ptr(src, ctypes.c_uint32),
                       _ptr(dst, ctypes.c_uint32), _ptr(op, ctypes.c_uint8))
    if rc != 0:
        raise ValueError("gen_uniform: bad arguments")
    return Stream(V, src, dst, op, f"uniform(V={V},ins={n_ins},del={n_del},seed={seed})")


def rmat_phased(V: int, abcd, target_edges: float, del_frac: float, seed: int) -> Stream:
    L = _load()
    a, b, c, d = abcd
    cap = int(target_edges * (1.0 + del_frac) * 1.02 + 64 * math.sqrt(target_edges) + 4096)
    src = np.empty(cap, np.uint32)
    dst = np.empty(cap, np.uint32)
    op = np.empty(cap, np.uint8)
    n = L.gen_rmat_phased(V, a, b, c, d, float(target_edges), del_frac, seed,
                          _ptr(src, ctypes.c_uint32), _ptr(dst, ctypes.c_uint32),
                          _ptr(op, ctypes.c_uint8), cap)
    if n < 0:
        raise ValueError("gen_rmat_phased failed (V must be a power of two)")
    return Stream(V, src[:n].copy(), dst[:n].copy(), op[:n].copy(),
                  f"rmat_phased(V={V},abcd={tuple(abcd)},E~{target_edges:g},del={del_frac},seed={seed})")


def rmat_interleaved(V: int, abcd, n_steps: int, del_prob: float, seed: int) -> Stream:
    L = _load()
    a, b, c, d = abcd
    src = np.empty(n_steps, np.uint32)
    dst = np.empty(n_steps, np.uint32)
    op = np.empty(n_steps, np.uint8)
    n = L.gen_rmat_interleaved(V, a, b, c, d, n_steps, del_prob, seed,
                               _ptr(src, ctypes.c_uint32), _ptr(dst, ctypes.c_uint32),
                               _ptr(op, ctypes.c_uint8))
    if n < 0:
        raise ValueError("gen_rmat_interleaved failed (V must be a power of two)")
    return Stream(V, src[:n].copy(), dst[:n].copy(), op[:n].copy(),
                  f"rmat_interleaved(V={V},abcd={tuple(abcd)},steps={n_steps},del={del_prob},seed={seed})")


def rmat_draws(V: int, abcd, n: int, seed: int, threads: int = 0) -> Stream:
    """n raw R-MAT draws (self-loops redrawn); a pair drawn again toggles its edge.
    The stream does not depend on `threads` (0 = one per CPU, at most 16)."""
    L = _load()
    a, b, c, _ = abcd
    src = np.empty(n, np.uint32)
    dst = np.empty(n, np.uint32)
    t = threads or min(16, os.cpu_count() or 1)
    if L.gen_rmat_draws(V, a, b, c, n, seed, t, _ptr(src, ctypes.c_uint32),
                        _ptr(dst, ctypes.c_uint32)) < 0:
        raise ValueError("gen_rmat_draws failed (V must be a power of two)")
    return Stream(V, src, dst, np.ones(n, np.uint8),
                  f"rmat_draws(V={V},abcd={tuple(abcd)},n={n},seed={seed})")


def gnp(V: int, p: float, del_frac: float, seed: int) -> Stream:
    L = _load()
    npairs = V * (V - 1) // 2
    mean = npairs * p
    cap = int((mean + 8 * math.sqrt(mean) + 64) * (1.0 + del_frac) + 64)
    src = np.empty(cap, np.uint32)
    dst = np.empty(cap, np.uint32)
    op = np.empty(cap, np.uint8)
    n = L.gen_gnp(V, p, del_frac, seed, _ptr(src, ctypes.c_uint32), _ptr(dst, ctypes.c_uint32),
                  _ptr(op, ctypes.c_uint8), cap)
    if n < 0:
        raise ValueError("gen_gnp failed")
    return Stream(V, src[:n].copy(), dst[:n].copy(), op[:n].copy(),
                  f"gnp(V={V},p={p:.5f},del={del_frac},seed={seed})")


def rmat_session(V: int, abcd, n_updates: int, del_prob: float, seed: int) -> tuple[Stream, int]:
    L = _load()
    a, b, c, d = abcd
    src = np.empty(n_updates, np.uint32)
    dst = np.empty(n_updates, np.uint32)
    op = np.empty(n_updates, np.uint8)
    fb = ctypes.c_uint64(0)
    n = L.gen_rmat_session(V, a, b, c, d, n_updates, del_prob, seed,
                           _ptr(src, ctypes.c_uint32), _ptr(dst, ctypes.c_uint32),
                           _ptr(op, ctypes.c_uint8), ctypes.byref(fb))
    if n < 0:
        raise ValueError("gen_rmat_session failed")
    return Stream(V, src, dst, op, f"rmat_session(V={V},n={n_updates},seed={seed})"), int(fb.value)


def uniform_ints(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    """n integers uniform on [lo, hi] (inclusive)."""
    L = _load()
    out = np.empty(n, np.uint64)
    L.gen_uniform_u64(seed, n, lo, hi, _ptr(out, ctypes.c_uint64))
    return out


def unit_floats(seed: int, stream: int, n: int) -> np.ndarray:
    """n doubles uniform on [0, 1)."""
    L = _load()
    out = np.empty(n, np.float64)
    L.gen_unit_f64(seed, stream, n, _ptr(out, ctypes.c_double))
    return out


# --------------------------------------------------------------- graph helpers


def final_edges(s: Stream) -> tuple[np.ndarray, np.ndarray]:
    """Edges present after the stream, as canonical (u < v) pairs.

    Each update toggles its pair, so the final graph is the set of pairs that
    occur an odd number of times.
    """
    u = np.minimum(s.src, s.dst).astype(np.int64)
    v = np.maximum(s.src, s.dst).astype(np.int64)
    key = u * s.V + v
    k, cnt = np.unique(key, return_counts=True)
    k = k[(cnt & 1) == 1]
    return (k // s.V).astype(np.uint32), (k % s.V).astype(np.uint32)


def union_find_labels(V: int, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Component label (smallest member id) of every node, by plain union-find."""
    parent = list(range(V))

    def find(x: int) -> int:
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in zip(u.tolist(), v.tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            if ra < rb:
                parent[rb] = ra
            else:
                parent[ra] = rb
    return np.array([find(x) for x in range(V)], np.uint32)


def scipy_labels(V: int, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Component labels (smallest member id) via scipy's connected_components (large graphs)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    m = sp.coo_matrix((np.ones(len(u), np.int8), (u.astype(np.int64), v.astype(np.int64))),
                      shape=(V, V)).tocsr()
    _, lab = connected_components(m, directed=False)
    # relabel each component by its smallest node id
    first = np.full(lab.max() + 1 if V else 0, V, np.int64)
    np.minimum.at(first, lab, np.arange(V))
    return first[lab].astype(np.uint32)


# ------------------------------------------------------------- workload recipes

RMAT_GRAPH500 = (0.57, 0.19, 0.19, 0.05)
RMAT_SKEWED = (0.7, 0.1, 0.1, 0.1)


def config_uniform_small(seed: int = 1) -> Stream:
    """V=1024, 150k uniform distinct inserts then 50k uniform live deletes."""
    return uniform_stream(1024, 150_000, 50_000, seed)


def config_rmat_dense(seed: int = 2, V: int = 1 << 14, edges: float = 50e6) -> Stream:
    """V=2^14 Graph500-initiator R-MAT, ~50M distinct inserts then 10% live deletes."""
    return rmat_phased(V, RMAT_GRAPH500, edges, 0.10, seed)


def config_rmat_skewed(seed: int = 3, V: int = 1 << 15, steps: int = 150_000_000) -> Stream:
    """V=2^15 skewed R-MAT, ~150M updates with 20% deletes interleaved."""
    return rmat_interleaved(V, RMAT_SKEWED, steps, 0.20, seed)


PHI64 = 0x9E3779B97F4A7C15  # floor(2^64 / golden ratio)


def many_graph_seed(base: int, g: int) -> int:
    """Sketch seed of graph g in the many-instance workload."""
    return (base ^ ((g + 1) * PHI64)) & 0xFFFFFFFFFFFFFFFF


def config_many_gnp(seed: int = 4, G: int = 4096, vlo: int = 64, vhi: int = 2048,
                    plo: float = 0.001, phi: float = 0.05, del_frac: float = 0.30):
    """G independent G(n,p) graphs: V ~ U{vlo..vhi}, p ~ U(plo, phi), 30% deletes."""
    Vs = uniform_ints(seed, G, vlo, vhi).astype(np.int64)
    ps = plo + (phi - plo) * unit_floats(seed, 1, G)
    streams = [gnp(int(Vs[g]), float(ps[g]), del_frac, seed * 1_000_003 + g) for g in range(G)]
    return streams


def serving_sessions(seed: int = 5, S: int = 256, vlo_log2: float = 10.0, vhi_log2: float = 16.0):
    """Per-session node counts V = round(2^U(10,16)) for the serving workload."""
    u = unit_floats(seed, 2, S)
    return [int(round(2.0 ** (vlo_log2 + (vhi_log2 - vlo_log2) * x))) for x in u]


def pareto_batch_sizes(seed: int, stream: int, n: int, xmin: int = 1000, xmax: int = 1_000_000,
                       alpha: float = 1.5) -> np.ndarray:
    """Truncated Pareto(alpha) batch lengths on [xmin, xmax]."""
    u = unit_floats(seed, stream, n)
    x = np.floor(xmin * np.power(1.0 - u, -1.0 / alpha))
    return np.minimum(x, xmax).astype(np.int64)
