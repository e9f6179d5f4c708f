"""Cache of autotuned ingest launch parameters.

The tuner itself runs in the library (gz_autotune: candidate launch shapes
timed with HIP events on a scratch graph).  This module keys its results by
device, workload kind and sketch shape.  Lookups read the cache packaged next
to this file (results of gz_autotune runs on MI355X, written by
``save_entry``), then the user cache; a shape found in neither is tuned on the
caller's sample and stored in the user cache.
"""
from __future__ import annotations

import json
import os

PACKAGED_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")
USER_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gz_mi355x_tuning.json")


def device_tag() -> str:
    try:
        import torch

        p = torch.cuda.get_device_properties(0)
        arch = getattr(p, "gcnArchName", "").split(":")[0]
        return f"{arch or p.name}|cu={p.multi_processor_count}"
    except Exception:
        return "unknown"


def key(graph, kind: str = "single") -> str:
    return f"{device_tag()}|{kind}|V={graph.V}|R={graph.R}|B={graph.B}"


def load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(graph, kind: str = "single"):
    """-> (tuning dict, source path) from the packaged or the user cache, or (None, None)."""
    k = key(graph, kind)
    for path in (PACKAGED_CACHE, USER_CACHE):
        entry = load(path).get(k)
        if entry:
            return dict(entry["tuning"]), path
    return None, None


def save_entry(graph, tuning: dict, ms: float, sample_updates: int, path: str = USER_CACHE,
               kind: str = "single") -> None:
    cache = load(path)
    cache[key(graph, kind)] = {"tuning": dict(tuning), "sample_updates": int(sample_updates),
                               "ingest_ms": float(ms)}
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned(graph, src_sample, dst_sample, kind: str = "single", refresh: bool = False,
          save_path: str = USER_CACHE):
    """Apply cached launch parameters for graph's shape, or tune on the sample and cache them.

    Returns (tuning dict, source): source names the cache file the tuple came
    from, or "gz_autotune" when it was tuned now.
    """
    if not refresh:
        t, path = lookup(graph, kind)
        if t is not None:
            graph.set_tuning(**t)
            return graph.tuning, path
    best, ms = graph.autotune(src_sample, dst_sample)
    try:
        save_entry(graph, best, ms, len(src_sample), save_path, kind)
    except OSError:
        pass
    return best, "gz_autotune"
