"""Persistent cache of autotuned ingest launch parameters.

The tuner itself runs in the library (gz_autotune: candidates timed with HIP
events on a scratch graph).  This module keys its results by device and sketch
shape and keeps them in a JSON file, so a shape is tuned once per device.
"""
from __future__ import annotations

import json
import os

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gz_mi355x_tuning.json")


def _device_name() -> str:
    try:
        import torch

        return torch.cuda.get_device_name(0)
    except Exception:
        return "unknown"


def _key(graph) -> str:
    return f"{_device_name()}|V={graph.V}|R={graph.R}|B={graph.B}"


def load(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned(graph, src_sample, dst_sample, path: str = DEFAULT_CACHE, refresh: bool = False):
    """Apply cached parameters for graph's shape, or tune on the sample and cache them.

    Returns (tuning dict, ingest ms of the sample or None when taken from the cache).
    """
    cache = load(path)
    key = _key(graph)
    if key in cache and not refresh:
        graph.set_tuning(**cache[key]["tuning"])
        return cache[key]["tuning"], None
    best, ms = graph.autotune(src_sample, dst_sample)
    cache[key] = {"tuning": best, "sample_updates": int(len(src_sample)), "ingest_ms": ms}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass
    return best, ms
