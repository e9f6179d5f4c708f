#!/usr/bin/env python3
"""Benchmark of the CubeSketch ingest + Boruvka connectivity hot path on one MI355X.

One step = zero the sketches, ingest the whole synthetic stream (device-side
grouping by endpoint + persistent LDS-staged sketch update) and answer a
connected-components query.  The stream is resident in HBM before timing.

Default workload: the dense R-MAT graph on V = 2^14 nodes (Graph500 initiator
a,b,c,d = 0.57,0.19,0.19,0.05, seed 2), ~50M distinct-edge inserts followed by
10% deletes of live edges, sketch shape R=15, C=8, B=28.

Besides the JSON line's `value` (whole-step updates/s) the line carries the
plain per-node-launch rate (one gz_update_sketch_batch launch per gutter of
half a node sketch, the paper's leaf-gutter size), the CC query time, the
roofline of the dominant kernel (measured with HIP events on its own stream)
and the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures used by the roofline (the design doc derives them)
PEAK_INT_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # VALU lane-instructions/s: 39.32 T
PEAK_HBM_GBS = 8000.0
# algorithmic integer ops per (update, round-column pair): the three hashes of the
# edge index (row hash 3, 64-bit checksum 6, depth 2) counted once per update,
# plus one exact-depth XOR of (alpha, gamma) per endpoint (4 each)
OPS_PER_UPDATE_PAIR = 19


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def make_workload(name: str):
    import workloads

    if name == "rmat_dense":
        s = workloads.config_rmat_dense()
        desc = ("R-MAT V=2^14 (a,b,c,d=0.57,0.19,0.19,0.05, seed 2): ~50M distinct inserts then "
                "10% live deletes")
        return s, 2, desc
    if name == "uniform_small":
        s = workloads.config_uniform_small()
        return s, 1, "uniform V=1024: 150k inserts then 50k deletes (seed 1)"
    if name == "rmat_skewed":
        s = workloads.config_rmat_skewed()
        desc = ("skewed R-MAT V=2^15 (0.7,0.1,0.1,0.1, seed 3): ~150M updates, 20% deletes "
                "interleaved")
        return s, 3, desc
    raise SystemExit(f"unknown workload {name}")


def traffic_from_profile(kernel_src_hash: str):
    """HBM bytes per launch of the update kernel from the committed PMC summary, or None.

    The summary records the hash of the kernel source it was taken with; a
    different hash means the kernel changed since, and the figure is stale.
    """
    path = os.path.join(ROOT, "profiles", "k_update_rmat_dense_pmc.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_src_hash:
        return None
    return float(t.group(1))


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2203_14927_amd", "csrc", "gz_ingest.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()


def cpu_baseline(stream, seed, seconds: float):
    """The oracle, untuned, single-threaded, on the first M updates of the same stream."""
    import oracle

    O = oracle.Oracle(stream.V, seed)
    probe = min(stream.N, 20000)
    t0 = time.perf_counter()
    O.ingest(stream.src[:probe], stream.dst[:probe])
    t1 = time.perf_counter()
    rate = probe / max(t1 - t0, 1e-9)
    M = int(min(stream.N - probe, max(1000, rate * seconds)))
    t0 = time.perf_counter()
    O.ingest(stream.src[probe:probe + M], stream.dst[probe:probe + M])
    t1 = time.perf_counter()
    del O
    return {"value": M / (t1 - t0), "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"updates {probe}..{probe + M} of the stream ({M} updates, ingest only, "
                      f"all {stream.V} node sketches, {t1 - t0:.1f} s)"}


def plain_pass(gz, g, stream, src_d, dst_d):
    """Plain path: one update_sketch_batch launch per node gutter, on pre-grouped input."""
    import torch

    V = stream.V
    u = torch.cat([src_d, dst_d]).long()
    v = torch.cat([dst_d, src_d])
    order = torch.sort(u, stable=False).indices
    nbrs = v[order].contiguous()
    counts = torch.bincount(u, minlength=V).cpu().numpy()
    del u, v, order
    offs = [0]
    for c in counts.tolist():
        offs.append(offs[-1] + c)
    gutter = max(1, (g.R * g.C * g.B * 16) // 2 // 4)  # half a node sketch at 4 B per update
    L = gz.lib()
    base = nbrs.data_ptr()
    h = g.handle
    flags = gz.GZ_DEVICE_PTR | gz.GZ_ASYNC | gz.GZ_UNCHECKED
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    calls = []
    for node in range(V):
        o, e = offs[node], offs[node + 1]
        for k in range(o, e, gutter):
            calls.append((node, base + 4 * k, min(gutter, e - k)))
    g.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for node, ptr, cnt in calls:
        st = L.gz_update_sketch_batch(h, node, ctypes.c_void_p(ptr), cnt, flags, s)
        if st:
            raise RuntimeError(f"plain batch failed: {st}")
    g.flush()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return stream.N / (t1 - t0), len(calls), gutter, (t1 - t0) * 1e3


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat_dense")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-node pass")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch parameters")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (a kernel of known traffic "
                         "that scales hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"this benchmark runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding is a design in DESIGN.md, not a built path", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2203_14927_amd as gz

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    stream, seed, desc = make_workload(args.workload)
    log(f"[bench] workload {args.workload}: V={stream.V} N={stream.N} "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    src_d = torch.from_numpy(stream.src.view(np.int32)).cuda()
    dst_d = torch.from_numpy(stream.dst.view(np.int32)).cuda()
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b
    g = gz.Graph(stream.V, seed=seed)
    tune_ms = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        best, tune_ms = g.autotune(src_d, dst_d)
        log(f"[bench] autotuned in {time.perf_counter() - t0:.1f} s: {best} "
            f"({tune_ms:.2f} ms per ingest)")
    g.profile(True)
    torch.cuda.synchronize()

    def step():
        g.reset()
        g.ingest(src_d, dst_d, flags=gz.GZ_ASYNC)
        prof = g.last_profile()
        st, labels, ncc = g.connected_components()
        return prof, st, ncc

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    profs, ncc, st = [], 0, 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        prof, st, ncc = step()
        profs.append(prof)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log(f"[bench] {args.steps} steps, {ms_per_step:.2f} ms/step, components={ncc}, status={st}")

    # CC query alone on the final sketches (wall time incl. labels D2H)
    qms = []
    for _ in range(5):
        q0 = time.perf_counter()
        g.connected_components()
        qms.append((time.perf_counter() - q0) * 1e3)
    cc_query_ms = statistics.median(qms)

    upd_ms = statistics.median(p["update_ms"] for p in profs)
    grp_ms = statistics.median(p["group_ms"] for p in profs)
    ing_ms = statistics.median(p["ingest_ms"] for p in profs)
    P = g.R * g.C
    ops = stream.N * P * OPS_PER_UPDATE_PAIR
    achieved = ops / (upd_ms * 1e-3) / 1e12
    traffic = traffic_from_profile(kernel_source_hash())

    out = {
        "metric": "edge updates/sec ingested (1 MI355X), batched vs plain; CC query ms; p99 latency",
        "value": stream.N / (ms_per_step * 1e-3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": desc, "V": stream.V, "updates": stream.N, "R": g.R, "C": g.C,
                   "B": g.B, "step": "reset + batched ingest + connected components"},
        "ingest_updates_per_s": stream.N / (ing_ms * 1e-3),
        "ingest_ms": ing_ms,
        "group_ms": grp_ms,
        "update_kernel_ms": upd_ms,
        "cc_query_ms": cc_query_ms,
        "components": ncc,
        "tuning": g.tuning,
        "autotuned": not args.no_autotune,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT_TOPS,
                     "unit": "TOP/s", "frac": achieved / PEAK_INT_TOPS,
                     "traffic": traffic,
                     "kernel": "k_update",
                     "ops_per_launch": ops,
                     "ops_rule": f"{OPS_PER_UPDATE_PAIR} int ops per (update, round-column pair), "
                                 f"{P} pairs per update"},
    }
    if not args.no_plain:
        rate, calls, gutter, pms = plain_pass(gz, g, stream, src_d, dst_d)
        out["plain_updates_per_s"] = rate
        out["plain_launches"] = calls
        out["plain_gutter_updates"] = gutter
        out["plain_ms"] = pms
        out["batched_vs_plain"] = out["ingest_updates_per_s"] / rate
        log(f"[bench] plain: {calls} launches, {pms:.1f} ms, {rate / 1e6:.1f} M updates/s")
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(stream, seed, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
