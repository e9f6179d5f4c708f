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

# Launch parameters the autotuner picks for a workload on MI355X (wg_size,
# lds_rows, chunk, wgs_per_cu, group_blocks), so that a default run times the
# same configuration every time; --autotune searches again.
TUNED = {"rmat_dense": "1024,28,16384,2,0", "many_gnp": "256,12,16384,8,0",
         "rmat_kron18": "512,16,4096,3,256"}

# MI355X figures used by the roofline: 256 CUs x 4 SIMD16 x 2.4 GHz, HBM3E 8 TB/s
PEAK_INT_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # VALU lane-instructions/s: 39.32 T
PEAK_HBM_GBS = 8000.0
# algorithmic integer ops per (update, round-column pair): the three hashes of the
# edge index (row hash 3, 64-bit checksum 6, depth 2) counted once per update,
# plus one exact-depth XOR of (alpha, gamma) per endpoint (4 each)
OPS_PER_UPDATE_PAIR = 19
# the same for graphs with V > 2^16, whose three hashes are keyed by the node
# pair (a*u + a2*v + b: two 64x32-bit multiply-adds and two 32-bit high-word
# products with their adds, 6 each), depth 2, and XORs of four 32-bit planes
# per endpoint (4 each)
OPS_PER_UPDATE_PAIR_WIDE = 28


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def make_workload(name: str):
    import workloads

    if name == "rmat_dense":
        s = workloads.config_rmat_dense()
        desc = ("R-MAT V=2^14 (a,b,c,d=0.57,0.19,0.19,0.05, seed 2): ~50M distinct inserts then "
                "10% live deletes")
        return s, 2, desc
    if name == "rmat_kron18":
        s = workloads.rmat_draws(1 << 18, workloads.RMAT_GRAPH500, 1 << 28, 18)
        desc = ("R-MAT V=2^18 (a,b,c,d=0.57,0.19,0.19,0.05, seed 18): 2^28 raw draws, a pair "
                "drawn again toggles its edge (pair-keyed contract, R=19, B=33)")
        return s, 18, desc
    if name == "uniform_small":
        s = workloads.config_uniform_small()
        return s, 1, "uniform V=1024: 150k inserts then 50k deletes (seed 1)"
    if name == "rmat_skewed":
        s = workloads.config_rmat_skewed()
        desc = ("skewed R-MAT V=2^15 (0.7,0.1,0.1,0.1, seed 3): ~150M updates, 20% deletes "
                "interleaved")
        return s, 3, desc
    raise SystemExit(f"unknown workload {name}")


PMC_SUMMARIES = {"rmat_dense": "k_update_rmat_dense_pmc.txt",
                 "rmat_kron18": "k_update_wide_rmat_kron18_pmc.txt"}


def traffic_from_profile(kernel_src_hash: str, workload: str = "rmat_dense"):
    """HBM bytes per launch of the update kernel from the committed PMC summary, or None.

    The summary records the hash of the kernel source it was taken with; a
    different hash means the kernel changed since, and the figure is stale.
    """
    if workload not in PMC_SUMMARIES:
        return None
    path = os.path.join(ROOT, "profiles", PMC_SUMMARIES[workload])
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_src_hash:
        return None
    return float(t.group(1))


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2203_14927_amd", "csrc", "gz_update.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()


def copy_calibration():
    """One plain 1 GiB device copy, the reference for scaling HBM traffic counters."""
    import torch

    a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)  # reads 1 GiB, writes 1 GiB
    torch.cuda.synchronize()
    del a, b


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
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default launch parameters")
    ap.add_argument("--autotune", action="store_true",
                    help="run the autotuner even where the workload has recorded launch parameters")
    ap.add_argument("--tuning", default="",
                    help="explicit launch parameters wg_size,lds_rows,chunk,wgs_per_cu,group_blocks "
                         "(skips the autotuner)")
    ap.add_argument("--sessions", type=int, default=256, help="serving: number of sessions")
    ap.add_argument("--batches", type=int, default=100, help="serving: batches per session")
    ap.add_argument("--hbm-budget-gb", type=float, default=120.0, help="serving: admission budget")
    ap.add_argument("--tick-updates", type=int, default=16 << 20, help="serving: updates per tick")
    ap.add_argument("--client-threads", type=int, default=16,
                    help="serving: host threads driving the sessions' closed-loop clients")
    ap.add_argument("--staging-mb", type=int, default=128,
                    help="host tier: device bytes of the two slab buffers")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (a kernel of known traffic "
                         "that scales hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"this benchmark runs on one GPU only (asked for {args.gpus}); sharding the path "
              "over several GPUs is a documented design, not a built path", file=sys.stderr)
        return 2

    import torch

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    if args.workload == "many_gnp":
        out = run_many(args)
    elif args.workload == "serving":
        out = run_serving(args)
    elif args.workload == "rmat_dense_host":
        out = run_host_tier(args)
    else:
        out = run_single(args)
    print(json.dumps(out), flush=True)
    return 0


# PCIe 5.0 x16 host link of the MI355X: 64 GB/s per direction
PEAK_HOST_LINK_GBS = 64.0


def run_host_tier(args) -> dict:
    """Dense R-MAT with the sketches in pinned host memory (host-DRAM tier)."""
    import torch

    import paper_2203_14927_amd as gz

    stream, seed, desc = make_workload("rmat_dense")
    src_d = torch.from_numpy(stream.src.view("int32")).cuda()
    dst_d = torch.from_numpy(stream.dst.view("int32")).cuda()
    g = gz.Graph(stream.V, seed=seed, host_tier=True, staging_bytes=args.staging_mb << 20)
    keys = ["wg_size", "lds_rows", "chunk", "wgs_per_cu", "group_blocks"]
    g.set_tuning(**dict(zip(keys, (int(x) for x in (args.tuning or TUNED["rmat_dense"]).split(",")))))
    sketch_bytes = g.storage()[1]

    def step():
        t0 = time.perf_counter()
        g.ingest(src_d, dst_d)  # synchronous
        t1 = time.perf_counter()
        st, labels, ncc = g.connected_components()
        t2 = time.perf_counter()
        return (t1 - t0) * 1e3, (t2 - t1) * 1e3, ncc

    for _ in range(args.warmup):
        g.reset()
        step()
    ing, qry, tot = [], [], []
    ncc = 0
    for _ in range(args.steps):
        g.reset()  # a host memset of the sketches: set-up, outside the timed step
        torch.cuda.synchronize()
        a, b, ncc = step()
        ing.append(a)
        qry.append(b)
        tot.append(a + b)
    ms = statistics.mean(tot)
    ims = statistics.median(ing)
    # every node has entries in this stream: each ingest moves the whole sketch
    # array host -> device and back, concurrently in the two directions
    link = sketch_bytes / (ims * 1e-3) / 1e9
    log(f"[bench] host tier: {ms:.2f} ms/step (ingest {ims:.2f} ms, components "
        f"{statistics.median(qry):.2f} ms), components={ncc}")
    return {
        "metric": "edge updates/sec ingested (1 MI355X), batched vs plain; CC query ms; p99 latency",
        "value": stream.N / (ms * 1e-3), "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": desc + "; sketches in pinned host memory (host-DRAM tier), "
                   f"{args.staging_mb} MiB of device slab buffers",
                   "V": stream.V, "updates": stream.N, "sketch_bytes": sketch_bytes,
                   "step": "ingest + connected components (sketch reset outside the timed step)"},
        "ingest_updates_per_s": stream.N / (ims * 1e-3), "ingest_ms": ims,
        "cc_query_ms": statistics.median(qry), "components": ncc,
        "roofline": {"bound": "host_link", "achieved": link, "peak": PEAK_HOST_LINK_GBS,
                     "unit": "GB/s", "frac": link / PEAK_HOST_LINK_GBS, "traffic": None,
                     "kernel": "slab copies of the ingest",
                     "bytes_rule": "sketch bytes per direction per ingest (every node is touched)"},
    }


def run_many(args) -> dict:
    """4096 independent G(n,p) graphs: one captured-plan ingest, then one fused query."""
    import numpy as np
    import torch

    import paper_2203_14927_amd as gz
    import workloads

    t0 = time.perf_counter()
    streams = workloads.config_many_gnp()
    seeds = [workloads.many_graph_seed(4, k) for k in range(len(streams))]
    offs = np.zeros(len(streams) + 1, np.uint64)
    offs[1:] = np.cumsum([s.N for s in streams])
    N = int(offs[-1])
    src_d = torch.from_numpy(np.concatenate([s.src for s in streams]).view(np.int32)).cuda()
    dst_d = torch.from_numpy(np.concatenate([s.dst for s in streams]).view(np.int32)).cuda()
    log(f"[bench] many G(n,p): {len(streams)} graphs, {N} updates, "
        f"{sum(s.V for s in streams)} nodes (generated in {time.perf_counter() - t0:.1f} s)")
    if args.copy_calibration:
        copy_calibration()
    graphs = [gz.Graph(s.V, seed=sd) for s, sd in zip(streams, seeds)]
    if not args.tuning and not args.no_autotune:
        args.tuning = TUNED["many_gnp"]
    if args.tuning:  # a fused launch takes the first graph's launch parameters
        keys = ["wg_size", "lds_rows", "chunk", "wgs_per_cu", "group_blocks"]
        graphs[0].set_tuning(**dict(zip(keys, (int(x) for x in args.tuning.split(",")))))
    sketch_bytes = sum(g.storage()[1] for g in graphs)
    plan = gz.Plan(graphs, [s.N for s in streams])
    stream_t = torch.cuda.current_stream()
    # the labels land in a caller-owned pinned buffer, reused by every step
    label_buf = torch.empty(sum(s.V for s in streams), dtype=torch.int32, pin_memory=True)
    label_out = label_buf.numpy().view(np.uint32)

    def reset_all():
        for g in graphs:
            g.reset()
        torch.cuda.synchronize()

    def step():
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream_t)
        plan.ingest(offs, src_d, dst_d, flags=gz.GZ_ASYNC)
        e1.record(stream_t)
        labels, ncc, stt = gz.connected_components_multi(graphs, out=label_out)
        e2.record(stream_t)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), ncc, stt

    for _ in range(args.warmup):
        reset_all()
        step()
    ingest_ms, total_ms = [], []
    for _ in range(args.steps):
        reset_all()  # sketch zeroing is set-up, outside the timed hot path
        t0 = time.perf_counter()
        ims, ncc, stt = step()
        total_ms.append((time.perf_counter() - t0) * 1e3)
        ingest_ms.append(ims)
    ms = statistics.mean(total_ms)
    ims = statistics.median(ingest_ms)
    log(f"[bench] {args.steps} steps, {ms:.2f} ms/step (ingest {ims:.2f} ms), "
        f"components={int(ncc.sum())}, failures={int((stt != 0).sum())}")
    # HBM roof of the fused ingest: every touched node tile is read and written
    # once, plus the stream reads of grouping and update
    touched = 12.0 * sum(g.B * g.R * g.C * s.V for g, s in zip(graphs, streams))
    algo_bytes = 2.0 * touched + 40.0 * N
    achieved = algo_bytes / (ims * 1e-3) / 1e9
    plan.close()
    return {
        "metric": "edge updates/sec ingested (1 MI355X), batched vs plain; CC query ms; p99 latency",
        "value": N / (ms * 1e-3), "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "4096 G(n,p) graphs, V~U{64..2048}, p~U(0.001,0.05), 30% deletes "
                               "(seed 4): one captured-plan ingest + fused components query",
                   "graphs": len(streams), "updates": N, "sketch_bytes": sketch_bytes,
                   "step": "captured-plan ingest + connected components of every graph"},
        "ingest_updates_per_s": N / (ims * 1e-3), "ingest_ms": ims,
        "cc_query_ms": ms - ims,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "captured ingest sequence",
                     "bytes_rule": "2 x node sketch bytes (read + write) + 40 B per update"},
    }


def _gen_session(arg):
    """(V, seed, n_updates) -> session stream arrays (runs in a worker process)."""
    import workloads

    V, seed, n = arg
    st, _ = workloads.rmat_session(V, workloads.RMAT_GRAPH500, n, 0.1, seed)
    return st.src, st.dst


def run_serving(args) -> dict:
    """Many graph sessions through the server: closed-loop clients, p50/p99 latencies."""
    import threading
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np

    import workloads
    from paper_2203_14927_amd.server import Server

    S = args.sessions
    Vs = workloads.serving_sessions(seed=5, S=S)
    plans = []
    for k, V in enumerate(Vs):
        sizes = workloads.pareto_batch_sizes(5, 100 + k, args.batches)
        plans.append((V, 5000 + k, sizes))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        data = list(ex.map(_gen_session, [(V, sd, int(sz.sum())) for V, sd, sz in plans]))
    total = sum(int(sz.sum()) for _, _, sz in plans)
    log(f"[bench] serving: {S} sessions, {total} updates generated in "
        f"{time.perf_counter() - t0:.1f} s")
    srv = Server(hbm_budget=int(args.hbm_budget_gb * (1 << 30)), tick_updates=args.tick_updates)
    lat_upd, lat_q, errors = [], [], []
    lock = threading.Lock()

    def clients(t):
        """Closed-loop clients of the sessions k = t, t + T, ...: each session keeps
        exactly one request outstanding (its next batch after the previous one
        completed, a query after every 50th batch and the last); one thread waits
        on the group's requests in submission order."""
        import collections

        try:
            mine = list(range(t, S, args.client_threads))
            st = {}
            pending = collections.deque()

            def next_request(k):
                c = st[k]
                V, seed, sizes = plans[k]
                if c["query_due"]:
                    c["query_due"] = False
                    c["ticket"], c["kind"] = c["sess"].submit_query(), "q"
                elif c["b"] < len(sizes):
                    n = int(sizes[c["b"]])
                    src, dst = data[k]
                    c["ticket"] = c["sess"].submit_updates(src[c["at"]:c["at"] + n],
                                                           dst[c["at"]:c["at"] + n])
                    c["kind"] = "u"
                    c["at"] += n
                    c["b"] += 1
                    c["query_due"] = c["b"] % 50 == 0 or c["b"] == len(sizes)
                else:
                    c["sess"].close()
                    return
                pending.append(k)

            for k in mine:
                V, seed, _ = plans[k]
                st[k] = {"sess": srv.open(V, seed), "at": 0, "b": 0, "query_due": False}
                next_request(k)
            while pending:
                k = pending.popleft()
                r = st[k]["ticket"].wait()
                with lock:
                    (lat_q if st[k]["kind"] == "q" else lat_upd).append(r["latency_ms"])
                next_request(k)
        except Exception as e:
            errors.append(e)

    th = [threading.Thread(target=clients, args=(t,)) for t in range(min(S, args.client_threads))]
    t0 = time.perf_counter()
    for t in th:
        t.start()
    for t in th:
        t.join()
    wall = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    if errors:
        raise errors[0]
    pct = lambda a, q: float(np.percentile(np.array(a), q)) if a else None  # noqa: E731
    log(f"[bench] serving: {wall:.1f} s, {total / wall / 1e6:.1f} M updates/s, "
        f"batch p50/p99 {pct(lat_upd, 50):.2f}/{pct(lat_upd, 99):.2f} ms, "
        f"query p50/p99 {pct(lat_q, 50):.2f}/{pct(lat_q, 99):.2f} ms, stats {stats}")
    return {
        "metric": "edge updates/sec ingested (1 MI355X), batched vs plain; CC query ms; p99 latency",
        "value": total / wall, "unit": "updates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"serving: {S} R-MAT sessions, V=round(2^U(10,16)), Pareto(1.5) "
                               f"batches in [1e3,1e6], {args.batches} batches each, a query every "
                               f"50 batches, closed-loop clients (one request outstanding per session, "
                               f"{min(S, args.client_threads)} host threads; seed 5)",
                   "sessions": S, "updates": total, "hbm_budget_gb": args.hbm_budget_gb,
                   "tick_updates": args.tick_updates},
        "batch_latency_ms": {"p50": pct(lat_upd, 50), "p99": pct(lat_upd, 99),
                             "n": len(lat_upd)},
        "query_latency_ms": {"p50": pct(lat_q, 50), "p99": pct(lat_q, 99), "n": len(lat_q)},
        "server": stats,
    }


def run_single(args) -> dict:
    import numpy as np
    import torch

    import paper_2203_14927_amd as gz

    t0 = time.perf_counter()
    stream, seed, desc = make_workload(args.workload)
    log(f"[bench] workload {args.workload}: V={stream.V} N={stream.N} "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    src_d = torch.from_numpy(stream.src.view(np.int32)).cuda()
    dst_d = torch.from_numpy(stream.dst.view(np.int32)).cuda()
    if args.copy_calibration:
        copy_calibration()
    g = gz.Graph(stream.V, seed=seed)
    tune_ms = None
    if not args.tuning and not args.autotune and not args.no_autotune:
        args.tuning = TUNED.get(args.workload, "")
    tuned_from = "explicit" if args.tuning else ("autotuner" if not args.no_autotune else "default")
    if args.tuning:
        keys = ["wg_size", "lds_rows", "chunk", "wgs_per_cu", "group_blocks"]
        g.set_tuning(**dict(zip(keys, (int(x) for x in args.tuning.split(",")))))
        args.no_autotune = True
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

    # the same ingest from host (pageable numpy) arrays: includes the PCIe copy
    hms = []
    for _ in range(3):
        g.reset()
        torch.cuda.synchronize()
        h0 = time.perf_counter()
        g.ingest(stream.src, stream.dst)
        torch.cuda.synchronize()
        hms.append((time.perf_counter() - h0) * 1e3)
    host_ingest_ms = statistics.median(hms)

    upd_ms = statistics.median(p["update_ms"] for p in profs)
    grp_ms = statistics.median(p["group_ms"] for p in profs)
    ing_ms = statistics.median(p["ingest_ms"] for p in profs)
    P = g.R * g.C
    opp = OPS_PER_UPDATE_PAIR_WIDE if stream.V > 65536 else OPS_PER_UPDATE_PAIR
    ops = stream.N * P * opp
    achieved = ops / (upd_ms * 1e-3) / 1e12
    traffic = traffic_from_profile(kernel_source_hash(), args.workload)

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
        "host_input_ingest_updates_per_s": stream.N / (host_ingest_ms * 1e-3),
        "components": ncc,
        "tuning": g.tuning,
        "tuning_source": tuned_from,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT_TOPS,
                     "unit": "TOP/s", "frac": achieved / PEAK_INT_TOPS,
                     "traffic": traffic,
                     "kernel": "k_update_wide" if stream.V > 65536 else "k_update",
                     "ops_per_launch": ops,
                     "ops_rule": f"{opp} int ops per (update, round-column pair), "
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
    return out


if __name__ == "__main__":
    sys.exit(main())
