#!/usr/bin/env python3
"""Benchmark of the CubeSketch ingest + Boruvka connectivity hot path on one MI355X.

One step = zero the sketches, ingest the whole synthetic stream (device-side
grouping by endpoint + persistent LDS-staged sketch update) and answer a
connected-components query.  The stream is resident in HBM before timing.

Default workload: the skewed R-MAT graph on V = 2^15 nodes (initiator
a,b,c,d = 0.7,0.1,0.1,0.1, seed 3), 150M updates with deletes of live edges
interleaved at rate 0.2, sketch shape R=16, C=8, B=30 (2 GB of sketches as
uint64 pairs; 1.5 GB in the library's 32-bit-word layout).

Besides the JSON line's `value` (whole-step updates/s) the line carries the
plain per-node-launch rate (one gz_update_sketch_batch launch per gutter of
half a node sketch, the paper's leaf-gutter size, each launch spread over the
chip), the CC query time, the roofline of the dominant kernel (measured with
HIP events on its own stream) and the CPU oracle's rate on a bounded sample,
single-threaded and over all host cores.
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

TUNING_KEYS = ["wg_size", "lds_rows", "chunk", "wgs_per_cu", "group_blocks"]

# MI355X figures used by the roofline.  VALU issue from unit counts: 256 CUs x
# 4 SIMDs x 16 lanes x 2.4 GHz = 39.32 T lane-instructions/s at one instruction
# per lane per clock, the rate of the 32-bit multiplies and 64-bit multiply-adds
# the hashes are made of; simple 32-bit operations (add, xor, logic, moves)
# dual-issue up to twice that, 78.64 T (the vector rate behind the chip's
# 157.3 TFLOP/s fp32 figure; gz_measure_peaks measures both classes).  HBM3E 8 TB/s.
PEAK_INT_1X = 256 * 4 * 16 * 2.4e9 / 1e12
PEAK_INT_2X = 2 * PEAK_INT_1X
PEAK_HBM_GBS = 8000.0
# algorithmic integer ops per (update, round-column pair), as (all, multiply-class):
# the three hashes of the edge index counted once per update (each 2 multiplies
# and an add), the depth (bit scan and clamp, counted at the multiply rate), and
# one exact-depth XOR of (alpha, gamma) per endpoint (4 each)
OPS_PER_UPDATE_PAIR = (19, 8)
# the same for graphs with V > 2^16, whose three hashes are keyed by the node
# pair (a*u + a2*v + b: two 64x32-bit multiply-adds and two 32-bit high-word
# products with their adds, 6 each, 4 of them multiplies), depth 2, and XORs of
# four 32-bit planes per endpoint (4 each)
OPS_PER_UPDATE_PAIR_WIDE = (28, 14)


def alu_peak(ops) -> float:
    """Peak rate (T ops/s) of an op mix: its multiply-class ops at 1x, the rest at 2x."""
    total, slow = ops
    return total / (slow / PEAK_INT_1X + (total - slow) / PEAK_INT_2X)


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
                "drawn again toggles its edge (pair-keyed contract, R=19, B=36)")
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
                 "rmat_skewed": "k_update_rmat_skewed_pmc.txt",
                 "rmat_kron18": "k_update_wide_rmat_kron18_pmc.txt",
                 "many_gnp": "k_update_many_gnp_kernel_trace.txt"}


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


def host_cpu():
    """(CPU model name, logical CPUs this process may run on)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def _oracle_part(arg):
    """One worker of the all-cores leg: the oracle over the sample, keeping only its nodes."""
    path, V, seed, nodes = arg
    import numpy as np

    import oracle

    d = np.load(path, mmap_mode="r")
    src = np.ascontiguousarray(d[0])
    dst = np.ascontiguousarray(d[1])
    O = oracle.Oracle(V, seed)
    t0 = time.perf_counter()
    O.ingest_nodes(src, dst, nodes)
    return time.perf_counter() - t0


def cpu_baseline(stream, seed, seconds: float, workers: int):
    """The oracle as it stands (untuned), timed on a bounded sample of the same stream.

    Single thread: the first M1 updates, every node sketch.  All cores: the
    next M updates, split by node over `workers` processes (each the same
    single-threaded oracle keeping only its nodes, the nodes dealt out so that
    every process gets about the same number of endpoint entries); the rate is
    M over the slowest process's ingest time.  Runs before the GPU is touched
    (the workers are forked).
    """
    import multiprocessing
    import tempfile

    import numpy as np

    import oracle

    model, nproc = host_cpu()
    O = oracle.Oracle(stream.V, seed)
    probe = min(stream.N, 20000)
    t0 = time.perf_counter()
    O.ingest(stream.src[:probe], stream.dst[:probe])
    rate1 = probe / max(time.perf_counter() - t0, 1e-9)
    M1 = int(min(stream.N - probe, max(1000, rate1 * seconds / 2)))
    t0 = time.perf_counter()
    O.ingest(stream.src[probe:probe + M1], stream.dst[probe:probe + M1])
    t1 = time.perf_counter()
    del O
    single = {"value": M1 / (t1 - t0), "cores": 1,
              "sample": f"updates {probe}..{probe + M1} ({M1} updates, all {stream.V} node "
                        f"sketches, {t1 - t0:.1f} s)"}
    out = {"value": single["value"], "unit": "updates/s", "cores": 1, "kind": "oracle",
           "sample": single["sample"], "single_thread": single, "cpu_model": model,
           "nproc": nproc}
    workers = max(1, min(workers, nproc))
    if workers == 1:
        return out
    lo = probe + M1
    M = int(min(stream.N - lo, max(10000, single["value"] * workers * seconds / 2)))
    src = stream.src[lo:lo + M]
    dst = stream.dst[lo:lo + M]
    # deal nodes to workers, heaviest first, each to the least loaded one
    deg = np.bincount(src, minlength=stream.V) + np.bincount(dst, minlength=stream.V)
    load = np.zeros(workers, np.int64)
    parts = [[] for _ in range(workers)]
    for v in np.argsort(-deg, kind="stable").tolist():
        w = int(np.argmin(load))
        parts[w].append(v)
        load[w] += int(deg[v])
    tmpdir = "/dev/shm" if os.path.isdir("/dev/shm") else tempfile.gettempdir()
    fd, path = tempfile.mkstemp(suffix=".npy", dir=tmpdir)
    os.close(fd)
    try:
        np.save(path, np.stack([src, dst]))
        ctx = multiprocessing.get_context("fork")
        with ctx.Pool(workers) as pool:
            times = pool.map(_oracle_part, [(path, stream.V, seed, np.array(p, np.int64))
                                            for p in parts])
    finally:
        os.unlink(path)
    out.update({"value": M / max(times), "cores": workers,
                "sample": f"updates {lo}..{lo + M} ({M} updates) split by node over {workers} "
                          f"processes of the single-threaded oracle; slowest process "
                          f"{max(times):.1f} s, fastest {min(times):.1f} s; ingest only"})
    return out


def plain_pass(gz, g, stream, src_d, dst_d):
    """Plain path: one gz_update_sketch_batch launch per node gutter (half a node sketch at
    4 B per update, the paper's leaf-gutter size), on input grouped by node beforehand.

    Each launch spreads its gutter over workgroups of node_chunk entries whose
    partial tiles merge by XOR; node_chunk is picked by timing a few values on
    the first gutters (1 << 30 is one workgroup per gutter).
    """
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

    def run(batch):
        g.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for node, ptr, cnt in batch:
            st = L.gz_update_sketch_batch(h, node, ctypes.c_void_p(ptr), cnt, flags, s)
            if st:
                raise RuntimeError(f"plain batch failed: {st}")
        g.flush()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    keep = g.tuning
    sweep = {}
    probe = calls[: min(len(calls), 3000)]
    probe_n = sum(c for _, _, c in probe)
    for nc in (0, 64, 128, 256, 512, 1024, 2048, 1 << 30):
        g.set_tuning(node_chunk=nc)
        run(probe[:200])  # warm-up
        sweep[nc] = probe_n / run(probe)
    best = max(sweep, key=sweep.get)
    g.set_tuning(node_chunk=best)
    dt = run(calls)
    g.set_tuning(**keep)
    return {"plain_updates_per_s": stream.N / dt, "plain_launches": len(calls),
            "plain_gutter_updates": gutter, "plain_ms": dt * 1e3, "plain_node_chunk": best,
            "plain_node_chunk_sweep": {str(k): v for k, v in sweep.items()},
            "plain_one_workgroup_updates_per_s": sweep[1 << 30]}


def l0_comparison(gz, g, stream, seed, src_d, dst_d, sample: int) -> dict:
    """Update cost of CubeSketch against the standard l0-sampler (Fig. agm_code) on the device,
    on the same first `sample` updates of the stream: each ingested into zeroed sketches of the
    same shape, the update kernels timed with HIP events (the paper's Fig. l0speedup makes the
    same comparison for one sampler on a CPU thread)."""
    import numpy as np
    import torch

    M = min(stream.N, sample)
    op_d = torch.from_numpy(np.ascontiguousarray(stream.op[:M])).cuda()
    s_src, s_dst = src_d[:M], dst_d[:M]
    l0 = gz.L0Sketch(stream.V, seed)
    l0.ingest(s_src, s_dst, op=op_d)  # warm-up
    l0_ms, cs_ms = [], []
    for _ in range(3):
        l0.reset()
        l0.ingest(s_src, s_dst, op=op_d)
        l0_ms.append(l0.last_update_ms())
        g.reset()
        g.ingest(s_src, s_dst, flags=gz.GZ_ASYNC)
        cs_ms.append(g.last_profile()["update_ms"])
    l0.close()
    torch.cuda.synchronize()
    l0m, csm = statistics.median(l0_ms), statistics.median(cs_ms)
    return {"sample": f"first {M} updates of the stream, both endpoints, sketches of the same "
                      f"shape (R={g.R}, C={g.C}, B={g.B})",
            "l0_update_ms": l0m, "cubesketch_update_ms": csm,
            "l0_updates_per_s": M / (l0m * 1e-3), "cubesketch_updates_per_s": M / (csm * 1e-3),
            "cubesketch_vs_l0": l0m / csm,
            "context": "Fig. l0speedup (one CPU thread): 127x at n = 10^6, 172x at 10^8, 196x at 10^9"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat_skewed",
                    help="rmat_skewed (default), rmat_dense, rmat_kron18, uniform_small, "
                         "many_gnp, serving, rmat_dense_host")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-node pass")
    ap.add_argument("--no-l0", action="store_true",
                    help="skip the comparison with the standard l0-sampler")
    ap.add_argument("--l0-sample", type=int, default=16_000_000,
                    help="updates of the stream the l0-sampler comparison ingests")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="CPU oracle budget (split between the single-thread and all-cores legs)")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="processes of the all-cores CPU leg (capped by the CPUs available)")
    ap.add_argument("--autotune", action="store_true",
                    help="run the autotuner even where the tuning cache has the shape")
    ap.add_argument("--tuning-cache-out", default="",
                    help="also store the launch parameters used in this JSON cache file")
    ap.add_argument("--tuning", default="",
                    help="explicit launch parameters wg_size,lds_rows,chunk,wgs_per_cu,group_blocks "
                         "(skips the cache and the autotuner)")
    ap.add_argument("--sessions", type=int, default=256, help="serving: number of sessions")
    ap.add_argument("--batches", type=int, default=200, help="serving: batches per session")
    ap.add_argument("--loads", default="0.5,0.8,1.0",
                    help="serving: open-loop offered loads as fractions of the closed-loop rate "
                         "(empty: closed loop only)")
    ap.add_argument("--hbm-budget-gb", type=float, default=120.0, help="serving: admission budget")
    ap.add_argument("--tick-updates", type=int, default=16 << 20, help="serving: updates per tick")
    ap.add_argument("--gutter-per-node", type=int, default=-1,
                    help="serving: gutter updates per session node (-1: the library's default, "
                         "0: no gutters)")
    ap.add_argument("--serving-dump", default="",
                    help="serving: write each open-loop run's schedule, latencies and tick "
                         "records to <prefix>_<load%%>.npz")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="serving: processes generating the session streams (1: in-process)")
    ap.add_argument("--client-threads", type=int, default=16,
                    help="serving: native client threads of the replay driver")
    ap.add_argument("--staging-mb", type=int, default=128,
                    help="host tier: device bytes of the two slab buffers")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure the device's copy bandwidth and integer VALU issue rates "
                         "(gz_measure_peaks) and print them as one JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (a kernel of known traffic "
                         "that scales hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"this benchmark runs on one GPU only (asked for {args.gpus}); sharding the path "
              "over several GPUs is a documented design, not a built path", file=sys.stderr)
        return 2

    if args.peaks:
        gpu_init()
        import paper_2203_14927_amd as gz

        runs = [gz.measure_peaks() for _ in range(3)]
        out = {k: (max(r[k] for r in runs) if isinstance(runs[0][k], float) else runs[0][k])
               for k in runs[0]}
        out["runs"] = 3
        out["unit_count_peaks"] = {"hbm_gbs": PEAK_HBM_GBS, "valu_1x_tops": PEAK_INT_1X,
                                   "valu_2x_tops": PEAK_INT_2X}
        print(json.dumps(out), flush=True)
        return 0
    if args.workload == "many_gnp":
        out = run_many(args)
    elif args.workload == "serving":
        out = run_serving(args)
    elif args.workload == "rmat_dense_host":
        out = run_host_tier(args)
    else:
        out = run_single(args)
    print(json.dumps(out), flush=True)
    import paper_2203_14927_amd as gz

    gz.close_all()  # every handle released while the runtime is up
    return 0


def gpu_init():
    import torch

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)


def apply_tuning(args, g, src_d, dst_d, kind="single"):
    """Launch parameters: explicit (--tuning), else the autotuner's cached tuple for this
    device and shape, else a fresh autotuner run.  Returns the source it came from."""
    from paper_2203_14927_amd import autotune

    if args.tuning:
        g.set_tuning(**dict(zip(TUNING_KEYS, (int(x) for x in args.tuning.split(",")))))
        source = "explicit"
    else:
        t0 = time.perf_counter()
        _, path = autotune.tuned(g, src_d, dst_d, kind=kind, refresh=args.autotune)
        source = ("gz_autotune (this run, %.1f s)" % (time.perf_counter() - t0)
                  if path == "gz_autotune" else "autotuner cache " + os.path.relpath(path, ROOT))
    if args.tuning_cache_out:
        autotune.save_entry(g, g.tuning, 0.0, len(src_d), args.tuning_cache_out, kind)
    log(f"[bench] launch parameters {g.tuning} from {source}")
    return source


# PCIe 5.0 x16 host link of the MI355X: 64 GB/s per direction
PEAK_HOST_LINK_GBS = 64.0


def run_host_tier(args) -> dict:
    """Dense R-MAT with the sketches in pinned host memory (host-DRAM tier)."""
    stream, seed, desc = make_workload("rmat_dense")
    gpu_init()
    import torch

    import paper_2203_14927_amd as gz
    from paper_2203_14927_amd import autotune

    src_d = torch.from_numpy(stream.src.view("int32")).cuda()
    dst_d = torch.from_numpy(stream.dst.view("int32")).cuda()
    g = gz.Graph(stream.V, seed=seed, host_tier=True, staging_bytes=args.staging_mb << 20)
    if args.tuning:
        g.set_tuning(**dict(zip(TUNING_KEYS, (int(x) for x in args.tuning.split(",")))))
    else:  # the HBM-resident graph of the same shape's tuned tuple, if cached
        t, _ = autotune.lookup(g)
        if t:
            g.set_tuning(**t)
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

    import workloads

    t0 = time.perf_counter()
    streams = workloads.config_many_gnp()
    seeds = [workloads.many_graph_seed(4, k) for k in range(len(streams))]
    offs = np.zeros(len(streams) + 1, np.uint64)
    offs[1:] = np.cumsum([s.N for s in streams])
    N = int(offs[-1])
    gpu_init()
    import torch

    import paper_2203_14927_amd as gz
    from paper_2203_14927_amd import autotune

    src_d = torch.from_numpy(np.concatenate([s.src for s in streams]).view(np.int32)).cuda()
    dst_d = torch.from_numpy(np.concatenate([s.dst for s in streams]).view(np.int32)).cuda()
    log(f"[bench] many G(n,p): {len(streams)} graphs, {N} updates, "
        f"{sum(s.V for s in streams)} nodes (generated in {time.perf_counter() - t0:.1f} s)")
    if args.copy_calibration:
        copy_calibration()
    graphs = [gz.Graph(s.V, seed=sd) for s, sd in zip(streams, seeds)]
    # a fused launch takes the first graph's launch parameters: explicit, else the
    # tuple cached for this workload, else the launch-shape sweep's best (wg 256,
    # 12 LDS rows, chunk 16384, 8 workgroups per CU)
    kind = f"many{len(graphs)}"
    if args.tuning:
        tuned_from = "explicit"
    else:
        t, path = autotune.lookup(graphs[0], kind)
        if t:
            graphs[0].set_tuning(**t)
            tuned_from = "autotuner cache " + os.path.relpath(path, ROOT)
        else:
            args.tuning = "256,12,16384,8,0"
            tuned_from = "launch-shape sweep"
    if args.tuning:
        graphs[0].set_tuning(**dict(zip(TUNING_KEYS, (int(x) for x in args.tuning.split(",")))))
    if args.tuning_cache_out:
        autotune.save_entry(graphs[0], graphs[0].tuning, 0.0, N, args.tuning_cache_out, kind)
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
    plan.close()
    # the update kernel alone, timed with HIP events on its stream by the library:
    # eager fused calls with the launch sequence the plan captured
    graphs[0].profile(True)
    upd = []
    for _ in range(3):
        reset_all()
        gz.ingest_multi(graphs, offs, src_d, dst_d, flags=gz.GZ_ASYNC)
        upd.append(graphs[0].last_profile()["update_ms"])
    graphs[0].profile(False)
    upd_ms = statistics.median(upd)
    tune = graphs[0].tuning
    moved = update_bytes_many(graphs, streams, tune["lds_rows"], tune["chunk"])
    achieved = moved["bytes"] / (upd_ms * 1e-3) / 1e9
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
        "cc_query_ms": ms - ims, "update_kernel_ms": upd_ms,
        "tuning": tune, "tuning_source": tuned_from,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic_from_profile(kernel_source_hash(), "many_gnp"),
                     "kernel": "k_update", "bytes_per_launch": moved["bytes"],
                     "bytes_rule": "per work item: 4 B per entry read, the rows d < DL of its "
                                   "node tile read and written (3 planes x DL x R x C x 4 B "
                                   "each way, DL as the kernel picks it from the item's size), "
                                   "24 B per expected entry-pair deeper than DL (HBM atomics), "
                                   "24 B of item record"},
    }


def update_bytes_many(graphs, streams, lds_rows: int, chunk: int) -> dict:
    """Bytes the update kernel must move for one fused ingest of these streams.

    Work items are a node's entries cut into pieces of at most `chunk`; an
    item of `count` entries keeps rows d < DL in LDS, DL = min(bitlen(count) +
    3, lds_rows) (every row, up to lds_rows, when that reaches B or the item
    has at least 16 entries per extra row), and reads and writes those rows of
    its node; entries deeper than DL (probability 2^-DL per pair) are applied
    to HBM with atomics.
    """
    import numpy as np

    total = 0.0
    deep = 0.0
    items = 0
    for g, s in zip(graphs, streams):
        deg = np.bincount(s.src, minlength=g.V) + np.bincount(s.dst, minlength=g.V)
        deg = deg[deg > 0].astype(np.int64)
        P = g.R * g.C
        full, rem = deg // chunk, deg % chunk
        counts = np.concatenate([np.full(int(full.sum()), chunk, np.int64), rem[rem > 0]])
        need = np.floor(np.log2(counts)).astype(np.int64) + 1 + 3
        all_rows = (need >= g.B) | ((g.B <= lds_rows) & (counts >= 16 * (g.B - need)))
        DL = np.where(all_rows, min(g.B, lds_rows), np.minimum(need, lds_rows))
        total += float((4 * counts + 24 * DL * P + 24).sum())
        d = (counts * P * np.exp2(-DL.astype(np.float64)) * (DL < g.B)).sum()
        deep += float(d)
        items += len(counts)
    return {"bytes": total + 24.0 * deep, "items": items, "deep_entry_pairs": deep}


def _gen_session(arg):
    """(V, seed, n_updates) -> session stream arrays (runs in a worker process)."""
    import workloads

    V, seed, n = arg
    st, _ = workloads.rmat_session(V, workloads.RMAT_GRAPH500, n, 0.1, seed)
    return st.src, st.dst


def _session_bytes(V: int) -> int:
    """Device bytes the server charges a session against its budget: sketches plus query
    scratch (12 bytes per bucket, R x C x B buckets per node)."""
    n = V * (V - 1) // 2
    R, B = (V - 1).bit_length() + 1, (n - 1).bit_length() + 1
    return 12 * B * R * 8 * V + V * (3 * B * 8 * 4 + 96)


def _mean(a) -> float:
    import numpy as np

    return float(np.mean(a)) if len(a) else 0.0


def _pcts(ns):
    """p50/p99 in ms of a latency array in ns."""
    import numpy as np

    if len(ns) == 0:
        return None
    x = np.asarray(ns, np.float64) / 1e6
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99)), "n": len(x)}


def run_serving(args) -> dict:
    """Many graph sessions through the server, driven by the library's native replay
    clients: a closed-loop run (capacity), then open-loop runs at fractions of it."""
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np

    import workloads

    S = args.sessions
    Vs = workloads.serving_sessions(seed=5, S=S)
    plans = []
    for k, V in enumerate(Vs):
        sizes = workloads.pareto_batch_sizes(5, 100 + k, args.batches)
        plans.append((V, 5000 + k, sizes))
    t0 = time.perf_counter()
    jobs = [(V, sd, int(sz.sum())) for V, sd, sz in plans]
    if args.gen_workers > 1:
        with ProcessPoolExecutor(max_workers=min(args.gen_workers, os.cpu_count() or 4)) as ex:
            data = list(ex.map(_gen_session, jobs))
    else:
        data = [_gen_session(j) for j in jobs]
    src = np.concatenate([d[0] for d in data])
    dst = np.concatenate([d[1] for d in data])
    sizes = np.concatenate([sz for _, _, sz in plans]).astype(np.uint64)
    offs = np.zeros(len(sizes) + 1, np.uint64)
    offs[1:] = np.cumsum(sizes)
    total, n_batches = int(offs[-1]), len(sizes)
    first = np.zeros(S + 1, np.int64)
    first[1:] = np.cumsum([len(sz) for _, _, sz in plans])
    log(f"[bench] serving: {S} sessions, {n_batches} batches, {total} updates generated in "
        f"{time.perf_counter() - t0:.1f} s")
    gpu_init()  # after the generator processes have forked
    from paper_2203_14927_amd.server import Server

    budget = int(args.hbm_budget_gb * (1 << 30))
    queries_of = lambda q: q[q > 0]  # noqa: E731

    def once(opens=None, arrival=None):
        srv = Server(hbm_budget=budget, tick_updates=args.tick_updates,
                     gutter_per_node=None if args.gutter_per_node < 0 else args.gutter_per_node)
        sess = [(V, sd, int(first[k]), len(sz), 0 if opens is None else int(opens[k]))
                for k, (V, sd, sz) in enumerate(plans)]
        r = srv.replay(sess, offs, src, dst, arrival, query_every=50,
                       client_threads=args.client_threads)
        st = srv.stats()
        st["timeline"] = srv.timeline()
        srv.close()
        return r, st

    r, stats = once()
    wall = r["wall_ns"] / 1e9
    cap = total / wall
    tl = stats.pop("timeline")
    timeline = {
        "ticks": len(tl),
        "device_busy_frac": float(tl["device_ms"].sum() / 1e3 / wall),
        "device_ms_per_tick": _mean(tl["device_ms"]),
        "updates_per_tick": _mean(tl["updates"]),
        "ingesting_ticks": int((tl["ingested"] > 0).sum()),
        "ingested_per_ingesting_tick": _mean(tl["ingested"][tl["ingested"] > 0]),
        "batches_per_tick": _mean(tl["batches"]),
        "graphs_per_tick": _mean(tl["graphs"]),
        "host_build_launch_ms_per_tick": _mean((tl["launched_ns"] - tl["take_ns"]) / 1e6),
        "launch_to_seen_done_ms_per_tick": _mean((tl["done_ns"] - tl["launched_ns"]) / 1e6),
        "device_updates_per_s": float(tl["updates"].sum() / max(tl["device_ms"].sum() / 1e3,
                                                                1e-9)),
    }
    log(f"[bench] serving timeline (closed loop): {timeline}")
    closed = {"batch": _pcts(r["batch_latency_ns"]),
              "query": _pcts(queries_of(r["query_latency_ns"]))}
    log(f"[bench] serving closed loop: {wall:.2f} s, {cap / 1e6:.1f} M updates/s, batch "
        f"{closed['batch']}, query {closed['query']}, stats {stats}")
    # Open loop: sessions arrive over time and live for their batches, so that about
    # n_conc of them (60% of what the budget holds on average: session sizes span 64x,
    # so the budget still binds at times) are open at once; each open session's
    # batches arrive as a Poisson process whose rate makes the steady offered load
    # `load` times the closed-loop rate.
    mean_bytes = float(np.mean([_session_bytes(V) for V in Vs]))
    n_conc = max(1, min(S, int(0.6 * budget / mean_bytes)))
    mean_batch = total / n_batches
    open_runs = []
    for load in ([float(x) for x in args.loads.split(",")] if args.loads else []):
        rate = load * cap / (n_conc * mean_batch)  # batches/s per open session
        life = args.batches / rate
        rng = np.random.default_rng([5, int(load * 1000)])
        opens = np.cumsum(rng.exponential(life / n_conc, S)) * 1e9
        arrival = np.zeros(n_batches, np.float64)
        for k in range(S):
            gaps = rng.exponential(1e9 / rate, int(first[k + 1] - first[k]))
            arrival[first[k]:first[k + 1]] = opens[k] + np.cumsum(gaps)
        r, st = once(opens.astype(np.uint64), arrival.astype(np.uint64))
        tl = st.pop("timeline")
        if args.serving_dump:
            np.savez_compressed(f"{args.serving_dump}_{int(load * 100)}.npz", opens=opens,
                                arrival=arrival, first=first, lat=r["batch_latency_ns"],
                                svc=r["batch_service_ns"], qlat=r["query_latency_ns"],
                                ticks=tl)
        w = r["wall_ns"] / 1e9
        log(f"[bench]   server stats: {st}")
        run = {"load": load, "offered_updates_per_s": load * cap, "sessions_open": n_conc,
               "achieved_updates_per_s": total / w, "wall_s": w,
               "batch_latency_ms": _pcts(r["batch_latency_ns"]),
               "batch_latency_in_service_ms": _pcts(r["batch_service_ns"]),
               "query_latency_ms": _pcts(queries_of(r["query_latency_ns"])),
               "ticks": st["ticks"]}
        open_runs.append(run)
        log(f"[bench] serving open loop at {load:.0%}: {w:.2f} s, "
            f"{total / w / 1e6:.1f} M updates/s over the run, batch {run['batch_latency_ms']}, "
            f"in service {run['batch_latency_in_service_ms']}, query {run['query_latency_ms']}")
    return {
        "metric": "edge updates/sec ingested (1 MI355X), batched vs plain; CC query ms; p99 latency",
        "value": cap, "unit": "updates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"serving: {S} R-MAT sessions, V=round(2^U(10,16)), Pareto(1.5) "
                               f"batches in [1e3,1e6], {args.batches} batches each, a query every "
                               f"50 batches and after the last; closed loop (one request "
                               f"outstanding per session, {args.client_threads} native client "
                               f"threads), then open-loop Poisson arrivals at {args.loads} of the "
                               f"closed-loop rate with sessions arriving over time; seed 5",
                   "sessions": S, "batches": n_batches, "updates": total,
                   "hbm_budget_gb": args.hbm_budget_gb, "tick_updates": args.tick_updates,
                   "gutter_per_node": args.gutter_per_node},
        "batch_latency_ms": closed["batch"],
        "query_latency_ms": closed["query"],
        "open_loop": open_runs,
        "timeline": timeline,
        "server": stats,
    }


def run_single(args) -> dict:
    import numpy as np

    t0 = time.perf_counter()
    stream, seed, desc = make_workload(args.workload)
    log(f"[bench] workload {args.workload}: V={stream.V} N={stream.N} "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    cpu = None
    if not args.no_cpu:
        # before the GPU is initialised: the all-cores leg forks its workers
        log("[bench] timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(stream, seed, args.cpu_seconds, args.cpu_workers)
        log(f"[bench] CPU oracle: {cpu['single_thread']['value'] / 1e6:.3f} M updates/s on one "
            f"thread, {cpu['value'] / 1e6:.3f} M updates/s on {cpu['cores']} processes")

    gpu_init()
    import torch

    import paper_2203_14927_amd as gz

    src_d = torch.from_numpy(stream.src.view(np.int32)).cuda()
    dst_d = torch.from_numpy(stream.dst.view(np.int32)).cuda()
    if args.copy_calibration:
        copy_calibration()
    g = gz.Graph(stream.V, seed=seed)
    tuned_from = apply_tuning(args, g, src_d, dst_d)
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
    mix = OPS_PER_UPDATE_PAIR_WIDE if stream.V > 65536 else OPS_PER_UPDATE_PAIR
    ops = stream.N * P * mix[0]
    achieved = ops / (upd_ms * 1e-3) / 1e12
    peak = alu_peak(mix)
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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TOP/s", "frac": achieved / peak,
                     "traffic": traffic,
                     "kernel": "k_update_wide" if stream.V > 65536 else "k_update",
                     "ops_per_launch": ops,
                     "ops_rule": f"{mix[0]} int ops per (update, round-column pair), {P} pairs "
                                 f"per update",
                     "peak_rule": f"{mix[1]} of the {mix[0]} ops multiply-class at "
                                  f"{PEAK_INT_1X:.2f} T/s, the rest at {PEAK_INT_2X:.2f} T/s "
                                  f"(VALU issue rates from unit counts)",
                     "frac_single_issue": achieved / PEAK_INT_1X},
    }
    if not args.no_plain:
        plain = plain_pass(gz, g, stream, src_d, dst_d)
        out.update(plain)
        out["batched_vs_plain"] = out["ingest_updates_per_s"] / plain["plain_updates_per_s"]
        log(f"[bench] plain: {plain['plain_launches']} launches, {plain['plain_ms']:.1f} ms, "
            f"{plain['plain_updates_per_s'] / 1e6:.1f} M updates/s (node_chunk "
            f"{plain['plain_node_chunk']}; one workgroup per gutter: "
            f"{plain['plain_one_workgroup_updates_per_s'] / 1e6:.1f} M updates/s)")
    if not args.no_l0 and stream.V <= 65536:
        out["l0_comparison"] = l0_comparison(gz, g, stream, seed, src_d, dst_d, args.l0_sample)
        log(f"[bench] standard l0-sampler: {out['l0_comparison']['l0_update_ms']:.2f} ms against "
            f"{out['l0_comparison']['cubesketch_update_ms']:.2f} ms for CubeSketch on the same "
            f"sample ({out['l0_comparison']['cubesketch_vs_l0']:.1f}x)")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    g.close()
    return out


if __name__ == "__main__":
    sys.exit(main())
