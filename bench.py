"""Benchmark: bounded sub-problems per second on one MI355X.

Workload: one 20-job x 20-machine instance (integer times uniform in [1, 99]),
a pool of 2^22 nodes whose prefix depth is uniform in 1..19, resident in HBM
before timing starts.  One step = one launch of the pool-bounding path over
the whole pool (decode, prefix recurrence, heads and tails, every machine pair
in Johnson order, max), through the C ABI.

Prints one JSON line with the throughput, the roofline of the bounding kernel
(algorithmic integer operations per launch over its measured duration, against
the INT32 vector peak) and the CPU oracle timed on a sample of the same pool.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bounded subproblems/sec (n=20,m=20) + B&B time-to-optimum, learned vs plain"

# MI355X: 256 compute units x 4 SIMDs x 16 lanes, one 32-bit integer
# operation per lane per clock at 2.4 GHz.
CUS, SIMDS, LANES, CLOCK = 256, 4, 16, 2.4e9
INT32_PEAK_TOPS = CUS * SIMDS * LANES * CLOCK / 1e12  # 39.3


def algorithmic_ops(depths: np.ndarray, n: int, m: int) -> int:
    """Integer operations the bound must perform, summed over a pool:
    per node, 4 per (machine pair, unscheduled job) for the two-machine walk,
    2 per (machine, scheduled job) for the prefix recurrence, 2 per
    (machine, unscheduled job) for the head and tail minima, 2 per machine
    for the heads, 2 per pair to add the tail and take the max."""
    d = depths.astype(np.int64)
    u = n - d
    P = m * (m - 1) // 2
    return int((4 * P * u + 2 * m * d + 2 * m * u + 2 * m + 2 * P).sum())


def measured_traffic() -> float | None:
    """HBM bytes per launch of the bounding kernel from the committed counter
    runs (profiles/bound_kernel_20x20_2p22.*), or None once the kernel
    sources differ from the ones that were measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "bound_kernel_20x20_2p22.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return float(rec["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(p, pool, target_s: float = 10.0) -> dict:
    from oracle import oracle as O
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    probe = pool[:4096]
    t0 = time.perf_counter()
    O.bound_pool(p, probe, nthreads=cores)
    dt = time.perf_counter() - t0
    per_node = dt / len(probe)
    k = int(min(len(pool), max(8192, target_s / max(per_node, 1e-9))))
    sample = pool[:k]
    t0 = time.perf_counter()
    O.bound_pool(p, sample, nthreads=cores)
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "nodes/s", "cores": cores, "kind": "oracle",
            "sample": f"first {k} nodes of the benchmark pool, {cores} threads, "
                      f"{dt:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2-pool", type=int, default=22)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy 5 times (the reference "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the pool "
              "bounding path shards across GPUs only by design",
              file=sys.stderr)
        return 2

    import torch
    from paper_1206_4973_amd import fsp, inputs

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 1 << 28, "launches": 5}))
        return 0
    n, m, seed = 20, 20, 2000
    count = 1 << args.log2_pool
    p = inputs.instance(n, m, seed)
    pool = inputs.random_pool(n, count, 1, n - 1, seed + 500000)
    inst = fsp.Instance(p)
    nodes = torch.from_numpy(pool).cuda()
    out = torch.empty(count, dtype=torch.int32, device="cuda")
    ops = algorithmic_ops(pool[:, 0], n, m)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        inst.bound_pool(nodes, out, stream=stream)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        inst.bound_pool(nodes, out, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_s = ev0.elapsed_time(ev1) / 1e3 / args.steps  # one launch per step

    ms_per_step = wall / args.steps * 1e3
    value = count / (wall / args.steps)
    achieved = ops / kernel_s / 1e12
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "pool bounding: 20 jobs x 20 machines, times uniform [1,99] "
                        f"(seed {seed}), 2^{args.log2_pool} nodes, prefix depth uniform 1..19",
            "n": n, "m": m, "pool": count, "stride": int(pool.shape[1]),
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": INT32_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": achieved / INT32_PEAK_TOPS,
            "traffic": measured_traffic(),
            "kernel": "bound_kernel<20,narrow>",
            "kernel_ms": kernel_s * 1e3,
            "algorithmic_ops_per_launch": ops,
        },
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(p, pool)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
