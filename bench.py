"""Benchmark: bounded sub-problems per second on one MI355X.

Workload: one 20-job x 20-machine instance (integer times uniform in [1, 99]),
a pool of 2^22 nodes whose prefix depth is uniform in 1..19, resident in HBM
before timing starts.  One step = one launch of the pool-bounding path over
the whole pool (decode, prefix recurrence, heads and tails, every machine pair
in Johnson order, max), through the C ABI.

Prints one JSON line with the throughput, the roofline of the bounding kernel
(algorithmic integer operations per launch over its measured duration, against
the vector peak of the arithmetic the kernel runs: packed 16-bit, two
operations per lane per clock, when the instance takes the two-nodes-per-lane
form), the same pool on the one-node-per-lane 32-bit form, a sweep of pool
sizes 2^16..2^22, the CPU oracle timed on a sample of the same pool (one core
and all host cores), and the branch-and-bound legs: time to a proven optimum
on 50 held-out 20x10 instances (plain adaptive vs batched vs batched +
learned) and a time-limited search of the 20x20 instance from NEH.

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

# MI355X: 256 compute units x 4 SIMDs x 16 lanes at 2.4 GHz.  A 32-bit
# integer instruction does one operation per lane per clock; a packed 16-bit
# instruction (v_pk_*) does two.
CUS, SIMDS, LANES, CLOCK = 256, 4, 16, 2.4e9
INT32_PEAK_TOPS = CUS * SIMDS * LANES * CLOCK / 1e12  # 39.3
PK16_PEAK_TOPS = 2 * INT32_PEAK_TOPS  # 78.6


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


def _oracle_rate(p, pool, threads: int, target_s: float):
    """(nodes/s, sample size, seconds) of the oracle on the first nodes of
    `pool`, sized from a short probe to take about target_s seconds."""
    from oracle import oracle as O
    probe = pool[:max(256, 512 * threads)]
    t0 = time.perf_counter()
    O.bound_pool(p, probe, nthreads=threads)
    per_node = (time.perf_counter() - t0) / len(probe)
    k = int(min(len(pool), max(len(probe), target_s / max(per_node, 1e-9))))
    t0 = time.perf_counter()
    O.bound_pool(p, pool[:k], nthreads=threads)
    dt = time.perf_counter() - t0
    return k / dt, k, dt


def cpu_baseline(p, pool, target_s: float = 10.0, one_core_s: float = 5.0) -> dict:
    """The oracle on all host cores (the reported baseline) and on one core
    (the paper's CPU baseline is a sequential search on one core)."""
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    rate, k, dt = _oracle_rate(p, pool, cores, target_s)
    rate1, k1, dt1 = _oracle_rate(p, pool, 1, one_core_s)
    return {"value": rate, "unit": "nodes/s", "cores": cores, "kind": "oracle",
            "sample": f"first {k} nodes of the benchmark pool, {cores} threads, "
                      f"{dt:.1f} s",
            "one_core": {"value": rate1, "unit": "nodes/s", "cores": 1,
                         "sample": f"first {k1} nodes of the benchmark pool, one thread, "
                                   f"{dt1:.1f} s"}}


# Held-out 20x10 instances: every seed of 4500..4549 (the policy network was
# trained on seeds 4000..4199).  The list is fixed before any run; a search
# that reaches the time limit is reported as censored at that limit.
HELD_OUT_SEEDS = list(range(4500, 4550))
BNB_TIME_LIMIT = 2.0


def progress(msg: str) -> None:
    """One line per finished step on stderr (the JSON result goes to stdout)."""
    print(msg, file=sys.stderr, flush=True)


def geomean(xs):
    xs = [max(float(x), 1e-9) for x in xs]
    return float(np.exp(np.mean(np.log(xs)))) if xs else None


def paired_summary(rows, base, kind, limit):
    """Paired comparison of `kind` against `base` over the seeds of `rows`.

    Time: a censored run counts at the time limit, so a ratio involving one
    is only a bound; the geomean over every seed and the one over the seeds
    both kinds proved are both given, with win/loss counts.  Nodes: geomean
    ratio over the seeds both proved (a censored run's count depends on the
    limit)."""
    both = [r for r in rows if r[base]["proven"] and r[kind]["proven"]]
    t = lambda r, k: r[k]["t_proof_s"] if r[k]["proven"] else limit
    return {
        "seeds": len(rows),
        "both_proven": len(both),
        "speedup_geomean_all_censored_at_limit": geomean([t(r, base) / t(r, kind) for r in rows]),
        "speedup_geomean_both_proven": geomean(
            [r[base]["t_proof_s"] / r[kind]["t_proof_s"] for r in both]),
        "node_ratio_geomean_both_proven": geomean(
            [r[kind]["nodes"] / r[base]["nodes"] for r in both]),
        "faster": sum(1 for r in rows if t(r, kind) < t(r, base)),
        "slower": sum(1 for r in rows if t(r, kind) > t(r, base)),
        "proven_only_by_" + kind: sum(1 for r in rows if r[kind]["proven"] and not r[base]["proven"]),
        "proven_only_by_" + base: sum(1 for r in rows if r[base]["proven"] and not r[kind]["proven"]),
    }


def bnb_leg(seeds, time_limit, only=None, prefilter=False, kinds=None,
            host_threads=0, bound_choice=0) -> dict:
    """Time to a proven optimum on held-out 20x10 instances: plain adaptive
    (the paper's Algorithm 1, launch by launch) vs batched (graph-replayed
    iterations, autotuned pool) vs batched + learned ordering and pool size.
    Every kind runs every seed of `seeds` with the same time limit; results
    are paired per seed.  `only` restricts the run to one kind (profiling)."""
    from paper_1206_4973_amd import fsp, inputs
    from paper_1206_4973_amd import train_policy
    model_path = os.path.join(ROOT, "paper_1206_4973_amd", "policy_20x10.npz")
    model = train_policy.load(model_path) if os.path.exists(model_path) else None
    if kinds is None:
        kinds = ["adaptive", "autotuned"] + (["learned"] if model is not None else [])
    if only:
        kinds = [only]
    rows = []
    t_leg = time.perf_counter()
    for s in seeds:
        inst = fsp.Instance(inputs.instance(20, 10, s))
        fsp.autotune_pool(inst)  # per-shape tuning, cached; not part of a run
        if bound_choice:
            depths = fsp.autotune_bounds(inst)  # likewise
        row = {"seed": s}
        for kind in kinds:
            kw = {"model": model} if kind == "learned" else {}
            r = fsp.branch_and_bound(inst, kind, time_limit=time_limit,
                                     prefilter=prefilter, host_threads=host_threads,
                                     bound_choice=bound_choice, **kw)
            progress(f"bnb seed {s} {kind}: {r.makespan} "
                     f"{'proven' if r.status == 0 else 'censored'} in {r.t_total_s:.3f} s")
            row[kind] = {"makespan": r.makespan, "proven": r.status == 0,
                         "t_proof_s": r.t_total_s, "t_found_s": r.t_found_s,
                         "t_search_s": r.t_search_s, "nodes": r.nodes_bounded,
                         "pools": r.pools, "pool": r.final_pool,
                         "proof_pools": r.proof_pools, "host_nodes": r.host_nodes}
        inst.close()
        rows.append(row)
    out = {"instances": f"20x10, seeds {seeds[0]}..{seeds[-1]} ({len(seeds)} held out)",
           "lb1_depths": depths if bound_choice else [],
           "time_limit_s": time_limit, "kinds": kinds, "one_machine_prefilter": prefilter,
           "host_threads": host_threads, "bound_choice": bound_choice,
           "leg_wall_s": time.perf_counter() - t_leg}
    # an exact search proves the same optimum whatever its kind: compare the
    # makespans of the kinds that proved it
    out["same_optimum"] = all(
        len({r[k]["makespan"] for k in kinds if r[k]["proven"]}) <= 1 for r in rows)
    for k in kinds:
        proven = [r for r in rows if r[k]["proven"]]
        out[k] = {"proven": len(proven),
                  "geomean_t_s_censored_at_limit": geomean(
                      [r[k]["t_proof_s"] if r[k]["proven"] else time_limit for r in rows]),
                  "geomean_nodes_proven": geomean([r[k]["nodes"] for r in proven])}
    if "adaptive" in kinds:
        for k in kinds:
            if k != "adaptive":
                out[f"{k}_vs_adaptive"] = paired_summary(rows, "adaptive", k, time_limit)
    out["per_instance"] = rows
    return out


def timed(fn, steps, warmup, stream):
    """Average seconds per call of fn over `steps` calls (HIP events on the
    launch stream), after `warmup` calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def pool_sweep(inst, nodes, out, depths, n, m, stream, peak, lo=16, hi=22) -> list:
    """The first 2^k nodes of the benchmark pool, k = lo..hi (the synthetic
    analogue of the paper's sweep of pool sizes): kernel time per launch
    (HIP events on the launch stream), nodes/s and the roofline fraction."""
    rows = []
    for k in range(lo, hi + 1):
        c = 1 << k
        if c > nodes.shape[0]:
            break
        sub, o = nodes[:c], out[:c]
        steps = max(5, min(200, (1 << 25) // c))
        t = timed(lambda: inst.bound_pool(sub, o, stream=stream), steps, 2, stream)
        ops = algorithmic_ops(depths[:c], n, m)
        rows.append({"log2_pool": k, "nodes": c, "steps": steps, "kernel_ms": t * 1e3,
                     "nodes_per_s": c / t, "achieved_TOPs": ops / t / 1e12,
                     "frac": ops / t / 1e12 / peak})
        progress(f"sweep 2^{k}: {t * 1e3:.3f} ms, {c / t / 1e9:.2f} G nodes/s")
    return rows


def timed_searches(inst, kinds, time_limit, model=None, prefilter=False, log_dir=None,
                   tag="") -> dict:
    """Searches of one instance from the NEH schedule with a time limit, one
    per kind; each reports the best UB, the smallest pending bound (a lower
    bound on the optimum), the gap and nodes per second."""
    from paper_1206_4973_amd import fsp
    rec = {}
    for kind in kinds:
        kw = {"model": model} if kind == "learned" else {}
        if kind == "learned" and model is None:
            continue
        if log_dir:
            os.makedirs(log_dir, exist_ok=True)
            kw["log_path"] = os.path.join(log_dir, f"{tag}_{kind}.jsonl")
        r = fsp.branch_and_bound(inst, kind, time_limit=time_limit, prefilter=prefilter, **kw)
        progress(f"{tag} {kind}: UB {r.makespan}, open bound {r.open_lb}, "
                 f"{r.nodes_bounded} nodes in {r.t_total_s:.1f} s")
        rec[kind] = {"best_ub": r.makespan, "open_lb": r.open_lb,
                     "gap": (r.makespan - r.open_lb) / r.makespan,
                     "proven": r.status == 0, "t_total_s": r.t_total_s,
                     "nodes": r.nodes_bounded,
                     "nodes_per_s": r.nodes_bounded / max(r.t_search_s, 1e-9),
                     "t_found_s": r.t_found_s, "pool": r.final_pool,
                     "proof_pools": r.proof_pools}
    return rec


def bnb20_leg(time_limit, kinds=None) -> dict:
    """The 20x20 benchmark instance (seed 2000): full searches from the NEH
    upper bound with the paper's adaptive pool size (Algorithm 1), the
    batched search with the autotuned pool, and the batched + learned search
    (20-machine network), each with a time limit; a search that proves the
    optimum reports it, one that does not reports its gap."""
    from paper_1206_4973_amd import fsp, inputs, train_policy
    model_path = os.path.join(ROOT, "paper_1206_4973_amd", "policy_m20.npz")
    model = train_policy.load(model_path) if os.path.exists(model_path) else None
    inst = fsp.Instance(inputs.instance(20, 20, 2000))
    neh_ub, _ = fsp.neh(inst)
    fsp.autotune_pool(inst)  # per-shape tuning, cached; not part of a run
    out = {"instance": "20x20, seed 2000", "neh_ub": neh_ub, "time_limit_s": time_limit}
    out.update(timed_searches(inst, kinds or ["adaptive", "autotuned", "learned"],
                              time_limit, model, tag="bnb 20x20"))
    inst.close()
    return out


def batch_workload(steps, warmup) -> dict:
    """64 instances (n in {20,50,100} x m in {5,10,20}, times uniform [1,99],
    seeds 3000+i), each with a pool of 2^e nodes, e uniform in 10..18 (depth
    uniform 1..n-1): one persistent graph-replayed launch vs 64 launches."""
    import torch
    from paper_1206_4973_amd import fsp, inputs
    shapes = [(n, m) for n in (20, 50, 100) for m in (5, 10, 20)]
    rng = np.random.default_rng(3000)
    exps = [int(e) for e in rng.integers(10, 19, size=64)]
    items, ops, nodes, seg_ops = [], 0, 0, []
    for i in range(64):
        n, m = shapes[i % 9]
        pool = inputs.random_pool(n, 1 << exps[i], 1, n - 1, 3000 + 500000 + i)
        items.append((fsp.Instance(inputs.instance(n, m, 3000 + i)),
                      torch.from_numpy(pool).cuda(), None))
        seg_ops.append(algorithmic_ops(pool[:, 0], n, m))
        ops += seg_ops[-1]
        nodes += len(pool)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    b = fsp.Batch(items, autotune=True)
    t_plan = time.perf_counter() - t0
    t_batch = timed(lambda: b.replay(stream), steps, warmup, stream)
    progress(f"batch, autotuned: {t_batch * 1e3:.3f} ms (planned in {t_plan:.2f} s)")
    b_def = fsp.Batch([(i, nd, None) for i, nd, _ in items])
    t_def = timed(lambda: b_def.replay(stream), steps, warmup, stream)
    b_one = fsp.Batch([(i, nd, None) for i, nd, _ in items], packed=False)
    t_one = timed(lambda: b_one.replay(stream), steps, warmup, stream)
    outs = [torch.empty(x[1].shape[0], dtype=torch.int32, device="cuda") for x in items]

    def separate():
        for (inst, nd, _), o in zip(items, outs):
            inst.bound_pool(nd, o, stream=stream)
    t_sep = timed(separate, steps, warmup, stream)
    torch.cuda.synchronize()
    same = all(torch.equal(a, c) and torch.equal(a, d) and torch.equal(a, e)
               for a, c, d, e in zip(b.outs, outs, b_def.outs, b_one.outs))
    paths, bpc = b.paths()
    # the packed segments count their work against the packed peak, the
    # others against the 32-bit peak: the launch's peak is the work-weighted
    # mean of the two
    ops_pk = sum(o for o, pth in zip(seg_ops, paths) if pth == "packed")
    peak = ops / (ops_pk / PK16_PEAK_TOPS + (ops - ops_pk) / INT32_PEAK_TOPS)
    achieved = ops / t_batch / 1e12
    form_count = {k: paths.count(k) for k in sorted(set(p for p in paths if p))}
    return {"workload": "batch: 64 instances, n in {20,50,100} x m in {5,10,20}, "
                        "pools 2^10..2^18 (seed 3000)",
            "nodes": nodes, "steps": steps, "warmup": warmup, "batch_info": b.info(),
            "autotuned": {"forms": form_count, "blocks_per_cu": bpc, "plan_s": t_plan},
            "one_launch": {"ms": t_batch * 1e3, "nodes_per_s": nodes / t_batch,
                           "achieved_TOPs": achieved, "peak_TOPs": peak,
                           "frac": achieved / peak},
            "one_launch_default_plan": {"ms": t_def * 1e3, "nodes_per_s": nodes / t_def},
            "one_launch_one_node_per_lane": {"ms": t_one * 1e3, "nodes_per_s": nodes / t_one,
                                             "frac_int32": ops / t_one / 1e12 / INT32_PEAK_TOPS},
            "separate_launches": {"ms": t_sep * 1e3, "nodes_per_s": nodes / t_sep},
            "identical_bounds": bool(same)}


def large_workload(steps, warmup, bnb_time, prefilter=False, shapes=None, kinds=None,
                   log_dir=None) -> dict:
    """50x20 (seed 5000) and 200x20 (seed 5001): pools of 2^22 nodes (depth
    uniform 1..n-1), then time-limited searches (plain adaptive, batched,
    batched + learned when a 20-machine policy is present) reporting the best
    UB, the smallest pending bound, the gap and nodes per second.  `shapes`
    and `kinds` select a subset; with `log_dir`, every search writes its
    per-batch log there (progress of long runs)."""
    import torch
    from paper_1206_4973_amd import fsp, inputs, train_policy
    out = {"workload": "large: 50x20 and 200x20", "bnb_time_limit_s": bnb_time,
           "one_machine_prefilter": prefilter}
    model_path = os.path.join(ROOT, "paper_1206_4973_amd", "policy_m20.npz")
    model = train_policy.load(model_path) if os.path.exists(model_path) else None
    stream = torch.cuda.current_stream()
    for n, m, seed in ((50, 20, 5000), (200, 20, 5001)):
        if shapes and f"{n}x{m}" not in shapes:
            continue
        p = inputs.instance(n, m, seed)
        inst = fsp.Instance(p)
        pool = inputs.random_pool(n, 1 << 22, 1, n - 1, seed + 500000)
        nodes = torch.from_numpy(pool).cuda()
        lb = torch.empty(len(pool), dtype=torch.int32, device="cuda")
        t = timed(lambda: inst.bound_pool(nodes, lb, stream=stream), steps, warmup, stream)
        progress(f"large {n}x{m}: pool of {len(pool)} nodes bounded in {t * 1e3:.3f} ms")
        ops = algorithmic_ops(pool[:, 0], n, m)
        rec = {"pool_bounding": {"nodes": len(pool), "ms": t * 1e3,
                                 "nodes_per_s": len(pool) / t,
                                 "frac": ops / t / 1e12 / INT32_PEAK_TOPS}}
        del nodes, lb
        run = [k for k in ("adaptive", "autotuned", "learned") if not kinds or k in kinds]
        rec.update(timed_searches(inst, run, bnb_time, model, prefilter, log_dir,
                                  tag=f"{n}x{m}"))
        out[f"{n}x{m}"] = rec
        inst.close()
    return out


BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 matrix cores


def policy_workload(steps, warmup) -> dict:
    """The policy network on 2^20 rows of 22 features (the 20x10 model):
    forward, and backward with weight gradients (forward recomputed), on the
    matrix cores.  Algorithmic FLOPs use the real layer sizes 22-128-128-2;
    the kernels run them padded to 32 inputs and 16 outputs."""
    import torch
    from paper_1206_4973_amd import train_policy
    model = train_policy.load(os.path.join(ROOT, "paper_1206_4973_amd", "policy_20x10.npz"))
    rows = 1 << 20
    g = torch.Generator(device="cpu").manual_seed(6000)
    x = torch.zeros((rows, 32), dtype=torch.float32)
    x[:, :22] = torch.rand((rows, 22), generator=g)
    x = x.to(torch.bfloat16).cuda()
    dy = torch.randn((rows, 2), generator=g).cuda()
    stream = torch.cuda.current_stream()
    t_fwd = timed(lambda: model.forward(x, stream=stream), steps, warmup, stream)
    t_bwd = timed(lambda: model.backward(x, dy, stream=stream), steps, warmup, stream)
    fwd = 2 * (22 * 128 + 128 * 128 + 128 * 2)
    bwd = fwd + 2 * (2 * 128 * 2) + 2 * (2 * 128 * 128) + 2 * 22 * 128
    out = {"workload": "policy network 22-128-128-2, 2^20 rows (seed 6000)", "rows": rows}
    for name, t, f in (("forward", t_fwd, fwd), ("backward", t_bwd, bwd)):
        tf = rows * f / t / 1e12
        out[name] = {"ms": t * 1e3, "rows_per_s": rows / t, "flop_per_row": f,
                     "achieved_TFLOPs": tf, "peak_TFLOPs": BF16_PEAK_TFLOPS,
                     "frac": tf / BF16_PEAK_TFLOPS}
        progress(f"policy {name}: {t * 1e3:.3f} ms, {tf:.1f} TFLOP/s")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2-pool", type=int, default=22)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-bnb", action="store_true", help="skip the B&B time-to-optimum leg")
    ap.add_argument("--pool-only", action="store_true",
                    help="only the timed launches of the benchmark pool (no 32-bit form, no "
                         "sweep, no oracle, no B&B): the run that profiles use")
    ap.add_argument("--bnb-kind", default=None, choices=["adaptive", "autotuned", "learned"],
                    help="with --workload bnb: run only this kind")
    ap.add_argument("--prefilter", action="store_true",
                    help="with --workload bnb or large: one-machine pre-filter in every search")
    ap.add_argument("--workload", default="pool",
                    choices=["pool", "batch", "large", "policy", "bnb"],
                    help="pool: the 20x20 line (default); batch: 64 mixed instances in one "
                         "launch; large: 50x20 and 200x20 pools and time-limited searches; "
                         "policy: the policy network's forward and backward kernels; "
                         "bnb: only the B&B time-to-optimum leg")
    ap.add_argument("--bnb-limit", type=float, default=BNB_TIME_LIMIT,
                    help="time limit of each held-out 20x10 search (s)")
    ap.add_argument("--bnb20-limit", type=float, default=8.0,
                    help="time limit of each search of the 20x20 instance (s)")
    ap.add_argument("--bnb-seeds", type=int, default=0,
                    help="with --workload bnb: only the first K held-out seeds")
    ap.add_argument("--bound-choice", type=int, default=0, choices=[0, 1],
                    help="with --workload bnb: 1 = the one-machine bound at the depths the "
                         "autotuner picks per shape (the two-machine bound elsewhere)")
    ap.add_argument("--host-threads", type=int, default=0,
                    help="with --workload bnb: hybrid search, this many CPU threads "
                         "exploring subtrees beside the device")
    ap.add_argument("--bnb-time", type=float, default=60.0,
                    help="time limit of each search of the large workload (s)")
    ap.add_argument("--large-shapes", default=None,
                    help="with --workload large: comma-separated subset of 50x20,200x20")
    ap.add_argument("--large-kinds", default=None,
                    help="with --workload large: comma-separated subset of "
                         "adaptive,autotuned,learned")
    ap.add_argument("--bnb-log-dir", default=None,
                    help="with --workload large: directory for the per-batch search logs")
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
    if args.workload == "batch":
        print(json.dumps(batch_workload(args.steps, args.warmup)), flush=True)
        return 0
    if args.workload == "large":
        split = lambda v: v.split(",") if v else None
        print(json.dumps(large_workload(args.steps, args.warmup, args.bnb_time, args.prefilter,
                                        split(args.large_shapes), split(args.large_kinds),
                                        args.bnb_log_dir)),
              flush=True)
        return 0
    if args.workload == "policy":
        print(json.dumps(policy_workload(args.steps, args.warmup)), flush=True)
        return 0
    if args.workload == "bnb":
        seeds = HELD_OUT_SEEDS[:args.bnb_seeds] if args.bnb_seeds else HELD_OUT_SEEDS
        print(json.dumps(bnb_leg(seeds, args.bnb_limit, args.bnb_kind, args.prefilter,
                                 host_threads=args.host_threads,
                                 bound_choice=args.bound_choice)),
              flush=True)
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
    packed = inst.bound_path == "packed"
    peak = PK16_PEAK_TOPS if packed else INT32_PEAK_TOPS

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
    progress(f"pool 20x20 2^{args.log2_pool}: {kernel_s * 1e3:.3f} ms per launch "
             f"({inst.bound_path} form)")
    if args.pool_only:
        args.no_cpu = args.no_bnb = True

    t32, sweep = None, None
    if not args.pool_only:
        # the same pool on the one-node-per-lane 32-bit form
        inst32 = fsp.Instance(p, packed=False)
        t32 = timed(lambda: inst32.bound_pool(nodes, out, stream=stream), args.steps,
                    args.warmup, stream)
        inst32.close()
        progress(f"pool 20x20 2^{args.log2_pool} on the 32-bit form: {t32 * 1e3:.3f} ms")
        sweep = pool_sweep(inst, nodes, out, pool[:, 0], n, m, stream, peak,
                           hi=args.log2_pool)
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
        "dtype": "int16x2" if packed else "int32",
        "data": "synthetic",
        "config": {
            "workload": "pool bounding: 20 jobs x 20 machines, times uniform [1,99] "
                        f"(seed {seed}), 2^{args.log2_pool} nodes, prefix depth uniform 1..19",
            "n": n, "m": m, "pool": count, "stride": int(pool.shape[1]),
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TOP/s",
            "frac": achieved / peak,
            "peak_basis": ("packed 16-bit vector ops: 256 CUs x 64 lanes x 2 per clock x "
                           "2.4 GHz" if packed else
                           "32-bit vector integer ops: 256 CUs x 64 lanes x 2.4 GHz"),
            "traffic": measured_traffic(),
            "kernel": {"packed": f"bound_kernel_p16<{m}, false> (two nodes per lane, 16-bit)",
                       "register": f"bound_kernel<{m}> (one node per lane)",
                       "masks": f"bound_kernel<{m}> (job masks)",
                       "bytes": f"bound_kernel<{m}> (flag bytes in LDS)"}[inst.bound_path],
            "kernel_ms": kernel_s * 1e3,
            "algorithmic_ops_per_launch": ops,
        },
    }
    if t32 is not None:
        res["int32_register_form"] = {
            "kernel": f"bound_kernel<{m}> (one node per lane, 32-bit)",
            "kernel_ms": t32 * 1e3, "nodes_per_s": count / t32,
            "achieved_TOPs": ops / t32 / 1e12, "peak_TOPs": INT32_PEAK_TOPS,
            "frac": ops / t32 / 1e12 / INT32_PEAK_TOPS,
        }
        res["pool_sweep"] = sweep
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(p, pool)
        progress("cpu baseline done")
    if not args.no_bnb:
        res["bnb_time_to_optimum"] = bnb_leg(HELD_OUT_SEEDS, args.bnb_limit)
        res["bnb_20x20"] = bnb20_leg(args.bnb20_limit)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
