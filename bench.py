#!/usr/bin/env python3
"""Throughput of the global Curveball super-step on one MI355X.

One step = one global trade (matching, dependency scan, trade kernel,
per-row rebuild) of the whole graph, inputs resident in HBM; the schedule
options come from the library's autotuner, run before the timed rounds. Default
workload: n = 2^24 nodes, degrees i.i.d. Pld([20, 2^20), gamma = 2.2), erased
configuration model (graph seed 1), chain seed 1: W warm-up rounds, then K
timed rounds, repeated R times from a fresh upload; value = m * K / (wall
seconds of the K steps), the median over the repetitions.

--workload batch runs the batched form: 512 independent chains (2^10..2^16
nodes each) advancing together, one step = one round of every chain,
launched as a captured graph, options from the autotuner; value = the sum
of the chains' edges * K / wall seconds. The same chains run one by one on
the single-chain path give the comparison figure.

Prints one JSON line. --gpus above 1 is refused: the library runs on one
GPU (independent chains would shard one per GPU with no exchange).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # bytes/s, MI355X HBM3E
WORKLOAD_TEXT = {
    "large": "n=2^24, degrees Pld([20,2^20),2.2), erased configuration model, graph seed 1",
    "mid": "n=2^20, degrees Pld([10,2^16),2.0), erased configuration model, graph seed 1",
    "small": "n=8192, degrees Pld([5,500),2.0), erased configuration model, graph seed 1",
    "hubs": "n=2^24, degrees Pld([1,2^16),2.5), erased configuration model, graph seed 3",
    "batch": ("512 chains: chain c has n_c=round(2^U[10,16]) nodes, degrees Pld([2,n_c/8),gamma_c), "
              "gamma_c~U[1.8,2.6], graph seed 1000+c, chain seed c"),
    "serve": ("Poisson requests: m=2^U[12,24] edges, degrees Pld([5,sqrt n),2), graph seed 10^6+q, "
              "k~U{1..32} samples, r~U{5..20} rounds, rate 0.7x the measured capacity"),
    "quality": ("mixing study: thinning on n=2000 Pld([5,b),2), b in {25,750}, global trades vs n/2 "
                "single trades per super-step; swap fractions on 10-regular and Pld([10,n/20),2) graphs"),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_{workload}.json")
KERNEL_SOURCES = ["cb_trade.hip", "cb_prep.hip", "cb_block.hpp", "cb_device.hpp", "cb_kernels.hpp"]


def kernel_source_digest() -> str:
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1804_08487_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_bytes(rec, name: str):
    """Scaled HBM bytes of one kernel in a traffic record, whose kernel names
    carry their namespace (cbx::k_trade), or None."""
    for key, value in rec["kernels"].items():
        if key == name or key.endswith("::" + name):
            return value
    return None


def measured_traffic(workload: str):
    """HBM bytes per step (per kernel) from the committed rocprofv3 counter
    runs, or None when the kernel sources changed since they were taken."""
    try:
        with open(TRAFFIC_FILE.format(workload=workload)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha1") != kernel_source_digest():
        return None
    return rec


def host_cpu():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, avail


def cpu_baseline(row_ptr, col, seed: int, trades: int):
    """The oracle (IM-CB form, single-threaded as the chain is sequential) on
    round 0 of the same graph: its per-round setup (matching, dependency
    counts, edge placement) plus the first `trades` trades, each phase timed
    inside the oracle. The round estimate is setup + (trade time / trades) *
    floor(n/2) (trades of a uniform matching are exchangeable); the oracle's
    final per-row rebuild is left out, which only favours the CPU figure."""
    import oracle
    o = oracle.default()
    _, st = o.global_trade(row_ptr, col, seed, 0, "o2", max_trades=trades)
    L = (len(row_ptr) - 1) // 2
    setup, tt = st["setup_seconds"], st["trade_seconds"]
    done = max(min(trades, L), 1)
    per_trade = tt / done
    round_s = setup + per_trade * L
    m = len(col) // 2
    model, ncpu, avail = host_cpu()
    return {
        "value": m / round_s,
        "unit": "edge-trades/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"IM-CB-form oracle, round 0 of this workload: setup {setup:.1f} s (measured) + first "
                   f"{min(trades, L)} of {L} trades {tt:.2f} s (measured), trades extrapolated to "
                   f"{per_trade * L:.1f} s; round estimate {round_s:.1f} s without the final row rebuild"),
        "host_cpu": model,
        "host_nproc": ncpu,
        "host_threads_available": avail,
    }


def cpu_baseline_batch(graphs, seeds, budget_s: float = 15.0):
    """The oracle (IM-CB form, single-threaded) on round 0 of the batch's
    chains, in order, until `budget_s` seconds of oracle time have passed."""
    import oracle
    o = oracle.default()
    edges, spent, done = 0, 0.0, 0
    for (rp, col), seed in zip(graphs, seeds):
        t0 = time.perf_counter()
        o.global_trade(rp, col, seed, 0, "o2")
        spent += time.perf_counter() - t0
        edges += len(col) // 2
        done += 1
        if spent >= budget_s:
            break
    model, ncpu, avail = host_cpu()
    return {"value": edges / spent, "unit": "edge-trades/s", "cores": 1, "kind": "oracle",
            "sample": f"IM-CB-form oracle, round 0 of the first {done} of {len(graphs)} chains "
                      f"({edges} edges) in {spent:.1f} s, rebuild included",
            "host_cpu": model, "host_nproc": ncpu, "host_threads_available": avail}


def copy_bandwidth(nbytes: int = 4 << 30):
    """Device-to-device copy of nbytes, best of 5 (read + write bytes / s)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / best


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return 0.0
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def timed_steps(step, steps: int):
    """Run `steps` steps on torch's current stream, bracketed by syncs; per-step
    durations from events on the same stream. Returns (wall_s, [ms])."""
    import torch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(steps):
        step(k)
        evs[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]


def run_single(args, cb, row_ptr, col):
    import torch
    n, m = len(row_ptr) - 1, len(col) // 2
    reps = []
    step_ms_all = []
    kernel_ms = None
    st = None
    tune = None
    for rep in range(args.reps):
        t_up = time.perf_counter()
        g = cb.Graph(row_ptr, col, validate=False)
        torch.cuda.synchronize()
        t_up = time.perf_counter() - t_up
        if args.tune:
            # the library's autotuner (cached per process by the graph's shape),
            # before the timed rounds
            tune = g.autotune(trial_rounds=2, use_cache=True)
        for opt, val in ((cb.OPT_SMALL_MAX, args.small_max), (cb.OPT_BIG_WORKERS, args.big_workers),
                         (cb.OPT_GRID_BLOCKS, args.grid_blocks), (cb.OPT_LOCAL_STACK, args.local_stack),
                         (cb.OPT_FUSE_NEXT, args.fuse)):
            if val is not None:
                g.set_option(opt, val)
        g.set_option(cb.OPT_TIMING, 1)
        for r in range(args.warmup):
            g.global_trade(args.seed, r)
            g.sync()
        g.kernel_times()  # discard warm-up timings
        wall, per_step = timed_steps(lambda k: g.global_trade(args.seed, args.warmup + k), args.steps)
        g.sync()
        km, _ = g.kernel_times()
        st = g.stats()
        g.close()
        reps.append(wall)
        step_ms_all += per_step
        kernel_ms = km if kernel_ms is None else [a + b for a, b in zip(kernel_ms, km)]
        print(f"[bench] repetition {rep}: {args.steps} rounds in {wall:.3f} s (upload {t_up:.2f} s); "
              f"kernel ms {[round(x, 2) for x in km]}", file=sys.stderr, flush=True)
    kernel_ms = [x / args.reps for x in kernel_ms]
    return reps, step_ms_all, kernel_ms, st, t_up, tune


def run_batch(args, cb, graphs, seeds):
    import torch
    reps, step_ms_all, tune = [], [], None
    for rep in range(args.reps):
        b = cb.Batch(graphs, seeds, validate=False)
        tune = b.autotune(trial_rounds=2, use_cache=True)
        if args.fuse is not None:
            b.set_option(cb.OPT_FUSE_NEXT, args.fuse)
        for _ in range(args.warmup):
            b.run(1)
        b.sync()
        wall, per_step = timed_steps(lambda k: b.run(1), args.steps)
        b.sync()
        b.close()
        reps.append(wall)
        step_ms_all += per_step
        print(f"[bench] repetition {rep}: {args.steps} rounds of {len(graphs)} chains in {wall:.3f} s; "
              f"tuned {tune}", file=sys.stderr, flush=True)
    # the same chains one by one on the single-chain path (plain kernel)
    torch.cuda.synchronize()
    t_single = 0.0
    for c, (rp, col) in enumerate(graphs):
        g = cb.Graph(rp, col, validate=False)
        for r in range(args.warmup):
            g.global_trade(seeds[c], r)
        g.sync()
        t0 = time.perf_counter()
        for r in range(args.warmup, args.warmup + args.steps):
            g.global_trade(seeds[c], r)
        g.sync()
        t_single += time.perf_counter() - t0
        g.close()
    return reps, step_ms_all, tune, t_single


def run_serve(args, cb, graphgen):
    """Closed batch (every request at t = 0) to measure capacity, then a
    Poisson stream at 0.7x that rate through the continuous-batching server.
    Returns the JSON fields of the serving run."""
    import numpy as np
    import torch
    spec = graphgen.serve_specs(args.requests)
    graphs = [graphgen.pld_graph(s["n"], s["a"], s["b"], s["gamma"], s["graph_seed"]) for s in spec]
    work = [len(c) // 2 * s["samples"] * s["rounds"] for (_, c), s in zip(graphs, spec)]
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.6 * free)

    def serve(arrivals):
        srv = cb.Server(budget)
        order = np.argsort(arrivals, kind="stable")
        pending = list(order)
        inflight = {}
        done_at = {}
        steps = 0
        t0 = time.perf_counter()
        while pending or inflight:
            now = time.perf_counter() - t0
            while pending and arrivals[pending[0]] <= now:
                q = pending.pop(0)
                s = spec[q]
                inflight[srv.submit(*graphs[q], s["samples"], s["rounds"], s["chain_seed"])] = q
            if not inflight:
                time.sleep(max(0.0, arrivals[pending[0]] - now))
                continue
            srv.step()
            steps += 1
            now = time.perf_counter() - t0
            for rid in [r for r in inflight if srv.finished(r)]:
                done_at[inflight.pop(rid)] = now
                srv.release(rid)
        srv.close()
        lat = [done_at[q] - arrivals[q] for q in range(len(spec))]
        return lat, max(done_at.values()), steps

    lat0, span0, steps0 = serve(np.zeros(len(spec)))
    capacity = len(spec) / span0
    rate = 0.7 * capacity
    rng = np.random.Generator(np.random.PCG64(11))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, len(spec)))
    arrivals -= arrivals[0]
    lat, span, steps = serve(arrivals)
    print(f"[bench] serve: capacity {capacity:.2f} req/s (closed batch {span0:.2f} s), "
          f"Poisson at {rate:.2f} req/s: span {span:.2f} s, p50 {np.median(lat):.2f} s", file=sys.stderr, flush=True)
    return {
        "requests": len(spec), "edge_trades": int(sum(work)), "budget_bytes": budget,
        "closed_batch_s": span0, "capacity_req_per_s": capacity, "rate_req_per_s": rate,
        "span_s": span, "server_steps": steps, "latency_p50_s": percentile(lat, 0.5),
        "latency_p99_s": percentile(lat, 0.99), "latency_max_s": max(lat),
        "closed_batch_edge_trades_per_s": sum(work) / span0,
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed rounds (default 10; batch 16)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed rounds (default 1; batch 2)")
    ap.add_argument("--reps", type=int, default=5, help="repetitions from a fresh upload (median reported)")
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-trades", type=int, default=1 << 19,
                    help="trades of the oracle sample (0 disables the CPU baseline)")
    ap.add_argument("--small-max", type=int, default=None)
    ap.add_argument("--big-workers", type=int, default=None)
    ap.add_argument("--grid-blocks", type=int, default=None)
    ap.add_argument("--local-stack", type=int, default=None)
    ap.add_argument("--tune", type=int, default=1, choices=[0, 1],
                    help="single chain: options from the library's autotuner (default on)")
    ap.add_argument("--fuse", type=int, default=None, choices=[0, 1],
                    help="prepare the next round in the rebuild (default on)")
    ap.add_argument("--requests", type=int, default=32, help="requests of the served workload")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one plain device-to-device copy of BYTES (for scaling "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args(argv)
    if args.steps is None:
        args.steps = 16 if args.workload == "batch" else 10
    if args.warmup is None:
        # a batch captures its round graph on the first two rounds (before and
        # after the first prepared round)
        args.warmup = 2 if args.workload == "batch" else 1

    if args.copy_calibration:
        import torch
        torch.cuda.set_device(0)
        src = torch.ones(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calibration}))
        return 0

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU; runs on several GPUs are not supported "
              "(independent chains shard one per GPU with no exchange).", file=sys.stderr)
        return 2

    import torch

    import graphgen
    import paper_1804_08487_amd as cb

    torch.cuda.set_device(0)
    # the library's work and the per-step events share this stream (on the
    # default stream's null handle the library would use a stream of its own)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    copy_bps = copy_bandwidth()
    print(f"[bench] device copy {copy_bps / 1e9:.0f} GB/s (read + write)", file=sys.stderr, flush=True)
    if args.workload == "quality":
        from paper_1804_08487_amd import quality
        t0 = time.perf_counter()
        q = quality.study(supersteps=args.steps if args.steps != 10 else 300)
        wall = time.perf_counter() - t0
        out = {"metric": "chain quality (fraction of edges still correlated vs thinning; swap fraction)",
               "value": None, "unit": "fraction", "n_gpus": 1, "steps": None, "warmup": 0,
               "higher_is_better": False, "data": "synthetic",
               "config": {"workload": f"quality: {WORKLOAD_TEXT['quality']}"}, "wall_s": wall, "quality": q}
        print(json.dumps(out), flush=True)
        return 0
    if args.workload == "serve":
        sv = run_serve(args, cb, graphgen)
        out = {"metric": "edge-trades/sec per global super-step (m x rounds / s)",
               "value": sv["edge_trades"] / sv["span_s"], "unit": "edge-trades/s", "n_gpus": 1,
               "steps": sv["server_steps"], "warmup": 0, "ms_per_step": sv["span_s"] * 1e3 / sv["server_steps"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
               "data": "synthetic", "config": {"workload": f"serve: {WORKLOAD_TEXT['serve']}",
                                               "requests": sv["requests"]},
               "serving": sv, "copy_kernel_gbps": copy_bps / 1e9, "hbm_peak_gbps": HBM_PEAK / 1e9}
        print(json.dumps(out), flush=True)
        return 0
    t_gen = time.perf_counter()
    if args.workload == "batch":
        spec = graphgen.batch_specs(512)
        graphs = [graphgen.batch_chain(s) for s in spec]
        seeds = [s["chain_seed"] for s in spec]
        n = sum(len(rp) - 1 for rp, _ in graphs)
        m = sum(len(c) // 2 for _, c in graphs)
    else:
        row_ptr, col = graphgen.workload(args.workload)
        n, m = len(row_ptr) - 1, len(col) // 2
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] workload {args.workload}: n={n} m={m} generated in {t_gen:.1f} s", file=sys.stderr, flush=True)

    if args.workload == "batch":
        reps, step_ms, tune, t_single = run_batch(args, cb, graphs, seeds)
    else:
        reps, step_ms, kernel_ms, st, t_up, tune = run_single(args, cb, row_ptr, col)
    wall = statistics.median(reps)
    ms_per_step = wall * 1e3 / args.steps
    value = m * args.steps / wall
    superstep_bytes = 16 * m + 16 * n
    out = {
        "metric": "edge-trades/sec per global super-step (m x rounds / s)",
        "value": value,
        "unit": "edge-trades/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}", "n": n, "m": m,
                   "chain_seed": args.seed if args.workload != "batch" else "c",
                   "rounds_timed": f"{args.warmup}..{args.warmup + args.steps - 1}",
                   "repetitions": args.reps},
        "step_ms_p50": percentile(step_ms, 0.5),
        "step_ms_p99": percentile(step_ms, 0.99),
        "wall_s_per_repetition": reps,
        "copy_kernel_gbps": copy_bps / 1e9,
        "hbm_peak_gbps": HBM_PEAK / 1e9,
        "superstep_algorithmic_frac": superstep_bytes / (ms_per_step / 1e3) / HBM_PEAK,
        "generate_s": t_gen,
    }
    traffic = measured_traffic(args.workload)
    if args.workload == "batch":
        single_value = m * args.steps / t_single
        out["config"]["chains"] = len(graphs)
        out["batched_vs_single_chain"] = {"single_chain_value": single_value, "single_chain_wall_s": t_single,
                                          "ratio": value / single_value}
        out["autotune"] = tune
        if args.cpu_trades > 0:
            print("[bench] timing the oracle sample on the host", file=sys.stderr, flush=True)
            out["cpu_baseline"] = cpu_baseline_batch(graphs, seeds)
        out["roofline"] = {"bound": "hbm", "kernel": "whole step", "achieved": superstep_bytes / (ms_per_step / 1e3) / 1e9,
                           "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                           "frac": superstep_bytes / (ms_per_step / 1e3) / HBM_PEAK,
                           "traffic": traffic["step_bytes"] if traffic else None,
                           "algorithmic_bytes_per_launch": superstep_bytes}
    else:
        names = ["matching", "depscan", "trade", "rebuild"]
        # Algorithmic bytes per launch of the trade kernel: read every
        # round-start adjacency entry and write every final entry once (2m
        # int32 each way).
        trade_bytes = 2 * (2 * m * 4)
        trade_s = kernel_ms[2] / 1e3
        achieved = trade_bytes / trade_s if trade_s > 0 else 0.0
        out["roofline"] = {"bound": "hbm", "kernel": "k_trade", "achieved": achieved / 1e9,
                           "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK,
                           "traffic": kernel_bytes(traffic, "k_trade") if traffic else None,
                           "algorithmic_bytes_per_launch": trade_bytes, "avg_launch_ms": kernel_ms[2]}
        out["step_ms"] = dict(zip(names, kernel_ms))
        if traffic:
            out["superstep_hbm_frac"] = traffic["step_bytes"] / (ms_per_step / 1e3) / HBM_PEAK
            out["superstep_traffic_bytes"] = traffic["step_bytes"]
        out["round_stats"] = st
        out["autotune"] = tune
        out["upload_s_pcie_inclusive"] = t_up
        if args.cpu_trades > 0:
            print("[bench] timing the oracle sample on the host", file=sys.stderr, flush=True)
            out["cpu_baseline"] = cpu_baseline(row_ptr, col, args.seed, args.cpu_trades)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
