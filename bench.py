"""Benchmark of the Monte Carlo IC / LT simulator on one MI355X.

A step is one full simulation of the workload (every trial, from graph in HBM
to per-trial counts, per-node counts and total).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default workload: LT on a directed Chung-Lu graph, n = 1,000,000, out-degree
exponent 2.1, mean out-degree 16, weights 1/indeg(v), the 100 nodes of largest
out-degree as seeds, 1,000 trials.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "edge-examinations/sec and trials/sec at 1 GPU; % HBM roofline; surrogate vs plain greedy"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "lt_chunglu_1m": "chung_lu_lt_1m",
    "ba_ic_100k": "ba_ic_100k",
    "er_ic_1k": "er_ic_1k",
}
# IC benchmark graphs after the paper's Section 4 (ER / Watts-Strogatz / a
# Barabasi-Albert stand-in for the Facebook graph x TV / UR / WC weights)
SUITE = ["er_tv", "er_ur", "er_wc", "ws_tv", "ws_ur", "ws_wc", "ba_fb_tv", "ba_fb_ur", "ba_fb_wc"]


def load_workload(name: str):
    import synth
    if name in WORKLOADS:
        return getattr(synth, WORKLOADS[name])()
    return synth.paper_ic_suite()[SUITE.index(name[len("paper_"):])]
KERNEL_SOURCES = ["paper_2404_17059_amd/csrc/sim_kernels.hpp", "paper_2404_17059_amd/csrc/philox.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def load_alg_bytes(workload: str, graph_sha: str, n_trials: int, rng_seed: int):
    path = os.path.join(ROOT, "tests", "golden", f"alg_bytes_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("graph_sha256") != graph_sha or d.get("n_trials") != n_trials or d.get("rng_seed") != rng_seed:
        return None
    return d


def load_traffic(workload: str):
    """Measured HBM bytes per launch from committed rocprofv3 counter runs,
    valid only while the kernel sources are unchanged."""
    path = os.path.join(ROOT, "profiles", f"traffic_simulate_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256") != kernel_source_sha():
        return None
    return d


def cpu_baseline(w, sample_trials: int, threads: int) -> dict:
    import oracle
    enc = oracle.encode(w.model, w.param)
    t0 = time.perf_counter()
    r = oracle.simulate(w.model, w.graph.n, w.graph.offsets, w.graph.indices, enc, w.seeds, sample_trials,
                        w.rng_seed, threads=threads, want_bits=False, want_node_counts=False)
    dt = time.perf_counter() - t0
    exams = int(r["exams"].sum())
    return {"value": exams / dt, "unit": "edge-examinations/s", "cores": threads, "kind": "oracle",
            "sample": f"trials 0..{sample_trials - 1} of {w.n_trials} of the same workload (same graph, seeds, rng_seed)",
            "trials_per_sec": sample_trials / dt, "seconds": round(dt, 3)}


def copy_calibration(mib: int) -> int:
    """A plain copy of known size: reads and writes mib MiB each time, so
    hardware byte counters can be scaled to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "bytes_read_per_copy": n * 4, "bytes_written_per_copy": n * 4}))
    return 0


def run_suite(args) -> int:
    """The nine IC benchmark workloads, each timed as in the main mode; one
    JSON line with the summed work over the summed time and the per-workload
    figures."""
    import torch

    import paper_2404_17059_amd as ims
    import synth

    rows, tot_exams, tot_s, tot_trials = [], 0, 0.0, 0
    for w in synth.paper_ic_suite():
        g = w.graph
        G = ims.Graph(g.n, g.offsets, g.indices, w.model, w.param)
        T = w.n_trials
        dev = torch.device("cuda", 0)
        tc = torch.empty(T, dtype=torch.int32, device=dev)
        tot = torch.empty(1, dtype=torch.int64, device=dev)
        nc = torch.empty(g.n, dtype=torch.int32, device=dev)
        for _ in range(args.warmup):
            ims.simulate_into(G, w.seeds, T, w.rng_seed, tc, tot, nc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ims.simulate_into(G, w.seeds, T, w.rng_seed, tc, tot, nc)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        counts = nc.cpu().numpy().view(np.uint32).astype(np.int64)
        exams = int((counts * g.outdeg()).sum())
        rows.append({"workload": w.name, "n": g.n, "m": g.m, "ms": round(dt * 1e3, 4), "mean_spread": int(tot.item()) / T,
                     "exams_per_s": exams / dt, "trials_per_s": T / dt})
        tot_exams += exams
        tot_s += dt
        tot_trials += T
        log(f"[bench] {w.name}: {dt * 1e3:.3f} ms per {T} trials, mean spread {int(tot.item()) / T:.1f}")
        G.close()
    print(json.dumps({"metric": METRIC, "value": tot_exams / tot_s, "unit": "edge-examinations/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(tot_s * 1e3, 4),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                      "data": "synthetic", "config": {"workload": "ic_paper_suite_9x1000_trials_100_seeds"},
                      "trials_per_sec": tot_trials / tot_s, "suite": rows}), flush=True)
    return 0


def run_batch(args) -> int:
    """The 64-item uneven batch (IC and LT mixed, 2,000 trials each) as one
    persistent launch replayed from its HIP graph: timed with the default
    schedule, then autotuned and timed again; one JSON line."""
    import torch

    import paper_2404_17059_amd as ims
    import synth

    t0 = time.perf_counter()
    ws = synth.batch_items()
    log(f"[bench] batch of {len(ws)} items generated in {time.perf_counter() - t0:.1f}s")
    items = [(ims.Graph(w.graph.n, w.graph.offsets, w.graph.indices, w.model, w.param), w.seeds, w.n_trials, w.rng_seed)
             for w in ws]
    B = ims.Batch(items)

    def timed() -> float:
        for _ in range(args.warmup):
            B.launch()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            B.launch()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / args.steps

    dt_default = timed()
    log(f"[bench] default schedule: {dt_default * 1e3:.2f} ms per launch")
    chosen = B.autotune(repeats=1)
    dt = timed()
    log(f"[bench] autotuned {chosen}: {dt * 1e3:.2f} ms per launch")
    res = B.results()
    exams = sum(int((r["node_counts"].astype(np.int64) * w.graph.outdeg()).sum()) for r, w in zip(res, ws))
    trials = sum(w.n_trials for w in ws)
    print(json.dumps({"metric": METRIC, "value": exams / dt, "unit": "edge-examinations/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 4),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                      "data": "synthetic",
                      "config": {"workload": "batch_64_items_er_ba_ic_lt_2000_trials", "items": len(ws),
                                 "sum_n": int(sum(w.graph.n for w in ws)), "sum_m": int(sum(w.graph.m for w in ws))},
                      "trials_per_sec": trials / dt, "default_ms_per_step": round(dt_default * 1e3, 4),
                      "tuning": {"blocks_per_cu": chosen[0], "order": chosen[1], "split": chosen[2]},
                      "mean_spreads": [r["mean"] for r in res]}), flush=True)
    B.close()
    for it in items:
        it[0].close()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lt_chunglu_1m",
                    choices=sorted(WORKLOADS) + ["paper_" + x for x in SUITE] + ["paper_suite", "batch64"])
    ap.add_argument("--cpu-sample", type=int, default=64, help="oracle trials timed for cpu_baseline (0 = skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported by this build "
              "(trials would shard across GPUs with one all-reduce of the counts at the end).", file=sys.stderr)
        return 2

    import torch

    import paper_2404_17059_amd as ims

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "paper_suite":
        return run_suite(args)
    if args.workload == "batch64":
        return run_batch(args)
    t0 = time.perf_counter()
    w = load_workload(args.workload)
    g = w.graph
    log(f"[bench] workload {w.name}: n={g.n} m={g.m} T={w.n_trials} seeds={len(w.seeds)} "
        f"generated in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    G = ims.Graph(g.n, g.offsets, g.indices, w.model, w.param)
    create_s = time.perf_counter() - t0
    T = w.n_trials
    dev = torch.device("cuda", 0)
    tc = torch.empty(T, dtype=torch.int32, device=dev)
    tot = torch.empty(1, dtype=torch.int64, device=dev)
    nc = torch.empty(g.n, dtype=torch.int32, device=dev)
    opts = ims.Opts(shape=0, blocks_per_cu=0, alpha=0.0, profile=1)
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        ims.simulate_into(G, w.seeds, T, w.rng_seed, tc, tot, nc, opts=opts)
    torch.cuda.synchronize()
    G.profile(reset=True)
    log(f"[bench] warmup done ({args.warmup} steps)")

    torch.cuda.synchronize()
    t_begin = time.perf_counter()
    for i in range(args.steps):
        ims.simulate_into(G, w.seeds, T, w.rng_seed, tc, tot, nc, opts=opts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_begin
    kern_ms, kern_n = G.profile(reset=True)
    steps_taken, guard = G.last_status(stream)
    if guard:
        raise RuntimeError("step guard fired")
    log(f"[bench] timed {args.steps} steps in {elapsed:.4f}s; kernel {kern_ms / max(kern_n, 1):.3f} ms/launch")

    node_counts = nc.cpu().numpy().view(np.uint32).astype(np.int64)
    total = int(tot.item())
    exams_per_step = int((node_counts * g.outdeg()).sum())  # sum over trials of out-degrees of active nodes
    ms_per_step = elapsed * 1e3 / args.steps
    exams_per_s = exams_per_step * args.steps / elapsed
    trials_per_s = T * args.steps / elapsed

    kernel_avg_s = kern_ms / 1e3 / max(kern_n, 1)
    alg = load_alg_bytes(args.workload, g.sha256(), T, w.rng_seed)
    traffic = load_traffic(args.workload)
    roofline = None
    if alg is not None:
        achieved = alg["bytes"] / kernel_avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None if traffic is None else traffic["bytes_per_launch"],
                    "kernel": "ims_simulate call (count-threshold table, ltg_sweep_kernel sweeps, final pass)", "kernel_ms": round(kernel_avg_s * 1e3, 4),
                    "alg_bytes_per_launch": alg["bytes"], "alg_units_per_launch": alg["units"]}

    cpu = None
    if args.cpu_sample > 0:
        import oracle
        threads = min(16, len(os.sched_getaffinity(0)))
        oracle.build() if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")) else None
        log(f"[bench] cpu_baseline: oracle on {args.cpu_sample} trials, {threads} threads")
        cpu = cpu_baseline(w, min(args.cpu_sample, T), threads)

    rec = {
        "metric": METRIC,
        "value": exams_per_s,
        "unit": "edge-examinations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w.name, "model": w.model, "n": g.n, "m": g.m, "trials": T,
                   "seeds": int(len(w.seeds)), "rng_seed": w.rng_seed, "parallelism": "trial-bit-parallel, 1 GPU"},
        "trials_per_sec": trials_per_s,
        "mean_spread": total / T,
        "exams_per_step": exams_per_step,
        "steps_per_run": steps_taken,
        "graph_create_s": round(create_s, 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    G.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
