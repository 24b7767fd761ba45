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
# every source that decides what the simulation kernels do and how they are
# launched (grid sizes, padding, threshold form): a measured traffic figure is
# reported only while all of them are unchanged
KERNEL_SOURCES = ["paper_2404_17059_amd/csrc/sim_kernels.hpp", "paper_2404_17059_amd/csrc/philox.hpp",
                  "paper_2404_17059_amd/csrc/imsim.hip"]


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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(w, sample_trials: int, threads: int) -> dict:
    import oracle
    enc = oracle.encode(w.model, w.param)
    t0 = time.perf_counter()
    r = oracle.simulate(w.model, w.graph.n, w.graph.offsets, w.graph.indices, enc, w.seeds, sample_trials,
                        w.rng_seed, threads=threads, want_bits=False, want_node_counts=False)
    dt = time.perf_counter() - t0
    exams = int(r["exams"].sum())
    return {"value": exams / dt, "trials_per_sec": sample_trials / dt, "seconds": round(dt, 3),
            "trials": sample_trials, "threads": threads}


def cpu_baseline(w, sample_all: int, sample_one: int) -> dict:
    """The oracle on the host: trial-parallel on every core this process may
    use (the affinity set, capped by OMP_NUM_THREADS when that is set, as on a
    host shared per GPU), and on one thread; each on a bounded sample of the
    workload's trials (same graph, seeds and rng_seed)."""
    visible = len(os.sched_getaffinity(0))
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    threads = min(visible, share) if share > 0 else visible
    log(f"[bench] cpu_baseline: oracle on {sample_all} trials x {threads} threads, then {sample_one} trials x 1 thread")
    allc = oracle_rate(w, sample_all, threads)
    one = oracle_rate(w, sample_one, 1)
    return {"value": allc["value"], "unit": "edge-examinations/s", "cores": threads, "kind": "oracle",
            "sample": f"trials 0..{sample_all - 1} of {w.n_trials} of the same workload (same graph, seeds, rng_seed); "
                      f"one-thread leg on trials 0..{sample_one - 1}",
            "trials_per_sec": allc["trials_per_sec"], "seconds": allc["seconds"],
            "one_thread": {"value": one["value"], "trials_per_sec": one["trials_per_sec"], "seconds": one["seconds"],
                           "trials": sample_one},
            "cpu_model": cpu_model(), "host_cpus_visible": visible,
            "omp_num_threads": share or None}


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


def _counter_sums(dirpath: str):
    """Per-kernel sums of one rocprofv3 --pmc run's counter (csv output)."""
    import csv
    import glob
    files = glob.glob(os.path.join(dirpath, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {dirpath}")
    per, disp = {}, {}
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                k = r["Kernel_Name"]
                per[k] = per.get(k, 0.0) + float(r["Counter_Value"])
                disp.setdefault(k, set()).add(r.get("Dispatch_Id"))
    return per, {k: len(v) for k, v in disp.items()}


def traffic_record(dirs, copy_mib: int, calls: int, workload: str) -> int:
    """Measured bytes per call from four rocprofv3 runs (FETCH_SIZE and
    WRITE_SIZE of the workload, then of the copy calibration): each counter is
    scaled by the bytes the copy is known to move per KiB it reads, summed over
    the library's kernels and divided by the calls in the run.  Prints the
    per-kernel table and writes profiles/traffic_simulate_<workload>.json,
    keyed to the kernel sources."""
    fetch, fd = _counter_sums(dirs[0])
    write, wd = _counter_sums(dirs[1])
    cfetch, _ = _counter_sums(dirs[2])
    cwrite, _ = _counter_sums(dirs[3])
    copy_bytes = 3 * copy_mib * (1 << 20)
    cf = max(cfetch.values())
    cw = max(cwrite.values())
    fscale, wscale = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    print(f"calibration: the copy reads FETCH_SIZE {cf:.1f} KiB and WRITE_SIZE {cw:.1f} KiB for {copy_bytes} B each way; "
          f"bytes = FETCH_SIZE x {fscale:.4f} KiB, WRITE_SIZE x {wscale:.4f} KiB")
    names = sorted(set(fetch) | set(write), key=lambda k: -(fetch.get(k, 0) + write.get(k, 0)))
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB |\n|---|---:|---:|---:|")
    for k in names:
        print(f"| `{k[:90]}` | {fd.get(k, wd.get(k, 0))} | {fetch.get(k, 0):.0f} | {write.get(k, 0):.0f} |")
    lib = [k for k in names if "imsim" in k]
    fb = sum(fetch.get(k, 0) for k in lib) * 1024 * fscale / calls
    wb = sum(write.get(k, 0) for k in lib) * 1024 * wscale / calls
    print(f"library kernels per call: read {fb / 1e9:.3f} GB, written {wb / 1e9:.3f} GB, total {(fb + wb) / 1e9:.3f} GB")
    out = os.path.join(ROOT, "profiles", f"traffic_simulate_{workload}.json")
    with open(out, "w") as f:
        json.dump({"workload": workload, "bytes_per_launch": int(fb + wb), "fetch_bytes": int(fb), "write_bytes": int(wb),
                   "fetch_scale": fscale, "write_scale": wscale, "kernel_source_sha256": kernel_source_sha(),
                   "source": f"profiles/simulate_{workload}_hbm_traffic.md"}, f, indent=1)
    print("wrote", out)
    return 0


def run_suite(args) -> int:
    """The nine IC benchmark workloads, each timed as in the main mode; one
    JSON line with the summed work over the summed time and the per-workload
    figures."""
    import torch

    import paper_2404_17059_amd as ims
    import synth

    rows, tot_exams, tot_s, tot_trials = [], 0, 0.0, 0
    opts = ims.Opts(shape=args.shape, ic_direction={"auto": 0, "push": 1, "pull": 2}[args.ic_direction])
    suite = synth.paper_ic_suite()
    if args.with_c1c2:
        suite = suite + [synth.er_ic_1k(), synth.ba_ic_100k()]
    for w in suite:
        g = w.graph
        G = ims.Graph(g.n, g.offsets, g.indices, w.model, w.param)
        T = w.n_trials
        dev = torch.device("cuda", 0)
        tc = torch.empty(T, dtype=torch.int32, device=dev)
        tot = torch.empty(1, dtype=torch.int64, device=dev)
        nc = torch.empty(g.n, dtype=torch.int32, device=dev)
        for _ in range(args.warmup):
            ims.simulate_into(G, w.seeds, T, w.rng_seed, tc, tot, nc, opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ims.simulate_into(G, w.seeds, T, w.rng_seed, tc, tot, nc, opts=opts)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        dirs = G.level_directions()
        counts = nc.cpu().numpy().view(np.uint32).astype(np.int64)
        exams = int((counts * g.outdeg()).sum())
        rows.append({"workload": w.name, "n": g.n, "m": g.m, "ms": round(dt * 1e3, 4), "mean_spread": int(tot.item()) / T,
                     "exams_per_s": exams / dt, "trials_per_s": T / dt,
                     "levels_pulled": f"{int((dirs == 2).sum())}/{len(dirs)}" if len(dirs) else None})
        tot_exams += exams
        tot_s += dt
        tot_trials += T
        log(f"[bench] {w.name}: {dt * 1e3:.3f} ms per {T} trials, mean spread {int(tot.item()) / T:.1f}")
        G.close()
    print(json.dumps({"metric": METRIC, "value": tot_exams / tot_s, "unit": "edge-examinations/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(tot_s * 1e3, 4),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                      "data": "synthetic", "config": {"workload": "ic_paper_suite_9x1000_trials_100_seeds"
                                                      + ("_plus_er_1k_ba_100k" if args.with_c1c2 else ""),
                                                      "shape": args.shape, "ic_direction": args.ic_direction},
                      "trials_per_sec": tot_trials / tot_s, "suite": rows}), flush=True)
    return 0


def run_sets(args) -> int:
    """Many-sets evaluation on the 200k-node Chung-Lu graph with
    weighted-cascade p (the influence-maximisation workload): every node as a
    singleton set, and the 2,000 largest-out-degree singletons (the largest
    cascades), each set's trials under common random numbers.  One JSON line
    with set-trials/s for each case."""
    import torch

    import paper_2404_17059_amd as ims
    import synth

    g, param = synth.chung_lu_wc_200k()
    G = ims.Graph(g.n, g.offsets, g.indices, "ic", param)
    order = np.argsort(-g.outdeg(), kind="stable")
    dev = torch.device("cuda", 0)
    rows, tot_st, tot_s = [], 0, 0.0
    for label, k, R in (("all_singletons", g.n, 1000), ("top2000_singletons", 2000, 1000), ("top2000_singletons", 2000, 10000)):
        offs, nodes = ims.pack_sets([[int(x)] for x in order[:k]])
        tot = torch.empty(k, dtype=torch.int64, device=dev)
        for _ in range(args.warmup):
            ims.simulate_sets_into(G, offs, nodes, R, 5, tot)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ims.simulate_sets_into(G, offs, nodes, R, 5, tot)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        mean = float(tot.sum().item()) / (k * R)
        rows.append({"case": label, "sets": k, "trials": R, "s": round(dt, 4), "set_trials_per_s": k * R / dt,
                     "mean_spread": round(mean, 3)})
        tot_st += k * R
        tot_s += dt
        log(f"[bench] {label} x{k} R={R}: {dt:.3f} s, {k * R / dt:.3e} set-trials/s")
    G.close()
    print(json.dumps({"metric": METRIC, "value": tot_st / tot_s, "unit": "set-trials/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(tot_s * 1e3, 4),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                      "data": "synthetic", "config": {"workload": "ic_sets_chung_lu_wc_n200000"}, "cases": rows}), flush=True)
    return 0


def batch_timeline(B, ws) -> dict:
    """One more launch with per-task timing: the span from the first task's
    start to the last task's end, how busy the workgroup slots were, and the
    items that took the most task time (device wall clock, 100 MHz)."""
    import torch
    B.task_timing(True)
    B.launch()
    torch.cuda.synchronize()
    codes, times = B.task_times()
    B.task_timing(False)
    if len(codes) == 0:
        return {}
    start, end, slot = times[:, 0].astype(np.int64), times[:, 1].astype(np.int64), times[:, 2].astype(np.int64)
    t0 = int(start.min())
    span = int(end.max()) - t0
    busy = int((end - start).sum())
    slots = int(slot.max()) + 1
    item = (codes >> np.uint64(32)).astype(np.int64)
    per_item = np.bincount(item, weights=(end - start).astype(np.float64), minlength=len(ws))
    top = np.argsort(-per_item)[:8]
    last_end = np.sort(end - t0)
    return {"clock_mhz": 100, "span_ms": span / 1e5, "slots": slots, "tasks": int(len(codes)),
            "slot_busy_frac": busy / (slots * span) if span > 0 else None,
            "median_task_us": float(np.median(end - start)) / 100.0, "max_task_us": float((end - start).max()) / 100.0,
            "ms_until_90pct_tasks_done": float(last_end[int(0.9 * (len(last_end) - 1))]) / 1e5,
            "top_items": [{"item": ws[i].name, "task_ms": float(per_item[i]) / 1e5,
                           "share": float(per_item[i] / per_item.sum())} for i in top]}


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
    timeline = batch_timeline(B, ws)
    exams = sum(int((r["node_counts"].astype(np.int64) * w.graph.outdeg()).sum()) for r, w in zip(res, ws))
    trials = sum(w.n_trials for w in ws)
    print(json.dumps({"metric": METRIC, "value": exams / dt, "unit": "edge-examinations/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 4),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                      "data": "synthetic",
                      "config": {"workload": "batch_64_items_er_ba_ic_lt_2000_trials", "items": len(ws),
                                 "sum_n": int(sum(w.graph.n for w in ws)), "sum_m": int(sum(w.graph.m for w in ws))},
                      "trials_per_sec": trials / dt, "default_ms_per_step": round(dt_default * 1e3, 4),
                      "tuning": {"blocks_per_cu": chosen[0], "order": chosen[1], "split": chosen[2],
                                 "ic_alpha": chosen[3], "ic_beta": chosen[4]},
                      "mean_spreads": [r["mean"] for r in res], "timeline": timeline}), flush=True)
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
                    choices=sorted(WORKLOADS) + ["paper_" + x for x in SUITE] + ["paper_suite", "batch64", "c5_sets"])
    ap.add_argument("--cpu-sample", type=int, default=64, help="oracle trials timed on all cores for cpu_baseline (0 = skip)")
    ap.add_argument("--cpu-sample-one", type=int, default=16, help="oracle trials timed on one thread for cpu_baseline")
    ap.add_argument("--shape", type=int, default=0, choices=[0, 1, 2],
                    help="paper_suite: execution shape (0 automatic, 1 word-local, 2 grid-wide)")
    ap.add_argument("--ic-direction", default="auto", choices=["auto", "push", "pull"],
                    help="paper_suite: IC direction (auto = the per-level rule)")
    ap.add_argument("--with-c1c2", action="store_true",
                    help="paper_suite: also run the 1k-node ER and 100k-node BA IC workloads")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB three times (HBM counter calibration)")
    ap.add_argument("--traffic-record", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="only summarise four rocprofv3 --pmc runs (the workload's FETCH_SIZE and WRITE_SIZE, then the "
                         "copy calibration's) into profiles/traffic_simulate_<workload>.json")
    ap.add_argument("--copy-mib", type=int, default=1024, help="--traffic-record: MiB per copy of the calibration run")
    ap.add_argument("--calls", type=int, default=1, help="--traffic-record: simulate calls in the counted run")
    args = ap.parse_args()
    if args.traffic_record:
        return traffic_record(args.traffic_record, args.copy_mib, args.calls, args.workload)
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
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
    if args.workload == "c5_sets":
        return run_sets(args)
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
        # frac: algorithmic bytes (the push traffic of the frontier expansion)
        # per second; frac_measured: the bytes the hardware counters saw
        measured = None if traffic is None else traffic["bytes_per_launch"] / kernel_avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None if traffic is None else traffic["bytes_per_launch"],
                    "achieved_measured": None if measured is None else round(measured, 1),
                    "frac_measured": None if measured is None else round(measured / HBM_PEAK_GBS, 4),
                    "kernel": "ims_simulate call (count-threshold table, ltg_sweep_kernel sweeps, final pass)", "kernel_ms": round(kernel_avg_s * 1e3, 4),
                    "alg_bytes_per_launch": alg["bytes"], "alg_units_per_launch": alg["units"]}

    cpu = None
    if args.cpu_sample > 0:
        import oracle
        oracle.build() if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")) else None
        cpu = cpu_baseline(w, min(args.cpu_sample, T), min(max(args.cpu_sample_one, 1), T))

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
