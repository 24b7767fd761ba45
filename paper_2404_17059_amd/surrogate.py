"""Training data, training loop and surrogate-guided greedy selection.

Influence maximization (paper Section 2, "Influence Maximization") picks k
seeds greedily by Monte Carlo estimates of sigma(S + v); CELF (Section 4)
saves evaluations but still needs sigma for every node in its first pass.  Here
a message-passing network (include/imsim_mpnn.h) trained on simulator
estimates ranks a candidate pool at every step, and only the top r candidates
are estimated by Monte Carlo; the best of those is taken.  The same pipeline
with the network replaced by degree order or random order is the ablation
(the paper's heuristics in Section 4, "Influence Maximization").

    python -m paper_2404_17059_amd.surrogate --out DIR [--stage data|train|select|all]

Every step (simulation, network forward/backward, Adam) runs in libimsim.so;
this module only samples seed sets, batches them and keeps the books.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import Graph, pack_sets, simulate_sets, simulate_sets_into
from . import im
from . import mpnn


# --------------------------------------------------------------------------
# training data

def sample_sets(n: int, deg: np.ndarray, count: int, seed: int, max_size: int = 50) -> tuple[np.ndarray, np.ndarray]:
    """`count` seed sets, sizes uniform on 1..max_size; each member is drawn
    uniformly with probability 1/2, else proportionally to degree + 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(1, max_size + 1, size=count)
    total = int(sizes.sum())
    cdf = np.cumsum(deg.astype(np.float64) + 1.0)
    cdf /= cdf[-1]
    uni = rng.integers(0, n, size=total)
    by_deg = np.minimum(np.searchsorted(cdf, rng.random(total), side="right"), n - 1)
    nodes = np.where(rng.random(total) < 0.5, uni, by_deg).astype(np.uint32)
    offs = np.zeros(count + 1, dtype=np.uint32)
    np.cumsum(sizes, out=offs[1:])
    return offs, nodes


def generate_dataset(graph: Graph, deg: np.ndarray, count: int, trials: int, rng_seed: int, sample_seed: int,
                     chunk: int = 8192, log=None) -> dict:
    """(sets, sigma-hat) pairs: sigma-hat = mean active count over `trials`
    Monte Carlo trials of the simulator (common random numbers)."""
    offs, nodes = sample_sets(graph.n, deg, count, sample_seed)
    totals = np.zeros(count, dtype=np.int64)
    dev = torch.device("cuda", torch.cuda.current_device())
    tot = torch.empty(chunk, dtype=torch.int64, device=dev)
    t0 = time.perf_counter()
    for i in range(0, count, chunk):
        j = min(count, i + chunk)
        o = (offs[i:j + 1] - offs[i]).astype(np.uint32)
        nd = np.ascontiguousarray(nodes[offs[i]:offs[j]])
        simulate_sets_into(graph, o, nd, trials, rng_seed, tot[:j - i])
        totals[i:j] = tot[:j - i].cpu().numpy()
        if log:
            log(f"[data] {j}/{count} sets, {time.perf_counter() - t0:.1f}s")
    return {"offs": offs, "nodes": nodes, "sigma": totals / float(trials), "trials": trials,
            "seconds": time.perf_counter() - t0}


def subset(data: dict, idx: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    offs, nodes = data["offs"], data["nodes"]
    starts, ends = offs[idx].astype(np.int64), offs[idx + 1].astype(np.int64)
    sizes = ends - starts
    o = np.zeros(len(idx) + 1, dtype=np.uint32)
    np.cumsum(sizes, out=o[1:])
    take = np.concatenate([np.arange(s, e) for s, e in zip(starts, ends)]) if len(idx) else np.zeros(0, np.int64)
    return o, np.ascontiguousarray(nodes[take], dtype=np.uint32)


# --------------------------------------------------------------------------
# training

def evaluate(S: mpnn.Surrogate, params, data: dict, idx: np.ndarray, batch: int) -> dict:
    preds = np.zeros(len(idx))
    for i in range(0, len(idx), batch):
        b = idx[i:i + batch]
        o, nd = subset(data, b)
        preds[i:i + len(b)] = S.forward_packed(params, o, nd).cpu().numpy()
    y = data["sigma"][idx]
    return {"mae": float(np.mean(np.abs(preds - y))), "rel": float(np.mean(np.abs(preds - y) / y)),
            "rmse_over_n": float(np.sqrt(np.mean(((preds - y) / S.n) ** 2)))}


def train(S: mpnn.Surrogate, data: dict, epochs: int, batch: int, lr: float, seed: int, val_frac: float = 0.05,
          checkpoint: str | None = None, log=None, time_budget_s: float | None = None, eps: float = 1e-20) -> dict:
    """Adam on the mean squared error of sigma / n; returns params and history.
    With `checkpoint`, state is saved after every epoch and resumed from.
    The loss is scaled by 1/n^2, so gradients are around 1e-9: Adam's eps must
    sit far below them or the steps shrink to nothing."""
    dev = torch.device("cuda", torch.cuda.current_device())
    count = data["sigma"].shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(count)
    n_val = max(1, int(count * val_frac))
    val, tr = perm[:n_val], perm[n_val:]
    state = {"epoch": 0, "step": 0, "history": []}
    params = torch.from_numpy(mpnn.init_params(seed)).to(dev)
    # start the readout bias at the mean per-node activation frequency
    mean_frac = float(np.clip(np.mean(data["sigma"]) / S.n, 1e-6, 1 - 1e-6))
    params[mpnn.OFF["bo"]] = float(np.log(mean_frac / (1 - mean_frac)))
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    if checkpoint and os.path.exists(checkpoint):
        ck = np.load(checkpoint, allow_pickle=False)
        params.copy_(torch.from_numpy(ck["params"]))
        m.copy_(torch.from_numpy(ck["m"]))
        v.copy_(torch.from_numpy(ck["v"]))
        state = json.loads(str(ck["state"]))
    target = torch.empty(batch, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    grads = torch.empty(mpnn.NPARAMS, dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    while state["epoch"] < epochs:
        order = rng.permutation(tr)
        run_loss, nb = 0.0, 0
        te = time.perf_counter()
        for i in range(0, len(order) - batch + 1, batch):
            b = order[i:i + batch]
            o, nd = subset(data, b)
            S.forward_packed(params, o, nd)
            target.copy_(torch.from_numpy(data["sigma"][b].astype(np.float32)), non_blocking=False)
            S.backward(params, target, grads=grads, loss=loss)
            state["step"] += 1
            mpnn.adam_step(params, grads, m, v, lr, state["step"], eps=eps)
            if nb % 200 == 0:
                run_loss += loss.item()
            nb += 1
        state["epoch"] += 1
        ev = evaluate(S, params, data, val, batch)
        rec = {"epoch": state["epoch"], "train_loss_sampled": run_loss, "val": ev, "seconds": time.perf_counter() - te}
        state["history"].append(rec)
        if log:
            log(f"[train] epoch {state['epoch']}: val rel err {ev['rel']:.4f}, mae {ev['mae']:.2f}, {rec['seconds']:.1f}s")
        if checkpoint:
            np.savez(checkpoint + ".tmp.npz", params=params.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(),
                     state=json.dumps(state))
            os.replace(checkpoint + ".tmp.npz", checkpoint)
        if time_budget_s is not None and time.perf_counter() - t0 > time_budget_s:
            break
    return {"params": params, "history": state["history"], "epochs_done": state["epoch"],
            "seconds": time.perf_counter() - t0}


# --------------------------------------------------------------------------
# selection

def guided_greedy(graph: Graph, k: int, trials: int, rng_seed: int, scorer, pool_deg: int = 512, pool_score: int = 512,
                  r: int = 8, deg: np.ndarray | None = None, tol: float | None = 0.1, log=None,
                  incremental: bool = True) -> dict:
    """Greedy with a scorer ranking a candidate pool and Monte Carlo on the
    top r.  scorer(S, pool) -> scores, larger first (the network's scores are
    its sigma(S + v) estimates).  The pool is the top `pool_deg` nodes by
    degree outside S plus the top `pool_score` of the previous step's ranking.
    With `tol` (estimating scorers only): when the estimate for the chosen
    node is off its Monte Carlo value by more than tol (relative), the next r
    candidates are validated too.  With `incremental` the Monte Carlo values
    come from the stored state of S (identical values, less work)."""
    t0 = time.perf_counter()
    mc_of = im._evaluator(graph, trials, rng_seed, 4096, incremental)
    deg_order = np.argsort(-deg, kind="stable")
    S: list[int] = []
    prev_rank = deg_order[:pool_score + pool_deg]
    sigma = 0.0
    mc_sets = 0
    widened = 0
    for _ in range(k):
        chosen = set(S)
        by_deg = [int(v) for v in deg_order[:pool_deg + len(S)] if int(v) not in chosen][:pool_deg]
        by_prev = [int(v) for v in prev_rank if int(v) not in chosen][:pool_score]
        pool = np.array(sorted(set(by_deg) | set(by_prev)), dtype=np.int64)
        est = scorer(S, pool)
        order = np.lexsort((pool, -est))
        ranked = pool[order]
        val = ranked[:r]
        mc = mc_of(S, [int(v) for v in val])
        mc_sets += len(val)
        best_i = int(np.lexsort((val, -mc))[0])
        best, best_mc = int(val[best_i]), int(mc[best_i])
        e = est[order][best_i]
        if tol is not None and abs(e - best_mc / trials) > tol * best_mc / trials and len(ranked) > r:
            more = ranked[r:2 * r]
            mc2 = mc_of(S, [int(v) for v in more])
            mc_sets += len(more)
            widened += 1
            allv = np.concatenate([val, more])
            allmc = np.concatenate([mc, mc2])
            j = int(np.lexsort((allv, -allmc))[0])
            best, best_mc = int(allv[j]), int(allmc[j])
        S.append(best)
        sigma = best_mc / trials
        prev_rank = ranked
        if log and (len(S) % 10 == 0 or len(S) == k):
            log(f"[guided] pick {len(S)}: sigma {sigma:.2f}, {time.perf_counter() - t0:.1f}s")
    return {"seeds": S, "sigma": sigma, "mc_sets": mc_sets, "widened": widened, "seconds": time.perf_counter() - t0}


def net_scorer(S_plan: mpnn.Surrogate, params, batch: int):
    def score(S, pool):
        base = np.array(S, dtype=np.uint32)
        out = []
        for i in range(0, len(pool), batch):
            sets = [np.append(base, np.uint32(v)) for v in pool[i:i + batch]]
            out.append(S_plan.forward(params, sets).clone())
        return torch.cat(out).cpu().numpy().astype(np.float64)
    return score


def degree_scorer(deg):
    """Order only (no sigma estimate): larger degree first."""
    return lambda S, pool: deg[pool].astype(np.float64)


def random_scorer(seed: int):
    """Order only: a fresh random order at every step."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return lambda S, pool: rng.random(len(pool))


def judge(graph: Graph, seeds, trials: int, rng_seed: int) -> float:
    return float(simulate_sets(graph, [np.array(seeds, dtype=np.uint32)], trials, rng_seed)["sigma"][0])


# --------------------------------------------------------------------------

def step_bench(g, wc, batch: int, log, steps: int = 10, warmup: int = 3) -> int:
    """Time training steps (forward, backward, Adam) on `batch` random sets of
    1-50 nodes with HIP events on the launch stream."""
    S = mpnn.Surrogate(g.n, g.offsets, g.indices, wc.astype(np.float32), max_batch=batch)
    params = torch.from_numpy(mpnn.init_params(1)).cuda()
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    offs, nodes = sample_sets(g.n, g.outdeg(), batch, seed=3)
    target = torch.full((batch,), 100.0, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tf = tb = 0.0
    for it in range(warmup + steps):
        ev[0].record()
        S.forward_packed(params, offs, nodes)
        ev[1].record()
        grads = S.backward(params, target)
        mpnn.adam_step(params, grads, m, v, 1e-3, it + 1, eps=1e-20)
        ev[2].record()
        torch.cuda.synchronize()
        if it >= warmup:
            tf += ev[0].elapsed_time(ev[1])
            tb += ev[1].elapsed_time(ev[2])
    log(json.dumps({"n": g.n, "m": g.m, "batch": batch, "forward_ms": tf / steps, "backward_adam_ms": tb / steps,
                    "us_per_set": (tf + tb) / steps / batch * 1e3}))
    S.close()
    return 0


def main(argv=None) -> int:
    import synth

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--stage", default="all", choices=["data", "train", "select", "all", "step-bench"])
    ap.add_argument("--pairs", type=int, default=100_000)
    ap.add_argument("--data-trials", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--train-budget", type=float, default=600.0, help="seconds of training per call")
    ap.add_argument("--k", type=int, default=50)
    ap.add_argument("--R", type=int, default=10_000)
    ap.add_argument("--judge-seed", type=int, default=999)
    ap.add_argument("--celf-batch", type=int, default=8, help="stale heap entries CELF re-evaluates at once")
    ap.add_argument("--full-mc", action="store_true",
                    help="evaluate sigma(S + v) by full simulations instead of from the stored state of S")
    ap.add_argument("--methods", default="surrogate,degree_ranked,random_ranked,heuristics,celf",
                    help="selection methods to run (comma-separated)")
    ap.add_argument("--n", type=int, default=200_000, help="nodes of the Chung-Lu graph (exponent 2.3, mean degree 10)")
    ap.add_argument("--weighting", default="wc", choices=["wc", "tv"],
                    help="arc probabilities: weighted cascade 1/indeg(v), or trivalency (each arc one of "
                         "0.1, 0.01, 0.001, seeded), the paper's Section 4 weightings")
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)
    log = lambda *a: print(*a, flush=True)
    torch.cuda.set_device(0)
    g, wc = synth.chung_lu_wc_200k(args.n)
    if args.weighting == "tv":
        wc = synth.trivalency(g, seed=106)
    deg = g.outdeg().astype(np.int64)
    G = Graph(g.n, g.offsets, g.indices, "ic", wc)
    if args.stage == "step-bench":
        return step_bench(g, wc, args.batch, log)
    data_path = os.path.join(args.out, "pairs.npz")
    ck_path = os.path.join(args.out, "surrogate.npz")
    report = {"graph": {"n": g.n, "m": g.m, "sha256": g.sha256()}, "weighting": args.weighting}
    if args.stage in ("data", "all"):
        d = generate_dataset(G, deg, args.pairs, args.data_trials, rng_seed=7, sample_seed=8, log=log)
        np.savez(data_path, offs=d["offs"], nodes=d["nodes"], sigma=d["sigma"], trials=d["trials"])
        report["data_seconds"] = d["seconds"]
        log(f"[data] {args.pairs} pairs in {d['seconds']:.1f}s")
    if args.stage in ("train", "all"):
        z = np.load(data_path, allow_pickle=False)
        d = {k: z[k] for k in ("offs", "nodes", "sigma")}
        S = mpnn.Surrogate(g.n, g.offsets, g.indices, wc.astype(np.float32), max_batch=args.batch)
        tr = train(S, d, args.epochs, args.batch, args.lr, seed=11, checkpoint=ck_path, log=log,
                   time_budget_s=args.train_budget)
        report["train"] = {"epochs_done": tr["epochs_done"], "seconds": tr["seconds"], "history": tr["history"]}
        S.close()
    if args.stage in ("select", "all"):
        ck = np.load(ck_path, allow_pickle=False)
        S = mpnn.Surrogate(g.n, g.offsets, g.indices, wc.astype(np.float32), max_batch=args.batch)
        params = torch.from_numpy(ck["params"]).cuda()
        sel = {}
        methods = set(args.methods.split(","))
        runs = [("surrogate", net_scorer(S, params, args.batch), 0.1), ("degree_ranked", degree_scorer(deg), None),
                ("random_ranked", random_scorer(12), None)]
        for name, scorer, tol in runs:
            if name not in methods:
                continue
            res = guided_greedy(G, args.k, args.R, rng_seed=5, scorer=scorer, deg=deg, tol=tol, log=log,
                                incremental=not args.full_mc)
            res["judge_sigma"] = judge(G, res["seeds"], args.R, args.judge_seed)
            sel[name] = res
            log(f"[select] {name}: judge sigma {res['judge_sigma']:.2f}, {res['seconds']:.1f}s")
        if "heuristics" in methods:
            top = np.argsort(-deg, kind="stable")[:args.k]
            sel["top_degree"] = {"seeds": [int(v) for v in top], "judge_sigma": judge(G, top, args.R, args.judge_seed)}
            rnd = np.random.Generator(np.random.PCG64(13)).choice(g.n, args.k, replace=False)
            sel["random"] = {"seeds": [int(v) for v in rnd], "judge_sigma": judge(G, rnd, args.R, args.judge_seed)}
            log(f"[select] top degree {sel['top_degree']['judge_sigma']:.2f}, random {sel['random']['judge_sigma']:.2f}")
        if "celf" in methods:
            c = im.celf(G, args.k, args.R, rng_seed=5, batch=args.celf_batch, log=log, incremental=not args.full_mc)
            c["judge_sigma"] = judge(G, c["seeds"], args.R, args.judge_seed)
            sel["celf"] = c
            log(f"[select] celf: judge sigma {c['judge_sigma']:.2f}, {c['seconds']:.1f}s")
        report["select"] = sel
        S.close()
    path = os.path.join(args.out, f"report_{args.stage}_{args.methods.replace(',', '_')}.json" if args.stage == "select"
                        else f"report_{args.stage}.json")
    with open(path, "w") as f:
        json.dump(report, f, indent=1, default=lambda o: o.tolist() if hasattr(o, "tolist") else str(o))
    log(f"[done] {path}")
    G.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
