"""Influence maximisation drivers on the GPU simulator (paper Section 2,
"Influence Maximization"; CELF in Section 4, "Influence Maximization").

sigma(S) is estimated by Monte Carlo with common random numbers: every
evaluation in one run uses the same rng_seed and trials 0 .. R-1, so the
estimate is itself a monotone submodular coverage function for IC, and lazy
greedy (CELF, Leskovec et al. KDD'07) returns exactly the plain greedy picks.
Ties go to the smallest node id.
"""
from __future__ import annotations

import heapq
import time

import numpy as np

from . import Graph, simulate, simulate_sets, simulate_sets_from


def _sigma_of(graph: Graph, base: list[int], extra: list[int], R: int, rng_seed: int, chunk: int) -> np.ndarray:
    """Totals (sum over trials of active nodes) of base + {v} for v in extra."""
    out = np.zeros(len(extra), dtype=np.int64)
    b = np.asarray(base, dtype=np.uint32)
    for i in range(0, len(extra), chunk):
        sets = [np.append(b, np.uint32(v)) for v in extra[i:i + chunk]]
        out[i:i + chunk] = simulate_sets(graph, sets, R, rng_seed)["totals"]
    return out


class _Incremental:
    """sigma(S + v) from the stored state of S: one full run of S (active
    bits kept on the device) per change of S, then only the cascades that the
    added nodes start (exact, see ims_simulate_sets_from)."""

    def __init__(self, graph: Graph, R: int, rng_seed: int, chunk: int):
        self.graph, self.R, self.rng_seed, self.chunk = graph, R, rng_seed, chunk
        self.key = None
        self.bits = None
        self.total = 0

    def __call__(self, base: list[int], extra: list[int]) -> np.ndarray:
        if not base:
            return _sigma_of(self.graph, base, extra, self.R, self.rng_seed, self.chunk)
        key = tuple(sorted(set(base)))
        if key != self.key:
            r = simulate(self.graph, np.array(key, dtype=np.uint32), self.R, self.rng_seed, want_bits=True,
                         want_node_counts=False)
            self.bits, self.total, self.key = r["active_bits"], int(r["total"]), key
        out = np.zeros(len(extra), dtype=np.int64)
        for i in range(0, len(extra), self.chunk):
            sets = [np.array([v], dtype=np.uint32) for v in extra[i:i + self.chunk]]
            out[i:i + self.chunk] = self.total + simulate_sets_from(self.graph, self.bits, sets, self.R,
                                                                    self.rng_seed)["new_totals"]
        return out


def _evaluator(graph, R: int, rng_seed: int, chunk: int, incremental: bool = False):
    """graph: a Graph (Monte Carlo on the GPU) or a callable
    (base, extra) -> totals standing in for it."""
    if callable(graph) and not isinstance(graph, Graph):
        return graph
    if incremental:
        return _Incremental(graph, R, rng_seed, chunk)
    return lambda base, extra: _sigma_of(graph, base, extra, R, rng_seed, chunk)


def greedy(graph, k: int, R: int, rng_seed: int, candidates=None, chunk: int = 4096, n: int | None = None,
           incremental: bool = False) -> dict:
    """Plain greedy: every round evaluates sigma(S + v) for every candidate."""
    n = graph.n if n is None else n
    sigma_of = _evaluator(graph, R, rng_seed, chunk, incremental)
    cand = list(range(n)) if candidates is None else [int(c) for c in candidates]
    S: list[int] = []
    cur = 0
    evals = 0
    for _ in range(k):
        rest = [v for v in cand if v not in set(S)]
        tot = sigma_of(S, rest)
        evals += len(rest)
        best = int(np.argmax(tot))  # first maximum = smallest id among ties (rest is sorted)
        S.append(rest[best])
        cur = int(tot[best])
    return {"seeds": S, "sigma": cur / R, "evaluations": evals}


def celf(graph, k: int, R: int, rng_seed: int, candidates=None, chunk: int = 4096, batch: int = 64,
         n: int | None = None, log=None, incremental: bool = False) -> dict:
    """Lazy greedy.  The heap holds (-gain upper bound, node, round evaluated);
    stale tops are re-evaluated `batch` at a time against the current S.
    `incremental` evaluates them from the stored state of S (same values).
    `log` (optional) receives a progress line per pick."""
    t0 = time.perf_counter()
    n = graph.n if n is None else n
    sigma_of = _evaluator(graph, R, rng_seed, chunk, incremental)
    cand = sorted(range(n) if candidates is None else {int(c) for c in candidates})
    first = sigma_of([], cand)
    evals = len(cand)
    if log:
        log(f"[celf] first pass: {len(cand)} singletons, {time.perf_counter() - t0:.1f}s")
    heap = [(-int(t), v, 0) for t, v in zip(first, cand)]
    heapq.heapify(heap)
    S: list[int] = []
    cur_total = 0
    gains = []
    while len(S) < k and heap:
        if heap[0][2] == len(S):
            g, v, _ = heapq.heappop(heap)
            S.append(v)
            cur_total += -g
            gains.append(-g / R)
            if log:
                log(f"[celf] pick {len(S)}: node {v}, sigma {cur_total / R:.2f}, {evals} evaluations, "
                    f"{time.perf_counter() - t0:.1f}s")
            continue
        stale = []
        while heap and heap[0][2] != len(S) and len(stale) < batch:
            stale.append(heapq.heappop(heap))
        vs = [v for _, v, _ in stale]
        tot = sigma_of(S, vs)
        evals += len(vs)
        for v, t in zip(vs, tot):
            heapq.heappush(heap, (-(int(t) - cur_total), v, len(S)))
    return {"seeds": S, "sigma": cur_total / R, "gains": gains, "evaluations": evals,
            "seconds": time.perf_counter() - t0}


def main(argv=None) -> int:
    """CELF timing on the paper's CELF benchmark graph (Section 4: a random
    7-regular graph, k = 10, trivalency or weighted-cascade probabilities)."""
    import argparse
    import json

    import synth

    ap = argparse.ArgumentParser(description="CELF on a random 7-regular graph")
    ap.add_argument("--n", type=int, default=5000)
    ap.add_argument("--ewm", choices=["tv", "wc"], default="tv")
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--R", type=int, default=1000)
    ap.add_argument("--rng-seed", type=int, default=5)
    ap.add_argument("--full-mc", action="store_true")
    args = ap.parse_args(argv)
    g = synth.random_regular(args.n, 7, seed=109)
    p = synth.trivalency(g, seed=330) if args.ewm == "tv" else synth.weighted_cascade(g)
    G = Graph(g.n, g.offsets, g.indices, "ic", p)
    celf(G, 2, min(args.R, 256), args.rng_seed, batch=8)  # warm-up (compilation, buffers)
    c = celf(G, args.k, args.R, args.rng_seed, batch=8, incremental=not args.full_mc)
    print(json.dumps({"graph": f"random_7_regular_n{g.n}", "ewm": args.ewm, "k": args.k, "R": args.R,
                      "incremental": not args.full_mc, "seeds": c["seeds"], "sigma": c["sigma"],
                      "evaluations": c["evaluations"], "seconds": round(c["seconds"], 3)}), flush=True)
    G.close()
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
