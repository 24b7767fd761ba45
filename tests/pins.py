"""Independent pins for the oracle, built from library routines and exact
enumeration only (numpy's Philox for the hash, scipy's graph search for
reachability, Python fractions for exact probabilities).  Nothing here calls
the oracle or the device path."""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

TWO32 = 1 << 32
MASK64 = (1 << 64) - 1


def numpy_philox_block(rng_seed: int, domain: int, c0: int, c1: int) -> list[int]:
    """Philox4x64-10 output block for counter (c0, c1, 0, 0) and key
    (rng_seed, domain) from numpy, whose generator increments the 256-bit
    counter before producing a block."""
    v = (c0 | (c1 << 64)) - 1
    v &= (1 << 256) - 1
    ctr = [(v >> (64 * i)) & MASK64 for i in range(4)]
    g = np.random.Philox(counter=np.array(ctr, dtype=np.uint64),
                         key=np.array([rng_seed, domain], dtype=np.uint64))
    return [int(x) for x in g.random_raw(4)]


def numpy_hash32(rng_seed: int, domain: int, trial: int, ident: int) -> int:
    blk = numpy_philox_block(rng_seed, domain, ident, trial >> 3)
    word = blk[(trial & 7) >> 1]
    return (word >> 32) if (trial & 1) else (word & 0xFFFFFFFF)


def numpy_hash32_table(rng_seed: int, domain: int, n_trials: int, n_ids: int) -> np.ndarray:
    """[n_trials, n_ids] table of 32-bit hashes from numpy's Philox."""
    out = np.zeros((n_trials, n_ids), dtype=np.uint64)
    for ident in range(n_ids):
        for g in range((n_trials + 7) // 8):
            blk = numpy_philox_block(rng_seed, domain, ident, g)
            for j in range(8):
                t = 8 * g + j
                if t >= n_trials:
                    break
                word = blk[j >> 1]
                out[t, ident] = (word >> 32) if (j & 1) else (word & 0xFFFFFFFF)
    return out


def bfs_distance(n: int, src: np.ndarray, dst: np.ndarray, seeds) -> np.ndarray:
    """Arcs on a shortest path from `seeds` to each node over arcs src->dst
    (-1 when unreachable), by scipy's unweighted shortest paths from an extra
    super-source."""
    seeds = np.unique(np.asarray(seeds, dtype=np.int64))
    if seeds.size == 0:
        return np.full(n, -1, dtype=np.int64)
    s = np.concatenate([np.asarray(src, dtype=np.int64), np.full(seeds.size, n)])
    d = np.concatenate([np.asarray(dst, dtype=np.int64), seeds])
    mat = sp.csr_matrix((np.ones(s.size, dtype=np.float64), (s, d)), shape=(n + 1, n + 1))
    dist = csg.shortest_path(mat, directed=True, unweighted=True, indices=n)[:n]
    return np.where(np.isinf(dist), -1, dist - 1).astype(np.int64)


def reachable(n: int, src: np.ndarray, dst: np.ndarray, seeds) -> np.ndarray:
    """Boolean mask of nodes reachable from `seeds` over arcs src->dst,
    by scipy's breadth-first search on a graph with one extra super-source."""
    seeds = np.unique(np.asarray(seeds, dtype=np.int64))
    if seeds.size == 0:
        return np.zeros(n, dtype=bool)
    s = np.concatenate([np.asarray(src, dtype=np.int64), np.full(seeds.size, n)])
    d = np.concatenate([np.asarray(dst, dtype=np.int64), seeds])
    mat = sp.csr_matrix((np.ones(s.size, dtype=np.int8), (s, d)), shape=(n + 1, n + 1))
    order = csg.breadth_first_order(mat, n, directed=True, return_predecessors=False)
    mask = np.zeros(n + 1, dtype=bool)
    mask[order] = True
    return mask[:n]


def p_eff(thr: int) -> Fraction:
    return Fraction(1) if thr == 0xFFFFFFFF else Fraction(int(thr), TWO32)


def brute_ic(n: int, src, dst, thr, seeds):
    """Exact IC spread by enumerating all 2^m live-arc subsets (live-edge
    view): returns (sigma, pi[v], distribution of |A|) as Fractions."""
    m = len(src)
    ps = [p_eff(int(t)) for t in thr]
    sigma = Fraction(0)
    pi = [Fraction(0)] * n
    dist: dict[int, Fraction] = {}
    src = list(map(int, src))
    dst = list(map(int, dst))
    for live in itertools.product((0, 1), repeat=m):
        pr = Fraction(1)
        for e in range(m):
            pr *= ps[e] if live[e] else (1 - ps[e])
            if pr == 0:
                break
        if pr == 0:
            continue
        adj = [[] for _ in range(n)]
        for e in range(m):
            if live[e]:
                adj[src[e]].append(dst[e])
        act = set(int(s) for s in seeds)
        stack = list(act)
        while stack:
            u = stack.pop()
            for v in adj[u]:
                if v not in act:
                    act.add(v)
                    stack.append(v)
        sigma += pr * len(act)
        for v in act:
            pi[v] += pr
        dist[len(act)] = dist.get(len(act), Fraction(0)) + pr
    return sigma, pi, dist


def lt_fixpoint(n: int, src, dst, w64, seeds, h) -> set:
    """Deterministic LT outcome for fixed threshold hashes h[v]: the least set
    containing the seeds closed under "v joins when its active in-weight
    exceeds h[v]", found by repeated single-node updates."""
    act = set(int(s) for s in seeds)
    changed = True
    while changed:
        changed = False
        for v in range(n):
            if v in act:
                continue
            tot = sum(int(w64[e]) for e in range(len(src)) if int(dst[e]) == v and int(src[e]) in act)
            if tot > h[v]:
                act.add(v)
                changed = True
    return act


def lt_sync_levels(n: int, src, dst, w64, seeds, h) -> list:
    """Synchronous LT steps for fixed threshold hashes h[v] (Section 2: a node
    joins at step s when the in-weight of the nodes active after step s - 1
    exceeds its threshold): the step at which each node joins, 0 for the
    seeds, -1 for nodes that never join."""
    level = [-1] * n
    for s in seeds:
        level[int(s)] = 0
    step = 0
    while True:
        step += 1
        joins = []
        for v in range(n):
            if level[v] >= 0:
                continue
            tot = sum(int(w64[e]) for e in range(len(src))
                      if int(dst[e]) == v and 0 <= level[int(src[e])] < step)
            if tot > h[v]:
                joins.append(v)
        if not joins:
            return level
        for v in joins:
            level[v] = step


def brute_lt_thresholds(n: int, src, dst, w64, seeds):
    """Exact LT spread by enumerating, per node, the intervals of its 32-bit
    threshold hash between consecutive distinct subset sums of its in-weights
    (the outcome is constant on each interval)."""
    cuts = []
    for v in range(n):
        ins = [int(w64[e]) for e in range(len(src)) if int(dst[e]) == v]
        sums = set()
        for r in range(len(ins) + 1):
            for comb in itertools.combinations(range(len(ins)), r):
                sums.add(sum(ins[i] for i in comb))
        # h ranges over [0, 2^32); "sum > h" flips at h = sum
        pts = sorted(x for x in sums if 0 < x <= TWO32)
        edges = [0] + pts + [TWO32]
        edges = sorted(set(edges))
        cuts.append([(edges[i], edges[i + 1]) for i in range(len(edges) - 1)])
    sigma = Fraction(0)
    pi = [Fraction(0)] * n
    for choice in itertools.product(*cuts):
        pr = Fraction(1)
        h = []
        for (lo, hi) in choice:
            pr *= Fraction(hi - lo, TWO32)
            h.append(lo)
        act = lt_fixpoint(n, src, dst, w64, seeds, h)
        sigma += pr * len(act)
        for v in act:
            pi[v] += pr
    return sigma, pi


def brute_lt_live_edge(n: int, src, dst, w64, seeds):
    """Exact LT spread through the live-edge equivalence of Kempe, Kleinberg
    and Tardos: each node keeps at most one in-arc, arc e with probability
    w_e / 2^32, none with the remaining probability; the active set is the
    set reachable from the seeds over kept arcs."""
    options = []
    for v in range(n):
        ins = [e for e in range(len(src)) if int(dst[e]) == v]
        opts = [(e, Fraction(int(w64[e]), TWO32)) for e in ins]
        rest = 1 - sum((p for _, p in opts), Fraction(0))
        opts.append((None, rest))
        options.append(opts)
    sigma = Fraction(0)
    pi = [Fraction(0)] * n
    for choice in itertools.product(*options):
        pr = Fraction(1)
        kept = []
        for (e, p) in choice:
            pr *= p
            if e is not None:
                kept.append(e)
        if pr == 0:
            continue
        adj = [[] for _ in range(n)]
        for e in kept:
            adj[int(src[e])].append(int(dst[e]))
        act = set(int(s) for s in seeds)
        stack = list(act)
        while stack:
            u = stack.pop()
            for v in adj[u]:
                if v not in act:
                    act.add(v)
                    stack.append(v)
        sigma += pr * len(act)
        for v in act:
            pi[v] += pr
    return sigma, pi


def csr_from_arcs(n: int, src, dst, param=None):
    """Stable CSR (rows in arc order) plus the permutation applied to arcs."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    order = np.argsort(src, kind="stable")
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=offsets[1:])
    out = [offsets, dst[order].astype(np.uint32)]
    if param is not None:
        out.append(np.asarray(param)[order])
    return out
