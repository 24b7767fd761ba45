"""Seeded synthetic inputs for the IC/LT Monte Carlo simulator.

This module is the only code shared by the device path and the CPU oracle.
It draws graphs, seed sets and real-valued per-arc parameters from numpy's
PCG64 streams and holds none of the diffusion arithmetic: no fixed-point
encoding, no hashing, no simulation.  Every array it returns is host memory.

Graph shapes follow the synthetic workloads of the paper's demonstration
(Section 4, "Benchmarks": Erdos-Renyi and small-world graphs, undirected
edges stored as two arcs, the TV / UR / WC edge-weight models) scaled up to
the sizes the GPU path is measured on.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np


@dataclasses.dataclass
class Graph:
    """Directed graph in CSR form: out-neighbours of u are
    indices[offsets[u]:offsets[u+1]] (Section 3, "Data Structures")."""

    n: int
    offsets: np.ndarray  # int64 [n+1]
    indices: np.ndarray  # uint32 [m]

    @property
    def m(self) -> int:
        return int(self.offsets[-1])

    def outdeg(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def indeg(self) -> np.ndarray:
        return np.bincount(self.indices.astype(np.int64), minlength=self.n).astype(np.int64)

    def arc_sources(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int64), self.outdeg())

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.offsets, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.indices, dtype=np.uint32).tobytes())
        return h.hexdigest()


def from_arcs(n: int, src: np.ndarray, dst: np.ndarray, dedupe: bool = True,
              drop_self_loops: bool = True) -> Graph:
    """CSR from an arc list, rows sorted by target id."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if drop_self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    key = src * np.int64(n) + dst
    if dedupe:
        key = np.unique(key)
    else:
        key = np.sort(key, kind="stable")
    src = key // n
    dst = key % n
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=offsets[1:])
    return Graph(n=n, offsets=offsets, indices=dst.astype(np.uint32))


def _targets_excluding_self(rng, src: np.ndarray, n: int) -> np.ndarray:
    """Uniform target in V \\ {src} for every entry of src."""
    t = rng.integers(0, n - 1, size=src.shape[0], dtype=np.int64)
    return t + (t >= src)


def erdos_renyi_directed(n: int, avg_out_degree: float, seed: int) -> Graph:
    """Directed G(n, p) with p = avg_out_degree/(n-1), no self-loops.

    Out-degrees are Binomial(n-1, p); targets are drawn uniformly from
    V minus the source with replacement and duplicate arcs are dropped."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = avg_out_degree / (n - 1)
    deg = rng.binomial(n - 1, p, size=n).astype(np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    dst = _targets_excluding_self(rng, src, n)
    return from_arcs(n, src, dst)


def erdos_renyi_undirected(n: int, p: float, seed: int) -> Graph:
    """Undirected G(n, p): each of the n(n-1)/2 pairs is an edge with
    probability p (edge count Binomial, pairs drawn without repetition);
    both arc directions kept."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pairs = n * (n - 1) // 2
    k = int(rng.binomial(pairs, p))
    idx = np.sort(rng.choice(pairs, size=k, replace=False))
    # pair index -> (a, b), a < b, row-major over the upper triangle
    a = (n - 2 - np.floor(np.sqrt(-8.0 * idx + 4.0 * n * (n - 1) - 7) / 2.0 - 0.5)).astype(np.int64)
    b = (idx + a + 1 - n * (n - 1) // 2 + (n - a) * ((n - a) - 1) // 2).astype(np.int64)
    return from_arcs(n, np.concatenate([a, b]), np.concatenate([b, a]))


def barabasi_albert(n: int, m_attach: int, seed: int) -> Graph:
    """Barabasi-Albert preferential attachment, both arc directions kept.

    Starts from m_attach isolated nodes; the first new node links to all of
    them, every later node to m_attach distinct targets drawn with
    probability proportional to current degree."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = m_attach
    rep = np.empty(2 * m * n, dtype=np.int64)  # node list, one entry per edge end
    rep_len = 0
    src_l = np.empty(m * n, dtype=np.int64)
    dst_l = np.empty(m * n, dtype=np.int64)
    e = 0
    targets = list(range(m))
    for v in range(m, n):
        for t in targets:
            src_l[e] = v
            dst_l[e] = t
            e += 1
        rep[rep_len:rep_len + m] = targets
        rep[rep_len + m:rep_len + 2 * m] = v
        rep_len += 2 * m
        chosen: set[int] = set()
        while len(chosen) < m:
            draws = rep[rng.integers(0, rep_len, size=2 * m)]
            for d in draws.tolist():
                chosen.add(d)
                if len(chosen) == m:
                    break
        targets = list(chosen)
    src = np.concatenate([src_l[:e], dst_l[:e]])
    dst = np.concatenate([dst_l[:e], src_l[:e]])
    return from_arcs(n, src, dst)


def _power_law_weights(n: int, gamma: float, total: float, rng) -> np.ndarray:
    """Chung-Lu expected degrees w_i proportional to (i+1)^(-1/(gamma-1)),
    scaled to sum to `total`, assigned to a random permutation of node ids."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    w *= total / w.sum()
    out = np.empty(n, dtype=np.float64)
    out[rng.permutation(n)] = w
    return out


def chung_lu_directed(n: int, gamma: float, mean_out_degree: float, seed: int) -> Graph:
    """Directed Chung-Lu graph whose out-degree is power law.

    d_u ~ Poisson(w_u) clipped to n-1; targets uniform in V minus u.  Rows
    with d_u >= 1024 draw targets without replacement; shorter rows draw
    with replacement and drop duplicate arcs (a small loss at these
    densities).  In-degrees are then close to Poisson(mean_out_degree)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = _power_law_weights(n, gamma, mean_out_degree * n, rng)
    deg = np.minimum(rng.poisson(w), n - 1).astype(np.int64)
    big = np.nonzero(deg >= 1024)[0]
    small_deg = deg.copy()
    small_deg[big] = 0
    src = np.repeat(np.arange(n, dtype=np.int64), small_deg)
    dst = _targets_excluding_self(rng, src, n)
    srcs = [src]
    dsts = [dst]
    for u in big.tolist():
        t = rng.choice(n - 1, size=int(deg[u]), replace=False).astype(np.int64)
        t += t >= u
        srcs.append(np.full(t.shape[0], u, dtype=np.int64))
        dsts.append(t)
    return from_arcs(n, np.concatenate(srcs), np.concatenate(dsts))


def chung_lu_undirected(n: int, gamma: float, mean_degree: float, seed: int) -> Graph:
    """Undirected Chung-Lu graph, both arc directions kept.

    n*mean_degree/2 endpoint pairs are drawn with probability proportional
    to the power-law weights; self-loops and duplicate edges are dropped."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = _power_law_weights(n, gamma, mean_degree * n, rng)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    n_pairs = int(round(n * mean_degree / 2))
    a = np.minimum(np.searchsorted(cdf, rng.random(n_pairs), side="right"), n - 1)
    b = np.minimum(np.searchsorted(cdf, rng.random(n_pairs), side="right"), n - 1)
    keep = a != b
    a, b = a[keep], b[keep]
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = np.unique(lo * np.int64(n) + hi)
    lo = key // n
    hi = key % n
    return from_arcs(n, np.concatenate([lo, hi]), np.concatenate([hi, lo]))


def random_regular(n: int, d: int, seed: int, max_rounds: int = 10000) -> Graph:
    """Random d-regular simple undirected graph, both arcs kept: one
    configuration-model pairing of the n*d stubs, then every self-loop or
    repeated edge is switched with a random edge (a degree-preserving swap of
    endpoints) until the graph is simple."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    stubs = rng.permutation(np.repeat(np.arange(n, dtype=np.int64), d))
    a, b = stubs[0::2].copy(), stubs[1::2].copy()
    for _ in range(max_rounds):
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        _, first = np.unique(lo * n + hi, return_index=True)
        repeated = np.ones(a.shape[0], dtype=bool)
        repeated[first] = False
        bad = np.flatnonzero((a == b) | repeated)
        if bad.size == 0:
            return from_arcs(n, np.concatenate([lo, hi]), np.concatenate([hi, lo]))
        for i in bad:
            j = int(rng.integers(0, a.shape[0]))
            if rng.random() < 0.5:
                a[i], b[j] = b[j], a[i]
            else:
                a[i], a[j] = a[j], a[i]
    raise RuntimeError("random_regular: switching did not reach a simple graph")


def watts_strogatz(n: int, k: int, p: float, seed: int) -> Graph:
    """Watts-Strogatz ring lattice (k nearest neighbours) with each edge's
    far end rewired with probability p to a uniform node, avoiding
    self-loops and duplicates; both arc directions kept."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = set()
    for j in range(1, k // 2 + 1):
        for u in range(n):
            edges.add((u, (u + j) % n))
    edge_list = sorted(edges)
    present = {(min(a, b), max(a, b)) for a, b in edge_list}
    out = []
    for (u, v) in edge_list:
        if rng.random() < p:
            for _ in range(64):
                w = int(rng.integers(0, n))
                key = (min(u, w), max(u, w))
                if w != u and key not in present:
                    present.discard((min(u, v), max(u, v)))
                    present.add(key)
                    v = w
                    break
        out.append((u, v))
    a = np.array([e[0] for e in out], dtype=np.int64)
    b = np.array([e[1] for e in out], dtype=np.int64)
    return from_arcs(n, np.concatenate([a, b]), np.concatenate([b, a]))


# ---------------------------------------------------------------- parameters

def uniform_p(g: Graph, p: float) -> np.ndarray:
    return np.full(g.m, p, dtype=np.float64)


def weighted_cascade(g: Graph) -> np.ndarray:
    """1/indeg(v) on every arc (u, v): the WC model of Section 4
    ("Benchmarks"); also the standard LT weights."""
    indeg = g.indeg()
    return 1.0 / indeg[g.indices.astype(np.int64)].astype(np.float64)


def trivalency(g: Graph, seed: int) -> np.ndarray:
    """TV model: each arc weight uniform from {0.1, 0.01, 0.001}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.array([0.1, 0.01, 0.001])[rng.integers(0, 3, size=g.m)]


def uniform_random(g: Graph, seed: int) -> np.ndarray:
    """UR model: each arc weight uniform on [0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(g.m)


def random_seeds(n: int, k: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.uint32)


def top_outdeg_seeds(g: Graph, k: int) -> np.ndarray:
    """k nodes of largest out-degree, ties to the smaller id."""
    order = np.lexsort((np.arange(g.n), -g.outdeg()))
    return np.sort(order[:k]).astype(np.uint32)


# ---------------------------------------------------------------- workloads

@dataclasses.dataclass
class Workload:
    name: str
    model: str  # "ic" or "lt"
    graph: Graph
    param: np.ndarray  # float64 per arc, out-CSR order: p (IC) or weight (LT)
    seeds: np.ndarray  # uint32
    n_trials: int
    rng_seed: int


def er_ic_1k(n_trials: int = 1000) -> Workload:
    """IC on directed Erdos-Renyi, n=1,000, mean out-degree 10, p=0.1,
    10 uniform seeds, 1,000 trials."""
    g = erdos_renyi_directed(1000, 10.0, seed=101)
    return Workload("ic_er_n1000_d10_p0.1_s10", "ic", g, uniform_p(g, 0.1),
                    random_seeds(g.n, 10, seed=201), n_trials, 1)


def paper_ic_suite(n_trials: int = 1000) -> list[Workload]:
    """IC benchmark workloads after Section 4 ("Benchmarks"): 100 random
    seeds, 1,000 trials, undirected edges as two arcs, on an Erdos-Renyi graph
    (n = 2,000, p = 0.002), a Watts-Strogatz graph (n = 10,000, k = 10,
    p = 0.007) and, standing in for the SNAP Facebook graph (4,039 nodes,
    88,234 edges, not available here), a Barabasi-Albert graph with 4,039
    nodes and m = 22; each with trivalency (TV), uniformly random (UR) and
    weighted-cascade (WC) arc probabilities."""
    graphs = [("er", erdos_renyi_undirected(2000, 0.002, seed=104)),
              ("ws", watts_strogatz(10000, 10, 0.007, seed=107)),
              ("ba_fb", barabasi_albert(4039, 22, seed=108))]
    out = []
    for gi, (gname, g) in enumerate(graphs):
        params = {"tv": trivalency(g, seed=300 + gi), "ur": uniform_random(g, seed=310 + gi), "wc": weighted_cascade(g)}
        seeds = random_seeds(g.n, 100, seed=320 + gi)
        for ename, par in params.items():
            out.append(Workload(f"ic_{gname}_{ename}_n{g.n}_s100", "ic", g, par, seeds, n_trials, 20 + gi))
    return out


def ba_ic_100k(n_trials: int = 10000, n: int = 100_000) -> Workload:
    """IC on Barabasi-Albert n=100,000, m=5 (both arcs), p=0.01, 50 uniform
    seeds, 10,000 trials."""
    g = barabasi_albert(n, 5, seed=102)
    return Workload(f"ic_ba_n{n}_m5_p0.01_s50", "ic", g, uniform_p(g, 0.01),
                    random_seeds(g.n, 50, seed=202), n_trials, 2)


def chung_lu_lt_1m(n_trials: int = 1000, n: int = 1_000_000) -> Workload:
    """LT on directed Chung-Lu n=1,000,000, out-degree exponent 2.1, mean
    out-degree 16, weights 1/indeg(v), 100 top-out-degree seeds, 1,000
    trials."""
    g = chung_lu_directed(n, 2.1, 16.0, seed=103)
    return Workload(f"lt_chunglu_n{n}_g2.1_d16_top100", "lt", g,
                    weighted_cascade(g), top_outdeg_seeds(g, 100), n_trials, 3)


def batch_items(n_items: int = 64, n_trials: int = 2000, n_lo: int = 1000,
                n_hi: int = 200_000, seed: int = 104) -> list[Workload]:
    """Uneven batch: n log-uniform in [n_lo, n_hi]; graphs alternate
    Erdos-Renyi (mean degree 8) and Barabasi-Albert (m=4); models alternate
    in pairs between IC with WC weights and LT with 1/indeg weights; 20
    uniform seeds each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = np.round(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=n_items))).astype(np.int64)
    items = []
    for i, n in enumerate(ns.tolist()):
        gs = 1000 + i
        g = erdos_renyi_directed(n, 8.0, gs) if i % 2 == 0 else barabasi_albert(n, 4, gs)
        model = "ic" if (i // 2) % 2 == 0 else "lt"
        items.append(Workload(f"batch{i}_{'er' if i % 2 == 0 else 'ba'}_{model}_n{n}", model, g,
                              weighted_cascade(g), random_seeds(n, 20, 2000 + i),
                              n_trials, 4000 + i))
    return items


def chung_lu_wc_200k(n: int = 200_000) -> tuple[Graph, np.ndarray]:
    """IC weighted-cascade graph for influence maximisation: undirected
    Chung-Lu n=200,000, mean degree 10, exponent 2.3."""
    g = chung_lu_undirected(n, 2.3, 10.0, seed=105)
    return g, weighted_cascade(g)
