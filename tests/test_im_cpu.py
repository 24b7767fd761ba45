"""CELF and greedy on the oracle's Monte Carlo (CPU): with common random
numbers the IC estimate is a coverage function, hence exactly monotone
submodular, so lazy greedy must return the greedy picks and greedy must reach
(1 - 1/e) of the best k-set of the same estimate (Nemhauser, Wolsey and
Fisher 1978; paper Section 2, "Influence Maximization")."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2404_17059_amd import im
from tests.pins import csr_from_arcs


def random_ic(seed, n=9, m=20):
    rng = np.random.default_rng(seed)
    arcs = set()
    while len(arcs) < m:
        u, v = (int(x) for x in rng.integers(0, n, size=2))
        if u != v:
            arcs.add((u, v))
    arcs = sorted(arcs)
    p = rng.uniform(0.1, 0.7, size=len(arcs))
    offsets, indices, p = csr_from_arcs(n, [a for a, _ in arcs], [b for _, b in arcs], p)
    return n, offsets, indices, oracle.encode("ic", p)


def evaluator(n, offsets, indices, thr, R, rng_seed):
    def sigma_of(base, extra):
        out = np.zeros(len(extra), dtype=np.int64)
        for i, v in enumerate(extra):
            seeds = np.array(sorted(set(base) | {int(v)}), dtype=np.uint32)
            r = oracle.simulate("ic", n, offsets, indices, thr, seeds, R, rng_seed, want_node_counts=False)
            out[i] = int(np.asarray(r["trial_counts"]).sum())
        return out
    return sigma_of


@pytest.mark.parametrize("gseed", [1, 2, 3])
def test_celf_equals_greedy_and_reaches_the_greedy_bound(gseed):
    n, off, idx, thr = random_ic(gseed)
    R, rs, k = 400, 17, 3
    ev = evaluator(n, off, idx, thr, R, rs)
    g = im.greedy(ev, k, R, rs, n=n)
    c = im.celf(ev, k, R, rs, n=n, batch=2)
    assert c["seeds"] == g["seeds"] and c["sigma"] == g["sigma"]
    best = max(ev(list(s[:-1]), [s[-1]])[0] for s in itertools.combinations(range(n), k)) / R
    assert g["sigma"] >= (1 - 1 / np.e) * best - 1e-12
    assert c["evaluations"] <= g["evaluations"]
