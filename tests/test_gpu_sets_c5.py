"""Many-sets and marginal-sets forms on the 200k-node weighted-cascade
Chung-Lu graph of the influence-maximisation workload (the forms CELF, the
estimator's training data and the guided greedy use there), against the
oracle set by set: totals and per-node counts over all 1,000 trials.  The
top-50-degree set puts more than 64 frontier nodes with over 512 out-arcs
into one step, so the word-local tasks take the branch where a wavefront
walks such a node alone (counted in the run's status word 3)."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ims():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2404_17059_amd as m
    return m


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def c5():
    g, param = synth.chung_lu_wc_200k()
    deg = g.outdeg()
    order = np.argsort(-deg, kind="stable")
    rng = np.random.default_rng(91)
    top50 = order[:50].tolist()
    sets = [top50,                                   # 50 largest hubs together
            [int(order[0])], [int(order[1])],        # single hubs
            [int(x) for x in rng.choice(g.n, 25, replace=False)],
            [int(x) for x in rng.choice(g.n, 1, replace=False)],
            order[50:90].tolist(),
            [int(x) for x in order[:10]] + [int(x) for x in rng.choice(g.n, 10, replace=False)],
            []]
    return g, param, sets


def test_sets_on_the_200k_graph_match_the_oracle(ims, c5):
    g, param, sets = c5
    big = int((g.outdeg() > 512).sum())
    say(f"[sets-c5] n={g.n} m={g.m} nodes with >512 out-arcs: {big}")
    assert big > 64
    G = ims.Graph(g.n, g.offsets, g.indices, "ic", param)
    T, rs = 1000, 5
    # push only: every step walks out-arcs, so the dense second step meets
    # more than 64 nodes with over 512 out-arcs
    r = ims.simulate_sets(G, sets, T, rs, want_node_counts=True, opts=ims.Opts(ic_direction=1))
    counters = G.last_counters()
    say(f"[sets-c5] status words {counters.tolist()}")
    assert counters[1] == 0
    assert counters[3] > 0, "no step handed more than 64 large nodes to single wavefronts"
    # the automatic direction and pull only give the same
    for d in (0, 2):
        r2 = ims.simulate_sets(G, sets, T, rs, want_node_counts=True, opts=ims.Opts(ic_direction=d))
        assert (r2["totals"] == r["totals"]).all(), d
        assert (r2["node_counts"] == r["node_counts"]).all(), d
    enc = oracle.encode("ic", param)
    for k, s in enumerate(sets):
        o = oracle.simulate("ic", g.n, g.offsets, g.indices, enc, s, T, rs, threads=16, want_bits=False)
        assert r["totals"][k] == o["total"], k
        assert (r["node_counts"][k] == o["node_counts"]).all(), k
    G.close()


def test_marginal_sets_on_the_200k_graph_match_the_oracle(ims, c5):
    g, param, sets = c5
    G = ims.Graph(g.n, g.offsets, g.indices, "ic", param)
    T, rs = 1000, 6
    base_set = sets[0][:25]
    base = ims.simulate(G, base_set, T, rs, want_bits=True)
    adds = [sets[0][25:], [sets[5][0]], sets[3], []]
    m = ims.simulate_sets_from(G, base["active_bits"], adds, T, rs, want_node_counts=True)
    enc = oracle.encode("ic", param)
    ob = oracle.simulate("ic", g.n, g.offsets, g.indices, enc, base_set, T, rs, threads=16, want_bits=False)
    assert base["total"] == ob["total"]
    for k, x in enumerate(adds):
        o = oracle.simulate("ic", g.n, g.offsets, g.indices, enc, base_set + list(x), T, rs, threads=16, want_bits=False)
        assert base["total"] + int(m["new_totals"][k]) == o["total"], k
        assert (m["node_counts"][k].astype(np.int64) + ob["node_counts"] == o["node_counts"]).all(), k
    G.close()
