"""IC pull side and the push / pull switch of the grid shape, through the C
ABI: forced push, forced pull and the automatic rule (at several switch
points) must give identical per-trial active sets, equal to the oracle's
(the final set of a trial is reachability over its live arcs, whichever side
draws an arc's coin, since both key it by the arc's out-CSR id)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import pins

pytestmark = pytest.mark.gpu

PUSH, PULL = 1, 2


@pytest.fixture(scope="module")
def ims():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2404_17059_amd as m
    return m


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def variants(ims):
    """(label, opts): grid shape with push only, pull only, the rule at its
    default switch points and at ones that pull early / late."""
    mk = lambda **kw: ims.Opts(shape=2, **kw)  # noqa: E731
    return [("push", mk(ic_direction=PUSH)), ("pull", mk(ic_direction=PULL)), ("auto", mk()),
            ("auto-eager", mk(ic_alpha=1e6, ic_beta=1e6)), ("auto-lazy", mk(ic_alpha=0.05, ic_beta=0.5))]


def check_all(ims, g, param, seeds, T, rs, oracle_trials="all", label=""):
    """Every variant's bits equal each other and the oracle; returns the
    per-level directions of every variant."""
    say(f"[ic-pull] {label} n={g.n} m={g.m} T={T} seeds={len(seeds)} rng={rs}")
    G = ims.Graph(g.n, g.offsets, g.indices, "ic", param)
    ref_bits = None
    dirs = {}
    for name, opts in variants(ims):
        r = ims.simulate(G, seeds, T, rs, want_bits=True, opts=opts)
        bits = r["active_bits"].cpu().numpy().view(np.uint64)
        dirs[name] = G.level_directions()
        if ref_bits is None:
            ref_bits, ref_tc, ref_nc, ref_total = bits, r["trial_counts"].cpu().numpy(), r["node_counts"].cpu().numpy(), r["total"]
        else:
            assert (bits == ref_bits).all(), name
            assert (r["trial_counts"].cpu().numpy() == ref_tc).all(), name
            assert (r["node_counts"].cpu().numpy() == ref_nc).all(), name
            assert r["total"] == ref_total, name
    assert (dirs["push"] == PUSH).all() and (dirs["pull"] == PULL).all()
    enc = oracle.encode("ic", param) if np.asarray(param).dtype == np.float64 else param
    if oracle_trials == "all":
        o = oracle.simulate("ic", g.n, g.offsets, g.indices, enc, seeds, T, rs, threads=8)
        assert (ref_bits == o["active_bits"]).all()
        assert ref_total == o["total"]
    else:
        for t0 in oracle_trials:
            cnt = min(64, T - t0)
            o = oracle.simulate("ic", g.n, g.offsets, g.indices, enc, seeds, cnt, rs, t_begin=t0, threads=8)
            assert (ref_bits[t0 // 64] == o["active_bits"][0]).all(), t0
    G.close()
    return dirs


@pytest.mark.parametrize("T", [1, 63, 65, 200, 1000])
def test_random_graphs_every_direction(ims, T):
    rng = np.random.default_rng(50 + T)
    n = 400
    src = rng.integers(0, n, size=4000)
    dst = rng.integers(0, n, size=4000)  # self-loops and repeated arcs kept
    off, idx = pins.csr_from_arcs(n, src, dst)
    g = synth.Graph(n=n, offsets=off, indices=idx)
    param = rng.choice([0.0, 0.02, 0.1, 0.3, 1.0], size=idx.shape[0])
    seeds = np.array([3, 9, 3, 399, 0], dtype=np.uint32)
    check_all(ims, g, param, seeds, T, 700 + T, label="random")


@pytest.mark.parametrize("case", range(9))
def test_paper_stand_ins_every_direction(ims, case):
    w = synth.paper_ic_suite()[case]
    dirs = check_all(ims, w.graph, w.param, w.seeds, w.n_trials, w.rng_seed, label=w.name)
    if w.name.startswith("ic_ba_fb_ur"):
        # hubs, p averaging 1/2: the frontier's arcs dwarf what is left to pull
        assert (dirs["auto"] == PULL).any()


def test_er_ic_1k_every_direction(ims):
    w = synth.er_ic_1k()
    check_all(ims, w.graph, w.param, w.seeds, w.n_trials, w.rng_seed, label=w.name)


def test_ba_ic_100k_grid_every_direction(ims):
    """The 100k-node BA workload (10,000 trials) on the grid shape; the rule
    keeps its sparse frontiers on the push side."""
    w = synth.ba_ic_100k()
    dirs = check_all(ims, w.graph, w.param, w.seeds, w.n_trials, w.rng_seed,
                     oracle_trials=[0, 64 * 77, w.n_trials - 16], label=w.name)
    assert (dirs["auto"] == PUSH).all()


def test_edge_cases_every_direction(ims):
    g = synth.erdos_renyi_directed(300, 4.0, seed=61)
    p = synth.uniform_p(g, 0.25)
    check_all(ims, g, p, np.zeros(0, dtype=np.uint32), 100, 1, label="empty seeds")
    check_all(ims, g, p, np.arange(g.n, dtype=np.uint32), 70, 2, label="all seeds")
    iso = np.nonzero(g.outdeg() == 0)[0][:2].astype(np.uint32)
    check_all(ims, g, p, iso, 130, 3, label="isolated seeds")
    for q in (0.0, 1.0):  # no in-arcs on the pull side at all / certain arcs
        check_all(ims, g, synth.uniform_p(g, q), [1, 2, 3], 100, 4, label=f"p={q}")


def test_repeated_runs_alternating_directions_start_clean(ims):
    """Path 0 -> ... -> K-1 with p = 1: runs from node 0 and from node K-3
    alternate push and pull on one handle and must not see each other's
    frontier masks or level counters."""
    for K in (3, 4, 9, 17, 33):
        src = np.arange(K - 1)
        off, idx = pins.csr_from_arcs(K, src, src + 1)
        G = ims.Graph(K, off, idx, "ic", np.ones(K - 1))
        for rep in range(2):
            for d in (PUSH, PULL, 0):
                opts = ims.Opts(shape=2, ic_direction=d)
                assert ims.simulate(G, [0], 64, 11, opts=opts)["total"] == K * 64, (K, rep, d)
                assert ims.simulate(G, [K - 3], 64, 12, opts=opts)["total"] == 3 * 64, (K, rep, d)
        G.close()


def word_local_variants(ims):
    mk = lambda **kw: ims.Opts(shape=1, **kw)  # noqa: E731
    return [("push", mk(ic_direction=PUSH)), ("pull", mk(ic_direction=PULL)), ("auto", mk()),
            ("auto-eager", mk(ic_alpha=1e6, ic_beta=1e6))]


@pytest.mark.parametrize("case", ["ic_ba_fb_tv", "ic_ws_ur", "ic_er_ur", "ba_wc_20k"])
def test_word_local_every_direction(ims, case):
    """Word-local tasks (one workgroup per 64-trial word with active bits, and
    the counts-only slot tasks of 4 to 16 trials) with every direction: identical to
    the oracle.  The BA graph has in-degrees above 64 (wavefront-wide
    pulls)."""
    if case == "ba_wc_20k":
        g = synth.barabasi_albert(20000, 4, seed=71)
        param, seeds, T, rs = synth.weighted_cascade(g), synth.random_seeds(g.n, 20, 72), 500, 73
        assert int(np.bincount(g.indices, minlength=g.n).max()) > 64
    else:
        w = [x for x in synth.paper_ic_suite() if x.name.startswith(case + "_")][0]
        g, param, seeds, T, rs = w.graph, w.param, w.seeds, w.n_trials, w.rng_seed
    say(f"[ic-pull] word-local {case} n={g.n} m={g.m} T={T}")
    G = ims.Graph(g.n, g.offsets, g.indices, "ic", param)
    o = oracle.simulate("ic", g.n, g.offsets, g.indices, oracle.encode("ic", param), seeds, T, rs, threads=8)
    for name, opts in word_local_variants(ims):
        r = ims.simulate(G, seeds, T, rs, want_bits=True, opts=opts)
        assert (r["active_bits"].cpu().numpy().view(np.uint64) == o["active_bits"]).all(), name
        c = ims.simulate(G, seeds, T, rs, want_bits=False, opts=opts)  # slot tasks
        assert c["total"] == o["total"], name
        assert (c["trial_counts"].cpu().numpy().view(np.uint32) == o["trial_counts"]).all(), name
        assert (c["node_counts"].cpu().numpy().view(np.uint32) == o["node_counts"]).all(), name
    # per-level counts (BFS distances) do not depend on the direction either
    lv = ims.simulate_levels(G, seeds, T, rs, max_levels=4096)
    o_levels = oracle.simulate("ic", g.n, g.offsets, g.indices, oracle.encode("ic", param), seeds, T, rs,
                               threads=8, want_levels=True, want_bits=False)["levels"]
    assert not lv["truncated"]
    for lev in range(lv["level_counts"].shape[0]):
        assert (lv["level_counts"][lev] == (o_levels == lev).sum(axis=1)).all(), lev
    G.close()


def test_sets_and_marginal_sets_every_direction(ims):
    g = synth.barabasi_albert(20000, 4, seed=81)
    param = synth.weighted_cascade(g)
    deg = g.outdeg()
    hubs = np.argsort(-deg, kind="stable")[:30].astype(np.uint32)
    rng = np.random.default_rng(82)
    sets = [[int(h)] for h in hubs[:6]] + [list(hubs), list(rng.choice(g.n, 40, replace=False)), []]
    G = ims.Graph(g.n, g.offsets, g.indices, "ic", param)
    T, rs = 700, 83
    ref = None
    for name, opts in word_local_variants(ims):
        r = ims.simulate_sets(G, sets, T, rs, want_node_counts=True, opts=opts)
        if ref is None:
            ref = r
        else:
            assert (r["totals"] == ref["totals"]).all(), name
            assert (r["node_counts"] == ref["node_counts"]).all(), name
    enc = oracle.encode("ic", param)
    for k in (0, 6):
        o = oracle.simulate("ic", g.n, g.offsets, g.indices, enc, sets[k], T, rs, threads=8, want_bits=False)
        assert ref["totals"][k] == o["total"]
        assert (ref["node_counts"][k] == o["node_counts"]).all()
    # marginal sets on top of the run of {hub 0}
    base = ims.simulate(G, [int(hubs[0])], T, rs, want_bits=True)
    mref = None
    for name, opts in word_local_variants(ims):
        m = ims.simulate_sets_from(G, base["active_bits"], [[int(h)] for h in hubs[1:8]], T, rs,
                                   want_node_counts=True, opts=opts)
        if mref is None:
            mref = m
        else:
            assert (m["new_totals"] == mref["new_totals"]).all(), name
            assert (m["node_counts"] == mref["node_counts"]).all(), name
    full = ims.simulate_sets(G, [[int(hubs[0]), int(h)] for h in hubs[1:8]], T, rs)
    assert (mref["new_totals"] + base["total"] == full["totals"]).all()
    G.close()


def test_batch_switch_points_leave_results_unchanged(ims):
    import torch
    ws = synth.batch_items(n_items=6, n_trials=300, n_hi=20000)
    items = [(ims.Graph(w.graph.n, w.graph.offsets, w.graph.indices, w.model, w.param), w.seeds, w.n_trials,
              w.rng_seed) for w in ws]
    ref = None
    for alpha in (1e-9, 0.0, 1e6):
        for split in (1, 8):
            B = ims.Batch(items, tuning=(2, 0, split, alpha, 0.0))
            B.launch()
            torch.cuda.synchronize()
            res = B.results()
            B.close()
            if ref is None:
                ref = res
                for (w, r) in zip(ws, res):
                    o = oracle.simulate(w.model, w.graph.n, w.graph.offsets, w.graph.indices,
                                        oracle.encode(w.model, w.param), w.seeds, w.n_trials, w.rng_seed,
                                        threads=8, want_bits=False)
                    assert r["total"] == o["total"]
                    assert (r["node_counts"] == o["node_counts"]).all()
            else:
                for a, b in zip(res, ref):
                    assert a["total"] == b["total"], (alpha, split)
                    assert (a["trial_counts"] == b["trial_counts"]).all(), (alpha, split)
                    assert (a["node_counts"] == b["node_counts"]).all(), (alpha, split)
    for it in items:
        it[0].close()
