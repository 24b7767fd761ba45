"""Bit-exact parity of the HIP simulator (through the C ABI) with the CPU
oracle: every trial's final active set, per-trial counts, per-node counts and
the total must be identical."""
import sys

import functools

import numpy as np
import pytest

import oracle
import synth
from tests import pins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ims():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2404_17059_amd as m
    return m


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_both(ims, model, n, off, idx, param, seeds, T, rs, t_sample=None, opts=None, threads=8):
    """GPU run over all T trials vs the oracle over all (or sampled) trials."""
    say(f"[parity] model={model} n={n} m={idx.shape[0]} T={T} seeds={len(seeds)} rng={rs}")
    G = ims.Graph(n, off, idx, model, param)
    got = ims.simulate(G, seeds, T, rs, want_bits=True, opts=opts)
    bits = got["active_bits"].cpu().numpy().view(np.uint64)
    tc = got["trial_counts"].cpu().numpy().view(np.uint32)
    nc = got["node_counts"].cpu().numpy().view(np.uint32)
    # the same run returning counts only (the word-local shape then runs
    # slot tasks of 4 to 16 trials that add their own counts)
    cnt_only = ims.simulate(G, seeds, T, rs, want_bits=False, opts=opts)
    assert cnt_only["total"] == got["total"]
    assert (cnt_only["trial_counts"].cpu().numpy().view(np.uint32) == tc).all()
    assert (cnt_only["node_counts"].cpu().numpy().view(np.uint32) == nc).all()
    enc = oracle.encode(model, param) if np.asarray(param).dtype == np.float64 else param
    if t_sample is None:
        ref = oracle.simulate(model, n, off, idx, enc, seeds, T, rs, threads=threads)
        assert (tc == ref["trial_counts"]).all()
        assert (nc == ref["node_counts"]).all()
        assert got["total"] == ref["total"]
        assert (bits == ref["active_bits"]).all()
    else:
        for t0 in t_sample:  # 64-trial words, compared bit for bit
            cnt = min(64, T - t0)
            ref = oracle.simulate(model, n, off, idx, enc, seeds, cnt, rs, t_begin=t0, threads=8)
            w = t0 // 64
            assert (bits[w] == ref["active_bits"][0]).all(), t0
            assert (tc[t0:t0 + cnt] == ref["trial_counts"]).all(), t0
        # properties over every trial
        assert int(tc.astype(np.int64).sum()) == got["total"] == int(nc.astype(np.int64).sum())
        pop = np.zeros(T, dtype=np.int64)
    G.close()
    return got, bits


def test_device_hash_matches_numpy_philox(ims):
    rng = np.random.default_rng(3)
    trials = rng.integers(0, 10**6, size=300)
    ids = rng.integers(0, 2**32, size=300).astype(np.uint64)
    ids[:8] = 0
    trials[:8] = np.arange(8)
    # counters above 2^32 (arc ids of graphs with more arcs) and the largest
    ids[8:16] = rng.integers(2**32, 2**63, size=8).astype(np.uint64)
    ids[16] = 2**64 - 1
    for dom in (1, 2):
        got = ims.debug_hash(12345, dom, trials, ids)
        exp = [pins.numpy_hash32(12345, dom, int(t), int(i)) for t, i in zip(trials, ids)]
        assert got.tolist() == exp


@pytest.mark.parametrize("model", ["ic", "lt"])
@pytest.mark.parametrize("T", [1, 63, 64, 65, 200, 777])
def test_small_random_graphs(ims, model, T):
    rng = np.random.default_rng(T)
    n = 300
    src = rng.integers(0, n, size=2400)
    dst = rng.integers(0, n, size=2400)  # self-loops and repeated arcs kept
    off, idx = pins.csr_from_arcs(n, src, dst)
    if model == "ic":
        param = rng.choice([0.0, 0.02, 0.1, 0.3, 1.0], size=idx.shape[0])
    else:
        indeg = np.bincount(idx, minlength=n)
        param = rng.choice([1.0, 0.7], size=n)[idx] / indeg[idx]
    seeds = np.array([5, 7, 5, 299, 0], dtype=np.uint32)  # duplicates on purpose
    run_both(ims, model, n, off, idx, param, seeds, T, 1000 + T)


@pytest.mark.parametrize("model", ["ic", "lt"])
def test_edge_cases(ims, model):
    g = synth.erdos_renyi_directed(400, 5.0, seed=3)
    param = synth.uniform_p(g, 0.2) if model == "ic" else synth.weighted_cascade(g)
    # empty seed set
    got, bits = run_both(ims, model, g.n, g.offsets, g.indices, param, np.array([], np.uint32), 100, 1)
    assert got["total"] == 0
    # isolated seed (no out-arcs) plus all nodes as seeds
    deg = g.outdeg()
    iso = np.nonzero(deg == 0)[0][:1].astype(np.uint32)
    run_both(ims, model, g.n, g.offsets, g.indices, param, iso, 130, 2)
    got, _ = run_both(ims, model, g.n, g.offsets, g.indices, param, np.arange(g.n, dtype=np.uint32), 70, 3)
    assert got["total"] == g.n * 70


def test_ic_probability_extremes(ims):
    g = synth.erdos_renyi_directed(500, 3.0, seed=4)
    for p in (0.0, 1.0):
        got, bits = run_both(ims, "ic", g.n, g.offsets, g.indices, synth.uniform_p(g, p), [1, 2, 3], 100, 5)
    reach = pins.reachable(g.n, g.arc_sources(), g.indices, [1, 2, 3])
    assert (got["node_counts"].cpu().numpy() == 100 * reach).all()


def test_ic_grid_repeated_runs_start_clean(ims):
    """Runs on one graph handle leave no frontier masks behind, whichever
    level the last step launch ends on: a path 0 -> 1 -> ... -> K-1 with p = 1
    is run from node 0 (K levels), then from node K-3, which must reach the
    last three nodes in every trial."""
    opts = ims.Opts(shape=2, blocks_per_cu=0, alpha=0.0, profile=0)
    for K in range(3, 40):
        src = np.arange(K - 1)
        off, idx = pins.csr_from_arcs(K, src, src + 1)
        G = ims.Graph(K, off, idx, "ic", np.ones(K - 1))
        for rep in range(2):
            r = ims.simulate(G, [0], 64, 11, opts=opts)
            assert r["total"] == K * 64, (K, rep)
        r = ims.simulate(G, [K - 3], 64, 12, opts=opts)
        assert r["total"] == 3 * 64, K
        G.close()


@pytest.mark.parametrize("first_shape", [1, 2])
def test_lt_word_local_runs_after_other_runs(ims, first_shape):
    """LT word-local runs (active bits, per-level counts) on a handle that
    already ran give what they give on a fresh handle."""
    g = synth.erdos_renyi_directed(3000, 6.0, seed=21)
    param = synth.weighted_cascade(g)
    seeds = synth.random_seeds(g.n, 10, 22)
    fresh = ims.Graph(g.n, g.offsets, g.indices, "lt", param)
    ref_bits = ims.simulate(fresh, seeds, 200, 5, want_bits=True, opts=ims.Opts(shape=1, blocks_per_cu=0, alpha=0.0, profile=0))
    ref_lv = ims.simulate_levels(fresh, seeds, 200, 5)
    fresh.close()
    G = ims.Graph(g.n, g.offsets, g.indices, "lt", param)
    ims.simulate(G, seeds, 200, 4, want_bits=True, opts=ims.Opts(shape=first_shape, blocks_per_cu=0, alpha=0.0, profile=0))
    for rep in range(2):
        got = ims.simulate(G, seeds, 200, 5, want_bits=True, opts=ims.Opts(shape=1, blocks_per_cu=0, alpha=0.0, profile=0))
        assert (got["active_bits"].cpu().numpy() == ref_bits["active_bits"].cpu().numpy()).all(), rep
        lv = ims.simulate_levels(G, seeds, 200, 5)
        assert lv["levels_processed"] == ref_lv["levels_processed"]
        assert (lv["level_counts"] == ref_lv["level_counts"]).all(), rep
    G.close()


def test_lt_full_weight_arcs(ims):
    # indegree-1 nodes carry a weight of exactly 2^32 (stored as two pieces)
    n = 200
    src = np.arange(n - 1)
    dst = np.arange(1, n)
    off, idx = pins.csr_from_arcs(n, src, dst)
    got, _ = run_both(ims, "lt", n, off, idx, np.ones(n - 1), [0], 100, 9)
    assert got["total"] == n * 100


def test_er_ic_1k_full(ims):
    w = synth.er_ic_1k()
    run_both(ims, w.model, w.graph.n, w.graph.offsets, w.graph.indices, w.param, w.seeds, w.n_trials, w.rng_seed)


def test_ba_ic_100k_full(ims):
    w = synth.ba_ic_100k()
    run_both(ims, w.model, w.graph.n, w.graph.offsets, w.graph.indices, w.param, w.seeds, w.n_trials, w.rng_seed)


def test_chung_lu_lt_1m_full(ims):
    """The benchmark workload in the benchmark's launch configuration: every
    trial's active set bit for bit against the oracle (the oracle takes about
    a minute on 16 host threads)."""
    import os
    w = synth.chung_lu_lt_1m()
    got, bits = run_both(ims, w.model, w.graph.n, w.graph.offsets, w.graph.indices, w.param, w.seeds,
                         w.n_trials, w.rng_seed, threads=max(1, min(16, len(os.sched_getaffinity(0)))))
    # seeds active in every trial
    nc = got["node_counts"].cpu().numpy()
    assert (nc[w.seeds] == w.n_trials).all()


@pytest.mark.parametrize("model", ["ic", "lt"])
def test_schedule_invariance(ims, model):
    """Word-local and grid-wide shapes, several occupancies: identical bits,
    equal to the oracle."""
    g = synth.barabasi_albert(3000, 3, seed=5)
    param = synth.weighted_cascade(g)
    seeds = synth.random_seeds(g.n, 10, 6)
    G = ims.Graph(g.n, g.offsets, g.indices, model, param)
    outs = []
    for shape in (1, 2):
        for bpc in (1, 3, 0):
            say(f"[parity] schedule model={model} shape={shape} bpc={bpc}")
            opts = ims.Opts(shape=shape, blocks_per_cu=bpc, alpha=0.0, profile=0)
            r = ims.simulate(G, seeds, 300, 4, want_bits=True, opts=opts)
            outs.append(r["active_bits"].cpu().numpy())
    assert all((o == outs[0]).all() for o in outs)
    ref = oracle.simulate(model, g.n, g.offsets, g.indices, oracle.encode(model, param), seeds, 300, 4)
    assert (outs[0].view(np.uint64) == ref["active_bits"]).all()
    G.close()


@pytest.mark.parametrize("model", ["ic", "lt"])
@pytest.mark.parametrize("shape", [1, 2])
def test_both_shapes_on_random_graphs(ims, model, shape):
    rng = np.random.default_rng(40 + shape)
    n = 2000
    src = rng.integers(0, n, size=12000)
    dst = rng.integers(0, n, size=12000)
    off, idx = pins.csr_from_arcs(n, src, dst)
    if model == "ic":
        param = rng.choice([0.0, 0.05, 0.2, 1.0], size=idx.shape[0])
    else:
        indeg = np.bincount(idx, minlength=n)
        param = 1.0 / indeg[idx]
    opts = ims.Opts(shape=shape, blocks_per_cu=0, alpha=0.0, profile=0)
    run_both(ims, model, n, off, idx, param, np.array([3, 9, 27], np.uint32), 333, 17, opts=opts)


@pytest.mark.parametrize("n", [4096, 4097])
@pytest.mark.parametrize("direction", [0, 1, 2])
def test_ic_slot_runs_either_side_of_the_lds_limit(ims, n, direction):
    """Count-only IC word-local runs keep the tasks' masks in LDS on graphs
    of at most 4,096 nodes and in global memory above: both against the
    oracle over every trial, with the push / pull rule (mean arc probability
    above 0.25), push only and pull only."""
    rng = np.random.default_rng(4100 + n + direction)
    m = 6 * n
    src = rng.integers(0, n, size=m)
    dst = rng.integers(0, n, size=m)
    off, idx = pins.csr_from_arcs(n, src, dst)
    param = rng.choice([0.0, 0.05, 0.3, 0.6, 1.0], size=idx.shape[0])
    opts = ims.Opts(shape=1, blocks_per_cu=0, alpha=0.0, profile=0, ic_direction=direction)
    run_both(ims, "ic", n, off, idx, param, np.array([1, 77, n - 1], np.uint32), 1000, 23, opts=opts)


@pytest.mark.parametrize("flags,alpha", [(0, 0.0), (1, 0.0), (8, 0.0), (8, 1.0), (0, 1.0), (0, 1e-9), (4, 0.0), (5, 1.0)])
def test_lt_grid_threshold_paths_and_direction_switch(ims, flags, alpha):
    """LT grid shape with count thresholds, full threshold hashes, hashes drawn
    in the kernel, with and without the equal-in-weights counting form, and
    with the marking direction always on (alpha=1) or always off (alpha
    tiny): identical bits."""
    g = synth.chung_lu_directed(20000, 2.1, 8.0, seed=31)
    param = synth.weighted_cascade(g)
    seeds = synth.top_outdeg_seeds(g, 20)
    opts = ims.Opts(shape=2, blocks_per_cu=0, alpha=alpha, profile=0, test_flags=flags)
    run_both(ims, "lt", g.n, g.offsets, g.indices, param, seeds, 200, 23, opts=opts)


@pytest.mark.parametrize("T,flags", [(300, 0), (400, 8), (600, 0), (832, 0), (832, 8), (900, 1), (1600, 0)])
def test_lt_grid_padded_rows(ims, T, flags):
    """9 to 15 words of trials (alone, or as the last 16-word run): the
    node-major rows are padded to 16 words, and the padding holds no trial;
    every threshold form, bits against the oracle."""
    g = synth.chung_lu_directed(20000, 2.1, 8.0, seed=35)
    param = synth.weighted_cascade(g)
    seeds = synth.top_outdeg_seeds(g, 20)
    opts = ims.Opts(shape=2, blocks_per_cu=0, alpha=0.0, profile=0, test_flags=flags)
    run_both(ims, "lt", g.n, g.offsets, g.indices, param, seeds, T, 31, opts=opts)


@pytest.mark.parametrize("T", [1025, 1500])
def test_lt_grid_count_thresholds_over_several_word_groups(ims, T):
    """Count-threshold table and sweep with more than one group of 16 words,
    the last one partial (W = 17 and 24)."""
    g = synth.chung_lu_directed(20000, 2.1, 8.0, seed=33)
    param = synth.weighted_cascade(g)
    seeds = synth.top_outdeg_seeds(g, 20)
    opts = ims.Opts(shape=2, blocks_per_cu=0, alpha=0.0, profile=0, test_flags=0)
    run_both(ims, "lt", g.n, g.offsets, g.indices, param, seeds, T, 29, opts=opts)


@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_lt_grid_count_thresholds_with_long_rows(ims, alpha):
    """Count-threshold sweeps on a graph where 24 nodes have more than 64
    in-arc pieces (Barabasi-Albert hubs, in-degree up to 280): those batches
    are evaluated by a second launch in every sweep, with marking always off
    or always on."""
    g = synth.barabasi_albert(5000, 4, seed=35)
    assert int(np.bincount(g.indices, minlength=g.n).max()) > 64
    param = synth.weighted_cascade(g)
    seeds = synth.random_seeds(g.n, 10, seed=36)
    opts = ims.Opts(shape=2, blocks_per_cu=0, alpha=alpha, profile=0, test_flags=0)
    run_both(ims, "lt", g.n, g.offsets, g.indices, param, seeds, 300, 31, opts=opts)


@pytest.mark.parametrize("T,alpha", [(1000, 0.0), (1000, 1.0), (64, 1.0)])
def test_lt_grid_trailing_nodes_without_in_arcs(ims, T, alpha):
    """Count-threshold sweeps on a graph whose last 300 of 2,000 nodes have
    no in-arcs, so the last batches hold no in-arc piece and start at the
    end of the in-CSR; marking off, and always on (every sweep after the
    first evaluates stamped batches only)."""
    rng = np.random.default_rng(41)
    n, m = 2000, 16000
    g = synth.from_arcs(n, rng.integers(0, n, m), rng.integers(0, 1700, m))
    indeg = np.bincount(g.indices, minlength=n)
    assert indeg[1700:].sum() == 0 and indeg[:1700].sum() == g.m
    param = synth.weighted_cascade(g)
    seeds = np.array([3, 1750, 1999, 421], np.uint32)
    opts = ims.Opts(shape=2, blocks_per_cu=0, alpha=alpha, profile=0, test_flags=0)
    run_both(ims, "lt", g.n, g.offsets, g.indices, param, seeds, T, 43, opts=opts)


@pytest.mark.parametrize("model", ["ic", "lt"])
def test_sets_equal_single_runs_and_oracle(ims, model):
    """Many seed sets at once (common random numbers) == each set alone."""
    g = synth.barabasi_albert(2000, 3, seed=21)
    param = synth.weighted_cascade(g)
    rng = np.random.default_rng(5)
    sets = [rng.choice(g.n, size=int(rng.integers(0, 6)), replace=True).astype(np.uint32) for _ in range(37)]
    sets[3] = np.array([], np.uint32)
    sets[4] = np.array([7, 7, 7], np.uint32)
    T, rs = 130, 77
    say(f"[parity] sets model={model} n_sets={len(sets)} T={T}")
    G = ims.Graph(g.n, g.offsets, g.indices, model, param)
    got = ims.simulate_sets(G, sets, T, rs, want_node_counts=True)
    enc = oracle.encode(model, param)
    for i, st in enumerate(sets):
        ref = oracle.simulate(model, g.n, g.offsets, g.indices, enc, st, T, rs, want_bits=False)
        assert int(got["totals"][i]) == ref["total"], i
        assert (got["node_counts"][i] == ref["node_counts"]).all(), i
    # a second call on the same handle (slot state reused) gives the same
    again = ims.simulate_sets(G, sets[::-1], T, rs)
    assert (again["totals"] == got["totals"][::-1]).all()
    G.close()


@functools.lru_cache(maxsize=1)
def paper_suite():
    return synth.paper_ic_suite()


@pytest.mark.parametrize("i", range(9))
def test_paper_benchmark_suite_full_parity(ims, i):
    """The Section 4 benchmark stand-ins (ER / WS / BA x TV / UR / WC, 100
    seeds, 1,000 trials): every trial's active set equals the oracle's."""
    w = paper_suite()[i]
    run_both(ims, w.model, w.graph.n, w.graph.offsets, w.graph.indices, w.param, w.seeds, w.n_trials, w.rng_seed)


@pytest.mark.parametrize("case", ["random", "er_ic_1k"])
def test_ic_level_counts_match_oracle_levels(ims, case):
    """Per-trial counts of nodes first active at each level equal the
    histogram of the oracle's activation levels."""
    if case == "random":
        rng = np.random.default_rng(31)
        n = 700
        src = rng.integers(0, n, size=2500)
        dst = rng.integers(0, n, size=2500)
        off, idx = pins.csr_from_arcs(n, src, dst)
        param = rng.choice([0.0, 0.2, 0.5, 1.0], size=idx.shape[0])
        seeds, T, rs = np.array([1, 2, 3, 400], np.uint32), 333, 55
    else:
        w = synth.er_ic_1k()
        n, off, idx, param, seeds, T, rs = w.graph.n, w.graph.offsets, w.graph.indices, w.param, w.seeds, w.n_trials, w.rng_seed
    say(f"[parity] levels case={case} n={n} T={T}")
    G = ims.Graph(n, off, idx, "ic", param)
    got = ims.simulate_levels(G, seeds, T, rs, max_levels=512)
    assert not got["truncated"]
    enc = oracle.encode("ic", param)
    r = oracle.simulate("ic", n, off, idx, enc, seeds, T, rs, want_levels=True, threads=8)
    L = got["level_counts"].shape[0]
    expect = np.zeros((max(L, int(r["levels"].max()) + 1), T), dtype=np.int64)
    for t in range(T):
        lv = r["levels"][t]
        expect[:, t] = np.bincount(lv[lv >= 0], minlength=expect.shape[0])
    np.testing.assert_array_equal(got["level_counts"].astype(np.int64), expect[:L])
    assert expect[L:].sum() == 0
    np.testing.assert_array_equal(got["level_counts"].sum(axis=0), got["trial_counts"])
    assert got["total"] == int(np.asarray(r["trial_counts"]).sum())
    # a short buffer keeps the first levels and reports the truncation
    short = ims.simulate_levels(G, seeds, T, rs, max_levels=3)
    np.testing.assert_array_equal(short["level_counts"], got["level_counts"][:3])
    assert short["truncated"] == (got["levels_processed"] + 1 > 3)


@pytest.mark.parametrize("case", ["random", "ba_hubs"])
def test_lt_level_counts_match_oracle_levels(ims, case):
    """LT with level counts runs synchronous steps: per-trial counts of nodes
    first active at each step equal the histogram of the oracle's levels,
    and the final state equals the oracle's (the in-place runs reach the same
    fixpoint).  ba_hubs has nodes with more than 64 in-arcs."""
    if case == "random":
        rng = np.random.default_rng(37)
        n = 800
        off, idx = pins.csr_from_arcs(n, rng.integers(0, n, size=4000), rng.integers(0, n, size=4000))
        indeg = np.bincount(idx, minlength=n)
        param = rng.choice([1.0, 0.7], size=n)[idx] / np.maximum(indeg[idx], 1)
        seeds, T, rs = np.array([4, 9, 100, 701], np.uint32), 200, 61
    else:
        g = synth.barabasi_albert(3000, 4, seed=38)
        n, off, idx = g.n, g.offsets, g.indices
        param = synth.weighted_cascade(g)
        seeds, T, rs = synth.random_seeds(n, 6, seed=39), 130, 62
    say(f"[parity] lt levels case={case} n={n} T={T}")
    G = ims.Graph(n, off, idx, "lt", param)
    got = ims.simulate_levels(G, seeds, T, rs, max_levels=512)
    assert not got["truncated"]
    enc = oracle.encode("lt", param)
    r = oracle.simulate("lt", n, off, idx, enc, seeds, T, rs, want_levels=True, threads=8)
    L = got["level_counts"].shape[0]
    deepest = int(r["levels"].max())
    assert deepest >= 3
    expect = np.zeros((max(L, deepest + 1), T), dtype=np.int64)
    for t in range(T):
        lv = r["levels"][t]
        expect[:, t] = np.bincount(lv[lv >= 0], minlength=expect.shape[0])
    np.testing.assert_array_equal(got["level_counts"].astype(np.int64), expect[:L])
    assert expect[L:].sum() == 0
    np.testing.assert_array_equal(got["trial_counts"], r["trial_counts"])
    assert got["total"] == r["total"]
    G.close()


@pytest.mark.parametrize("model,shape", [("ic", 0), ("lt", 0), ("lt", 2)])
def test_sets_from_stored_state_equal_full_sets(ims, model, shape):
    """Marginal runs from the active bits of S: new activations of S + X equal
    sigma(S + X) - sigma(S) of full runs, per set and per node, and the oracle
    agrees on one set."""
    g = synth.barabasi_albert(3000, 3, seed=22)
    param = synth.weighted_cascade(g)
    rng = np.random.default_rng(12)
    S = rng.choice(g.n, size=6, replace=False).astype(np.uint32)
    T, rs = 200, 41
    say(f"[parity] sets_from model={model} shape={shape} T={T}")
    G = ims.Graph(g.n, g.offsets, g.indices, model, param)
    base = ims.simulate(G, S, T, rs, want_bits=True, opts=ims.Opts(shape=shape, blocks_per_cu=0, alpha=0.0, profile=0))
    extra = [rng.choice(g.n, size=int(rng.integers(1, 5)), replace=True).astype(np.uint32) for _ in range(40)]
    extra[0] = np.array([], np.uint32)             # nothing added
    extra[1] = S[:2].copy()                        # already seeds
    extra[2] = np.array([7, 7, 7], np.uint32)      # duplicates
    inc = ims.simulate_sets_from(G, base["active_bits"], extra, T, rs, want_node_counts=True)
    full = ims.simulate_sets(G, [np.concatenate([S, x]) for x in extra], T, rs, want_node_counts=True)
    np.testing.assert_array_equal(inc["new_totals"], full["totals"] - base["total"])
    nc_base = base["node_counts"].cpu().numpy().view(np.uint32).astype(np.int64)
    np.testing.assert_array_equal(inc["node_counts"].astype(np.int64), full["node_counts"].astype(np.int64) - nc_base[None, :])
    assert inc["new_totals"][0] == 0 and inc["new_totals"][1] == 0
    enc = oracle.encode(model, param)
    o_s = oracle.simulate(model, g.n, g.offsets, g.indices, enc, S, T, rs, want_bits=False, want_node_counts=False, threads=8)
    o_x = oracle.simulate(model, g.n, g.offsets, g.indices, enc, np.concatenate([S, extra[5]]), T, rs, want_bits=False,
                          want_node_counts=False, threads=8)
    assert inc["new_totals"][5] == o_x["total"] - o_s["total"]
    with pytest.raises(ims.ImsError) as e:
        ims.simulate_sets_from(G, base["active_bits"], [np.array([g.n], np.uint32)], T, rs)
    assert e.value.code == -4


def test_incremental_celf_equals_full_celf(ims):
    from paper_2404_17059_amd import im
    g = synth.barabasi_albert(2000, 3, seed=23)
    param = synth.weighted_cascade(g)
    for model in ("ic", "lt"):
        G = ims.Graph(g.n, g.offsets, g.indices, model, param)
        a = im.celf(G, 5, 300, 13, batch=8, incremental=True)
        b = im.celf(G, 5, 300, 13, batch=8, incremental=False)
        assert a["seeds"] == b["seeds"] and a["sigma"] == b["sigma"], model


def test_celf_equals_greedy_and_oracle_greedy(ims):
    """CELF on sigma with common random numbers returns exactly the plain
    greedy picks (submodular coverage), and the plain greedy equals a greedy
    computed from oracle spreads."""
    from paper_2404_17059_amd import im
    g = synth.random_regular(300, 4, seed=8)
    param = synth.weighted_cascade(g)
    G = ims.Graph(g.n, g.offsets, g.indices, "ic", param)
    R, rs, k = 256, 9, 4
    a = im.celf(G, k, R, rs)
    b = im.greedy(G, k, R, rs)
    assert a["seeds"] == b["seeds"]
    assert a["sigma"] == b["sigma"]
    # oracle greedy
    enc = oracle.encode("ic", param)
    S = []
    for _ in range(k):
        best, best_t = None, -1
        for v in range(g.n):
            if v in S:
                continue
            t = oracle.simulate("ic", g.n, g.offsets, g.indices, enc, S + [v], R, rs, want_bits=False,
                                want_node_counts=False, threads=8)["total"]
            if t > best_t:
                best, best_t = v, t
        S.append(best)
    assert S == a["seeds"]
    assert a["evaluations"] < b["evaluations"]
    G.close()


def _batch_items(ims, count=10, seed=3, unequal_lt=False):
    """Uneven IC/LT items; with unequal_lt every other LT item gets random
    in-weights (sums 0.9 per node) instead of 1/indeg."""
    rng = np.random.default_rng(seed)
    items, specs = [], []
    for i in range(count):
        n = int(rng.integers(300, 4000))
        g = synth.erdos_renyi_directed(n, 6.0, 50 + i) if i % 2 == 0 else synth.barabasi_albert(n, 3, 50 + i)
        model = "ic" if (i // 2) % 2 == 0 else "lt"
        param = synth.weighted_cascade(g)
        if unequal_lt and model == "lt" and i % 4 == 3:
            u = rng.uniform(0.05, 1.0, size=g.m)
            insum = np.bincount(g.indices, weights=u, minlength=g.n)
            param = 0.9 * u / insum[g.indices]
        seeds = synth.random_seeds(n, int(rng.integers(0, 12)), 70 + i)
        T = int(rng.choice([1, 64, 100, 190]))
        G = ims.Graph(g.n, g.offsets, g.indices, model, param)
        items.append((G, seeds, T, 900 + i))
        specs.append((model, g, param, seeds, T, 900 + i))
    return items, specs


def test_batch_equals_single_runs_across_graph_replays(ims):
    """One persistent launch over uneven graphs, IC and LT mixed; the captured
    HIP graph is replayed several times with eager work in between, and every
    replay equals the per-item runs (and the oracle totals)."""
    import torch
    items, specs = _batch_items(ims)
    singles = [ims.simulate(G, sd, T, rs) for (G, sd, T, rs) in items]
    B = ims.Batch(items)
    for rep in range(3):
        say(f"[parity] batch replay {rep}")
        B.launch()
        torch.cuda.synchronize()
        x = torch.randn(1000, device="cuda").sum()  # eager work between replays
        res = B.results()
        for k, (r, s1) in enumerate(zip(res, singles)):
            assert r["total"] == s1["total"], (rep, k)
            assert (r["trial_counts"] == s1["trial_counts"].cpu().numpy().view(np.uint32)).all(), (rep, k)
            assert (r["node_counts"] == s1["node_counts"].cpu().numpy().view(np.uint32)).all(), (rep, k)
    for (model, g, param, sd, T, rs), r in zip(specs, res):
        ref = oracle.simulate(model, g.n, g.offsets, g.indices, oracle.encode(model, param), sd, T, rs, want_bits=False)
        assert r["total"] == ref["total"]
    chosen = B.autotune(repeats=1)
    assert chosen[0] >= 1 and chosen[2] >= 1
    B.launch()
    torch.cuda.synchronize()
    assert [r["total"] for r in B.results()] == [s1["total"] for s1 in singles]
    B.close()
    for it in items:
        it[0].close()


@pytest.mark.parametrize("split", [1, 2, 4, 8, 16, 32, 64])
def test_batch_split_tasks_equal_single_runs(ims, split):
    """Words split into `split` tasks of 64 / split trials each (trial
    counts with ragged last words: parts past the last trial are skipped)
    give the per-item results of whole-word runs, over two replays.  From 8
    on a task's trials lie in one 8-trial group and lanes take whole nodes
    (hubs with more arcs go through the wavefront-wide walk); LT items with
    equal and with unequal in-weights."""
    import torch
    items, specs = _batch_items(ims, count=12, unequal_lt=True)
    singles = [ims.simulate(G, sd, T, rs) for (G, sd, T, rs) in items]
    B = ims.Batch(items, tuning=(2, 0, split))
    for rep in range(2):
        say(f"[parity] batch split {split} replay {rep}")
        B.launch()
        torch.cuda.synchronize()
        for k, (r, s1) in enumerate(zip(B.results(), singles)):
            assert r["total"] == s1["total"], (rep, k)
            assert (r["trial_counts"] == s1["trial_counts"].cpu().numpy().view(np.uint32)).all(), (rep, k)
            assert (r["node_counts"] == s1["node_counts"].cpu().numpy().view(np.uint32)).all(), (rep, k)
    B.close()
    for it in items:
        it[0].close()


def test_batch_lt_push_form_edge_weights(ims):
    """The push form of the 8-trial LT tasks (threshold remainders) on LT
    weights that reach its edge cases: an arc of weight exactly 1 (its
    target's only in-weight: it always joins), arcs of weight 0 (never
    counted), in-weights summing to exactly 1, a node whose in-weights are
    one tiny and one large arc, seeds that point at each other and at
    already-active nodes, a hub with more out-arcs than a wavefront; every
    item equals the oracle over all trials, on launches with 8, then 64, then
    16, then 8 trials per task again (push, pull, push over two 8-trial
    groups, push: remainder words written by earlier tasks on the same slots
    must not leak into later ones)."""
    import torch
    rng = np.random.default_rng(41)
    items, specs = [], []
    # 1: a path with weight-1 arcs and a cycle back (every node joins)
    n = 300
    src = np.arange(n - 1); dst = src + 1
    g = synth.from_arcs(n, np.concatenate([src, [n - 1]]), np.concatenate([dst, [0]]))
    specs.append((g, np.ones(g.m), [0], 200, 11))
    # 2: ER with a third of the arcs at weight 0 and the rest summing to 1
    g = synth.erdos_renyi_directed(800, 5.0, 42)
    u = rng.uniform(0.0, 1.0, size=g.m)
    u[rng.random(g.m) < 0.33] = 0.0
    insum = np.bincount(g.indices, weights=u, minlength=g.n)
    w = np.where(insum[g.indices] > 0, u / np.maximum(insum[g.indices], 1e-300), 0.0)
    specs.append((g, w, synth.random_seeds(g.n, 6, 43), 190, 12))
    # 3: a star hub (out-degree 700) into nodes with one tiny and one large in-arc
    n = 1500
    hub_src = np.zeros(700, dtype=np.int64); hub_dst = np.arange(1, 701)
    side_src = np.arange(701, 1401); side_dst = np.arange(1, 701)
    g = synth.from_arcs(n, np.concatenate([hub_src, side_src]), np.concatenate([hub_dst, side_dst]))
    wt = np.where(np.repeat(np.arange(g.n), np.diff(g.offsets)) == 0, 1e-9, 0.999)
    specs.append((g, wt, [0, 701, 702, 5], 64, 13))
    # 4: BA graph, 1/indeg weights, seeds adjacent to each other
    g = synth.barabasi_albert(2000, 3, 44)
    sd = [int(x) for x in g.indices[g.offsets[0]:g.offsets[0] + 5]] + [0]
    specs.append((g, synth.weighted_cascade(g), sd, 100, 14))
    for g, w, sd, T, rs in specs:
        items.append((ims.Graph(g.n, g.offsets, g.indices, "lt", w), np.asarray(sd, dtype=np.int64), T, rs))
    refs = [oracle.simulate("lt", g.n, g.offsets, g.indices, oracle.encode("lt", w), np.unique(np.asarray(sd)), T, rs)
            for g, w, sd, T, rs in specs]
    for split in (8, 1, 4, 8):
        B = ims.Batch(items, tuning=(2, 0, split))
        for rep in range(2):
            say(f"[parity] LT push-form edge weights, split {split}, replay {rep}")
            B.launch()
            torch.cuda.synchronize()
            for k, (r, ref) in enumerate(zip(B.results(), refs)):
                assert r["total"] == ref["total"], (split, rep, k)
                assert (r["trial_counts"] == ref["trial_counts"]).all(), (split, rep, k)
                assert (r["node_counts"] == ref["node_counts"]).all(), (split, rep, k)
        B.close()
    for it in items:
        it[0].close()


def test_batch_64_items_full(ims):
    """The 64-item uneven batch (ER / BA, IC-WC / LT-1/indeg, n 1k-200k, 2,000
    trials each) in one persistent launch with the default schedule: every
    item's per-trial counts, per-node counts and total equal the oracle's over
    all trials."""
    import os

    import torch
    ws = synth.batch_items()
    items = [(ims.Graph(w.graph.n, w.graph.offsets, w.graph.indices, w.model, w.param), w.seeds, w.n_trials, w.rng_seed)
             for w in ws]
    B = ims.Batch(items)
    say("[parity] batch of 64 items, default schedule")
    B.launch()
    torch.cuda.synchronize()
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    for k, (w, r) in enumerate(zip(ws, B.results())):
        ref = oracle.simulate(w.model, w.graph.n, w.graph.offsets, w.graph.indices, oracle.encode(w.model, w.param),
                              w.seeds, w.n_trials, w.rng_seed, threads=threads, want_bits=False)
        assert r["total"] == ref["total"], (k, w.name)
        assert (r["trial_counts"] == ref["trial_counts"]).all(), (k, w.name)
        assert (r["node_counts"] == ref["node_counts"]).all(), (k, w.name)
    B.close()
    for it in items:
        it[0].close()
