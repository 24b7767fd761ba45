"""Pins for the CPU oracle against what the paper and mathematics fix.

* hash: numpy's Philox4x64-10 (library routine) as known answers;
* per-trial sets: IC = reachability over live arcs (coins from numpy's
  Philox, search by scipy); LT = least fixpoint of the threshold rule found
  by single-node updates in node order (Section 2, "Diffusion Models");
* exact spread by brute-force enumeration (|E| <= 12) in rationals, with the
  LT value computed two independent ways (threshold intervals and the
  Kempe-Kleinberg-Tardos live-edge equivalence);
* closed forms on paths and stars;
* invariants: p = 1 gives reachability, p = 0 gives the seeds, per-trial
  monotonicity in the seed set, seeds always active, the locality observation
  of Section 3 ("Algorithms") per step, totals.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import pins


def bits_to_sets(bits, T, n):
    out = []
    for t in range(T):
        w, b = divmod(t, 64)
        out.append(set(np.nonzero((bits[w] >> np.uint64(b)) & np.uint64(1))[0].tolist()))
    return out


def random_digraph(n, m, rng, self_loops=False):
    src = rng.integers(0, n, size=m)
    dst = rng.integers(0, n, size=m)
    if not self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    return src, dst


# ------------------------------------------------------------------ hash

@pytest.mark.parametrize("seed,dom,c0,c1", [(0, 1, 0, 0), (1, 1, 0, 0), (3, 2, 1, 5),
                                            (2**63 + 11, 1, 2**64 - 1, 77), (999, 2, 123456789, 2**40)])
def test_philox_block_matches_numpy(seed, dom, c0, c1):
    got = [int(x) for x in oracle.philox4x64_10([c0, c1, 0, 0], [seed, dom])]
    assert got == pins.numpy_philox_block(seed, dom, c0, c1)


def test_hash32_matches_numpy_over_trials_and_ids():
    rng = np.random.default_rng(5)
    for _ in range(200):
        seed = int(rng.integers(0, 2**63))
        dom = int(rng.integers(1, 3))
        t = int(rng.integers(0, 10**6))
        ident = int(rng.integers(0, 2**32))
        assert oracle.hash32(seed, dom, t, ident) == pins.numpy_hash32(seed, dom, t, ident)
    # every lane of one block, including id 0 (counter borrow in numpy)
    for t in range(16):
        assert oracle.hash32(7, 1, t, 0) == pins.numpy_hash32(7, 1, t, 0)


# -------------------------------------------------------------- encoders

def test_encode_p_closed_forms():
    p = np.array([0.0, 2.0**-33, 0.01, 0.1, 0.5, 1 - 2.0**-33, 1.0, 2.0**-32, 0.25])
    thr = oracle.encode_p(p)
    assert thr.tolist() == [0, 0, 0x028F5C28, 0x19999999, 0x80000000, 0xFFFFFFFF, 0xFFFFFFFF, 1, 0x40000000]


@pytest.mark.parametrize("bad", [float("nan"), -1e-9, 1.0 + 1e-12, float("inf")])
def test_encode_rejects(bad):
    with pytest.raises(oracle.OracleError):
        oracle.encode_p(np.array([0.1, bad]))
    with pytest.raises(oracle.OracleError):
        oracle.encode_w(np.array([0.1, bad]))


def test_encode_w_closed_forms():
    d = np.arange(1, 200)
    got = oracle.encode_w(1.0 / d)
    assert got.tolist() == [(1 << 32) // int(k) for k in d]
    assert oracle.encode_w(np.array([0.0, 0.5, 1.0])).tolist() == [0, 1 << 31, 1 << 32]


def test_validate():
    off = np.array([0, 2, 3, 3], dtype=np.int64)
    idx = np.array([1, 2, 2], dtype=np.uint32)
    assert oracle.validate("lt", 3, off, idx, np.array([1 << 31, 1 << 31, 1 << 31], dtype=np.uint64)) == 0
    assert oracle.validate("lt", 3, off, idx, np.array([1 << 31, 1 << 31, (1 << 31) + 1], dtype=np.uint64)) == oracle.E_WSUM
    assert oracle.validate("ic", 3, off, np.array([1, 2, 3], dtype=np.uint32)) == oracle.E_GRAPH
    assert oracle.validate("ic", 3, np.array([0, 2, 1, 3], dtype=np.int64), idx) == oracle.E_GRAPH
    with pytest.raises(oracle.OracleError):
        oracle.simulate("ic", 3, off, idx, np.zeros(3, np.uint32), [3], 4, 0)


# ------------------------------------------------ per-trial exact sets

@pytest.mark.parametrize("gseed", [0, 1, 2])
def test_ic_sets_equal_live_arc_reachability(gseed):
    rng = np.random.default_rng(gseed)
    n = 40
    src, dst = random_digraph(n, 160, rng, self_loops=True)
    off, idx, psrc = pins.csr_from_arcs(n, src, dst, src)
    m = idx.shape[0]
    pr = rng.choice([0.0, 0.05, 0.3, 0.7, 1.0], size=m)
    thr = oracle.encode_p(pr)
    seeds = np.array([3, 17, 3, 30], dtype=np.uint32)  # duplicate seed on purpose
    T, rs = 150, 1000 + gseed
    r = oracle.simulate("ic", n, off, idx, thr, seeds, T, rs)
    coins = pins.numpy_hash32_table(rs, 1, T, m)
    sets = bits_to_sets(r["active_bits"], T, n)
    arc_src = np.repeat(np.arange(n), np.diff(off))
    for t in range(T):
        live = (thr == 0xFFFFFFFF) | (coins[t] < thr)
        expect = set(np.nonzero(pins.reachable(n, arc_src[live], idx[live], seeds))[0].tolist())
        assert sets[t] == expect, t
        assert r["trial_counts"][t] == len(expect)
    assert r["node_counts"].tolist() == [sum(v in s for s in sets) for v in range(n)]


@pytest.mark.parametrize("gseed", [0, 1])
def test_ic_levels_equal_live_arc_bfs_distance(gseed):
    """A node's activation level is its shortest live-arc distance from the
    seed set (the synchronous step of Section 2 at which it activates)."""
    rng = np.random.default_rng(20 + gseed)
    n = 40
    src, dst = random_digraph(n, 160, rng, self_loops=True)
    off, idx = pins.csr_from_arcs(n, src, dst)
    m = idx.shape[0]
    thr = oracle.encode_p(rng.choice([0.0, 0.1, 0.4, 0.8, 1.0], size=m))
    seeds = np.array([5, 11, 5], dtype=np.uint32)
    T, rs = 100, 300 + gseed
    r = oracle.simulate("ic", n, off, idx, thr, seeds, T, rs, want_levels=True)
    coins = pins.numpy_hash32_table(rs, 1, T, m)
    arc_src = np.repeat(np.arange(n), np.diff(off))
    for t in range(T):
        live = (thr == 0xFFFFFFFF) | (coins[t] < thr)
        np.testing.assert_array_equal(r["levels"][t], pins.bfs_distance(n, arc_src[live], idx[live], seeds))


@pytest.mark.parametrize("gseed", [0, 1])
def test_lt_sets_equal_least_fixpoint(gseed):
    rng = np.random.default_rng(10 + gseed)
    n = 24
    src, dst = random_digraph(n, 90, rng, self_loops=True)
    off, idx = pins.csr_from_arcs(n, src, dst)
    m = idx.shape[0]
    indeg = np.bincount(idx, minlength=n)
    # weights: a random share of 1/indeg, some nodes at exactly sum 1
    frac = rng.choice([1.0, 0.5, 0.9], size=n)
    wreal = frac[idx] / indeg[idx]
    w64 = oracle.encode_w(wreal)
    assert oracle.validate("lt", n, off, idx, w64) == 0
    seeds = np.array([1, 5], dtype=np.uint32)
    T, rs = 70, 77 + gseed
    r = oracle.simulate("lt", n, off, idx, w64, seeds, T, rs)
    h = pins.numpy_hash32_table(rs, 2, T, n)
    arc_src = np.repeat(np.arange(n), np.diff(off))
    sets = bits_to_sets(r["active_bits"], T, n)
    for t in range(T):
        expect = pins.lt_fixpoint(n, arc_src, idx, w64, seeds, [int(x) for x in h[t]])
        assert sets[t] == expect, t


@pytest.mark.parametrize("gseed", [0, 1])
def test_lt_levels_equal_synchronous_steps(gseed):
    """The oracle's LT activation levels are the synchronous steps of Section
    2, recomputed here step by step from the weights and the threshold
    hashes (numpy Philox)."""
    rng = np.random.default_rng(60 + gseed)
    n = 30
    src, dst = random_digraph(n, 110, rng, self_loops=True)
    off, idx = pins.csr_from_arcs(n, src, dst)
    indeg = np.bincount(idx, minlength=n)
    frac = rng.choice([1.0, 0.6, 0.9], size=n)
    w64 = oracle.encode_w(frac[idx] / indeg[idx])
    seeds = np.array([2, 17], dtype=np.uint32)
    T, rs = 40, 90 + gseed
    r = oracle.simulate("lt", n, off, idx, w64, seeds, T, rs, want_levels=True)
    h = pins.numpy_hash32_table(rs, 2, T, n)
    arc_src = np.repeat(np.arange(n), np.diff(off))
    deepest = 0
    for t in range(T):
        expect = pins.lt_sync_levels(n, arc_src, idx, w64, seeds, [int(x) for x in h[t]])
        np.testing.assert_array_equal(r["levels"][t], np.array(expect, dtype=np.int32))
        deepest = max(deepest, max(expect))
    assert deepest >= 3  # the cases reach several steps


def test_ic_coin_comparison_is_strict():
    # one arc 0 -> 1; the coin of (trial 0, arc 0) decides
    off = np.array([0, 1, 1], dtype=np.int64)
    idx = np.array([1], dtype=np.uint32)
    c = pins.numpy_hash32(5, 1, 0, 0)
    assert c not in (0, 0xFFFFFFFF)
    dead = oracle.simulate("ic", 2, off, idx, np.array([c], np.uint32), [0], 1, 5)
    live = oracle.simulate("ic", 2, off, idx, np.array([c + 1], np.uint32), [0], 1, 5)
    assert dead["trial_counts"][0] == 1 and live["trial_counts"][0] == 2


def test_lt_threshold_comparison_is_strict():
    off = np.array([0, 1, 1], dtype=np.int64)
    idx = np.array([1], dtype=np.uint32)
    h = pins.numpy_hash32(9, 2, 0, 1)
    no = oracle.simulate("lt", 2, off, idx, np.array([h], np.uint64), [0], 1, 9)
    yes = oracle.simulate("lt", 2, off, idx, np.array([h + 1], np.uint64), [0], 1, 9)
    assert no["trial_counts"][0] == 1 and yes["trial_counts"][0] == 2


# ----------------------------------------------- brute force, statistics

def mc_close(mean, exact, var, T, k=5.0):
    return abs(mean - exact) <= k * math.sqrt(max(var, 1e-12) / T) + 1e-12


TINY_GRAPHS = [
    # (n, arcs, p per arc, seeds)
    (4, [(0, 1), (1, 2), (2, 3), (0, 2), (3, 1)], [0.5, 0.3, 0.9, 0.2, 0.6], [0]),
    (5, [(0, 1), (0, 2), (1, 3), (2, 3), (3, 4), (4, 0), (1, 2)], [0.7, 0.4, 0.5, 0.5, 0.8, 0.3, 0.25], [0]),
    (6, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5), (5, 3), (2, 3), (0, 0), (1, 2)],
     [0.6, 0.6, 0.6, 0.3, 0.9, 0.1, 0.5, 1.0, 0.4], [0, 4]),
]


@pytest.mark.parametrize("case", range(len(TINY_GRAPHS)))
def test_ic_brute_force(case):
    n, arcs, pr, seeds = TINY_GRAPHS[case]
    src = [a for a, _ in arcs]
    dst = [b for _, b in arcs]
    off, idx, pp = pins.csr_from_arcs(n, src, dst, pr)
    thr = oracle.encode_p(pp)
    arc_src = np.repeat(np.arange(n), np.diff(off))
    sigma, pi, dist = pins.brute_ic(n, arc_src, idx, thr, seeds)
    T = 40000
    r = oracle.simulate("ic", n, off, idx, thr, seeds, T, 31 + case, threads=4, want_bits=False)
    var = float(sum(p * k * k for k, p in dist.items()) - sigma * sigma)
    assert mc_close(r["mean"], float(sigma), var, T)
    for v in range(n):
        q = float(pi[v])
        assert mc_close(r["node_counts"][v] / T, q, q * (1 - q), T), v
    # distribution of |A|: chi-square against the exact law
    hist = np.bincount(r["trial_counts"], minlength=n + 1)
    chi = 0.0
    dof = 0
    for k, p in dist.items():
        e = float(p) * T
        if e >= 5:
            chi += (hist[k] - e) ** 2 / e
            dof += 1
    assert chi < dof + 6 * math.sqrt(2 * dof) + 10


LT_TINY = [
    (4, [(0, 1), (0, 2), (1, 2), (2, 3), (1, 3), (3, 1)], [0]),
    (5, [(0, 2), (1, 2), (2, 3), (3, 4), (2, 4), (1, 4), (4, 3)], [0, 1]),
]


@pytest.mark.parametrize("case", range(len(LT_TINY)))
def test_lt_two_exact_enumerations_agree_and_match_mc(case):
    n, arcs, seeds = LT_TINY[case]
    src = [a for a, _ in arcs]
    dst = [b for _, b in arcs]
    off, idx = pins.csr_from_arcs(n, src, dst)
    indeg = np.bincount(idx, minlength=n)
    rng = np.random.default_rng(case)
    share = rng.choice([1.0, 0.75, 0.5], size=n)
    w64 = oracle.encode_w(share[idx] / indeg[idx])
    arc_src = np.repeat(np.arange(n), np.diff(off))
    s1, pi1 = pins.brute_lt_thresholds(n, arc_src, idx, w64, seeds)
    s2, pi2 = pins.brute_lt_live_edge(n, arc_src, idx, w64, seeds)
    assert s1 == s2 and pi1 == pi2
    T = 40000
    r = oracle.simulate("lt", n, off, idx, w64, seeds, T, 55 + case, threads=4, want_bits=False)
    for v in range(n):
        q = float(pi1[v])
        assert mc_close(r["node_counts"][v] / T, q, q * (1 - q), T), v


# --------------------------------------------------------- closed forms

def _run(model, n, arcs, param, seeds, T=40000, rs=3):
    src = [a for a, _ in arcs]
    dst = [b for _, b in arcs]
    off, idx, pp = pins.csr_from_arcs(n, src, dst, param)
    enc = oracle.encode_p(pp) if model == "ic" else oracle.encode_w(pp)
    return oracle.simulate(model, n, off, idx, enc, seeds, T, rs, threads=4, want_bits=False), enc


def test_ic_path_closed_form():
    k, p = 6, 0.6
    r, thr = _run("ic", k + 1, [(i, i + 1) for i in range(k)], [p] * k, [0])
    pe = float(pins.p_eff(int(thr[0])))
    T = 40000
    for i in range(k + 1):
        q = pe ** i
        assert mc_close(r["node_counts"][i] / T, q, q * (1 - q), T)
    assert mc_close(r["mean"], sum(pe ** i for i in range(k + 1)), k * k, T)


def test_ic_out_star_and_in_star_closed_forms():
    ps = [0.1, 0.5, 0.9, 0.3]
    r, thr = _run("ic", 5, [(0, i + 1) for i in range(4)], ps, [0])
    pe = [float(pins.p_eff(int(t))) for t in thr]
    assert mc_close(r["mean"], 1 + sum(pe), 4, 40000)
    r, thr = _run("ic", 5, [(i + 1, 0) for i in range(4)], ps, [1, 2, 3, 4])
    q = 1 - np.prod([1 - float(pins.p_eff(int(t))) for t in thr])
    assert mc_close(r["node_counts"][0] / 40000, q, q * (1 - q), 40000)


def test_ic_two_disjoint_paths_closed_form():
    arcs = [(0, 1), (1, 3), (0, 2), (2, 3)]
    ps = [0.5, 0.6, 0.3, 0.8]
    r, thr = _run("ic", 4, arcs, ps, [0])
    off_order = np.argsort([a for a, _ in arcs], kind="stable")
    pe = dict(zip([arcs[i] for i in off_order], [float(pins.p_eff(int(t))) for t in thr]))
    q = 1 - (1 - pe[(0, 1)] * pe[(1, 3)]) * (1 - pe[(0, 2)] * pe[(2, 3)])
    assert mc_close(r["node_counts"][3] / 40000, q, q * (1 - q), 40000)


def test_lt_path_and_in_star_closed_forms():
    ws = [0.9, 0.5, 0.7, 0.4]
    r, w64 = _run("lt", 5, [(i, i + 1) for i in range(4)], ws, [0])
    prod = 1.0
    for i in range(4):
        prod *= int(w64[i]) / 2**32
        assert mc_close(r["node_counts"][i + 1] / 40000, prod, prod * (1 - prod), 40000)
    ws = [0.2, 0.3, 0.1, 0.25]
    r, w64 = _run("lt", 5, [(i + 1, 0) for i in range(4)], ws, [1, 3])
    q = (int(w64[0]) + int(w64[2])) / 2**32
    assert mc_close(r["node_counts"][0] / 40000, q, q * (1 - q), 40000)


# ------------------------------------------------------------ invariants

def _mid_graph(seed=4, n=300, m=1500):
    rng = np.random.default_rng(seed)
    src, dst = random_digraph(n, m, rng)
    off, idx = pins.csr_from_arcs(n, src, dst)
    return n, off, idx, rng


def test_p_one_is_reachability_and_p_zero_is_seeds():
    n, off, idx, rng = _mid_graph()
    seeds = rng.choice(n, 4, replace=False).astype(np.uint32)
    arc_src = np.repeat(np.arange(n), np.diff(off))
    reach = pins.reachable(n, arc_src, idx, seeds)
    r = oracle.simulate("ic", n, off, idx, oracle.encode_p(np.ones(idx.size)), seeds, 100, 1)
    assert (r["node_counts"] == 100 * reach).all()
    r = oracle.simulate("ic", n, off, idx, oracle.encode_p(np.zeros(idx.size)), seeds, 100, 1)
    assert r["trial_counts"].tolist() == [4] * 100
    # LT: one in-arc of weight 1 per node is reachability along those arcs
    first = {}
    for e, v in enumerate(idx.tolist()):
        first.setdefault(v, e)
    keep = np.array(sorted(first.values()))
    w = np.zeros(idx.size)
    w[keep] = 1.0
    r = oracle.simulate("lt", n, off, idx, oracle.encode_w(w), seeds, 100, 1)
    reach = pins.reachable(n, arc_src[keep], idx[keep], seeds)
    assert (r["node_counts"] == 100 * reach).all()


@pytest.mark.parametrize("model", ["ic", "lt"])
def test_monotone_in_seed_set_per_trial_and_locality(model):
    n, off, idx, rng = _mid_graph(7)
    if model == "ic":
        param = oracle.encode_p(np.full(idx.size, 0.25))
    else:
        indeg = np.bincount(idx, minlength=n)
        param = oracle.encode_w(1.0 / indeg[idx])
    small = np.array([1, 2], dtype=np.uint32)
    big = np.array([1, 2, 50, 99], dtype=np.uint32)
    T = 130
    a = oracle.simulate(model, n, off, idx, param, small, T, 9, want_levels=True)
    b = oracle.simulate(model, n, off, idx, param, big, T, 9)
    assert ((a["active_bits"] & ~b["active_bits"]) == 0).all()
    for s in big:
        assert b["node_counts"][s] == T
    assert int(a["trial_counts"].astype(np.int64).sum()) == int(a["node_counts"].astype(np.int64).sum())
    # locality: every non-seed active at step l has an in-neighbour active at step l-1
    arc_src = np.repeat(np.arange(n), np.diff(off))
    lv = a["levels"]
    for t in range(0, T, 13):
        L = lv[t]
        for v in np.nonzero(L > 0)[0]:
            ins = arc_src[idx == v]
            assert (L[ins] == L[v] - 1).any()
        # exams = sum of out-degrees of active nodes
        assert a["exams"][t] == int(np.diff(off)[L >= 0].sum())


def test_ic_per_trial_submodular():
    n, off, idx, rng = _mid_graph(11)
    thr = oracle.encode_p(np.full(idx.size, 0.3))
    T = 64
    S = [1, 2]
    Sp = [1, 2, 40]
    x = 77
    f = {}
    for name, s in {"S": S, "Sx": S + [x], "Sp": Sp, "Spx": Sp + [x]}.items():
        f[name] = oracle.simulate("ic", n, off, idx, thr, np.array(s, np.uint32), T, 5)["trial_counts"].astype(np.int64)
    assert ((f["Sx"] - f["S"]) >= (f["Spx"] - f["Sp"])).all()


def test_thread_count_does_not_change_outputs():
    n, off, idx, rng = _mid_graph(12)
    indeg = np.bincount(idx, minlength=n)
    w64 = oracle.encode_w(1.0 / np.maximum(indeg[idx], 1))
    a = oracle.simulate("lt", n, off, idx, w64, [0, 1, 2], 200, 4, threads=1)
    b = oracle.simulate("lt", n, off, idx, w64, [0, 1, 2], 200, 4, threads=4)
    assert (a["active_bits"] == b["active_bits"]).all()


def test_trial_range_offsets_bits():
    n, off, idx, rng = _mid_graph(13)
    thr = oracle.encode_p(np.full(idx.size, 0.2))
    full = oracle.simulate("ic", n, off, idx, thr, [5, 6], 256, 8)
    part = oracle.simulate("ic", n, off, idx, thr, [5, 6], 64, 8, t_begin=128)
    assert (full["active_bits"][2] == part["active_bits"][0]).all()
    assert (full["trial_counts"][128:192] == part["trial_counts"]).all()


def test_empty_seed_set():
    n, off, idx, rng = _mid_graph(14)
    r = oracle.simulate("ic", n, off, idx, oracle.encode_p(np.full(idx.size, 0.5)), [], 70, 1)
    assert r["total"] == 0 and (r["active_bits"] == 0).all()
