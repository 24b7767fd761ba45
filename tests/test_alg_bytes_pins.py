"""Pins of the algorithmic byte count (the roofline numerator) on graphs small
enough to count by hand.

The count's unit is a (64-trial word, step, frontier node u) triple: u is in
the frontier of a step of the word when some trial of the word activated u in
the step before (Section 3, "Algorithms").  Each unit costs 16 B of row
offsets, per out-arc a 4 B index, a b_p B parameter (4 for the IC threshold,
8 for the LT weight) and an 8 B target-state update, and 16 B to read the
frontier mask and write the active mask.  The expected values below are
written from that rule, node by node; activation steps that depend on coins
or thresholds come from numpy's Philox (tests/pins.py), not from the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import alg_bytes as AB

from pins import numpy_hash32

TWO32 = 1 << 32


def graph(n, arcs):
    """Graph whose out-rows keep the given arc order (arc ids are positions)."""
    src = np.array([a for a, _ in arcs], dtype=np.int64)
    dst = np.array([b for _, b in arcs], dtype=np.uint32)
    assert np.all(np.diff(src) >= 0), "arcs must be listed by source"
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=offsets[1:])
    return synth.Graph(n=n, offsets=offsets, indices=dst)


def unit_bytes(outdeg, b_p):
    return 16 + outdeg * (4 + b_p + 8) + 16


def run(model, g, param, seeds, T, rs=5):
    enc = np.asarray(param, dtype=np.uint32 if model == "ic" else np.uint64)
    return AB.alg_bytes(model, g, enc, np.asarray(seeds, dtype=np.uint32), T, rs, threads=1)


@pytest.mark.parametrize("T", [1, 64, 130])
def test_certain_path_one_unit_per_node_and_word(T):
    # 0 -> 1 -> 2 -> 3, every arc certain: each word sees nodes 0..3 once each
    g = graph(4, [(0, 1), (1, 2), (2, 3)])
    W = (T + 63) // 64
    for model, param, b_p in (("ic", [0xFFFFFFFF] * 3, 4), ("lt", [TWO32] * 3, 8)):
        r = run(model, g, param, [0], T)
        per_word = 3 * unit_bytes(1, b_p) + unit_bytes(0, b_p)
        assert r["units"] == 4 * W
        assert r["bytes"] == per_word * W
        assert r["exams"] == 3 * T  # outdeg 1 + 1 + 1 + 0 per trial


def test_certain_out_star():
    # seed 0 with five certain out-arcs to leaves without out-arcs
    g = graph(6, [(0, v) for v in range(1, 6)])
    for model, param, b_p in (("ic", [0xFFFFFFFF] * 5, 4), ("lt", [TWO32] * 5, 8)):
        r = run(model, g, param, [0], 64)
        assert r["units"] == 6
        assert r["bytes"] == unit_bytes(5, b_p) + 5 * unit_bytes(0, b_p)
        assert r["exams"] == 5 * 64


def test_p_zero_counts_only_the_seed_rows():
    # IC with every threshold 0: the seeds form the only frontier
    g = graph(4, [(0, 1), (0, 2), (1, 3), (2, 3)])
    r = run("ic", g, [0] * 4, [0, 3], 100)
    assert r["units"] == 2 * 2  # two seeds, two words
    assert r["bytes"] == 2 * (unit_bytes(2, 4) + unit_bytes(0, 4))
    assert r["exams"] == 2 * 100


def _levels_of_x_ic(rs, T):
    # s = 0, y = 1, x = 2; arcs (ids) 0: s->y certain, 1: s->x at 1/2, 2: y->x certain.
    # x joins at step 1 in trials where arc 1 is live, else at step 2 through y.
    thr = 0x80000000
    return [1 if numpy_hash32(rs, 1, t, 1) < thr else 2 for t in range(T)]


def _levels_of_x_lt(rs, T):
    # s = 0, y = 1, x = 2; w(s->y) = 1, w(s->x) = w(y->x) = 1/2.  y joins at step 1
    # in every trial (2^32 > any hash); x joins at step 1 when 2^31 > h_x(t),
    # else at step 2, when its active in-weight is 2^32.
    return [1 if (TWO32 >> 1) > numpy_hash32(rs, 2, t, 2) else 2 for t in range(T)]


@pytest.mark.parametrize("model", ["ic", "lt"])
@pytest.mark.parametrize("T", [64, 128, 100])
def test_node_joining_at_two_steps_in_one_word_is_two_units(model, T):
    g = graph(3, [(0, 1), (0, 2), (1, 2)])
    rs = 5
    if model == "ic":
        param, b_p, lev = [0xFFFFFFFF, 0x80000000, 0xFFFFFFFF], 4, _levels_of_x_ic(rs, T)
    else:
        param, b_p, lev = [TWO32, TWO32 >> 1, TWO32 >> 1], 8, _levels_of_x_lt(rs, T)
    expect_units = expect_bytes = 0
    for w0 in range(0, T, 64):
        distinct = len(set(lev[w0:w0 + 64]))
        assert distinct == 2, "premise: x joins at both steps within the word"
        expect_units += 1 + 1 + distinct
        expect_bytes += unit_bytes(2, b_p) + unit_bytes(1, b_p) + distinct * unit_bytes(0, b_p)
    r = run(model, g, param, [0], T, rs)
    assert r["units"] == expect_units
    assert r["bytes"] == expect_bytes
    assert r["exams"] == 3 * T
    # and the step numbers themselves: the oracle's levels for x equal the
    # ones derived from numpy's hash
    enc = np.asarray(param, dtype=np.uint32 if model == "ic" else np.uint64)
    o = oracle.simulate(model, 3, g.offsets, g.indices, enc, [0], T, rs, want_levels=True)
    assert o["levels"][:, 2].tolist() == lev
