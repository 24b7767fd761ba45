"""Pins of the FP64 reference of the spread estimator (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import mpnn_ref as R


def tiny_graph(seed=0, n=9, m=24):
    rng = np.random.default_rng(seed)
    arcs = set()
    while len(arcs) < m:
        u, v = rng.integers(0, n - 1, size=2)  # node n-1 stays isolated
        if u != v:
            arcs.add((int(u), int(v)))
    # one node with in-degree above 4 (the GPU's unrolled path and its tail)
    for u in range(5):
        if u != 7:
            arcs.add((u, 7))
    arcs = sorted(arcs)
    src = np.array([a for a, _ in arcs])
    dst = np.array([b for _, b in arcs], dtype=np.uint32)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=offsets[1:])
    a = rng.uniform(0.05, 0.9, size=len(arcs)).astype(np.float32)
    return n, offsets, dst, a


def random_params(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, scale, size=R.NPARAMS)
    p[R.OFF["b0"]:R.OFF["b0"] + 64] += 0.3  # keep most ReLUs away from their kink
    return p


def test_bf16_rounding_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 10, 5000), [1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -0.0, 1e-40, 3e38]])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(R.bf16_round(x), ref)
    assert R.bf16_round(np.float32(1 + 2.0 ** -8))[()] == 1.0
    assert R.bf16_round(np.float32(1 + 3 * 2.0 ** -8))[()] == 1 + 2.0 ** -6


def test_backward_matches_central_differences():
    n, off, idx, a = tiny_graph()
    sets = [[0], [2, 5, 2], [], [1, 3, 4, 6]]  # duplicate member, empty set
    params = random_params(1)
    target = np.array([3.0, 1.0, 2.0, 6.5])
    fwd = R.forward(params, n, off, idx, a, sets)
    grads, L = R.backward(fwd, target)

    def f(p):
        return R.loss(R.forward(p, n, off, idx, a, sets)["pred"], target, n)

    assert abs(f(params) - L) < 1e-15
    rng = np.random.default_rng(2)
    real_w0 = [r * 64 + c for r in (0, 1, 2, 3, 16, 17, 18, 19) for c in range(64)]
    picks = np.unique(np.concatenate([rng.choice(real_w0, 60, replace=False),
                                      R.OFF["b0"] + rng.choice(64, 10, replace=False),
                                      R.OFF["W1"] + rng.choice(8192, 60, replace=False),
                                      R.OFF["b1"] + rng.choice(64, 10, replace=False),
                                      R.OFF["W2"] + rng.choice(8192, 60, replace=False),
                                      R.OFF["b2"] + rng.choice(64, 10, replace=False),
                                      R.OFF["wo"] + np.arange(64), [R.OFF["bo"]]]))
    h = 1e-6
    fd = np.empty(picks.shape[0])
    for i, j in enumerate(picks):
        p1, p2 = params.copy(), params.copy()
        p1[j] += h
        p2[j] -= h
        fd[i] = (f(p1) - f(p2)) / (2 * h)
    scale = np.abs(grads[picks]).max()
    assert scale > 0
    np.testing.assert_allclose(grads[picks], fd, rtol=1e-5, atol=1e-6 * scale)
    # inputs that are always zero (padded features) get zero gradient
    pad_rows = [r for r in range(32) if r not in (0, 1, 2, 3, 16, 17, 18, 19)]
    W0g = grads[:2048].reshape(32, 64)
    assert np.all(W0g[pad_rows] == 0)


def test_aggregation_direction_on_two_nodes():
    # one arc 0 -> 1 with a = 0.5: node 1 aggregates node 0, node 0 gets nothing
    off = np.array([0, 1, 1], dtype=np.int64)
    idx = np.array([1], dtype=np.uint32)
    a = np.array([0.5], dtype=np.float32)
    fwd = R.forward(random_params(4), 2, off, idx, a, [[0], [1]])
    M0 = fwd["cache"]["M"][0]
    assert M0[1, 0, 0] == 0.5 and M0[0, 0, 0] == 0.0   # seed indicator of set {0}
    assert M0[1, 1, 0] == 0.0 and M0[0, 1, 0] == 0.0   # set {1}: nothing flows backwards
    X = fwd["cache"]["H"][0]
    np.testing.assert_array_equal(M0[1], 0.5 * X[0])
    np.testing.assert_array_equal(M0[0], 0.0 * X[0])


def test_relabelling_nodes_leaves_predictions_unchanged():
    n, off, idx, a = tiny_graph(5)
    sets = [[0, 4], [7], [2, 3, 8]]
    params = random_params(6)
    base = R.forward(params, n, off, idx, a, sets)["pred"]
    perm = np.random.default_rng(7).permutation(n)          # old id -> new id
    src = np.repeat(np.arange(n), np.diff(off))
    new_src, new_dst = perm[src], perm[idx.astype(np.int64)]
    order = np.lexsort((np.arange(len(src)), new_src))       # keep arcs, regroup by new source
    off2 = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(new_src, minlength=n), out=off2[1:])
    got = R.forward(params, n, off2, new_dst[order].astype(np.uint32), a[order],
                    [[perm[v] for v in s] for s in sets])["pred"]
    np.testing.assert_allclose(got, base, rtol=1e-12)


def test_closed_form_with_zero_weights_and_seed_counting():
    n, off, idx, a = tiny_graph(8)
    p = np.zeros(R.NPARAMS)
    rng = np.random.default_rng(9)
    b = {k: rng.normal(0, 1, 64) for k in ("b0", "b1", "b2")}
    for k, v in b.items():
        p[R.OFF[k]:R.OFF[k] + 64] = v
    wo = rng.normal(0, 1, 64)
    p[R.OFF["wo"]:R.OFF["wo"] + 64] = wo
    p[R.OFF["bo"]] = 0.25
    sets = [[1, 1, 2], [], [0, 3, 4, 5]]
    pred = R.forward(p, n, off, idx, a, sets)["pred"]
    yz = 1.0 / (1.0 + np.exp(-(np.maximum(b["b2"], 0) @ wo + 0.25)))
    for s, got in zip(sets, pred):
        k = len(set(s))
        assert abs(got - (k + (n - k) * yz)) < 1e-12
    p[R.OFF["bo"]] = -800.0
    pred = R.forward(p, n, off, idx, a, sets)["pred"]
    np.testing.assert_array_equal(pred, [2.0, 0.0, 4.0])


def _header_offsets():
    """Parameter offsets as the C header declares them."""
    import os
    import re
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "imsim_mpnn.h")
    with open(path) as f:
        return {k: int(v) for k, v in re.findall(r"#define IMS_MPNN_OFF_(\w+) (\d+)", f.read())}


def test_forward_by_hand_from_the_header_definition():
    """Three nodes, arcs 0->1 (a = 1/2), 2->1 (1/4), 1->0 (3/4), nonzero
    weights everywhere; every layer written out scalar by scalar from the
    header: z_v[c] = b[c] + sum_k h_v[k] W[k][c] + sum_k m_v[k] W[d + k][c]
    with m_v = sum over arcs (u, v) of a_uv h_u, W row-major [2d][64] at the
    header's offsets; readout 1 for seeds, else sigmoid(h_v . w_o + b_o)."""
    import math
    off_h = _header_offsets()
    n = 3
    offsets = np.array([0, 1, 2, 3], dtype=np.int64)
    indices = np.array([1, 0, 1], dtype=np.uint32)
    a = np.array([0.5, 0.75, 0.25], dtype=np.float32)
    arcs = [(0, 1, 0.5), (1, 0, 0.75), (2, 1, 0.25)]
    rng = np.random.default_rng(21)
    params = rng.normal(0.0, 0.3, size=off_h["BO"] + 1)
    sets = [[0], [2], [0, 2], []]

    outdeg = [1, 1, 1]
    indeg = [1, 2, 0]
    asum = [0.5, 0.75, 0.25]
    f32 = lambda x: float(np.float32(x))  # noqa: E731  (features are stored as float32)
    widths = [16, 64, 64, 64]
    preds = []
    for s in sets:
        h = [[0.0] * 16 for _ in range(n)]
        for v in range(n):
            h[v][0] = 1.0 if v in s else 0.0
            h[v][1] = f32(math.log1p(outdeg[v]))
            h[v][2] = f32(math.log1p(indeg[v]))
            h[v][3] = f32(math.log1p(asum[v]))
        for layer in range(3):
            d = widths[layer]
            wo_, bo_ = off_h[f"W{layer}"], off_h[f"B{layer}"]
            m = [[0.0] * d for _ in range(n)]
            for (u, v, w) in arcs:
                for k in range(d):
                    m[v][k] += w * h[u][k]
            nh = [[0.0] * 64 for _ in range(n)]
            for v in range(n):
                for c in range(64):
                    z = params[bo_ + c]
                    for k in range(d):
                        z += h[v][k] * params[wo_ + k * 64 + c]          # self rows 0 .. d-1
                        z += m[v][k] * params[wo_ + (d + k) * 64 + c]    # aggregate rows d .. 2d-1
                    nh[v][c] = max(z, 0.0)
            h = nh
        total = 0.0
        for v in range(n):
            if v in s:
                total += 1.0
            else:
                z = params[off_h["BO"]] + sum(h[v][c] * params[off_h["WO"] + c] for c in range(64))
                total += 1.0 / (1.0 + math.exp(-z))
        preds.append(total)
    got = R.forward(params, n, offsets, indices, a, sets)["pred"]
    np.testing.assert_allclose(got, preds, rtol=1e-12, atol=0)
    # the offsets of the reference equal the header's
    for k, v in R.OFF.items():
        assert off_h[k.upper()] == v
    assert R.NPARAMS == off_h["BO"] + 1
    # swapping the self and aggregate halves of any one layer changes the answer
    for layer in range(3):
        d = widths[layer]
        sw = params.copy()
        base = R.OFF[f"W{layer}"]
        Wl = sw[base:base + 2 * d * 64].reshape(2 * d, 64).copy()
        sw[base:base + 2 * d * 64] = np.concatenate([Wl[d:], Wl[:d]]).ravel()
        assert np.max(np.abs(R.forward(sw, n, offsets, indices, a, sets)["pred"] - preds)) > 1e-6
