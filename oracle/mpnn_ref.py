"""FP64 reference of the learned spread estimator (test infrastructure only).

Plain numpy forward and hand-derived backward of the message-passing network
that the GPU library trains to estimate sigma(S) (the expected number of
active nodes, paper Section 2, "Influence Maximization"); the paper defines no
network, the definition is the library's (3 layers of
h' = ReLU([h | sum_in a_uv h_u] W + b), width 64, per-node sigmoid readout with
seeds fixed to 1, summed over nodes).  Nothing here is shared with the HIP
path; only tests import it.  Every array is float64; optional bf16 rounding of
the weights reproduces what the GPU multiplies by.

Pins (tests/test_mpnn_reference.py): the backward against central finite
differences of this forward, node relabelling invariance, the aggregation
direction on a two-node graph, and closed forms with no arcs.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64
IN = 16
N_FEATURES = 4
OFF = {"W0": 0, "b0": 2048, "W1": 2112, "b1": 10304, "W2": 10368, "b2": 18560, "wo": 18624, "bo": 18688}
NPARAMS = 18689
SHAPES = {"W0": (2 * IN, HIDDEN), "b0": (HIDDEN,), "W1": (2 * HIDDEN, HIDDEN), "b1": (HIDDEN,),
          "W2": (2 * HIDDEN, HIDDEN), "b2": (HIDDEN,), "wo": (HIDDEN,), "bo": (1,)}


def bf16_round(x) -> np.ndarray:
    """Round float32 values to bf16 (nearest, ties to even), returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    r = np.where(nan, (u >> 16) | 0x40, r).astype(np.uint32)
    return (r << 16).view(np.float32).astype(np.float64)


def bf16_bits_to_float(bits) -> np.ndarray:
    b = np.ascontiguousarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def unpack(params) -> dict:
    p = np.asarray(params, dtype=np.float64)
    return {k: p[OFF[k]:OFF[k] + int(np.prod(s))].reshape(s) for k, s in SHAPES.items()}


def pack(d: dict) -> np.ndarray:
    out = np.zeros(NPARAMS, dtype=np.float64)
    for k, s in SHAPES.items():
        out[OFF[k]:OFF[k] + int(np.prod(s))] = np.asarray(d[k], dtype=np.float64).ravel()
    return out


def in_csr(n, offsets, indices, a):
    """(in_off, src, weight) listing, for each v, the arcs (u, v) in out-CSR order."""
    offsets = np.asarray(offsets, dtype=np.int64)
    indices = np.asarray(indices, dtype=np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(offsets))
    order = np.argsort(indices, kind="stable")
    in_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(indices, minlength=n), out=in_off[1:])
    return in_off, src[order], np.asarray(a, dtype=np.float64)[order]


def features(n, offsets, indices, a) -> np.ndarray:
    """Static node features [log(1+outdeg), log(1+indeg), log(1 + sum of a over
    out-arcs)], rounded to float32 as the library stores them."""
    offsets = np.asarray(offsets, dtype=np.int64)
    outdeg = np.diff(offsets)
    indeg = np.bincount(np.asarray(indices, dtype=np.int64), minlength=n)
    src = np.repeat(np.arange(n), outdeg)
    asum = np.bincount(src, weights=np.asarray(a, dtype=np.float64), minlength=n)
    f = np.stack([np.log1p(outdeg.astype(np.float64)), np.log1p(indeg.astype(np.float64)), np.log1p(asum)], axis=1)
    return f.astype(np.float32).astype(np.float64)


def aggregate(n, in_off, src, w, H):
    """M[v] = sum over arcs (u, v) of a_uv H[u]; H has shape [n, B, D]."""
    dst = np.repeat(np.arange(n), np.diff(in_off))
    M = np.zeros_like(H)
    np.add.at(M, dst, w[:, None, None] * H[src])
    return M


def aggregate_transpose(n, in_off, src, w, G):
    """Adjoint of aggregate: out[u] = sum over arcs (u, v) of a_uv G[v]."""
    dst = np.repeat(np.arange(n), np.diff(in_off))
    out = np.zeros_like(G)
    np.add.at(out, src, w[:, None, None] * G[dst])
    return out


def input_features(n, feat, sets) -> np.ndarray:
    """X0 [n, B, 16]: seed indicator, the three static features, zeros."""
    B = len(sets)
    X = np.zeros((n, B, IN), dtype=np.float64)
    X[:, :, 1:4] = feat[:, None, :]
    for b, s in enumerate(sets):
        X[np.asarray(s, dtype=np.int64), b, 0] = 1.0
    return X


def forward(params, n, offsets, indices, a, sets, bf16_weights: bool = False, feat=None) -> dict:
    """Prediction pred[b] for every set and every intermediate (fp64)."""
    P = unpack(params)
    if bf16_weights:
        for k in ("W0", "W1", "W2", "wo"):
            P[k] = bf16_round(P[k])
    in_off, src, w = in_csr(n, offsets, indices, np.asarray(a, dtype=np.float32).astype(np.float64))
    if feat is None:
        feat = features(n, offsets, indices, a)
    X = input_features(n, feat, sets)
    if bf16_weights:
        X = bf16_round(X)
    cache = {"P": P, "in": (in_off, src, w), "H": [X], "M": []}
    H = X
    for layer in range(3):
        M = aggregate(n, in_off, src, w, H)
        Z = np.concatenate([H, M], axis=2) @ P[f"W{layer}"] + P[f"b{layer}"]
        cache["M"].append(M)
        H = np.maximum(Z, 0.0)
        cache["H"].append(H)
    z = H @ P["wo"] + P["bo"][0]
    seed = X[:, :, 0] != 0
    with np.errstate(over="ignore"):
        y = np.where(seed, 1.0, 1.0 / (1.0 + np.exp(-z)))
    cache["yhat"] = y
    cache["n"] = n
    return {"pred": y.sum(axis=0), "cache": cache}


def loss(pred, target, n) -> float:
    d = (np.asarray(pred, dtype=np.float64) - np.asarray(target, dtype=np.float64)) / n
    return float(np.mean(d * d))


def backward(fwd: dict, target) -> tuple[np.ndarray, float]:
    """Gradient of loss(pred, target) with respect to the flat parameters."""
    c = fwd["cache"]
    P, n = c["P"], c["n"]
    in_off, src, w = c["in"]
    pred = fwd["pred"]
    B = pred.shape[0]
    target = np.asarray(target, dtype=np.float64)
    g = 2.0 * (pred - target) / (n * n) / B                     # d loss / d pred[b]
    y = c["yhat"]
    dz = g[None, :] * y * (1.0 - y)                              # zero for seeds (y = 1)
    grads = {"wo": np.einsum("vb,vbc->c", dz, c["H"][3]), "bo": np.array([dz.sum()])}
    dH = dz[:, :, None] * P["wo"][None, None, :]
    for layer in (2, 1, 0):
        Hout, Hin, M = c["H"][layer + 1], c["H"][layer], c["M"][layer]
        dZ = dH * (Hout > 0)
        Xcat = np.concatenate([Hin, M], axis=2)
        grads[f"W{layer}"] = np.einsum("vbk,vbc->kc", Xcat, dZ)
        grads[f"b{layer}"] = dZ.sum(axis=(0, 1))
        if layer == 0:
            break
        dX = dZ @ P[f"W{layer}"].T
        D = Hin.shape[2]
        dH = dX[:, :, :D] + aggregate_transpose(n, in_off, src, w, dX[:, :, D:])
    return pack(grads), loss(pred, target, n)
