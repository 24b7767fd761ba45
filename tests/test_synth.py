"""Synthetic input generators: structure of each family and SHA-256 pins of
the arrays (a changed generator changes every stored expectation)."""
import numpy as np
import pytest

import synth

PINS = {
    "er": ("ecf8ed6b58fa4ef6a379e5479c0b5a2b3c3dca987143697d1a116020903bf28f", 19794),
    "ba": ("09db0413fc07545a4b054368be94b231afe7ece968523961ea02347f317b42bd", 29950),
    "cld": ("e561ecfaba7eba5fe35dd353e4dbe173bbaa36d030fcb1924d9c4ca8ce66e18d", 78498),
    "clu": ("7fe10a9f7fb5752eb8f0473cfa9f1870944d31575390a869b5e494801ba37fab", 46266),
    "rr": ("4c8b6d33563d4ffe54ad7c32dc6a7f4b7e44282ebe8b146a2726eda900f9f110", 35000),
    "ws": ("938fbfb3588cc5a0a416884d9533ae4c0611b5387f4e52f81ebf3a601ded28ed", 100000),
}


def make(name):
    return {
        "er": lambda: synth.erdos_renyi_directed(2000, 10.0, 5),
        "ba": lambda: synth.barabasi_albert(3000, 5, 6),
        "cld": lambda: synth.chung_lu_directed(5000, 2.1, 16.0, 7),
        "clu": lambda: synth.chung_lu_undirected(5000, 2.3, 10.0, 8),
        "rr": lambda: synth.random_regular(5000, 7, 9),
        "ws": lambda: synth.watts_strogatz(10000, 10, 0.007, 10),
    }[name]()


def simple(g):
    src = g.arc_sources()
    dst = g.indices.astype(np.int64)
    key = src * g.n + dst
    return not np.any(src == dst) and np.unique(key).shape[0] == key.shape[0]


@pytest.mark.parametrize("name", sorted(PINS))
def test_generator_pins_and_structure(name):
    g = make(name)
    sha, m = PINS[name]
    assert g.m == m and g.sha256() == sha
    assert simple(g)
    src, dst = g.arc_sources(), g.indices.astype(np.int64)
    if name in ("ba", "clu", "rr", "ws"):      # undirected: both arcs present
        fwd = set(zip(src.tolist(), dst.tolist()))
        assert all((v, u) in fwd for u, v in fwd)
    if name == "rr":
        assert np.all(g.outdeg() == 7) and np.all(g.indeg() == 7)
    if name == "ws":
        assert np.all(g.outdeg() >= 1) and abs(g.m / g.n - 10.0) < 1e-9
    if name == "er":
        assert abs(g.m / g.n - 10.0) < 0.5
    if name == "cld":
        assert abs(g.m / g.n - 16.0) < 1.0 and g.outdeg().max() > 20 * 16   # heavy out-degree tail


def test_weight_models():
    g = make("er")
    wc = synth.weighted_cascade(g)
    sums = np.bincount(g.indices.astype(np.int64), weights=wc, minlength=g.n)
    assert np.allclose(sums[g.indeg() > 0], 1.0)
    tv = synth.trivalency(g, 1)
    assert set(np.unique(tv)) <= {0.1, 0.01, 0.001}
    ur = synth.uniform_random(g, 2)
    assert ur.min() >= 0.0 and ur.max() <= 1.0


def test_workload_seeds():
    w = synth.er_ic_1k()
    assert w.graph.sha256() == "e6ea131b9e7b73d6f362c3d0fc750e45da9be6e47935760181992bb87477bd58"
    assert len(set(w.seeds.tolist())) == len(w.seeds) == 10
    g = make("cld")
    top = synth.top_outdeg_seeds(g, 10)
    d = g.outdeg()
    assert np.all(d[top] >= np.sort(d)[-10])


def test_paper_ic_suite():
    ws = synth.paper_ic_suite()
    assert [w.name.split("_n")[0] for w in ws] == ["ic_er_tv", "ic_er_ur", "ic_er_wc", "ic_ws_tv", "ic_ws_ur", "ic_ws_wc",
                                                     "ic_ba_fb_tv", "ic_ba_fb_ur", "ic_ba_fb_wc"]
    pins = {0: ("5f9b8905d935f4f872c0603b1c2bff7de006f191bd385de07151ea8c3424a443", 8040),
            3: ("22e811e27c6f2e8c999a9478ee8ea7aa4cb876232c0e3d4fbeb42ff23fa50e04", 100000),
            6: ("e4e30eda7573108b412019075b431f3b2c6e90e65c923f1d7f3908da2512e337", 176748)}
    for i, (sha, m) in pins.items():
        g = ws[i].graph
        assert g.m == m and g.sha256() == sha and simple(g)
        src, dst = g.arc_sources(), g.indices.astype(np.int64)
        fwd = set(zip(src.tolist(), dst.tolist()))
        assert all((v, u) in fwd for u, v in fwd)       # undirected edges as two arcs
    for w in ws:
        assert w.n_trials == 1000 and len(set(w.seeds.tolist())) == 100
        kind = w.name.split("_")[-3]
        if kind == "tv":
            assert set(np.unique(w.param)) <= {0.1, 0.01, 0.001}
        elif kind == "ur":
            assert w.param.min() >= 0 and w.param.max() <= 1
        else:
            indeg = w.graph.indeg()
            np.testing.assert_allclose(w.param, 1.0 / indeg[w.graph.indices.astype(np.int64)])


def test_undirected_erdos_renyi_pairs():
    g = synth.erdos_renyi_undirected(60, 0.3, seed=3)
    assert simple(g)
    src, dst = g.arc_sources(), g.indices.astype(np.int64)
    assert np.all(np.bincount(src, minlength=60) == np.bincount(dst, minlength=60))
    # expected edge count n(n-1)/2 * p within 5 sd
    e = g.m // 2
    mu = 60 * 59 / 2 * 0.3
    assert abs(e - mu) < 5 * np.sqrt(mu * 0.7)
