"""The allocation-free entry point (ims_simulate_noalloc) against ims_simulate
through the C ABI: identical per-trial counts, per-node counts and totals, on
calls in a row whose later inputs are smaller than the earlier ones (the fixed
device array keeps the previous call's contents), plus its size limit."""
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


def run_noalloc(ims, G, seeds, T, rs):
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    tc = torch.full((T,), -1, dtype=torch.int32, device=dev)
    nc = torch.full((G.n,), -1, dtype=torch.int32, device=dev)
    tot = torch.full((1,), -1, dtype=torch.int64, device=dev)
    ims.simulate_noalloc_into(G, seeds, T, rs, tc, tot, nc)
    steps, guard = G.last_status()
    assert guard == 0
    return tc.cpu().numpy().view(np.uint32), nc.cpu().numpy().view(np.uint32), int(tot.item())


def check_case(ims, model, g, param, seeds, T, rs, with_oracle=False):
    say(f"[noalloc] model={model} n={g.n} m={g.m} T={T} seeds={len(seeds)} rng={rs}")
    G = ims.Graph(g.n, g.offsets, g.indices, model, param)
    ref = ims.simulate(G, seeds, T, rs)
    tc, nc, tot = run_noalloc(ims, G, seeds, T, rs)
    assert tot == ref["total"]
    assert (tc == ref["trial_counts"].cpu().numpy().view(np.uint32)).all()
    assert (nc == ref["node_counts"].cpu().numpy().view(np.uint32)).all()
    if with_oracle:
        o = oracle.simulate(model, g.n, g.offsets, g.indices, oracle.encode(model, param), seeds, T, rs,
                            threads=8, want_bits=False)
        assert tot == o["total"]
        assert (tc == o["trial_counts"]).all()
        assert (nc == o["node_counts"]).all()
    G.close()
    return tot


@pytest.mark.parametrize("model", ["ic", "lt"])
def test_noalloc_equals_simulate_on_calls_in_a_row(ims, model):
    big = synth.barabasi_albert(20000, 4, seed=31)
    small = synth.erdos_renyi_directed(700, 5.0, seed=32)
    par = (lambda g: synth.weighted_cascade(g)) if model == "lt" else (lambda g: synth.uniform_p(g, 0.12))
    seeds_big = synth.random_seeds(big.n, 40, seed=33)
    seeds_small = synth.random_seeds(small.n, 6, seed=34)
    # a larger run, then smaller ones: fewer nodes, trials and seeds
    check_case(ims, model, big, par(big), seeds_big, 1000, 5)
    check_case(ims, model, small, par(small), seeds_small, 130, 6, with_oracle=True)
    # duplicates, an empty seed set, one trial
    check_case(ims, model, small, par(small), np.concatenate([seeds_small, seeds_small[:3]]), 77, 7, with_oracle=True)
    check_case(ims, model, small, par(small), np.zeros(0, dtype=np.uint32), 64, 8)
    check_case(ims, model, small, par(small), seeds_small[:2], 1, 9, with_oracle=True)


def test_noalloc_graph_that_fits_few_slots(ims):
    # about 200k nodes: the fixed array holds only a handful of workgroup slots
    g = synth.barabasi_albert(200000, 3, seed=41)
    check_case(ims, "ic", g, synth.uniform_p(g, 0.05), synth.random_seeds(g.n, 30, seed=42), 512, 11)


def test_noalloc_rejects_graphs_beyond_its_array(ims):
    import torch
    n = 1_500_000  # one slot of 48 B per node alone exceeds 64 MiB
    off = np.zeros(n + 1, dtype=np.int64)
    G = ims.Graph(n, off, np.zeros(0, dtype=np.uint32), "ic", np.zeros(0, dtype=np.uint32))
    dev = torch.device("cuda", torch.cuda.current_device())
    tc = torch.zeros(64, dtype=torch.int32, device=dev)
    tot = torch.zeros(1, dtype=torch.int64, device=dev)
    with pytest.raises(ims.ImsError) as e:
        ims.simulate_noalloc_into(G, [0, 1], 64, 1, tc, tot)
    assert e.value.code == -8
    assert "scratch" in str(e.value)
    with pytest.raises(ims.ImsError) as e:
        ims.simulate_noalloc_into(G, [n], 64, 1, tc, tot)
    assert e.value.code == -4
    G.close()
