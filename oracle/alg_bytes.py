"""Algorithmic HBM bytes of a bit-parallel frontier simulation, from the
oracle's per-trial activation steps.

Unit of work: a (64-trial word, step, frontier node u) triple, where u is in
the frontier of step l for the word when some trial of the word activated u
at step l - 1 (Section 3, "Algorithms": each step examines the out-arcs of
the nodes activated in the previous step).  Its compulsory traffic is the
node's CSR row (16 B of offsets plus outdeg(u) * (4 B index + b_p B
parameter)), one 8 B state update per examined arc, and 16 B to read the
frontier mask and write the active mask:

    B_alg = sum over (word, step, u in F) of  32 + outdeg(u) * (12 + b_p)

with b_p = 4 (uint32 IC threshold) or 8 (uint64 LT weight).

TEST / MEASUREMENT INFRASTRUCTURE: calls only the oracle and the seeded
input generators, and writes its result under tests/golden/.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def alg_bytes(model: str, g: synth.Graph, enc, seeds, n_trials: int, rng_seed: int, threads: int) -> dict:
    b_p = 4 if model == "ic" else 8
    outdeg = g.outdeg()
    per_node = 32 + outdeg * (12 + b_p)
    total = 0
    units = 0
    exams = 0
    for t0 in range(0, n_trials, 64):
        cnt = min(64, n_trials - t0)
        r = oracle.simulate(model, g.n, g.offsets, g.indices, enc, seeds, cnt, rng_seed, t_begin=t0,
                            threads=threads, want_bits=False, want_levels=True, want_node_counts=False)
        lv = r["levels"]  # [cnt, n], -1 = never active
        exams += int(r["exams"].sum())
        # distinct activation steps of each node across the word's trials
        lv_sorted = np.sort(lv, axis=0)
        distinct = (lv_sorted[0] >= 0).astype(np.int64)
        distinct += ((lv_sorted[1:] != lv_sorted[:-1]) & (lv_sorted[1:] >= 0)).sum(axis=0)
        units += int(distinct.sum())
        total += int((distinct * per_node).sum())
        print(f"word {t0 // 64}: units {int(distinct.sum())}", flush=True)
    return {"bytes": total, "units": units, "exams": exams}


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="lt_chunglu_1m", choices=["lt_chunglu_1m", "ba_ic_100k", "er_ic_1k"])
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    args = ap.parse_args()
    w = {"lt_chunglu_1m": synth.chung_lu_lt_1m, "ba_ic_100k": synth.ba_ic_100k, "er_ic_1k": synth.er_ic_1k}[args.workload]()
    enc = oracle.encode(w.model, w.param)
    t = time.time()
    res = alg_bytes(w.model, w.graph, enc, w.seeds, w.n_trials, w.rng_seed, args.threads)
    res.update({"workload": w.name, "graph_sha256": w.graph.sha256(), "n_trials": w.n_trials,
                "rng_seed": w.rng_seed, "seconds": round(time.time() - t, 1)})
    out = os.path.join(ROOT, "tests", "golden", f"alg_bytes_{args.workload}.json")
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
