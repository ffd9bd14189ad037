"""Writes batch512_subset.json: the oracle's refinement (tau 0.75, limit 12) of a subset of the
512-hypergraph batch workload (workloads.batch_set(seed=3): n log-uniform in [1e3, 1e5], m = 1.2 n,
Zipf(2.1) net sizes capped at 1,000, k in {2, 8, 32}): the 12 largest hypergraphs and, for each k,
10 more spread evenly over the sizes of that k -- every k and the largest sizes are covered.

Only oracle/ computes the values.  tests/test_gpu_batch.py refines the whole batch through the
library and compares these hypergraphs' partitions (SHA-256) and statistics.
Run: python tests/golden/make_batch_subset.py   (single-threaded; a few minutes)
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def subset(items):
    sizes = np.array([h.p for h, _ in items])
    ks = np.array([h.k for h, _ in items])
    chosen = list(np.argsort(-sizes, kind="stable")[:12])
    for k in (2, 8, 32):
        idx = np.nonzero(ks == k)[0]
        idx = idx[np.argsort(sizes[idx], kind="stable")]
        for j in np.linspace(0, len(idx) - 1, 10).round().astype(int):
            if idx[j] not in chosen:
                chosen.append(idx[j])
    return sorted(int(i) for i in chosen)


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def main(out_path=os.path.join(HERE, "batch512_subset.json")):
    t0 = time.time()
    items = W.batch_set(seed=3)
    rows = []
    for i in subset(items):
        hg, part = items[i]
        out, rc, st, _ = O.refine(hg, part, tau=(0.75,), limit=12)
        rows.append({"index": i, "n": int(hg.n), "pins": int(hg.p), "k": int(hg.k), "rc": rc,
                     "sha256_out": sha(out), "km1_in": st["km1_in"], "km1_out": st["km1_out"],
                     "iterations": st["iterations"], "rebalance_rounds": st["rebalance_rounds"],
                     "moves_executed": st["moves_executed"]})
        print(f"hypergraph {i}: n {hg.n} k {hg.k} km1 {st['km1_in']} -> {st['km1_out']} ({time.time() - t0:.0f}s)",
              flush=True)
    doc = {"source": "oracle/ (jo_refine), written by tests/golden/make_batch_subset.py; inputs from "
                     "workloads.batch_set(seed=3)", "tau": [0.75], "limit": 12, "hypergraphs": rows}
    with open(out_path, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"wrote {out_path} ({len(rows)} hypergraphs)", flush=True)


if __name__ == "__main__":
    main()
