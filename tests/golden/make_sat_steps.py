"""Writes sat20M_k128_steps.json: the oracle's results for every step of one Jet iteration on the
full-size SAT-like workload (20M vertices, 200M pins, Zipf(1.8) nets up to 10^6 pins, vertex weights
U{1..8}, k = 128), from a seeded uniform partition:

  * candidates (Section 4.1, tau 0.75): SHA-256 of M, and of t and g on the candidates;
  * recomputed gains of Algorithm 2 on those candidates: SHA-256 of rg, count of rg > 0;
  * one rebalancing round (Section 4.3) from an overloaded partition (1% of the vertices moved to
    block 0): SHA-256 of the selection and of the resulting partition, vertices moved;
  * one whole Jet iteration (Algorithm 1, limit 1, max_iters 1) with its rebalancing rounds:
    SHA-256 of the output partition, statistics and the iteration record.

Only oracle/ computes the values; inputs come from workloads/.  tests/test_gpu_fullsize.py runs the
same steps through the library and compares.  Run: python tests/golden/make_sat_steps.py
(single-threaded; about twenty minutes).
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


def sha(a, dtype=np.int32):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def overloaded_start(part, n, seed=5):
    over = part.copy()
    over[np.random.default_rng(seed).choice(n, n // 100, replace=False)] = 0
    return over


def main(out_path=os.path.join(HERE, "sat20M_k128_steps.json")):
    t0 = time.time()
    hg = W.sat_like(seed=5)
    part = W.part_uniform(hg.n, hg.k, seed=5)
    doc = {"source": "oracle/ (jo_candidates, jo_afterburner, jo_rebalance_round, jo_refine), written by "
                     "tests/golden/make_sat_steps.py; inputs from workloads/ (sat_like seed 5, part_uniform seed 5)",
           "workload": "sat-20000000-k128", "pins": int(hg.p), "nets": int(hg.m), "tau": 0.75}
    doc["km1"] = O.km1(hg, part)
    tq = O.quantize_tau(0.75)
    t, g, m = O.candidates(hg, part, tq)
    sel = m.astype(bool)
    doc["candidates"] = {"count": int(sel.sum()), "sha256_in_m": sha(m, np.uint8),
                         "sha256_t_on_candidates": sha(np.where(sel, t, -1)),
                         "sha256_g_on_candidates": sha(np.where(sel, g, 0))}
    print(f"candidates {time.time() - t0:.0f}s", flush=True)
    rg = O.afterburner(hg, part, t, g, m)
    doc["afterburner"] = {"sha256_rg": sha(rg), "kept": int((rg > 0).sum())}
    print(f"afterburner {time.time() - t0:.0f}s", flush=True)
    over = overloaded_start(part, hg.n)
    new, sel_t, moved = O.rebalance_round(hg, over)
    doc["rebalance_round"] = {"start": "part_uniform seed 5, then 1% of the vertices (numpy default_rng(5).choice) "
                                       "moved to block 0", "moved": moved, "sha256_sel_target": sha(sel_t),
                              "sha256_part": sha(new)}
    print(f"rebalancing round {time.time() - t0:.0f}s", flush=True)
    out, rc, st, tr = O.refine(hg, part, tau=(0.75,), limit=1, max_iters=1)
    doc["iteration"] = {"rc": rc, "sha256_part": sha(out), "stats": st, "trace": tr}
    print(f"iteration {time.time() - t0:.0f}s", flush=True)
    with open(out_path, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"wrote {out_path}", flush=True)


if __name__ == "__main__":
    main()
