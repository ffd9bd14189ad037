"""Writes flows_vlsi1M_round.json: the oracle's result for the flow-refinement benchmark workload,
the VLSI-like hypergraph (1M vertices, k = 8) refined by Jet (temperatures 0.75 / 0.375 / 0, limit
8, Algorithm 1) from its seeded start, then one round of the k-way flow schedule (Section 5, α = 16)
-- exactly what one step of the benchmark computes.

Only oracle/ computes the values; the inputs come from the seeded generators in workloads/.  The
GPU test (tests/test_gpu_flow.py) runs the same through the library and compares the partitions
(SHA-256) and every count with this file.

Run: python tests/golden/make_flows_round.py   (single-threaded; about 20 minutes)
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

SEED, N = 2, 1_000_000
TAU, LIMIT, ALPHA, ROUNDS = (0.75, 0.375, 0.0), 8, 16, 1


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def main():
    t0 = time.time()
    hg, start = W.vlsi_like(seed=SEED, n=N, m=int(1.1 * N))
    jet, rc, st, _ = O.refine(hg, start, trace_cap=0, tau=TAU, limit=LIMIT)
    print(f"Jet: km1 {st['km1_in']} -> {st['km1_out']}, {st['iterations']} iterations, {time.time() - t0:.0f}s",
          flush=True)
    out, fst = O.flow_refine(hg, jet, alpha=ALPHA, max_rounds=ROUNDS)
    print(f"flows: km1 {fst['km1_in']} -> {fst['km1_out']}, {fst['flow_calls']} flows, {time.time() - t0:.0f}s",
          flush=True)
    res = {"workload": "vlsi_like(seed=2, n=1000000, m=1100000), k=8, eps=0.03", "tau": list(TAU), "limit": LIMIT,
           "alpha": ALPHA, "rounds": ROUNDS, "pins": int(hg.p), "sha256_start": sha(start), "jet_rc": rc,
           "jet_km1": st["km1_out"], "jet_iterations": st["iterations"], "sha256_jet": sha(jet),
           "sha256_flows": sha(out), "flows": fst}
    path = os.path.join(HERE, "flows_vlsi1M_round.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print(f"wrote {path} in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
