"""Writes rownet4M_k64_levels.json: the oracle's result on every level of the 4M-vertex row-net
workload's 12-level hierarchy, refined from the coarsest level to the finest exactly as the
benchmark does (greedy start on the coarsest level, projection between levels, temperatures
0.75 / 0.375 / 0, limit 8 -- Algorithm 1 with the final setting of the paper's experiments).

Only oracle/ computes the values; the inputs come from the seeded generators in workloads/.  The
GPU test (tests/test_gpu_fullsize.py) runs the same chain through the library and compares every
level's output partition (SHA-256), metric, iteration and rebalancing counts with this file.

The coarse levels are the slow ones for the oracle (about half an hour for the coarsest alone), so
the file is rewritten after every level with the levels done so far, and the last output partition
is kept in rownet4M_k64_levels.resume.npz; a later run continues from there (after checking it
against the stored SHA-256) and deletes it when the chain is complete.

Run: python tests/golden/make_rownet_levels.py   (single-threaded; many hours for all 12 levels)
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

SEED, N, K, LEVELS = 4, 4_000_000, 64, 12
TAU, LIMIT = (0.75, 0.375, 0.0), 8


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def write(out_path, levels):
    doc = {"source": "oracle/ (jo_refine), written by tests/golden/make_rownet_levels.py; inputs from workloads/ "
                     "(rownet_matrix seed 4, hierarchy seed 4, greedy_initial seed 4)",
           "workload": f"rownet-{N}-k{K}", "levels_total": LEVELS, "tau": list(TAU), "limit": LIMIT,
           "complete": len(levels) == LEVELS, "levels": levels}
    tmp = out_path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(doc, fh, indent=1)
    os.replace(tmp, out_path)


def main(out_path=os.path.join(HERE, "rownet4M_k64_levels.json")):
    t0 = time.time()
    hg = W.rownet_matrix(seed=SEED, n=N, k=K)
    hgs, parents = W.hierarchy(hg, LEVELS, seed=SEED)
    part = W.greedy_initial(hgs[-1], seed=SEED)
    print(f"hierarchy built in {time.time() - t0:.0f}s", flush=True)
    levels = []
    resume = out_path.replace(".json", ".resume.npz")
    if os.path.exists(out_path) and os.path.exists(resume):
        with open(out_path) as fh:
            levels = json.load(fh)["levels"]
        part = np.load(resume)["part"]
        assert levels and sha(part) == levels[-1]["sha256_out"] and len(part) == hgs[levels[-1]["level"]].n
        print(f"resuming after level {levels[-1]['level']}", flush=True)
    for lvl in range(LEVELS - 1 - len(levels), -1, -1):
        if lvl < LEVELS - 1:
            part = part[parents[lvl]]
        t1 = time.time()
        sha_in = sha(part)
        part, rc, st, _ = O.refine(hgs[lvl], part, tau=TAU, limit=LIMIT)
        levels.append({"level": lvl, "n": int(hgs[lvl].n), "pins": int(hgs[lvl].p), "sha256_in": sha_in,
                       "sha256_out": sha(part), "rc": rc, "km1_in": st["km1_in"], "km1_out": st["km1_out"],
                       "iterations": st["iterations"], "rebalance_rounds": st["rebalance_rounds"],
                       "moves_executed": st["moves_executed"], "max_block_weight": st["max_block_weight"]})
        print(f"level {lvl}: km1 {st['km1_in']} -> {st['km1_out']}, {st['iterations']} iterations, "
              f"{time.time() - t1:.0f}s", flush=True)
        np.savez(resume, part=part)
        write(out_path, levels)
    os.remove(resume)
    print(f"wrote {out_path} in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
