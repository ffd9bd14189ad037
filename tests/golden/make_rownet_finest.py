"""Writes rownet4M_k64_finest.json: the oracle's refinement of the finest level of the 4M-vertex
row-net workload (4M vertices, Zipf(2.1) row nets up to 10^4 pins, k = 64) with the full schedule
of the paper's final setting (temperatures 0.75 / 0.375 / 0, limit 8, Algorithm 1), from a seeded
start: contiguous ID ranges with 40,000 vertices reassigned at random (part_ranges_noise seed 4).

Only oracle/ computes the values; inputs come from workloads/.  tests/test_gpu_fullsize.py refines
the same start through the library and compares the partition (SHA-256), the statistics and every
iteration record.  Run: python tests/golden/make_rownet_finest.py   (single-threaded; about 15
minutes)
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


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def main(out_path=os.path.join(HERE, "rownet4M_k64_finest.json")):
    t0 = time.time()
    hg = W.rownet_matrix(seed=4, n=4_000_000, k=64)
    part = W.part_ranges_noise(hg.n, 64, 40_000, seed=4)
    out, rc, st, tr = O.refine(hg, part, tau=(0.75, 0.375, 0.0), limit=8)
    doc = {"source": "oracle/ (jo_refine), written by tests/golden/make_rownet_finest.py; inputs from workloads/ "
                     "(rownet_matrix seed 4, part_ranges_noise(n, 64, 40000, seed 4))",
           "workload": "rownet-4000000-k64, finest level", "tau": [0.75, 0.375, 0.0], "limit": 8,
           "sha256_in": sha(part), "rc": rc, "sha256_out": sha(out), "stats": st, "trace": tr,
           "seconds": round(time.time() - t0, 1)}
    with open(out_path, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"wrote {out_path}: km1 {st['km1_in']} -> {st['km1_out']}, {st['iterations']} iterations, "
          f"{time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
