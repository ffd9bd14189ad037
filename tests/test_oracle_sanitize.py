"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle is built a second time with -fsanitize=address,undefined (no recovery: the first
finding aborts) and run in a child process on the hand-derived worked example, on a random
refinement with weights, several temperatures and rebalancing, on the failure paths (a vertex
heavier than the balance limit), with both orders of the original Jet rebalancer, on a clustering
pass of the coarsening phase, and on k-way flow refinements (one with regions over many levels).
The child must exit cleanly and print the same results as the ordinary build.
"""
import json
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle as O, workloads as W
out = {}
hg = W.Hypergraph(n=4, m=3, off=np.array([0, 2, 4, 6], dtype=np.int64),
                  pins=np.array([0, 1, 1, 2, 2, 3], dtype=np.int32), k=2, eps=0.03)
p, rc, st, tr = O.refine(hg, np.array([0, 1, 0, 1]), tau=(0.75,), limit=12)
out["path4"] = [p.tolist(), rc, st["km1_out"], len(tr)]
hg = W.random_hypergraph(400, 700, 8, seed=5, nw_max=4, vw_max=5)
part = W.part_uniform(hg.n, hg.k, seed=5)
p, rc, st, tr = O.refine(hg, part, tau=(0.75, 0.375, 0.0), limit=8)
out["random"] = [int(np.int64(p.astype(np.int64) @ np.arange(1, hg.n + 1))), rc, st["km1_out"], len(tr)]
t, g, m = O.candidates(hg, part, O.quantize_tau(0.75))
rg = O.afterburner(hg, part, t, g, m)
out["ab"] = int(np.abs(rg.astype(np.int64)).sum())
vw = np.ones(40, dtype=np.int32); vw[0] = 60  # heavier than Lmax = 51
hg = W.random_hypergraph(40, 60, 2, seed=7)
hg.vtx_w = vw
p, rc, st = O.rebalance(hg, np.zeros(40, dtype=np.int32))
out["heavy"] = [p.tolist(), rc, st["balanced"]]
hg = W.random_hypergraph(500, 800, 4, seed=9, smax=12, nw_max=3, vw_max=3)
lab, cnt = O.coarsen(hg, np.random.default_rng(9).permutation(hg.n).astype(np.int32), 8)
out["coarsen"] = [int(lab.astype(np.int64) @ np.arange(1, hg.n + 1)), cnt]
hg = W.random_hypergraph(300, 400, 4, seed=11, smax=6, nw_max=3, vw_max=2)
p, st = O.flow_refine(hg, W.part_roundrobin(hg.n, hg.k, 11), max_rounds=3)
out["flows"] = [int(p.astype(np.int64) @ np.arange(1, hg.n + 1)), st["km1_out"], st["pairs"]]
hg = W.random_hypergraph(200, 300, 3, seed=13, smax=6, nw_max=4, vw_max=6)
part = W.part_uniform(hg.n, hg.k, seed=13)
part[: hg.n // 2] = 0
for order in (1, 2):
    p, rc, st, tr = O.refine(hg, part, tau=(0.75, 0.0), limit=6, rb_unweighted=order)
    out[f"order{order}"] = [int(p.astype(np.int64) @ np.arange(1, hg.n + 1)), rc, st["km1_out"], len(tr)]
hg, part = W.banded_hypergraph(800, 4, 14, vw_max=3)
r = O.flow_region(hg, part, 1, 2, 100)
p, st = O.flow_refine(hg, part, max_rounds=2)
out["banded"] = [int((r > 0).sum()), int(p.astype(np.int64) @ np.arange(1, hg.n + 1)), st["km1_out"]]
print(json.dumps(out))
"""


def run_child(env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_oracle_clean_under_asan_ubsan():
    san = oracle.build(force=True, sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime")
    plain = run_child({"JET_ORACLE_LIB": oracle.build(force=False)})
    checked = run_child({"JET_ORACLE_LIB": san, "LD_PRELOAD": asan,
                         "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                         "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    assert checked == plain
    assert plain["path4"] == [[0, 0, 1, 1], 0, 1, plain["path4"][3]]
    assert plain["heavy"][1] == 1 and plain["heavy"][2] == 0  # JET_IMBALANCED, valid partition
