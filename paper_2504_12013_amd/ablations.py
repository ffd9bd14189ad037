"""Original-Jet variants against the paper's deterministic Jet settings, on the benchmark workloads.

The paper changes three settings of the original Jet refinement (Sections 4.3 and 7):
  * temperatures: the original uses one round per level with tau_c = 0.75 on the coarse levels and
    tau_f = 0.25 on the finest; the paper runs three rounds, 0.75 / 0.375 / 0, on every level;
  * iteration limit: 12 iterations without improvement in the original, 8 in the paper;
  * rebalancing priority: the original orders moves by gain alone; the paper weighs the gain by
    the vertex weight (gain / c(v) below zero, gain * c(v) above), which it reports reduces the
    penalty of rebalancing.
  * rebalancing selection: the original takes moves by a bucket-based partial order of their loss
    (all of a lower bucket before any of the next) instead of a sort; which vertices of the last
    bucket it takes depends on arrival order, so here a bucket's vertices go in vertex-ID order.

Variants (each refines the whole hierarchy coarsest to finest, on the GPU, from the same start):
  detjet               0.75 / 0.375 / 0 on every level, limit 8, weighted priority (the paper)
  jet-tau              tau_c 0.75 on coarse levels, tau_f 0.25 on the finest, limit 12, weighted
  jet-rebalance        the paper's temperatures and limit, unweighted priority
  jet-bucket           the paper's temperatures and limit, bucket order of the loss
  jet-original         tau_c / tau_f, limit 12, unweighted priority
  jet-original-bucket  tau_c / tau_f, limit 12, bucket order of the loss

    python -m paper_2504_12013_amd.ablations --workload rownet      (4M vertices, k = 64, 12 levels)
    python -m paper_2504_12013_amd.ablations --workload sat         (20M vertices, k = 128, 12 levels)
    python -m paper_2504_12013_amd.ablations --workload graph       (4.2M-vertex mesh, k = 64, 1 level)
Prints one JSON object: per variant the final metric, its ratio to detjet, GPU seconds and
iterations.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from .jet import JetContext

VARIANTS = {
    "detjet": dict(coarse=(0.75, 0.375, 0.0), finest=(0.75, 0.375, 0.0), limit=8, rb_unweighted=0),
    "jet-tau": dict(coarse=(0.75,), finest=(0.25,), limit=12, rb_unweighted=0),
    "jet-rebalance": dict(coarse=(0.75, 0.375, 0.0), finest=(0.75, 0.375, 0.0), limit=8, rb_unweighted=1),
    "jet-bucket": dict(coarse=(0.75, 0.375, 0.0), finest=(0.75, 0.375, 0.0), limit=8, rb_unweighted=2),
    "jet-original": dict(coarse=(0.75,), finest=(0.25,), limit=12, rb_unweighted=1),
    "jet-original-bucket": dict(coarse=(0.75,), finest=(0.25,), limit=12, rb_unweighted=2),
}


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_variant(ctxs, parents, start, v):
    """Refines every level coarsest to finest with the variant's settings; returns (final metric,
    GPU seconds, Jet iterations, rebalancing rounds, balanced)."""
    levels = len(ctxs)
    pars = [torch.from_numpy(p).to("cuda").long() for p in parents]
    part = torch.from_numpy(np.ascontiguousarray(start)).to("cuda", torch.int32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = rounds = 0
    st = None
    for lvl in range(levels - 1, -1, -1):
        if lvl < levels - 1:
            part = part[pars[lvl]].contiguous()
        tau = v["finest"] if lvl == 0 else v["coarse"]
        _, st, _ = ctxs[lvl].refine(part, tau=tau, limit=v["limit"], rb_unweighted=v["rb_unweighted"])
        iters += st["iterations"]
        rounds += st["rebalance_rounds"]
    torch.cuda.synchronize()
    return st["km1_out"], time.perf_counter() - t0, iters, rounds, bool(st["balanced"])


def build(workload, seed):
    import workloads as W
    if workload == "graph":
        hg, start = W.mesh_graph(seed=6)
        return [hg], [], start
    if workload == "rownet":
        hg = W.rownet_matrix(seed=seed, n=4_000_000, k=64)
    else:
        hg = W.sat_like(seed=seed)
    hgs, parents = [hg], []
    for lvl in range(11):
        c, par = W.coarsen(hgs[-1], seed * 1000 + lvl)
        hgs.append(c)
        parents.append(par)
        _log(f"  level {lvl + 1} n={c.n} pins={c.p}")
    return hgs, parents, W.greedy_initial(hgs[-1], seed=seed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["rownet", "sat", "graph"], default="rownet")
    ap.add_argument("--seed", type=int, default=None, help="workload seed (default: the benchmark's)")
    ap.add_argument("--variants", default=",".join(VARIANTS),
                    help="comma-separated subset of the variants (detjet always runs: the ratios need it)")
    args = ap.parse_args()
    names = ["detjet"] + [x for x in args.variants.split(",") if x and x != "detjet"]
    for x in names:
        if x not in VARIANTS:
            ap.error(f"unknown variant {x}")
    seed = args.seed if args.seed is not None else {"rownet": 4, "sat": 5, "graph": 6}[args.workload]
    t0 = time.time()
    hgs, parents, start = build(args.workload, seed)
    _log(f"built in {time.time() - t0:.0f}s")
    ctxs = [JetContext(h) for h in hgs]
    run_variant(ctxs, parents, start, VARIANTS["detjet"])  # graph capture, untimed
    rows = {}
    for name in names:
        v = VARIANTS[name]
        km1, secs, iters, rounds, bal = run_variant(ctxs, parents, start, v)
        rows[name] = {"km1": km1, "seconds": round(secs, 4), "iterations": iters, "rebalance_rounds": rounds,
                      "balanced": bal}
        _log(f"{name}: km1 {km1}, {secs:.2f}s, {iters} iterations, {rounds} rebalancing rounds")
    base = rows["detjet"]["km1"]
    for r in rows.values():
        r["km1_over_detjet"] = round(r["km1"] / base, 5) if base else None
    print(json.dumps({"workload": args.workload, "seed": seed, "levels": len(hgs), "variants": rows}), flush=True)


if __name__ == "__main__":
    main()
