"""Multilevel deterministic Jet with the synchronous clustering of Section 6 on the GPU.

The coarsening phase alternates a clustering pass (jet_coarsen, Algorithm 4) with the contraction
of its clusters until the hypergraph is small enough for initial partitioning; the refinement
then runs deterministic Jet on every level, coarsest to finest (Sections 2 and 4).  The paper
reuses an existing contraction; here it is the host contraction of the synthetic-input library
(summed vertex weights, nets mapped and deduplicated, single-pin nets dropped).

Clustering schedules compared (Section 6 and its experiments on coarsening):
  prefix-doubling  100 single-vertex sub-rounds, then doubling up to 1 % of the vertices (the paper)
  three-equal      the vertex order split into three sub-rounds of equal size (the earlier
                   deterministic coarsening's schedule; the rating fix and swap prevention stay on)
and, for reference, the random-matching hierarchy the refinement benchmarks use.

Readings where the paper is silent: coarsening stops once a level has at most 160 k vertices or
a pass removes fewer than 1 % of them; the maximum cluster weight is ceil(c(V) / (160 k)); each
level's vertex order is a seeded permutation; coarse vertices are numbered in increasing order of
their cluster's label.

    python -m paper_2504_12013_amd.multilevel --workload rownet    (4M vertices, k = 64)
    python -m paper_2504_12013_amd.multilevel --workload vlsi      (1M vertices, k = 8)
    ... --flows 1    also DetJet with one round of flow-based refinement after every level
Prints one JSON object with, per hierarchy, its levels, coarsening and refinement seconds and the
final connectivity metric.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from .ablations import VARIANTS, run_variant
from .jet import JetContext

SCHEDULES = ("prefix-doubling", "three-equal")


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def level_order(n: int, seed: int, level: int) -> np.ndarray:
    """The seeded vertex order of one clustering pass."""
    return np.random.default_rng([seed, level]).permutation(n).astype(np.int32)


def max_cluster_weight(hg, contraction_limit: int) -> int:
    total = int(hg.n if hg.vtx_w is None else hg.vtx_w.astype(np.int64).sum())
    return -(-total // contraction_limit)


def cluster_level(ctx: JetContext, hg, order: np.ndarray, wmax: int, schedule: str):
    """One clustering pass on the GPU: returns (label int32[n] as vertex IDs, clusters)."""
    if schedule == "prefix-doubling":
        label, cnt = ctx.coarsen(torch.from_numpy(order).to("cuda"), wmax)
        return label.cpu().numpy(), cnt
    if schedule != "three-equal":
        raise ValueError(f"unknown schedule {schedule}")
    label = torch.arange(hg.n, dtype=torch.int32, device="cuda")
    vw = np.ones(hg.n, np.int64) if hg.vtx_w is None else hg.vtx_w.astype(np.int64)
    cw = torch.from_numpy(vw).to("cuda")
    for part in np.array_split(order, 3):
        ctx.coarsen_subround(label, cw, torch.from_numpy(np.ascontiguousarray(part)).to("cuda"), wmax)
    lab = label.cpu().numpy()
    return lab, int(np.unique(lab).size)


def compact(label: np.ndarray):
    """parent[v] = coarse vertex of v, numbered 0..c-1 in increasing order of the cluster labels."""
    uniq, inv = np.unique(label, return_inverse=True)
    return inv.astype(np.int32), int(uniq.size)


def cluster_hierarchy(hg, seed: int, schedule: str = "prefix-doubling", max_levels: int = 64, log=None):
    """Coarsens with GPU clustering passes and host contraction.  Returns (hypergraphs finest
    first, parents[l] mapping level l to l + 1, contexts per level, per-level records)."""
    import workloads as W
    limit = 160 * hg.k
    wmax = max_cluster_weight(hg, limit)
    hgs, parents, ctxs, recs = [hg], [], [JetContext(hg)], []
    while hgs[-1].n > limit and len(hgs) < max_levels:
        cur, ctx = hgs[-1], ctxs[-1]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        label, cnt = cluster_level(ctx, cur, level_order(cur.n, seed, len(hgs) - 1), wmax, schedule)
        t1 = time.perf_counter()
        if cnt > cur.n - cur.n // 100:
            break
        parent, nc = compact(label)
        assert nc == cnt
        coarse = W.contract(cur, parent, nc)
        t2 = time.perf_counter()
        recs.append({"n": cur.n, "clusters": nc, "cluster_s": round(t1 - t0, 4), "contract_s": round(t2 - t1, 4)})
        if log:
            log(f"  {schedule} level {len(hgs)}: n={nc} pins={coarse.p} (clustering {1000 * (t1 - t0):.1f} ms, "
                f"contraction {1000 * (t2 - t1):.0f} ms)")
        hgs.append(coarse)
        parents.append(parent)
        ctxs.append(JetContext(coarse))
    return hgs, parents, ctxs, recs


def matching_hierarchy(hg, seed: int, levels: int, log=None):
    import workloads as W
    hgs, parents = [hg], []
    t0 = time.perf_counter()
    for lvl in range(levels - 1):
        c, par = W.coarsen(hgs[-1], seed * 1000 + lvl)
        hgs.append(c)
        parents.append(par)
    secs = time.perf_counter() - t0
    if log:
        log(f"  random matching: {levels} levels, coarsest n={hgs[-1].n} ({secs:.1f} s)")
    return hgs, parents, [JetContext(h) for h in hgs], secs


def refine_with_flows(ctxs, parents, start, flow_rounds: int):
    """DetJet on every level, coarsest to finest, each level followed by flow_rounds rounds of the
    k-way flow schedule (Section 5), as the paper's configuration with flows runs them.  Returns
    (final metric, total seconds, seconds in flows, metric gained by flows)."""
    v = VARIANTS["detjet"]
    pars = [torch.from_numpy(p).to("cuda").long() for p in parents]
    part = torch.from_numpy(np.ascontiguousarray(start)).to("cuda", torch.int32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flow_s, gained = 0.0, 0
    for lvl in range(len(ctxs) - 1, -1, -1):
        if lvl < len(ctxs) - 1:
            part = part[pars[lvl]].contiguous()
        ctxs[lvl].refine(part, tau=v["coarse"], limit=v["limit"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = ctxs[lvl].flow_refine(part, max_rounds=flow_rounds)
        torch.cuda.synchronize()
        flow_s += time.perf_counter() - t1
        gained += st["km1_in"] - st["km1_out"]
        _log(f"  level {lvl}: flows km1 {st['km1_in']} -> {st['km1_out']} in {time.perf_counter() - t1:.1f} s "
             f"({st['flow_calls']} maximum-flow iterations)")
    km1 = ctxs[0].km1(part)
    torch.cuda.synchronize()
    return km1, time.perf_counter() - t0, flow_s, gained


def build_input(workload: str, seed: int, n: int = 0):
    import workloads as W
    if workload == "rownet":
        return W.rownet_matrix(seed=seed, n=n or 4_000_000, k=64)
    if workload == "vlsi":
        n = n or 1_000_000
        return W.vlsi_like(seed=seed, n=n, m=int(1.1 * n))[0]
    return W.sat_like(seed=seed)


def main():
    import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["rownet", "vlsi", "sat"], default="rownet")
    ap.add_argument("--seed", type=int, default=None, help="workload seed (default: the benchmark's)")
    ap.add_argument("--n", type=int, default=0, help="vertices of the row-net or VLSI-like input (default: full size)")
    ap.add_argument("--flows", type=int, default=0,
                    help="also refine the prefix-doubling hierarchy with this many rounds of flows after Jet "
                         "on every level (0: no)")
    args = ap.parse_args()
    seed = args.seed if args.seed is not None else {"rownet": 4, "vlsi": 2, "sat": 5}[args.workload]
    t0 = time.time()
    hg = build_input(args.workload, seed, args.n)
    _log(f"{args.workload}: n={hg.n} m={hg.m} pins={hg.p} k={hg.k} ({time.time() - t0:.0f} s)")
    out = {"workload": args.workload, "seed": seed, "n": hg.n, "pins": hg.p, "k": hg.k, "hierarchies": {}}
    detjet = VARIANTS["detjet"]
    runs = []
    for sched in SCHEDULES:
        t1 = time.perf_counter()
        hgs, parents, ctxs, recs = cluster_hierarchy(hg, seed, sched, log=_log)
        runs.append((sched, hgs, parents, ctxs, {"coarsening_s": round(time.perf_counter() - t1, 3),
                                                  "clustering_s": round(sum(r["cluster_s"] for r in recs), 4),
                                                  "levels": len(hgs), "coarsest_n": hgs[-1].n}))
    hgs, parents, ctxs, secs = matching_hierarchy(hg, seed, 12, log=_log)
    runs.append(("random-matching", hgs, parents, ctxs, {"coarsening_s": round(secs, 3), "levels": len(hgs),
                                                         "coarsest_n": hgs[-1].n}))
    for name, hgs, parents, ctxs, rec in runs:
        start = W.greedy_initial(hgs[-1], seed=seed)
        run_variant(ctxs, parents, start, detjet)  # graph capture, untimed
        km1, secs, iters, rounds, bal = run_variant(ctxs, parents, start, detjet)
        rec.update({"km1": km1, "refine_s": round(secs, 4), "iterations": iters, "rebalance_rounds": rounds,
                    "balanced": bal})
        _log(f"{name}: km1 {km1}, refinement {secs:.2f} s, {iters} iterations")
        out["hierarchies"][name] = rec
    if args.flows > 0:
        name, hgs, parents, ctxs, _ = runs[0]
        start = W.greedy_initial(hgs[-1], seed=seed)
        km1, secs, fsecs, gained = refine_with_flows(ctxs, parents, start, args.flows)
        out["hierarchies"][name + "+flows"] = {"km1": km1, "refine_s": round(secs, 3), "flows_s": round(fsecs, 3),
                                               "km1_gained_by_flows": gained, "flow_rounds_per_level": args.flows}
        _log(f"{name}+flows: km1 {km1}, {secs:.2f} s ({fsecs:.2f} s in flows)")
    base = out["hierarchies"]["prefix-doubling"]["km1"]
    for r in out["hierarchies"].values():
        r["km1_over_prefix_doubling"] = round(r["km1"] / base, 5) if base else None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
