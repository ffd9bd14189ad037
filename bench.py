"""Benchmark: Jet refinement throughput (pins per second per iteration) at k = 64.

Workload (default, "rownet-4M-k64"): the row-net hypergraph of a banded sparse matrix with 4M rows
(4M vertices, 4M nets, Zipf(2.1) net sizes on [2, 10^4], ~40M pins), k = 64, eps = 0.03, seeded
synthetic data.  A 12-level hierarchy (seeded random matching, 2x shrink per level) gives the
multilevel starting point; the coarsest level starts from a seeded greedy balanced partition.

One step = the whole refinement hot path over that hierarchy: for every level from coarsest to
finest, project the partition and run Jet refinement (three temperatures 0.75 / 0.375 / 0, limit 8)
through the C ABI.  Hierarchy construction and context set-up are untimed.

value = sum over levels of (pins of the level x Jet iterations executed there) / step time.

roofline: the first warm-up step brackets every kernel family with device clock marks, nodes of
the captured iteration graphs on the library's stream (per-level breakdown, "kernels_warmup"); the
graphs are then recaptured with marks around the family with the largest total time only, whose
algorithmic bytes per launch (counted on the device) divided by its average launch duration over
the timed steps is reported against the MI355X HBM peak (8 TB/s).  traffic: the counter bytes of
that family per step (TRAFFIC_RECORDS) over its launches per step, while the sources match.

cpu_baseline: the single-threaded CPU oracle, pinned to one core, timed on a bounded sample of the
same workload (one Jet iteration, tau = 0.75, with its rebalancing, on the finest level from the
partition projected from level 1; on the SAT-like workload a 1/20-scale instance of the same
generator), in the same unit, next to the GPU's rate on the same level or sample.

Other workloads: --workload vlsi | sat | batch | graph | coarsen | flows | small (see
build_workload, run_batch, run_coarsen and run_flows).

Prints one JSON line.  Only one GPU is used: --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rownet",
                    choices=["rownet", "vlsi", "sat", "small", "batch", "coarsen", "graph", "flows"])
    ap.add_argument("--autotune-cache", default=None, help="JSON cache of the batch autotuner (batch workload)")
    ap.add_argument("--retune", action="store_true", help="sweep the batch knobs even if cached")
    ap.add_argument("--levels", type=int, default=12, help="hierarchy levels (rownet and sat workloads)")
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the full vertex count (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tau-net", default=os.path.join(ROOT, "paper_2504_12013_amd", "tau_net.bin"),
                    help="temperature network for the learned-vs-fixed comparison (skipped if missing)")
    ap.add_argument("--tau-eval-seeds", default="",
                    help="comma-separated extra workload seeds for the learned-vs-fixed comparison")
    ap.add_argument("--summarize", metavar="DIR", default=None,
                    help="no run: summarise the rocprofv3 CSV output under DIR (kernel stats or one PMC counter) "
                         "per kernel family and exit")
    ap.add_argument("--flow-workers", type=int, default=4,
                    help="flows workload: block pairs of a matching refined at once (JET_OPT_FLOW_WORKERS)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB device to device five times (a kernel of "
                         "known traffic for calibrating the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


WORKLOAD_SEED = {"rownet": 4, "sat": 5}


def build_hierarchy(args, seed):
    """Finest hypergraph of the multilevel workloads for a seed, its hierarchy and the coarsest
    level's greedy start: (hgs finest first, parents, start)."""
    import workloads as W
    if args.workload == "rownet":
        hg = W.rownet_matrix(seed=seed, n=int(4_000_000 * args.scale), k=64)
    else:
        hg = W.sat_like(seed=seed, n=int(20_000_000 * args.scale), p_total=int(200_000_000 * args.scale))
    hgs, parents = [hg], []
    for lvl in range(args.levels - 1):   # as W.hierarchy, with a progress line per level
        c, par = W.coarsen(hgs[-1], seed * 1000 + lvl)
        hgs.append(c)
        parents.append(par)
        log(f"  seed {seed}: level {lvl + 1} n={c.n} pins={c.p}")
    return hgs, parents, W.greedy_initial(hgs[-1], seed=seed)


def build_workload(args):
    import workloads as W
    t0 = time.time()
    if args.workload == "rownet":
        n = int(4_000_000 * args.scale)
        hgs, parents, start = build_hierarchy(args, WORKLOAD_SEED["rownet"])
        hg = hgs[0]
        cfg = {"workload": f"rownet-{n}-k64", "n": n, "m": hg.m, "pins": hg.p, "k": 64, "eps": 0.03,
               "levels": args.levels, "net_sizes": "zipf(2.1) on [2,1e4]", "tau": [0.75, 0.375, 0.0], "limit": 8}
    elif args.workload == "sat":
        n = int(20_000_000 * args.scale)
        hgs, parents, start = build_hierarchy(args, WORKLOAD_SEED["sat"])
        hg = hgs[0]
        cfg = {"workload": f"sat-{n}-k128", "n": n, "m": hg.m, "pins": hg.p, "k": 128, "eps": 0.03,
               "levels": args.levels, "net_sizes": "zipf(1.8) on [2,1e6]", "vertex_weights": "U{1..8}",
               "tau": [0.75, 0.375, 0.0], "limit": 8}
    elif args.workload == "vlsi":
        n = int(1_000_000 * args.scale)
        hg, start = W.vlsi_like(seed=2, n=n, m=int(1.1 * n))
        hgs, parents = [hg], []
        cfg = {"workload": f"vlsi-{n}-k8", "n": n, "m": hg.m, "pins": hg.p, "k": 8, "eps": 0.03, "levels": 1,
               "tau": [0.75], "limit": 12}
    elif args.workload == "graph":
        side = int(round(2048 * args.scale ** 0.5))
        hg, start = W.mesh_graph(side=side, k=64, seed=6)
        hgs, parents = [hg], []
        cfg = {"workload": f"mesh-{hg.n}-k64", "n": hg.n, "m": hg.m, "pins": hg.p, "k": 64, "eps": 0.03, "levels": 1,
               "graph": "triangulated grid, every net of two pins", "tau": [0.75, 0.375, 0.0], "limit": 8}
    else:
        hg, start = W.small_uniform(seed=1)
        hgs, parents = [hg], []
        cfg = {"workload": "uniform-2000-k4", "n": 2000, "m": 4000, "pins": hg.p, "k": 4, "eps": 0.03, "levels": 1,
               "tau": [0.75], "limit": 12}
    log(f"workload built in {time.time() - t0:.1f}s: " + ", ".join(f"L{i}: n={h.n} p={h.p}" for i, h in enumerate(hgs)))
    return hgs, parents, start, cfg


# kernels of each timed family (the names rocprofv3 reports): (kernels of which exactly one runs
# once per family launch, the other kernels of the family)
FAMILIES = {
    "candidates": (("k_candidates", "k_candidates_bits"), ()),
    "candidates_hub": (("k_candidates_hub",), ()),
    "afterburner": (("k_ab_chunks", "k_ab_graph"), ("k_ab_nets", "k_ab_overflow", "k_rg_reduce")),
    "select_moves": (("k_select_moves",), ()),
    "apply": (("k_apply",), ("k_apply_chunks", "k_apply_nets")),
    "rebalance_gain": (("k_rb_list", "k_rb_list_union"), ("k_rb_gain", "k_rb_gain_bits", "k_rb_hub_list",
                                                          "k_rb_hub_accum", "k_rb_hub_finish")),
    "rebalance_select": (("k_rb_select",), ("k_rb_sel_hist", "k_rb_sel_split")),
    "clustering_subround": (("k_co_join", "k_co_settle_small"), ("k_co_rate", "k_co_swap", "k_co_group", "k_co_scan",
                                                                 "k_co_scatter", "k_co_approve", "k_co_apply")),
    # one launch per maximum-flow iteration of the piercing loop: the side weights
    "flow_iteration": (("k_fl_sidew",), ("k_fl_reach", "k_fl_reach_init", "k_fl_gr_level", "k_fl_gr_init",
                                         "k_fl_gr_rest", "k_fl_sweep", "k_fl_active", "k_fl_saturate", "k_fl_sinkflow",
                                         "k_fl_absorb", "k_fl_cand", "k_fl_pierce")),
}


def kernel_base_name(name):
    """k_apply from 'void jet::(anonymous namespace)::k_apply<1>(int4 const*, ...)' or 'k_apply'."""
    name = name.replace("(anonymous namespace)::", "").split("(")[0].split("<")[0].strip()
    return name.split("::")[-1].split(" ")[-1]


# HBM traffic of a family per step, from the two counter passes over whole bench runs (FETCH_SIZE
# x 2.0 + WRITE_SIZE x 1.0, scaled by the copy calibration, divided by the steps traced), valid only
# for the workload and kernel sources it was measured on: the file holding the family's kernels and
# the headers of the kernel directory.  Per launch it is divided by the launches that ran (the
# device loop also dispatches gated launches that return at once; the counters see those too).
TRAFFIC_RECORDS = [
    {"family": "rebalance_gain", "workload": "rownet-4000000-k64", "sources": ["k_rebal.hip"],
     "sources_sha256": "eef8d73e95e5e1be22057613aec8e8888654eb623a815b500085538c59fd30e1", "bytes_per_step": (4193624.4 + 126110.7) * 1e6 / 3},
    {"family": "apply", "workload": "rownet-4000000-k64", "sources": ["k_iter.hip"],
     "sources_sha256": "af9ebc85d5c34ab5edb617c60d490e4d70860a9d5b5993983667048ec65fdf30", "bytes_per_step": (548190.9 + 807364.5) * 1e6 / 3},
    {"family": "candidates", "workload": "rownet-4000000-k64", "sources": ["k_iter.hip"],
     "sources_sha256": "af9ebc85d5c34ab5edb617c60d490e4d70860a9d5b5993983667048ec65fdf30", "bytes_per_step": (804338.3 + 17651.3) * 1e6 / 3},
    {"family": "candidates", "workload": "mesh-4194304-k64", "sources": ["k_iter.hip"],
     "sources_sha256": "af9ebc85d5c34ab5edb617c60d490e4d70860a9d5b5993983667048ec65fdf30", "bytes_per_step": (309890.1 + 21371.1) * 1e6 / 9},
    {"family": "candidates", "workload": "vlsi-1000000-k8", "sources": ["k_iter.hip"],
     "sources_sha256": "af9ebc85d5c34ab5edb617c60d490e4d70860a9d5b5993983667048ec65fdf30", "bytes_per_step": (3516.3 + 575.4) * 1e6 / 5},
]


def traffic_per_launch(family, workload, launches_per_step):
    for rec in TRAFFIC_RECORDS:
        if (rec["family"] == family and rec["workload"] == workload and launches_per_step > 0
                and rec["sources_sha256"] == kernel_sources_sha256(rec["sources"])):
            return rec["bytes_per_step"] / launches_per_step
    return None


def kernel_sources_sha256(files):
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_12013_amd", "csrc")
    for p in sorted([os.path.join(csrc, f) for f in files] + glob.glob(os.path.join(csrc, "*.h"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def summarize(directory, copy_mib):
    """Per-family figures from rocprofv3 CSV output (no GPU needed).

    *_kernel_stats.csv (from --kernel-trace --stats): calls, total and average duration per kernel;
    per family, launches = the calls of the kernels that run once per family launch, and the
    average time per family launch.  *_counter_collection.csv (from --pmc FETCH_SIZE or WRITE_SIZE, KiB per dispatch):
    the counter summed per family and per family launch; with --copy-mib, the last five copy-kernel
    dispatches are the calibration copies of copy_mib MiB each and scale the counter to bytes."""
    import csv
    import glob
    lines = []
    for path in sorted(glob.glob(os.path.join(directory, "*_kernel_stats.csv"))):
        rows = {}
        for r in csv.DictReader(open(path)):  # template instances of one kernel are merged
            b = kernel_base_name(r["Name"])
            if b in rows:
                o = rows[b]
                calls = int(o["Calls"]) + int(r["Calls"])
                tot = float(o["TotalDurationNs"]) + float(r["TotalDurationNs"])
                rows[b] = {"Name": b, "Calls": calls, "TotalDurationNs": tot, "AverageNs": tot / calls}
            else:
                rows[b] = dict(r, Name=b)
        lines.append(f"kernel stats: {os.path.basename(path)}")
        lines.append(f"{'family':18s} {'launches':>9s} {'total ms':>10s} {'avg us/launch':>14s}  kernels")
        for fam, (heads, rest) in FAMILIES.items():
            got = [rows[k] for k in heads + rest if k in rows]
            if not got:
                continue
            hc = [int(rows[k]["Calls"]) for k in heads if k in rows]
            launches = sum(hc) if hc else max(int(r["Calls"]) for r in got)
            tot = sum(float(r["TotalDurationNs"]) for r in got) / 1e6
            det = ", ".join(f"{r['Name']} {r['Calls']}x{float(r['AverageNs']) / 1e3:.1f}us" for r in got)
            lines.append(f"{fam:18s} {launches:9d} {tot:10.1f} {1000 * tot / launches:14.1f}  {det}")
    for path in sorted(glob.glob(os.path.join(directory, "*_counter_collection.csv"))):
        per_kernel, calls, copies = {}, {}, []
        counter = None
        for r in csv.DictReader(open(path)):
            counter = r["Counter_Name"]
            name, val = kernel_base_name(r["Kernel_Name"]), float(r["Counter_Value"])
            per_kernel[name] = per_kernel.get(name, 0.0) + val
            calls[name] = calls.get(name, 0) + 1
            if name == "__amd_rocclr_copyBuffer":
                copies.append(val)
        scale = 1024.0
        lines.append(f"counter {counter}: {os.path.basename(path)} (KiB per dispatch as read)")
        if copy_mib > 0 and len(copies) >= 5:
            cal = sum(copies[-5:]) / 5
            scale = copy_mib * 1048576.0 / cal
            lines.append(f"calibration: a copy of {copy_mib} MiB counts {cal:.1f} KiB -> {scale:.2f} bytes per unit")
        lines.append(f"{'family':18s} {'launches':>9s} {'MB total':>10s} {'MB/launch':>10s}")
        for fam, (heads, rest) in FAMILIES.items():
            got = [k for k in heads + rest if k in per_kernel]
            if not got:
                continue
            hc = [calls[k] for k in heads if k in calls]
            launches = sum(hc) if hc else max(calls[k] for k in got)
            tot = sum(per_kernel[k] for k in got) * scale / 1e6
            lines.append(f"{fam:18s} {launches:9d} {tot:10.1f} {tot / launches:10.3f}")
    for path in sorted(glob.glob(os.path.join(directory, "*_kernel_trace.csv"))):
        lines.extend(summarize_levels(path))
    print("\n".join(lines))


def summarize_levels(path, top=6):
    """Kernel time per level refinement from a *_kernel_trace.csv: each refinement starts with the
    state build of its level (k_build_ns), so with --steps 1 --warmup 0 the groups are the levels
    refined coarsest first, numbered as in the bench's level lines (0 = finest); kernels before
    the first group are set-up."""
    import csv
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    groups, cur = [], {}
    for r in rows:
        name = kernel_base_name(r["Kernel_Name"])
        if name == "k_build_ns":
            groups.append(cur)
            cur = {}
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        c, t = cur.get(name, (0, 0.0))
        cur[name] = (c + 1, t + d)
    groups.append(cur)
    out = [f"kernel time per level refinement: {os.path.basename(path)} (coarsest first; top {top} kernels)"]
    nlev = len(groups) - 1
    for i, g in enumerate(groups):
        tot = sum(t for _, t in g.values()) / 1e3
        det = ", ".join(f"{k} {c}x{t / c:.0f}us" for k, (c, t) in sorted(g.items(), key=lambda kv: -kv[1][1])[:top])
        out.append(f"{'set-up' if i == 0 else f'level {nlev - i}':>8s} {tot:8.1f} ms  {det}")
    return out


def main():
    args = parse()
    if args.summarize:
        summarize(args.summarize, args.copy_mib)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2504_12013_amd import JetContext
    from paper_2504_12013_amd import jet

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "coarsen":
        return run_coarsen(args)
    if args.workload == "flows":
        return run_flows(args)
    hgs, parents, start, cfg = build_workload(args)
    tau, limit = tuple(cfg["tau"]), cfg["limit"]
    t0 = time.time()
    ctxs = [JetContext(h) for h in hgs]
    par_dev = [torch.from_numpy(p).to("cuda").long() for p in parents]
    start_dev = torch.from_numpy(start).to("cuda")
    torch.cuda.synchronize()
    log(f"contexts ready in {time.time() - t0:.1f}s")

    finest_in = {}
    loop_counts = [0, 0]  # host polls and iteration pieces over the timed steps
    finest_time = [0.0, 0]  # seconds and pins x iterations of the finest level over the timed steps

    def step(verbose=False, timed=False):
        part = start_dev.clone()
        work = 0
        km1 = None
        iters = 0
        for lvl in range(len(hgs) - 1, -1, -1):
            if lvl < len(hgs) - 1:
                part = part[par_dev[lvl]].contiguous()
            if lvl == 0 and "part" not in finest_in:
                finest_in["part"] = part.cpu().numpy()
            t_l = time.perf_counter()
            rc, st, _ = ctxs[lvl].refine(part, tau=tau, limit=limit)
            if verbose:
                log(f"  level {lvl}: n={hgs[lvl].n} p={hgs[lvl].p} iterations {st['iterations']} "
                    f"rebalance rounds {st['rebalance_rounds']} km1 {st['km1_in']} -> {st['km1_out']} "
                    f"{1000 * (time.perf_counter() - t_l):.1f} ms")
            work += hgs[lvl].p * st["iterations"]
            iters += st["iterations"]
            if timed:
                polls, pieces = ctxs[lvl].loop_counts()
                loop_counts[0] += polls
                loop_counts[1] += pieces
            if timed and lvl == 0:  # refine returns after the level's work finished (it synchronises)
                finest_time[0] += time.perf_counter() - t_l
                finest_time[1] += hgs[lvl].p * st["iterations"]
            km1 = st["km1_out"]
            balanced = st["balanced"]
        return work, km1, iters, balanced, part

    # The first warm-up step brackets every kernel family with events (per-level breakdown); the
    # timed steps bracket only the family that dominated it, which keeps the events' host work
    # (a few microseconds per launch) small inside the timed region.
    warm_fams = {}
    for i in range(args.warmup):
        if i == 0:
            for c in ctxs:
                c.prof_enable(True)
        w, km1, it, bal, _ = step(verbose=(i == 0))
        log(f"warmup {i}: km1 {km1} iterations {it} balanced {bal}")
        if i == 0:
            for lvl in range(len(hgs) - 1, -1, -1):
                fam = ctxs[lvl].prof_read()
                log(f"  level {lvl} kernels: " + ", ".join(
                    f"{k} {v['launches']}x{1000 * v['total_ms'] / max(1, v['launches']):.0f}us"
                    for k, v in sorted(fam.items(), key=lambda kv: -kv[1]["total_ms"])))
                for name, e in fam.items():
                    f = warm_fams.setdefault(name, {"launches": 0, "total_ms": 0.0, "alg_bytes": 0.0})
                    for key in f:
                        f[key] += e[key]
                ctxs[lvl].prof_enable(False)
    mask = (1 << len(jet.PROF_FAMILIES)) - 1
    if warm_fams:
        mask = 1 << jet.PROF_FAMILIES.index(max(warm_fams.items(), key=lambda kv: kv[1]["total_ms"])[0])
    for c in ctxs:
        c.set_option(jet.JET_OPT_PROF_FAMILIES, mask)
        c.prof_enable(True)
    # one more untimed step: the iteration graphs, recaptured with the new marks, are built here
    step()
    for c in ctxs:
        c.prof_enable(True)  # counters back to zero (the graphs stay)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    total_work = 0
    for i in range(args.steps):
        w, km1, it, bal, part = step(timed=True)
        total_work += w
        log(f"step {i}: km1 {km1} iterations {it} pins*iterations {w}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    value = total_work / elapsed
    fams = {}
    for c in ctxs:
        for name, e in c.prof_read().items():
            f = fams.setdefault(name, {"launches": 0, "total_ms": 0.0, "alg_bytes": 0.0})
            for key in f:
                f[key] += e[key]
        c.prof_enable(False)
    for name, f in sorted(fams.items(), key=lambda kv: -kv[1]["total_ms"]):
        log(f"  {name:18s} launches {f['launches']:7d}  total {f['total_ms']:9.1f} ms  "
            f"avg {1000 * f['total_ms'] / max(1, f['launches']):8.1f} us  "
            f"alg {f['alg_bytes'] / max(1e-9, f['total_ms']) / 1e6:8.1f} GB/s")
    dom_name, dom = max(fams.items(), key=lambda kv: kv[1]["total_ms"])
    achieved = dom["alg_bytes"] / (dom["total_ms"] * 1e-3) / 1e9 if dom["alg_bytes"] > 0 else None
    traffic = traffic_per_launch(dom_name, cfg["workload"], dom["launches"] / args.steps)
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                "frac": None if achieved is None else achieved / 8000.0, "traffic": traffic,
                "launches": dom["launches"], "avg_launch_us": 1000.0 * dom["total_ms"] / dom["launches"],
                "alg_bytes_per_launch": dom["alg_bytes"] / dom["launches"],
                "share_of_step_time": dom["total_ms"] / (elapsed * 1000.0)}
    general = None
    if args.workload == "graph":  # untimed: the same step with the general (per-net) afterburner
        general = {}
        for on in (0, 1):
            for c in ctxs:
                c.set_option(jet.JET_OPT_GRAPH_KERNELS, on)
                c.set_option(jet.JET_OPT_PROF_FAMILIES, (1 << len(jet.PROF_FAMILIES)) - 1)
                c.prof_enable(True)
            step()  # graphs recaptured
            for c in ctxs:
                c.prof_enable(True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            fam = {}
            for c in ctxs:
                for name, e in c.prof_read().items():
                    fam[name] = fam.get(name, 0.0) + e["total_ms"]
                c.prof_enable(False)
            general["graph_kernels" if on else "general"] = {
                "ms_per_step": 1000.0 * (time.perf_counter() - t1), "afterburner_ms": round(fam.get("afterburner", 0.0), 3)}
        log(f"afterburner per step: graph kernels {general['graph_kernels']}, general {general['general']}")
    learned = None
    if os.path.exists(args.tau_net) and args.workload in WORKLOAD_SEED:
        learned = learned_vs_fixed(args, hgs, parents, start, ctxs)
    cpu = None
    if args.no_cpu_baseline:
        pass
    elif args.workload == "sat":
        # one oracle iteration on the finest level takes some twenty minutes: the sample is a
        # 1/20-scale instance of the same generator instead, timed on the GPU too
        import workloads as W
        n_s, p_s = hgs[0].n // 20, hgs[0].p // 20
        hs = W.sat_like(seed=5, n=n_s, p_total=p_s)
        ps = W.part_uniform(hs.n, hs.k, seed=5)
        cpu = cpu_baseline(hs, ps, f"a 1/20-scale SAT-like instance of the same generator (seed 5, n={hs.n}, "
                                   f"pins={hs.p}, k={hs.k}) from a seeded uniform partition")
        cpu["gpu_same_sample"] = gpu_same_sample(hs, ps)
    else:
        cpu = cpu_baseline(hgs[0], finest_in["part"], f"the finest level (n={hgs[0].n}, pins={hgs[0].p}, "
                                                      f"k={hgs[0].k}) from the partition projected from level 1")
    if cpu is not None and finest_time[0] > 0:
        cpu["gpu_same_level"] = {"value": finest_time[1] / finest_time[0], "unit": "pins/s",
                                 "what": "GPU pins x iterations / time on the finest level alone, timed steps"}
    out = {"metric": "Jet pins/s per iteration at k=64" if cfg["k"] == 64 else "Jet pins/s per iteration",
           "value": value, "unit": "pins/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1000.0 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int32", "data": "synthetic", "config": cfg,
           "km1_final": km1, "balanced": bool(bal), "roofline": roofline, "cpu_baseline": cpu,
           "learned_tau": learned, "afterburner_forms": general,
           "host_polls_per_step": loop_counts[0] / args.steps, "pieces_per_step": loop_counts[1] / args.steps,
           "kernels": {k: {"launches": v["launches"], "total_ms": round(v["total_ms"], 3)} for k, v in fams.items()},
           "kernels_warmup": {k: {"launches": v["launches"], "total_ms": round(v["total_ms"], 3)}
                              for k, v in warm_fams.items()}}
    print(json.dumps(out), flush=True)
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 5 copies of {args.copy_mib} MiB")


def run_batch(args):
    """512 independent hypergraphs (n log-uniform in [1e3, 1e5], m = 1.2 n, Zipf(2.1) sizes capped at
    1000, k in {2, 8, 32}) refined in one batched call per step (tau 0.75, limit 12); knobs from the
    autotuner.  value = sum over hypergraphs of pins x iterations / step time."""
    import torch
    import workloads as W
    from paper_2504_12013_amd import JetBatch
    from paper_2504_12013_amd import autotune
    t0 = time.time()
    items = W.batch_set(seed=3)
    hgs = [h for h, _ in items]
    starts = [torch.from_numpy(p).to("cuda") for _, p in items]
    log(f"batch built in {time.time() - t0:.1f}s: {len(hgs)} hypergraphs, {sum(h.n for h in hgs)} vertices, "
        f"{sum(h.p for h in hgs)} pins")
    t0 = time.time()
    batch = JetBatch(hgs)
    log(f"batch contexts ready in {time.time() - t0:.1f}s")
    kw = dict(tau=(0.75,), limit=12)
    key, knobs = autotune.tuned(batch, hgs, starts, cache_path=args.autotune_cache or autotune.DEFAULT_CACHE,
                                retune=args.retune, log=log, **kw)
    log(f"autotuned {key}: {knobs}")

    def step():
        parts = [p.clone() for p in starts]
        torch.cuda.synchronize()
        rc, stats, rcs = batch.refine(parts, replays=knobs["replays"], **kw)
        return parts, stats

    # warm-up with every family marked (breakdown), then the dominant family only, graph recaptured
    # in one more untimed step
    from paper_2504_12013_amd import jet
    batch.prof_enable(True)
    for i in range(args.warmup):
        step()
    warm = batch.prof_read()
    for name, e in sorted(warm.items(), key=lambda kv: -kv[1]["total_ms"]):
        log(f"  warm-up {name:18s} launches {e['launches']:6d} total {e['total_ms']:8.1f} ms")
    dom_name = max(warm.items(), key=lambda kv: kv[1]["total_ms"])[0] if warm else "candidates"
    batch.set_option(jet.JET_OPT_PROF_FAMILIES, 1 << jet.PROF_FAMILIES.index(dom_name))
    batch.prof_enable(True)
    step()
    batch.prof_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    work = 0
    for i in range(args.steps):
        parts, stats = step()
        w = sum(h.p * s["iterations"] for h, s in zip(hgs, stats))
        work += w
        log(f"step {i}: pins*iterations {w}, km1 total {sum(s['km1_out'] for s in stats)}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    fams = batch.prof_read()
    dom = fams.get(dom_name, {"launches": 0, "total_ms": 0.0, "alg_bytes": 0.0})
    achieved = dom["alg_bytes"] / (dom["total_ms"] * 1e-3) / 1e9 if dom["total_ms"] > 0 else None
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                "frac": None if achieved is None else achieved / 8000.0, "traffic": None,
                "launches": dom["launches"],
                "avg_launch_us": 1000.0 * dom["total_ms"] / max(1, dom["launches"]),
                "alg_bytes_per_launch": dom["alg_bytes"] / max(1, dom["launches"]),
                "share_of_step_time": dom["total_ms"] / (elapsed * 1000.0)}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        order = sorted(range(len(hgs)), key=lambda i: hgs[i].p)
        done, pw, t1 = 0, 0, time.perf_counter()
        allowed = sorted(os.sched_getaffinity(0))
        os.sched_setaffinity(0, {allowed[-1]})  # one core, restored afterwards
        try:
            for i in order[::16]:        # every 16th hypergraph by size, about 32 of them
                _, _, st, _ = oracle.refine(hgs[i], items[i][1], **kw)
                pw += hgs[i].p * st["iterations"]
                done += 1
                if time.perf_counter() - t1 > 20:
                    break
            dt = time.perf_counter() - t1
        finally:
            os.sched_setaffinity(0, allowed)
        cpu = {"value": pw / dt, "unit": "pins/s", "cores": 1, "kind": "oracle", "nproc": os.cpu_count(),
               "sample": f"{done} of the 512 hypergraphs (every 16th by size, from the smallest), whole "
                         f"refinement each, single thread on {cpu_model()}; {dt:.1f} s"}
    out = {"metric": "Jet pins/s per iteration (batched)", "value": work / elapsed, "unit": "pins/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000.0 * elapsed / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "batch-512-mixed", "hypergraphs": len(hgs), "pins": sum(h.p for h in hgs),
                      "k": [2, 8, 32], "eps": 0.03, "tau": [0.75], "limit": 12, "autotune": knobs},
           "km1_total": sum(s["km1_out"] for s in stats), "roofline": roofline, "cpu_baseline": cpu,
           "kernels_warmup": {k: {"launches": v["launches"], "total_ms": round(v["total_ms"], 3)}
                              for k, v in warm.items()}}
    print(json.dumps(out), flush=True)


def run_coarsen(args):
    """The clustering pass of one coarsening level (jet_coarsen, Section 6 / Algorithm 4) on the
    VLSI-like hypergraph (1M vertices, 3.85M pins): seeded vertex order, the paper's schedule (100
    one-vertex sub-rounds, doubling up to 1% of n), maximum cluster weight ceil(W / (160 k)) at
    k = 8.  A step is one pass; value = pins / pass time.  The roofline is the pass's: algorithmic
    bytes = 16 n + 28 p + 8 sum_e |e| (|e| - 1) (incidence offsets; per incident net its ID, offsets
    and rating; per other pin of the net its ID and cluster label) over the pass time."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2504_12013_amd import JetContext
    hg, _ = W.vlsi_like(seed=2, n=int(1_000_000 * args.scale), m=int(1_100_000 * args.scale))
    Wt = int(hg.vtx_w.astype(np.int64).sum())
    wmax = -(-Wt // (160 * 8))
    order_h = np.random.default_rng(2).permutation(hg.n).astype(np.int32)
    order = torch.from_numpy(order_h).to("cuda")
    ctx = JetContext(hg)
    sizes = np.diff(hg.off).astype(np.int64)
    alg = 16.0 * hg.n + 28.0 * hg.p + 8.0 * float((sizes * (sizes - 1)).sum())
    for _ in range(args.warmup):
        _, cnt = ctx.coarsen(order, wmax)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, cnt = ctx.coarsen(order, wmax)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    log(f"coarsen: {cnt} clusters from {hg.n} vertices, {1000 * dt:.2f} ms per pass")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        allowed = sorted(os.sched_getaffinity(0))
        os.sched_setaffinity(0, {allowed[-1]})
        try:
            reps, t1 = 0, time.perf_counter()
            while reps < 3 or time.perf_counter() - t1 < 10:
                olab, ocnt = oracle.coarsen(hg, order_h, wmax)
                reps += 1
            cdt = (time.perf_counter() - t1) / reps
        finally:
            os.sched_setaffinity(0, allowed)
        cpu = {"value": hg.p / cdt, "unit": "pins/s", "cores": 1, "kind": "oracle", "nproc": os.cpu_count(),
               "sample": f"the same pass ({reps} repetitions), single thread on {cpu_model()}; "
                         f"{cdt:.2f} s per pass; same clusters: {ocnt == cnt}"}
    achieved = alg / dt / 1e9
    out = {"metric": "clustering pass pins/s", "value": hg.p / dt, "unit": "pins/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000.0 * dt, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": f"coarsen-vlsi-{hg.n}", "n": hg.n, "m": hg.m, "pins": hg.p,
                      "max_cluster_weight": wmax, "initial_single": 100, "cap_div": 100, "clusters": cnt},
           "roofline": {"bound": "hbm", "kernel": "clustering pass", "achieved": achieved, "peak": 8000.0,
                        "unit": "GB/s", "frac": achieved / 8000.0, "traffic": None, "alg_bytes_per_pass": alg},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def run_flows(args):
    """Flow-based refinement (Section 5) after Jet, as the paper runs it on a level: the VLSI-like
    hypergraph (1M vertices, 3.85M pins, k = 8) refined by Jet (0.75 / 0.375 / 0, limit 8), then one
    round of the k-way flow schedule (every quotient-graph edge once), untimed warm-up.  A step is
    that round from the same Jet partition; value = pins / round time.  roofline: the round's
    algorithmic bytes are one read of the flow network per maximum-flow iteration (16 bytes per arc:
    head, tail, residual), a lower bound on what the piercing loop must touch, over the round time;
    the loop is bound by the latency of its dependent searches, not by bandwidth."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2504_12013_amd import JetContext
    n = int(1_000_000 * args.scale)
    hg, start = W.vlsi_like(seed=2, n=n, m=int(1.1 * n))
    ctx = JetContext(hg)
    from paper_2504_12013_amd import jet as J
    ctx.set_option(J.JET_OPT_FLOW_WORKERS, args.flow_workers)
    p = torch.from_numpy(start).to("cuda", torch.int32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.refine(p, tau=(0.75, 0.375, 0.0), limit=8)
    torch.cuda.synchronize()
    jet_s = time.perf_counter() - t0
    jet_part = p.clone()
    for _ in range(args.warmup):
        ctx.flow_refine(jet_part.clone(), max_rounds=1)
    torch.cuda.synchronize()
    times, st = [], None
    for _ in range(args.steps):
        q = jet_part.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.flow_refine(q, max_rounds=1)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"flows: round {1000 * times[-1]:.0f} ms, km1 {st['km1_in']} -> {st['km1_out']}, {st['flow_calls']} "
            f"maximum-flow iterations over {st['pairs']} pairs")
    dt = sum(times) / len(times)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # a bounded sample: the same generator at 20,000 vertices, after the oracle's Jet, one round
        sh, sstart = W.vlsi_like(seed=2, n=20_000, m=22_000)
        spart, _, _, _ = oracle.refine(sh, sstart, tau=(0.75, 0.375, 0.0), limit=8)
        sctx = JetContext(sh)
        sq = torch.from_numpy(spart).to("cuda", torch.int32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gst = sctx.flow_refine(sq, max_rounds=1)
        torch.cuda.synchronize()
        gdt = time.perf_counter() - t0
        allowed = sorted(os.sched_getaffinity(0))
        os.sched_setaffinity(0, {allowed[-1]})
        try:
            t1 = time.perf_counter()
            out, ost = oracle.flow_refine(sh, spart, max_rounds=1)
            cdt = time.perf_counter() - t1
        finally:
            os.sched_setaffinity(0, allowed)
        same = bool(np.array_equal(out, sq.cpu().numpy()))
        cpu = {"value": sh.p / cdt, "unit": "pins/s", "cores": 1, "kind": "oracle", "nproc": os.cpu_count(),
               "sample": f"one round of the k-way flow schedule after Jet on the same generator at 20,000 vertices "
                         f"({sh.p} pins), single thread on {cpu_model()}; {cdt:.1f} s; same partition as the GPU: "
                         f"{same}",
               "gpu_same_sample": {"value": sh.p / gdt, "unit": "pins/s", "seconds": round(gdt, 3),
                                   "km1": [gst["km1_in"], gst["km1_out"]]}}
    alg = 16.0 * st["arcs"]
    achieved = alg / dt / 1e9
    out = {"metric": "flow refinement round pins/s", "value": hg.p / dt, "unit": "pins/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000.0 * dt, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"flows-vlsi-{n}-k8", "n": n, "m": hg.m, "pins": hg.p, "k": 8, "eps": 0.03,
                      "alpha": 16, "rounds": 1, "after": "Jet 0.75/0.375/0, limit 8",
                      "flow_workers": args.flow_workers},
           "flows": {"km1_jet": st["km1_in"], "km1_flows": st["km1_out"], "pairs": st["pairs"],
                     "accepted": st["accepted"], "iterations": st["flow_calls"], "moved": st["moved"],
                     "jet_seconds": round(jet_s, 4), "flows_over_jet_time": round(dt / jet_s, 1)},
           "roofline": {"bound": "hbm", "kernel": "flow round (network reads)", "achieved": achieved,
                        "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0, "traffic": None,
                        "alg_bytes_per_round": alg},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def learned_vs_fixed(args, hgs, parents, start, ctxs):
    """Final metric and GPU time of the whole hierarchy with the fixed schedule and with network
    temperatures, on this workload and on --tau-eval-seeds.  If the learned run takes more than
    1.05x the fixed run's time, the fixed run gets extra tau = 0 rounds until its time matches."""
    import numpy as np
    from paper_2504_12013_amd import TauNet
    from paper_2504_12013_amd.tau_training import fixed_at_equal_time, run_hierarchy
    net = TauNet(path=args.tau_net)
    rows = []
    cases = [WORKLOAD_SEED[args.workload]] + [int(x) for x in args.tau_eval_seeds.split(",") if x.strip()]
    for sd in cases:
        if sd == WORKLOAD_SEED[args.workload]:
            hh, pp, st0, cc = hgs, parents, start, ctxs
        else:
            t0 = time.time()
            hh, pp, st0 = build_hierarchy(args, sd)
            cc = None
            log(f"learned vs fixed: seed {sd} built in {time.time() - t0:.0f}s")
        kf, tf, itf, _, _ = run_hierarchy(hh, pp, st0, None, ctxs=cc)
        kl, tl, itl, taus, fell_back = run_hierarchy(hh, pp, st0, net, ctxs=cc)
        kfe, tfe, rounds = (kf, tf, 3) if tl <= 1.05 * tf else fixed_at_equal_time(hh, pp, st0, tl, ctxs=cc)
        rows.append({"seed": sd, "km1_fixed": kf, "s_fixed": round(tf, 4), "iters_fixed": itf, "km1_learned": kl,
                     "s_learned": round(tl, 4), "iters_learned": itl, "km1_fixed_equal_time": kfe,
                     "fixed_rounds_equal_time": rounds, "s_fixed_equal_time": round(tfe, 4),
                     "rounds_on_fixed_tau": fell_back, "rounds_total": 3 * len(hh),
                     "tau_finest": [round(t, 4) for t in taus[-1]], "tau_coarsest": [round(t, 4) for t in taus[0]]})
        log(f"learned vs fixed, seed {sd}: km1 {kl} vs {kf} (equal time {kfe}), {tl:.2f}s vs {tf:.2f}s")
    ratio = float(np.exp(np.mean([np.log(r["km1_learned"] / r["km1_fixed_equal_time"]) for r in rows])))
    return {"net": os.path.relpath(args.tau_net, ROOT), "geomean_km1_learned_over_fixed": ratio, "runs": rows}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def gpu_same_sample(hg, part):
    """The library on the cpu_baseline's sample, same call (one iteration, tau 0.75): pins x
    iterations / s over three runs after one untimed run (graph capture)."""
    import torch
    from paper_2504_12013_amd import JetContext
    ctx = JetContext(hg)
    src = torch.from_numpy(part).to("cuda")
    ctx.refine(src.clone(), tau=(0.75,), limit=1, max_iters=1)
    work, dt = 0, 0.0
    for _ in range(3):
        p = src.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st, _ = ctx.refine(p, tau=(0.75,), limit=1, max_iters=1)
        torch.cuda.synchronize()
        dt += time.perf_counter() - t0
        work += hg.p * st["iterations"]
    ctx.close()
    return {"value": work / dt, "unit": "pins/s", "what": "GPU, same sample and call, mean of 3 runs"}


def cpu_baseline(hg, part, what):
    """The oracle (single thread, pinned to one core) on one Jet iteration of hg from part:
    pins x iterations / s."""
    import oracle
    nproc = os.cpu_count()
    allowed = sorted(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {allowed[-1]})  # this thread only, restored afterwards
    try:
        t0 = time.perf_counter()
        _, rc, st, _ = oracle.refine(hg, part, tau=(0.75,), limit=1, max_iters=1)
        dt = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, allowed)
    log(f"cpu baseline: oracle {st['iterations']} iteration(s), {st['rebalance_rounds']} rebalancing rounds, "
        f"{dt:.1f} s")
    return {"value": hg.p * st["iterations"] / dt, "unit": "pins/s", "cores": 1, "kind": "oracle",
            "pinned_cpu": allowed[-1], "nproc": nproc, "cpus_allowed": len(allowed),
            "sample": f"one Jet iteration (tau 0.75, limit 1, with its {st['rebalance_rounds']} rebalancing rounds) "
                      f"on {what}; single thread on {cpu_model()}; {dt:.1f} s"}


if __name__ == "__main__":
    main()
