"""Training data, training and evaluation of the temperature network.

The paper runs every level with a fixed schedule of temperatures (three rounds, tau = 0.75, 0.375,
0; Section 4.1 and the temperature study of Section 7).  Here a network may pick tau per level and
round instead.  Its labels come from sweeps of the plain method:

  for every level (coarsest first) and round r: from the current partition, run one Jet round
  (jet_refine, one temperature, limit 8) for every tau on a grid, followed by the fixed schedule's
  remaining rounds (look-ahead); the label tau* is the grid value whose end-of-level result is best
  by the quality key (overload, metric), ties broken toward the fixed schedule's tau_r, then toward
  the smaller tau; the sweep continues from tau*'s one-round partition.  Without look-ahead the
  key is that of the one-round result.

The features are those of jet_tau_features (level statistics from jet_level_stats).  Training is
mean squared error with Adam on minibatches, all in the library's FP32 kernels (TauNet).  Sweeps,
training and evaluation all run the library on the GPU; nothing here computes partitions itself.

    python -m paper_2504_12013_amd.tau_training --out paper_2504_12013_amd/tau_net.bin
    python -m paper_2504_12013_amd.tau_training --evaluate sat --seeds 51,52,53   (held-out evaluation)
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

from .jet import JetContext, TauNet, jet_tau_features

GRID = tuple(i / 8 for i in range(9))
FIXED = (0.75, 0.375, 0.0)
LIMIT = 8


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _key(st):
    return (max(0, st["max_block_weight"] - st["lmax"]), st["km1_out"])


def sweep(hgs, parents, start, grid=GRID, fixed=FIXED, limit=LIMIT, lookahead=True):
    """Labelled (features, tau*) pairs of one hierarchy (hgs finest first, parents[l] maps level l to
    l + 1, start = partition of the coarsest level).  Returns (X[N][16], y[N], final metric)."""
    levels, n0, rounds = len(hgs), hgs[0].n, len(fixed)
    part = torch.from_numpy(np.ascontiguousarray(start)).to("cuda", torch.int32)
    X, y = [], []
    km1 = None
    for lvl in range(levels - 1, -1, -1):
        if lvl < levels - 1:
            part = part[torch.from_numpy(parents[lvl]).to("cuda").long()].contiguous()
        ctx = JetContext(hgs[lvl])
        prev = 0.0
        for r in range(rounds):
            st = ctx.level_stats(part)
            X.append(jet_tau_features(st, hgs[lvl].eps, lvl, levels, n0, r, rounds, prev))
            before = int(st[9])
            best = None
            for tau in grid:
                p = part.clone()
                _, s, _ = ctx.refine(p, tau=(tau,), limit=limit)
                key = _key(s)
                if lookahead and r + 1 < rounds:
                    p2 = p.clone()
                    _, s2, _ = ctx.refine(p2, tau=fixed[r + 1:], limit=limit)
                    key = _key(s2)
                pref = (0 if tau == fixed[r] else 1, tau)
                cand = (key, pref, tau, p, s)
                if best is None or cand[:2] < best[:2]:
                    best = cand
            _, _, tau_star, part, s = best
            y.append(tau_star)
            prev = (before - s["km1_out"]) / before if before > 0 else 0.0
            km1 = s["km1_out"]
        ctx.close()
    return np.array(X, np.float32), np.array(y, np.float32), km1


def standardisation(X):
    mean = X.mean(axis=0).astype(np.float32)
    std = X.std(axis=0).astype(np.float32)
    std[std < 1e-6] = 1.0   # constant features (eps, k of a one-k set) pass through centred
    return mean, std


def train(net: TauNet, X, y, epochs=300, batch=256, lr=1e-3, seed=0):
    """Minibatch Adam on the GPU kernels; returns the mean loss of every epoch."""
    mean, std = standardisation(X)
    net.set(mean=mean, std=std)
    rng = np.random.default_rng(seed)
    Xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y).cuda()
    hist = []
    for _ in range(epochs):
        order = torch.from_numpy(rng.permutation(len(X))).cuda()
        losses = []
        for i in range(0, len(X), batch):
            idx = order[i:i + batch]
            losses.append(net.train_step(Xd[idx], yd[idx], lr=lr))
        hist.append(float(np.mean(losses)))
    return hist


def run_hierarchy(hgs, parents, start, net=None, fixed=FIXED, limit=LIMIT, ctxs=None):
    """Refines a hierarchy coarsest to finest with the fixed schedule (net None) or with network
    temperatures; returns (final metric, GPU seconds, Jet iterations, temperatures used, rounds that
    used the fixed temperature because a feature was out of the network's range)."""
    levels, n0 = len(hgs), hgs[0].n
    own = ctxs is None
    if own:
        ctxs = [JetContext(h) for h in hgs]
    part = torch.from_numpy(np.ascontiguousarray(start)).to("cuda", torch.int32)
    pars = [torch.from_numpy(p).to("cuda").long() for p in parents]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, taus, st, fell_back = 0, [], None, 0
    for lvl in range(levels - 1, -1, -1):
        if lvl < levels - 1:
            part = part[pars[lvl]].contiguous()
        if net is None:
            _, st, _ = ctxs[lvl].refine(part, tau=fixed, limit=limit)
            taus.append(list(fixed))
        else:
            _, st, used = ctxs[lvl].refine_learned(part, net, lvl, levels, n0, tau=fixed, limit=limit)
            taus.append(used)
            fell_back += st["tau_from_net"].count(0)
        iters += st["iterations"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if own:
        for c in ctxs:
            c.close()
    return st["km1_out"], dt, iters, taus, fell_back


def fixed_at_equal_time(hgs, parents, start, t_learned, fixed=FIXED, slack=1.05, max_rounds=8, ctxs=None, log=None):
    """The fixed schedule given as much GPU time as a learned run took: while the learned run's time
    t_learned exceeds slack x the fixed run's, one more tau = 0 round is appended (up to max_rounds
    rounds).  Returns (final metric, GPU seconds, rounds of the schedule)."""
    sched = list(fixed)
    km1, t, _, _, _ = run_hierarchy(hgs, parents, start, None, fixed=tuple(sched), ctxs=ctxs)
    while t_learned > slack * t and len(sched) < max_rounds:
        sched.append(0.0)
        km1, t, _, _, _ = run_hierarchy(hgs, parents, start, None, fixed=tuple(sched), ctxs=ctxs)
        if log:
            log(f"  fixed schedule with {len(sched)} rounds: {km1} in {t:.2f}s")
    return km1, t, len(sched)


def training_set(specs):
    """specs: list of (family, n, k, seed); family 'rownet' (row-net of a banded matrix, Zipf(2.1)
    sizes) or 'sat' (Zipf(1.8) sizes, uniform pins, weights 1..8)."""
    import workloads as W
    for fam, n, k, seed in specs:
        if fam == "rownet":
            hg = W.rownet_matrix(seed=seed, n=n, k=k)
        else:
            hg = W.sat_like(seed=seed, n=n, p_total=10 * n, k=k, cap=max(64, n // 4))
        levels = max(1, int(np.floor(np.log2(n / 2000.0))) + 1)
        hgs, parents = W.hierarchy(hg, levels, seed=seed)
        yield (fam, n, k, seed), hgs, parents, W.greedy_initial(hgs[-1], seed=seed)


DEFAULT_SPECS = ([("rownet", n, k, 1000 + i) for i, (n, k) in
                  enumerate([(n, k) for n in (1 << 14, 1 << 16, 1 << 18) for k in (16, 32, 64, 128)] +
                            [(1 << 20, 64), (1 << 20, 128)])] +
                 [("sat", n, k, 1040 + i) for i, (n, k) in
                  enumerate([(n, k) for n in (1 << 14, 1 << 16, 1 << 18) for k in (32, 128)])])


def evaluate(family, seeds, net_path, levels=12, scale=1.0, log=_log):
    """The network against the fixed schedule on full-size workloads of one family ('rownet': 4M
    vertices, k = 64; 'sat': 20M vertices, 200M pins, k = 128), one seeded hierarchy per seed:
    final metric and GPU time of both, and the fixed schedule given equal GPU time."""
    import workloads as W
    net = TauNet(path=net_path)
    rows = []
    for sd in seeds:
        t0 = time.time()
        if family == "rownet":
            hg = W.rownet_matrix(seed=sd, n=int(4_000_000 * scale), k=64)
        else:
            hg = W.sat_like(seed=sd, n=int(20_000_000 * scale), p_total=int(200_000_000 * scale))
        hgs, parents = [hg], []
        for lvl in range(levels - 1):
            c, par = W.coarsen(hgs[-1], sd * 1000 + lvl)
            hgs.append(c)
            parents.append(par)
            log(f"  seed {sd}: level {lvl + 1} n={c.n} pins={c.p}")
        start = W.greedy_initial(hgs[-1], seed=sd)
        log(f"seed {sd}: hierarchy built in {time.time() - t0:.0f}s")
        ctxs = [JetContext(h) for h in hgs]
        kf, tf, itf, _, _ = run_hierarchy(hgs, parents, start, None, ctxs=ctxs)
        log(f"  fixed schedule: {kf} in {tf:.2f}s")
        kl, tl, itl, taus, fell_back = run_hierarchy(hgs, parents, start, net, ctxs=ctxs)
        log(f"  network: {kl} in {tl:.2f}s")
        kfe, tfe, rounds = (kf, tf, len(FIXED)) if tl <= 1.05 * tf else \
            fixed_at_equal_time(hgs, parents, start, tl, ctxs=ctxs, log=log)
        for c in ctxs:
            c.close()
        row = {"seed": sd, "km1_fixed": kf, "s_fixed": round(tf, 4), "iters_fixed": itf, "km1_learned": kl,
               "s_learned": round(tl, 4), "iters_learned": itl, "km1_fixed_equal_time": kfe,
               "fixed_rounds_equal_time": rounds, "s_fixed_equal_time": round(tfe, 4),
               "rounds_on_fixed_tau": fell_back, "rounds_total": len(FIXED) * len(hgs)}
        log(f"seed {sd}: learned {kl} ({tl:.2f}s) vs fixed {kf} ({tf:.2f}s), fixed at equal time {kfe}")
        rows.append(row)
    ratio = float(np.exp(np.mean([np.log(r["km1_learned"] / r["km1_fixed_equal_time"]) for r in rows])))
    return {"family": family, "net": net_path, "geomean_km1_learned_over_fixed_equal_time": ratio, "runs": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--evaluate", choices=["rownet", "sat"], default=None,
                    help="no training: compare the network in --net with the fixed schedule on --seeds")
    ap.add_argument("--seeds", default="51,52,53")
    ap.add_argument("--net", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tau_net.bin"))
    ap.add_argument("--out", default=None, help="network file to write")
    ap.add_argument("--data", default=None, help="optional .npz to store / reuse the sweep data")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-lookahead", action="store_true", help="label by the one-round result")
    args = ap.parse_args()
    if args.evaluate:
        import json
        res = evaluate(args.evaluate, [int(x) for x in args.seeds.split(",") if x.strip()], args.net)
        print(json.dumps(res), flush=True)
        return
    if not args.out:
        ap.error("--out is required for training")
    if args.data and os.path.exists(args.data):
        d = np.load(args.data)
        X, y = d["X"], d["y"]
        _log(f"sweep data loaded: {len(X)} samples")
    else:
        Xs, ys = [], []
        t0 = time.time()
        for spec, hgs, parents, start in training_set(DEFAULT_SPECS):
            X, y, km1 = sweep(hgs, parents, start, lookahead=not args.no_lookahead)
            Xs.append(X)
            ys.append(y)
            _log(f"sweep {spec}: {len(hgs)} levels, {len(X)} samples, final km1 {km1}, labels "
                 f"{np.bincount((y * 8).astype(int), minlength=9).tolist()}, {time.time() - t0:.0f}s")
        X, y = np.concatenate(Xs), np.concatenate(ys)
        if args.data:
            np.savez(args.data, X=X, y=y)
    net = TauNet(seed=args.seed)
    hist = train(net, X, y, epochs=args.epochs, seed=args.seed)
    _log(f"training: {len(X)} samples, loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    net.save(args.out)
    _log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
