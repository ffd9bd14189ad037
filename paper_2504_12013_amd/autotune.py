"""Autotuner for batched refinement: picks the launch knobs of a batch by a timed sweep on the GPU and
caches the choice as JSON keyed by (GPU architecture, shape bucket).

Knobs (none of them changes any result, only the time):
  lanes          streams (each driven by a host thread) that take the hypergraphs largest first;
  apply_divisor  switch point of move application from per-move atomics to per-net recounting.

The sweep refines copies of the batch's starting partitions once per setting (after one untimed
warm-up) and keeps the fastest.  The cache file is plain JSON; a missing entry triggers a sweep.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from .jet import JET_OPT_APPLY_DIVISOR

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune.json")
LANES = (1, 2, 4, 8, 16)
DIVISORS = (4, 8, 16, 32)


def _bucket(x: float) -> int:
    return 1 << max(0, int(round(math.log2(max(1.0, x)))))


def shape_key(hgs, arch: str = "gfx950") -> str:
    ks = sorted({int(h.k) for h in hgs})
    mean_p = sum(int(h.p) for h in hgs) / len(hgs)
    return f"{arch}|count{_bucket(len(hgs))}|pins{_bucket(mean_p)}|k{'-'.join(map(str, ks))}"


def _load(path):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _time(batch, parts, settings, kw):
    batch.set_option(JET_OPT_APPLY_DIVISOR, settings["apply_divisor"])
    work = [p.clone() for p in parts]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.refine(work, lanes=settings["lanes"], **kw)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def sweep(batch, parts, lanes=LANES, divisors=DIVISORS, log=None, **kw):
    """Times every (lanes, apply_divisor) pair; returns (best settings, {setting: seconds})."""
    _time(batch, parts, {"lanes": max(lanes), "apply_divisor": 8}, kw)  # warm-up
    times = {}
    for d in divisors:
        for l in lanes:
            s = {"lanes": l, "apply_divisor": d}
            times[(l, d)] = _time(batch, parts, s, kw)
            if log:
                log(f"autotune lanes {l} divisor {d}: {times[(l, d)]:.3f}s")
    (l, d) = min(times, key=times.get)
    return {"lanes": l, "apply_divisor": d}, times


def tuned(batch, hgs, parts, cache_path: str = DEFAULT_CACHE, retune: bool = False, log=None, **kw):
    """Settings for this batch from the cache, sweeping (and storing) them when absent."""
    key = shape_key(hgs)
    cache = _load(cache_path)
    if key in cache and not retune:
        settings = {"lanes": int(cache[key]["lanes"]), "apply_divisor": int(cache[key]["apply_divisor"])}
    else:
        settings, times = sweep(batch, parts, log=log, **kw)
        cache[key] = dict(settings, seconds={f"{l}x{d}": round(t, 4) for (l, d), t in times.items()})
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    batch.set_option(JET_OPT_APPLY_DIVISOR, settings["apply_divisor"])
    return key, settings
