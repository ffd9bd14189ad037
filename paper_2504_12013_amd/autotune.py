"""Autotuner for batched refinement: picks the launch knobs of a batch by a timed sweep on the GPU and
caches the choice as JSON keyed by (GPU architecture, shape bucket).

Knobs (none of them changes any result, only the time):
  replays        iterations of the whole batch's captured graph between two host polls;
  grid           workgroups of the persistent kernels (tiles per workgroup = work / grid);
  lane_degree    lanes per vertex of the bit-sliced candidate kernel: one lane below this mean degree,
                 eight above (0: always eight);
  apply_divisor  switch point of move application from per-move atomics to per-net recounting;
  rb_slots       rebalancing rounds a replayed iteration holds room for.

The sweep is coordinate descent from the library defaults: each knob in turn is timed at every
value with the others fixed at their best so far (one refinement of copies of the batch's starting
partitions per setting, after one untimed warm-up), twice over the knobs.  The cache file is plain
JSON; a missing entry triggers a sweep.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from .jet import JET_OPT_APPLY_DIVISOR, JET_OPT_CAND_LANE_DEGREE, JET_OPT_GRID, JET_OPT_RB_SLOTS

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune.json")
KNOBS = {
    "replays": (2, 8, 32),
    "grid": (1024, 2048, 4096),
    "lane_degree": (0, 24),
    "apply_divisor": (4, 16, 64),
    "rb_slots": (1, 2),
}
DEFAULTS = {"replays": 8, "grid": 2048, "lane_degree": 24, "apply_divisor": 16, "rb_slots": 1}
_OPTION = {"grid": JET_OPT_GRID, "lane_degree": JET_OPT_CAND_LANE_DEGREE, "apply_divisor": JET_OPT_APPLY_DIVISOR,
           "rb_slots": JET_OPT_RB_SLOTS}


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


def apply(batch, settings):
    """Sets the batch's launch options (everything but replays, which is a refine argument)."""
    for name, opt in _OPTION.items():
        batch.set_option(opt, int(settings[name]))


def _time(batch, parts, settings, kw):
    apply(batch, settings)
    batch.refine([p.clone() for p in parts], replays=settings["replays"], **kw)  # graph capture, untimed
    work = [p.clone() for p in parts]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.refine(work, replays=settings["replays"], **kw)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def sweep(batch, parts, knobs=None, passes=2, log=None, **kw):
    """Coordinate descent over the knobs; returns (best settings, {setting string: seconds})."""
    knobs = knobs or KNOBS
    best = dict(DEFAULTS)
    times = {}

    def key(s):
        return ",".join(f"{k}={s[k]}" for k in sorted(s))

    best_t = times.setdefault(key(best), _time(batch, parts, best, kw))
    for _ in range(passes):
        for name, values in knobs.items():
            for v in values:
                s = dict(best, **{name: v})
                if key(s) not in times:
                    times[key(s)] = _time(batch, parts, s, kw)
                    if log:
                        log(f"autotune {key(s)}: {times[key(s)]:.3f}s")
                if times[key(s)] < best_t:
                    best, best_t = s, times[key(s)]
    return best, times


def tuned(batch, hgs, parts, cache_path: str = DEFAULT_CACHE, retune: bool = False, log=None, **kw):
    """Settings for this batch from the cache, sweeping (and storing) them when absent; the batch's
    options are set to them."""
    key = shape_key(hgs)
    cache = _load(cache_path)
    if key in cache and not retune and all(k in cache[key] for k in DEFAULTS):
        settings = {k: int(cache[key][k]) for k in DEFAULTS}
    else:
        settings, times = sweep(batch, parts, log=log, **kw)
        cache[key] = dict(settings, seconds={k: round(t, 4) for k, t in times.items()})
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    apply(batch, settings)
    return key, settings
