"""Batched refinement (union contexts, one graph for the whole batch): every hypergraph of a batch
refined by jet_batch_refine equals jet_refine on it alone and the oracle, for any number of replays
per poll and any value of the launch knobs; the full 512-hypergraph workload equals the oracle's
results on a covering subset; errors name the hypergraph; the autotuner's cache round-trips.
"""
import json
import os
import sys
import tempfile

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def J():
    import paper_2504_12013_amd.jet as jet
    return jet


@pytest.fixture(scope="module")
def small_batch():
    items = W.batch_set(seed=7, count=24, nmin=200, nmax=3000)
    refs = []
    for hg, part in items:
        out, rc, st, _ = O.refine(hg, part, tau=(0.75,), limit=12)
        refs.append((out, rc, st))
    return items, refs


@pytest.mark.parametrize("replays", [1, 3, 8])
def test_batch_equals_oracle_and_single(small_batch, replays):
    items, refs = small_batch
    say(f"batch of {len(items)}, replays {replays}")
    batch = J().JetBatch([h for h, _ in items])
    parts = [torch.from_numpy(p).to("cuda") for _, p in items]
    rc, stats, rcs = batch.refine(parts, replays=replays, tau=(0.75,), limit=12)
    for i, ((hg, part), (out, orc, ost)) in enumerate(zip(items, refs)):
        assert rcs[i] == orc, i
        assert np.array_equal(parts[i].cpu().numpy(), out), i
        for key in ("km1_in", "km1_out", "iterations", "rebalance_rounds", "moves_executed", "balanced"):
            assert stats[i][key] == ost[key], (i, key)
    # the same hypergraph alone
    hg, part = items[5]
    ctx = J().JetContext(hg)
    p = torch.from_numpy(part).to("cuda")
    ctx.refine(p, tau=(0.75,), limit=12)
    assert torch.equal(p, parts[5])


@pytest.mark.parametrize("knob", ["APPLY_DIVISOR", "GRID", "CAND_LANE_DEGREE", "RB_SLOTS", "GRAPH"])
def test_batch_knobs_do_not_change_results(small_batch, knob):
    """Every value the autotuner may choose (and the extremes) gives the oracle's partitions."""
    from paper_2504_12013_amd import autotune
    items, refs = small_batch
    batch = J().JetBatch([h for h, _ in items])
    values = {"APPLY_DIVISOR": (0, 1, 4, 16, 64, 1 << 20), "GRID": (64, 1024, 4096),
              "CAND_LANE_DEGREE": (0, 24, 1 << 20), "RB_SLOTS": (1, 2, 5), "GRAPH": (0, 1)}[knob]
    for tuned_name, opt in autotune._OPTION.items():  # the tuner's knob names map to these options
        assert opt == getattr(J(), "JET_OPT_" + {"grid": "GRID", "lane_degree": "CAND_LANE_DEGREE",
                                                 "apply_divisor": "APPLY_DIVISOR", "rb_slots": "RB_SLOTS"}[tuned_name])
    for v in values:
        say(f"{knob} = {v}")
        batch.set_option(getattr(J(), "JET_OPT_" + knob), v)
        parts = [torch.from_numpy(p).to("cuda") for _, p in items]
        _, stats, _ = batch.refine(parts, replays=4, tau=(0.75,), limit=12)
        for i, (out, _, ost) in enumerate(refs):
            assert np.array_equal(parts[i].cpu().numpy(), out), (knob, v, i)
            assert stats[i]["iterations"] == ost["iterations"], (knob, v, i)


def test_batch_error_names_hypergraph(small_batch):
    items, _ = small_batch
    batch = J().JetBatch([h for h, _ in items[:6]])
    parts = [torch.from_numpy(p).to("cuda") for _, p in items[:6]]
    bad = parts[4].clone()
    bad[0] = items[4][0].k          # block id out of range
    parts[4] = bad
    with pytest.raises(J().JetError) as ei:
        batch.refine(parts, replays=2, tau=(0.75,), limit=12)
    assert ei.value.code == J().JET_EINVAL
    assert "hypergraph 4" in str(ei.value)
    with pytest.raises(J().JetError):
        batch.refine(parts, replays=0)
    # a pin outside its own hypergraph's vertex range is rejected at set-up, naming the hypergraph
    hg = items[2][0]
    bad_hg = W.Hypergraph(n=hg.n, m=hg.m, off=hg.off, pins=hg.pins.copy(), k=hg.k, eps=hg.eps)
    bad_hg.pins[3] = hg.n
    with pytest.raises(J().JetError) as ei:
        J().JetBatch([items[0][0], items[1][0], bad_hg])
    assert ei.value.code == J().JET_EINVAL and "hypergraph 2" in str(ei.value)


def test_autotuner_cache_roundtrip(small_batch):
    from paper_2504_12013_amd import autotune
    items, _ = small_batch
    hgs = [h for h, _ in items]
    batch = J().JetBatch(hgs)
    parts = [torch.from_numpy(p).to("cuda") for _, p in items]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        key, knobs = autotune.tuned(batch, hgs, parts, cache_path=path, tau=(0.75,), limit=12)
        with open(path) as f:
            cache = json.load(f)
        assert key in cache and key.startswith("gfx950|count32|")
        for name, values in autotune.KNOBS.items():
            assert knobs[name] in values or knobs[name] == autotune.DEFAULTS[name]
        assert len(cache[key]["seconds"]) >= sum(len(v) for v in autotune.KNOBS.values()) - len(autotune.KNOBS)
        key2, knobs2 = autotune.tuned(batch, hgs, parts, cache_path=path, tau=(0.75,), limit=12)
        assert (key2, knobs2) == (key, knobs)
    # the partitions handed to the tuner are not modified
    for (_, p0), p in zip(items, parts):
        assert np.array_equal(p.cpu().numpy(), p0)


def test_full_batch_workload_covering_subset():
    """The 512-hypergraph batch workload (n log-uniform in [1e3, 1e5], Zipf(2.1) nets capped at
    1,000, k in {2, 8, 32}) refined in one batch call, as the benchmark runs it: the hypergraphs of
    tests/golden/batch512_subset.json (the 12 largest and 10 per k spread over the sizes) equal the
    oracle's partitions (SHA-256) and statistics; every other hypergraph's metric recounts."""
    import hashlib
    with open(os.path.join(os.path.dirname(__file__), "golden", "batch512_subset.json")) as f:
        gold = json.load(f)
    items = W.batch_set(seed=3)
    say(f"full batch: {len(items)} hypergraphs")
    batch = J().JetBatch([h for h, _ in items])
    parts = [torch.from_numpy(p).to("cuda") for _, p in items]
    _, stats, _ = batch.refine(parts, replays=8, tau=tuple(gold["tau"]), limit=gold["limit"])
    for row in gold["hypergraphs"]:
        i = row["index"]
        out = parts[i].cpu().numpy()
        assert hashlib.sha256(np.ascontiguousarray(out, np.int32).tobytes()).hexdigest() == row["sha256_out"], i
        for key in ("km1_in", "km1_out", "iterations", "rebalance_rounds", "moves_executed"):
            assert stats[i][key] == row[key], (i, key)
    for i in range(0, len(items), 37):
        assert stats[i]["km1_out"] == O.km1(items[i][0], parts[i].cpu().numpy()), i
