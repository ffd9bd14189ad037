"""Batched refinement: every hypergraph of a batch refined by jet_batch_refine equals jet_refine on it
alone and the oracle, for any number of lanes and any value of the performance knobs; errors name
the hypergraph; the autotuner's cache round-trips.
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


@pytest.mark.parametrize("lanes", [1, 3, 8])
def test_batch_equals_oracle_and_single(small_batch, lanes):
    items, refs = small_batch
    say(f"batch of {len(items)}, lanes {lanes}")
    batch = J().JetBatch([h for h, _ in items])
    parts = [torch.from_numpy(p).to("cuda") for _, p in items]
    rc, stats, rcs = batch.refine(parts, lanes=lanes, tau=(0.75,), limit=12)
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


def test_batch_knobs_do_not_change_results(small_batch):
    items, refs = small_batch
    batch = J().JetBatch([h for h, _ in items])
    for div in (0, 1, 8, 1 << 20):
        say(f"apply divisor {div}")
        batch.set_option(J().JET_OPT_APPLY_DIVISOR, div)
        parts = [torch.from_numpy(p).to("cuda") for _, p in items]
        batch.refine(parts, lanes=4, tau=(0.75,), limit=12)
        for i, (out, _, _) in enumerate(refs):
            assert np.array_equal(parts[i].cpu().numpy(), out), (div, i)


def test_batch_error_names_hypergraph(small_batch):
    items, _ = small_batch
    batch = J().JetBatch([h for h, _ in items[:6]])
    parts = [torch.from_numpy(p).to("cuda") for _, p in items[:6]]
    bad = parts[4].clone()
    bad[0] = items[4][0].k          # block id out of range
    parts[4] = bad
    with pytest.raises(J().JetError) as ei:
        batch.refine(parts, lanes=2, tau=(0.75,), limit=12)
    assert ei.value.code == J().JET_EINVAL
    assert "hypergraph 4" in str(ei.value)
    with pytest.raises(J().JetError):
        batch.refine(parts, lanes=0)


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
        assert knobs["lanes"] in autotune.LANES and knobs["apply_divisor"] in autotune.DIVISORS
        assert len(cache[key]["seconds"]) == len(autotune.LANES) * len(autotune.DIVISORS)
        key2, knobs2 = autotune.tuned(batch, hgs, parts, cache_path=path, tau=(0.75,), limit=12)
        assert (key2, knobs2) == (key, knobs)
    # the partitions handed to the tuner are not modified
    for (_, p0), p in zip(items, parts):
        assert np.array_equal(p.cpu().numpy(), p0)
