"""GPU parity of the flow-based refinement (Section 5) with the oracle, through the C ABI:

* maximum flow and both residual reachable sets (S_r, T_r) for given terminals, element by element
  (the flow assignment of push-relabel is free; these are not);
* the region of a block pair;
* two-way refinement of block pairs: partition and every count (cuts, maximum flows computed,
  region sizes, moved vertices);
* k-way refinement with the matching schedule: partition and every count, on random hypergraphs
  with and without weights, k from 2 to 16, and a VLSI-like netlist, with the pairs of a matching
  refined at once and one after the other;
* argument errors.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

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


def dev(a, dtype=torch.int32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def terminals(part, a, b, seed):
    rng = np.random.default_rng(seed)
    term = np.zeros(len(part), np.int8)
    pair = np.flatnonzero(np.isin(part, [a, b]))
    r = rng.random(len(pair))
    term[pair[(r < 0.3) & (part[pair] == a)]] = 1
    term[pair[(r < 0.3) & (part[pair] == b)]] = 2
    return term


@pytest.mark.parametrize("seed", range(10))
def test_mincut_matches_oracle(seed):
    n = [40, 300, 2000, 5000][seed % 4]
    hg = W.random_hypergraph(n, int(1.3 * n), 3, 500 + seed, smin=2, smax=6, nw_max=4 if seed % 2 else 1)
    part = np.random.default_rng(seed).integers(0, 3, n).astype(np.int32)
    term = terminals(part, 0, 2, seed)
    say(f"mincut seed {seed}: n={n}")
    F, sr, tr = J().JetContext(hg).flow_mincut(dev(part), 0, 2, dev(term, torch.int8))
    oF, osr, otr = O.flow_mincut(hg, part, 0, 2, term)
    assert F == oF
    assert np.array_equal(sr.cpu().numpy().astype(bool), osr)
    assert np.array_equal(tr.cpu().numpy().astype(bool), otr)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("alpha", [0, 2, 16])
def test_region_matches_oracle(seed, alpha):
    hg = W.random_hypergraph(3000, 3500, 4, 600 + seed, smin=2, smax=5, vw_max=3 if seed % 2 else 1)
    part = W.part_roundrobin(hg.n, 4, seed)
    ctx = J().JetContext(hg)
    for a, b in ((0, 1), (3, 2)):
        got = ctx.flow_region(dev(part), a, b, alpha).cpu().numpy()
        assert np.array_equal(got, O.flow_region(hg, part, a, b, alpha)), (a, b)


PAIR_KEYS = ("old_cut", "new_cut", "iterations", "region_a", "region_b", "moved")


@pytest.mark.parametrize("seed", range(2))
def test_deep_regions_pair_and_refine(seed):
    """A banded hypergraph in contiguous blocks: regions over many breadth-first levels up to a
    third block, a pair refinement and the k-way schedule on it, against the oracle."""
    hg, part = W.banded_hypergraph(4000, 8, seed, vw_max=3 if seed % 2 else 1)
    say("banded", seed)
    ctx = J().JetContext(hg)
    for alpha in (16, 100):
        for a, b in ((0, 1), (1, 2), (5, 4)):
            got = ctx.flow_region(dev(part), a, b, alpha).cpu().numpy()
            assert np.array_equal(got, O.flow_region(hg, part, a, b, alpha)), (alpha, a, b)
    d = dev(part)
    st = ctx.flow_pair(d, 1, 2)
    onew, orep, ost = O.flow_pair(hg, part, 1, 2)
    assert bool(st["replaced"]) == orep and np.array_equal(d.cpu().numpy(), onew)
    for key in PAIR_KEYS:
        assert st[key] == ost[key], key
    d = dev(part)
    st = ctx.flow_refine(d, max_rounds=2)
    onew, ost = O.flow_refine(hg, part, max_rounds=2)
    for key in REFINE_KEYS:
        assert st[key] == ost[key], key
    assert np.array_equal(d.cpu().numpy(), onew)
    ctx.close()


@pytest.mark.parametrize("seed", range(6))
def test_pair_matches_oracle(seed):
    k = 4
    n = [500, 2000, 6000][seed % 3]
    hg = W.random_hypergraph(n, int(1.4 * n), k, 700 + seed, smin=2, smax=6, vw_max=3 if seed % 2 else 1,
                             nw_max=3 if seed % 3 == 0 else 1)
    part = W.part_roundrobin(hg.n, k, seed)
    ctx = J().JetContext(hg)
    p = dev(part)
    for a, b in ((0, 1), (2, 3), (1, 3), (0, 2)):
        say(f"pair seed {seed} n={n}: ({a},{b})")
        st = ctx.flow_pair(p, a, b)
        part, replaced, ost = O.flow_pair(hg, part, a, b)
        assert bool(st["replaced"]) == replaced
        for key in PAIR_KEYS:
            assert st[key] == ost[key], key
        assert np.array_equal(p.cpu().numpy(), part)


REFINE_KEYS = ("km1_in", "km1_out", "rounds", "matchings", "pairs", "accepted", "flow_calls", "moved")

CASES = {
    "k2": lambda: (W.random_hypergraph(3000, 4000, 2, 81, smin=2, smax=6), 1),
    "k4-weighted": lambda: (W.random_hypergraph(4000, 5000, 4, 82, smin=2, smax=7, vw_max=4, nw_max=3), 2),
    "k8": lambda: (W.random_hypergraph(6000, 8000, 8, 83, smin=2, smax=5), 3),
    "k16": lambda: (W.random_hypergraph(8000, 10000, 16, 84, smin=2, smax=4, vw_max=2), 4),
    "vlsi-k8": lambda: (W.vlsi_like(seed=85, n=8000, m=8800)[0], 5),
}


@pytest.mark.parametrize("workers", [4, 1], ids=["pairs-at-once", "one-after-another"])
@pytest.mark.parametrize("name", list(CASES))
def test_refine_matches_oracle(name, workers):
    hg, seed = CASES[name]()
    part = W.part_roundrobin(hg.n, hg.k, seed)
    say(f"flow refine {name}: n={hg.n} pins={hg.p} k={hg.k}, {workers} workers")
    p = dev(part)
    ctx = J().JetContext(hg)
    ctx.set_option(J().JET_OPT_FLOW_WORKERS, workers)
    st = ctx.flow_refine(p, max_rounds=3)
    out, ost = O.flow_refine(hg, part, max_rounds=3)
    say(f"  km1 {ost['km1_in']} -> {ost['km1_out']}, pairs {ost['pairs']}, flows {ost['flow_calls']}")
    for key in REFINE_KEYS:
        assert st[key] == ost[key], key
    assert np.array_equal(p.cpu().numpy(), out)


def test_refine_after_jet_matches_oracle():
    """Flows after Jet, as the paper runs them on a level: the Jet-refined partition of a VLSI-like
    netlist refined further by the k-way schedule."""
    hg, start = W.vlsi_like(seed=86, n=20000, m=22000)
    ctx = J().JetContext(hg)
    p = dev(start)
    ctx.refine(p, tau=(0.75, 0.375, 0.0), limit=8)
    jet_part = p.cpu().numpy()
    st = ctx.flow_refine(p, max_rounds=4)
    out, ost = O.flow_refine(hg, jet_part, max_rounds=4)
    say(f"after Jet: km1 {ost['km1_in']} -> {ost['km1_out']}")
    for key in REFINE_KEYS:
        assert st[key] == ost[key], key
    assert np.array_equal(p.cpu().numpy(), out)


def test_argument_errors():
    hg = W.random_hypergraph(200, 300, 4, 90)
    part = dev(W.part_roundrobin(hg.n, 4, 1))
    ctx = J().JetContext(hg)
    for call in (lambda: ctx.flow_pair(part, 1, 1), lambda: ctx.flow_pair(part, 0, 4),
                 lambda: ctx.flow_region(part, 0, 1, alpha=-1), lambda: ctx.flow_refine(part, max_rounds=-1),
                 lambda: ctx.set_option(J().JET_OPT_FLOW_WORKERS, 0), lambda: ctx.set_option(J().JET_OPT_FLOW_WORKERS, 9)):
        with pytest.raises(J().JetError) as ei:
            call()
        assert ei.value.code == J().JET_EINVAL
    bad = part.clone()
    bad[5] = 7
    with pytest.raises(J().JetError):
        ctx.flow_refine(bad)


def test_flow_round_full_size_bit_identical():
    """The flow benchmark's step at full size: the VLSI-like hypergraph (1M vertices, k = 8) refined
    by Jet from its seeded start, then one round of the k-way flow schedule, as bench.py --workload
    flows runs it (four workers); partitions (SHA-256) and every count equal the oracle's stored
    result (tests/golden/make_flows_round.py)."""
    import hashlib
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "flows_vlsi1M_round.json")
    if not os.path.exists(path):
        pytest.skip("the oracle's result is not stored yet (tests/golden/make_flows_round.py)")
    with open(path) as f:
        gold = json.load(f)

    def sha(a):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()

    say("flows 1M: generate")
    hg, start = W.vlsi_like(seed=2, n=1_000_000, m=1_100_000)
    assert hg.p == gold["pins"] and sha(start) == gold["sha256_start"]
    ctx = J().JetContext(hg)
    p = dev(start)
    say("flows 1M: Jet")
    rc, st, _ = ctx.refine(p, tau=tuple(gold["tau"]), limit=gold["limit"])
    assert rc == gold["jet_rc"] and st["km1_out"] == gold["jet_km1"] and st["iterations"] == gold["jet_iterations"]
    assert sha(p.cpu().numpy()) == gold["sha256_jet"]
    say("flows 1M: one round")
    fst = ctx.flow_refine(p, alpha=gold["alpha"], max_rounds=gold["rounds"])
    for key in REFINE_KEYS:
        assert fst[key] == gold["flows"][key], key
    assert sha(p.cpu().numpy()) == gold["sha256_flows"]
