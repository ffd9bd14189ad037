"""GPU parity: every step of the HIP path against the CPU oracle, element by element.

All comparisons are exact (integer partition arithmetic): pin counts, metric, candidate targets,
gains and flags, recomputed gains, rebalancing selections, and whole refinements including the
per-iteration trace.
"""
import hashlib
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads import Hypergraph

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def jet_mod():
    import paper_2504_12013_amd.jet as J
    return J


def dev(a, dtype=torch.int32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=dtype)


def host(t):
    return t.cpu().numpy()


def ctx_for(hg):
    return jet_mod().JetContext(hg)


def hg_from_nets(n, nets, k, eps=0.03, net_w=None, vtx_w=None):
    off = np.zeros(len(nets) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(e) for e in nets])
    pins = np.array([v for e in nets for v in e], dtype=np.int32)
    return Hypergraph(n=n, m=len(nets), off=off, pins=pins, k=k, eps=eps,
                      net_w=None if net_w is None else np.asarray(net_w, np.int32),
                      vtx_w=None if vtx_w is None else np.asarray(vtx_w, np.int32))


def mixed_sizes(seed, n, m, k, smax, vw_max=1, nw_max=1, big=()):
    """Random hypergraph with sizes U[2, smax] plus a few large nets (sizes in `big`)."""
    hg = W.random_hypergraph(n, m, k, seed, smin=2, smax=smax, vw_max=vw_max, nw_max=nw_max)
    if not big:
        return hg
    rng = np.random.default_rng(seed)
    nets = [hg.pins[hg.off[e]:hg.off[e + 1]].tolist() for e in range(hg.m)]
    for s in big:
        nets.insert(int(rng.integers(0, len(nets) + 1)), sorted(rng.choice(n, size=s, replace=False).tolist()))
    nw = None if hg.net_w is None else rng.integers(1, nw_max + 1, len(nets)).astype(np.int32)
    return hg_from_nets(n, nets, k, net_w=nw, vtx_w=hg.vtx_w)


CASES = [
    # (seed, n, m, k, smax, vw_max, nw_max, big nets)
    (1, 200, 300, 2, 6, 1, 1, ()),
    (2, 300, 500, 3, 8, 3, 1, ()),
    (3, 500, 800, 8, 10, 1, 4, (100,)),
    (4, 800, 1000, 11, 12, 2, 2, (70, 300)),
    (5, 2500, 1500, 16, 20, 1, 1, (65, 1025, 2000)),
    (6, 1500, 2000, 33, 30, 4, 3, (200,)),
    (7, 3000, 3000, 64, 40, 1, 1, (64, 65, 500, 1100)),
    (8, 6000, 2500, 100, 16, 2, 1, (1500, 5000)),
    (9, 6000, 4000, 128, 24, 1, 2, (3000, 4100, 5500)),
    # vertices with more than 256 incident nets (workgroup-per-vertex paths)
    (10, 600, 26000, 64, 10, 3, 2, ()),
    (11, 400, 30000, 128, 8, 1, 1, (300,)),
    (12, 500, 20000, 8, 10, 2, 1, ()),
    # incidence lists longer than 8192 (radix-sorted at set-up)
    (13, 40, 40000, 4, 20, 1, 1, ()),
]


@pytest.mark.parametrize("case", CASES, ids=[f"k{c[3]}-s{c[0]}" for c in CASES])
def test_phi_and_metric(case):
    seed, n, m, k, smax, vw, nwm, big = case
    say("case", case)
    hg = mixed_sizes(seed, n, m, k, smax, vw, nwm, big)
    part = W.part_uniform(hg.n, k, seed)
    ctx = ctx_for(hg)
    phi = host(ctx.phi(dev(part)))
    assert (phi == O.phi(hg, part)).all()
    assert ctx.km1(dev(part)) == O.km1(hg, part)
    ctx.close()


@pytest.mark.parametrize("case", CASES, ids=[f"k{c[3]}-s{c[0]}" for c in CASES])
def test_candidates(case):
    seed, n, m, k, smax, vw, nwm, big = case
    say("case", case)
    hg = mixed_sizes(seed, n, m, k, smax, vw, nwm, big)
    part = W.part_uniform(hg.n, k, seed + 1)
    rng = np.random.default_rng(seed)
    lock = (rng.random(hg.n) < 0.2).astype(np.uint8)
    ctx = ctx_for(hg)
    for tau in (0.0, 0.375, 0.75, 1.0):
        tq = O.quantize_tau(tau)
        for lk in (None, lock):
            t, g, inM = ctx.candidates(dev(part), tq, None if lk is None else dev(lk, torch.uint8))
            ot, og, oin = O.candidates(hg, part, tq, lk)
            assert (host(t) == ot).all()
            assert (host(g)[ot >= 0] == og[ot >= 0]).all()
            assert (host(inM) == oin).all()
    ctx.close()


@pytest.mark.parametrize("lane_degree,xcd", [(0, 0), (1 << 20, 0), (0, 1), (1 << 20, 1)],
                         ids=["lane-groups", "one-lane", "lane-groups-xcd", "one-lane-xcd"])
@pytest.mark.parametrize("case", CASES, ids=[f"k{c[3]}-s{c[0]}" for c in CASES])
def test_candidates_each_kernel(case, lane_degree, xcd, monkeypatch):
    """Unit net weights and k <= 64 have two kernels for the candidates and for the rebalancing gains
    (a group of lanes per vertex, or one lane per vertex with bit-sliced counts); forcing either,
    with or without contiguous vertex and list ranges per XCD, gives the oracle's targets, gains and
    candidate set, the oracle's rebalancing round, and the oracle's refinement."""
    monkeypatch.setenv("JET_CAND_LANE_DEGREE", str(lane_degree))
    monkeypatch.setenv("JET_CAND_XCD", str(xcd))
    monkeypatch.setenv("JET_RB_XCD", str(xcd))
    seed, n, m, k, smax, vw, nwm, big = case
    hg = mixed_sizes(seed, n, m, k, smax, vw, nwm, big)
    part = W.part_uniform(hg.n, k, seed + 3)
    rng = np.random.default_rng(seed + 3)
    lock = (rng.random(hg.n) < 0.2).astype(np.uint8)
    ctx = ctx_for(hg)
    for tau in (0.0, 0.75):
        tq = O.quantize_tau(tau)
        t, g, inM = ctx.candidates(dev(part), tq, dev(lock, torch.uint8))
        ot, og, oin = O.candidates(hg, part, tq, lock)
        assert (host(t) == ot).all()
        assert (host(g)[ot >= 0] == og[ot >= 0]).all()
        assert (host(inM) == oin).all()
    # a rebalancing round (its gain pass has the same two kernels)
    over = part.copy()
    over[: hg.n // 3] = rng.integers(0, max(1, k // 3), hg.n // 3)
    for dz in (100_000, 0):
        d = dev(over)
        sel, moved = ctx.rebalance_round(d, dz)
        new, osel, omoved = O.rebalance_round(hg, over, dz)
        assert moved == omoved
        assert (host(sel) == osel).all()
        assert (host(d) == new).all()
    ctx.close()
    if seed in (1, 7, 10):
        check_refine(hg, W.part_roundrobin(hg.n, k, seed + 5), tau=(0.75, 0.0), limit=6)


@pytest.mark.parametrize("case", CASES, ids=[f"k{c[3]}-s{c[0]}" for c in CASES])
def test_rebalance_selection_split_pass(case, monkeypatch):
    """The rebalancing selection's first radix pass over all compute units (histogram and split
    kernels, used on large levels) forced on every level: the oracle's rebalancing rounds, with
    blocks overloaded by little and by much (emit-all, kept-bucket and one-pass-done cases), and
    the oracle's refinement."""
    monkeypatch.setenv("JET_SEL_SPLIT_MIN", "0")
    seed, n, m, k, smax, vw, nwm, big = case
    say("case", case)
    hg = mixed_sizes(seed, n, m, k, smax, vw, nwm, big)
    rng = np.random.default_rng(seed + 11)
    ctx = ctx_for(hg)
    part = W.part_uniform(hg.n, k, seed + 4)
    for frac in (3, 12):
        over = part.copy()
        over[: hg.n // frac] = rng.integers(0, max(1, k // 3), hg.n // frac)
        for dz in (100_000, 0):
            d = dev(over)
            for r in range(3):
                say("overload 1 /", frac, "deadzone", dz, "round", r)
                before = host(d)
                sel, moved = ctx.rebalance_round(d, dz)
                new, osel, omoved = O.rebalance_round(hg, before, dz)
                assert moved == omoved
                assert (host(sel) == osel).all()
                assert (host(d) == new).all()
    ctx.close()
    if seed in (2, 5, 9, 11):
        check_refine(hg, W.part_roundrobin(hg.n, k, seed + 6), tau=(0.75, 0.0), limit=6)


@pytest.mark.parametrize("seed", [19, 85, 116, 139, 182, 199, 209, 230, 239, 266])
def test_heavy_vertex_with_a_valid_target(seed):
    """Overloaded block 0 holds a vertex heavier than 3/2 (c(V_0) - ceil(c(V)/k)) that still has a
    valid target, so Section 4.3's heavy-vertex rule alone keeps it: one rebalancing round, and
    whole rebalancing calls in all three orders, against the oracle."""
    hg, part, heavy = W.overloaded_with_heavy_vertex(seed)
    say("heavy vertex", seed, heavy)
    ctx = ctx_for(hg)
    d = dev(part)
    sel, moved = ctx.rebalance_round(d, 100_000)
    new, osel, omoved = O.rebalance_round(hg, part, 100_000)
    assert osel[heavy] == -1
    assert moved == omoved and (host(sel) == osel).all() and (host(d) == new).all()
    for order in (0, 1, 2):
        d = dev(part)
        rc, st = ctx.rebalance(d, rb_unweighted=order)
        ob, orc, ost = O.rebalance(hg, part, rb_unweighted=order)
        assert rc == orc and (host(d) == ob).all() and st["rebalance_rounds"] == ost["rebalance_rounds"], order
    ctx.close()


@pytest.mark.parametrize("slices", [2, 7, 64])
@pytest.mark.parametrize("case", [CASES[0], CASES[4], CASES[8], CASES[11]], ids=lambda c: f"k{c[3]}-s{c[0]}")
def test_rebalance_selection_split_pass_slices(case, slices, monkeypatch):
    """The split pass with several workgroups per overloaded block (JET_SEL_SLICES): histograms
    merged across workgroups and the kept entries compacted by atomics from several slices, against
    the oracle's rebalancing rounds with several overloaded blocks."""
    monkeypatch.setenv("JET_SEL_SPLIT_MIN", "0")
    monkeypatch.setenv("JET_SEL_SLICES", str(slices))
    seed, n, m, k, smax, vw, nwm, big = case
    say("case", case, "slices", slices)
    hg = mixed_sizes(seed, n, m, k, smax, vw, nwm, big)
    rng = np.random.default_rng(seed + 13)
    ctx = ctx_for(hg)
    part = W.part_uniform(hg.n, k, seed + 4)
    for frac in (3, 12):
        over = part.copy()
        over[: hg.n // frac] = rng.integers(0, max(1, k // 3), hg.n // frac)
        d = dev(over)
        for r in range(3):
            before = host(d)
            sel, moved = ctx.rebalance_round(d, 100_000)
            new, osel, omoved = O.rebalance_round(hg, before, 100_000)
            assert moved == omoved
            assert (host(sel) == osel).all()
            assert (host(d) == new).all()
    ctx.close()


@pytest.mark.parametrize("case", CASES, ids=[f"k{c[3]}-s{c[0]}" for c in CASES])
def test_afterburner_method_candidates(case):
    seed, n, m, k, smax, vw, nwm, big = case
    say("case", case)
    hg = mixed_sizes(seed, n, m, k, smax, vw, nwm, big)
    part = W.part_uniform(hg.n, k, seed + 2)
    ctx = ctx_for(hg)
    for tau in (0.0, 0.75, 1.0):
        ot, og, oin = O.candidates(hg, part, O.quantize_tau(tau))
        rg = host(ctx.afterburner(dev(part), dev(ot), dev(og), dev(oin, torch.uint8)))
        assert (rg == O.afterburner(hg, part, ot, og, oin)).all()
    ctx.close()


@pytest.mark.parametrize("case", CASES, ids=[f"k{c[3]}-s{c[0]}" for c in CASES])
def test_afterburner_arbitrary_moves(case):
    """Random candidate sets, targets and heavily tied gains: exercises every per-block class of
    the large-net kernels (inert, arrival-only, departure-only, interleaved)."""
    seed, n, m, k, smax, vw, nwm, big = case
    say("case", case)
    hg = mixed_sizes(seed, n, m, k, smax, vw, nwm, big)
    rng = np.random.default_rng(100 + seed)
    ctx = ctx_for(hg)
    for frac in (0.05, 0.5, 0.95):
        kk = min(k, 4) if frac > 0.9 else k      # few blocks: blocks that every pin leaves are common
        part = rng.integers(0, kk, hg.n).astype(np.int32)
        inM = (rng.random(hg.n) < frac).astype(np.uint8)
        t = ((part + rng.integers(1, kk, hg.n)) % kk).astype(np.int32)
        g = rng.integers(-3, 4, hg.n).astype(np.int32)
        rg = host(ctx.afterburner(dev(part), dev(t), dev(g), dev(inM, torch.uint8)))
        assert (rg == O.afterburner(hg, part, t, g, inM)).all()
    ctx.close()


def huge_net_case(all_leave):
    n, k = 12000, 4
    rng = np.random.default_rng(5)
    nets = [list(range(10000))] + [[int(a), int(b)] for a, b in rng.integers(0, n, (3000, 2)) if a != b]
    hg = hg_from_nets(n, nets, k)
    part = rng.integers(1, k, n).astype(np.int32)
    part[:150] = 0                                   # 150 pins of the huge net in block 0
    t = (part % 3) + 1                               # a different block in 1..3 (or 1 for block 0)
    t[t == part] = np.where(part[t == part] == 3, 1, part[t == part] + 1)
    t[1000:1500] = 0                                 # 500 arrivals in block 0
    inM = (rng.random(n) < 0.5).astype(np.uint8)
    inM[:150] = 1                                    # every block-0 pin leaves
    inM[1000:1500] = 1
    if all_leave:
        inM[:] = 1
    g = rng.integers(-2, 3, n).astype(np.int32)
    return hg, part, t.astype(np.int32), g, inM


def test_afterburner_huge_net_interleaved_events():
    """One net larger than the in-LDS capacity whose candidates interleave on one block: the
    kernel streams the pins again and keeps only the events of that block."""
    hg, part, t, g, inM = huge_net_case(False)
    assert (part != t).all()
    ctx = ctx_for(hg)
    rg = host(ctx.afterburner(dev(part), dev(t), dev(g), dev(inM, torch.uint8)))
    assert (rg == O.afterburner(hg, part, t, g, inM)).all()
    ctx.close()


def test_afterburner_huge_net_scratch_path():
    """Every pin of a 10,000-pin net is a candidate: more interleaved events than LDS holds, so the
    net goes through the global-scratch radix sort and segmented walk."""
    hg, part, t, g, inM = huge_net_case(True)
    ctx = ctx_for(hg)
    rg = host(ctx.afterburner(dev(part), dev(t), dev(g), dev(inM, torch.uint8)))
    assert (rg == O.afterburner(hg, part, t, g, inM)).all()
    ctx.close()


@pytest.mark.parametrize("case", CASES, ids=[f"k{c[3]}-s{c[0]}" for c in CASES])
def test_rebalance_round(case):
    seed, n, m, k, smax, vw, nwm, big = case
    say("case", case)
    hg = mixed_sizes(seed, n, m, k, smax, vw, nwm, big)
    rng = np.random.default_rng(200 + seed)
    part = rng.integers(0, k, hg.n).astype(np.int32)
    part[: hg.n // 3] = rng.integers(0, max(1, k // 3), hg.n // 3)     # overload the low blocks
    ctx = ctx_for(hg)
    for dz in (100_000, 0):
        d = dev(part)
        sel, moved = ctx.rebalance_round(d, dz)
        new, osel, omoved = O.rebalance_round(hg, part, dz)
        assert moved == omoved
        assert (host(sel) == osel).all()
        assert (host(d) == new).all()
    ctx.close()


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def check_refine(hg, part, **kw):
    ctx = ctx_for(hg)
    d = dev(part)
    rc, st, tr = ctx.refine(d, trace_cap=4096, **kw)
    out = host(d)
    opart, orc, ost, otr = O.refine(hg, part, **kw)
    say("gpu", st, "\noracle", ost)
    assert rc == orc
    assert sha(out) == sha(opart)
    for key in ("km1_in", "km1_out", "lmax", "max_block_weight", "iterations", "rebalance_rounds", "balanced",
                "moves_executed", "tau_q_used"):
        assert st[key] == ost[key], key
    assert tr == otr
    ctx.close()
    return out, st


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_refine_small_uniform(seed):
    """2,000 vertices, 4,000 nets of size U[2,8], k=4, tau=0.75, limit 12 (the small workload)."""
    hg, part = W.small_uniform(seed)
    out, st = check_refine(hg, part, tau=(0.75,), limit=12)
    assert st["km1_out"] <= st["km1_in"]


@pytest.mark.parametrize("case", CASES, ids=[f"k{c[3]}-s{c[0]}" for c in CASES])
def test_refine_schedule(case):
    seed, n, m, k, smax, vw, nwm, big = case
    say("case", case)
    hg = mixed_sizes(seed, n, m, k, smax, vw, nwm, big)
    part = W.part_roundrobin(hg.n, k, seed)
    check_refine(hg, part, tau=(0.75, 0.375, 0.0), limit=8)


def test_refine_imbalanced_input():
    hg = W.random_hypergraph(2000, 3000, 8, 77, smin=2, smax=9, vw_max=5)
    part = np.zeros(hg.n, np.int32)
    part[::3] = np.arange(len(part[::3])) % 8
    check_refine(hg, part, tau=(1.0, 0.0), limit=6)


def test_rebalance_entry_point():
    hg = W.random_hypergraph(5000, 8000, 16, 78, smin=2, smax=12, vw_max=4)
    rng = np.random.default_rng(78)
    part = rng.integers(0, 4, hg.n).astype(np.int32)
    ctx = ctx_for(hg)
    d = dev(part)
    rc, st = ctx.rebalance(d)
    opart, orc, ost = O.rebalance(hg, part)
    assert rc == orc and (host(d) == opart).all()
    assert st["rebalance_rounds"] == ost["rebalance_rounds"] and st["km1_out"] == ost["km1_out"]
    ctx.close()


def test_worked_example_on_gpu(golden_dir):
    import json
    import os
    with open(os.path.join(golden_dir, "path4_worked_example.json")) as f:
        G = json.load(f)
    hg = hg_from_nets(4, G["hypergraph"]["nets"], 2)
    out, st = check_refine(hg, np.array(G["part_in"], np.int32), tau=(G["tau"],), limit=12)
    assert out.tolist() == G["part_out"] and st["km1_out"] == G["km1_out"]


def test_determinism_repeat():
    hg = mixed_sizes(9, 6000, 4000, 128, 24, 1, 2, (3000, 4100, 5500))
    part = W.part_roundrobin(hg.n, 128, 9)
    hashes = set()
    ctx = ctx_for(hg)
    for _ in range(3):
        d = dev(part)
        ctx.refine(d, tau=(0.75, 0.0), limit=5)
        hashes.add(sha(host(d)))
    ctx.close()
    assert len(hashes) == 1


def test_errors():
    J = jet_mod()
    hg = W.random_hypergraph(100, 100, 4, 3)
    ctx = ctx_for(hg)
    bad = np.zeros(100, np.int32)
    bad[7] = 4
    with pytest.raises(J.JetError) as ei:
        ctx.km1(dev(bad))
    assert ei.value.code == J.JET_EINVAL
    # context still usable
    assert ctx.km1(dev(np.zeros(100, np.int32))) == 0
    ctx.close()
    dup = hg_from_nets(10, [[1, 2, 1], [3, 4]], 2)
    with pytest.raises(J.JetError):
        ctx_for(dup)
    oob = hg_from_nets(10, [[1, 2, 10]], 2)
    with pytest.raises(J.JetError):
        ctx_for(oob)


@pytest.mark.parametrize("xcd", [0, 1], ids=["strided", "xcd-ranges"])
@pytest.mark.parametrize("divisor", [0, 1 << 20], ids=["vertex-centric", "net-centric"])
@pytest.mark.parametrize("case", [CASES[2], CASES[6], CASES[8], CASES[10]], ids=lambda c: f"k{c[3]}-s{c[0]}")
def test_refine_each_apply_path(case, divisor, xcd, monkeypatch):
    """Move application has a vertex-centric (atomics) and a net-centric (recount) path; forcing
    each one, with the workgroups striding or each XCD taking one contiguous range, must give the
    same partitions as the oracle."""
    monkeypatch.setenv("JET_APPLY_DIVISOR", str(divisor))
    monkeypatch.setenv("JET_APPLY_XCD", str(xcd))
    seed, n, m, k, smax, vw, nwm, big = case
    say("case", case, "divisor", divisor)
    hg = mixed_sizes(seed, n, m, k, smax, vw, nwm, big)
    part = W.part_roundrobin(hg.n, k, seed + 7)
    check_refine(hg, part, tau=(1.0, 0.5, 0.0), limit=6)


@pytest.mark.parametrize("divisor", [0, 1 << 20], ids=["vertex-centric", "net-centric"])
@pytest.mark.parametrize("size", [65535, 70000], ids=["16-bit-counts-at-limit", "32-bit-counts"])
def test_refine_largest_net_sizes(size, divisor, monkeypatch):
    """Pin counts are 16-bit when no net exceeds 65,535 pins and 32-bit otherwise.  One net of
    exactly 65,535 pins, all in block 0 at the start (its count at the 16-bit maximum while the
    rebalancing empties the block), and one of 70,000 pins (32-bit counts); both application paths
    against the oracle."""
    monkeypatch.setenv("JET_APPLY_DIVISOR", str(divisor))
    rng = np.random.default_rng(size)
    n, k = 72000, 4
    nets = [list(range(size))] + [sorted(rng.choice(n, size=int(sz), replace=False).tolist())
                                  for sz in rng.integers(2, 9, 30000)]
    hg = hg_from_nets(n, nets, k)
    part = (np.arange(n) % k).astype(np.int32)
    part[:size] = 0
    say("largest net", size, "divisor", divisor)
    ctx = ctx_for(hg)
    assert ctx.km1(dev(part)) == O.km1(hg, part)
    ctx.close()
    check_refine(hg, part, tau=(0.75, 0.0), limit=4)


def test_afterburner_many_overflow_nets_repeatable():
    """Hundreds of nets beyond the in-LDS capacity, k = 128, almost every pin a candidate (the shape
    of the SAT-like workload): every run equals the oracle."""
    rng = np.random.default_rng(77)
    n, k = 30000, 128
    nets = [sorted(rng.choice(n, size=int(s), replace=False).tolist()) for s in rng.integers(4200, 12000, 150)]
    nets += [sorted(rng.choice(n, size=int(s), replace=False).tolist()) for s in rng.integers(2, 11, 20000)]
    order = rng.permutation(len(nets))
    hg = hg_from_nets(n, [nets[i] for i in order], k)
    part = rng.integers(0, k, n).astype(np.int32)
    t = ((part + rng.integers(1, k, n)) % k).astype(np.int32)
    g = rng.integers(-3, 4, n).astype(np.int32)
    inM = (rng.random(n) < 0.9995).astype(np.uint8)
    ref = O.afterburner(hg, part, t, g, inM)
    ctx = ctx_for(hg)
    for rep in range(3):
        say("repeat", rep)
        rg = host(ctx.afterburner(dev(part), dev(t), dev(g), dev(inM, torch.uint8)))
        bad = np.nonzero(rg != ref)[0]
        assert bad.size == 0, (rep, bad[:10].tolist(), rg[bad[:10]].tolist(), ref[bad[:10]].tolist())
    ctx.close()


@pytest.mark.parametrize("k", [2, 8])
def test_imbalanced_heavy_vertex(k):
    """A vertex heavier than Lmax (Section 2's balance constraint cannot hold; Section 4.3's
    heavy-vertex rule keeps it in place): refinement and rebalancing return JET_IMBALANCED with a
    valid partition equal to the oracle's, and the same statistics and trace."""
    J = jet_mod()
    hg = W.random_hypergraph(600, 900, k, seed=21 + k, vw_max=3)
    vw = hg.vtx_w.copy()
    vw[17] = 2 * int(vw.sum())  # two thirds of the total weight: above Lmax for every k >= 2
    hg.vtx_w = vw
    part = W.part_roundrobin(hg.n, k, 5)
    out, st = check_refine(hg, part, tau=(0.75, 0.0), limit=6)
    assert st["balanced"] == 0
    assert out.min() >= 0 and out.max() < k
    ctx = ctx_for(hg)
    d = dev(part)
    rc, gst = ctx.rebalance(d)
    ref, orc, ost = O.rebalance(hg, part)
    assert rc == orc == J.JET_IMBALANCED
    assert np.array_equal(host(d), ref)
    assert gst["rebalance_rounds"] == ost["rebalance_rounds"] and gst["max_block_weight"] == ost["max_block_weight"]
    ctx.close()


def test_overflow_errors():
    """jet_init rejects a vertex whose incident net weights sum to 2^31 or more, and a total vertex
    weight of 2^31 or more, with JET_EOVERFLOW (the integer ranges of the exact arithmetic)."""
    J = jet_mod()
    big = (1 << 30) + 1
    hg = hg_from_nets(4, [[0, 1], [0, 2], [2, 3]], 2, net_w=[big, big, 1])  # vertex 0: 2^31 + 2
    with pytest.raises(J.JetError) as ei:
        ctx_for(hg)
    assert ei.value.code == J.JET_EOVERFLOW
    ok = hg_from_nets(4, [[0, 1], [0, 2], [2, 3]], 2, net_w=[big - 2, big - 2, 1])  # 2^31 - 2: accepted
    ctx_for(ok).close()
    heavy = hg_from_nets(3, [[0, 1], [1, 2]], 2, vtx_w=[1 << 30, 1 << 30, 1])
    with pytest.raises(J.JetError) as ei:
        ctx_for(heavy)
    assert ei.value.code == J.JET_EOVERFLOW


@pytest.mark.parametrize("knobs", [dict(graph=0, slots=1, replays=1), dict(graph=1, slots=1, replays=8),
                                   dict(graph=1, slots=3, replays=2), dict(graph=1, slots=1, replays=64)],
                         ids=["eager", "graph-1x8", "graph-3x2", "graph-1x64"])
@pytest.mark.parametrize("case", [CASES[1], CASES[4], CASES[8], CASES[10]], ids=lambda c: f"k{c[3]}-s{c[0]}")
def test_refine_device_loop_knobs(case, knobs):
    """The device-resident loop (Algorithm 1 on the device): launched one kernel at a time or replayed
    from a captured graph, with 1 or 3 rebalancing rounds per replay and 1 to 64 replays between host
    polls, gives the oracle's partition, statistics and per-iteration records every time."""
    J = jet_mod()
    seed, n, m, k, smax, vw, nwm, big = case
    say("case", case, "knobs", knobs)
    hg = mixed_sizes(seed, n, m, k, smax, vw, nwm, big)
    part = W.part_roundrobin(hg.n, k, seed + 3)
    part[: hg.n // 5] = 0  # overloaded start: rebalancing rounds in the first iterations
    kw = dict(tau=(0.75, 0.375, 0.0), limit=6)
    ctx = ctx_for(hg)
    ctx.set_option(J.JET_OPT_GRAPH, knobs["graph"])
    ctx.set_option(J.JET_OPT_RB_SLOTS, knobs["slots"])
    ctx.set_option(J.JET_OPT_REPLAYS, knobs["replays"])
    ref = O.refine(hg, part, **kw)
    for rep in range(2):  # the second call replays the graph captured by the first
        d = dev(part)
        rc, st, tr = ctx.refine(d, trace_cap=4096, **kw)
        assert rc == ref[1]
        assert sha(host(d)) == sha(ref[0])
        for key in ("km1_in", "km1_out", "iterations", "rebalance_rounds", "moves_executed", "max_block_weight"):
            assert st[key] == ref[2][key], key
        assert tr == ref[3]
    d = dev(part)
    rc, st = ctx.rebalance(d)
    ob, orc, ost = O.rebalance(hg, part)
    assert rc == orc and np.array_equal(host(d), ob) and st["rebalance_rounds"] == ost["rebalance_rounds"]
    ctx.close()


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("case", [CASES[1], CASES[3], CASES[5], CASES[7], CASES[9], CASES[11]],
                         ids=lambda c: f"k{c[3]}-s{c[0]}")
def test_unweighted_rebalancing_priority(case, order):
    """The original Jet rebalancer's orders, ablations Section 4.3 contrasts with its weighted
    priority: the gain alone (jet_params.rb_unweighted = 1) and the bucket order of the loss (2).
    On weighted inputs: whole refinements with an overloaded start and the rebalancing call,
    against the oracle run with the same order; and the batch of several such hypergraphs."""
    J = jet_mod()
    seed, n, m, k, smax, vw, nwm, big = case
    say("case", case)
    hg = mixed_sizes(seed, n, m, k, smax, max(vw, 4), nwm, big)
    part = W.part_roundrobin(hg.n, k, seed + 9)
    part[: hg.n // 4] = 0
    out, st = check_refine(hg, part, tau=(0.75, 0.0), limit=6, rb_unweighted=order)
    ctx = ctx_for(hg)
    d = dev(part)
    rc, rst = ctx.rebalance(d, rb_unweighted=order)
    ob, orc, ost = O.rebalance(hg, part, rb_unweighted=order)
    assert rc == orc and (host(d) == ob).all() and rst["rebalance_rounds"] == ost["rebalance_rounds"]
    ctx.close()
    batch = J.JetBatch([hg, hg])
    parts = [dev(part), dev(W.part_roundrobin(hg.n, k, seed + 10))]
    starts = [host(p).copy() for p in parts]
    brc, bst, brcs = batch.refine(parts, tau=(0.75, 0.0), limit=6, rb_unweighted=order)
    for i in range(2):
        opart, orc, ost, _ = O.refine(hg, starts[i], tau=(0.75, 0.0), limit=6, rb_unweighted=order)
        assert brcs[i] == orc and sha(host(parts[i])) == sha(opart) and bst[i]["km1_out"] == ost["km1_out"]
    batch.close()
