"""Pins of the oracle's rebalancing round for each order (Section 4.3): the paper's priority, which
divides a negative gain by the vertex weight and multiplies a non-negative one by it; the original
Jet rebalancer's, the gain alone; and the original's bucket order of the loss (ablations the paper
contrasts with its own). Buckets: a move that does not lose is in bucket 0, a loss L in bucket
L.bit_length(); a bucket's vertices go in ID order.

The expected round is derived here from the definitions with brute-force gains (the metric
recomputed after each single move), independently of the oracle's gain code: heavy-vertex rule,
valid targets (room for the vertex, outside the deadzone), best target (largest gain, lowest block),
priority order (exact rationals, then vertex ID), and per overloaded block the shortest prefix whose
weight removes the overload.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W


def expected_round(hg, part, unweighted, dz_ppm=100_000):
    vw = np.ones(hg.n, dtype=np.int64) if hg.vtx_w is None else hg.vtx_w.astype(np.int64)
    bw = np.bincount(part, weights=vw, minlength=hg.k).astype(np.int64)
    A, lmax, dz = O.limits(int(vw.sum()), hg.k, hg.eps, dz_ppm)
    per_block = {}
    for v in range(hg.n):
        s, c = int(part[v]), int(vw[v])
        if bw[s] <= lmax or 2 * c > 3 * (bw[s] - A):
            continue
        best, bg = -1, None
        for b in range(hg.k):
            if b == s or bw[b] + c > lmax or bw[b] >= dz:
                continue
            g = O.gain_bruteforce(hg, part, v, b)
            if best < 0 or g > bg:
                best, bg = b, g
        if best < 0:
            continue
        if unweighted == 2:
            prio = Fraction(-(0 if bg >= 0 else (-bg).bit_length()))
        elif unweighted:
            prio = Fraction(bg)
        else:
            prio = Fraction(bg * c) if bg >= 0 else Fraction(bg, c)
        per_block.setdefault(s, []).append((-prio, v, best, c))
    sel = np.full(hg.n, -1, dtype=np.int32)
    for s, items in per_block.items():
        items.sort()
        need, run = int(bw[s] - lmax), 0
        for _, v, t, c in items:
            if run >= need:
                break
            sel[v] = t
            run += c
    return sel


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("unweighted", [0, 1, 2])
def test_round_from_definitions(seed, unweighted):
    hg = W.random_hypergraph(60, 90, 3, 700 + seed, smin=2, smax=5, vw_max=6, nw_max=3)
    rng = np.random.default_rng(seed)
    part = rng.integers(0, 3, hg.n).astype(np.int32)
    part[: hg.n // 2] = 0  # block 0 overloaded
    new, sel, moved = O.rebalance_round(hg, part, unweighted=unweighted)
    exp = expected_round(hg, part, unweighted)
    assert np.array_equal(sel, exp)
    assert moved == int((exp >= 0).sum()) > 0
    assert np.array_equal(new, np.where(exp >= 0, exp, part))


def test_priorities_differ_with_weights_and_agree_without():
    # with vertex weights the two orders select different vertices on some seed ...
    differ = 0
    for seed in range(8):
        hg = W.random_hypergraph(80, 120, 3, 800 + seed, smin=2, smax=5, vw_max=8)
        part = np.random.default_rng(seed).integers(0, 3, hg.n).astype(np.int32)
        part[: hg.n // 2] = 0
        differ += not np.array_equal(O.rebalance_round(hg, part, unweighted=0)[1],
                                     O.rebalance_round(hg, part, unweighted=1)[1])
    assert differ > 0
    # ... and with unit weights they are the same order (g * 1 = g / 1 = g)
    for seed in range(4):
        hg = W.random_hypergraph(80, 120, 3, 900 + seed, smin=2, smax=5)
        part = np.random.default_rng(seed).integers(0, 3, hg.n).astype(np.int32)
        part[: hg.n // 2] = 0
        a = O.refine(hg, part, tau=(0.75, 0.0), limit=6, rb_unweighted=0)
        b = O.refine(hg, part, tau=(0.75, 0.0), limit=6, rb_unweighted=1)
        assert np.array_equal(a[0], b[0]) and a[2] == b[2]


def test_bucket_order_differs_from_the_sort():
    # coarse buckets change the selection against the exact order on some seeds, with and without
    # vertex weights (unit weights: the gain order and the bucket order split ties differently)
    for vw_max in (1, 8):
        differ = 0
        for seed in range(8):
            hg = W.random_hypergraph(80, 120, 3, 1100 + seed, smin=2, smax=6, vw_max=vw_max, nw_max=4)
            part = np.random.default_rng(seed).integers(0, 3, hg.n).astype(np.int32)
            part[: hg.n // 2] = 0
            differ += not np.array_equal(O.rebalance_round(hg, part, unweighted=1)[1],
                                         O.rebalance_round(hg, part, unweighted=2)[1])
        assert differ > 0, vw_max


def test_bucket_order_worked_example():
    # k = 2, unit weights, vertices 0..7 in block 0 and 8, 9 in block 1: c(V) = 10, A = 5,
    # Lmax = floor(1.03 * 5) = 5, so 3 must leave block 0; block 1 (weight 2) is a valid target
    # for every vertex and the heavy-vertex rule (2 > 3 * 3) excludes none.  Nets and weights:
    # {0, 8} 1, {1, 2} 1, {2, 3} 2, {4, 5} 3, {6, 7} 8.  Gains of moving v to block 1, by hand:
    # 0: +1 (its net leaves the cut); 1: -1; 2: -1 - 2 = -3; 3: -2; 4, 5: -3; 6, 7: -8.
    # Buckets: 0 | 1 | 2, 3, 4, 5 (losses 2..3) | 6, 7 (loss 8).
    # Sorted by gain: 0, 1, 3, 2, 4, 5, 6, 7 -> the first three are {0, 1, 3}.
    # Bucket order: 0 | 1 | 2, 3, 4, 5 in ID order -> {0, 1, 2}.
    nets = [(0, 8), (1, 2), (2, 3), (4, 5), (6, 7)]
    pins = np.array(nets, np.int32).ravel()
    off = np.arange(0, 2 * len(nets) + 1, 2, dtype=np.int64)
    hg = W.Hypergraph(n=10, m=len(nets), off=off, pins=pins, k=2, eps=0.03,
                      net_w=np.array([1, 1, 2, 3, 8], np.int32), vtx_w=None)
    part = np.array([0] * 8 + [1, 1], np.int32)
    _, lmax, _ = O.limits(10, 2, 0.03, 100_000)
    assert lmax == 5
    assert [O.gain_bruteforce(hg, part, v, 1) for v in range(8)] == [1, -1, -3, -2, -3, -3, -8, -8]
    expect = {0: [1, 1, -1, 1, -1, -1, -1, -1], 2: [1, 1, 1, -1, -1, -1, -1, -1]}
    for order in (0, 1, 2):
        new, sel, moved = O.rebalance_round(hg, part, unweighted=order)
        assert sel[:8].tolist() == expect[2 if order == 2 else 0], order
        assert moved == 3 and (sel[8:] == -1).all()


@pytest.mark.parametrize("seed", [19, 85, 116, 139, 182, 199, 209, 230, 239, 266])
@pytest.mark.parametrize("unweighted", [0, 1, 2])
def test_round_with_a_heavy_vertex(seed, unweighted):
    # one vertex of the overloaded block 0 weighs more than 3/2 (c(V_0) - ceil(c(V)/k)) and still
    # has a valid target: Section 4.3's rule alone keeps it in place
    hg, part, heavy = W.overloaded_with_heavy_vertex(seed)
    k = hg.k
    vw = hg.vtx_w.astype(np.int64)
    bw = np.bincount(part, weights=vw, minlength=k).astype(np.int64)
    A, lmax, dz = O.limits(int(vw.sum()), k, hg.eps)
    c = int(vw[heavy])
    assert bw[0] > lmax and 2 * c > 3 * (bw[0] - A)
    assert any(b != 0 and bw[b] + c <= lmax and bw[b] < dz for b in range(k))
    new, sel, moved = O.rebalance_round(hg, part, unweighted=unweighted)
    assert np.array_equal(sel, expected_round(hg, part, unweighted))
    assert sel[heavy] == -1
