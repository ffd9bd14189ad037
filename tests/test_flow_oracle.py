"""Pins of the oracle's flow-based refinement (Section 5), CPU only.

* Maximum flow and both reachable sets against brute force: every assignment of the free vertices
  gives a cut of the pair's induced subhypergraph; the flow must equal the least such cut, S_r the
  intersection of the source sides of all least cuts (inclusion-minimal source side) and T_r the
  complement of their union (inclusion-minimal sink side) (Section 5.1, after Picard and
  Queyranne).
* The region (reading F1) against a breadth-first search written here.
* Two-way refinement: the metric drops by exactly the pair's cut reduction, only the pair's
  vertices move and only between its blocks, and a replaced pair is balanced; a worked example
  with one misplaced vertex per side finds the single bridging net.
* The k-way schedule (reading F4) restated here over the oracle's two-way refinement gives the same
  partition and counts.
"""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W


def induced_cut(hg, part, a, b):
    cut = 0
    for e in range(hg.m):
        bl = {int(part[x]) for x in hg.pins[hg.off[e]:hg.off[e + 1]]}
        if a in bl and b in bl:
            cut += 1 if hg.net_w is None else int(hg.net_w[e])
    return cut


def side_cut(hg, part, a, b, src):
    """Weight of the nets with pair pins on both sides of the source set src (bool over vertices)."""
    cut = 0
    for e in range(hg.m):
        pe = [int(x) for x in hg.pins[hg.off[e]:hg.off[e + 1]] if part[x] in (a, b)]
        sides = {bool(src[x]) for x in pe}
        if len(sides) == 2:
            cut += 1 if hg.net_w is None else int(hg.net_w[e])
    return cut


def brute_force_cuts(hg, part, a, b, term):
    free = [v for v in range(hg.n) if part[v] in (a, b) and term[v] == 0]
    best, sides = None, []
    for bits in itertools.product([0, 1], repeat=len(free)):
        src = np.array([part[v] in (a, b) and term[v] == 1 for v in range(hg.n)])
        for v, bit in zip(free, bits):
            src[v] = bool(bit)
        c = side_cut(hg, part, a, b, src)
        if best is None or c < best:
            best, sides = c, [src]
        elif c == best:
            sides.append(src)
    inter = np.logical_and.reduce(sides)
    union = np.logical_or.reduce(sides)
    pair = np.isin(part, [a, b])
    return best, inter, pair & ~union


@pytest.mark.parametrize("seed", range(12))
def test_mincut_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    weighted = seed % 3 == 1
    hg = W.random_hypergraph(16, 22, 3, 100 + seed, smin=2, smax=4, nw_max=4 if weighted else 1)
    part = rng.integers(0, 3, hg.n).astype(np.int32)
    a, b = 0, 1
    pair = np.flatnonzero(np.isin(part, [a, b]))
    term = np.zeros(hg.n, np.int8)
    # a few terminals on each side, the rest free (at most 12 free vertices)
    for i, v in enumerate(pair):
        if i % 4 == 0:
            term[v] = 1
        elif i % 4 == 1:
            term[v] = 2
    F, sr, tr = O.flow_mincut(hg, part, a, b, term)
    best, inter, sink_min = brute_force_cuts(hg, part, a, b, term)
    assert F == best
    assert np.array_equal(sr, inter)
    assert np.array_equal(tr, sink_min)
    assert not (sr & tr).any()


def test_mincut_chain_closed_form():
    # a path of 2-pin nets 0-1-2-...-9 with weights 5,4,3,2,1,2,3,4,5; source 0, sink 9: the least
    # cut is the weight-1 net in the middle, unique, so S_r = {0..4} and T_r = {5..9}
    n = 10
    pins = np.array([[i, i + 1] for i in range(n - 1)], np.int32).ravel()
    off = np.arange(0, 2 * (n - 1) + 1, 2, dtype=np.int64)
    nw = np.array([5, 4, 3, 2, 1, 2, 3, 4, 5], np.int32)
    hg = W.Hypergraph(n=n, m=n - 1, off=off, pins=pins, k=2, eps=0.03, net_w=nw, vtx_w=None)
    part = np.array([0] * 5 + [1] * 5, np.int32)
    term = np.zeros(n, np.int8)
    term[0], term[9] = 1, 2
    F, sr, tr = O.flow_mincut(hg, part, 0, 1, term)
    assert F == 1
    assert sr.tolist() == [True] * 5 + [False] * 5
    assert tr.tolist() == [False] * 5 + [True] * 5
    # two equal least cuts (weights 1 at both ends of the middle): S_r stops at the first, T_r at the second
    nw2 = np.array([5, 4, 1, 3, 3, 3, 1, 4, 5], np.int32)
    hg2 = W.Hypergraph(n=n, m=n - 1, off=off, pins=pins, k=2, eps=0.03, net_w=nw2, vtx_w=None)
    F2, sr2, tr2 = O.flow_mincut(hg2, part, 0, 1, term)
    assert F2 == 1
    assert sr2.tolist() == [True] * 3 + [False] * 7
    assert tr2.tolist() == [False] * 7 + [True] * 3


def region_reference(hg, part, a, b, alpha):
    vw = np.ones(hg.n, np.int64) if hg.vtx_w is None else hg.vtx_w.astype(np.int64)
    bw = np.bincount(part, weights=vw, minlength=hg.k).astype(np.int64)
    A, lmax, _ = O.limits(int(vw.sum()), hg.k, hg.eps, 0)
    big = int(np.floor((1.0 + alpha * hg.eps) * A))
    nets_of = [[] for _ in range(hg.n)]
    for e in range(hg.m):
        for x in hg.pins[hg.off[e]:hg.off[e + 1]]:
            nets_of[x].append(e)
    out = np.zeros(hg.n, np.int8)
    for side, other, mark in ((a, b, 1), (b, a, 2)):
        bound = max(0, min(big - int(bw[other]), int(bw[side]) - 1))
        level = sorted(v for v in range(hg.n) if part[v] == side and any(
            any(part[x] == other for x in hg.pins[hg.off[e]:hg.off[e + 1]]) for e in nets_of[v]))
        seen, used = set(level), 0
        while level:
            lw = int(vw[level].sum())
            if used + lw <= bound:
                out[level] = mark
                used += lw
            else:
                for v in level:
                    if used + vw[v] > bound:
                        break
                    used += int(vw[v])
                    out[v] = mark
                break
            nxt = set()
            for u in level:
                for e in nets_of[u]:
                    for x in hg.pins[hg.off[e]:hg.off[e + 1]]:
                        if part[x] == side and x not in seen:
                            seen.add(int(x))
                            nxt.add(int(x))
            level = sorted(nxt)
    return out


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("alpha", [0, 1, 4, 16])
def test_region_against_bfs(seed, alpha):
    hg = W.random_hypergraph(400, 300, 4, 200 + seed, smin=2, smax=4, vw_max=3 if seed % 2 else 1)
    part = W.part_roundrobin(hg.n, hg.k, seed)
    for a, b in ((0, 1), (2, 3), (1, 3)):
        assert np.array_equal(O.flow_region(hg, part, a, b, alpha), region_reference(hg, part, a, b, alpha))


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("alpha", [4, 16, 100])
def test_region_deep_levels(seed, alpha):
    # a banded hypergraph in contiguous blocks of 100: the boundary of two blocks is a few vertices
    # wide, so the search runs over many levels and, with a large alpha, reaches the far end of the
    # block, next to a third block
    hg, part = W.banded_hypergraph(400, 4, seed, vw_max=3 if seed % 2 else 1)
    deep = 0
    for a, b in ((0, 1), (1, 2), (2, 1), (3, 2)):
        got = O.flow_region(hg, part, a, b, alpha)
        assert np.array_equal(got, region_reference(hg, part, a, b, alpha)), (a, b)
        deep = max(deep, int((got == 1).sum()))
    assert alpha < 16 or deep > 30  # with room for it, the search went well past the boundary


@pytest.mark.parametrize("seed", range(8))
def test_pair_moves_and_metric(seed):
    k = 4
    hg = W.random_hypergraph(500, 700, k, 300 + seed, smin=2, smax=6, vw_max=3 if seed % 2 else 1,
                             nw_max=3 if seed % 3 == 0 else 1)
    part = W.part_roundrobin(hg.n, k, seed)
    vw = np.ones(hg.n, np.int64) if hg.vtx_w is None else hg.vtx_w.astype(np.int64)
    _, lmax, _ = O.limits(int(vw.sum()), k, hg.eps, 0)
    for a, b in ((0, 1), (1, 2), (0, 3)):
        before = O.km1(hg, part)
        new, replaced, st = O.flow_pair(hg, part, a, b)
        assert st["old_cut"] == induced_cut(hg, part, a, b)
        changed = new != part
        if not replaced:
            assert not changed.any() and st["new_cut"] == st["old_cut"]
            continue
        assert np.isin(part[changed], [a, b]).all() and np.isin(new[changed], [a, b]).all()
        assert st["moved"] == int(changed.sum())
        assert st["new_cut"] == induced_cut(hg, new, a, b) <= st["old_cut"]
        assert O.km1(hg, new) == before - (st["old_cut"] - st["new_cut"])
        bw = np.bincount(new, weights=vw, minlength=k)
        assert bw[a] <= lmax and bw[b] <= lmax
        part = new


def test_pair_worked_example():
    # two groups, the even and the odd vertices of 0..11, every pair inside a group joined by a
    # 2-pin net, and one net {10, 11} between them; vertices 0 and 1 start on the wrong sides.  The
    # regions (two vertices a side at eps = 0.03) hold both, and the least balanced cut is the
    # bridging net alone.
    groups = (range(0, 12, 2), range(1, 12, 2))
    nets = [(i, j) for g in groups for i in g for j in g if i < j] + [(10, 11)]
    pins = np.array(nets, np.int32).ravel()
    off = np.arange(0, 2 * len(nets) + 1, 2, dtype=np.int64)
    hg = W.Hypergraph(n=12, m=len(nets), off=off, pins=pins, k=2, eps=0.03, net_w=None, vtx_w=None)
    part = np.array([1, 0] + [v % 2 for v in range(2, 12)], np.int32)
    assert O.km1(hg, part) == 11
    assert O.flow_region(hg, part, 0, 1).tolist() == [2, 1, 1, 2] + [0] * 8
    new, replaced, st = O.flow_pair(hg, part, 0, 1)
    assert replaced and st["old_cut"] == 11 and st["new_cut"] == 1 and st["moved"] == 2
    assert new.tolist() == [v % 2 for v in range(12)]
    assert O.km1(hg, new) == 1


def schedule_reference(hg, part, alpha, max_rounds):
    """Reading F4 restated over the oracle's two-way refinement."""
    k = hg.k
    active = [True] * k
    part = part.copy()
    counts = dict(rounds=0, matchings=0, pairs=0, accepted=0)
    for _ in range(max_rounds):
        edges = set()
        for e in range(hg.m):
            bl = sorted({int(part[x]) for x in hg.pins[hg.off[e]:hg.off[e + 1]]})
            for i, j in itertools.combinations(bl, 2):
                if active[i] or active[j]:
                    edges.add((i, j))
        if not edges:
            break
        counts["rounds"] += 1
        nxt = [False] * k
        while edges:
            deg = [sum(1 for (i, j) in edges if b in (i, j)) for b in range(k)]
            order = sorted(range(k), key=lambda b: (-deg[b], b))
            mate = [-1] * k
            for i in order:
                if mate[i] >= 0 or deg[i] == 0:
                    continue
                cands = [j for j in range(k) if (min(i, j), max(i, j)) in edges and mate[j] < 0 and j != i]
                if cands:
                    j = min(cands, key=lambda c: (-deg[c], c))
                    mate[i], mate[j] = j, i
            counts["matchings"] += 1
            for i in range(k):
                j = mate[i]
                if j < 0 or j < i:
                    continue
                edges.discard((i, j))
                part, replaced, st = O.flow_pair(hg, part, i, j, alpha)
                counts["pairs"] += 1
                if replaced:
                    counts["accepted"] += 1
                    if st["new_cut"] < st["old_cut"]:
                        nxt[i] = nxt[j] = True
        active = nxt
        if not any(active):
            break
    return part, counts


@pytest.mark.parametrize("seed,k", [(0, 4), (1, 5), (2, 8), (3, 3)])
def test_kway_schedule_restated(seed, k):
    hg = W.random_hypergraph(300, 420, k, 400 + seed, smin=2, smax=5, vw_max=2 if seed % 2 else 1)
    part = W.part_roundrobin(hg.n, k, seed)
    got, st = O.flow_refine(hg, part, max_rounds=4)
    ref, counts = schedule_reference(hg, part, O.FLOW_ALPHA, 4)
    assert np.array_equal(got, ref)
    for key, val in counts.items():
        assert st[key] == val, key
    assert st["km1_in"] == O.km1(hg, part) and st["km1_out"] == O.km1(hg, got) <= st["km1_in"]
    vw = np.ones(hg.n, np.int64) if hg.vtx_w is None else hg.vtx_w.astype(np.int64)
    _, lmax, _ = O.limits(int(vw.sum()), k, hg.eps, 0)
    assert np.bincount(got, weights=vw, minlength=k).max() <= max(lmax, np.bincount(part, weights=vw).max())


def test_bad_arguments():
    hg = W.random_hypergraph(50, 60, 3, 7)
    part = W.part_roundrobin(hg.n, 3, 1)
    with pytest.raises(ValueError):
        O.flow_pair(hg, part, 1, 1)
    with pytest.raises(ValueError):
        O.flow_region(hg, part, 0, 3)
    with pytest.raises(ValueError):
        O.flow_refine(hg, part, alpha=-1)


def pair_loop_reference(hg, part, a, b, alpha):
    """Algorithm 3 with readings F1-F3 restated here, every minimum cut found by enumerating the
    free vertices' sides (brute force, no flow algorithm): returns (new part, replaced, new cut,
    iterations, moved)."""
    vw = np.ones(hg.n, np.int64) if hg.vtx_w is None else hg.vtx_w.astype(np.int64)
    bw = np.bincount(part, weights=vw, minlength=hg.k).astype(np.int64)
    _, lmax, _ = O.limits(int(vw.sum()), hg.k, hg.eps, 0)
    old_cut = induced_cut(hg, part, a, b)
    if old_cut == 0:
        return part.copy(), False, old_cut, 0, 0
    region = region_reference(hg, part, a, b, alpha)
    pair = np.isin(part, [a, b])
    term = np.zeros(hg.n, np.int8)
    term[(part == a) & (region == 0)] = 1
    term[(part == b) & (region == 0)] = 2
    wab = int(bw[a] + bw[b])
    heavier_old = max(int(bw[a]), int(bw[b]))
    iterations = 0
    while True:
        F, sr, tr = brute_force_cuts(hg, part, a, b, term)
        iterations += 1
        if F > old_cut:
            return part.copy(), False, old_cut, iterations, 0
        w1, w2 = int(vw[sr].sum()), int(vw[tr].sum())
        h1, h2 = max(w1, wab - w1), max(w2, wab - w2)
        bal1 = w1 <= lmax and wab - w1 <= lmax
        bal2 = w2 <= lmax and wab - w2 <= lmax
        if bal1 or bal2:
            use1 = bal1 and (not bal2 or h1 <= h2)
            if F < old_cut or (h1 if use1 else h2) < heavier_old:
                src = sr if use1 else (pair & ~tr)
                new = part.copy()
                new[pair] = np.where(src[pair], a, b)
                return new, True, F, iterations, int((new != part).sum())
            return part.copy(), False, old_cut, iterations, 0
        if F >= old_cut:
            return part.copy(), False, old_cut, iterations, 0
        source_side = w1 <= w2
        mine, theirs = (sr, tr) if source_side else (tr, sr)
        term[pair & mine & (term == 0)] = 1 if source_side else 2
        best = None
        for e in range(hg.m):
            pe = [int(x) for x in hg.pins[hg.off[e]:hg.off[e + 1]] if pair[x]]
            if not any(mine[x] for x in pe) or all(mine[x] for x in pe):
                continue
            for x in pe:
                if not mine[x] and term[x] == 0:
                    key = (1 if theirs[x] else 0, x)
                    best = key if best is None or key < best else best
        if best is None:
            return part.copy(), False, old_cut, iterations, 0
        term[best[1]] = 1 if source_side else 2


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("alpha", [4, 16, 100])
def test_pair_loop_against_brute_force(seed, alpha):
    # two blocks of about seven vertices, so a region holds at most a dozen free vertices; some
    # starts are out of balance, so that equal-cut results and balance decide too
    rng = np.random.default_rng(seed)
    hg = W.random_hypergraph(14, 24, 2, 1000 + seed, smin=2, smax=4, vw_max=3 if seed % 2 else 1,
                             nw_max=3 if seed % 3 == 0 else 1)
    part = rng.permutation(np.arange(hg.n) % 2).astype(np.int32)
    if seed % 4 == 3:
        part[rng.choice(np.flatnonzero(part == 1), 2, replace=False)] = 0
    new, replaced, st = O.flow_pair(hg, part, 0, 1, alpha)
    rnew, rrep, rcut, rit, rmoved = pair_loop_reference(hg, part, 0, 1, alpha)
    assert replaced == rrep
    assert st["new_cut"] == rcut and st["iterations"] == rit and st["moved"] == rmoved
    assert np.array_equal(new, rnew)


@pytest.mark.parametrize("seed,k", [(5, 4), (6, 6)])
def test_kway_schedule_restated_unbalanced_start(seed, k):
    # an overloaded block: some pairs are replaced at an equal cut for balance alone, which must
    # not make their blocks active
    hg = W.random_hypergraph(240, 330, k, 500 + seed, smin=2, smax=4)
    part = W.part_roundrobin(hg.n, k, seed)
    rng = np.random.default_rng(seed)
    part[rng.choice(np.flatnonzero(part != 0), 12, replace=False)] = 0
    got, st = O.flow_refine(hg, part, max_rounds=4)
    ref, counts = schedule_reference(hg, part, O.FLOW_ALPHA, 4)
    assert np.array_equal(got, ref)
    for key, val in counts.items():
        assert st[key] == val, key


@pytest.mark.parametrize("seed", [3, 10, 12, 22, 170, 234])
def test_pair_loop_both_sides_balanced_ties(seed):
    # inputs where the two canonical cuts differ, both are balanced and the heavier blocks tie, so
    # only the tie rule of Section 5.2 (prefer the source-side cut) decides; brute force as above
    rng = np.random.default_rng(seed)
    n = 10 + seed % 7
    hg = W.random_hypergraph(n, int(n * 1.7), 2, 5000 + seed, smin=2, smax=4,
                             vw_max=1 + seed % 3, nw_max=1 + (seed // 3) % 2)
    part = rng.permutation(np.arange(hg.n) % 2).astype(np.int32)
    if seed % 4 == 3:
        part[rng.choice(np.flatnonzero(part == 1), 2, replace=False)] = 0
    for alpha in (4, 16, 100):
        new, replaced, st = O.flow_pair(hg, part, 0, 1, alpha)
        rnew, rrep, rcut, rit, rmoved = pair_loop_reference(hg, part, 0, 1, alpha)
        assert replaced == rrep and st["new_cut"] == rcut and st["iterations"] == rit
        assert np.array_equal(new, rnew), alpha


@pytest.mark.parametrize("seed", [4, 75])
def test_kway_schedule_activity_rule(seed):
    # starts where some pairs are replaced at an equal cut, for balance alone; the next round's
    # pairs then depend on such pairs leaving their blocks inactive (reading F4)
    rng = np.random.default_rng(seed)
    k = 3 + seed % 5
    n = 120 + 20 * (seed % 5)
    hg = W.random_hypergraph(n, int(n * 1.4), k, 7000 + seed, smin=2, smax=4, vw_max=1 + seed % 2)
    part = W.part_roundrobin(hg.n, k, seed)
    part[rng.choice(np.flatnonzero(part != 0), n // 20, replace=False)] = 0
    got, st = O.flow_refine(hg, part, max_rounds=4)
    ref, counts = schedule_reference(hg, part, O.FLOW_ALPHA, 4)
    assert np.array_equal(got, ref)
    for key, val in counts.items():
        assert st[key] == val, key


@pytest.mark.parametrize("seed", [4, 6, 18, 19, 24, 42])
def test_pair_loop_equal_cut_rebalances(seed):
    # overloaded starts whose cut is already minimal: the pair is replaced at an equal cut when a
    # balanced bipartition has a lighter heavier block than the start (reading F3); brute force
    rng = np.random.default_rng(seed)
    n = 10 + seed % 7
    hg = W.random_hypergraph(n, int(n * 1.2), 2, 9000 + seed, smin=2, smax=4,
                             vw_max=1 + seed % 2, nw_max=1 + (seed // 2) % 3)
    part = rng.permutation(np.arange(hg.n) % 2).astype(np.int32)
    part[rng.choice(np.flatnonzero(part == 1), 1 + seed % 3, replace=False)] = 0
    equal = 0
    for alpha in (4, 100):
        new, replaced, st = O.flow_pair(hg, part, 0, 1, alpha)
        rnew, rrep, rcut, rit, rmoved = pair_loop_reference(hg, part, 0, 1, alpha)
        assert replaced == rrep and st["new_cut"] == rcut and st["iterations"] == rit
        assert np.array_equal(new, rnew), alpha
        equal += replaced and st["new_cut"] == st["old_cut"]
    assert equal > 0  # the case this test is for happens
