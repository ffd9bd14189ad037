"""The host contraction that builds coarse levels from a clustering (Section 6 reuses an existing
contraction): summed vertex weights, every net mapped to its coarse pins with duplicates removed,
nets left with one pin dropped, parallel nets kept, net order and weights preserved.  Checked
against that definition written out with Python sets, and against the random-matching levels."""
import numpy as np
import pytest

import workloads as W


def expected(hg, parent, nc):
    vw = np.ones(hg.n, np.int64) if hg.vtx_w is None else hg.vtx_w.astype(np.int64)
    cvw = np.zeros(nc, np.int64)
    np.add.at(cvw, parent, vw)
    nets, weights = [], []
    for e in range(hg.m):
        s = sorted({int(parent[v]) for v in hg.pins[hg.off[e]:hg.off[e + 1]]})
        if len(s) >= 2:
            nets.append(s)
            weights.append(1 if hg.net_w is None else int(hg.net_w[e]))
    return cvw, nets, weights


@pytest.mark.parametrize("seed", range(4))
def test_contract_matches_definition(seed):
    hg = W.random_hypergraph(300, 400, 4, 40 + seed, smin=1, smax=7, nw_max=5 if seed % 2 else 1, vw_max=4)
    rng = np.random.default_rng(seed)
    nc = [1, 7, 150, 300][seed]
    parent = rng.integers(0, nc, hg.n).astype(np.int32)
    c = W.contract(hg, parent, nc)
    cvw, nets, weights = expected(hg, parent, nc)
    assert c.n == nc and np.array_equal(c.vtx_w.astype(np.int64), cvw)
    assert c.m == len(nets)
    assert [c.pins[c.off[e]:c.off[e + 1]].tolist() for e in range(c.m)] == nets
    if hg.net_w is None:
        assert c.net_w is None
    else:
        assert c.net_w.tolist() == weights


def test_contract_reproduces_matching_levels():
    hg = W.random_hypergraph(4000, 6000, 4, 9, smin=2, smax=9, nw_max=3, vw_max=3)
    hgs, parents = W.hierarchy(hg, 4, 13)
    for lvl in range(3):
        c = W.contract(hgs[lvl], parents[lvl], hgs[lvl + 1].n)
        nxt = hgs[lvl + 1]
        for a, b in ((c.off, nxt.off), (c.pins, nxt.pins), (c.vtx_w, nxt.vtx_w), (c.net_w, nxt.net_w)):
            assert np.array_equal(a, b)


def test_contract_rejects_bad_parent():
    hg = W.random_hypergraph(50, 60, 2, 3, smin=2, smax=4)
    parent = np.zeros(hg.n, np.int32)
    parent[7] = 5
    with pytest.raises(ValueError):
        W.contract(hg, parent, 5)
    parent[7] = -1
    with pytest.raises(ValueError):
        W.contract(hg, parent, 5)
