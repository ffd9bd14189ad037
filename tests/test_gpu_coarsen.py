"""GPU parity of the synchronous clustering (Section 6, Algorithm 4; jet_coarsen and
jet_coarsen_subround) against the oracle: cluster labels and counts bit for bit.

* single sub-rounds on random clusterings (targets after swap prevention, labels and cluster
  weights after the moves), sub-rounds of one vertex up to all vertices;
* whole passes on random hypergraphs with weights, the paper's schedule and schedules with large
  sub-rounds (many conflicting proposals, swaps, groups above the LDS sort capacity);
* the rating tables split over many launches (a tiny table-slot option) give the same labels;
* bad orders are rejected;
* the VLSI-like benchmark hypergraph (1M vertices) at full size, and a row-net hypergraph with
  Zipf net sizes up to 10^4 pins (100k vertices).
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


def random_clustering(hg, seed, frac=0.3):
    rng = np.random.default_rng(seed)
    vw = np.ones(hg.n, dtype=np.int64) if hg.vtx_w is None else hg.vtx_w.astype(np.int64)
    label = np.arange(hg.n, dtype=np.int32)
    cw = vw.copy()
    for v in rng.choice(hg.n, int(hg.n * frac), replace=False):
        t = int(rng.integers(hg.n))
        if label[v] == v and cw[v] == vw[v] and t != v and label[t] == t:
            label[v] = t
            cw[t] += vw[v]
            cw[v] -= vw[v]
    return label, cw


@pytest.mark.parametrize("seed,nb,wmax", [(1, 1, 8), (2, 17, 8), (3, 600, 6), (4, 2000, 12), (5, 2000, 3)])
def test_subround_matches_oracle(seed, nb, wmax):
    say(f"coarsen sub-round seed={seed} nb={nb} wmax={wmax}")
    hg = W.random_hypergraph(2000, 3000, 4, 400 + seed, smin=2, smax=10, nw_max=4 if seed % 2 else 1,
                             vw_max=3 if seed > 2 else 1)
    label, cw = random_clustering(hg, seed)
    B = np.random.default_rng(seed).permutation(hg.n)[:nb].astype(np.int32)
    olab, ocw, oT, _ = O.coarsen_subround(hg, label, cw, B, wmax)
    ctx = J().JetContext(hg)
    dl, dc = dev(label), dev(cw, torch.int64)
    T = ctx.coarsen_subround(dl, dc, dev(B), wmax)
    assert np.array_equal(T.cpu().numpy(), oT)
    assert np.array_equal(dl.cpu().numpy(), olab)
    assert np.array_equal(dc.cpu().numpy(), ocw)
    # an empty sub-round leaves everything alone
    T = ctx.coarsen_subround(dl, dc, dev(np.zeros(0, np.int32)), wmax)
    assert int((T >= 0).sum()) == 0 and np.array_equal(dl.cpu().numpy(), olab)


CASES = [
    # (seed, n, m, smax, nw_max, vw_max, wmax, initial_single, cap_div)
    (1, 3000, 5000, 8, 1, 1, 4, 100, 100),
    (2, 5000, 6000, 12, 5, 3, 10, 100, 100),
    (3, 5000, 6000, 12, 1, 2, 20, 0, 4),      # sub-rounds up to n/4: many conflicts and swaps
    (4, 8000, 4000, 30, 3, 1, 50, 0, 1),      # doubling up to n: groups above the LDS sort capacity
    (5, 400, 900, 6, 2, 4, 7, 100, 100),      # every sub-round holds one vertex
]


@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
def test_pass_matches_oracle(case):
    seed, n, m, smax, nwm, vwm, wmax, first, div = case
    say(f"coarsen pass {case}")
    hg = W.random_hypergraph(n, m, 4, 500 + seed, smin=2, smax=smax, nw_max=nwm, vw_max=vwm)
    order = np.random.default_rng(seed).permutation(n).astype(np.int32)
    olab, ocnt = O.coarsen(hg, order, wmax, first, div)
    ctx = J().JetContext(hg)
    lab, cnt = ctx.coarsen(dev(order), wmax, first, div)
    assert cnt == ocnt
    assert np.array_equal(lab.cpu().numpy(), olab)
    # again on the same context (state left clean between calls)
    lab2, cnt2 = ctx.coarsen(dev(order), wmax, first, div)
    assert cnt2 == cnt and torch.equal(lab, lab2)


def test_star_group_above_sort_capacity():
    """A centre with 5,000 two-pin nets to leaves; one sub-round holds thousands of leaves that all
    propose the centre: the group exceeds the LDS sort and takes the rank-sum path."""
    n = 5001
    nets = [[0, i] for i in range(1, n)]
    off = np.arange(0, 2 * len(nets) + 1, 2, dtype=np.int64)
    pins = np.array([v for e in nets for v in e], dtype=np.int32)
    vw = (np.arange(n) % 5 + 1).astype(np.int32)
    hg = W.Hypergraph(n=n, m=len(nets), off=off, pins=pins, k=2, eps=0.03, vtx_w=vw)
    order = np.concatenate([[0], np.random.default_rng(7).permutation(np.arange(1, n))]).astype(np.int32)
    for wmax in (40, 3000):
        olab, ocnt = O.coarsen(hg, order, wmax, 0, 1)
        ctx = J().JetContext(hg)
        lab, cnt = ctx.coarsen(dev(order), wmax, 0, 1)
        assert cnt == ocnt and np.array_equal(lab.cpu().numpy(), olab)


def test_table_split_over_launches():
    hg = W.random_hypergraph(4000, 6000, 4, 77, smin=2, smax=20, nw_max=3, vw_max=2)
    order = np.random.default_rng(77).permutation(hg.n).astype(np.int32)
    olab, ocnt = O.coarsen(hg, order, 12, 10, 10)
    ctx = J().JetContext(hg)
    ctx.set_option(J().JET_OPT_CO_TABLE_SLOTS, 64)
    lab, cnt = ctx.coarsen(dev(order), 12, 10, 10)
    assert cnt == ocnt and np.array_equal(lab.cpu().numpy(), olab)


def test_bad_orders_rejected():
    hg = W.random_hypergraph(300, 400, 4, 3)
    ctx = J().JetContext(hg)
    bad = np.arange(hg.n, dtype=np.int32)
    bad[5] = 6
    with pytest.raises(J().JetError, match="order"):
        ctx.coarsen(dev(bad), 10)
    bad[5] = hg.n
    with pytest.raises(J().JetError, match="order"):
        ctx.coarsen(dev(bad), 10)
    with pytest.raises(J().JetError):
        ctx.coarsen(dev(np.arange(hg.n, dtype=np.int32)), 0)
    lab, cnt = ctx.coarsen(dev(np.arange(hg.n, dtype=np.int32)), 10)  # the context still works
    assert 0 < cnt < hg.n


def test_vlsi_full_size_pass():
    say("coarsen: VLSI-like 1M vertices")
    hg, _ = W.vlsi_like(seed=2)
    W_total = int(hg.vtx_w.astype(np.int64).sum())
    wmax = -(-W_total // (160 * 8))   # ceil(W / (160 k)) at k = 8
    order = np.random.default_rng(2).permutation(hg.n).astype(np.int32)
    ctx = J().JetContext(hg)
    lab, cnt = ctx.coarsen(dev(order), wmax)
    say(f"coarsen: GPU {cnt} clusters; oracle")
    olab, ocnt = O.coarsen(hg, order, wmax)
    assert cnt == ocnt and np.array_equal(lab.cpu().numpy(), olab)
    assert cnt < hg.n * 0.75


def test_rownet_zipf_pass():
    say("coarsen: row-net 100k vertices, nets up to 10^4 pins")
    hg = W.rownet_matrix(seed=9, n=100_000, k=64)
    wmax = -(-hg.n // (160 * 64))
    order = np.random.default_rng(9).permutation(hg.n).astype(np.int32)
    ctx = J().JetContext(hg)
    lab, cnt = ctx.coarsen(dev(order), wmax)
    olab, ocnt = O.coarsen(hg, order, wmax)
    assert cnt == ocnt and np.array_equal(lab.cpu().numpy(), olab)
