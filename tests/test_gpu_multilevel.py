"""Multilevel deterministic Jet with GPU clustering (Section 6, Algorithm 4; Sections 2 and 4):
every level's clustering, with the paper's prefix-doubling schedule and with three equal
sub-rounds, equals the oracle's on an oracle-built chain of levels (the oracle clusters, the host
contraction contracts), and the refinement of the whole hierarchy, coarsest to finest, ends in the
oracle's partition."""
import hashlib
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


def oracle_level(hg, order, wmax, schedule):
    if schedule == "prefix-doubling":
        return O.coarsen(hg, order, wmax)[0]
    label = np.arange(hg.n, dtype=np.int32)
    cw = np.ones(hg.n, np.int64) if hg.vtx_w is None else hg.vtx_w.astype(np.int64)
    for part in np.array_split(order, 3):
        label, cw, _, _ = O.coarsen_subround(hg, label, cw, part, wmax)
    return label


def oracle_chain(hg, seed, schedule, ML):
    limit = 160 * hg.k
    wmax = ML.max_cluster_weight(hg, limit)
    hgs, parents = [hg], []
    while hgs[-1].n > limit:
        cur = hgs[-1]
        lab = oracle_level(cur, ML.level_order(cur.n, seed, len(hgs) - 1), wmax, schedule)
        uniq, inv = np.unique(lab, return_inverse=True)
        if uniq.size > cur.n - cur.n // 100:
            break
        parents.append(inv.astype(np.int32))
        hgs.append(W.contract(cur, parents[-1], int(uniq.size)))
    return hgs, parents


CASES = {
    "random-k8": lambda: W.random_hypergraph(24000, 30000, 8, 61, smin=2, smax=8, nw_max=3, vw_max=3),
    "rownet-k4": lambda: W.rownet_matrix(seed=62, n=20000, k=4, cap=400),
}


@pytest.mark.parametrize("schedule", ["prefix-doubling", "three-equal"])
@pytest.mark.parametrize("case", list(CASES))
def test_multilevel_matches_oracle(case, schedule):
    import paper_2504_12013_amd.multilevel as ML
    hg = CASES[case]()
    say(f"multilevel {case} {schedule}: n={hg.n} pins={hg.p} k={hg.k}")
    hgs, parents, ctxs, _ = ML.cluster_hierarchy(hg, 5, schedule)
    ohgs, oparents = oracle_chain(hg, 5, schedule, ML)
    say(f"  levels gpu {[h.n for h in hgs]} oracle {[h.n for h in ohgs]}")
    assert len(hgs) == len(ohgs) >= 3
    for a, b in zip(parents, oparents):
        assert np.array_equal(a, b)
    start = W.greedy_initial(hgs[-1], seed=5)
    from paper_2504_12013_amd.ablations import VARIANTS, run_variant
    v = VARIANTS["detjet"]
    pars = [torch.from_numpy(p).to("cuda").long() for p in parents]
    part = torch.from_numpy(start).to("cuda", torch.int32)
    opart = start.copy()
    for lvl in range(len(hgs) - 1, -1, -1):
        if lvl < len(hgs) - 1:
            part = part[pars[lvl]].contiguous()
            opart = opart[oparents[lvl]]
        rc, st, _ = ctxs[lvl].refine(part, tau=v["coarse"], limit=v["limit"])
        opart, orc, ost, _ = O.refine(ohgs[lvl], opart, tau=v["coarse"], limit=v["limit"])
        assert rc == orc and st["km1_out"] == ost["km1_out"], lvl
        assert np.array_equal(part.cpu().numpy(), opart), lvl
    say(f"  final km1 {st['km1_out']} sha {hashlib.sha256(opart.tobytes()).hexdigest()[:12]}")
    # the driver's own refinement gives the same result
    km1, _, _, _, _ = run_variant(ctxs, parents, start, v)
    assert km1 == st["km1_out"]
