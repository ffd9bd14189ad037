"""What the trained temperature network gains over the fixed schedule (GPU).

The benchmark's row-net workload (4M vertices, k = 64, 12-level hierarchy) on held-out seeds 41-43
(training used seeds 1000-1045 at 2^14-2^20 vertices): the whole hierarchy is refined once with
the paper's fixed schedule and once with the shipped network's temperatures.  The network's final
metric is lower on every seed, also against the fixed schedule given equal GPU time (extra tau = 0
rounds appended while the learned run took more than 1.05x its time).  (At 2^18 vertices the
network is not better on average: seeds 44-46 give ratios 0.975, 1.041, 0.998.)
"""
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

torch = pytest.importorskip("torch")

NET = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2504_12013_amd", "tau_net.bin")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_network_beats_fixed_schedule_on_held_out_seeds():
    from paper_2504_12013_amd import TauNet
    from paper_2504_12013_amd.tau_training import fixed_at_equal_time, run_hierarchy
    net = TauNet(path=NET)
    ratios = []
    for seed in (41, 42, 43):
        hg = W.rownet_matrix(seed=seed, n=4_000_000, k=64)
        hgs, parents = W.hierarchy(hg, 12, seed=seed)
        start = W.greedy_initial(hgs[-1], seed=seed)
        kf, tf, itf, _, _ = run_hierarchy(hgs, parents, start, None)
        kl, tl, itl, taus, fell_back = run_hierarchy(hgs, parents, start, net)
        kfe, tfe, rounds = fixed_at_equal_time(hgs, parents, start, tl)
        print(f"seed {seed}: fixed km1 {kf} ({tf:.2f}s, {itf} it), learned km1 {kl} ({tl:.2f}s, {itl} it, "
              f"{fell_back} rounds on the fixed temperature), fixed at equal time {kfe} ({rounds} rounds, "
              f"{tfe:.2f}s), finest-level tau {taus[-1]}", flush=True)
        assert tl <= 1.05 * tfe or rounds == 8
        assert kl <= kfe
        ratios.append(kl / kf)
    print("km1 learned / fixed:", [round(r, 4) for r in ratios], "geomean", float(np.exp(np.mean(np.log(ratios)))))
    assert max(ratios) < 1.0
