"""Host logic of the multilevel driver (CPU): compaction of cluster labels into coarse vertex
numbers, the seeded per-level vertex order and the maximum cluster weight ⌈c(V) / (160 k)⌉."""
import numpy as np

import workloads as W


def ML():
    import paper_2504_12013_amd.multilevel as m
    return m


def test_compact_numbers_clusters_by_label():
    parent, c = ML().compact(np.array([5, 5, 2, 9, 2, 5], np.int32))
    assert c == 3 and parent.tolist() == [1, 1, 0, 2, 0, 1] and parent.dtype == np.int32


def test_level_order_is_a_seeded_permutation():
    a = ML().level_order(1000, 4, 0)
    assert np.array_equal(np.sort(a), np.arange(1000)) and a.dtype == np.int32
    assert np.array_equal(a, ML().level_order(1000, 4, 0))
    assert not np.array_equal(a, ML().level_order(1000, 4, 1))
    assert not np.array_equal(a, ML().level_order(1000, 5, 0))


def test_max_cluster_weight():
    hg = W.random_hypergraph(1000, 1200, 8, 3, vw_max=5)
    total = int(hg.vtx_w.astype(np.int64).sum())
    assert ML().max_cluster_weight(hg, 160 * 8) == -(-total // 1280)
    hg1 = W.random_hypergraph(1281, 1200, 8, 3)
    assert ML().max_cluster_weight(hg1, 1280) == 2
