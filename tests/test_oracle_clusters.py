"""Pins for the oracle's connected components and weighted precision /
recall (Section VI-B, Table II).

Components are checked against scipy's connected_components (a library
routine; the partitions must agree and the labels must be each component's
smallest vertex) and hand-built graphs; the scores against hand-worked
contingency tables and the closed forms of the extreme clusterings."""

import numpy as np
import pytest


def test_components_hand_built(orc):
    # 0-1-2 chain, 3 alone, 4-5 and 6-5, a self-contained 7-7 loop
    lab = orc.components(8, [1, 2, 5, 6, 7], [0, 1, 4, 5, 7])
    assert lab.tolist() == [0, 0, 0, 3, 4, 4, 4, 7]
    assert orc.components(0, [], []).size == 0
    assert orc.components(3, [], []).tolist() == [0, 1, 2]
    with pytest.raises(ValueError):
        orc.components(2, [0], [2])


def test_components_match_scipy(orc):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    rng = np.random.default_rng(11)
    for n, m in [(50, 30), (300, 280), (1000, 2000), (2000, 500)]:
        i = rng.integers(0, n, m)
        j = rng.integers(0, n, m)
        lab = orc.components(n, i, j)
        g = sp.coo_matrix((np.ones(m), (i, j)), shape=(n, n))
        k, ref = connected_components(g, directed=False)
        # same partition
        pairs = set(zip(lab.tolist(), ref.tolist()))
        assert len(pairs) == k == np.unique(lab).size
        # canonical labels: the smallest member of each component
        for c in np.unique(ref):
            members = np.nonzero(ref == c)[0]
            assert (lab[members] == members.min()).all()


def test_weighted_scores_hand_worked(orc):
    # clusters {0,1,2} {3,4}; families {0,1} {2,3,4}
    # n_cf: C0: F0 2, F1 1; C1: F1 2 -> precision (2 + 2) / 5, recall (2 + 2) / 5
    p, r = orc.weighted_scores([0, 0, 0, 3, 3], [7, 7, 9, 9, 9])
    assert (p, r) == (4 / 5, 4 / 5)
    # clusters {0,1} {2} {3,4,5}; families {0,1,2,3} {4,5}
    # C0: F0 2; C1: F0 1; C2: F0 1, F1 2 -> precision (2+1+2)/6; recall F0 max 2, F1 2 -> 4/6
    p, r = orc.weighted_scores([0, 0, 2, 3, 3, 3], [1, 1, 1, 1, 2, 2])
    assert (p, r) == (5 / 6, 4 / 6)


def test_weighted_scores_extremes(orc):
    rng = np.random.default_rng(2)
    fam = rng.integers(0, 7, 200)
    fam[:20] = -1  # sequences outside every family: a family each
    sizes = np.bincount(fam[fam >= 0])
    n = fam.size
    # the families themselves: both 1
    clus = np.where(fam >= 0, fam, 100 + np.arange(n))
    assert orc.weighted_scores(clus, fam) == (1.0, 1.0)
    # everything in one cluster: precision = largest family / N, recall = 1
    p, r = orc.weighted_scores(np.zeros(n, int), fam)
    assert p == sizes.max() / n and r == 1.0
    # every sequence alone: precision 1, recall = number of families / N
    p, r = orc.weighted_scores(np.arange(n), fam)
    assert p == 1.0 and r == (sizes.size + 20) / n
