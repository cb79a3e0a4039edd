"""Oracle: connected components of the similarity graph taken as protein
families, scored against reference families (Section VI-B, Table II).
TEST INFRASTRUCTURE ONLY (see the package docstring).

  * ``components``: plain union-find over the edges; every vertex is
    labelled with the smallest sequence index of its component (a canonical
    labelling, so two correct implementations agree element for element).
  * ``weighted_scores``: weighted precision and recall of a clustering
    against families, in the sense of the protein clustering study the paper
    cites for them: with n_cf the sequences of cluster c in family f and N
    the sequences, precision = sum_c max_f n_cf / N (a cluster mixing
    families loses precision) and recall = sum_f max_c n_cf / N (a family
    split over clusters loses recall).  A sequence outside every family
    (family < 0) is a family of its own.
"""

from __future__ import annotations

import numpy as np


def components(n: int, i, j) -> np.ndarray:
    """Component label of every vertex 0..n-1 of the undirected graph with
    edges (i[e], j[e]): the smallest vertex of its component."""
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    for u, v in zip(np.asarray(i).tolist(), np.asarray(j).tolist()):
        if not (0 <= u < n and 0 <= v < n):
            raise ValueError("edge endpoint out of range")
        ru, rv = find(u), find(v)
        if ru != rv:
            # the smaller root stays the root: it is the smallest vertex of the union
            lo, hi = (ru, rv) if ru < rv else (rv, ru)
            parent[hi] = lo
    return np.array([find(x) for x in range(n)], dtype=np.uint32)


def weighted_scores(cluster, family) -> tuple[float, float]:
    """(weighted precision, weighted recall) of the clustering `cluster`
    against the families `family` (both per sequence; family < 0: a family
    of its own)."""
    cluster = np.asarray(cluster).tolist()
    family = np.asarray(family).tolist()
    n = len(cluster)
    if n == 0:
        return 1.0, 1.0
    counts: dict = {}
    for v, (c, f) in enumerate(zip(cluster, family)):
        key = (c, f if f >= 0 else ("alone", v))
        counts[key] = counts.get(key, 0) + 1
    best_in_cluster: dict = {}
    best_in_family: dict = {}
    for (c, f), m in counts.items():
        best_in_cluster[c] = max(best_in_cluster.get(c, 0), m)
        best_in_family[f] = max(best_in_family.get(f, 0), m)
    return sum(best_in_cluster.values()) / n, sum(best_in_family.values()) / n
