"""Connected components of the similarity graph and their weighted precision
and recall against family labels (Section VI-B, Table II), on the GPU
against the oracle: component labels element by element (each vertex gets
the smallest vertex of its component, a canonical labelling), scores exactly
(both are ratios of the same integer counts)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _edges_dev(i, j, gpu):
    import torch

    from paper_2009_14467_amd._binding import EDGE_DTYPE

    e = np.zeros(len(i), EDGE_DTYPE)
    e["i"], e["j"] = i, j
    return torch.from_numpy(e.view(np.uint8).copy()).to(gpu)


def _dev(x, gpu):
    import torch

    a = np.ascontiguousarray(x)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(gpu)


def _graphs():
    rng = np.random.default_rng(17)
    out = []
    for n, m in [(1, 0), (5, 0), (100, 50), (3000, 2000), (100_000, 300_000), (200_000, 60_000)]:
        out.append((f"random-{n}-{m}", n, rng.integers(0, n, m), rng.integers(0, n, m)))
    # a long path given in random order: deep trees for the hooks to merge
    n = 50_000
    perm = rng.permutation(n)
    order = rng.permutation(n - 1)
    out.append(("path", n, perm[order], perm[order + 1]))
    # a star around the largest vertex, and self-loops
    out.append(("star", 1000, np.full(999, 999), np.arange(999)))
    out.append(("loops", 10, np.arange(10), np.arange(10)))
    return out


@pytest.mark.parametrize("case", _graphs(), ids=lambda c: c[0])
def test_components_match_oracle(gpu, orc, case):
    import paper_2009_14467_amd as P

    _, n, i, j = case
    ctx = P.Context(P.Params())
    got = ctx.components(_edges_dev(i, j, gpu), n).cpu().numpy().view(np.uint32)
    want = orc.components(n, i, j)
    np.testing.assert_array_equal(got, want)


def test_components_reject_bad_endpoints(gpu):
    import paper_2009_14467_amd as P

    ctx = P.Context(P.Params())
    with pytest.raises(P.PastisError, match="endpoint"):
        ctx.components(_edges_dev([0, 5], [1, 2], gpu), 5)


@pytest.mark.parametrize("n,n_clusters,n_fams", [(1, 1, 1), (50, 7, 5), (20_000, 300, 900), (250_000, 40_000, 10_000)])
def test_scores_match_oracle(gpu, orc, n, n_clusters, n_fams):
    import paper_2009_14467_amd as P

    rng = np.random.default_rng(n)
    clus = rng.integers(0, n_clusters, n).astype(np.uint32)
    fam = rng.integers(0, n_fams, n).astype(np.int32)
    fam[rng.random(n) < 0.2] = -1  # sequences outside every family
    ctx = P.Context(P.Params())
    got = ctx.cluster_scores(_dev(clus, gpu), _dev(fam, gpu))
    assert got == orc.weighted_scores(clus, fam)


def test_scores_reject_labels_out_of_range(gpu):
    import paper_2009_14467_amd as P

    ctx = P.Context(P.Params())
    with pytest.raises(P.PastisError, match=">= n"):
        ctx.cluster_scores(_dev(np.array([0, 5], np.uint32), gpu), _dev(np.array([0, 0], np.int32), gpu))
    with pytest.raises(P.PastisError, match=">= n"):
        ctx.cluster_scores(_dev(np.array([0, 1], np.uint32), gpu), _dev(np.array([0, 2], np.int32), gpu))


@pytest.mark.parametrize("m", [0, 10, 25])
def test_search_components_as_families(gpu, orc, m):
    """The Table II pipeline at test scale: search edges (30% identity, 70%
    coverage), their components as families, scored against the generator's
    family labels; components and scores against the oracle on the same edges."""
    import paper_2009_14467_amd as P
    from synth import workload

    s = workload("mid", n_families=40)
    res, off = _dev(s.residues, gpu), _dev(s.offsets, gpu)
    ctx = P.Context(P.Params(k=6, n_subs=m, ck_min=2))
    edges = ctx.search(res, off)
    assert edges.size > 0
    lab = ctx.components(_edges_dev(edges["i"], edges["j"], gpu), s.n)
    want = orc.components(s.n, edges["i"], edges["j"])
    np.testing.assert_array_equal(lab.cpu().numpy().view(np.uint32), want)
    p, r = ctx.cluster_scores(lab, _dev(s.labels.astype(np.int32), gpu))
    assert (p, r) == orc.weighted_scores(want, s.labels)
    assert 0 < p <= 1 and 0 < r <= 1
