"""Parity of the HIP candidate discovery with the CPU oracle (Sections IV-A to
IV-C, threshold of Section VI): every candidate field compared bit for bit."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("lo", "hi", "count", "seed1", "seed2")


def _dev(x, gpu):
    import torch

    a = np.ascontiguousarray(x)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(gpu)


def _gpu_candidates(gpu, residues, offsets, **params):
    import paper_2009_14467_amd as P

    ctx = P.Context(P.Params(**params))
    nc = ctx.discover(_dev(residues, gpu), _dev(offsets, gpu))
    c = ctx.candidates(nc)
    return {k: v.cpu().numpy().view(np.uint32) for k, v in c.items()}


def _compare(got, want):
    for f in FIELDS:
        assert got[f].shape == want[f].shape, f"{f}: {got[f].shape} vs {want[f].shape}"
        bad = np.nonzero(got[f] != want[f])[0]
        assert bad.size == 0, f"{f}: {bad.size} mismatches at {bad[:5]}: got {got[f][bad[:5]]} want {want[f][bad[:5]]}"


def _set_from(seqs):
    from synth.families import FamilySet

    lens = np.array([len(x) for x in seqs], np.int64)
    off = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    res = np.frombuffer(b"".join(seqs), np.uint8).copy() if seqs else np.zeros(0, np.uint8)
    return FamilySet(res, off, np.zeros(len(seqs), np.int32), {})


def _random_set(seed, n, lo, hi, letters):
    rng = np.random.default_rng(seed)
    alpha = np.frombuffer(letters.encode(), np.uint8)
    return _set_from([rng.choice(alpha, int(rng.integers(lo, hi + 1))).tobytes() for _ in range(n)])


def test_exact_tiny(gpu, orc):
    from synth import workload

    s = workload("tiny")
    want = orc.candidates(orc.encode(s.residues), s.offsets, 6, ck_min=1)
    _compare(_gpu_candidates(gpu, s.residues, s.offsets, k=6, ck_min=1), want)


@pytest.mark.parametrize("k,ck", [(3, 1), (3, 2), (4, 3), (2, 1)])
def test_exact_dense_sharing(gpu, orc, k, ck):
    """Few letters: long posting lists, many products per row."""
    s = _random_set(10 + k + ck, 120, 0, 90, "ACDE")
    want = orc.candidates(orc.encode(s.residues), s.offsets, k, ck_min=ck)
    _compare(_gpu_candidates(gpu, s.residues, s.offsets, k=k, ck_min=ck), want)


def test_exact_large_rows_use_global_tables(gpu, orc):
    """Rows with more than 12,288 products go through the global-memory path."""
    s = _random_set(77, 300, 100, 400, "AC")
    want = orc.candidates(orc.encode(s.residues), s.offsets, 3, ck_min=1)
    _compare(_gpu_candidates(gpu, s.residues, s.offsets, k=3, ck_min=1), want)


@pytest.mark.parametrize("ck", [1, 2])
def test_exact_rows_of_every_table_size(gpu, orc, ck):
    """Posting lists of ~1,600 entries: rows of 1 to 38 k-mers span the
    larger table sizes (4K to 32K LDS slots, global memory), and most rows
    have more candidates than their LDS table stages, so the global redo of
    those rows is exercised too."""
    s = _random_set(91 + ck, 5000, 3, 40, "ACDE")
    want = orc.candidates(orc.encode(s.residues), s.offsets, 3, ck_min=ck)
    _compare(_gpu_candidates(gpu, s.residues, s.offsets, k=3, ck_min=ck), want)


@pytest.mark.parametrize("ck", [1, 2])
def test_exact_rows_of_the_small_tables(gpu, orc, ck):
    """Posting lists of ~260 entries: rows of 1 to 18 k-mers fill the 2K, 4K
    and 8K-slot tables."""
    s = _random_set(57 + ck, 6000, 3, 20, "ACDEFG")
    want = orc.candidates(orc.encode(s.residues), s.offsets, 3, ck_min=ck)
    assert len(want["lo"]) > 10000
    _compare(_gpu_candidates(gpu, s.residues, s.offsets, k=3, ck_min=ck), want)


@pytest.mark.parametrize("case", ["exact", "substitutes", "global_rows"])
def test_redone_with_room_for_every_candidate(gpu, orc, case):
    """A candidate room far below the directional entries overflows in the
    LDS and global-table kernels; the discovery is redone with enough room
    and gives the same candidates."""
    from synth import workload

    if case == "exact":
        s, kw = workload("tiny"), dict(k=6, ck_min=1)
    elif case == "substitutes":
        s, kw = workload("tiny", n_families=6), dict(k=6, ck_min=2, n_subs=25)
    else:
        s, kw = _random_set(77, 300, 100, 400, "AC"), dict(k=3, ck_min=1)
    want = orc.candidates(orc.encode(s.residues), s.offsets, kw["k"], ck_min=kw["ck_min"],
                          n_subs=kw.get("n_subs", 0))
    assert len(want["lo"]) > 1000
    _compare(_gpu_candidates(gpu, s.residues, s.offsets, candidate_room=64, **kw), want)


def test_negative_candidate_room_is_rejected(gpu):
    import paper_2009_14467_amd as P

    with pytest.raises(P.PastisError):
        P.Context(P.Params(candidate_room=-1))


@pytest.mark.parametrize("k,m,ck,alpha", [(3, 5, 2, 20), (4, 10, 2, 20), (6, 25, 2, 20), (3, 8, 1, 24)])
def test_substitutes(gpu, orc, k, m, ck, alpha):
    from synth import workload

    if k == 6:
        s = workload("tiny", n_families=6)
    else:
        s = _random_set(5 + k + m, 80, 0, 60, "ACDEFGSTW")
    want = orc.candidates(orc.encode(s.residues), s.offsets, k, ck_min=ck, n_subs=m, alpha=alpha)
    got = _gpu_candidates(gpu, s.residues, s.offsets, k=k, ck_min=ck, n_subs=m, sub_alphabet=alpha)
    _compare(got, want)


def test_heavy_tail_discovery_k5_m25(gpu, orc):
    """The heavy-tail setting: k = 5 with 25 substitute k-mers, >= 2 shared,
    on the heavy recipe (40% divergence) scaled to 16 families, one of which
    descends from a 28k-residue ancestor, so A S rows of tens of thousands of
    entries and k = 5 postings shared by many sequences are both present."""
    from synth import workload

    s = workload("heavy", n_families=16)
    assert np.diff(s.offsets).max() > 20000
    want = orc.candidates(orc.encode(s.residues), s.offsets, 5, ck_min=2, n_subs=25)
    assert len(want["lo"]) > 20000
    got = _gpu_candidates(gpu, s.residues, s.offsets, k=5, ck_min=2, n_subs=25)
    _compare(got, want)


@pytest.mark.parametrize("k,m,ck", [(7, 0, 1), (8, 0, 1), (7, 10, 2), (8, 25, 2), (8, 25, 1)])
def test_long_kmers_without_dense_map(gpu, orc, k, m, ck):
    """k = 7 and 8: ids past 32 bits (24^8 > 2^36), no dense id map (the
    substitutes' compact indices come from a binary search of the sorted
    distinct ids); candidates, counts and seeds against the oracle."""
    from synth import workload

    s = workload("tiny", n_families=6)
    want = orc.candidates(orc.encode(s.residues), s.offsets, k, ck_min=ck, n_subs=m)
    assert len(want["lo"]) > 200
    _compare(_gpu_candidates(gpu, s.residues, s.offsets, k=k, ck_min=ck, n_subs=m), want)


@pytest.mark.parametrize("mode", ["sw", "xd"])
def test_search_k8(gpu, orc, mode):
    """The whole search at k = 8 (seeds of 8 columns in XD) against the oracle."""
    import paper_2009_14467_amd as P
    from synth import workload

    from test_gpu_search import _compare_edges

    s = workload("tiny", n_families=8)
    want = orc.search(s.residues, s.offsets, k=8, n_subs=10, ck_min=1, mode=mode)
    got = P.Context(P.Params(k=8, n_subs=10, ck_min=1, align_mode=mode)).search(_dev(s.residues, gpu),
                                                                             _dev(s.offsets, gpu))
    _compare_edges(got, want)


def test_k_out_of_range_is_rejected(gpu):
    import paper_2009_14467_amd as P

    for k in (0, 9):
        with pytest.raises(P.PastisError):
            P.Context(P.Params(k=k))


def test_substitutes_m0_equals_exact(gpu, orc):
    s = _random_set(3, 60, 0, 50, "ACDEF")
    a = _gpu_candidates(gpu, s.residues, s.offsets, k=3, ck_min=1, n_subs=0)
    want = orc.candidates(orc.encode(s.residues), s.offsets, 3, ck_min=1, method="brute")
    _compare(a, want)


@pytest.mark.parametrize("k,m,alpha", [(6, 25, 20), (5, 25, 20), (3, 40, 24), (2, 10, 20), (7, 25, 20), (8, 25, 20),
                                       (8, 10, 24)])
def test_subkmers_neighbourhoods(gpu, orc, k, m, alpha):
    import paper_2009_14467_amd as P

    rng = np.random.default_rng(k * 100 + m)
    ids = []
    for _ in range(64):
        c = rng.integers(0, 24 if alpha == 24 else 20, k)
        ids.append(sum(int(c[t]) * 24 ** (k - 1 - t) for t in range(k)))
    # a few k-mers with X (negative expenses) and the extremes
    ids += [orc.kmer_id("X" * k), orc.kmer_id("W" * k), orc.kmer_id("A" * (k - 1) + "C")]
    ctx = P.Context(P.Params(k=k, n_subs=m, sub_alphabet=alpha))
    gi, gd, gn = ctx.subkmers(_dev(np.array(ids, np.int64), gpu))
    gi, gd, gn = gi.cpu().numpy(), gd.cpu().numpy(), gn.cpu().numpy()
    for q, r in enumerate(ids):
        wi, wd = orc.subkmers(r, k, m, alpha)
        assert gn[q] == len(wi)
        got = sorted(zip(gd[q, : gn[q]].tolist(), gi[q, : gn[q]].tolist()))
        assert got == list(zip(wd.tolist(), wi.tolist())), orc.kmer_string(r, k)


def test_edge_cases(gpu, orc):
    seqs = [b"", b"AC", b"ACDEFG", b"ACDEFGH", b"", b"ACDEFG", b"W"]
    s = _set_from(seqs)
    want = orc.candidates(orc.encode(s.residues), s.offsets, 6, ck_min=1)
    _compare(_gpu_candidates(gpu, s.residues, s.offsets, k=6, ck_min=1), want)
    one = _set_from([b"ACDEFGHIK"])
    got = _gpu_candidates(gpu, one.residues, one.offsets, k=6, ck_min=1)
    assert all(v.size == 0 for v in got.values())
    empty = _set_from([])
    got = _gpu_candidates(gpu, empty.residues, empty.offsets, k=6, ck_min=1)
    assert all(v.size == 0 for v in got.values())
