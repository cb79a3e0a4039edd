"""Parity of the HIP Smith-Waterman path with the CPU oracle (Section IV-E).

Every record field is compared element by element; all of it is integer work,
so the bar is bit-exact.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("score", "beg_a", "end_a", "beg_b", "end_b", "matches", "columns", "seed_used", "passed", "swapped", "cells")


def _to_dev(x, dev, dtype=None):
    import torch

    a = np.ascontiguousarray(x)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(dev)


def _gpu_records(dev, s, lo, hi, s1=None, s2=None, tuning=None, **params):
    import paper_2009_14467_amd as P

    ctx = P.Context(P.Params(**params))
    if tuning:
        ctx.set_tuning(**tuning)
    out = ctx.align_pairs(
        _to_dev(s.residues, dev), _to_dev(s.offsets, dev), _to_dev(lo, dev), _to_dev(hi, dev),
        None if s1 is None else _to_dev(s1, dev), None if s2 is None else _to_dev(s2, dev),
    )
    return P.records_to_numpy(out)


def _compare(got, want, fields=FIELDS, mask=None):
    assert got.shape == want.shape
    for f in fields:
        g, w = got[f], want[f]
        if mask is not None:
            g, w = g[mask], w[mask]
        bad = np.nonzero(g != w)[0]
        assert bad.size == 0, f"{f}: {bad.size} mismatches, first at {bad[:5]}: got {g[bad[:5]]} want {w[bad[:5]]}"


@pytest.fixture(scope="module")
def tiny(orc):
    from synth import workload

    s = workload("tiny")
    codes = orc.encode(s.residues)
    cand = orc.candidates(codes, s.offsets, 6, ck_min=1)
    want = orc.align_pairs(codes, s.offsets, cand["lo"], cand["hi"], mode="sw")
    return s, cand, want


def test_sw_full_records_tiny(gpu, tiny):
    s, cand, want = tiny
    got = _gpu_records(gpu, s, cand["lo"], cand["hi"], full_records=True)
    _compare(got, want)


def test_sw_fast_records_tiny(gpu, tiny):
    s, cand, want = tiny
    got = _gpu_records(gpu, s, cand["lo"], cand["hi"], full_records=False)
    _compare(got, want, ("score", "end_a", "end_b", "passed", "swapped", "cells"))
    _compare(got, want, FIELDS, mask=want["passed"] == 1)


def test_sw_reversed_pair_order(gpu, tiny):
    """(j, i) gives the same alignment as (i, j): orientation is by length."""
    s, cand, want = tiny
    got = _gpu_records(gpu, s, cand["hi"], cand["lo"], full_records=True)
    w2 = want.copy()
    # same rows/columns unless the lengths tie, where the first of the pair is a
    L = np.diff(s.offsets)
    tie = L[cand["lo"]] == L[cand["hi"]]
    _compare(got[~tie], w2[~tie], tuple(f for f in FIELDS if f != "swapped"))
    assert (got["swapped"][~tie] == 1 - w2["swapped"][~tie]).all()


def test_sw_multi_strip_long_pairs(gpu, orc):
    """Rows beyond 512 cross strips through the global boundary buffer."""
    from synth import make_family_set

    s = make_family_set(n_families=4, family_size=4, mean_len=900, min_len=500, max_len=1800, divergence=0.3,
                        stream=91)
    codes = orc.encode(s.residues)
    n = s.n
    lo, hi = np.triu_indices(n, 1)
    lo = lo.astype(np.uint32)
    hi = hi.astype(np.uint32)
    want = orc.align_pairs(codes, s.offsets, lo, hi, mode="sw")
    got = _gpu_records(gpu, s, lo, hi, full_records=True)
    assert (want["end_a"] >= 512).any()
    _compare(got, want)


def test_sw_edge_cases(gpu, orc):
    from synth.families import FamilySet

    seqs = [b"", b"W", b"WW", b"A", b"WWWWWWWWWW", b"WWWWWGWWWWW", b"PPP", b"X*BZ", b"A" * 700, b"A" * 700 + b"W"]
    lens = np.array([len(x) for x in seqs])
    off = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    s = FamilySet(np.frombuffer(b"".join(seqs), np.uint8).copy(), off, np.zeros(len(seqs), np.int32), {})
    codes = orc.encode(s.residues)
    lo, hi = np.triu_indices(len(seqs), 1)
    lo = lo.astype(np.uint32)
    hi = hi.astype(np.uint32)
    want = orc.align_pairs(codes, s.offsets, lo, hi, mode="sw")
    got = _gpu_records(gpu, s, lo, hi, full_records=True)
    _compare(got, want)


def test_sw_rejects_bad_input(gpu):
    import paper_2009_14467_amd as P
    from synth.families import FamilySet

    res = np.frombuffer(b"ACDEFJKL", np.uint8).copy()
    off = np.array([0, 4, 8], np.int64)
    s = FamilySet(res, off, np.zeros(2, np.int32), {})
    with pytest.raises(P.PastisError, match="BAD_RESIDUE"):
        _gpu_records(gpu, s, np.array([0], np.uint32), np.array([1], np.uint32))
    s = FamilySet(np.frombuffer(b"ACDEFGKL", np.uint8).copy(), off, np.zeros(2, np.int32), {})
    with pytest.raises(P.PastisError, match="INVAL"):
        _gpu_records(gpu, s, np.array([0], np.uint32), np.array([2], np.uint32))
    with pytest.raises(P.PastisError, match="INVAL"):
        _gpu_records(gpu, s, np.array([1], np.uint32), np.array([1], np.uint32))


def test_sw_every_length_bin(gpu, orc):
    """One pair per side of every bin boundary (64 R rows in one strip; 2, 3
    and 4 strips of 64 R rows, R = 5..8), against the oracle."""
    from synth.families import FamilySet

    rng = np.random.default_rng(5)
    lens = [1, 64, 65, 128, 129, 448, 449, 512, 513, 640, 641, 768, 769, 896, 897, 1024, 1025, 1152, 1153, 1344,
            1345, 1536, 1537, 1792, 2048, 2049, 2500]
    seqs = []
    for L in lens:
        a = rng.integers(0, 20, L)
        b = a.copy()
        sub = rng.random(L) < 0.25
        b[sub] = rng.integers(0, 20, int(sub.sum()))
        b = np.concatenate([rng.integers(0, 20, 7), b, rng.integers(0, 20, 11)])
        seqs += [a, b]
    letters = np.frombuffer(b"ARNDCQEGHILKMFPSTWYV", np.uint8)
    res = np.concatenate([letters[x] for x in seqs]).astype(np.uint8)
    off = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum([len(x) for x in seqs], out=off[1:])
    s = FamilySet(res, off, np.zeros(len(seqs), np.int32), {})
    codes = orc.encode(s.residues)
    lo = np.arange(0, len(seqs), 2, dtype=np.uint32)
    hi = lo + 1
    want = orc.align_pairs(codes, s.offsets, lo, hi, mode="sw")
    for full in (True, False):
        got = _gpu_records(gpu, s, lo, hi, full_records=full)
        if full:
            _compare(got, want)
        else:
            _compare(got, want, ("score", "end_a", "end_b", "passed", "swapped", "cells"))


def _check16(got, want):
    """16-bit pass 1: score, end row and the cut are exact for every pair; the
    end column and statistics exist where the statistics pass ran, and every
    pair without them fails the cut."""
    _compare(got, want, ("score", "end_a", "passed", "swapped", "cells"))
    have = got["beg_a"] >= 0
    assert (want["passed"][~have] == 0).all()
    _compare(got, want, ("beg_a", "beg_b", "matches", "columns"), mask=have)
    _compare(got, want, ("end_b",), mask=got["end_b"] != -1)
    assert (got["end_b"][have] >= 0).all()
    return have


def test_sw16_records_tiny(gpu, tiny):
    s, cand, want = tiny
    got = _gpu_records(gpu, s, cand["lo"], cand["hi"], score_width=16)
    have = _check16(got, want)
    assert have.sum() >= (want["passed"] == 1).sum() > 0


@pytest.mark.parametrize("narrow", [0, 4])
def test_sw16_every_one_strip_bin_and_odd_counts(gpu, orc, narrow):
    """Rows 1..1024 (one-strip bins R = 1..16) with odd pair counts per bin,
    so the last wave of a bin carries one pair, and several pairs sharing
    their shorter sequence (the 16-bit pass pairs those in one wave).  Bins
    of up to 8 rows per lane run in two rows classes (up to 64 R - 32 rows,
    and more): both sides of every class boundary are here, in strips of 32
    lanes (narrow 0) and, up to 4 rows per lane, of 16 (narrow 4)."""
    from synth.families import FamilySet

    rng = np.random.default_rng(8)
    lens = [1, 2, 63, 64, 65, 100, 128, 129, 191, 192, 193, 255, 256, 257, 320, 321, 383, 384, 385, 448, 449, 511,
            512, 513, 640, 641, 768, 769, 896, 897, 1023, 1024]
    lens += [64 * R - 32 + d for R in range(1, 9) for d in (0, 1)]
    seqs = []
    for L in lens:
        a = rng.integers(0, 20, L)
        b = a.copy()
        sub = rng.random(L) < 0.3
        b[sub] = rng.integers(0, 20, int(sub.sum()))
        b = np.concatenate([rng.integers(0, 20, int(rng.integers(0, 40))), b, rng.integers(0, 20, 5)])
        seqs += [a, b]
    letters = np.frombuffer(b"ARNDCQEGHILKMFPSTWYV", np.uint8)
    res = np.concatenate([letters[x] for x in seqs]).astype(np.uint8)
    off = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum([len(x) for x in seqs], out=off[1:])
    s = FamilySet(res, off, np.zeros(len(seqs), np.int32), {})
    codes = orc.encode(s.residues)
    lo = np.arange(0, len(seqs), 2, dtype=np.uint32)
    hi = lo + 1
    # plus every cross pair among the first 16 sequences: many pairs per bin
    a, b = np.triu_indices(16, 1)
    lo = np.concatenate([lo, a.astype(np.uint32)])
    hi = np.concatenate([hi, b.astype(np.uint32)])
    want = orc.align_pairs(codes, s.offsets, lo, hi, mode="sw")
    tuning = dict(sw16_max_rows=16, sw16_narrow_rows=narrow)
    got = _gpu_records(gpu, s, lo, hi, tuning=tuning, score_width=16)
    _check16(got, want)


def test_sw16_multi_strip_bins(gpu, orc):
    """Rows 1025..2978 run in 16-bit lanes over strips of 64 R rows (R = 9..16)
    with the boundary row passed through a per-wave buffer; 2979 rows and more
    stay in 32 bits.  Identical runs of W (11 per row) put the score at the
    16-bit limit: 11 * 2978 = 32758 in 16 bits, 32769 in 32."""
    from synth.families import FamilySet

    rng = np.random.default_rng(9)
    lens = [1025, 1100, 1152, 1153, 1344, 1345, 1536, 1537, 1792, 2048, 2049, 2500, 2977, 2978, 2979, 3100]
    seqs = []
    for L in lens:
        a = rng.integers(0, 20, L)
        b = a.copy()
        sub = rng.random(L) < 0.3
        b[sub] = rng.integers(0, 20, int(sub.sum()))
        b = np.concatenate([rng.integers(0, 20, int(rng.integers(0, 40))), b, rng.integers(0, 20, 5)])
        seqs += [a, b]
    w = np.full(2978, 17)  # W
    seqs += [w, w.copy(), np.full(2979, 17), np.full(2979, 17)]
    letters = np.frombuffer(b"ARNDCQEGHILKMFPSTWYV", np.uint8)
    res = np.concatenate([letters[x] for x in seqs]).astype(np.uint8)
    off = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum([len(x) for x in seqs], out=off[1:])
    s = FamilySet(res, off, np.zeros(len(seqs), np.int32), {})
    codes = orc.encode(s.residues)
    lo = np.arange(0, len(seqs), 2, dtype=np.uint32)
    hi = lo + 1
    # several pairs sharing their shorter sequence (1025 rows), one wave apart
    a = np.zeros(9, np.uint32)
    lo = np.concatenate([lo, a])
    hi = np.concatenate([hi, np.arange(3, 30, 3, dtype=np.uint32)])
    want = orc.align_pairs(codes, s.offsets, lo, hi, mode="sw")
    assert want["score"][len(lens)] == 11 * 2978 and want["score"][len(lens) + 1] == 11 * 2979
    got = _gpu_records(gpu, s, lo, hi, score_width=16)
    _check16(got, want)
    _compare(_gpu_records(gpu, s, lo, hi, full_records=True, score_width=16), want)


def test_intra_pair_mode(gpu, orc):
    """One workgroup per pair (strips pipelined across four waves) for
    sequences a over 2,978 rows, and for every multi-strip pair once 16-bit
    lanes are off: 1 to 20 strips, pairs sharing sequences, against the oracle."""
    from synth.families import FamilySet

    rng = np.random.default_rng(13)
    lens = [1100, 2500, 2979, 3100, 4100, 5000, 9000, 20000]
    seqs = []
    for L in lens:
        a = rng.integers(0, 20, L)
        b = a.copy()
        sub = rng.random(L) < 0.25
        b[sub] = rng.integers(0, 20, int(sub.sum()))
        b = np.concatenate([rng.integers(0, 20, int(rng.integers(0, 60))), b, rng.integers(0, 20, 9)])
        seqs += [a, b]
    letters = np.frombuffer(b"ARNDCQEGHILKMFPSTWYV", np.uint8)
    res = np.concatenate([letters[x] for x in seqs]).astype(np.uint8)
    off = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum([len(x) for x in seqs], out=off[1:])
    s = FamilySet(res, off, np.zeros(len(seqs), np.int32), {})
    codes = orc.encode(s.residues)
    lo = np.arange(0, len(seqs), 2, dtype=np.uint32)
    hi = lo + 1
    # unrelated pairs and pairs sharing their shorter sequence
    lo = np.concatenate([lo, np.array([4, 4, 6, 8, 10], np.uint32)])
    hi = np.concatenate([hi, np.array([9, 13, 11, 15, 13], np.uint32)])
    want = orc.align_pairs(codes, s.offsets, lo, hi, mode="sw")
    intra = dict(sw_intra_pair=1)
    _compare(_gpu_records(gpu, s, lo, hi, tuning=intra, full_records=True), want)
    _compare(_gpu_records(gpu, s, lo, hi, tuning=intra), want, ("score", "end_a", "end_b", "passed", "swapped", "cells"))
    _check16(_gpu_records(gpu, s, lo, hi, tuning=intra, score_width=16), want)


def test_search_same_edges_in_16_and_32_bits(gpu):
    import paper_2009_14467_amd as P
    from synth import workload

    s = workload("tiny", n_families=15)
    res, off = _to_dev(s.residues, gpu), _to_dev(s.offsets, gpu)
    e16 = P.Context(P.Params(k=6, ck_min=1, score_width=16)).search(res, off)
    e32 = P.Context(P.Params(k=6, ck_min=1, score_width=32)).search(res, off)
    assert e16.size == e32.size > 0
    assert e16.tobytes() == e32.tobytes()


def test_longest_pairs_sw_and_xd(gpu, orc):
    """Pairs of 20,000-30,000 residues (the heavy tail's range): many strips
    of 1024 rows, scores far beyond 16 bits, the start bound skipped for
    rectangles taller than its packing allows; SW and XD against the oracle."""
    from synth.families import FamilySet

    rng = np.random.default_rng(12)
    anc = rng.integers(0, 20, 30000)
    a = anc.copy()
    sub = rng.random(a.size) < 0.2
    a[sub] = rng.integers(0, 20, int(sub.sum()))
    b = np.concatenate([anc[:12000], rng.integers(0, 20, 40), anc[12000:29000]])
    c = rng.integers(0, 20, 20000)
    seqs = [a, b, c]
    letters = np.frombuffer(b"ARNDCQEGHILKMFPSTWYV", np.uint8)
    res = np.concatenate([letters[x] for x in seqs]).astype(np.uint8)
    off = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum([len(x) for x in seqs], out=off[1:])
    s = FamilySet(res, off, np.zeros(len(seqs), np.int32), {})
    codes = orc.encode(s.residues)
    lo = np.array([0, 0, 1], np.uint32)
    hi = np.array([1, 2, 2], np.uint32)
    want = orc.align_pairs(codes, s.offsets, lo, hi, mode="sw")
    assert want["score"][0] > 1 << 16 and want["passed"][0] == 1
    _compare(_gpu_records(gpu, s, lo, hi, full_records=True), want)
    _compare(_gpu_records(gpu, s, lo, hi), want, ("score", "end_a", "end_b", "passed", "swapped", "cells"))
    p = orc.pair_counts(codes, s.offsets, lo, hi, 6)
    wx = orc.align_pairs(codes, s.offsets, lo, hi, p["seed1"], p["seed2"], mode="xd", k=6)
    gx = _gpu_records(gpu, s, lo, hi, p["seed1"], p["seed2"], align_mode="xd", full_records=True)
    _compare(gx, wx)


def test_rejects_sequences_beyond_u16_positions(gpu):
    import paper_2009_14467_amd as P
    from synth.families import FamilySet

    res = np.full(65536 + 10, ord("A"), np.uint8)
    off = np.array([0, 65536, 65546], np.int64)
    s = FamilySet(res, off, np.zeros(2, np.int32), {})
    with pytest.raises(P.PastisError):
        _gpu_records(gpu, s, np.array([0], np.uint32), np.array([1], np.uint32))
    ctx = P.Context(P.Params())
    with pytest.raises(P.PastisError):
        ctx.search(_to_dev(s.residues, gpu), _to_dev(s.offsets, gpu))


@pytest.mark.parametrize("go,ge", [(5, 2), (250, 10), (2, 1), (240, 4)])
def test_sw_other_gap_costs(gpu, orc, tiny, go, ge):
    """Gap costs away from 11/1: the 16-bit profile holds s + o + e in a byte,
    so o + e above 244 (and below 4) must run in 32-bit lanes; every width and
    record mode still matches the oracle, and so do the search's edges."""
    import paper_2009_14467_amd as P

    s, cand, _ = tiny
    codes = orc.encode(s.residues)
    want = orc.align_pairs(codes, s.offsets, cand["lo"], cand["hi"], mode="sw", gap_open=go, gap_extend=ge)
    gaps = dict(gap_open=go, gap_extend=ge)
    _compare(_gpu_records(gpu, s, cand["lo"], cand["hi"], full_records=True, **gaps), want)
    for width in (0, 16, 32):
        _check16(_gpu_records(gpu, s, cand["lo"], cand["hi"], score_width=width, **gaps), want)
    res, off = _to_dev(s.residues, gpu), _to_dev(s.offsets, gpu)
    want_e = orc.search(s.residues, s.offsets, k=6, ck_min=1, mode="sw", **gaps)
    for width in (0, 16):
        got_e = P.Context(P.Params(k=6, ck_min=1, score_width=width, **gaps)).search(res, off)
        assert got_e.size == want_e.size and got_e.tobytes() == want_e.tobytes()
