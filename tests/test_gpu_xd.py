"""Parity of the HIP x-drop seed extension (Section IV-E, XD) with the CPU
oracle: every record field, the evaluated-cell count included, bit for bit."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("score", "beg_a", "end_a", "beg_b", "end_b", "matches", "columns", "seed_used", "passed", "swapped", "cells")


def _dev(x, gpu):
    import torch

    a = np.ascontiguousarray(x)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(gpu)


def _gpu_xd(gpu, s, lo, hi, s1, s2, **params):
    import paper_2009_14467_amd as P

    ctx = P.Context(P.Params(align_mode="xd", **params))
    out = ctx.align_pairs(_dev(s.residues, gpu), _dev(s.offsets, gpu), _dev(lo, gpu), _dev(hi, gpu), _dev(s1, gpu),
                          _dev(s2, gpu))
    return P.records_to_numpy(out)


def _compare(got, want):
    for f in FIELDS:
        bad = np.nonzero(got[f] != want[f])[0]
        assert bad.size == 0, f"{f}: {bad.size} mismatches at {bad[:5]}: got {got[f][bad[:5]]} want {want[f][bad[:5]]}"


@pytest.mark.parametrize("n_subs,ck", [(0, 1), (25, 2)])
def test_xd_candidates(gpu, orc, n_subs, ck):
    from synth import workload

    s = workload("tiny", n_families=10 if n_subs else 25)
    codes = orc.encode(s.residues)
    c = orc.candidates(codes, s.offsets, 6, ck_min=ck, n_subs=n_subs)
    want = orc.align_pairs(codes, s.offsets, c["lo"], c["hi"], c["seed1"], c["seed2"], mode="xd", k=6)
    got = _gpu_xd(gpu, s, c["lo"], c["hi"], c["seed1"], c["seed2"], k=6)
    assert (want["seed_used"] >= 0).all()
    _compare(got, want)


def test_xd_unbounded_drop_uses_wide_bands(gpu, orc):
    """X = 1e6 never prunes: bands grow past the 256-cell LDS ring."""
    from synth import make_family_set

    s = make_family_set(n_families=3, family_size=4, mean_len=500, min_len=300, max_len=700, divergence=0.3,
                        stream=33)
    codes = orc.encode(s.residues)
    c = orc.candidates(codes, s.offsets, 4, ck_min=1)
    want = orc.align_pairs(codes, s.offsets, c["lo"], c["hi"], c["seed1"], c["seed2"], mode="xd", k=4, xdrop=10**6)
    got = _gpu_xd(gpu, s, c["lo"], c["hi"], c["seed1"], c["seed2"], k=4, xdrop=10**6)
    _compare(got, want)


def test_xd_seed_positions_and_missing_seeds(gpu, orc):
    from synth.families import FamilySet

    seqs = [b"ACDEFGHIKLMNPQRSTVWY", b"ACDEFGHIKLMNPQRSTVWY", b"WWACDEFG", b"ACDEFG", b"PPPP", b"PPPPPPPP"]
    lens = np.array([len(x) for x in seqs])
    off = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    s = FamilySet(np.frombuffer(b"".join(seqs), np.uint8).copy(), off, np.zeros(len(seqs), np.int32), {})
    codes = orc.encode(s.residues)
    NO = 0xFFFFFFFF
    # (lo, hi, seed1, seed2): seeds at the first / last k-mer, one or no seed,
    # and an out-of-range seed (ignored by both sides)
    rows = [
        (0, 1, (0 << 16) | 0, (14 << 16) | 14),
        (0, 1, (14 << 16) | 14, NO),
        (2, 3, (2 << 16) | 0, NO),
        (2, 3, NO, NO),
        (4, 5, (0 << 16) | 4, (0 << 16) | 0),
        (0, 1, (60 << 16) | 0, (3 << 16) | 3),
    ]
    lo = np.array([r[0] for r in rows], np.uint32)
    hi = np.array([r[1] for r in rows], np.uint32)
    s1 = np.array([r[2] for r in rows], np.uint32)
    s2 = np.array([r[3] for r in rows], np.uint32)
    want = orc.align_pairs(codes, s.offsets, lo, hi, s1, s2, mode="xd", k=6)
    got = _gpu_xd(gpu, s, lo, hi, s1, s2, k=6)
    _compare(got, want)


@pytest.mark.parametrize("weight", ["ani", "ns"])
def test_search_xd_tiny(gpu, orc, weight):
    """XD search edges against the oracle, with the identity weight and cut,
    and with the normalised score (no cut, no traceback fields)."""
    import paper_2009_14467_amd as P
    from synth import workload

    from test_gpu_search import _compare_edges

    s = workload("tiny")
    want = orc.search(s.residues, s.offsets, k=6, ck_min=1, mode="xd", weight=weight)
    ctx = P.Context(P.Params(k=6, ck_min=1, align_mode="xd", weight_mode=weight))
    got = ctx.search(_dev(s.residues, gpu), _dev(s.offsets, gpu))
    _compare_edges(got, want)
