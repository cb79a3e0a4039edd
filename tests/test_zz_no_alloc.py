"""The no-allocation variant of the pair alignment entry point, called
through the C ABI: the same records as pastis_align_pairs on two calls in a
row (the second on a smaller input, over the workspace the first one left),
and its limits (Smith-Waterman only, inputs that fit the static workspace)."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NOALLOC_BYTES = 48 << 20


def _dev(x, gpu):
    import torch

    a = np.ascontiguousarray(x)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(gpu)


def _noalloc(P, ctx, res, off, pi, pj, s1, s2, out):
    import torch

    ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
    return P.lib().pastis_align_pairs_noalloc(ctx._ctx, ptr(res), ptr(off), off.numel() - 1, ptr(pi), ptr(pj),
                                              ptr(s1), ptr(s2), pi.numel(), ptr(out),
                                              torch.cuda.current_stream().cuda_stream)


def _subset(s, keep):
    from synth.families import FamilySet

    L = np.diff(s.offsets)
    parts = [s.residues[s.offsets[i]:s.offsets[i + 1]] for i in keep]
    off = np.zeros(len(keep) + 1, np.int64)
    np.cumsum(L[keep], out=off[1:])
    return FamilySet(np.concatenate(parts).astype(np.uint8), off, s.labels[keep], {})


@pytest.mark.parametrize("params", [dict(), dict(full_records=True), dict(score_width=16)])
def test_noalloc_matches_align_pairs_on_two_calls(gpu, orc, params):
    import torch

    import paper_2009_14467_amd as P
    from synth import workload

    s = workload("tiny")
    assert np.diff(s.offsets).max() <= 1024
    codes = orc.encode(s.residues)
    cand = orc.candidates(codes, s.offsets, 6, ck_min=1)
    small = _subset(s, np.arange(0, s.n, 3))
    cs = orc.candidates(orc.encode(small.residues), small.offsets, 6, ck_min=1)
    ctx = P.Context(P.Params(k=6, ck_min=1, **params))
    for fs, c in ((s, cand), (small, cs)):  # the second call is smaller
        res, off = _dev(fs.residues, gpu), _dev(fs.offsets, gpu)
        pi, pj = _dev(c["lo"], gpu), _dev(c["hi"], gpu)
        s1, s2 = _dev(c["seed1"], gpu), _dev(c["seed2"], gpu)
        want = ctx.align_pairs(res, off, pi, pj, s1, s2)
        out = torch.full((pi.numel() * 48,), 0xAB, dtype=torch.uint8, device=gpu)
        st = _noalloc(P, ctx, res, off, pi, pj, s1, s2, out)
        assert st == 0, P.lib().pastis_last_error(ctx._ctx)
        torch.cuda.synchronize()
        got, ref = P.records_to_numpy(out), P.records_to_numpy(want)
        assert got.tobytes() == ref.tobytes()
        # and the oracle agrees on every field the record mode fills
        orc_rec = orc.align_pairs(orc.encode(fs.residues), fs.offsets, c["lo"], c["hi"], mode="sw")
        for f in ("score", "end_a", "passed", "swapped", "cells"):
            assert (got[f] == orc_rec[f]).all(), f
        assert ctx.stats()["n_aligned"] == pi.numel()


def test_noalloc_limits(gpu):
    import torch

    import paper_2009_14467_amd as P
    from synth.families import FamilySet

    rng = np.random.default_rng(3)
    letters = np.frombuffer(b"ARNDCQEGHILKMFPSTWYV", np.uint8)
    seqs = [letters[rng.integers(0, 20, L)] for L in (300, 320, 1500, 1600)]
    off = np.zeros(5, np.int64)
    np.cumsum([x.size for x in seqs], out=off[1:])
    s = FamilySet(np.concatenate(seqs), off, np.zeros(4, np.int32), {})
    res, offd = _dev(s.residues, gpu), _dev(s.offsets, gpu)
    pi, pj = _dev(np.array([0, 2], np.uint32), gpu), _dev(np.array([1, 3], np.uint32), gpu)
    out = torch.full((2 * 48,), 0xAB, dtype=torch.uint8, device=gpu)
    ctx = P.Context(P.Params(k=6))
    # a 1,500-residue sequence needs boundary rows beyond the workspace
    assert _noalloc(P, ctx, res, offd, pi, pj, None, None, out) == 5  # PASTIS_E_CAPACITY
    assert b"no-allocation workspace" in P.lib().pastis_last_error(ctx._ctx)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 0xAB).all()  # nothing written
    # the short pair alone fits; x-drop is refused
    p1, q1 = pi[:1].contiguous(), pj[:1].contiguous()
    short = FamilySet(np.concatenate(seqs[:2]), off[:3].copy(), np.zeros(2, np.int32), {})
    r2, o2 = _dev(short.residues, gpu), _dev(short.offsets, gpu)
    assert _noalloc(P, ctx, r2, o2, p1, q1, None, None, out) == 0
    want = ctx.align_pairs(r2, o2, p1, q1)
    torch.cuda.synchronize()
    assert out[:48].cpu().numpy().tobytes() == want.cpu().numpy().tobytes()
    xd = P.Context(P.Params(k=6, align_mode="xd"))
    assert _noalloc(P, xd, r2, o2, p1, q1, None, None, out) == 1  # PASTIS_E_INVAL
