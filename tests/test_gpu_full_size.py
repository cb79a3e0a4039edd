"""Parity at the benchmark's full sizes, in the launch configurations
bench.py times (one pastis_search):
  * large: 250,000 sequences (10,000 families x 20 + 50,000 singletons,
    lengths up to 5,000), exact 6-mers, >= 2 shared; schedule chosen by the
    autotuner and the SW stage replayed as a captured HIP graph;
  * mid: 50,000 sequences (2,000 families x 25), 25 substitute 6-mers,
    >= 2 shared; the library's schedule, direct launches.
Both are searched with SW and with XD.

The oracle cannot redo a whole search in test time, so it computes sampled
pairs one by one: every same-family pair of 24 random families, and 3,000
random pairs.  The sample is drawn from the generator's labels and a seeded
RNG, never from the GPU's output.  Properties that hold at any size are
checked on the whole output."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PARAMS = {"mid": dict(k=6, n_subs=25, ck_min=2), "large": dict(k=6, n_subs=0, ck_min=2)}


def _dev(x, gpu):
    import torch

    a = np.ascontiguousarray(x)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(gpu)


def _key(lo, hi):
    return (np.asarray(lo, np.uint64) << np.uint64(32)) | np.asarray(hi, np.uint64)


@pytest.fixture(scope="module", params=["mid", "large"])
def mid(request, gpu, orc):
    import paper_2009_14467_amd as P
    from synth import workload

    name = request.param
    prm = PARAMS[name]
    s = workload(name)
    res, off = _dev(s.residues, gpu), _dev(s.offsets, gpu)
    if name == "large":
        ctx = P.Context(P.Params(graph_mode=True, **prm))
        ctx.autotune(res, off, max_pairs=400_000)
    else:
        ctx = P.Context(P.Params(**prm))
    edges = ctx.search(res, off)
    if name == "large":
        assert ctx.search(res, off).tobytes() == edges.tobytes()  # a replay of the captured graph
        assert ctx.stats()["sw_graph"] > 0
    st = ctx.stats()
    nc = int(st["n_candidates"])
    xd_edges = P.Context(P.Params(align_mode="xd", **prm)).search(res, off)
    c = {k: v.cpu().numpy().view(np.uint32) for k, v in ctx.candidates(nc).items()}
    codes = orc.encode(s.residues)
    # the sample: all pairs inside 24 random families, and random pairs
    rng = np.random.default_rng(2024)
    fams = rng.choice(np.unique(s.labels[s.labels >= 0]), 24, replace=False)
    lo, hi = [], []
    for f in fams:
        members = np.nonzero(s.labels == f)[0]
        a, b = np.triu_indices(members.size, 1)
        lo.append(members[a])
        hi.append(members[b])
    x = rng.integers(0, s.n, 3300)
    y = rng.integers(0, s.n, 3300)
    ok = x != y
    lo.append(np.minimum(x, y)[ok][:3000])
    hi.append(np.maximum(x, y)[ok][:3000])
    lo = np.concatenate(lo).astype(np.uint32)
    hi = np.concatenate(hi).astype(np.uint32)
    k = np.unique(_key(lo, hi))
    lo, hi = (k >> np.uint64(32)).astype(np.uint32), (k & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    want = orc.pair_counts(codes, s.offsets, lo, hi, prm["k"], n_subs=prm["n_subs"])
    return dict(s=s, res=res, off=off, edges=edges, xd_edges=xd_edges, stats=st, cand=c, codes=codes, lo=lo, hi=hi,
                want=want, prm=prm, name=name)


def test_candidates_on_sampled_pairs(mid):
    c, want = mid["cand"], mid["want"]
    keys = _key(c["lo"], c["hi"])
    order = np.argsort(keys)
    skeys = keys[order]
    q = _key(mid["lo"], mid["hi"])
    at = np.minimum(np.searchsorted(skeys, q), skeys.size - 1)
    found = skeys[at] == q
    expect = want["count"] >= mid["prm"]["ck_min"]
    assert expect.sum() > 2000  # family pairs and chance candidates are both present
    np.testing.assert_array_equal(found, expect)
    g = order[at[found]]
    for f in ("count", "seed1", "seed2"):
        np.testing.assert_array_equal(c[f][g], want[f][expect], err_msg=f)


def test_candidate_set_properties(mid):
    c, s = mid["cand"], mid["s"]
    L = np.diff(s.offsets)
    assert (c["lo"] < c["hi"]).all() and (c["hi"] < s.n).all()
    keys = _key(c["lo"], c["hi"])
    assert np.unique(keys).size == keys.size
    prm = mid["prm"]
    assert (c["count"] >= prm["ck_min"]).all()
    # two shared k-mers give two distinct seed keys, inside both sequences
    assert (c["seed1"] < c["seed2"]).all() and (c["seed2"] != 0xFFFFFFFF).all()
    for f in ("seed1", "seed2"):
        p_lo, p_hi = c[f] >> 16, c[f] & 0xFFFF
        assert (p_lo <= L[c["lo"]] - prm["k"]).all() and (p_hi <= L[c["hi"]] - prm["k"]).all()


@pytest.mark.parametrize("mode", ["sw", "xd"])
def test_edges_on_sampled_pairs(mid, orc, mode):
    from test_gpu_search import _compare_edges

    s, want, prm = mid["s"], mid["want"], mid["prm"]
    cand = want["count"] >= prm["ck_min"]
    lo, hi = mid["lo"][cand], mid["hi"][cand]
    rec = orc.align_pairs(mid["codes"], s.offsets, lo, hi, want["seed1"][cand], want["seed2"][cand], mode=mode,
                          k=prm["k"])
    oe = orc.records_to_edges(lo, hi, want["count"][cand], rec, np.diff(s.offsets))
    e = mid["edges"] if mode == "sw" else mid["xd_edges"]
    sel = np.isin(_key(e["i"], e["j"]), _key(mid["lo"], mid["hi"]))
    assert oe.size > 1000
    _compare_edges(e[sel], oe)


def test_edge_set_properties(mid):
    e, c, s = mid["edges"], mid["cand"], mid["s"]
    L = np.diff(s.offsets)
    keys = _key(e["i"], e["j"])
    assert (keys[1:] > keys[:-1]).all()  # sorted, unique
    assert mid["stats"]["n_edges"] == e.size
    ck = _key(c["lo"], c["hi"])
    order = np.argsort(ck)
    at = np.searchsorted(ck[order], keys)
    assert (ck[order][at] == keys).all()  # every edge is a candidate
    assert (e["shared_kmers"] == np.minimum(c["count"][order][at], 65535)).all()
    assert (100 * e["matches"].astype(np.int64) >= 30 * e["columns"].astype(np.int64)).all()
    short_is_i = (L[e["i"]] < L[e["j"]]) | ((L[e["i"]] == L[e["j"]]) & (e["i"] < e["j"]))
    span = np.where(short_is_i, e["end_i"].astype(np.int64) - e["beg_i"] + 1,
                    e["end_j"].astype(np.int64) - e["beg_j"] + 1)
    assert (100 * span >= 70 * np.minimum(L[e["i"]], L[e["j"]])).all()
    ident = e["matches"].astype(np.float32) / e["columns"].astype(np.float32)
    np.testing.assert_array_equal(e["identity"].view(np.uint32), ident.view(np.uint32))


@pytest.mark.parametrize("mode", ["sw", "xd"])
def test_align_pairs_sample(gpu, mid, orc, mode):
    """2,000 sampled pairs aligned through pastis_align_pairs with full
    records, every field against the oracle."""
    import paper_2009_14467_amd as P

    from test_gpu_xd import FIELDS, _compare

    s, want = mid["s"], mid["want"]
    rng = np.random.default_rng(7)
    pick = np.sort(rng.choice(mid["lo"].size, 2000, replace=False))
    lo, hi = mid["lo"][pick], mid["hi"][pick]
    s1, s2 = want["seed1"][pick], want["seed2"][pick]
    ref = orc.align_pairs(mid["codes"], s.offsets, lo, hi, s1, s2, mode=mode, k=mid["prm"]["k"])
    ctx = P.Context(P.Params(align_mode=mode, full_records=True, **mid["prm"]))
    got = P.records_to_numpy(ctx.align_pairs(mid["res"], mid["off"], _dev(lo, gpu), _dev(hi, gpu), _dev(s1, gpu),
                                             _dev(s2, gpu)))
    assert FIELDS[-1] == "cells"
    _compare(got, ref)
