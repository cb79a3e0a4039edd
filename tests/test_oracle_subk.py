"""Pins for the oracle's m-nearest substitute k-mers (Section IV-B).

Pinned by the paper's AAC example, by plain Python enumeration of every k-mer
for small k, and by the agreement of the oracle's two routes (full scan and
distance-bounded enumeration) at k = 5, 6.
"""

import itertools

import numpy as np
import pytest

ALPHA = "ARNDCQEGHILKMFPSTWYVBZX*"


def _py_nearest(orc, r: str, m: int, alpha: int):
    B = orc.blosum62()
    rc = [ALPHA.index(x) for x in r]
    k = len(r)
    out = []
    for s in itertools.product(range(alpha), repeat=k):
        sid = 0
        for x in s:
            sid = sid * 24 + x
        if list(s) == rc:
            continue
        d = sum(int(B[a, a] - B[a, b]) for a, b in zip(rc, s))
        out.append((d, sid))
    out.sort()
    return out[:m]


def test_aac_neighbourhood(orc):
    r = orc.kmer_id("AAC")
    ids, d = orc.subkmers(r, 3, 2, 20)
    assert sorted(orc.kmer_string(i, 3) for i in ids) == ["ASC", "SAC"]
    assert list(d) == [3, 3]
    ids, d = orc.subkmers(r, 3, 10, 20)
    names = [orc.kmer_string(i, 3) for i in ids]
    assert set(names[2:]) == {"CAC", "GAC", "TAC", "VAC", "ACC", "AGC", "ATC", "AVC"}
    assert list(d) == [3, 3] + [4] * 8
    # all 16 of {C,G,T,V}{C,G,T,V}C (distance 8) come before any AAx, x != C
    ids, d = orc.subkmers(r, 3, 200, 20)
    names = [orc.kmer_string(i, 3) for i in ids]
    pos = {n: t for t, n in enumerate(names)}
    two_hop = [a + b + "C" for a in "CGTV" for b in "CGTV"]
    aax = [n for n in names if n.startswith("AA") and n != "AAC"]
    assert aax, "200 nearest should reach some AAx"
    assert max(pos[n] for n in two_hop) < min(pos[n] for n in aax)


@pytest.mark.parametrize("alpha", [20, 24])
def test_against_python_enumeration_k3(orc, alpha):
    rng = np.random.default_rng(11)
    for _ in range(12):
        r = "".join(ALPHA[int(x)] for x in rng.integers(0, alpha, 3))
        m = int(rng.integers(1, 60))
        want = _py_nearest(orc, r, m, alpha)
        for method in ("bounded", "brute"):
            ids, d = orc.subkmers(orc.kmer_id(r), 3, m, alpha, method)
            assert [(int(a), int(b)) for a, b in zip(d, ids)] == want, (r, m, method)


def test_bounded_equals_full_scan(orc):
    rng = np.random.default_rng(3)
    for k, trials in ((4, 30), (5, 4), (6, 2)):
        for _ in range(trials):
            r = orc.kmer_id("".join(ALPHA[int(x)] for x in rng.integers(0, 20, k)))
            full = orc.subkmers(r, k, 50, 20, "brute")
            for m in (1, 10, 25, 50):
                a = orc.subkmers(r, k, m, 20, "bounded")
                # the m nearest under a total order are a prefix of the 50 nearest
                assert (a[0] == full[0][:m]).all() and (a[1] == full[1][:m]).all()


def test_distances_sorted_and_exclude_root(orc):
    rng = np.random.default_rng(4)
    for _ in range(50):
        r = orc.kmer_id("".join(ALPHA[int(x)] for x in rng.integers(0, 20, 6)))
        ids, d = orc.subkmers(r, 6, 25, 20)
        assert len(ids) == 25 and r not in set(ids.tolist())
        keys = list(zip(d.tolist(), ids.tolist()))
        assert keys == sorted(keys)
