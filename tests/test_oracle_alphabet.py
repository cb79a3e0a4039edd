"""Pins for the oracle's alphabet, BLOSUM62 and k-mer functions.

Each check ties the oracle to something outside itself: numbers printed in the
paper (tests/golden/paper_examples.txt), a second independent transcription of
BLOSUM62 (the input generator's), or brute force.
"""

import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.txt")
ALPHA = "ARNDCQEGHILKMFPSTWYVBZX*"


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if line:
            rows.append(line.split())
    return rows


def _score(B, x, y):
    return sum(int(B[ALPHA.index(p), ALPHA.index(q)]) for p, q in zip(x, y))


def test_paper_examples(orc):
    B = orc.blosum62()
    rows = _golden()
    assert len(rows) >= 10
    for row in rows:
        kind = row[0]
        if kind == "kmer_id":
            assert orc.kmer_id(row[1]) == int(row[2])
        elif kind == "kmer_score":
            assert _score(B, row[1], row[2]) == int(row[3])
        elif kind == "blosum":
            assert B[ALPHA.index(row[1]), ALPHA.index(row[2])] == int(row[3])
        elif kind == "expense_prefix":
            base, ex = orc.expense_row(ALPHA.index(row[1]), 24)
            want = [tuple(t.split(":")) for t in row[2].split(",")]
            got = [(ALPHA[b], str(e)) for b, e in zip(base[: len(want)], ex[: len(want)])]
            assert got == want
        elif kind == "dist":
            r, s = row[1], row[2]
            d = sum(orc.lib().orc_expense(ALPHA.index(p), ALPHA.index(q)) for p, q in zip(r, s))
            assert d == int(row[3])
        elif kind == "closer_than_all":
            r, s, pat = row[1], row[2], row[3]
            ds = sum(orc.lib().orc_expense(ALPHA.index(p), ALPHA.index(q)) for p, q in zip(r, s))
            for x in ALPHA[:20]:
                other = pat.replace("*", x)
                if other == r:
                    continue
                d = sum(orc.lib().orc_expense(ALPHA.index(p), ALPHA.index(q)) for p, q in zip(r, other))
                assert ds < d, (other, d)
        else:
            raise AssertionError(f"unknown golden kind {kind}")


def test_blosum62_structure(orc):
    B = orc.blosum62()
    assert B.shape == (24, 24)
    assert (B == B.T).all()
    diag20 = [4, 5, 6, 6, 9, 5, 5, 6, 8, 4, 4, 5, 5, 6, 7, 4, 5, 11, 7, 4]
    assert list(np.diag(B)[:20]) == diag20
    off = B[:20, :20] - np.diag(np.diag(B[:20, :20])) - np.eye(20, dtype=int) * 100
    # every substitution among the 20 standard residues scores below every match
    assert off.max() <= 3 < min(diag20)
    assert B[:, 23][:23].max() == -4 and B[23, 23] == 1


def test_blosum62_matches_generator_transcription(orc):
    """The input generator carries its own 20x20 copy; the two must agree."""
    from synth.families import _B62_20

    assert (orc.blosum62()[:20, :20] == _B62_20).all()


def test_encode(orc):
    assert list(orc.encode("ARNDCQEGHILKMFPSTWYVBZX*")) == list(range(24))
    with pytest.raises(ValueError, match="index 3"):
        orc.encode("ACDJ")
    with pytest.raises(ValueError, match="index 0"):
        orc.encode("a")
    assert orc.encode("").size == 0


def test_kmer_id_radix24(orc):
    rng = np.random.default_rng(5)
    for k in range(1, 8):
        for _ in range(20):
            c = rng.integers(0, 24, k)
            assert orc.kmer_id(c.astype(np.uint8)) == sum(int(c[t]) * 24 ** (k - 1 - t) for t in range(k))


def test_kmer_set_bruteforce(orc):
    rng = np.random.default_rng(7)
    for _ in range(60):
        L = int(rng.integers(0, 40))
        k = int(rng.integers(1, 6))
        # small alphabet so that k-mers repeat inside a sequence
        c = rng.integers(0, 3, L).astype(np.uint8)
        ids, pos = orc.kmer_set(c, k)
        first = {}
        for t in range(L - k + 1):
            key = tuple(c[t : t + k])
            first.setdefault(key, t)
        want = sorted((orc.kmer_id(np.array(key, np.uint8)), t) for key, t in first.items())
        assert [(int(a), int(b)) for a, b in zip(ids, pos)] == want
