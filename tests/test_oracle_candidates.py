"""Pins for the oracle's candidate discovery (Sections IV-A, IV-C, VI).

B = A A^T counts shared k-mers (Section IV-A) and is symmetric; with the
substitute semiring the m = 0 case must reduce to it.  Both are checked
against plain Python sets on small random inputs, and the two oracle routes
(all-pairs merge and row-wise inverted index) against each other.
"""

import itertools

import numpy as np
import pytest

ALPHA = "ARNDCQEGHILKMFPSTWYVBZX*"
NO = 0xFFFFFFFF


def _random_set(rng, n, lo, hi, letters):
    lens = rng.integers(lo, hi + 1, n)
    off = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    codes = rng.choice(np.array(letters, np.uint8), int(off[-1]))
    return codes.astype(np.uint8), off


def _kset(codes, off, i, k):
    s = codes[off[i] : off[i + 1]]
    d = {}
    for t in range(len(s) - k + 1):
        d.setdefault(tuple(int(x) for x in s[t : t + k]), t)
    return d


def _py_exact(codes, off, k, ck):
    n = len(off) - 1
    ks = [_kset(codes, off, i, k) for i in range(n)]
    out = []
    for i, j in itertools.combinations(range(n), 2):
        common = set(ks[i]) & set(ks[j])
        if len(common) >= max(ck, 1):
            keys = sorted((ks[i][t] << 16) | ks[j][t] for t in common)
            keys += [NO, NO]
            out.append((i, j, len(common), keys[0], keys[1]))
    return out


def _as_tuples(c):
    return list(zip(*(c[k].tolist() for k in ("lo", "hi", "count", "seed1", "seed2"))))


@pytest.mark.parametrize("k,ck", [(3, 1), (3, 2), (4, 1), (2, 3)])
def test_exact_against_python_sets(orc, k, ck):
    rng = np.random.default_rng(100 + k + ck)
    codes, off = _random_set(rng, 30, 0, 40, [0, 1, 4, 17])
    want = _py_exact(codes, off, k, ck)
    for method in ("brute", "index"):
        got = _as_tuples(orc.candidates(codes, off, k, ck_min=ck, method=method))
        assert got == want, method


def test_b_symmetric_and_diagonal(orc):
    """B_ij = B_ji and B_ii = |K(i)|: count row i against a copy of itself."""
    rng = np.random.default_rng(9)
    codes, off = _random_set(rng, 12, 5, 30, [0, 1, 2])
    n = len(off) - 1
    # duplicate every sequence: pair (i, i + n) shares exactly K(i)
    codes2 = np.concatenate([codes, codes])
    off2 = np.concatenate([off, off[1:] + off[-1]])
    c = orc.candidates(codes2, off2, 3)
    table = {(a, b): cnt for a, b, cnt in zip(c["lo"].tolist(), c["hi"].tolist(), c["count"].tolist())}
    for i in range(n):
        assert table.get((i, i + n), 0) == len(_kset(codes, off, i, 3))
        for j in range(n):
            if i != j:
                assert table.get((min(i, j), max(i, j)), 0) == table.get((min(i, j) + n, max(i, j) + n), 0)


def _py_subs(orc, codes, off, k, m, ck, alpha=20):
    B = orc.blosum62()
    n = len(off) - 1
    ks = [_kset(codes, off, i, k) for i in range(n)]
    cache = {}

    def S(p):
        if p not in cache:
            lst = []
            for s in itertools.product(range(alpha), repeat=k):
                if s == p:
                    continue
                d = sum(int(B[a, a] - B[a, b]) for a, b in zip(p, s))
                sid = 0
                for x in s:
                    sid = sid * 24 + x
                lst.append((d, sid, s))
            lst.sort()
            cache[p] = [(p, 0)] + [(s, d) for d, _, s in lst[:m]]
        return cache[p]

    AS = []
    for i in range(n):
        row = {}
        for p, pos in ks[i].items():
            for s, d in S(p):
                if s not in row or (d, pos) < row[s]:
                    row[s] = (d, pos)
        AS.append(row)

    def direction(r, c):
        common = [s for s in ks[c] if s in AS[r]]
        keys = []
        for s in common:
            pr, pc = AS[r][s][1], ks[c][s]
            keys.append((pr << 16 | pc) if r < c else (pc << 16 | pr))
        keys = sorted(keys) + [NO, NO]
        return len(common), keys[0], keys[1]

    out = []
    for i, j in itertools.combinations(range(n), 2):
        f = direction(i, j)
        b = direction(j, i)
        best = b if b[0] > f[0] else f
        if best[0] >= max(ck, 1):
            out.append((i, j) + best)
    return out


def test_substitutes_against_python_definition(orc):
    rng = np.random.default_rng(21)
    codes, off = _random_set(rng, 14, 0, 25, [0, 15, 16, 4, 7])
    want = _py_subs(orc, codes, off, 3, 6, 2)
    got = _as_tuples(orc.candidates(codes, off, 3, ck_min=2, n_subs=6))
    assert got == want


def test_substitutes_m0_reduces_to_exact(orc):
    rng = np.random.default_rng(22)
    codes, off = _random_set(rng, 40, 0, 60, [0, 1, 4, 17, 8])
    a = orc.candidates(codes, off, 3, ck_min=1, n_subs=0)
    b = orc.candidates(codes, off, 3, ck_min=1, method="brute")
    assert _as_tuples(a) == _as_tuples(b)


def test_row_subset_matches_full(orc):
    rng = np.random.default_rng(23)
    codes, off = _random_set(rng, 40, 5, 40, [0, 15, 16, 4, 7])
    full = _as_tuples(orc.candidates(codes, off, 3, ck_min=2, n_subs=5))
    rows = [3, 17, 29]
    sub = _as_tuples(orc.candidates(codes, off, 3, ck_min=2, n_subs=5, rows=rows))
    assert sub == [t for t in full if t[0] in rows or t[1] in rows]


def test_family_workload_candidates_are_mostly_family_pairs(orc):
    from synth import workload

    s = workload("tiny")
    codes = orc.encode(s.residues)
    c = orc.candidates(codes, s.offsets, 6, ck_min=1)
    same = s.labels[c["lo"]] == s.labels[c["hi"]]
    assert same.mean() > 0.9
    assert (c["lo"] < c["hi"]).all() and (c["count"] >= 1).all()


@pytest.mark.parametrize("m,ck", [(0, 1), (6, 2)])
def test_pair_counts_match_python_definition_on_every_pair(orc, m, ck):
    """The per-pair route (used at full size on sampled pairs) against the
    plain-Python definition over all pairs of a small random set."""
    rng = np.random.default_rng(24 + m)
    codes, off = _random_set(rng, 14, 0, 25, [0, 15, 16, 4, 7])
    want = _py_subs(orc, codes, off, 3, m, ck) if m else _as_tuples(orc.candidates(codes, off, 3, ck_min=ck,
                                                                                    method="brute"))
    lo, hi = np.triu_indices(off.size - 1, 1)
    p = orc.pair_counts(codes, off, lo, hi, 3, n_subs=m)
    keep = p["count"] >= ck
    got = _as_tuples(dict(lo=lo[keep], hi=hi[keep], count=p["count"][keep], seed1=p["seed1"][keep],
                          seed2=p["seed2"][keep]))
    assert got == want
    assert (p["count"][~keep] < ck).all()
    with pytest.raises(ValueError):
        orc.pair_counts(codes, off, [3], [3], 3)
