"""Pins for the oracle's alignment (Section IV-E) and filter (Section IV-F).

Independent of the oracle's DP: exhaustive enumeration of every alignment of
tiny sequences (maximum score, canonical end, and the canonical path chosen by
comparing whole alignments), hand-worked cases, self-alignment, swap symmetry,
the XD <= SW bound (every x-drop alignment is a local alignment), and x-drop
at finite X against a dictionary enumeration of the grid (scores, ends, paths
and the live-predecessor cell count) plus hand-worked pruning cases.
"""

import functools
import itertools

import numpy as np
import pytest

ALPHA = "ARNDCQEGHILKMFPSTWYVBZX*"
O, E = 11, 1


def enc(s):
    return np.array([ALPHA.index(c) for c in s], np.uint8)


@functools.lru_cache(maxsize=None)
def _paths(m, n):
    """All global alignment op strings of lengths m and n over M (diagonal),
    E (consumes a column of b) and F (consumes a row of a)."""
    if m == 0 and n == 0:
        return [""]
    out = []
    if m > 0 and n > 0:
        out += [p + "M" for p in _paths(m - 1, n - 1)]
    if n > 0:
        out += [p + "E" for p in _paths(m, n - 1)]
    if m > 0:
        out += [p + "F" for p in _paths(m - 1, n)]
    return out


def _score_path(B, a, b, ops):
    i = j = 0
    s = 0
    matches = 0
    prev = None
    for op in ops:
        if op == "M":
            s += int(B[a[i], b[j]])
            matches += int(a[i] == b[j])
            i += 1
            j += 1
        else:
            s -= E + (O if prev != op else 0)
            if op == "E":
                j += 1
            else:
                i += 1
        prev = op
    return s, matches


# state-dependent preference read backwards from the end of the alignment:
# in H: stop < diagonal < E < F; in a gap: extend first, then as in H.
_RANK = {
    "H": {"": 0, "M": 1, "E": 2, "F": 3},
    "E": {"E": 0, "": 1, "M": 2, "F": 3},
    "F": {"F": 0, "": 1, "M": 2, "E": 3},
}


def _canon_key(ops):
    back = ops[::-1]
    key = []
    state = "H"
    for t in range(len(back) + 1):
        op = back[t] if t < len(back) else ""
        key.append(_RANK[state][op])
        if op == "":
            break
        state = "H" if op == "M" else op
    return key


def _enumerate_local(B, a, b):
    """Every local alignment: (score, end_a, end_b, key, beg_a, beg_b, matches, columns)."""
    out = []
    for i0 in range(len(a)):
        for i1 in range(i0 + 1, len(a) + 1):
            for j0 in range(len(b)):
                for j1 in range(j0 + 1, len(b) + 1):
                    for ops in _paths(i1 - i0, j1 - j0):
                        if ops[0] != "M" or ops[-1] != "M":
                            continue  # a gap at either end never helps
                        s, m = _score_path(B, a[i0:i1], b[j0:j1], ops)
                        out.append((s, i1 - 1, j1 - 1, _canon_key(ops), i0, j0, m, len(ops)))
    return out


def _check_sw(orc, B, a, b):
    r = orc.sw(a, b, O, E)
    al = _enumerate_local(B, a, b)
    best = max([x[0] for x in al] + [0])
    assert r["score"] == best
    if best == 0:
        assert r["columns"] == 0 and r["end_a"] == -1
        return
    opt = [x for x in al if x[0] == best]
    end = min((x[1], x[2]) for x in opt)
    assert (r["end_a"], r["end_b"]) == end
    canon = min((x for x in opt if (x[1], x[2]) == end), key=lambda x: x[3])
    assert (r["beg_a"], r["beg_b"], r["matches"], r["columns"]) == (canon[4], canon[5], canon[6], canon[7])


def test_sw_exhaustive_small(orc):
    B = orc.blosum62()
    rng = np.random.default_rng(1)
    for _ in range(60):
        a = rng.integers(0, 20, int(rng.integers(1, 5))).astype(np.uint8)
        b = rng.integers(0, 20, int(rng.integers(1, 5))).astype(np.uint8)
        _check_sw(orc, B, a, b)


def test_sw_exhaustive_tie_rich(orc):
    """Few letters with close scores create many co-optimal paths."""
    B = orc.blosum62()
    rng = np.random.default_rng(2)
    letters = np.array([ALPHA.index(c) for c in "ASTW"], np.uint8)
    for _ in range(40):
        a = rng.choice(letters, int(rng.integers(2, 6)))
        b = rng.choice(letters, int(rng.integers(2, 6)))
        _check_sw(orc, B, a, b)


def test_sw_hand_worked(orc):
    # one mismatch: 8 W/W pairs (11 each) + A/C (0)
    r = orc.sw(enc("WWWWAWWWW"), enc("WWWWCWWWW"))
    assert (r["score"], r["matches"], r["columns"]) == (88, 8, 9)
    # a gap of one costs 11 + 1: 10 W pairs - 12
    r = orc.sw(enc("W" * 10), enc("WWWWWGWWWWW"))
    assert (r["score"], r["matches"], r["columns"], r["beg_b"], r["end_b"]) == (98, 10, 11, 0, 10)
    # a gap of three costs 11 + 3
    r = orc.sw(enc("W" * 10), enc("WWWWWGGGWWWWW"))
    assert (r["score"], r["columns"]) == (96, 13)
    # no positive cell: no alignment
    r = orc.sw(enc("WWW"), enc("PPP"))
    assert r["score"] == 0 and r["columns"] == 0


def test_sw_self_alignment(orc):
    B = orc.blosum62()
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = rng.integers(0, 20, int(rng.integers(1, 300))).astype(np.uint8)
        r = orc.sw(a, a)
        assert r["score"] == int(sum(B[x, x] for x in a))
        assert (r["beg_a"], r["end_a"], r["matches"], r["columns"]) == (0, len(a) - 1, len(a), len(a))


def test_sw_swap_symmetry_and_nonnegative(orc):
    rng = np.random.default_rng(4)
    for _ in range(40):
        a = rng.integers(0, 20, int(rng.integers(0, 80))).astype(np.uint8)
        b = rng.integers(0, 20, int(rng.integers(0, 80))).astype(np.uint8)
        s1 = orc.sw(a, b)["score"]
        assert s1 == orc.sw(b, a)["score"] and s1 >= 0


def _enumerate_anchored(B, a, b):
    """Every global alignment of a[:u], b[:v] for all u, v (anchored at 0)."""
    out = [(0, 0, 0, [], 0, 0)]
    for u in range(len(a) + 1):
        for v in range(len(b) + 1):
            if u == 0 and v == 0:
                continue
            for ops in _paths(u, v):
                s, m = _score_path(B, a[:u], b[:v], ops)
                key = _canon_key(ops)[:-1]  # the anchor ends every path
                out.append((s, u + v, u, key, m, len(ops)))
    return out


def test_xdrop_unbounded_equals_enumeration(orc):
    B = orc.blosum62()
    rng = np.random.default_rng(5)
    letters = np.array([ALPHA.index(c) for c in "ASTWC"], np.uint8)
    for _ in range(50):
        a = rng.choice(letters, int(rng.integers(0, 5)))
        b = rng.choice(letters, int(rng.integers(0, 5)))
        r = orc.xdrop_extend(a, b, O, E, 10**6)
        al = _enumerate_anchored(B, a, b)
        best = max(x[0] for x in al)
        assert r["score"] == best
        opt = [x for x in al if x[0] == best]
        d, u = min((x[1], x[2]) for x in opt)
        assert (r["u"] + r["v"], r["u"]) == (d, u)
        canon = min((x for x in opt if (x[1], x[2]) == (d, u)), key=lambda x: x[3])
        assert (r["matches"], r["columns"]) == (canon[4], canon[5])


def test_xdrop_stops_on_drop(orc):
    a = enc("WWWW" + "P" * 12 + "W" * 10)
    b = enc("WWWW" + "G" * 12 + "W" * 10)
    # P/G scores -2: twelve of them fall 24 below the best, which X = 20 does not
    # survive but X = 49 does (4*11 - 24 + 10*11 = 130).
    r20 = orc.xdrop_extend(a, b, O, E, 20)
    assert (r20["score"], r20["u"], r20["v"]) == (44, 4, 4)
    r49 = orc.xdrop_extend(a, b, O, E, 49)
    assert (r49["score"], r49["u"], r49["v"], r49["matches"], r49["columns"]) == (130, 26, 26, 14, 26)
    assert r20["cells"] < r49["cells"]


def _xdrop_dense(B, a, b, x):
    """x-drop extension (Section IV-E) enumerated over a dictionary of every
    grid cell: anti-diagonal d = u + v visits all of its cells, computes those
    with a live predecessor, then marks live the computed cells that are not
    below the best score of the earlier anti-diagonals minus x, and only then
    raises the best.  Stops at the first anti-diagonal without a live cell.
    Returns the same fields as the oracle, with the live-predecessor cell count."""
    neg = -(10**9)
    la, lb = len(a), len(b)
    H, Eg, Fg = {(0, 0): 0}, {(0, 0): neg}, {(0, 0): neg}
    live = {(0, 0)}
    best, end, cells = 0, (0, 0), 0
    for d in range(1, la + lb + 1):
        computed = []
        for u in range(la + 1):
            v = d - u
            if not 0 <= v <= lb:
                continue
            up, left, dia = (u - 1, v), (u, v - 1), (u - 1, v - 1)
            has_up, has_left, has_dia = up in live, left in live, dia in live
            if not (has_up or has_left or has_dia):
                continue
            cells += 1
            Eg[(u, v)] = max(Eg[left] - E, H[left] - O - E) if has_left else neg
            Fg[(u, v)] = max(Fg[up] - E, H[up] - O - E) if has_up else neg
            dval = H[dia] + int(B[a[u - 1], b[v - 1]]) if has_dia else neg
            H[(u, v)] = max(dval, Eg[(u, v)], Fg[(u, v)])
            computed.append((u, v))
        survivors = [c for c in computed if H[c] >= best - x]
        if not survivors:
            break
        live.update(survivors)
        top = max(H[c] for c in survivors)
        if top > best:
            best, end = top, min(c for c in survivors if H[c] == top)
    # canonical path back to the anchor: diagonal, then E, then F; extend first
    (u, v), state, matches, columns = end, "H", 0, 0
    while (u, v, state) != (0, 0, "H"):
        if state == "H":
            dia = (u - 1, v - 1)
            if dia in live and H[(u, v)] == H[dia] + int(B[a[u - 1], b[v - 1]]):
                columns += 1
                matches += int(a[u - 1] == b[v - 1])
                u, v = u - 1, v - 1
            else:
                state = "E" if H[(u, v)] == Eg[(u, v)] else "F"
        elif state == "E":
            columns += 1
            left = (u, v - 1)
            state = "E" if Eg[left] - E >= H[left] - O - E else "H"
            v -= 1
        else:
            columns += 1
            up = (u - 1, v)
            state = "F" if Fg[up] - E >= H[up] - O - E else "H"
            u -= 1
    return dict(score=best, u=end[0], v=end[1], matches=matches, columns=columns, cells=cells)


def test_xdrop_cell_exactly_x_below_stays_live(orc):
    # A against A: anti-diagonal 1 holds the two gap cells at -12 = 0 - 12.
    # With X = 12 they stay live (only scores below best - X die), and the
    # diagonal cell (1,1) = 4 follows: 3 cells, score 4.  With X = 11 both gap
    # cells die, anti-diagonal 1 has no live cell and the extension stops.
    a, b = enc("A"), enc("A")
    assert orc.xdrop_extend(a, b, O, E, 12) == dict(score=4, u=1, v=1, matches=1, columns=1, cells=3)
    assert orc.xdrop_extend(a, b, O, E, 11) == dict(score=0, u=0, v=0, matches=0, columns=0, cells=2)
    # WWWW against AWWWW: the best path opens with the gap cell (0,1) at
    # exactly best - X = -12 and then matches four W: -12 + 4 * 11 = 32 at
    # (4,5), one gap column and four matches.  The gap-free path scores only
    # -3 + 3 * 11 = 30 at (4,4); no path with four matches avoids a gap.
    r = orc.xdrop_extend(enc("WWWW"), enc("AWWWW"), O, E, 12)
    assert (r["score"], r["u"], r["v"], r["matches"], r["columns"]) == (32, 4, 5, 4, 5)
    assert orc.xdrop_extend(enc("WWWW"), enc("AWWWW"), O, E, 11)["score"] == 0


def test_xdrop_prunes_against_earlier_antidiagonals_only(orc):
    # WKA (rows) against W (one column), X = 16, worked by hand:
    #   d=1: (1,0) = (0,1) = -12, both live (>= 0 - 16); best stays 0.  2 cells
    #   d=2: (1,1) = 0 + W/W 11 = 11; (2,0) = -13.  Both are judged against the
    #        best of anti-diagonals < 2, which is 0: both live (-13 >= -16).
    #        A best raised within the anti-diagonal (11 - 16 = -5) would have
    #        killed (2,0).  best = 11.  4 cells
    #   d=3: (2,1) = max(-12 + K/W -3, 11 - 12, (2,0) - 12) = -1 (live);
    #        (3,0) = -14 from the live (2,0) (dead, < -5).  6 cells
    #   d=4: (3,1) = max((2,0) + A/W -3 = -16, -1 - 12 = -13) = -13, dead: stop.
    #        7 cells; without (2,0) there would be no (3,0) and 6 cells.
    assert orc.xdrop_extend(enc("WKA"), enc("W"), O, E, 16) == dict(score=11, u=1, v=1, matches=1, columns=1,
                                                                      cells=7)
    # a case where the rule changes the score: a best raised within an
    # anti-diagonal would prune the start of the optimal path and end at 3
    B = orc.blosum62()
    a, b = enc("CPKPKW"), enc("EPPW")
    r = orc.xdrop_extend(a, b, O, E, 14)
    assert r == _xdrop_dense(B, a, b, 14)
    assert (r["score"], r["u"], r["v"], r["matches"], r["columns"], r["cells"]) == (5, 6, 4, 2, 6, 30)


def test_xdrop_matches_dense_enumeration(orc):
    # every field, the live-predecessor cell count included, at drops small
    # enough that pruning and ties at exactly best - X happen often
    B = orc.blosum62()
    rng = np.random.default_rng(8)
    letters = np.array([ALPHA.index(c) for c in "WAGCSPKE"], np.uint8)
    for _ in range(1500):
        a = rng.choice(letters, int(rng.integers(0, 9)))
        b = rng.choice(letters, int(rng.integers(0, 9)))
        x = int(rng.integers(0, 30))
        assert orc.xdrop_extend(a, b, O, E, x) == _xdrop_dense(B, a, b, x), (a, b, x)
    for _ in range(40):
        a = rng.integers(0, 20, int(rng.integers(20, 60))).astype(np.uint8)
        b = a.copy()
        for t in rng.choice(b.size, b.size // 3, replace=False):
            b[t] = rng.integers(0, 20)
        x = int(rng.integers(5, 50))
        assert orc.xdrop_extend(a, b, O, E, x) == _xdrop_dense(B, a, b, x)


def test_xd_self_pair_and_bound_by_sw(orc):
    from synth import workload

    B = orc.blosum62()
    s = workload("tiny")
    codes = orc.encode(s.residues)
    rng = np.random.default_rng(6)
    a = codes[s.offsets[0] : s.offsets[1]]
    r = orc.xd_seed(a, a, 10, 10, 6)
    assert r["score"] == int(sum(B[x, x] for x in a)) and r["matches"] == len(a)
    # family pairs: every x-drop alignment from any seed is a local alignment
    fam = np.nonzero(s.labels == s.labels[0])[0]
    for i, j in itertools.islice(itertools.combinations(fam, 2), 12):
        ai = codes[s.offsets[i] : s.offsets[i + 1]]
        bj = codes[s.offsets[j] : s.offsets[j + 1]]
        sw = orc.sw(ai, bj)["score"]
        for _ in range(3):
            pa = int(rng.integers(0, len(ai) - 6))
            pb = int(rng.integers(0, len(bj) - 6))
            assert orc.xd_seed(ai, bj, pa, pb, 6)["score"] <= sw


@pytest.mark.parametrize(
    "matches,columns,beg,end,la,ok",
    [
        (3, 10, 0, 6, 10, True),  # identity exactly 30%, coverage exactly 70%
        (3, 10, 0, 5, 10, False),  # coverage 60%
        (29, 100, 0, 99, 100, False),  # identity 29%
        (30, 100, 0, 99, 100, True),
        (7, 23, 0, 6, 10, True),  # 7/23 = 30.4%
        (7, 24, 0, 6, 10, False),  # 7/24 = 29.2%
    ],
)
def test_filter_boundaries(orc, matches, columns, beg, end, la, ok):
    rec = dict(score=5, matches=matches, columns=columns, beg_a=beg, end_a=end)
    assert orc.passes(rec, la, 30, 70) is ok


def test_search_edges_sorted_unique(orc):
    from synth import workload

    s = workload("tiny", n_families=4)
    e = orc.search(s.residues, s.offsets, k=6, ck_min=1)
    keys = list(zip(e["i"].tolist(), e["j"].tolist()))
    assert keys == sorted(set(keys)) and all(i < j for i, j in keys)
    assert (e["identity"] >= 0.3).all()
