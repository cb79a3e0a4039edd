"""CPU oracle for the PASTIS hot path — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct implementations written from the paper
(Selvitopi et al., "Distributed Many-to-Many Protein Sequence Alignment using
Sparse Matrices", SC20).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never calls it and it never calls the GPU library; the two share no code.

What each function follows:
  * ``encode``/``kmer_id``/``kmer_set``: Section V-B (bases 0..23, radix-24 ids,
    leftmost residue most significant) and Section IV-A (A_ij = start position).
  * ``subkmers``: Section IV-B (E = Sort(Diag(C) - C), m nearest k-mers).
  * ``candidates``: Sections IV-A and IV-C (B = A A^T, A S A^T semirings) and
    the common-k-mer threshold of Section VI.
  * ``align_pairs``/``sw``/``xdrop_extend``: Section IV-E (SW and XD).
  * ``search``: the pipeline of Section IV with the filter of Section IV-F.
  * ``components``/``weighted_scores`` (``oracle.clusters``): connected
    components of the similarity graph as families, scored as in Section VI-B.
Points where the paper is silent are resolved in the C sources' headers.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

ALPHABET = "ARNDCQEGHILKMFPSTWYVBZX*"
NO_SEED = 0xFFFFFFFF

_lib = None

_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")

ALN_DTYPE = np.dtype(
    [
        ("score", np.int32),
        ("beg_a", np.int32),
        ("end_a", np.int32),
        ("beg_b", np.int32),
        ("end_b", np.int32),
        ("matches", np.int32),
        ("columns", np.int32),
        ("seed_used", np.int32),
        ("passed", np.int32),
        ("swapped", np.int32),
        ("cells", np.int64),
    ],
    align=True,
)

EDGE_DTYPE = np.dtype(
    [
        ("i", np.uint32),
        ("j", np.uint32),
        ("score", np.int32),
        ("matches", np.uint32),
        ("columns", np.uint32),
        ("beg_i", np.uint32),
        ("end_i", np.uint32),
        ("beg_j", np.uint32),
        ("end_j", np.uint32),
        ("shared_kmers", np.uint16),
        ("seed_used", np.uint8),
        ("flags", np.uint8),
        ("identity", np.float32),
        ("ns_weight", np.float32),
    ]
)
assert EDGE_DTYPE.itemsize == 48


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_blosum62.restype = ctypes.c_int
        L.orc_blosum62.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_encode.restype = ctypes.c_int64
        L.orc_encode.argtypes = [_u8p, ctypes.c_int64, _u8p]
        L.orc_kmer_id.restype = ctypes.c_int64
        L.orc_kmer_id.argtypes = [_u8p, ctypes.c_int]
        L.orc_kmer_set.restype = ctypes.c_int64
        L.orc_kmer_set.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int, _i64p, _i32p]
        L.orc_expense.restype = ctypes.c_int
        L.orc_expense.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_expense_row.restype = ctypes.c_int
        L.orc_expense_row.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, _i32p]
        for name in ("orc_subk_bruteforce", "orc_subk_bounded"):
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64p, _i32p]
        L.orc_candidates_bruteforce.restype = ctypes.c_int64
        L.orc_candidates_bruteforce.argtypes = [_u8p, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_int64, _u32p, _u32p, _u32p, _u32p, _u32p]
        L.orc_candidates_index.restype = ctypes.c_int64
        L.orc_candidates_index.argtypes = [_u8p, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int64, _u32p, _u32p,
                                           _u32p, _u32p, _u32p]
        L.orc_pair_counts.restype = ctypes.c_int64
        L.orc_pair_counts.argtypes = [_u8p, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _u32p,
                                      _u32p, ctypes.c_int64, _u32p, _u32p, _u32p]
        aln_p = np.ctypeslib.ndpointer(dtype=ALN_DTYPE, flags="C_CONTIGUOUS")
        L.orc_sw.restype = None
        L.orc_sw.argtypes = [_u8p, ctypes.c_int, _u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, aln_p]
        L.orc_xdrop_extend.restype = ctypes.c_int32
        L.orc_xdrop_extend.argtypes = [_u8p, ctypes.c_int, _u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, _i32p, _i32p, _i32p, _i32p, _i64p]
        L.orc_xd_seed.restype = None
        L.orc_xd_seed.argtypes = [_u8p, ctypes.c_int, _u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, aln_p]
        L.orc_align_pairs.restype = None
        L.orc_align_pairs.argtypes = [_u8p, _i64p, _u32p, _u32p, _u32p, _u32p, ctypes.c_int64, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, aln_p]
        L.orc_passes.restype = ctypes.c_int
        L.orc_passes.argtypes = [aln_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (n <= 0: all cores); results do not depend on it."""
    lib().orc_set_threads(int(n))


# ---------------------------------------------------------------- alphabet


def blosum62() -> np.ndarray:
    L = lib()
    return np.array([[L.orc_blosum62(a, b) for b in range(24)] for a in range(24)], dtype=np.int64)


def encode(ascii) -> np.ndarray:
    """ASCII letters -> codes 0..23; ValueError names the first bad byte."""
    if isinstance(ascii, (bytes, str)):
        ascii = np.frombuffer(ascii.encode() if isinstance(ascii, str) else ascii, dtype=np.uint8)
    a = np.ascontiguousarray(ascii, dtype=np.uint8)
    out = np.zeros(max(a.size, 1), dtype=np.uint8)
    bad = lib().orc_encode(a if a.size else np.zeros(1, np.uint8), a.size, out)
    if bad >= 0:
        raise ValueError(f"bad residue at index {bad}")
    return out[: a.size]


def kmer_id(kmer, k=None) -> int:
    c = encode(kmer) if isinstance(kmer, (str, bytes)) else np.ascontiguousarray(kmer, dtype=np.uint8)
    return int(lib().orc_kmer_id(c, len(c) if k is None else k))


def kmer_string(kid: int, k: int) -> str:
    s = []
    for _ in range(k):
        s.append(ALPHABET[kid % 24])
        kid //= 24
    return "".join(reversed(s))


def kmer_set(codes, k: int):
    c = np.ascontiguousarray(codes, dtype=np.uint8)
    w = max(c.size - k + 1, 1)
    ids = np.zeros(w, dtype=np.int64)
    pos = np.zeros(w, dtype=np.int32)
    m = lib().orc_kmer_set(c if c.size else np.zeros(1, np.uint8), c.size, k, ids, pos)
    return ids[:m], pos[:m]


def expense_row(a: int, alpha: int = 24):
    base = np.zeros(alpha, np.int32)
    ex = np.zeros(alpha, np.int32)
    lib().orc_expense_row(a, alpha, base, ex)
    return base, ex


def subkmers(r: int, k: int, m: int, alpha: int = 20, method: str = "bounded"):
    """The m nearest substitute k-mers of k-mer id r: (ids, distances)."""
    ids = np.zeros(max(m, 1), np.int64)
    dist = np.zeros(max(m, 1), np.int32)
    f = lib().orc_subk_bounded if method == "bounded" else lib().orc_subk_bruteforce
    got = f(int(r), k, m, alpha, ids, dist)
    return ids[:got], dist[:got]


# ---------------------------------------------------------------- candidates


def candidates(codes, offsets, k: int, ck_min: int = 1, n_subs: int = 0, alpha: int = 20, rows=None,
               method: str = "index", cap: int | None = None) -> dict:
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = offsets.size - 1
    if codes.size == 0:
        codes = np.zeros(1, np.uint8)
    cap = cap or max(1024, 4 * n)
    while True:
        lo = np.zeros(cap, np.uint32)
        hi = np.zeros(cap, np.uint32)
        cnt = np.zeros(cap, np.uint32)
        s1 = np.zeros(cap, np.uint32)
        s2 = np.zeros(cap, np.uint32)
        if method == "brute":
            assert n_subs == 0 and rows is None
            got = lib().orc_candidates_bruteforce(codes, offsets, n, k, ck_min, cap, lo, hi, cnt, s1, s2)
        else:
            r = np.ascontiguousarray(rows if rows is not None else np.zeros(1), dtype=np.int64)
            nr = -1 if rows is None else len(rows)
            got = lib().orc_candidates_index(codes, offsets, n, k, n_subs, alpha, ck_min, r, nr, cap, lo, hi, cnt,
                                             s1, s2)
        if got >= 0:
            return dict(lo=lo[:got], hi=hi[:got], count=cnt[:got], seed1=s1[:got], seed2=s2[:got])
        cap *= 4


def pair_counts(codes, offsets, lo, hi, k: int, n_subs: int = 0, alpha: int = 20) -> dict:
    """Shared (substitute) k-mer count and seeds of the listed pairs lo < hi,
    as candidate discovery defines them, without the threshold (count 0 when
    the pair shares nothing).  Needs only the listed pairs' sequences."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    lo = np.ascontiguousarray(lo, dtype=np.uint32)
    hi = np.ascontiguousarray(hi, dtype=np.uint32)
    if codes.size == 0:
        codes = np.zeros(1, np.uint8)
    m = lo.size
    cnt = np.zeros(max(m, 1), np.uint32)
    s1 = np.zeros(max(m, 1), np.uint32)
    s2 = np.zeros(max(m, 1), np.uint32)
    got = lib().orc_pair_counts(codes, offsets, offsets.size - 1, k, n_subs, alpha, lo if m else np.zeros(1, np.uint32),
                                hi if m else np.zeros(1, np.uint32), m, cnt, s1, s2)
    if got < 0:
        raise ValueError("pairs must satisfy lo < hi < n")
    return dict(count=cnt[:m], seed1=s1[:m], seed2=s2[:m])


# ---------------------------------------------------------------- alignment


def sw(a, b, gap_open: int = 11, gap_extend: int = 1) -> dict:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.zeros(1, ALN_DTYPE)
    lib().orc_sw(a if a.size else np.zeros(1, np.uint8), a.size, b if b.size else np.zeros(1, np.uint8), b.size,
                 gap_open, gap_extend, out)
    return {k: int(out[0][k]) for k in ALN_DTYPE.names}


def xdrop_extend(a, b, gap_open: int = 11, gap_extend: int = 1, xdrop: int = 49) -> dict:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    u = np.zeros(1, np.int32)
    v = np.zeros(1, np.int32)
    m = np.zeros(1, np.int32)
    c = np.zeros(1, np.int32)
    cells = np.zeros(1, np.int64)
    s = lib().orc_xdrop_extend(a if a.size else np.zeros(1, np.uint8), a.size, b if b.size else np.zeros(1, np.uint8),
                               b.size, gap_open, gap_extend, xdrop, u, v, m, c, cells)
    return dict(score=int(s), u=int(u[0]), v=int(v[0]), matches=int(m[0]), columns=int(c[0]), cells=int(cells[0]))


def xd_seed(a, b, pos_a: int, pos_b: int, k: int, gap_open=11, gap_extend=1, xdrop=49) -> dict:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.zeros(1, ALN_DTYPE)
    lib().orc_xd_seed(a, a.size, b, b.size, pos_a, pos_b, k, gap_open, gap_extend, xdrop, out)
    return {kk: int(out[0][kk]) for kk in ALN_DTYPE.names}


def passes(rec: dict, la: int, min_identity: int = 30, min_coverage: int = 70) -> bool:
    """The similarity filter of Section IV-F on one alignment record."""
    r = np.zeros(1, ALN_DTYPE)
    for key, val in rec.items():
        r[0][key] = val
    return bool(lib().orc_passes(r, la, min_identity, min_coverage))


def align_pairs(codes, offsets, pi, pj, seed1=None, seed2=None, *, mode: str = "sw", k: int = 6, gap_open: int = 11,
                gap_extend: int = 1, xdrop: int = 49, min_identity: int = 30, min_coverage: int = 70) -> np.ndarray:
    """Per-pair records (ALN_DTYPE) in the rows=a / columns=b orientation."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    pi = np.ascontiguousarray(pi, dtype=np.uint32)
    pj = np.ascontiguousarray(pj, dtype=np.uint32)
    npairs = pi.size
    s1 = np.ascontiguousarray(seed1 if seed1 is not None else np.full(max(npairs, 1), NO_SEED), dtype=np.uint32)
    s2 = np.ascontiguousarray(seed2 if seed2 is not None else np.full(max(npairs, 1), NO_SEED), dtype=np.uint32)
    out = np.zeros(max(npairs, 1), ALN_DTYPE)
    if npairs:
        lib().orc_align_pairs(codes if codes.size else np.zeros(1, np.uint8), offsets, pi, pj, s1, s2, npairs,
                              0 if mode == "sw" else 1, k, gap_open, gap_extend, xdrop, min_identity, min_coverage,
                              out)
    return out[:npairs]


def records_to_edges(pi, pj, counts, rec, lengths, weight: str = "ani") -> np.ndarray:
    """Similarity-graph edges (EDGE_DTYPE, sorted by (i, j)) from pair records.

    ANI mode keeps pairs that pass the identity/coverage cut, weight =
    matches/columns in float32 (Section VI-B).  NS mode keeps every pair with
    a positive score, weight = score / shorter length, and no cut-off
    (Section VI-B); the weight needs only the score, so its edges carry no
    traceback statistics and no alignment coordinates (begins and ends
    reported as 0xFFFFFFFF, matches, columns and identity as 0).
    """
    pi = np.asarray(pi, dtype=np.uint32)
    pj = np.asarray(pj, dtype=np.uint32)
    keep = rec["passed"] == 1 if weight == "ani" else rec["score"] > 0
    idx = np.nonzero(keep)[0]
    e = np.zeros(idx.size, EDGE_DTYPE)
    r = rec[idx]
    i = pi[idx]
    j = pj[idx]
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    # a is the first of (i, j) unless swapped; map (a, b) back onto (lo, hi)
    a_is_lo = (r["swapped"] == 0) == (i < j)
    e["i"] = lo
    e["j"] = hi
    e["score"] = r["score"]
    e["matches"] = r["matches"]
    e["columns"] = r["columns"]
    e["beg_i"] = np.where(a_is_lo, r["beg_a"], r["beg_b"])
    e["end_i"] = np.where(a_is_lo, r["end_a"], r["end_b"])
    e["beg_j"] = np.where(a_is_lo, r["beg_b"], r["beg_a"])
    e["end_j"] = np.where(a_is_lo, r["end_b"], r["end_a"])
    e["shared_kmers"] = np.minimum(np.asarray(counts)[idx], 65535)
    e["seed_used"] = np.where(r["seed_used"] < 0, 255, r["seed_used"]).astype(np.uint8)
    e["flags"] = r["swapped"].astype(np.uint8)
    e["identity"] = r["matches"].astype(np.float32) / np.maximum(r["columns"], 1).astype(np.float32)
    lens = np.asarray(lengths)
    short = np.minimum(lens[lo], lens[hi]).astype(np.float32)
    e["ns_weight"] = r["score"].astype(np.float32) / short
    if weight == "ns":
        # the normalised score needs only the score (Section VI-B): the
        # traceback statistics and the alignment's extent are not part of an
        # NS edge
        e["beg_i"] = e["beg_j"] = e["end_i"] = e["end_j"] = 0xFFFFFFFF
        e["matches"] = e["columns"] = 0
        e["identity"] = 0.0
    order = np.lexsort((e["j"], e["i"]))
    return e[order]


def encode_set(residues, offsets) -> np.ndarray:
    return encode(np.asarray(residues, dtype=np.uint8))


def search(residues, offsets, *, k: int = 6, n_subs: int = 0, alpha: int = 20, ck_min: int = 1, mode: str = "sw",
           gap_open: int = 11, gap_extend: int = 1, xdrop: int = 49, min_identity: int = 30, min_coverage: int = 70,
           weight: str = "ani", return_all: bool = False):
    """Sequences in, weighted similarity edges out (the whole pipeline)."""
    codes = encode_set(residues, offsets)
    offsets = np.asarray(offsets, dtype=np.int64)
    cand = candidates(codes, offsets, k, ck_min=ck_min, n_subs=n_subs, alpha=alpha)
    rec = align_pairs(codes, offsets, cand["lo"], cand["hi"], cand["seed1"], cand["seed2"], mode=mode, k=k,
                      gap_open=gap_open, gap_extend=gap_extend, xdrop=xdrop, min_identity=min_identity,
                      min_coverage=min_coverage)
    edges = records_to_edges(cand["lo"], cand["hi"], cand["count"], rec, np.diff(offsets), weight=weight)
    if return_all:
        return edges, cand, rec
    return edges


# ---------------------------------------------------------------- graph

from .clusters import components, weighted_scores  # noqa: E402,F401
