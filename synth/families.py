"""Family-structured random protein sets (seeded).

Recipe (stated once here, recorded in every set's ``meta``):

* Residues of ancestors and insertions are drawn i.i.d. from the background
  frequencies implied by BLOSUM62 over the 20 standard amino acids: the vector p
  solving  sum_b p_b * exp(lambda * s_ab) = 1  for every a, lambda = ln(2)/2
  (BLOSUM62 is in half-bit units), normalised to sum 1.
* Ancestor lengths are lognormal with sigma = 0.6 and mu = ln(mean) - sigma^2/2,
  rounded and clamped to [min_len, max_len]; an optional fraction of ancestors
  instead takes a uniform length in a long range (heavy-tail workload).
* Every family member is mutated independently from its ancestor (star
  phylogeny): each position is substituted with probability ``divergence`` by
  b != a drawn with probability proportional to p_b * exp(lambda * s_ab); then
  each position starts an indel event with probability ``indel_rate``
  (insertion or deletion, 50/50) of geometric length with mean ``indel_mean``.
  Members are truncated at ``max_len``.  The ancestor itself is not a member.
* Unrelated singletons are fresh ancestors of their own.
* The sequence order is a seeded random permutation; ``labels`` keeps the
  family id (or -1 for a singleton).
* Workload w's stream is ``SeedSequence(seed, spawn_key=(w,))``.

The substitution table below is BLOSUM62 (Henikoff & Henikoff 1992) restricted
to the 20 standard residues; it is used only to draw mutations.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

ALPHABET20 = "ARNDCQEGHILKMFPSTWYV"

_B62_20 = np.array(
    [
        # A  R  N  D  C  Q  E  G  H  I  L  K  M  F  P  S  T  W  Y  V
        [4, -1, -2, -2, 0, -1, -1, 0, -2, -1, -1, -1, -1, -2, -1, 1, 0, -3, -2, 0],
        [-1, 5, 0, -2, -3, 1, 0, -2, 0, -3, -2, 2, -1, -3, -2, -1, -1, -3, -2, -3],
        [-2, 0, 6, 1, -3, 0, 0, 0, 1, -3, -3, 0, -2, -3, -2, 1, 0, -4, -2, -3],
        [-2, -2, 1, 6, -3, 0, 2, -1, -1, -3, -4, -1, -3, -3, -1, 0, -1, -4, -3, -3],
        [0, -3, -3, -3, 9, -3, -4, -3, -3, -1, -1, -3, -1, -2, -3, -1, -1, -2, -2, -1],
        [-1, 1, 0, 0, -3, 5, 2, -2, 0, -3, -2, 1, 0, -3, -1, 0, -1, -2, -1, -2],
        [-1, 0, 0, 2, -4, 2, 5, -2, 0, -3, -3, 1, -2, -3, -1, 0, -1, -3, -2, -2],
        [0, -2, 0, -1, -3, -2, -2, 6, -2, -4, -4, -2, -3, -3, -2, 0, -2, -2, -3, -3],
        [-2, 0, 1, -1, -3, 0, 0, -2, 8, -3, -3, -1, -2, -1, -2, -1, -2, -2, 2, -3],
        [-1, -3, -3, -3, -1, -3, -3, -4, -3, 4, 2, -3, 1, 0, -3, -2, -1, -3, -1, 3],
        [-1, -2, -3, -4, -1, -2, -3, -4, -3, 2, 4, -2, 2, 0, -3, -2, -1, -2, -1, 1],
        [-1, 2, 0, -1, -3, 1, 1, -2, -1, -3, -2, 5, -1, -3, -1, 0, -1, -3, -2, -2],
        [-1, -1, -2, -3, -1, 0, -2, -3, -2, 1, 2, -1, 5, 0, -2, -1, -1, -1, -1, 1],
        [-2, -3, -3, -3, -2, -3, -3, -3, -1, 0, 0, -3, 0, 6, -4, -2, -2, 1, 3, -1],
        [-1, -2, -2, -1, -3, -1, -1, -2, -2, -3, -3, -1, -2, -4, 7, -1, -1, -4, -3, -2],
        [1, -1, 1, 0, -1, 0, 0, 0, -1, -2, -2, 0, -1, -2, -1, 4, 1, -3, -2, -2],
        [0, -1, 0, -1, -1, -1, -1, -2, -2, -1, -1, -1, -1, -2, -1, 1, 5, -2, -2, 0],
        [-3, -3, -4, -4, -2, -2, -3, -2, -2, -3, -2, -3, -1, 1, -4, -3, -2, 11, 2, -3],
        [-2, -2, -2, -3, -2, -1, -2, -3, 2, -1, -1, -2, -1, 3, -3, -2, -2, 2, 7, -1],
        [0, -3, -3, -3, -1, -2, -2, -3, -3, 3, 1, -2, 1, -1, -2, -2, 0, -3, -1, 4],
    ],
    dtype=np.int64,
)

_LAMBDA = math.log(2.0) / 2.0
_ASCII20 = np.frombuffer(ALPHABET20.encode(), dtype=np.uint8)


def background_frequencies() -> np.ndarray:
    """BLOSUM62-implied background over ALPHABET20 (float64, sums to 1)."""
    m = np.exp(_LAMBDA * _B62_20.astype(np.float64))
    p = np.linalg.solve(m, np.ones(20))
    p = np.clip(p, 1e-6, None)
    return p / p.sum()


def _substitution_cdf(p: np.ndarray) -> np.ndarray:
    """Row a: cumulative P(b | a, substituted), zero mass on b == a."""
    w = p[None, :] * np.exp(_LAMBDA * _B62_20.astype(np.float64))
    np.fill_diagonal(w, 0.0)
    w /= w.sum(axis=1, keepdims=True)
    cdf = np.cumsum(w, axis=1)
    cdf[:, -1] = 1.0
    return cdf


@dataclasses.dataclass
class FamilySet:
    residues: np.ndarray  # uint8 ASCII letters, all sequences concatenated
    offsets: np.ndarray  # int64 [n + 1]
    labels: np.ndarray  # int32 [n]: family id, or -1 for a singleton
    meta: dict

    @property
    def n(self) -> int:
        return int(self.offsets.size - 1)

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def seq(self, i: int) -> bytes:
        return self.residues[self.offsets[i] : self.offsets[i + 1]].tobytes()

    def subset(self, idx) -> "FamilySet":
        idx = np.asarray(idx, dtype=np.int64)
        parts = [self.residues[self.offsets[i] : self.offsets[i + 1]] for i in idx]
        lens = np.array([len(x) for x in parts], dtype=np.int64)
        off = np.zeros(idx.size + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        res = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
        return FamilySet(res.astype(np.uint8), off, self.labels[idx].copy(), dict(self.meta, subset=True))


def _draw_lengths(rng, count, mean, min_len, max_len, long_frac, long_range):
    sigma = 0.6
    mu = math.log(mean) - sigma * sigma / 2.0
    lens = np.rint(np.exp(rng.normal(mu, sigma, count))).astype(np.int64)
    lens = np.clip(lens, min_len, max_len)
    if long_frac > 0.0:
        is_long = rng.random(count) < long_frac
        nl = int(is_long.sum())
        if nl:
            lens[is_long] = rng.integers(long_range[0], long_range[1] + 1, nl)
    return lens


def _sample_substitutes(rng, a, sub_cdf_flat):
    """For residues a (int array) draw b != a from the substitution rows."""
    u = rng.random(a.size)
    b = np.searchsorted(sub_cdf_flat, a + u, side="right") - 20 * a
    return np.minimum(b, 19)


def _mutate_family(rng, anc, size, divergence, indel_rate, indel_mean, sub_cdf_flat, p_cdf, max_len):
    """All members of one family at once.

    An indel event at position t is an insertion of g random residues right
    after t, or a deletion of the g residues starting at t (g geometric).
    """
    n = anc.size
    x = np.broadcast_to(anc, (size, n)).copy()
    hit = rng.random((size, n)) < divergence
    x[hit] = _sample_substitutes(rng, x[hit], sub_cdf_flat)

    mem, pos = np.nonzero(rng.random((size, n)) < indel_rate)
    is_ins = rng.random(mem.size) < 0.5
    glen = rng.geometric(1.0 / indel_mean, mem.size)
    delta = np.zeros((size, n + 1), dtype=np.int64)
    dm, dp, dl = mem[~is_ins], pos[~is_ins], glen[~is_ins]
    np.add.at(delta, (dm, dp), 1)
    np.add.at(delta, (dm, np.minimum(dp + dl, n)), -1)
    keep = (np.cumsum(delta, axis=1)[:, :n] == 0).astype(np.int64)
    extra = np.zeros((size, n), dtype=np.int64)
    np.add.at(extra, (mem[is_ins], pos[is_ins]), glen[is_ins])

    width = (keep + extra).ravel()
    src = np.repeat(np.arange(size * n), width)
    first = np.zeros(src.size, dtype=bool)
    starts = np.cumsum(width) - width
    first[starts[width > 0]] = True
    orig = first & np.repeat(keep.ravel().astype(bool), width)
    vals = np.empty(src.size, dtype=np.int64)
    vals[orig] = x.ravel()[src[orig]]
    n_new = int((~orig).sum())
    vals[~orig] = np.searchsorted(p_cdf, rng.random(n_new), side="right").clip(0, 19)
    row_len = (keep + extra).sum(axis=1)
    bounds = np.concatenate([[0], np.cumsum(row_len)])
    return [vals[bounds[m] : bounds[m + 1]][:max_len] for m in range(size)]


def make_family_set(
    *,
    n_families: int,
    family_size: int,
    n_singletons: int = 0,
    mean_len: float,
    min_len: int,
    max_len: int,
    divergence: float,
    indel_rate: float = 0.02,
    indel_mean: float = 3.0,
    long_frac: float = 0.0,
    long_range=(5000, 35000),
    seed: int = 0,
    stream: int = 0,
    name: str = "custom",
) -> FamilySet:
    rng = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(stream,)))
    p = background_frequencies()
    p_cdf = np.cumsum(p)
    p_cdf[-1] = 1.0
    # rows shifted by their index so one sorted array serves every residue
    sub_cdf_flat = (_substitution_cdf(p) + np.arange(20)[:, None]).ravel()

    n_anc = n_families + n_singletons
    anc_lens = _draw_lengths(rng, n_anc, mean_len, min_len, max_len, long_frac, long_range)
    top = max(max_len, long_range[1] if long_frac > 0 else max_len)
    seqs = []
    labels = []
    for f in range(n_families):
        anc = np.searchsorted(p_cdf, rng.random(anc_lens[f]), side="right").clip(0, 19)
        seqs.extend(
            _mutate_family(rng, anc, family_size, divergence, indel_rate, indel_mean, sub_cdf_flat, p_cdf, top)
        )
        labels.extend([f] * family_size)
    for s in range(n_singletons):
        anc = np.searchsorted(p_cdf, rng.random(anc_lens[n_families + s]), side="right").clip(0, 19)
        seqs.append(anc)
        labels.append(-1)

    perm = rng.permutation(len(seqs))
    lens = np.array([seqs[i].size for i in perm], dtype=np.int64)
    offsets = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    codes = np.concatenate([seqs[i] for i in perm]) if seqs else np.zeros(0, np.int64)
    residues = _ASCII20[codes.astype(np.int64)].astype(np.uint8)
    meta = dict(
        name=name,
        n_families=n_families,
        family_size=family_size,
        n_singletons=n_singletons,
        mean_len=mean_len,
        min_len=min_len,
        max_len=max_len,
        divergence=divergence,
        indel_rate=indel_rate,
        indel_mean=indel_mean,
        long_frac=long_frac,
        long_range=list(long_range),
        length_sigma=0.6,
        seed=seed,
        stream=stream,
    )
    return FamilySet(residues, offsets, np.array(labels, dtype=np.int32)[perm], meta)


# The five workloads: sizes, length mixes and mutation rates; the method
# parameters that go with each live beside the callers (tests, bench).
WORKLOADS = {
    # 500 sequences, 25 families x 20, mean length 200 clamped to [50, 600].
    "tiny": dict(n_families=25, family_size=20, mean_len=200, min_len=50, max_len=600, divergence=0.30, stream=0),
    # 50,000 sequences, 2,000 families x 25, mean length 350 clamped to [30, 2000].
    "mid": dict(n_families=2000, family_size=25, mean_len=350, min_len=30, max_len=2000, divergence=0.30, stream=1),
    # 250,000 sequences: 10,000 families x 20 plus 50,000 singletons, clamp [30, 5000].
    "large": dict(
        n_families=10000, family_size=20, n_singletons=50000, mean_len=350, min_len=30, max_len=5000,
        divergence=0.30, stream=2,
    ),
    # 100,000 sequences, 4,000 families x 25: 95% lognormal(mean 300) ancestors,
    # 5% uniform in [5,000, 35,000]; 40% divergence.
    "heavy": dict(
        n_families=4000, family_size=25, mean_len=300, min_len=30, max_len=5000, divergence=0.40,
        long_frac=0.05, long_range=(5000, 35000), stream=4,
    ),
}


def workload(name: str, *, seed: int = 0, **overrides) -> FamilySet:
    """One of WORKLOADS, optionally scaled (e.g. ``n_families=40``)."""
    cfg = dict(WORKLOADS[name])
    cfg.update(overrides)
    return make_family_set(seed=seed, name=name, **cfg)


def pair_list(fs: FamilySet, *, random_per_seq: float = 10.0, seed: int = 0, stream: int = 100):
    """A seeded pair list over a family set: every within-family pair plus
    about ``random_per_seq * n`` uniformly random unrelated pairs (i < j).
    Input generation only (no k-mers, no scoring): it stands in for a
    candidate list when a stage is timed on its own."""
    rng = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(stream,)))
    lab = fs.labels
    order = np.argsort(lab, kind="stable")
    fam_pairs = []
    sl = lab[order]
    bounds = np.flatnonzero(np.diff(np.concatenate([[-2], sl, [-3]])))
    for s0, s1 in zip(bounds[:-1], bounds[1:]):
        if sl[s0] < 0 or s1 - s0 < 2:
            continue
        members = order[s0:s1]
        a, b = np.triu_indices(members.size, 1)
        fam_pairs.append(np.stack([members[a], members[b]], 1))
    fam = np.concatenate(fam_pairs) if fam_pairs else np.zeros((0, 2), np.int64)
    m = int(random_per_seq * fs.n)
    x = rng.integers(0, fs.n, m)
    y = rng.integers(0, fs.n, m)
    keep = (x != y) & ((lab[x] != lab[y]) | (lab[x] < 0))
    rnd = np.stack([x[keep], y[keep]], 1)
    allp = np.concatenate([fam, rnd])
    lo = np.minimum(allp[:, 0], allp[:, 1]).astype(np.uint32)
    hi = np.maximum(allp[:, 0], allp[:, 1]).astype(np.uint32)
    key = np.unique((lo.astype(np.uint64) << np.uint64(32)) | hi.astype(np.uint64))
    return (key >> np.uint64(32)).astype(np.uint32), (key & np.uint64(0xFFFFFFFF)).astype(np.uint32)
