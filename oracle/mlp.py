"""CPU oracle of the learned pre-alignment filter -- TEST INFRASTRUCTURE ONLY.

Not part of the paper: a small MLP scores each candidate pair from 16 cheap
features and pairs predicted to fail the identity/coverage cut (Section IV-F)
skip alignment.  Written in float64 numpy:

  features (16 per pair, a = the shorter sequence, lengths La <= Lb):
    f0      shared (substitute) k-mer count of the candidate
    f1      (pos_b - pos_a) / Lb of seed 1 (oriented positions)
    f2      |diag2 - diag1| / Lb, 0 without a second seed
    f3, f4  ln La, ln Lb
    f5      La / Lb
    f6..15  |comp_a[g] - comp_b[g]|, comp = fraction of residues in group g of
            {AG}{ST}{DE}{NQ}{KRH}{IV}{LM}{FYW}{C}{P}
  normalisation: z = (f - mean) / std (training statistics), cast to bf16.
  network: h1 = relu(W1 z + b1) -> bf16; h2 = relu(W2 h1 + b2) -> bf16;
           y = w3 . h2 + b3 (logit); weights bf16 copies of fp32 masters.
  loss: mean over the batch of pos_weight * t * softplus(-y) + (1 - t) * softplus(y).

bf16 casts round to nearest, ties to even.  Gradients follow the same cast
points: the weight gradients are products of bf16 activations and bf16
upstream gradients.
"""

from __future__ import annotations

import numpy as np

GROUPS = ["AG", "ST", "DE", "NQ", "KRH", "IV", "LM", "FYW", "C", "P"]
ALPHABET = "ARNDCQEGHILKMFPSTWYVBZX*"
N_IN, N_H = 16, 128
NO_SEED = 0xFFFFFFFF


def bf16(x) -> np.ndarray:
    """Round float64/float32 values to the nearest bfloat16 (ties to even),
    returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> np.uint64(16)) & np.uint64(1)) + np.uint64(0x7FFF)
    r = ((u + rounding) >> np.uint64(16)) << np.uint64(16)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def group_of_code() -> np.ndarray:
    """Residue code 0..23 -> group 0..9, or -1 outside the groups."""
    g = np.full(24, -1, np.int64)
    for gi, letters in enumerate(GROUPS):
        for ch in letters:
            g[ALPHABET.index(ch)] = gi
    return g


def composition(codes: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """[n, 10] fraction of each sequence's residues in each group (0 when empty)."""
    gmap = group_of_code()
    n = offsets.size - 1
    out = np.zeros((n, 10), np.float64)
    g = gmap[codes.astype(np.int64)]
    seq = np.repeat(np.arange(n), np.diff(offsets))
    ok = g >= 0
    np.add.at(out, (seq[ok], g[ok]), 1.0)
    L = np.diff(offsets).astype(np.float64)
    return out / np.maximum(L, 1.0)[:, None]


def features(codes, offsets, lo, hi, count, seed1, seed2) -> np.ndarray:
    """[N, 16] raw features of candidate pairs (lo < hi)."""
    lo = np.asarray(lo, np.int64)
    hi = np.asarray(hi, np.int64)
    L = np.diff(offsets).astype(np.int64)
    comp = composition(codes, offsets)
    Li, Lj = L[lo], L[hi]
    swap = ~((Li < Lj) | ((Li == Lj) & (lo < hi)))  # a = shorter, the first on a tie
    La = np.where(swap, Lj, Li).astype(np.float64)
    Lb = np.where(swap, Li, Lj).astype(np.float64)
    f = np.zeros((lo.size, N_IN), np.float64)
    f[:, 0] = np.asarray(count, np.float64)

    def diag(seed):
        seed = np.asarray(seed, np.uint64)
        p_lo = (seed >> np.uint64(16)).astype(np.int64)
        p_hi = (seed & np.uint64(0xFFFF)).astype(np.int64)
        pa = np.where(swap, p_hi, p_lo)
        pb = np.where(swap, p_lo, p_hi)
        return (pb - pa).astype(np.float64), seed != NO_SEED

    d1, h1 = diag(seed1)
    d2, h2 = diag(seed2)
    f[:, 1] = np.where(h1, d1 / Lb, 0.0)
    f[:, 2] = np.where(h1 & h2, np.abs(d2 - d1) / Lb, 0.0)
    f[:, 3] = np.log(La)
    f[:, 4] = np.log(Lb)
    f[:, 5] = La / Lb
    ca = np.where(swap[:, None], comp[hi], comp[lo])
    cb = np.where(swap[:, None], comp[lo], comp[hi])
    f[:, 6:16] = np.abs(ca - cb)
    return f


# flat parameter vector: W1 [128,16], b1 [128], W2 [128,128], b2 [128], w3 [128], b3 [1]
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("w3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[o : o + size], np.float64).reshape(shape)
        o += size
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], np.float64).ravel() for name, _ in SHAPES])


def init_params(seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.normal(0, np.sqrt(2.0 / N_IN), (N_H, N_IN)),
        "b1": np.zeros(N_H),
        "W2": rng.normal(0, np.sqrt(2.0 / N_H), (N_H, N_H)),
        "b2": np.zeros(N_H),
        "w3": rng.normal(0, np.sqrt(1.0 / N_H), N_H),
        "b3": np.zeros(1),
    }
    return pack(p)


def normalise(f, mean, std) -> np.ndarray:
    """z-score in float32 (as the GPU does), then the bf16 cast."""
    z = (np.asarray(f, np.float32) - np.asarray(mean, np.float32)) / np.asarray(std, np.float32)
    return bf16(z)


def _identity(x):
    return np.asarray(x, np.float64)


def forward(theta, z, cast=bf16):
    """Logits of normalised, bf16-valued inputs z [N, 16]; also the cache.

    cast is the rounding applied to weights and activations (bf16; the
    identity gives the exact float64 network the gradient pins use)."""
    p = {k: cast(v) for k, v in unpack(theta).items() if k not in ("b1", "b2", "b3")}
    q = unpack(theta)
    a1 = z @ p["W1"].T + q["b1"]
    h1 = cast(np.maximum(a1, 0.0))
    a2 = h1 @ p["W2"].T + q["b2"]
    h2 = cast(np.maximum(a2, 0.0))
    y = h2 @ p["w3"] + q["b3"][0]
    return y, dict(z=z, a1=a1, h1=h1, a2=a2, h2=h2, p=p)


def softplus(x):
    return np.logaddexp(0.0, x)


def loss(y, t, pos_weight: float) -> float:
    t = np.asarray(t, np.float64)
    return float(np.mean(pos_weight * t * softplus(-y) + (1.0 - t) * softplus(y)))


def backward(theta, z, t, pos_weight: float, cast=bf16):
    """Mean weighted BCE and its gradient with respect to the fp32 masters.

    dL/dy = (pos_weight * t * (sigmoid(y) - 1) + (1 - t) * sigmoid(y)) / N;
    the upstream gradients entering a weight product are cast to bf16 like
    the activations they multiply."""
    y, c = forward(theta, z, cast)
    t = np.asarray(t, np.float64)
    n = y.size
    s = 1.0 / (1.0 + np.exp(-y))
    dy = (pos_weight * t * (s - 1.0) + (1.0 - t) * s) / n
    p = c["p"]
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(dy, p["w3"]) * (c["a2"] > 0)
    dh2b = cast(dh2)
    g["W2"] = dh2b.T @ c["h1"]
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2b @ p["W2"]) * (c["a1"] > 0)
    dh1b = cast(dh1)
    g["W1"] = dh1b.T @ c["z"]
    g["b1"] = dh1.sum(axis=0)
    return loss(y, t, pos_weight), pack(g)


class Adam:
    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, grad):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad
        self.v = self.b2 * self.v + (1 - self.b2) * grad * grad
        mh = self.m / (1 - self.b1**self.t)
        vh = self.v / (1 - self.b2**self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)
