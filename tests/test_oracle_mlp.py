"""Pins of the CPU oracle of the learned pre-alignment filter (oracle/mlp.py).

The filter is not part of the paper; its oracle is pinned against a library
bfloat16 conversion, hand-computed features, closed forms of the loss and of
Adam, and central finite differences of the exact (cast-free) network."""

import numpy as np
import pytest

from oracle import mlp as M


def exact(x):
    return np.asarray(x, np.float64)


def test_bf16_hand_values():
    one = 1.0
    assert M.bf16(one)[()] == 1.0
    assert M.bf16(1.0 + 2.0**-8)[()] == 1.0  # halfway, even neighbour is 1.0
    assert M.bf16(1.0 + 3 * 2.0**-8)[()] == 1.0 + 2.0**-6  # halfway, even neighbour is the upper one
    assert M.bf16(1.0 + 2.0**-8 + 2.0**-20)[()] == 1.0 + 2.0**-7  # just above halfway
    assert M.bf16(-3.0)[()] == -3.0
    assert M.bf16(0.0)[()] == 0.0
    assert M.bf16(3.0e38)[()] == 226 / 128 * 2.0**127  # 3e38 = 1.7633 * 2^127; 7 mantissa bits


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1, 50000), rng.normal(0, 1e-30, 1000), rng.normal(0, 1e30, 1000),
                        rng.uniform(-4, 4, 50000)]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), want)


def _fs(seqs):
    lens = np.array([len(s) for s in seqs])
    off = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    codes = np.array([M.ALPHABET.index(ch) for ch in "".join(seqs)], np.uint8)
    return codes, off


def test_features_hand_example():
    codes, off = _fs(["ACDE", "AAGGKP", "WWXX"])
    NO = M.NO_SEED
    f = M.features(codes, off, lo=[0, 0], hi=[1, 2], count=[3, 1], seed1=[(1 << 16) | 3, NO],
                   seed2=[(0 << 16) | 0, NO])
    # pair (0, 1): a = "ACDE" (4), b = "AAGGKP" (6); seed diagonals 2 and 0
    want = [3, 2 / 6, 2 / 6, np.log(4), np.log(6), 4 / 6,
            abs(0.25 - 4 / 6), 0, 0.5, 0, 1 / 6, 0, 0, 0, 0.25, 1 / 6]
    np.testing.assert_allclose(f[0], want, rtol=0, atol=1e-15)
    # pair (0, 2): equal lengths, a = the first; no seeds; X is in no group
    want = [1, 0, 0, np.log(4), np.log(4), 1, 0.25, 0, 0.5, 0, 0, 0, 0, 0.5, 0.25, 0]
    np.testing.assert_allclose(f[1], want, rtol=0, atol=1e-15)


def test_features_orient_the_shorter_sequence_first():
    codes, off = _fs(["AAGGKP", "ACDE"])
    # the same pair as the hand example with the longer sequence first: the
    # seed key holds (position in sequence 0) << 16 | (position in sequence 1)
    f = M.features(codes, off, lo=[0], hi=[1], count=[3], seed1=[(3 << 16) | 1], seed2=[(0 << 16) | 0])
    codes2, off2 = _fs(["ACDE", "AAGGKP"])
    g = M.features(codes2, off2, lo=[0], hi=[1], count=[3], seed1=[(1 << 16) | 3], seed2=[0])
    np.testing.assert_allclose(f, g, rtol=0, atol=1e-15)


def test_loss_closed_forms():
    t = np.array([1, 0, 1, 0, 0])
    assert M.loss(np.zeros(5), t, 3.0) == pytest.approx((3 * 2 + 3) / 5 * np.log(2.0), rel=1e-15)
    # confident and right: ~0; confident and wrong: ~|y| per example
    assert M.loss(np.array([50.0, -50.0]), np.array([1, 0]), 1.0) < 1e-20
    assert M.loss(np.array([-800.0]), np.array([1]), 2.0) == pytest.approx(1600.0, rel=1e-12)


def _rand_case(n=12, seed=0):
    rng = np.random.default_rng(seed)
    theta = M.init_params(seed)
    theta[M.N_PARAMS - 1] = 0.3
    z = rng.normal(0, 1, (n, M.N_IN))
    t = (rng.random(n) < 0.4).astype(np.float64)
    return theta, z, t


def test_gradient_matches_finite_differences_of_exact_network():
    theta, z, t = _rand_case()
    _, g = M.backward(theta, z, t, 2.5, cast=exact)
    rng = np.random.default_rng(1)
    sizes = [int(np.prod(s)) for _, s in M.SHAPES]
    starts = np.cumsum([0] + sizes[:-1])
    idx = np.concatenate([s + rng.choice(n, min(n, 12), replace=False) for s, n in zip(starts, sizes)])
    h = 1e-6
    for q in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[q] += h
        tm[q] -= h
        fd = (M.loss(M.forward(tp, z, exact)[0], t, 2.5) - M.loss(M.forward(tm, z, exact)[0], t, 2.5)) / (2 * h)
        assert abs(g[q] - fd) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (q, g[q], fd)


def test_bf16_gradient_is_close_to_exact():
    """The bf16 cast points move each gradient block by a few bf16 ulps
    (2^-8 relative) compounded over three casts and ReLU masks: well under 10%."""
    theta, z, t = _rand_case(n=64, seed=5)
    zb = M.bf16(z)
    _, ge = M.backward(theta, zb, t, 1.0, cast=exact)
    _, gb = M.backward(theta, zb, t, 1.0)
    for name, sl in zip([n for n, _ in M.SHAPES], np.split(np.arange(M.N_PARAMS), np.cumsum(
            [int(np.prod(s)) for _, s in M.SHAPES])[:-1])):
        err = np.linalg.norm(gb[sl] - ge[sl]) / max(np.linalg.norm(ge[sl]), 1e-30)
        assert err < 0.1, (name, err)


def test_adam_closed_forms():
    opt = M.Adam(3, lr=0.01)
    th = np.array([1.0, 2.0, 3.0])
    g = np.array([0.5, -2.0, 0.0])
    th1 = opt.step(th, g)
    # first step: m^ = g, v^ = g^2, so the update is lr * g / (|g| + eps)
    np.testing.assert_allclose(th1, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps m^ = g and v^ = g^2 at every step
    th2 = opt.step(th1, g)
    np.testing.assert_allclose(th2, th1 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_training_separates_a_linear_rule():
    rng = np.random.default_rng(11)
    X = rng.normal(0, 1, (2048, M.N_IN))
    t = (X[:, 0] + 0.5 * X[:, 3] > 0.2).astype(np.float64)
    mean, std = X.mean(0), X.std(0)
    z = M.normalise(X, mean, std)
    theta = M.init_params(2)
    opt = M.Adam(M.N_PARAMS, lr=3e-3)
    for step in range(150):
        sel = rng.choice(X.shape[0], 256, replace=False)
        _, g = M.backward(theta, z[sel], t[sel], 1.0)
        theta = opt.step(theta, g)
    y, _ = M.forward(theta, z)
    assert ((y > 0) == (t > 0)).mean() > 0.95
