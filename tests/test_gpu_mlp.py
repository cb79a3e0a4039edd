"""Parity of the learned pre-alignment filter's HIP kernels with the CPU
oracle (oracle/mlp.py): features, bf16 MFMA forward, gradients, an Adam
step, calibration, and the filtered search."""

import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _dev(x, gpu):
    import torch

    a = np.ascontiguousarray(x)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(gpu)


def _key(lo, hi):
    return (np.asarray(lo, np.uint64) << np.uint64(32)) | np.asarray(hi, np.uint64)


def _net(seed=0, scale_b=0.1):
    theta = M.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    p = M.unpack(theta)
    p["b1"] = rng.normal(0, scale_b, M.N_H)
    p["b2"] = rng.normal(0, scale_b, M.N_H)
    p["b3"] = np.array([0.2])
    return M.pack(p).astype(np.float32).astype(np.float64)


def _features(n, seed):
    """Seeded feature-like rows: counts, diagonals, log lengths, ratios, composition gaps."""
    rng = np.random.default_rng(seed)
    X = np.zeros((n, M.N_IN), np.float32)
    X[:, 0] = rng.integers(1, 40, n)
    X[:, 1] = rng.normal(0, 0.2, n)
    X[:, 2] = np.abs(rng.normal(0, 0.05, n))
    la = rng.lognormal(np.log(300), 0.5, n)
    lb = la * rng.uniform(1, 3, n)
    X[:, 3], X[:, 4], X[:, 5] = np.log(la), np.log(lb), la / lb
    X[:, 6:] = np.abs(rng.normal(0, 0.03, (n, 10)))
    return X


@pytest.mark.parametrize("n_subs,ck", [(0, 1), (25, 2)])
def test_features_match_oracle(gpu, orc, n_subs, ck):
    import paper_2009_14467_amd as P
    from synth import workload

    s = workload("tiny", n_families=12)
    codes = orc.encode(s.residues)
    c = orc.candidates(codes, s.offsets, 6, ck_min=ck, n_subs=n_subs)
    want = M.features(codes, s.offsets, c["lo"], c["hi"], c["count"], c["seed1"], c["seed2"])
    ctx = P.Context(P.Params(k=6, n_subs=n_subs, ck_min=ck))
    res, off = _dev(s.residues, gpu), _dev(s.offsets, gpu)
    nc = ctx.discover(res, off)
    assert nc == c["lo"].size
    g = ctx.candidates(nc)
    F = ctx.mlp_features(res, off, nc).cpu().numpy().astype(np.float64)
    kg = _key(g["lo"].cpu().numpy().view(np.uint32), g["hi"].cpu().numpy().view(np.uint32))
    kw = _key(c["lo"], c["hi"])
    F = F[np.argsort(kg)]
    want = want[np.argsort(kw)]
    # fp32 on the GPU: logs and quotients to a few float32 ulps
    np.testing.assert_allclose(F, want, rtol=4e-7, atol=1e-6)


@pytest.mark.parametrize("n", [1, 17, 1000, 70001])
def test_forward_matches_oracle(gpu, n):
    import paper_2009_14467_amd as P

    theta = _net(1)
    X = _features(n, seed=n)
    mean, std = X.mean(0), X.std(0) + 1e-3
    ctx = P.Context()
    ctx.mlp_set(theta, mean, std)
    y = ctx.mlp_forward(_dev(X, gpu)).cpu().numpy().astype(np.float64)
    want, _ = M.forward(theta, M.normalise(X, mean, std))
    rel = np.abs(y - want) / (1 + np.abs(want))
    # fp32 accumulation against fp64: float32 rounding almost everywhere; a
    # pre-activation within that rounding of a bf16 rounding boundary can
    # round to the neighbouring bf16 value, which moves the logit by up to a
    # few 1e-3 (a float32 model of the kernel's sums, in another order, does
    # so for 0.04% of 70,001 rows, by at most 3.9e-3)
    assert np.median(rel) <= 1e-6
    assert (rel > 1e-4).sum() <= max(1, 5e-3 * n), np.sort(rel)[-10:]
    assert rel.max() <= 1e-2, rel.max()


@pytest.mark.parametrize("n,pw", [(16, 1.0), (999, 3.0), (4096, 10.0), (65536, 2.0)])
def test_gradient_matches_oracle(gpu, n, pw):
    """One minibatch gradient, from 16 pairs to the largest batch (65,536
    pairs: 1,024 blocks of partial sums, 256 chunks of the weight-gradient
    reduction); the reductions run in a fixed order, so a second call gives
    the same bits."""
    import paper_2009_14467_amd as P

    theta = _net(2)
    X = _features(n, seed=7 + n)
    rng = np.random.default_rng(n)
    t = (rng.random(n) < 0.3).astype(np.uint8)
    mean, std = X.mean(0), X.std(0) + 1e-3
    ctx = P.Context()
    ctx.mlp_set(theta, mean, std)
    loss, g = ctx.mlp_grad(_dev(X, gpu), _dev(t, gpu), pos_weight=pw)
    loss2, g2 = ctx.mlp_grad(_dev(X, gpu), _dev(t, gpu), pos_weight=pw)
    assert loss2 == loss and g2.tobytes() == g.tobytes()
    wl, wg = M.backward(theta, M.normalise(X, mean, std), t, pw)
    assert loss == pytest.approx(wl, rel=1e-5)
    o = 0
    for name, shape in M.SHAPES:
        sz = int(np.prod(shape))
        a, b = g[o : o + sz].astype(np.float64), wg[o : o + sz]
        o += sz
        scale = max(np.abs(b).max(), 1e-12)
        assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b) + 1e-7 * scale, name
        assert (np.abs(a - b) <= 1e-2 * scale).all(), name


def test_adam_step_matches_oracle(gpu):
    import torch

    import paper_2009_14467_amd as P

    n = 2048
    theta = _net(3)
    X = _features(n, seed=3)
    t = (np.random.default_rng(3).random(n) < 0.5).astype(np.uint8)
    mean, std = X.mean(0), X.std(0) + 1e-3
    ctx = P.Context()
    ctx.mlp_set(theta, mean, std)
    order = torch.arange(n, dtype=torch.int32, device=gpu)
    ctx.mlp_train_epoch(_dev(X, gpu), _dev(t, gpu), order, batch=n, lr=1e-3)
    got = ctx.mlp_get()["params"].astype(np.float64)
    _, wg = M.backward(theta, M.normalise(X, mean, std), t, 1.0)
    want = M.Adam(M.N_PARAMS, lr=1e-3).step(theta, wg)
    # the first Adam step moves each weight by lr * g / (|g| + eps): compare
    # where the gradient is well above float32 noise
    big = np.abs(wg) > 1e-4 * np.abs(wg).max()
    assert big.mean() > 0.3
    np.testing.assert_allclose(got[big], want[big], rtol=0, atol=2e-5)
    # no step exceeds lr (plus the float32 rounding of the stored weight)
    assert (np.abs(got - theta) <= 1e-3 + 2e-7).all()


def test_training_learns_and_calibration_holds_recall(gpu):
    import torch

    import paper_2009_14467_amd as P

    n = 20000
    X = _features(n, seed=21)
    t = ((X[:, 5] > 0.55) & (X[:, 0] > 8)).astype(np.uint8)
    ctx = P.Context()
    ctx.mlp_set(M.init_params(4), np.zeros(16), np.ones(16))
    Xd, td = _dev(X, gpu), _dev(t, gpu)
    ctx.mlp_fit_normalizer(Xd)
    net = ctx.mlp_get()
    np.testing.assert_allclose(net["mean"], X.astype(np.float64).mean(0), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(net["std"], X.astype(np.float64).std(0), rtol=1e-4)
    g = torch.Generator().manual_seed(0)
    losses = []
    for ep in range(15):
        order = torch.randperm(n, generator=g).to(torch.int32).to(gpu)
        losses.append(ctx.mlp_train_epoch(Xd, td, order, batch=1024, lr=2e-3, pos_weight=2.0))
    assert losses[-1] < 0.5 * losses[0]
    tau = ctx.mlp_calibrate(Xd, td, 0.99)
    y = ctx.mlp_forward(Xd).cpu().numpy()
    recall = (y[t == 1] >= tau).mean()
    assert recall >= 0.99
    assert (y[t == 0] >= tau).mean() < 0.3  # it does discriminate
    assert ctx.mlp_get()["tau"] == tau


def test_filtered_search_aligns_exactly_the_kept_pairs(gpu):
    import paper_2009_14467_amd as P
    from synth import workload

    s = workload("tiny")
    res, off = _dev(s.residues, gpu), _dev(s.offsets, gpu)
    plain = P.Context(P.Params(k=6, ck_min=1))
    want = plain.search(res, off)
    nc = plain.discover(res, off)
    c = plain.candidates(nc)
    F = plain.mlp_features(res, off, nc)

    ctx = P.Context(P.Params(k=6, ck_min=1, filter_mode="mlp"))
    theta = _net(5)
    Fh = F.cpu().numpy()
    ctx.mlp_set(theta, Fh.mean(0), Fh.std(0) + 1e-3, tau=-np.inf)
    got = ctx.search(res, off)  # keeps everything
    from test_gpu_search import _compare_edges

    _compare_edges(got, want)
    y = ctx.mlp_forward(F).cpu().numpy()
    tau = float(np.median(y))
    ctx.mlp_set(theta, Fh.mean(0), Fh.std(0) + 1e-3, tau=tau)
    got = ctx.search(res, off)
    st = ctx.stats()
    keep = y >= tau
    assert st["n_candidates"] == nc and st["n_aligned"] == int(keep.sum())
    kept = set(_key(c["lo"].cpu().numpy().view(np.uint32)[keep], c["hi"].cpu().numpy().view(np.uint32)[keep]))
    sel = np.array([k in kept for k in _key(want["i"], want["j"])], bool)
    _compare_edges(got, want[sel])


def test_filter_needs_a_network(gpu):
    import paper_2009_14467_amd as P
    from synth import workload

    s = workload("tiny", n_families=3)
    ctx = P.Context(P.Params(k=6, ck_min=1, filter_mode="mlp"))
    with pytest.raises(P.PastisError, match="network"):
        ctx.search(_dev(s.residues, gpu), _dev(s.offsets, gpu))


def test_trained_filter_keeps_recall_and_skips_work(gpu):
    """End to end: train inside the library on one sequence set (labels from
    exact alignment; candidates of substitute and of exact k-mers), filter
    another one from the same recipe; the filtered search finds at least 99%
    of the exact edges while aligning a small share of the candidates, and
    its edges are a subset of the exact ones, bit for bit."""
    import paper_2009_14467_amd as P
    from paper_2009_14467_amd import learned_filter as LF
    from synth import workload

    params = dict(k=6, n_subs=25, ck_min=2)
    tr = workload("mid", n_families=240, seed=1)
    te = workload("mid", n_families=120, seed=0)
    rt, ot = _dev(tr.residues, gpu), _dev(tr.offsets, gpu)
    tf = LF.train(P.Params(**params), sets=[(rt, ot, None), (rt, ot, P.Params(k=6, n_subs=0, ck_min=2))],
                  epochs=6, batch=1024)
    assert tf.heldout_recall >= 0.98
    res, off = _dev(te.residues, gpu), _dev(te.offsets, gpu)
    exact = P.Context(P.Params(**params)).search(res, off)
    ctx = P.Context(P.Params(filter_mode="mlp", **params))
    tf.install(ctx)
    got = ctx.search(res, off)
    st = ctx.stats()
    keys = lambda e: (e["i"].astype(np.uint64) << np.uint64(32)) | e["j"].astype(np.uint64)  # noqa: E731
    sel = np.isin(keys(exact), keys(got))
    assert sel.sum() == got.size  # a subset of the exact edges ...
    assert got.tobytes() == exact[sel].tobytes()  # ... with identical fields
    assert got.size >= 0.99 * exact.size
    assert st["n_aligned"] < 0.5 * st["n_candidates"]


def test_library_training_lifecycle_and_network_file(gpu, tmp_path):
    """Collection, training and calibration through the C ABI alone, then a
    save / load round trip of the network: the loaded network gives the same
    logits bit for bit; foreign or truncated files are refused and leave the
    network in place."""
    import paper_2009_14467_amd as P
    from synth import workload

    tr = workload("mid", n_families=60, seed=2)
    res, off = _dev(tr.residues, gpu), _dev(tr.offsets, gpu)
    ctx = P.Context(P.Params(k=6, n_subs=25, ck_min=2))
    with pytest.raises(P.PastisError, match="fewer than 64"):
        ctx.mlp_train()
    n1 = ctx.mlp_collect(res, off)
    plain = P.Context(P.Params(k=6, n_subs=25, ck_min=2))
    assert n1 == plain.discover(res, off) > 0
    n2 = ctx.mlp_collect(res, off, P.Params(k=6, n_subs=0, ck_min=2))
    assert n2 == P.Context(P.Params(k=6, n_subs=0, ck_min=2)).discover(res, off)
    assert ctx.mlp_pool_size() == n1 + n2
    rep = ctx.mlp_train(epochs=5, batch=512, seed=3, heldout=0.25)
    assert rep["n_examples"] == n1 + n2 and rep["epochs"] == 5
    assert rep["n_train"] == n1 + n2 - int(0.25 * (n1 + n2))
    assert 0 < rep["n_positive"] < rep["n_train"] and rep["pos_weight"] > 0
    assert rep["epoch_loss"][-1] < rep["epoch_loss"][0]
    assert rep["heldout_recall"] >= 0.95 and rep["heldout_kept"] < 0.9
    net = ctx.mlp_get()
    assert net["tau"] == rep["tau"]
    # labels are the exact pass/fail: the pool's positives equal the passing pairs
    with pytest.raises(P.PastisError):
        ctx.mlp_train(batch=24)  # not a multiple of 16
    path = str(tmp_path / "net.bin")
    ctx.mlp_save(path)
    other = P.Context(P.Params(k=6, n_subs=25, ck_min=2))
    other.mlp_load(path)
    got = other.mlp_get()
    for key in ("params", "mean", "std"):
        assert got[key].tobytes() == net[key].tobytes()
    assert got["tau"] == net["tau"]
    plain.discover(res, off)
    F = plain.mlp_features(res, off, n1)
    assert other.mlp_forward(F).cpu().numpy().tobytes() == ctx.mlp_forward(F).cpu().numpy().tobytes()
    raw = open(path, "rb").read()
    bad = tmp_path / "bad.bin"
    bad.write_bytes(raw[:-4])
    with pytest.raises(P.PastisError, match="not a network file"):
        other.mlp_load(str(bad))
    bad.write_bytes(b"XXXXXXXX" + raw[8:])
    with pytest.raises(P.PastisError, match="not a network file"):
        other.mlp_load(str(bad))
    with pytest.raises(P.PastisError, match="cannot read"):
        other.mlp_load(str(tmp_path / "missing.bin"))
    assert other.mlp_get()["params"].tobytes() == net["params"].tobytes()
    ctx.mlp_clear()
    assert ctx.mlp_pool_size() == 0
