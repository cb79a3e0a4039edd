"""Training driver of the learned pre-alignment filter.

Labels come from the exact pipeline: every candidate pair of a training set
is aligned and its pass/fail under the identity/coverage cut (Section IV-F)
is the target.  Feature extraction, the forward/backward passes, the Adam
steps and the threshold calibration all run in the HIP library; this module
only sequences the calls (epochs, shuffles, the train/held-out split).
"""

from __future__ import annotations

import dataclasses
import time

import numpy as np

from ._binding import MLP_FEATURES, MLP_PARAMS, RECORD_DTYPE, Context, Params

_PASSED_WORD = list(RECORD_DTYPE.names).index("passed")  # int32 word of the record


@dataclasses.dataclass
class TrainedFilter:
    params: np.ndarray
    mean: np.ndarray
    std: np.ndarray
    tau: float
    n_examples: int
    positive_frac: float
    heldout_recall: float
    heldout_kept_frac: float
    losses: list
    seconds: float

    def install(self, ctx: Context):
        ctx.mlp_set(self.params, self.mean, self.std, self.tau)


def labelled_candidates(ctx: Context, residues, offsets):
    """(features [n, 16], labels [n] uint8) of every candidate the discovery
    of ctx's parameters finds, labelled by aligning them exactly."""
    import torch

    nc = ctx.discover(residues, offsets)
    c = ctx.candidates(nc)
    X = ctx.mlp_features(residues, offsets, nc)
    rec = ctx.align_pairs(residues, offsets, c["lo"], c["hi"], c["seed1"], c["seed2"])
    words = rec.view(torch.int32).view(nc, RECORD_DTYPE.itemsize // 4)
    labels = words[:, _PASSED_WORD].to(torch.uint8).contiguous()
    return X, labels


def initial_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, in the flat PASTIS_MLP_PARAMS layout
    (W1 [128][16], b1, W2 [128][128], b2, w3 [128], b3)."""
    rng = np.random.default_rng(seed)
    h, f = 128, MLP_FEATURES
    parts = [rng.normal(0, np.sqrt(2.0 / f), h * f), np.zeros(h), rng.normal(0, np.sqrt(2.0 / h), h * h),
             np.zeros(h), rng.normal(0, np.sqrt(1.0 / h), h), np.zeros(1)]
    out = np.concatenate(parts).astype(np.float32)
    assert out.size == MLP_PARAMS
    return out


def train(params: Params, residues, offsets, epochs: int = 4, batch: int = 8192, lr: float = 2e-3,
          pos_weight: float | None = None, target_recall: float = 0.995, heldout: float = 0.2, seed: int = 0,
          device: int = 0) -> TrainedFilter:
    """Train a filter on the candidates of one sequence set (device tensors)
    and calibrate its threshold on a held-out fraction of them.  The
    positive class weight defaults to the negative / positive ratio."""
    import torch

    t0 = time.perf_counter()
    ctx = Context(dataclasses.replace(params, filter_mode="none"), device)
    X, y = labelled_candidates(ctx, residues, offsets)
    n = X.shape[0]
    if n < 32:
        raise ValueError("too few candidates to train on")
    gen = torch.Generator().manual_seed(seed)
    perm = torch.randperm(n, generator=gen).to(torch.int32)
    n_hold = max(16, int(heldout * n))
    hold = perm[:n_hold].to(X.device, torch.int64)
    train_idx = perm[n_hold:]
    if pos_weight is None:
        n_pos = max(int(y.sum()), 1)
        pos_weight = float(n - n_pos) / n_pos
    ctx.mlp_set(initial_params(seed), np.zeros(MLP_FEATURES), np.ones(MLP_FEATURES), 0.0)
    ctx.mlp_fit_normalizer(X[train_idx.to(X.device, torch.int64)].contiguous())
    losses = []
    for _ in range(epochs):
        order = train_idx[torch.randperm(train_idx.numel(), generator=gen)].to(X.device)
        losses.append(ctx.mlp_train_epoch(X, y, order, batch=batch, lr=lr, pos_weight=pos_weight))
    # the threshold comes from one half of the held-out pairs, the reported
    # recall and kept fraction from the other half
    cal, test = hold[: n_hold // 2], hold[n_hold // 2 :]
    tau = ctx.mlp_calibrate(X[cal].contiguous(), y[cal].contiguous(), target_recall)
    Xh, yh = X[test].contiguous(), y[test].contiguous()
    logit = ctx.mlp_forward(Xh)
    pos = yh.bool()
    recall = float((logit[pos] >= tau).float().mean()) if bool(pos.any()) else 1.0
    kept = float((logit >= tau).float().mean())
    net = ctx.mlp_get()
    torch.cuda.synchronize()
    return TrainedFilter(net["params"], net["mean"], net["std"], net["tau"], int(n), float(y.float().mean()),
                         recall, kept, losses, time.perf_counter() - t0)
