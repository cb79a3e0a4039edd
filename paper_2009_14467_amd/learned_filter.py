"""Training of the learned pre-alignment filter, through the library's calls.

Labels come from the exact pipeline: every candidate pair of a training set
is aligned and its pass/fail under the identity/coverage cut (Section IV-F)
is the target.  Collection (pastis_mlp_collect), the split, the positive
class weight, the epochs and the threshold calibration (pastis_mlp_train)
all run in the HIP library; this module only names the sequence sets.
"""

from __future__ import annotations

import dataclasses
import time

import numpy as np

from ._binding import Context, Params


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
    report: dict

    def install(self, ctx: Context):
        ctx.mlp_set(self.params, self.mean, self.std, self.tau)


def train(params: Params, residues=None, offsets=None, *, sets=None, epochs: int = 4, batch: int = 8192,
          lr: float = 2e-3, pos_weight: float = 0.0, target_recall: float = 0.995, heldout: float = 0.2,
          seed: int = 0, device: int = 0) -> TrainedFilter:
    """Train a filter on the candidates of one or more sequence sets (device
    tensors) and calibrate its threshold on a held-out share of them.

    sets: list of (residues, offsets, discovery) where discovery (Params or
    None) overrides the k-mer parameters of that set's collection; without
    it the one set (residues, offsets) is collected with `params`.
    pos_weight <= 0 takes the negative / positive ratio of the training share."""
    t0 = time.perf_counter()
    ctx = Context(dataclasses.replace(params, filter_mode="none", graph_mode=False), device)
    if sets is None:
        sets = [(residues, offsets, None)]
    for res, off, disc in sets:
        ctx.mlp_collect(res, off, disc)
    rep = ctx.mlp_train(epochs=epochs, batch=batch, lr=lr, pos_weight=pos_weight, target_recall=target_recall,
                        heldout=heldout, seed=seed)
    net = ctx.mlp_get()
    return TrainedFilter(net["params"], net["mean"], net["std"], net["tau"], int(rep["n_examples"]),
                         rep["n_positive"] / max(rep["n_train"], 1), rep["heldout_recall"], rep["heldout_kept"],
                         rep["epoch_loss"], time.perf_counter() - t0, rep)
