"""ctypes binding of libpastis_hip.so (the C ABI in include/pastis.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  torch supplies device memory and the current stream.  There is no
fallback: if the library is missing this module raises.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpastis_hip.so")

OK = 0
STATUS_NAMES = {0: "OK", 1: "E_INVAL", 2: "E_BAD_RESIDUE", 3: "E_NOMEM", 4: "E_DEVICE", 5: "E_CAPACITY", 6: "E_STATE"}

RECORD_DTYPE = np.dtype(
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
assert RECORD_DTYPE.itemsize == 48

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


class PastisError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {detail}")
        self.status = status
        self.detail = detail


class _Params(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("n_subs", ctypes.c_int32),
        ("sub_alphabet", ctypes.c_int32),
        ("ck_min", ctypes.c_int32),
        ("align_mode", ctypes.c_int32),
        ("gap_open", ctypes.c_int32),
        ("gap_extend", ctypes.c_int32),
        ("xdrop", ctypes.c_int32),
        ("min_identity_pct", ctypes.c_int32),
        ("min_coverage_pct", ctypes.c_int32),
        ("weight_mode", ctypes.c_int32),
        ("score_width", ctypes.c_int32),
        ("full_records", ctypes.c_int32),
        ("filter_mode", ctypes.c_int32),
        ("graph_mode", ctypes.c_int32),
        ("candidate_room", ctypes.c_int32),
        ("block_entries", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


class _Tuning(ctypes.Structure):
    _fields_ = [
        ("sw16_max_rows", ctypes.c_int32),
        ("sw_direct_pct", ctypes.c_int32),
        ("sw_grid_scale", ctypes.c_int32),
        ("sw_grid_scale_wide", ctypes.c_int32),
        ("sw_intra_pair", ctypes.c_int32),
        ("sw16_narrow_rows", ctypes.c_int32),
        ("sw_long_blocks", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 1),
    ]


class _TrainOpts(ctypes.Structure):
    _fields_ = [
        ("epochs", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("lr", ctypes.c_float),
        ("pos_weight", ctypes.c_float),
        ("target_recall", ctypes.c_double),
        ("heldout", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("reserved", ctypes.c_int32 * 4),
    ]


class _TrainReport(ctypes.Structure):
    _fields_ = [
        ("n_examples", ctypes.c_int64),
        ("n_train", ctypes.c_int64),
        ("n_positive", ctypes.c_int64),
        ("pos_weight", ctypes.c_float),
        ("tau", ctypes.c_float),
        ("heldout_recall", ctypes.c_double),
        ("heldout_kept", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("epochs", ctypes.c_int32),
        ("epoch_loss", ctypes.c_float * 32),
    ]


def _tuning_dict(t) -> dict:
    return {"sw16_max_rows": t.sw16_max_rows, "sw_direct_pct": t.sw_direct_pct, "sw_grid_scale": t.sw_grid_scale,
            "sw_grid_scale_wide": t.sw_grid_scale_wide, "sw_intra_pair": t.sw_intra_pair,
            "sw16_narrow_rows": t.sw16_narrow_rows, "sw_long_blocks": t.sw_long_blocks}


class _Stats(ctypes.Structure):
    _fields_ = [
        ("n_sequences", ctypes.c_int64),
        ("n_residues", ctypes.c_int64),
        ("n_kmers", ctypes.c_int64),
        ("n_candidates", ctypes.c_int64),
        ("n_aligned", ctypes.c_int64),
        ("n_edges", ctypes.c_int64),
        ("cells", ctypes.c_int64),
        ("stats_pass_pairs", ctypes.c_int64),
        ("int32_pairs", ctypes.c_int64),
        ("ms_total", ctypes.c_double),
        ("ms_stage", ctypes.c_double * 9),
        ("sw_bins", ctypes.c_int32),
        ("sw_bin_rows", ctypes.c_int32 * 32),
        ("sw_bin_multi", ctypes.c_int32 * 32),
        ("sw_bin_bits", ctypes.c_int32 * 32),
        ("sw_bin_pairs", ctypes.c_int64 * 32),
        ("sw_bin_cells", ctypes.c_int64 * 32),
        ("sw_bin_ms", ctypes.c_double * 32),
        ("bound_pass_pairs", ctypes.c_int64),
        ("bound_pass_cells", ctypes.c_int64),
        ("stats_pass_cells", ctypes.c_int64),
        ("sw_graph", ctypes.c_int32),
        ("sw_graph_pad", ctypes.c_int32),
        ("spgemm_products", ctypes.c_int64),
        ("n_subs_entries", ctypes.c_int64),
        ("n_row_blocks", ctypes.c_int64),
    ]


@dataclasses.dataclass
class Params:
    """Mirror of pastis_params; defaults are the paper's Section VI settings."""

    k: int = 6
    n_subs: int = 0
    sub_alphabet: int = 20
    ck_min: int = 1
    align_mode: str = "sw"  # "sw" | "xd"
    gap_open: int = 11
    gap_extend: int = 1
    xdrop: int = 49
    min_identity_pct: int = 30
    min_coverage_pct: int = 70
    weight_mode: str = "ani"  # "ani" | "ns"
    score_width: int = 0
    full_records: bool = False
    filter_mode: str = "none"  # "none" | "mlp" (the learned filter, set with Context.mlp_set)
    graph_mode: bool = False  # replay the alignment stage as a captured HIP graph
    candidate_room: int = 0  # initial room for directional candidates (0: automatic)
    block_entries: int = 0  # search: most directional entries per row block (0: the 32-bit limit)

    def to_c(self) -> _Params:
        p = _Params()
        p.k = self.k
        p.n_subs = self.n_subs
        p.sub_alphabet = self.sub_alphabet
        p.ck_min = self.ck_min
        p.align_mode = {"sw": 0, "xd": 1}[self.align_mode]
        p.gap_open = self.gap_open
        p.gap_extend = self.gap_extend
        p.xdrop = self.xdrop
        p.min_identity_pct = self.min_identity_pct
        p.min_coverage_pct = self.min_coverage_pct
        p.weight_mode = {"ani": 0, "ns": 1}[self.weight_mode]
        p.score_width = self.score_width
        p.full_records = int(self.full_records)
        p.filter_mode = {"none": 0, "mlp": 1}[self.filter_mode]
        p.graph_mode = int(self.graph_mode)
        p.candidate_room = self.candidate_room
        p.block_entries = self.block_entries
        return p


_lib = None

# (name, restype, argtypes) of every exported entry point
_VP = ctypes.c_void_p
_SIGNATURES = [
    ("pastis_default_params", None, [ctypes.POINTER(_Params)]),
    ("pastis_create", ctypes.c_int, [ctypes.POINTER(_Params), ctypes.c_int, ctypes.POINTER(_VP)]),
    ("pastis_destroy", None, [_VP]),
    ("pastis_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("pastis_last_error", ctypes.c_char_p, [_VP]),
    ("pastis_bad_residue_index", ctypes.c_int64, [_VP]),
    ("pastis_encode", ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int, _VP, _VP]),
    ("pastis_align_pairs", ctypes.c_int,
     [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int, _VP, _VP, _VP, _VP, ctypes.c_int64, _VP, _VP]),
    ("pastis_align_pairs_noalloc", ctypes.c_int,
     [_VP, _VP, _VP, ctypes.c_int64, _VP, _VP, _VP, _VP, ctypes.c_int64, _VP, _VP]),
    ("pastis_stats", ctypes.c_int, [_VP, ctypes.POINTER(_Stats)]),
    ("pastis_discover", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int, _VP, ctypes.POINTER(ctypes.c_int64)]),
    ("pastis_candidates_copy", ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_int, _VP]),
    ("pastis_subkmers", ctypes.c_int, [_VP, _VP, ctypes.c_int64, _VP, _VP, _VP, _VP]),
    ("pastis_search", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int, _VP, ctypes.POINTER(_VP)]),
    ("pastis_result_count", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64)]),
    ("pastis_result_device_ptr", _VP, [_VP]),
    ("pastis_result_copy", ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int, _VP]),
    ("pastis_result_free", None, [_VP]),
    ("pastis_mlp_features", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int, _VP, ctypes.c_int64, _VP]),
    ("pastis_mlp_set", ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_float]),
    ("pastis_mlp_get", ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_float)]),
    ("pastis_mlp_fit_normalizer", ctypes.c_int, [_VP, _VP, ctypes.c_int64, _VP]),
    ("pastis_mlp_forward", ctypes.c_int, [_VP, _VP, ctypes.c_int64, _VP, _VP]),
    ("pastis_mlp_grad", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_float, _VP, _VP, _VP]),
    ("pastis_mlp_train_epoch", ctypes.c_int,
     [_VP, _VP, _VP, ctypes.c_int64, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_float, _VP, _VP]),
    ("pastis_mlp_calibrate", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_double, _VP, _VP]),
    ("pastis_mlp_collect", ctypes.c_int,
     [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(_Params), _VP, ctypes.POINTER(ctypes.c_int64)]),
    ("pastis_mlp_clear", ctypes.c_int, [_VP]),
    ("pastis_mlp_pool_size", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64)]),
    ("pastis_mlp_default_train_opts", None, [ctypes.POINTER(_TrainOpts)]),
    ("pastis_mlp_train", ctypes.c_int, [_VP, ctypes.POINTER(_TrainOpts), _VP, ctypes.POINTER(_TrainReport)]),
    ("pastis_mlp_save", ctypes.c_int, [_VP, ctypes.c_char_p]),
    ("pastis_mlp_load", ctypes.c_int, [_VP, ctypes.c_char_p]),
    ("pastis_components", ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int64, _VP, _VP]),
    ("pastis_cluster_scores", ctypes.c_int,
     [_VP, _VP, _VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _VP]),
    ("pastis_get_tuning", ctypes.c_int, [_VP, ctypes.POINTER(_Tuning)]),
    ("pastis_set_tuning", ctypes.c_int, [_VP, ctypes.POINTER(_Tuning)]),
    ("pastis_autotune", ctypes.c_int,
     [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int, ctypes.c_int64, _VP, ctypes.POINTER(_Tuning)]),
]

MLP_FEATURES = 16
MLP_PARAMS = 18817


def lib():
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first (python -c "
                "'import __graft_entry__; __graft_entry__.build()')"
            )
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return [name for name, _, _ in _SIGNATURES]


def _torch():
    import torch

    return torch


def _dev_ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream_ptr(stream) -> int | None:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Context:
    """A pastis_ctx bound to one GPU.  Not thread-safe."""

    def __init__(self, params: Params | None = None, device: int = 0):
        self.params = params or Params()
        self.device = device
        self._ctx = _VP()
        self._cp = self.params.to_c()
        st = lib().pastis_create(ctypes.byref(self._cp), device, ctypes.byref(self._ctx))
        if st != OK:
            raise PastisError(st, "pastis_create failed (bad parameters or device)")

    def close(self):
        if self._ctx:
            lib().pastis_destroy(self._ctx)
            self._ctx = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != OK:
            detail = lib().pastis_last_error(self._ctx) or b""
            raise PastisError(st, detail.decode(errors="replace"))

    @property
    def bad_residue_index(self) -> int:
        return int(lib().pastis_bad_residue_index(self._ctx))

    def stats(self) -> dict:
        s = _Stats()
        self._check(lib().pastis_stats(self._ctx, ctypes.byref(s)))
        arrays = ("ms_stage", "sw_bin_rows", "sw_bin_multi", "sw_bin_bits", "sw_bin_pairs", "sw_bin_cells",
                  "sw_bin_ms")
        out = {f: getattr(s, f) for f, _ in _Stats._fields_ if f not in arrays}
        out["ms_stage"] = list(s.ms_stage)
        nb = s.sw_bins
        out["sw_bins"] = [
            {"rows_per_lane": s.sw_bin_rows[b], "multi_strip": bool(s.sw_bin_multi[b]), "bits": s.sw_bin_bits[b],
             "pairs": s.sw_bin_pairs[b],
             "cells": s.sw_bin_cells[b], "ms": s.sw_bin_ms[b]}
            for b in range(nb)
        ]
        return out

    def encode(self, residues, stream=None):
        """residues: uint8 torch tensor (device or host) -> device codes tensor."""
        torch = _torch()
        on_dev = int(residues.is_cuda)
        codes = torch.empty(residues.numel(), dtype=torch.uint8, device=f"cuda:{self.device}")
        self._check(lib().pastis_encode(self._ctx, _dev_ptr(residues), residues.numel(), on_dev,
                                        _dev_ptr(codes), _stream_ptr(stream)))
        return codes

    def align_pairs(self, residues, offsets, pi, pj, seed1=None, seed2=None, stream=None):
        """Align pairs (pi[q], pj[q]); returns a device uint8 tensor of npairs
        48-byte pastis_pair_record entries (view with RECORD_DTYPE on the host)."""
        torch = _torch()
        n = offsets.numel() - 1
        npairs = pi.numel()
        on_dev = int(residues.is_cuda)
        if on_dev != int(offsets.is_cuda):
            raise ValueError("residues and offsets must both be on the device or both on the host")
        out = torch.empty(max(npairs, 1) * RECORD_DTYPE.itemsize, dtype=torch.uint8, device=f"cuda:{self.device}")
        self._check(lib().pastis_align_pairs(self._ctx, _dev_ptr(residues), _dev_ptr(offsets), n, on_dev,
                                             _dev_ptr(pi), _dev_ptr(pj), _dev_ptr(seed1), _dev_ptr(seed2), npairs,
                                             _dev_ptr(out), _stream_ptr(stream)))
        return out[: npairs * RECORD_DTYPE.itemsize]


    def discover(self, residues, offsets, stream=None) -> int:
        """Candidate discovery; returns the number of candidates (kept in ctx)."""
        n = offsets.numel() - 1
        on_dev = int(residues.is_cuda)
        nc = ctypes.c_int64(0)
        self._check(lib().pastis_discover(self._ctx, _dev_ptr(residues), _dev_ptr(offsets), n, on_dev,
                                          _stream_ptr(stream), ctypes.byref(nc)))
        return int(nc.value)

    def candidates(self, n_candidates: int, stream=None) -> dict:
        """Device tensors (int32 views of uint32) of the last discovery's candidates."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        out = {k: torch.empty(max(n_candidates, 1), dtype=torch.int32, device=dev)
               for k in ("lo", "hi", "count", "seed1", "seed2")}
        self._check(lib().pastis_candidates_copy(self._ctx, *(_dev_ptr(out[k]) for k in
                                                            ("lo", "hi", "count", "seed1", "seed2")),
                                                 n_candidates, 1, _stream_ptr(stream)))
        return {k: v[:n_candidates] for k, v in out.items()}

    def subkmers(self, kmer_ids, stream=None):
        """kmer_ids: int64 device tensor of radix-24 ids -> (ids [n, m] int64, dist [n, m], count [n])."""
        torch = _torch()
        if kmer_ids.dtype != torch.int64:
            raise ValueError("k-mer ids are 64-bit")
        n = kmer_ids.numel()
        m = self.params.n_subs
        dev = f"cuda:{self.device}"
        ids = torch.empty((max(n, 1), m), dtype=torch.int64, device=dev)
        dist = torch.empty((max(n, 1), m), dtype=torch.int32, device=dev)
        cnt = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        self._check(lib().pastis_subkmers(self._ctx, _dev_ptr(kmer_ids), n, _dev_ptr(ids), _dev_ptr(dist),
                                          _dev_ptr(cnt), _stream_ptr(stream)))
        return ids[:n], dist[:n], cnt[:n]

    def search(self, residues, offsets, stream=None) -> np.ndarray:
        """Sequences in, edges out (host numpy array of EDGE_DTYPE)."""
        n = offsets.numel() - 1
        on_dev = int(residues.is_cuda)
        res = _VP()
        self._check(lib().pastis_search(self._ctx, _dev_ptr(residues), _dev_ptr(offsets), n, on_dev,
                                        _stream_ptr(stream), ctypes.byref(res)))
        try:
            ne = ctypes.c_int64(0)
            self._check(lib().pastis_result_count(res, ctypes.byref(ne)))
            out = np.zeros(ne.value, dtype=EDGE_DTYPE)
            if ne.value:
                self._check(lib().pastis_result_copy(res, out.ctypes.data, ne.value, 0, _stream_ptr(stream)))
            return out
        finally:
            lib().pastis_result_free(res)

    # ---- schedule of the alignment stage ----

    def get_tuning(self) -> dict:
        t = _Tuning()
        self._check(lib().pastis_get_tuning(self._ctx, ctypes.byref(t)))
        return _tuning_dict(t)

    def set_tuning(self, sw16_max_rows: int = 16, sw_direct_pct: int = 50, sw_grid_scale: int = 1,
                   sw_grid_scale_wide: int = 1, sw_intra_pair: int = 0, sw16_narrow_rows: int = 4,
                   sw_long_blocks: int = 4):
        t = _Tuning()
        t.sw16_max_rows, t.sw_direct_pct = sw16_max_rows, sw_direct_pct
        t.sw_grid_scale, t.sw_grid_scale_wide = sw_grid_scale, sw_grid_scale_wide
        t.sw_intra_pair, t.sw16_narrow_rows = sw_intra_pair, sw16_narrow_rows
        t.sw_long_blocks = sw_long_blocks
        self._check(lib().pastis_set_tuning(self._ctx, ctypes.byref(t)))

    def autotune(self, residues, offsets, max_pairs: int = 1 << 21, stream=None) -> dict:
        """Time schedule settings on a sample of these sequences' candidates and keep the fastest."""
        t = _Tuning()
        n = offsets.numel() - 1
        self._check(lib().pastis_autotune(self._ctx, _dev_ptr(residues), _dev_ptr(offsets), n, int(residues.is_cuda),
                                          int(max_pairs), _stream_ptr(stream), ctypes.byref(t)))
        return _tuning_dict(t)

    # ---- learned pre-alignment filter ----

    def mlp_features(self, residues, offsets, n_candidates: int, stream=None):
        """Raw features [n_candidates, 16] (device fp32) of the last discovery's candidates."""
        torch = _torch()
        n = offsets.numel() - 1
        out = torch.empty((max(n_candidates, 1), MLP_FEATURES), dtype=torch.float32, device=f"cuda:{self.device}")
        self._check(lib().pastis_mlp_features(self._ctx, _dev_ptr(residues), _dev_ptr(offsets), n,
                                              int(residues.is_cuda), _dev_ptr(out), n_candidates,
                                              _stream_ptr(stream)))
        return out[:n_candidates]

    def mlp_set(self, params, mean, std, tau: float = 0.0):
        """Install a network (host arrays, fp32): params [MLP_PARAMS], mean / std [16]."""
        th = np.ascontiguousarray(params, np.float32)
        mu = np.ascontiguousarray(mean, np.float32)
        sd = np.ascontiguousarray(std, np.float32)
        if th.size != MLP_PARAMS or mu.size != MLP_FEATURES or sd.size != MLP_FEATURES:
            raise ValueError("network arrays have the wrong size")
        self._check(lib().pastis_mlp_set(self._ctx, th.ctypes.data, mu.ctypes.data, sd.ctypes.data, float(tau)))

    def mlp_get(self) -> dict:
        th = np.zeros(MLP_PARAMS, np.float32)
        mu = np.zeros(MLP_FEATURES, np.float32)
        sd = np.zeros(MLP_FEATURES, np.float32)
        tau = ctypes.c_float(0.0)
        self._check(lib().pastis_mlp_get(self._ctx, th.ctypes.data, mu.ctypes.data, sd.ctypes.data,
                                         ctypes.byref(tau)))
        return {"params": th, "mean": mu, "std": sd, "tau": float(tau.value)}

    def mlp_fit_normalizer(self, X, stream=None):
        self._check(lib().pastis_mlp_fit_normalizer(self._ctx, _dev_ptr(X), X.shape[0], _stream_ptr(stream)))

    def mlp_forward(self, X, stream=None):
        """Logits [n] (device fp32) of raw features X [n, 16] (device fp32)."""
        torch = _torch()
        out = torch.empty(max(X.shape[0], 1), dtype=torch.float32, device=f"cuda:{self.device}")
        self._check(lib().pastis_mlp_forward(self._ctx, _dev_ptr(X), X.shape[0], _dev_ptr(out),
                                             _stream_ptr(stream)))
        return out[: X.shape[0]]

    def mlp_grad(self, X, labels, pos_weight: float = 1.0, stream=None):
        """(loss, gradient [MLP_PARAMS]) of the weighted BCE over X / labels (device)."""
        g = np.zeros(MLP_PARAMS, np.float32)
        loss = np.zeros(1, np.float32)
        self._check(lib().pastis_mlp_grad(self._ctx, _dev_ptr(X), _dev_ptr(labels), X.shape[0], float(pos_weight),
                                          g.ctypes.data, loss.ctypes.data, _stream_ptr(stream)))
        return float(loss[0]), g

    def mlp_train_epoch(self, X, labels, order, batch: int = 4096, lr: float = 1e-3, pos_weight: float = 1.0,
                        stream=None) -> float:
        """One Adam pass over order (device int32 example indices); returns the mean batch loss."""
        loss = np.zeros(1, np.float32)
        self._check(lib().pastis_mlp_train_epoch(self._ctx, _dev_ptr(X), _dev_ptr(labels), X.shape[0],
                                                 _dev_ptr(order), order.numel(), int(batch), float(lr), float(pos_weight),
                                                 loss.ctypes.data, _stream_ptr(stream)))
        return float(loss[0])

    def mlp_calibrate(self, X, labels, target_recall: float, stream=None) -> float:
        """Set (and return) the logit threshold keeping >= target_recall of the positives."""
        tau = np.zeros(1, np.float32)
        self._check(lib().pastis_mlp_calibrate(self._ctx, _dev_ptr(X), _dev_ptr(labels), X.shape[0],
                                               float(target_recall), tau.ctypes.data, _stream_ptr(stream)))
        return float(tau[0])


    def mlp_collect(self, residues, offsets, discovery: Params | None = None, stream=None) -> int:
        """Append the labelled candidates of one sequence set to the training
        pool (discovery overrides k, n_subs, sub_alphabet and ck_min); returns
        the number of examples added."""
        n = offsets.numel() - 1
        added = ctypes.c_int64(0)
        dp = None if discovery is None else ctypes.byref(discovery.to_c())
        self._check(lib().pastis_mlp_collect(self._ctx, _dev_ptr(residues), _dev_ptr(offsets), n,
                                             int(residues.is_cuda), dp, _stream_ptr(stream), ctypes.byref(added)))
        return int(added.value)

    def mlp_clear(self):
        self._check(lib().pastis_mlp_clear(self._ctx))

    def mlp_pool_size(self) -> int:
        n = ctypes.c_int64(0)
        self._check(lib().pastis_mlp_pool_size(self._ctx, ctypes.byref(n)))
        return int(n.value)

    def mlp_train(self, stream=None, **opts) -> dict:
        """Train a new network on the pool inside the library (options as in
        pastis_mlp_train_opts; unnamed ones keep the library defaults)."""
        o = _TrainOpts()
        lib().pastis_mlp_default_train_opts(ctypes.byref(o))
        for k, v in opts.items():
            if k not in dict(_TrainOpts._fields_) or k == "reserved":
                raise ValueError(f"unknown training option {k}")
            setattr(o, k, v)
        r = _TrainReport()
        self._check(lib().pastis_mlp_train(self._ctx, ctypes.byref(o), _stream_ptr(stream), ctypes.byref(r)))
        out = {f: getattr(r, f) for f, _ in _TrainReport._fields_ if f != "epoch_loss"}
        out["epoch_loss"] = list(r.epoch_loss)[: min(r.epochs, 32)]
        return out

    def mlp_save(self, path: str):
        self._check(lib().pastis_mlp_save(self._ctx, os.fsencode(path)))

    def mlp_load(self, path: str):
        self._check(lib().pastis_mlp_load(self._ctx, os.fsencode(path)))


    # ---- the similarity graph as families ----

    def components(self, edges, n: int, stream=None):
        """Component labels [n] (device uint32 as int32: the smallest vertex of
        each component) of the graph of `edges` (device uint8 tensor of
        48-byte pastis_edge entries, or a pastis_result's device pointer
        with its count as (ptr, count))."""
        torch = _torch()
        if isinstance(edges, tuple):
            ptr, m = edges
        else:
            ptr, m = _dev_ptr(edges), edges.numel() // EDGE_DTYPE.itemsize
        out = torch.empty(max(n, 1), dtype=torch.int32, device=f"cuda:{self.device}")
        self._check(lib().pastis_components(self._ctx, ptr if m else None, m, n, _dev_ptr(out), _stream_ptr(stream)))
        return out[:n]

    def cluster_scores(self, cluster, family, stream=None):
        """(weighted precision, weighted recall) of device labels against device families."""
        p, r = ctypes.c_double(0), ctypes.c_double(0)
        self._check(lib().pastis_cluster_scores(self._ctx, _dev_ptr(cluster), _dev_ptr(family), cluster.numel(),
                                                ctypes.byref(p), ctypes.byref(r), _stream_ptr(stream)))
        return p.value, r.value


def records_to_numpy(t) -> np.ndarray:
    return t.cpu().numpy().view(RECORD_DTYPE)
