#!/usr/bin/env python3
"""Benchmark of the gfx950 many-to-many protein similarity search hot path.

Prints ONE JSON line.  `value` is whole-step alignment throughput in GCUPS
(DP cells per second over the whole timed step, inputs already resident in
HBM); `pairs_per_s`, the roofline of the dominant kernel, the learned filter
against the plain search, and a CPU oracle baseline are reported beside it.

Default workload ("large"): 250,000 synthetic protein sequences (10,000
families x 20 plus 50,000 unrelated singletons, lengths lognormal mean 350
clamped to [30, 5000], 30% divergence, indels 0.02 / mean 3, seed 0), exact
6-mers, pairs sharing >= 2 k-mers aligned by Smith-Waterman (BLOSUM62, gaps
11/1) and cut at 30% identity / 70% coverage.  One step is one pastis_search
call from HBM-resident sequences to HBM-resident edges, with the SW schedule
chosen by the library's autotuner on a candidate sample and the SW stage
replayed as a captured HIP graph.  The learned filter is trained on the mid
recipe (50,000 sequences, another seed; candidates of 25 substitute 6-mers
and of exact 6-mers, both >= 2 shared) and applied to this workload.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "alignment GCUPS + aligned pairs/s, 1 GPU; MLP-filtered vs plain at ≥99% recall"
# int32 VALU lane-ops per second on MI355X: 256 CUs x 64 lanes x 2.4 GHz;
# packed 16-bit ops (v_pk_*_i16) do two lane-ops each
PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_INT16_TOPS = 2 * PEAK_INT32_TOPS
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
# algorithmic integer ops per pass-1 DP cell, as each lane width computes the
# recurrence with the gap states floored at zero (E' = max(E, 0), F' = max(F, 0)):
#   16-bit, per two cells (one packed op each): spread of the two scores (1),
#     d = G + s (1), E' and F' (clamped subtract + max: 2 + 2), h = max(d, E', F')
#     (2), G = h - (o + e) (1), row maximum (1)                       -> 10
#   32-bit one strip: d (1), E' (2), F' (2), h (one 3-way max: 1), G (1),
#     end key (h << 16 | ~column) and its maximum (2)                -> 9
#   32-bit multi-strip: as one strip, but the row maximum and its column (3) -> 10
#   16-bit multi-strip: as 16-bit (the strip boundary is a lane move)        -> 10
OPS_PER_SW_CELL = {(16, False): 10, (16, True): 10, (32, False): 9, (32, True): 10}
# the method's own count per SW cell, independent of the formulation: the gap
# open term (1), E and F (2 + 2), the diagonal with its score (1), the 3-way
# maximum with zero (2), and the running best with its position (3)
ALGO_OPS_PER_SW_CELL = 11
# x-drop: the same recurrence plus the drop test per live cell
ALGO_OPS_PER_XD_CELL = 12
# HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (KiB per
# dispatch, profiles/sw_search_<workload>_kernel_stats.md), scaled by what the
# counters read for a 1 GiB device copy (FETCH x 2.0, WRITE x 1.0); keyed by
# workload and kernel (a strip bin's two launches: their sum), and only for
# kernels unchanged since those counters were taken
MEASURED_TRAFFIC_KIB = {
    ("large", "sw16s_pass1_kernel<32, 9, 4> + sw16s_pass1_kernel<32, 10, 4>"): (690858.6, 61411.7),
    ("large", "sw16s_pass1_kernel<32, 11, 4> + sw16s_pass1_kernel<32, 12, 4>"): (547507.7, 46009.6),
    ("large", "sw16s_pass1_kernel<32, 13, 4> + sw16s_pass1_kernel<32, 14, 4>"): (455684.8, 36387.2),
    ("large", "sw16s_pass1_kernel<32, 15, 4> + sw16s_pass1_kernel<32, 16, 4>"): (338121.6, 25849.5),
    ("mid", "sw16s_pass1_kernel<32, 9, 4> + sw16s_pass1_kernel<32, 10, 4>"): (1448426.2, 152314.0),
    ("mid", "sw16s_pass1_kernel<32, 11, 4> + sw16s_pass1_kernel<32, 12, 4>"): (1247509.3, 129182.3),
    ("mid", "sw16s_pass1_kernel<32, 13, 4> + sw16s_pass1_kernel<32, 14, 4>"): (963776.0, 99906.1),
    ("mid", "sw16s_pass1_kernel<32, 15, 4> + sw16s_pass1_kernel<32, 16, 4>"): (720457.1, 75910.6),
    ("mid", "sw16_pass1_kernel<9, 2, false>"): (599028.2, 65327.9),
    ("mid", "sw16_pass1_kernel<10, 2, false>"): (348941.0, 40720.7),
}
# the same counters for the kernels of the sparse-product stage (one launch of
# each per step): the row scan that sizes each row's table, the headed
# posting records, and the product kernels (LDS tables of 2K..32K slots, and
# global-memory tables for the largest rows).  A row entry's posting list is a
# scattered read (a header and its records share a line), so the traffic
# exceeds the compulsory bytes several times over.  Exact rows carry their
# entries' posting lengths, so on large the row scan reads rows only; the
# substitute rows of mid still read each entry's header.
SPGEMM_TRAFFIC_KIB = {
    "large": {"work_kernel": (168184.7, 2846.7),
              "posting_records_kernel": (507979.7, 957138.4),
              "spgemm_lds_kernel<2048, 1024>": (3272152.0, 1548491.2),
              "spgemm_lds_kernel<4096, 2048>": (3412106.8, 1716966.8),
              "spgemm_lds_kernel<8192, 3072>": (1335173.5, 687799.4),
              "spgemm_lds_kernel<16384, 2048>": (166611.3, 89088.7),
              "spgemm_lds_kernel<32768, 4096>": (6703.3, 3697.6),
              "spgemm_global_kernel": (23.3, 131072.0)},
    "mid": {"work_kernel": (10991613.1, 3746.7),
            "posting_records_kernel": (114679.5, 241049.4),
            "spgemm_lds_kernel<2048, 1024>": (189456.2, 47655.7),
            "spgemm_lds_kernel<4096, 2048>": (1779433.5, 507194.9),
            "spgemm_lds_kernel<8192, 3072>": (5913474.1, 2197085.2),
            "spgemm_lds_kernel<16384, 2048>": (5810882.0, 2948496.0),
            "spgemm_lds_kernel<32768, 4096>": (2212974.0, 1422669.8),
            "spgemm_global_kernel": (1747741.1, 1480869.8)},
}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0

# method parameters of each workload (Section VI settings: BLOSUM62, gaps
# 11/1, x-drop 49, identity >= 30%, coverage >= 70%)
WORKLOAD_PARAMS = {
    "tiny": dict(k=6, n_subs=0, ck_min=1),
    "mid": dict(k=6, n_subs=25, ck_min=2),
    "large": dict(k=6, n_subs=0, ck_min=2),
    "heavy": dict(k=5, n_subs=25, ck_min=2),
}
WORKLOAD_TEXT = {
    "tiny": "25 families x 20, lengths lognormal mean 200 in [50, 600], 30% divergence; k=6 exact, >=1 shared",
    "mid": "2,000 families x 25, lengths lognormal mean 350 in [30, 2000], 30% divergence; k=6, 25 substitute "
    "k-mers, >=2 shared",
    "large": "10,000 families x 20 + 50,000 singletons, lengths mean 350 in [30, 5000]; k=6 exact, >=2 shared",
    "heavy": "4,000 families x 25, 95% lognormal(300) / 5% uniform [5000, 35000] lengths, 40% divergence; "
    "k=5, 25 substitute k-mers, >=2 shared",
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=["tiny", "mid", "large", "heavy"])
    ap.add_argument("--families", type=int, default=None, help="scale the workload down (tests)")
    ap.add_argument("--block-entries", type=int, default=0,
                    help="search in row blocks of at most this many directional candidate entries (0: one block)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-filter leg")
    ap.add_argument("--mlp-epochs", type=int, default=4)
    ap.add_argument("--no-xd", action="store_true", help="skip the x-drop leg")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the library's default schedule instead of tuning it on a candidate sample first")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the step with direct launches only (default: the SW stage replayed as a HIP graph)")
    ap.add_argument("--no-mid", action="store_true", help="skip the mid-workload sub-object")
    ap.add_argument("--no-ns", action="store_true",
                    help="skip the normalised-score weight leg (no statistics pass)")
    ap.add_argument("--pairs", type=int, default=0,
                    help="also time the alignment stage alone on this many seeded pairs (0: off)")
    ap.add_argument("--tune-pairs", type=int, default=2_000_000, help="candidate sample size of the autotuner")
    ap.add_argument("--schedule", default=None,
                    help="explicit SW schedule, e.g. sw16_max_rows=16,sw_direct_pct=50,sw_grid_scale=1,"
                    "sw_grid_scale_wide=1 (unnamed knobs keep the library default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one 1 GiB device-to-device copy (a reference for HBM byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    return ap.parse_args()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(fs, lo, hi, target_s):
    """The CPU oracle (textbook SW with traceback, OpenMP over pairs) on a
    bounded random sample of the step's candidate pairs: once on every host
    core the process may use, once on one core (a smaller sample)."""
    import numpy as np

    import oracle

    codes = oracle.encode(fs.residues)
    L = np.diff(fs.offsets)
    rng = np.random.default_rng(7)
    take = rng.permutation(lo.size)

    def timed(sel):
        t0 = time.perf_counter()
        rec = oracle.align_pairs(codes, fs.offsets, lo[sel], hi[sel], mode="sw")
        dt = time.perf_counter() - t0
        cells = float((L[lo[sel]].astype(np.int64) * L[hi[sel]]).sum())
        assert int(rec["cells"].sum()) == int(cells)
        return dt, cells

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    oracle.set_threads(cores)
    n0 = min(256, lo.size)
    dt0, _ = timed(take[:n0])
    n1 = int(min(lo.size, max(n0, n0 * target_s / max(dt0, 1e-3))))
    dt, cells = timed(take[:n1])
    used = oracle.num_threads()
    # one core: a sample sized for about a third of the target time
    oracle.set_threads(1)
    n2 = int(min(lo.size, max(64, n1 / max(used, 1) / 3)))
    dt1, cells1 = timed(take[:n2])
    oracle.set_threads(cores)
    return {
        "value": cells / dt / 1e9,
        "unit": "GCUPS",
        "pairs_per_s": n1 / dt,
        "cores": used,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": f"{n1} random candidate pairs of the step ({cells:.3e} cells), SW with full traceback, "
        f"{dt:.1f} s on {used} threads",
        "single_core": {"value": cells1 / dt1 / 1e9, "unit": "GCUPS", "pairs_per_s": n2 / dt1,
                        "sample": f"the first {n2} pairs of the same sample ({cells1:.3e} cells), {dt1:.1f} s"},
    }


def set_tuning(ctx, tuning):
    if isinstance(tuning, dict):
        ctx.set_tuning(**{k: tuning[k] for k in ("sw16_max_rows", "sw_direct_pct", "sw_grid_scale",
                                                  "sw_grid_scale_wide", "sw_intra_pair", "sw16_narrow_rows",
                                                  "sw_long_blocks")})


def timed_steps(ctx, args, res, off):
    """W untimed steps, then K timed ones; (ms per step, last edges, summed stage ms, last stats)."""
    import torch

    for _ in range(args.warmup):
        ctx.search(res, off)
    torch.cuda.synchronize()
    stage = [0.0] * 9
    t0 = time.perf_counter()
    for _ in range(args.steps):
        edges = ctx.search(res, off)
        st = ctx.stats()
        stage = [a + b for a, b in zip(stage, st["ms_stage"])]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / args.steps, edges, [x / args.steps for x in stage], st


STAGE_NAMES = ["encode", "kmers", "subs_AS", "spgemm", "schedule", "sw_pass1", "sw_pass2", "edges", "mlp_filter"]


def kernel_name(b, narrow):
    """The pass-1 kernel(s) of a length bin.  A 16-bit strip bin (up to 8 rows
    per lane) is two launches back to back on one stream: the sequences of up
    to 64 R - 32 rows with one row per lane less (two in 16-lane strips),
    then the rest; its events span both."""
    R = b["rows_per_lane"]
    if b["bits"] == 16:
        if b["multi_strip"]:
            return "sw16_pass1_kernel<%d, 4, true>" % R
        if R <= 8:
            S = 16 if R <= min(narrow, 4) else 32
            rp = 64 * R // S
            return "sw16s_pass1_kernel<%d, %d, 4> + sw16s_pass1_kernel<%d, %d, 4>" % (S, rp - 32 // S, S, rp)
        return "sw16_pass1_kernel<%d, 2, false>" % R
    return "sw_pass1_kernel<%d, %s>" % (R, "true" if b["multi_strip"] else "false")


def roofline(st, pass1_ms, traffic_ok, workload, narrow):
    """The dominant pass-1 kernel (the length bin with the most DP work; one
    launch per step, or for a 16-bit strip bin its two rows classes back to
    back on one stream) against the integer VALU peak of its lane width: its
    cells x the method's 11 ops per cell over its HIP-event time on the
    stream it was launched on.  The kernel's own formulation count (10 or 9
    ops per cell) is reported beside it."""

    def ops(b):
        return OPS_PER_SW_CELL[(b["bits"], bool(b["multi_strip"]))]

    def peak_of(b):
        return PEAK_INT16_TOPS if b["bits"] == 16 else PEAK_INT32_TOPS

    # chosen by work, not by event time: the multi-strip bins run on a second
    # stream beside the one-strip bins, so their event spans include time
    # shared with other kernels
    dom = max(st["sw_bins"], key=lambda b: b["cells"] / peak_of(b))
    name = kernel_name(dom, narrow)
    peak = peak_of(dom)
    achieved = dom["cells"] * ALGO_OPS_PER_SW_CELL / (dom["ms"] * 1e-3) / 1e12
    kernel_ops = dom["cells"] * ops(dom) / (dom["ms"] * 1e-3) / 1e12
    mix_peak_s = sum(b["cells"] * ALGO_OPS_PER_SW_CELL / (peak_of(b) * 1e12) for b in st["sw_bins"])
    traffic = None
    if traffic_ok and (workload, name) in MEASURED_TRAFFIC_KIB:
        f, w = MEASURED_TRAFFIC_KIB[(workload, name)]
        traffic = 1024 * (FETCH_SCALE * f + WRITE_SCALE * w)
    return {
        "kernel": name,
        "bound": "alu",
        "achieved": achieved,
        "peak": peak,
        "unit": "Tops/s",
        "frac": achieved / peak,
        "traffic": traffic,
        "kernel_ms": dom["ms"],
        "kernel_cells": dom["cells"],
        "ops_per_cell": ALGO_OPS_PER_SW_CELL,
        "kernel_ops_per_cell": ops(dom),
        "frac_kernel_ops": kernel_ops / peak,
        "all_pass1_bins": {"frac_of_mix_peak": mix_peak_s / (pass1_ms * 1e-3)},
    }


def spgemm_line(st, ms, traffic_workload):
    """Candidate discovery's sparse product against HBM bandwidth.  The
    compulsory bytes are A and its transpose read once (12 B per nonzero),
    the candidates written (20 B each) and, with substitutes, S read once (5 B
    per entry); the stage time also holds the symmetrisation and sort.
    `traffic` is the counted HBM bytes per step of the stage's row scan,
    posting records and product kernels."""
    compulsory = 12 * st["n_kmers"] + 20 * st["n_candidates"] + 5 * st["n_subs_entries"]
    gbs = compulsory / (ms * 1e-3) / 1e9
    traffic = None
    if traffic_workload in SPGEMM_TRAFFIC_KIB:
        traffic = 1024 * sum(FETCH_SCALE * f + WRITE_SCALE * w for f, w in SPGEMM_TRAFFIC_KIB[traffic_workload].values())
    return {
        "products": int(st["spgemm_products"]),
        "nnz_A": int(st["n_kmers"]),
        "nnz_S": int(st["n_subs_entries"]),
        "ms": ms,
        "products_per_s": st["spgemm_products"] / (ms * 1e-3),
        "compulsory_bytes": compulsory,
        "achieved_gb_s": gbs,
        "peak_gb_s": PEAK_HBM_GBS,
        "frac": gbs / PEAK_HBM_GBS,
        "traffic": traffic,
    }


def xd_leg(P, args, params, res, off, n_cand, tuning=None):
    """The same workload with x-drop seed extension from the stored seeds (X = 49)."""
    ctx = P.Context(P.Params(align_mode="xd", **params))
    ms, xedges, stage, st = timed_steps(ctx, args, res, off)
    align_ms = stage[5] + stage[6]
    live = float(st["cells"])
    return {
        "ms_per_step": ms,
        "pairs_per_s": n_cand / (ms * 1e-3),
        "live_cells": live,
        "gcups_live": live / (ms * 1e-3) / 1e9,
        "align_ms": align_ms,
        "register_band_ms": stage[5],
        "wide_band_redo_ms": stage[6],
        "align_pairs_per_s": n_cand / (align_ms * 1e-3),
        "align_frac_int32_peak": live * ALGO_OPS_PER_XD_CELL / (align_ms * 1e-3) / 1e12 / PEAK_INT32_TOPS,
        "edges": int(xedges.size),
    }


def pairs_leg(P, args, params, fs, res, off, tuning):
    """The alignment stage alone on a seeded list of --pairs pairs of the
    workload's sequences (every within-family pair, then uniformly random
    unrelated pairs, shuffled), through the pair-list entry point."""
    import numpy as np
    import torch

    from synth.families import pair_list

    lab = fs.labels[fs.labels >= 0]
    fam = int(sum(c * (c - 1) // 2 for c in np.unique(lab, return_counts=True)[1]))
    per_seq = max(0.0, (args.pairs - fam) / fs.n) * 1.05 + 1.0  # a little over: duplicates are dropped
    lo, hi = pair_list(fs, random_per_seq=per_seq, seed=0)
    rng = np.random.default_rng(np.random.SeedSequence(0, spawn_key=(200,)))
    sel = rng.permutation(lo.size)[: args.pairs]
    lo, hi = lo[sel], hi[sel]
    print(f"bench.py: pair list of {lo.size} pairs ({fam} within families)", file=sys.stderr, flush=True)
    lens = np.diff(fs.offsets)
    cells = float((lens[lo].astype(np.float64) * lens[hi].astype(np.float64)).sum())
    dev = res.device
    pi = torch.from_numpy(lo.view(np.int32)).to(dev)
    pj = torch.from_numpy(hi.view(np.int32)).to(dev)
    ctx = P.Context(P.Params(score_width=16, **params))
    set_tuning(ctx, tuning)
    for _ in range(max(args.warmup, 1)):
        recs = ctx.align_pairs(res, off, pi, pj)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        recs = ctx.align_pairs(res, off, pi, pj)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    passed = int(recs.view(torch.int32).view(-1, 12)[:, 8].sum().item())  # pastis_pair_record.passed
    return {"pairs": int(lo.size), "family_pairs": fam, "ms_per_step": ms, "pairs_per_s": lo.size / (ms * 1e-3),
            "gcups": cells / (ms * 1e-3) / 1e9, "cells": cells, "passed": passed}


# training sets of the learned filter: the mid recipe with another seed, its
# candidates collected with 25 substitute 6-mers and with exact 6-mers (both
# >= 2 shared), so both feature regimes are covered
TRAIN_COLLECTIONS = [dict(k=6, n_subs=25, ck_min=2), dict(k=6, n_subs=0, ck_min=2)]


def mlp_leg(P, args, params, res, off, edges, plain_ms, tuning, graph):
    """Train the learned pre-alignment filter inside the library on other
    sequences (labels from exact alignment), then time the filtered search on
    the bench workload and measure its recall of the exact edges."""
    import numpy as np
    import torch

    from paper_2009_14467_amd import learned_filter as LF
    from synth import workload

    train_over = {} if args.families is None else {"n_families": max(4, args.families // 2)}
    fs_tr = workload("mid", seed=1, **train_over)
    dev = res.device
    rt, ot = torch.from_numpy(fs_tr.residues).to(dev), torch.from_numpy(fs_tr.offsets).to(dev)
    tf = LF.train(P.Params(**params), sets=[(rt, ot, P.Params(**c)) for c in TRAIN_COLLECTIONS],
                  epochs=args.mlp_epochs)
    del rt, ot
    torch.cuda.empty_cache()
    ctx = P.Context(P.Params(filter_mode="mlp", graph_mode=graph, **params))
    set_tuning(ctx, tuning)
    tf.install(ctx)
    fms, fedges, fstage, st = timed_steps(ctx, args, res, off)

    def keys(e):
        return (e["i"].astype(np.uint64) << np.uint64(32)) | e["j"].astype(np.uint64)

    found = np.isin(keys(edges), keys(fedges)).sum()
    return {
        "recall": float(found / max(edges.size, 1)),
        "edges": int(fedges.size),
        "aligned_frac": st["n_aligned"] / max(st["n_candidates"], 1),
        "pairs_skipped": int(st["n_candidates"] - st["n_aligned"]),
        "precision": int(fedges.size) / max(int(st["n_aligned"]), 1),
        "ms_per_step": fms,
        "plain_ms_per_step": plain_ms,
        "speedup": plain_ms / fms,
        "filter_ms": fstage[8],
        "align_ms": fstage[5] + fstage[6],
        "train": {
            "workload": f"mid recipe, seed 1: {fs_tr.n} sequences; collections "
            + "; ".join(f"k={c['k']} n_subs={c['n_subs']} ck>={c['ck_min']}" for c in TRAIN_COLLECTIONS),
            "examples": tf.n_examples,
            "positive_frac": tf.positive_frac,
            "epochs": args.mlp_epochs,
            "seconds": tf.seconds,
            "losses": tf.losses,
            "heldout_recall": tf.heldout_recall,
            "heldout_kept_frac": tf.heldout_kept_frac,
            "tau": tf.tau,
        },
    }


def mid_leg(P, args, dev):
    """The mid workload (50,000 sequences, 25 substitute 6-mers): the plain
    SW step with the library's schedule, and the x-drop step."""
    from synth import workload

    import torch

    over = {} if args.families is None else {"n_families": args.families}
    fs = workload("mid", **over)
    params = WORKLOAD_PARAMS["mid"]
    res = torch.from_numpy(fs.residues).to(dev)
    off = torch.from_numpy(fs.offsets).to(dev)
    ctx = P.Context(P.Params(**params))
    ms, edges, stage, st = timed_steps(ctx, args, res, off)
    cells = float(st["cells"])
    out = {
        "workload": f"mid: {fs.n} sequences ({fs.residues.size} residues), " + WORKLOAD_TEXT["mid"],
        "ms_per_step": ms,
        "gcups": cells / (ms * 1e-3) / 1e9,
        "pairs_per_s": st["n_candidates"] / (ms * 1e-3),
        "candidates": int(st["n_candidates"]),
        "cells": cells,
        "edges": int(edges.size),
        "stage_ms": dict(zip(STAGE_NAMES, stage)),
        "roofline": roofline(st, stage[5], args.families is None, "mid", ctx.get_tuning()["sw16_narrow_rows"]),
        "spgemm": spgemm_line(st, stage[3], "mid" if args.families is None else None),
    }
    if not args.no_xd:
        out["xd"] = xd_leg(P, args, params, res, off, int(st["n_candidates"]))
    del res, off
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2009_14467_amd as P
    from synth import workload

    def note(msg):
        print(f"bench.py: {msg}", file=sys.stderr, flush=True)

    over = {} if args.families is None else {"n_families": args.families}
    fs = workload(args.workload, **over)
    params = dict(WORKLOAD_PARAMS[args.workload])
    if args.block_entries > 0:
        params["block_entries"] = args.block_entries
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    res = torch.from_numpy(fs.residues).to(dev)
    off = torch.from_numpy(fs.offsets).to(dev)
    ctx = P.Context(P.Params(**params))
    tuning = None
    if args.schedule:
        knobs = dict(kv.split("=") for kv in args.schedule.split(","))
        ctx.set_tuning(**{k: int(v) for k, v in knobs.items()})
        tuning = dict(ctx.get_tuning(), source="--schedule")
    elif not args.no_autotune:
        note(f"tuning the schedule on a sample of up to {args.tune_pairs} candidates")
        t0 = time.perf_counter()
        tuning = ctx.autotune(res, off, max_pairs=args.tune_pairs)
        torch.cuda.synchronize()
        tuning = dict(tuning, source="pastis_autotune", seconds=time.perf_counter() - t0,
                      sample_pairs=args.tune_pairs)
    note(f"schedule {tuning}")

    # direct launches: per-stage and per-bin HIP-event times (the roofline's source)
    d_ms, edges, stage, st = timed_steps(ctx, args, res, off)
    note(f"direct launches: {d_ms:.1f} ms per step")
    cells = float(st["cells"])
    n_cand = int(st["n_candidates"])
    graph = not args.no_graph
    ms_step = d_ms
    if graph:
        gctx = P.Context(P.Params(graph_mode=True, **params))
        set_tuning(gctx, tuning)
        ms_step, gedges, _, gst = timed_steps(gctx, args, res, off)
        assert gedges.tobytes() == edges.tobytes(), "graph replay changed the edges"
        graph_info = {"ms_per_step": ms_step, "sw_graph": gst["sw_graph"]}
        del gctx
        note(f"graph mode: {ms_step:.1f} ms per step")
    line = {
        "metric": METRIC,
        "value": cells / (ms_step * 1e-3) / 1e9,
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16+int32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {fs.n} sequences ({fs.residues.size} residues), "
            + ("" if args.families is None else f"scaled to {args.families} families; ")
            + WORKLOAD_TEXT[args.workload],
            "step": "pastis_search: sequences resident in HBM -> edges in HBM (discovery, SW, cut, edges)"
            + ("; SW stage replayed as a captured HIP graph" if graph else "; direct launches"),
            "schedule": "autotuned" if tuning is not None and not args.schedule else
            ("--schedule" if args.schedule else "library default"),
            **{k: v for k, v in params.items()},
        },
        "pairs_per_s": n_cand / (ms_step * 1e-3),
        "candidates": n_cand,
        "row_blocks": int(st["n_row_blocks"]),
        "cells": cells,
        "edges": int(edges.size),
        "direct_launch": {"ms_per_step": d_ms, "gcups": cells / (d_ms * 1e-3) / 1e9},
        "stats_pass_pairs": int(st["stats_pass_pairs"]),
        "stats_pass_cells": int(st["stats_pass_cells"]),
        "bound_pass_pairs": int(st["bound_pass_pairs"]),
        "bound_pass_cells": int(st["bound_pass_cells"]),
        "stage_ms": dict(zip(STAGE_NAMES, stage)),
        "align_gcups": cells / ((stage[5] + stage[6]) * 1e-3) / 1e9,
        "spgemm": spgemm_line(st, stage[3], args.workload if args.families is None else None),
        "roofline": roofline(st, stage[5], args.families is None, args.workload,
                             ctx.get_tuning()["sw16_narrow_rows"]),
        "sw_bins": [dict(b, gcups=b["cells"] / max(b["ms"], 1e-9) / 1e6) for b in st["sw_bins"] if b["pairs"]],
        "schedule": tuning if tuning is not None else dict(ctx.get_tuning(), source="library default"),
    }
    if graph:
        line["graph_mode"] = graph_info
    if not args.no_xd:
        line["xd"] = xd_leg(P, args, params, res, off, n_cand)
        note(f"xd: {line['xd']['ms_per_step']:.1f} ms per step")
    if not args.no_ns:
        nctx = P.Context(P.Params(weight_mode="ns", **params))
        set_tuning(nctx, tuning)
        nms, _, nstage, _ = timed_steps(nctx, args, res, off)
        line["ns_weight"] = {"ms_per_step": nms, "gcups": cells / (nms * 1e-3) / 1e9,
                             "align_ms": nstage[5] + nstage[6]}
    if not args.no_mlp:
        line["mlp_filter"] = mlp_leg(P, args, params, res, off, edges, ms_step, tuning, graph)
        note(f"learned filter: {line['mlp_filter']['speedup']:.2f}x at recall {line['mlp_filter']['recall']:.4f}")
    if args.pairs > 0:
        line["pair_list"] = pairs_leg(P, args, params, fs, res, off, tuning)
    c = None
    if not args.no_cpu_baseline:
        c = ctx.candidates(n_cand)
        lo = c["lo"].cpu().numpy().view(np.uint32)
        hi = c["hi"].cpu().numpy().view(np.uint32)
    del ctx, res, off
    torch.cuda.empty_cache()
    if not args.no_mid and args.workload != "mid":
        line["mid"] = mid_leg(P, args, dev)
        note(f"mid: {line['mid']['ms_per_step']:.1f} ms per step")
    if c is not None:
        line["cpu_baseline"] = cpu_baseline(fs, lo, hi, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
