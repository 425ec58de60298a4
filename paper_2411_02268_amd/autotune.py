"""Autotuner for the sketch size and the schedule.

k is semantic (it changes labels): it is chosen on a calibration sample by the
paper's quality rule (Section 4.1: the smallest sketch whose modularity stays within
1 % of the exact table), taking the fastest k that meets it.  The schedule knobs
(row_lanes, where rows of at most k entries go, exact tier bounds) never change
results: they are chosen by time, and
the tuner checks that every candidate reproduces the default's labels exactly.
The chosen values are written to a JSON params file.
"""
from __future__ import annotations

import json
import time

import numpy as np

SKETCH_K = (1, 2, 4, 8, 16, 32, 64)
ROW_LANES = (8, 16, 32, 64)
SHORT_ROWS = (0, 1, 2)
EXACT_TIERS = ((32, 512, 4096), (16, 256, 4096), (64, 512, 4096), (32, 128, 2048))


def choose_k(table, quality: float = 0.99):
    """table: {k: (worst quality ratio over the sample, seconds)}.  The fastest k
    whose worst ratio is >= quality; if none qualifies, the best ratio (ties: the
    faster).  Returns (k, met)."""
    ok = [k for k, (r, _) in table.items() if r >= quality]
    if ok:
        return min(ok, key=lambda k: (table[k][1], k)), True
    return max(table, key=lambda k: (table[k][0], -table[k][1])), False


def choose_fastest(times):
    """times: {candidate: seconds} -> the fastest candidate (ties: the first)."""
    return min(times, key=lambda c: times[c])


def _runner(mg, algo, batched):
    if batched:
        return lambda graphs, **kw: [lab for lab in mg.run_batched(algo, graphs, **kw)[0]]
    fn = {mg.ALGO_LPA: mg.lpa, mg.ALGO_LOUVAIN: mg.louvain, mg.ALGO_LEIDEN: mg.leiden}[algo]
    return lambda graphs, **kw: [fn(g, **kw)[0] for g in graphs]


def _timed(mg, run, graphs, repeats, **kw):
    import torch
    labels = run(graphs, **kw)  # warm-up, also the labels
    torch.cuda.synchronize()
    ts = []
    for _ in range(repeats):
        a = time.perf_counter()
        run(graphs, **kw)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - a)
    return float(np.median(ts)), labels


def tune(mg, sample, algo: int, ks=SKETCH_K, quality: float = 0.99, repeats: int = 3,
         batched: bool = False, chunk_len: int = 128):
    """Tune on `sample` (list of mg.DeviceGraph).  batched=True times the sample as one
    batched call (LPA and Louvain only).  Returns a dict of chosen params plus a
    report."""
    run = _runner(mg, algo, batched)
    base = {"chunk_len": chunk_len}
    # exact reference and its tier bounds (schedule only)
    tier_t, ref, q_exact = {}, None, None
    for t0, t1, t2 in EXACT_TIERS:
        kw = dict(base, mode=mg.MODE_EXACT, exact_small=t0, exact_lds=t1, exact_lds_big=t2)
        sec, labels = _timed(mg, run, sample, repeats, **kw)
        if q_exact is None:
            q_exact = [mg.modularity(g, lab) for g, lab in zip(sample, labels)]
        labels = [lab.cpu().numpy() for lab in labels]
        if ref is None:
            ref = labels
        elif any(not np.array_equal(a, b) for a, b in zip(ref, labels)):
            raise RuntimeError(f"exact tiers {(t0, t1, t2)} changed the labels")
        tier_t[(t0, t1, t2)] = sec
    tiers = choose_fastest(tier_t)
    # k by the quality rule
    table = {}
    for k in ks:
        sec, labels = _timed(mg, run, sample, repeats, **dict(base, k=k))
        ratios = [mg.modularity(g, lab) / q if q > 0 else 1.0
                  for g, lab, q in zip(sample, labels, q_exact)]
        table[k] = (float(min(ratios)), sec)
    k, met = choose_k(table, quality)
    # row lanes at the chosen k (schedule only)
    lane_t, ref_k = {}, None
    for rl in ROW_LANES:
        sec, labels = _timed(mg, run, sample, repeats, **dict(base, k=k, row_lanes=rl))
        labels = [lab.cpu().numpy() for lab in labels]
        if ref_k is None:
            ref_k = labels
        elif any(not np.array_equal(a, b) for a, b in zip(ref_k, labels)):
            raise RuntimeError(f"row_lanes={rl} changed the labels")
        lane_t[rl] = sec
    rl = choose_fastest(lane_t)
    # where rows of at most k entries go (k <= 16; schedule only): by the level's average
    # row, never or always to the exact one-lane kernel
    short_t = {}
    if k <= 16:
        for sr in SHORT_ROWS:
            sec, labels = _timed(mg, run, sample, repeats, **dict(base, k=k, row_lanes=rl, short_rows=sr))
            labels = [lab.cpu().numpy() for lab in labels]
            if any(not np.array_equal(a, b) for a, b in zip(ref_k, labels)):
                raise RuntimeError(f"short_rows={sr} changed the labels")
            short_t[sr] = sec
    sr = choose_fastest(short_t) if short_t else 0
    return {
        "algo": int(algo), "mode": int(mg.MODE_ALG1), "k": int(k), "k_aggregate": int(k),
        "chunk_len": int(chunk_len), "row_lanes": int(rl), "short_rows": int(sr),
        "exact_small": tiers[0], "exact_lds": tiers[1], "exact_lds_big": tiers[2],
        "report": {
            "quality_rule": quality, "quality_met": met, "batched": batched,
            "sample": [[g.n, g.nnz] for g in sample],
            "k_table": {str(kk): {"worst_Q_ratio": r, "seconds": s} for kk, (r, s) in table.items()},
            "row_lanes_seconds": {str(c): s for c, s in lane_t.items()},
            "short_rows_seconds": {str(c): s for c, s in short_t.items()},
            "exact_tier_seconds": {str(c): s for c, s in tier_t.items()},
            "Q_exact": q_exact,
        },
    }


PARAM_KEYS = ("mode", "k", "k_aggregate", "chunk_len", "row_lanes", "short_rows", "exact_small",
              "exact_lds", "exact_lds_big")


def save(tuned: dict, path: str):
    with open(path, "w") as f:
        json.dump(tuned, f, indent=1)


def load(path: str) -> dict:
    with open(path) as f:
        return json.load(f)


def run_kwargs(tuned: dict, exact: bool = False) -> dict:
    """Keyword arguments for mg.lpa/louvain/leiden/run_batched from a tuned dict;
    exact=True gives the exact-mode run with the tuned tier bounds."""
    kw = {k: tuned[k] for k in PARAM_KEYS if k in tuned}
    if exact:
        kw["mode"] = 0
        kw.pop("short_rows", None)
    return kw
