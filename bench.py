"""Benchmark: community detection with weighted Misra-Gries sketches on one MI355X.

Default workload (louvain-mg-k8-rmat20): Louvain, MG sketch k=8 (Algorithm 1) vs the
exact table, on an R-MAT graph with 2^20 vertices and 16 * 2^20 undirected edge
samples (a, b, c = 0.57, 0.19, 0.19; self-loops dropped, duplicates collapsed,
weights uniform in [1, 8]; ~31.4M CSR entries), plus a serving leg (Poisson stream of
R-MAT requests) and a batched leg (planted graphs, autotuned).  Other workloads:
leiden-mg-k16-cl24 (Leiden k=16 on a 2^24-vertex Chung-Lu graph) and
lpa-mg-k8-planted (LPA on the 10,000-vertex planted partition).  One step = one whole
run (every sweep of every pass, refinement, renumbering and aggregation) on the graph
already resident in HBM.

Prints one JSON line.  `value` = local-move edges/s of the whole job: CSR entries
streamed by local-moving sweeps divided by the wall time of the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from paper_2411_02268_amd.quality import nmi

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "local-move edges/s (sketch vs exact), batched p99 latency, equal modularity"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, GB/s

# HBM bytes of one level-0 launch of the main sweep kernel, per (workload, level 0 on
# the storage copy, short_rows), from FETCH_SIZE and WRITE_SIZE (rocprofv3 --pmc, one
# counter per run) scaled by what the counters read for a 512 MiB device copy (FETCH
# x 2.0, WRITE x 1.0); commands and figures in profiles/k_move_rows_rmat20_counters.md
# and profiles/k_move_rows_cl24_leiden_counters.md.  Each figure is valid only for the
# kernel sources it was taken on (the SHA-256 of TRAFFIC_SOURCES beside it, checked at
# run time); traffic is reported as null when the sources differ.
TRAFFIC_BYTES = {
    ("louvain-mg-k8-rmat20", False, 0): (2223564784, "14135e926398dd07a7f2c1975aa01f1d5d0505a6324d9e01db2eb465472917e9"),
    ("leiden-mg-k16-cl24", False, 0): (79392629096, "14135e926398dd07a7f2c1975aa01f1d5d0505a6324d9e01db2eb465472917e9"),
    ("leiden-mg-k16-cl24", True, 0): (67723806128, "14135e926398dd07a7f2c1975aa01f1d5d0505a6324d9e01db2eb465472917e9"),
}
TRAFFIC_SOURCES = ["csrc/move.hip", "csrc/move.hpp", "csrc/sketch.hpp", "csrc/common.hpp", "csrc/staging.hpp"]


def sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2411_02268_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def class_bytes(g, L: int, k: int, cands: float = 0.0, short: int = 0, label: int = 4):
    """Algorithmic bytes of one level-0 MG sweep per kernel class (reads and writes
    the method must make; a second pass over a row of at most 64 chunks counts as
    on-chip, a second pass over a longer row re-reads its keys and weights):
      per CSR entry 12 B (index 4, weight 4, gathered C[j] 4; `label` = 0 for the
      first sweep from singletons, where C[j] = j is not read);
      per decided vertex 28 B (list 4, offsets 8, C 4, C_new 4, K 4, Sigma_d 4);
      per candidate community c != d scored by class 0, 4 B (its total Sigma_c;
      `cands` = candidates per launch, counted on the device);
      rows of more than 64 chunks: one sketch of 8k + 4 B per group of 64 chunks,
      written by class 0 and read by class 1; class 1 re-reads their entries'
      keys and weights (8 B) and writes and reads 4 (k + 1) B of counts per chunk.
    Class 0: the main sweep kernel (k_move_rows).  Class 1: long-row merge, second
    pass and decision (k_long_merge, k_long_count, k_long_decide).  Class 2: rows of
    1..short entries on the exact one-lane kernel (12 B per entry, 28 B per vertex;
    their candidates' totals are not counted)."""
    deg = np.diff(g.offsets)
    nch = (deg + L - 1) // L
    big = nch > 64
    sh = (deg >= 1) & (deg <= short)
    groups = int(((nch[big] + 63) // 64).sum())
    per_entry = 8 + label
    c0 = per_entry * int(deg[~sh].sum()) + 28 * int((~sh).sum()) + (8 * k + 4) * groups + int(round(4 * cands))
    c1 = (8 * k + 4) * groups + 8 * int(deg[big].sum()) + 2 * 4 * (k + 1) * int(nch[big].sum())
    c2 = per_entry * int(deg[sh].sum()) + 28 * int(sh.sum())
    return [c0, c1, c2]


def serving_leg(mg, torch, requests: int, slots: int, resident: int, sweeps: int, budget_gb: float,
                seed: int = 5):
    """Louvain MG k=8 requests from synth.serving_stream: every request is its own
    R-MAT graph (2^s vertices, s uniform in [14, 21], 8 * 2^s edge samples, weights
    [1, 8]; drawn on the GPU by synth.rmat_torch from the request's seed), arriving as
    a Poisson stream.  Three ways to serve it, each in a device arena of budget_gb:
      plain -- one whole call at a time (the server with one slot: a FIFO of plain
               launches),
      calls -- `slots` worker streams, each running whole calls,
      steps -- up to `resident` requests advancing together, up to `sweeps` sweeps per
               step (0: each step takes every resident level to its end).
    Capacities are measured closed-loop (all requests queued at once); latencies
    open-loop at 0.8 * mu_plain for all three, and at 0.8 * mu of each server.
    Latency = completion minus submission (server clock).  Every served result is
    compared on the device with the request's own plain call (labels, bit-identical,
    hence equal modularity)."""
    import threading
    from paper_2411_02268_amd import synth
    reqs = synth.serving_stream(count=requests, smin=14, smax=21, deg=16, rate_hz=1.0, seed=seed)
    t0 = time.time()
    graphs = [mg.DeviceGraph(*synth.rmat_torch(s, 8, seed=gs)) for _, s, gs in reqs]
    torch.cuda.synchronize()
    nnz = np.array([g.nnz for g in graphs], dtype=np.int64)
    print(f"[bench] serving: {requests} distinct R-MAT requests ({int(nnz.sum())} entries) generated "
          f"in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    mg.louvain(graphs[0])
    solo, svc = [], np.zeros(requests)
    for i, g in enumerate(graphs):
        torch.cuda.synchronize()
        a = time.perf_counter()
        lab, st = mg.louvain(g)
        torch.cuda.synchronize()
        svc[i] = time.perf_counter() - a
        solo.append(lab)
    scales = np.array([s for _, s, _ in reqs])
    unit = np.array([t for t, _, _ in reqs])  # arrival times at one request per second
    budget = int(budget_gb * (1 << 30))
    same = [True]

    def run(kind, rate):
        arrivals = np.zeros(requests) if rate is None else unit / rate
        tickets = [None] * requests
        ready = threading.Semaphore(0)
        out = [None] * requests
        nsl = {"plain": 1, "calls": slots, "steps": resident}[kind]
        with mg.Server(mg.ALGO_LOUVAIN, budget, slots=nsl, stepped=kind == "steps",
                       sweeps_per_step=sweeps) as srv:
            def waiter():
                for k in range(requests):
                    ready.acquire()
                    lab, st, tm = srv.wait(tickets[k])
                    out[k] = (tm, st["edges_scanned"], bool(torch.equal(lab, solo[k])))
            th = threading.Thread(target=waiter)
            th.start()
            start = time.perf_counter()
            for k in range(requests):
                delay = start + arrivals[k] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets[k] = srv.submit(graphs[k])
                ready.release()
            th.join()
            peak = srv.info()["peak_bytes"]
            step_stats = srv.step_stats() if kind == "steps" else None
        lat = np.array([o[0][2] - o[0][0] for o in out])
        t_first = min(o[0][0] for o in out)
        t_last = max(o[0][2] for o in out)
        edges = sum(o[1] for o in out)
        same[0] &= all(o[2] for o in out)
        r = {"kind": kind, "slots": nsl, "rate_rps": rate, "p50_ms": float(np.percentile(lat, 50) * 1e3),
             "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
             "throughput_rps": requests / (t_last - t_first),
             "edges_per_s": edges / (t_last - t_first), "peak_blocks_GB": peak / 2**30}
        if step_stats:
            r["step_stats"] = step_stats
        print(f"[bench] serving {kind} rate {'closed' if rate is None else f'{rate:.1f}/s'}: "
              f"{r['throughput_rps']:.1f} req/s, p50 {r['p50_ms']:.2f} ms, p99 {r['p99_ms']:.2f} ms",
              file=sys.stderr, flush=True)
        return r

    kinds = ("plain", "calls", "steps")
    cap = {kd: run(kd, None) for kd in kinds}
    mu_p = cap["plain"]["throughput_rps"]
    res = {
        "requests": requests, "algorithm": "louvain", "k": 8, "budget_GB": budget_gb,
        "calls_slots": slots, "steps_resident": resident, "steps_sweeps_per_step": sweeps,
        "workload": "synth.serving_stream: distinct R-MAT graphs, 2^14..2^21 vertices (scale "
                    "uniform), 8 * 2^s edge samples, weights [1, 8], Poisson arrivals",
        "entries_total": int(nnz.sum()),
        "plain_service_ms_by_scale": {str(s): float(svc[scales == s].mean() * 1e3)
                                      for s in sorted(set(scales.tolist()))},
        "capacity": cap,
        "at_0.8_mu_plain": {kd: run(kd, 0.8 * mu_p) for kd in kinds},
        "at_0.8_own_mu": {kd: run(kd, 0.8 * cap[kd]["throughput_rps"]) for kd in ("calls", "steps")},
    }
    res["labels_identical_to_plain"] = same[0]
    return res


def batched_leg(mg, torch, count: int, nmax: float, workers: int):
    """LPA and Louvain (MG) on `count` planted-partition graphs (vertex counts
    log-uniform in [1e3, nmax], communities log-uniform in [20, 2000], intra:inter
    degree 12:4, weight 1; graph g seeded 4000 + g) in one batched call, against the
    plain per-graph launches of the same graphs.  k and the schedule knobs come from
    the autotuner on a 32-graph sample (batched).  Labels of the batched call must
    equal the plain launches' (bit-identical, hence equal modularity)."""
    from paper_2411_02268_amd import autotune, synth
    t0 = time.time()
    graphs = synth.planted_batch(count=count, nmax=nmax, workers=workers)
    dgs = [mg.to_device(g) for g in graphs]
    del graphs
    N = sum(g.n for g in dgs)
    E = sum(g.nnz for g in dgs)
    print(f"[bench] batch of {count} graphs: n={N} nnz={E}, built in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    sample = dgs[:: max(1, count // 32)][:32]
    out = {"graphs": count, "n": N, "nnz": E, "nmax": nmax}
    for name, algo, fn in (("lpa", mg.ALGO_LPA, mg.lpa), ("louvain", mg.ALGO_LOUVAIN, mg.louvain)):
        tuned = autotune.tune(mg, sample, algo, repeats=3, batched=True)  # median of 3 per config
        kw = autotune.run_kwargs(tuned)
        mg.run_batched(algo, dgs, **kw)  # warm-up
        torch.cuda.synchronize()
        t_runs = []
        for _ in range(3):  # the median of three (single runs vary by up to 10 %)
            a = time.perf_counter()
            labs, per, tot = mg.run_batched(algo, dgs, **kw)
            torch.cuda.synchronize()
            t_runs.append(time.perf_counter() - a)
        t_batch = float(np.median(t_runs))
        fn(dgs[0], **kw)
        torch.cuda.synchronize()
        a = time.perf_counter()
        same = True
        plain_labels = []
        for g in dgs:
            lab, _ = fn(g, **kw)
            plain_labels.append(lab)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - a
        for x, y in zip(labs, plain_labels):
            same &= bool(torch.equal(x, y))
        sample_labs = labs[:: max(1, count // 32)][:32]
        qs = [mg.modularity(g, lab) for g, lab in zip(sample, sample_labs)]
        nmis = [nmi(lab.cpu().numpy(), synth.planted_batch_truth(gi, nmax=nmax)[1])
                for gi, lab in zip(range(0, count, max(1, count // 32)), sample_labs)]
        edges = sum(p["edges_scanned"] for p in per)
        out[name] = {"k": tuned["k"], "row_lanes": tuned["row_lanes"],
                     "quality_rule_met": tuned["report"]["quality_met"],
                     "batched_s": t_batch, "batched_runs_s": t_runs, "plain_s": t_plain, "speedup": t_plain / t_batch,
                     "batched_edges_per_s": edges / t_batch, "labels_identical_to_plain": same,
                     "mean_Q_sample": float(np.mean(qs)),
                     "mean_nmi_sample_vs_planted": float(np.mean(nmis))}
        print(f"[bench] batched {name}: k={tuned['k']} batch {t_batch*1e3:.1f} ms vs plain "
              f"{t_plain*1e3:.1f} ms ({t_plain/t_batch:.2f}x), identical={same}",
              file=sys.stderr, flush=True)
        del labs, plain_labels
    return out


def k_sweep_leg(mg, torch, dg, repeats: int = 3, chunk_len: int = 128):
    """Synthetic analogue of the paper's k sweeps (Figs. 4-6): for LPA, Louvain and
    Leiden, each sketch variant (Algorithm 1, unconditional subtraction, LPA 1-scan)
    at k = 1..256 and the weighted Boyer-Moore mode, the run time and modularity
    relative to the exact table on the same graph (median of `repeats` runs); and the
    small mod-based table at slot counts of 1e-5 .. 1e-1 of |V|."""
    def timed(fn, **kw):
        lab, _ = fn(dg, chunk_len=chunk_len, **kw)
        torch.cuda.synchronize()
        ts = []
        for _ in range(repeats):
            a = time.perf_counter()
            lab, _ = fn(dg, chunk_len=chunk_len, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - a)
        return float(np.median(ts)), mg.modularity(dg, lab)

    out = {}
    for name in ("lpa", "louvain", "leiden"):
        fn = getattr(mg, name)
        t_x, q_x = timed(fn, mode=mg.MODE_EXACT)
        res = {"exact": {"ms": t_x * 1e3, "Q": q_x}}
        variants = [("alg1", dict(mode=mg.MODE_ALG1)), ("uncond", dict(mode=mg.MODE_UNCOND))]
        if name == "lpa":
            variants.append(("alg1_1scan", dict(mode=mg.MODE_ALG1, one_scan=1)))
        for vname, kw in variants:
            res[vname] = {}
            for k in (1, 2, 4, 8, 16, 32, 64, 128, 256):
                t, q = timed(fn, k=k, **kw)
                res[vname][str(k)] = {"rel_time": t / t_x, "rel_Q": q / q_x if q_x else None}
        t, q = timed(fn, mode=mg.MODE_BM)
        res["bm"] = {"rel_time": t / t_x, "rel_Q": q / q_x if q_x else None}
        # the small mod-based table (Appendix A.2) by slots fraction of |V|
        res["small"] = {}
        for frac in (1e-5, 1e-4, 3e-4, 1e-3, 1e-2, 1e-1):
            slots = max(1, int(round(frac * dg.n)))
            t, q = timed(fn, mode=mg.MODE_SMALL, k=slots)
            res["small"][f"{frac:g}"] = {"slots": slots, "rel_time": t / t_x,
                                         "rel_Q": q / q_x if q_x else None}
        out[name] = res
        best = min((v for v in res["alg1"].values() if v["rel_Q"] and v["rel_Q"] >= 0.99),
                   key=lambda v: v["rel_time"], default=None)
        print(f"[bench] k sweep {name}: exact {t_x*1e3:.2f} ms Q={q_x:.4f}; alg1 rel_Q by k "
              + " ".join(f"{k}:{v['rel_Q']:.3f}" for k, v in res["alg1"].items())
              + f"; fastest within 1 %: {best}", file=sys.stderr, flush=True)
    return out


WORKLOADS = {
    # name: (algorithm, k, graph description, generator -> (CSR, planted communities or None))
    # (the large graphs sort their edge samples on the GPU: the same CSR as on the host)
    "louvain-mg-k8-rmat20": (
        "louvain", 8, "R-MAT scale 20, edge factor 16, a/b/c=0.57/0.19/0.19, weights U[1,8], seed 2",
        lambda synth: (synth.rmat(scale=20, edge_factor=16, seed=2, device="cuda"), None)),
    "leiden-mg-k16-cl24": (
        "leiden", 16, "Chung-Lu 2^24 vertices, mean degree 32, exponent 2.1, weights U[1,4], seed 3",
        lambda synth: (synth.chung_lu(n=1 << 24, avg_deg=32, seed=3, device="cuda"), None)),
    "leiden-mg-k64-cl24": (
        "leiden", 64, "Chung-Lu 2^24 vertices, mean degree 32, exponent 2.1, weights U[1,4], seed 3",
        lambda synth: (synth.chung_lu(n=1 << 24, avg_deg=32, seed=3, device="cuda"), None)),
    "louvain-mg-k64-rmat20": (
        "louvain", 64, "R-MAT scale 20, edge factor 16, a/b/c=0.57/0.19/0.19, weights U[1,8], seed 2",
        lambda synth: (synth.rmat(scale=20, edge_factor=16, seed=2, device="cuda"), None)),
    "louvain-mg-k8-road": (
        "louvain", 8, "road-network stand-in: 1,620^2 grid intersections, segments kept with p 0.6, "
        "0..6 points per segment, unit weights, seed 4 (about 12 M vertices, 2.09 entries per vertex)",
        lambda synth: (synth.road_like(side=1620, seed=4, device="cuda"), None)),
    "louvain-mg-k8-kmer": (
        "louvain", 8, "k-mer stand-in: 2^24 vertices in chains of mean length 16, ends joined "
        "with p 0.9, unit weights, seed 5 (about 2.1 entries per vertex)",
        lambda synth: (synth.kmer_like(n=1 << 24, seed=5, device="cuda"), None)),
    "lpa-mg-k8-planted": (
        "lpa", 8, "planted partition 20 x 500, 12 intra + 4 inter edges per vertex, weight 1, seed 1",
        lambda synth: synth.planted_exact(n_comm=20, comm_size=500, seed=1)),
}
DEFAULT_WORKLOAD = "louvain-mg-k8-rmat20"


def host_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--exact-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=None,
                    help="requests of the serving leg (0 skips it; default 2000 with the "
                         "default workload, else 0)")
    ap.add_argument("--serve-slots", type=int, default=4, help="worker streams of the whole-call server")
    ap.add_argument("--serve-resident", type=int, default=64,
                    help="resident requests of the step-level server")
    ap.add_argument("--serve-sweeps", type=int, default=0,
                    help="sweeps per step of the step-level server (0: a whole level per step)")
    ap.add_argument("--batch-graphs", type=int, default=None,
                    help="graphs of the batched leg (0 skips it; default 4096 with the "
                         "default workload, else 0)")
    ap.add_argument("--batch-nmax", type=float, default=2e5)
    ap.add_argument("--storage-order", type=int, default=0, choices=(0, 1, 2),
                    help="level-0 storage copy in degree order: 0 by size (default), 1 off, 2 on "
                         "(schedule only: results are the same)")
    ap.add_argument("--short-rows", type=int, default=0, choices=(0, 1, 2),
                    help="MG rows of at most k entries on the exact one-lane kernel: 0 (default) "
                         "when the average row has at most k entries, 1 never, 2 always "
                         "(schedule only: results are the same)")
    ap.add_argument("--no-quality-split", dest="quality_split", action="store_false",
                    help="skip the modularity of L = 4096 and of aggregation decoupled "
                         "from local moving")
    ap.add_argument("--k-sweep", action="store_true",
                    help="also run the k sweep of every sketch variant on the workload graph")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="finish with three 512 MiB device-to-device copies, the reference "
                         "kernel for scaling FETCH_SIZE / WRITE_SIZE counters to bytes")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding notes in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    default = args.workload == DEFAULT_WORKLOAD
    if args.serve_requests is None:
        args.serve_requests = 2000 if default else 0
    if args.batch_graphs is None:
        args.batch_graphs = 4096 if default else 0

    import torch
    import paper_2411_02268_amd as mg
    from paper_2411_02268_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mg.lib()
    algo_name, k, graph_desc, gen = WORKLOADS[args.workload]
    L = 128
    fn = {"lpa": mg.lpa, "louvain": mg.louvain, "leiden": mg.leiden}[algo_name]
    t0 = time.time()
    g, truth = gen(synth)
    gen_s = time.time() - t0
    print(f"[bench] {args.workload}: graph n={g.n} nnz={g.nnz} W={g.total_weight()} generated in "
          f"{gen_s:.1f}s", file=sys.stderr, flush=True)
    dg = mg.to_device(g)

    def run(mode, steps, warm):
        so = args.storage_order
        for _ in range(warm):
            fn(dg, mode=mode, k=k, chunk_len=L, storage_order=so, short_rows=args.short_rows)
        torch.cuda.synchronize()
        stats = []
        a = time.perf_counter()
        for _ in range(steps):
            lab, st = fn(dg, mode=mode, k=k, chunk_len=L, storage_order=so, short_rows=args.short_rows)
            stats.append(st)
        torch.cuda.synchronize()
        b = time.perf_counter()
        return lab, stats, b - a

    lab, stats, secs = run(mg.MODE_ALG1, args.steps, args.warmup)
    edges = sum(s["edges_scanned"] for s in stats)
    value = edges / secs
    q_mg = mg.modularity(dg, lab)
    print(f"[bench] MG k={k}: {args.steps} steps in {secs:.3f}s, {value/1e9:.3f} G edges/s, "
          f"Q={q_mg:.6f}", file=sys.stderr, flush=True)

    # dominant level-0 kernel class, its live HIP-event time, algorithmic bytes
    ms = np.zeros(3)
    sweeps = 0
    for s in stats:
        ms += np.array(s["ms_l0_kernel"])
        sweeps += s["l0_sweeps"]
    cands = sum(s["l0_candidates"] for s in stats) / max(sweeps, 1)
    # MG Algorithm 1 here: rows of at most k entries on the exact kernel (level 0)
    short = k if (k <= 16 and (args.short_rows == 2 or (args.short_rows == 0 and g.nnz <= k * g.n))) else 0
    cb = class_bytes(g, L, k, cands, short)
    used_copy = args.storage_order == 2 or (args.storage_order == 0 and g.nnz >= (1 << 26))
    if not used_copy:
        # the first level-0 sweep of every run starts from singletons and reads no
        # labels: average the bytes over the same launches as the time
        per_run = sweeps / max(len(stats), 1)
        cb1 = class_bytes(g, L, k, cands, short, label=0)
        cb = [int(round((c1 + (per_run - 1) * c) / per_run)) for c1, c in zip(cb1, cb)]
    dom = int(np.argmax(ms))
    names = ["k_move_rows (every row of more than k entries: staged sketch, merge tree, second "
             "pass, decision; chunk sketches of rows longer than 64 chunks)",
             "k_long_merge + k_long_count + k_long_decide (rows longer than 64 chunks)",
             "k_exact_small (rows of at most k entries: their sketch is their exact table)"]
    per_launch_ms = ms[dom] / max(sweeps, 1)
    achieved = cb[dom] / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
    sweep_ms = ms.sum() / max(sweeps, 1)
    sweep_gbs = sum(cb) / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else 0.0

    exact = None
    q_x = None
    if args.exact_steps > 0:
        lab_x, stats_x, secs_x = run(mg.MODE_EXACT, args.exact_steps, 1)
        edges_x = sum(s["edges_scanned"] for s in stats_x)
        q_x = mg.modularity(dg, lab_x)
        exact = {"value": edges_x / secs_x, "unit": "edges/s",
                 "ms_per_step": secs_x / args.exact_steps * 1e3}
        print(f"[bench] exact: {args.exact_steps} steps in {secs_x:.3f}s, "
              f"{edges_x/secs_x/1e9:.3f} G edges/s, Q={q_x:.6f}", file=sys.stderr, flush=True)

    # where a sketch's modularity loss comes from (Louvain/Leiden, when the exact run
    # is there): the chunk length L = 4096 against the default, and aggregation
    # decoupled from local moving (sketch moving with exact rows; exact moving with
    # sketch rows of k slots)
    split = None
    if q_x and algo_name != "lpa" and args.quality_split:
        split = {}
        for key, kw in (("L4096", dict(mode=mg.MODE_ALG1, k=k, chunk_len=4096)),
                        ("mg_move_exact_agg", dict(mode=mg.MODE_ALG1, k=k, chunk_len=L,
                                                   aggregation=1)),
                        ("exact_move_mg_agg", dict(mode=mg.MODE_EXACT, k_aggregate=k,
                                                   chunk_len=L, aggregation=2))):
            lab_s, _ = fn(dg, **kw)
            qs = mg.modularity(dg, lab_s)
            split[key] = {"Q": qs, "ratio": qs / q_x}
        print(f"[bench] quality split: " + ", ".join(f"{a} {b['ratio']:.3f}" for a, b in split.items()),
              file=sys.stderr, flush=True)

    ground_truth = None
    if truth is not None:  # planted partition: NMI of the labels against it
        ground_truth = {"nmi_mg": nmi(lab.cpu().numpy(), truth)}
        if args.exact_steps > 0:
            ground_truth["nmi_exact"] = nmi(lab_x.cpu().numpy(), truth)
        print(f"[bench] NMI vs planted partition: {ground_truth}", file=sys.stderr, flush=True)

    serving = None
    if args.serve_requests > 0:
        serving = serving_leg(mg, torch, args.serve_requests, args.serve_slots, args.serve_resident,
                              args.serve_sweeps, 64.0)

    batched = None
    if args.batch_graphs > 0:
        batched = batched_leg(mg, torch, args.batch_graphs, args.batch_nmax,
                              min(16, host_threads()))

    ksweep = k_sweep_leg(mg, torch, dg) if args.k_sweep else None

    if args.calibrate_copy:
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        threads = host_threads()
        a = time.perf_counter()
        reps, e_cpu = 0, 0
        if g.nnz <= 100_000_000:
            ofn = {"lpa": oracle.lpa, "louvain": oracle.louvain, "leiden": oracle.leiden}[algo_name]
            while reps < 3 or time.perf_counter() - a < 10.0:
                _, est = ofn(g, mode=oracle.MODE_ALG1, k=k, chunk_len=L, threads=threads)
                e_cpu += est.edges_scanned
                reps += 1
                if time.perf_counter() - a > 30.0:
                    break
            sample = f"whole MG k={k} {algo_name} runs on the same graph"
        else:
            C0 = np.arange(g.n, dtype=np.int32)
            oalgo = oracle.ALGO_LPA if algo_name == "lpa" else oracle.ALGO_MOVE
            while reps < 1 or time.perf_counter() - a < 10.0:
                oracle.move_sweep(g, oalgo, C0, mode=oracle.MODE_ALG1, k=k, chunk_len=L)
                e_cpu += g.nnz
                reps += 1
                if time.perf_counter() - a > 30.0:
                    break
            sample = (f"level-0 MG k={k} local-moving sweeps from singletons on the same graph "
                      f"(a whole run exceeds the time bound)")
        cs = time.perf_counter() - a
        cpu = {"value": e_cpu / cs, "unit": "edges/s", "cores": threads, "kind": "oracle",
               "sample": f"{sample}, {reps} repetitions ({cs:.1f}s), OpenMP threads={threads}"}
        if g.nnz <= 100_000_000:  # one run on one thread as well (same sample kind)
            a1 = time.perf_counter()
            _, est = ofn(g, mode=oracle.MODE_ALG1, k=k, chunk_len=L, threads=1)
            cpu["value_1_thread"] = est.edges_scanned / (time.perf_counter() - a1)
        print(f"[bench] oracle: {reps} reps in {cs:.1f}s -> {e_cpu/cs/1e9:.3f} G edges/s",
              file=sys.stderr, flush=True)

    traffic = None
    known = TRAFFIC_BYTES.get((args.workload, used_copy, args.short_rows))
    if dom == 0 and known and sources_sha256() == known[1]:
        traffic = known[0]
    st_last = stats[-1]
    out = {
        "metric": METRIC, "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": secs / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": args.workload, "graph": graph_desc, "n": g.n, "nnz": g.nnz,
                   "k": k, "chunk_len": L, "algorithm": algo_name, "parallelism": "single-gpu",
                   "storage_order": args.storage_order, "short_rows": args.short_rows,
                   "level0_storage_copy": args.storage_order == 2 or
                                          (args.storage_order == 0 and g.nnz >= (1 << 26))},
        "modularity": {"mg": q_mg, "exact": q_x, "ratio": q_mg / q_x if q_x else None,
                       "split": split},
        "ground_truth": ground_truth,
        "k_sweep": ksweep,
        "exact": exact,
        "stats": {key: st_last[key] for key in ("iterations", "passes", "communities",
                                                 "ms_local_move", "ms_refine", "ms_aggregate",
                                                 "ms_total")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": names[dom],
                     "ms_per_launch": per_launch_ms, "bytes_per_launch": cb[dom],
                     "sweep": {"ms": sweep_ms, "bytes": sum(cb), "GBs": sweep_gbs,
                               "class_ms": (ms / max(sweeps, 1)).tolist(), "class_bytes": cb}},
        "cpu_baseline": cpu,
        "serving": serving,
        "batched": batched,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
