"""CPU oracle for the weighted Misra-Gries community-detection path.

TEST INFRASTRUCTURE ONLY.  A plain C implementation (``mgcd_oracle.c``) written
from the paper, loaded through ctypes.  Only the test suite, the smoke check and
the CPU-baseline leg of ``bench.py`` may import this package; the product path
(``paper_2411_02268_amd``) never does, and the two share no code.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mgcd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

MODE_EXACT, MODE_ALG1, MODE_UNCOND, MODE_STD = 0, 1, 2, 3
# weighted Boyer-Moore (Section 4.1): Algorithm 1 with one slot for local moving and
# refinement and four for aggregation (resolved in _params)
MODE_BM = 4
# small mod-based table (Appendix A.2): k is the number of slots; aggregation is exact
MODE_SMALL = 5
ALGO_LPA, ALGO_MOVE, ALGO_REFINE = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain -O2, OpenMP, no vector intrinsics)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-function", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True, cwd=HERE)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Params(ct.Structure):
    _fields_ = [("mode", ct.c_int32), ("k", ct.c_int32), ("k_aggregate", ct.c_int32),
                ("max_iterations", ct.c_int32), ("max_passes", ct.c_int32),
                ("threads", ct.c_int32), ("chunk_len", ct.c_int64),
                ("tolerance", ct.c_double), ("tolerance_drop", ct.c_double),
                ("aggregation_tolerance", ct.c_double), ("one_scan", ct.c_int32),
                ("aggregation", ct.c_int32)]


class _Stats(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("passes", ct.c_int32), ("communities", ct.c_int32),
                ("reserved", ct.c_int32), ("edges_scanned", ct.c_int64),
                ("moved_last", ct.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ct.CDLL(LIB)
        P = ct.c_void_p
        i32, i64 = ct.c_int32, ct.c_int64
        L.oracle_sketch_stream.argtypes = [P, P, i64, ct.c_int, ct.c_int, i64, P, P]
        L.oracle_sketch_stream.restype = ct.c_int
        L.oracle_mg_merge.argtypes = [P, P, ct.c_int, P, P, ct.c_int, ct.c_int, P, P]
        L.oracle_mg_merge.restype = ct.c_int
        L.oracle_canonical.argtypes = [i32, P, P]
        L.oracle_canonical.restype = None
        L.oracle_move_sweep.argtypes = [i32, P, P, P, ct.c_int, ct.c_int, ct.c_int, i64, P, P, P, P,
                                        P, i64, ct.c_int, ct.c_int, P, P]
        L.oracle_move_sweep.restype = ct.c_int
        L.oracle_refine.argtypes = [i32, P, P, P, P, P, i64, ct.c_int, ct.c_int, i64, P]
        L.oracle_refine.restype = ct.c_int
        L.oracle_aggregate.argtypes = [i32, P, P, P, P, i32, ct.c_int, ct.c_int, i64, ct.c_int, P,
                                       P, P]
        L.oracle_aggregate.restype = i64
        L.oracle_modularity.argtypes = [i32, P, P, P, P]
        L.oracle_modularity.restype = ct.c_double
        for name in ("oracle_lpa", "oracle_louvain", "oracle_leiden"):
            f = getattr(L, name)
            f.argtypes = [i32, P, P, P, ct.POINTER(_Params), P, ct.POINTER(_Stats)]
            f.restype = ct.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


def _csr(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    idx = np.ascontiguousarray(g.indices, dtype=np.int32)
    w = np.ascontiguousarray(g.weights, dtype=np.uint32)
    return off, idx, w


@dataclass
class Stats:
    iterations: int
    passes: int
    communities: int
    edges_scanned: int
    moved_last: int


# ---------------------------------------------------------------------------------
# sketch level
# ---------------------------------------------------------------------------------

def sketch_stream(keys, weights, mode=MODE_ALG1, k=8, chunk_len=1 << 62):
    """Final sketch of a (key, weight) stream: dict key -> value (positive only)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    weights = np.ascontiguousarray(weights, dtype=np.uint32)
    n = keys.shape[0]
    cap = max(n, k, 1)
    ok = np.zeros(cap, dtype=np.uint32)
    ov = np.zeros(cap, dtype=np.uint32)
    m = lib().oracle_sketch_stream(_p(keys), _p(weights), n, mode, k, chunk_len, _p(ok), _p(ov))
    if m < 0:
        raise ValueError("bad sketch arguments")
    return {int(a): int(b) for a, b in zip(ok[:m], ov[:m])}


def mg_merge(a: dict, b: dict, k: int) -> dict:
    ak = np.array(list(a.keys()), dtype=np.uint32)
    av = np.array(list(a.values()), dtype=np.uint32)
    bk = np.array(list(b.keys()), dtype=np.uint32)
    bv = np.array(list(b.values()), dtype=np.uint32)
    ok = np.zeros(max(k, 1), dtype=np.uint32)
    ov = np.zeros(max(k, 1), dtype=np.uint32)
    m = lib().oracle_mg_merge(_p(ak), _p(av), len(a), _p(bk), _p(bv), len(b), k, _p(ok), _p(ov))
    if m < 0:
        raise ValueError("bad merge arguments")
    return {int(x): int(y) for x, y in zip(ok[:m], ov[:m])}


def canonical(C) -> np.ndarray:
    C = np.ascontiguousarray(C, dtype=np.int32)
    out = np.zeros_like(C)
    lib().oracle_canonical(C.shape[0], _p(C), _p(out))
    return out


# ---------------------------------------------------------------------------------
# phase level
# ---------------------------------------------------------------------------------

def weighted_degree(g) -> np.ndarray:
    off, _, w = _csr(g)
    cs = np.concatenate([[0], np.cumsum(w.astype(np.int64))])
    return cs[off[1:]] - cs[off[:-1]]


def move_sweep(g, algo, C, mode=MODE_ALG1, k=8, chunk_len=128, bound=None, K=None, Sigma=None,
               size=None, W=None, direction=0, one_scan=0):
    """One synchronous sweep.  Returns (C_new, gain): for Louvain moves C_new holds
    the moves allowed by ``direction`` (-1 lower ids only, +1 higher ids only, 0 all);
    gain holds the integer gain of every vertex's best move.  one_scan=1 (LPA): the
    1-scan variant of Section 4.3, deciding from the sketch's values."""
    off, idx, w = _csr(g)
    n = off.shape[0] - 1
    C = np.ascontiguousarray(C, dtype=np.int32)
    if K is None:
        K = weighted_degree(g)
    K = np.ascontiguousarray(K, dtype=np.int64)
    if W is None:
        W = int(K.sum())
    if Sigma is None:
        Sigma = np.bincount(C, weights=K, minlength=n).astype(np.int64)
    if size is None:
        size = np.bincount(C, minlength=n).astype(np.int32)
    Sigma = np.ascontiguousarray(Sigma, dtype=np.int64)
    size = np.ascontiguousarray(size, dtype=np.int32)
    bnd = np.ascontiguousarray(bound, dtype=np.int32) if bound is not None else None
    Cn = np.zeros(n, dtype=np.int32)
    gain = np.zeros(n, dtype=np.int64)
    rc = lib().oracle_move_sweep(n, _p(off), _p(idx), _p(w), algo, mode, k, chunk_len, _p(C),
                                 _p(bnd), _p(K), _p(Sigma), _p(size), int(W), direction,
                                 int(one_scan), _p(Cn), _p(gain))
    if rc:
        raise ValueError("bad sweep arguments")
    return Cn, gain


def refine(g, bound, mode=MODE_ALG1, k=8, chunk_len=128, K=None, W=None) -> np.ndarray:
    off, idx, w = _csr(g)
    n = off.shape[0] - 1
    if K is None:
        K = weighted_degree(g)
    K = np.ascontiguousarray(K, dtype=np.int64)
    if W is None:
        W = int(K.sum())
    bound = np.ascontiguousarray(bound, dtype=np.int32)
    R = np.zeros(n, dtype=np.int32)
    lib().oracle_refine(n, _p(off), _p(idx), _p(w), _p(bound), _p(K), int(W), mode, k, chunk_len,
                        _p(R))
    return R


def aggregate(g, D, m, mode=MODE_ALG1, k=8, chunk_len=128, symmetric=False):
    """Aggregated CSR (offsets, indices, weights) under dense membership D."""
    from types import SimpleNamespace
    off, idx, w = _csr(g)
    n = off.shape[0] - 1
    D = np.ascontiguousarray(D, dtype=np.int32)
    L = lib()
    nnz = L.oracle_aggregate(n, _p(off), _p(idx), _p(w), _p(D), m, mode, k, chunk_len,
                             int(symmetric), None, None, None)
    o2 = np.zeros(m + 1, dtype=np.int64)
    i2 = np.zeros(max(nnz, 1), dtype=np.int32)
    w2 = np.zeros(max(nnz, 1), dtype=np.uint32)
    L.oracle_aggregate(n, _p(off), _p(idx), _p(w), _p(D), m, mode, k, chunk_len, int(symmetric),
                       _p(o2), _p(i2), _p(w2))
    return SimpleNamespace(offsets=o2, indices=i2[:nnz], weights=w2[:nnz])


def modularity(g, C) -> float:
    off, idx, w = _csr(g)
    C = np.ascontiguousarray(C, dtype=np.int32)
    return float(lib().oracle_modularity(off.shape[0] - 1, _p(off), _p(idx), _p(w), _p(C)))


# ---------------------------------------------------------------------------------
# whole runs
# ---------------------------------------------------------------------------------

DEFAULTS = dict(mode=MODE_ALG1, k=8, k_aggregate=None, chunk_len=128, max_iterations=20,
                max_passes=10, tolerance=None, tolerance_drop=10.0, aggregation_tolerance=0.8,
                threads=0, one_scan=0, aggregation=0)


def _params(algo: str, **kw) -> _Params:
    o = dict(DEFAULTS)
    o.update(kw)
    if o["k_aggregate"] is None:
        o["k_aggregate"] = o["k"]
    if o["mode"] == MODE_BM:
        o["mode"], o["k"], o["k_aggregate"] = MODE_ALG1, 1, 4
    if o["tolerance"] is None:
        o["tolerance"] = 0.05 if algo == "lpa" else 1e-2
    return _Params(o["mode"], o["k"], o["k_aggregate"], o["max_iterations"], o["max_passes"],
                   o["threads"], o["chunk_len"], o["tolerance"], o["tolerance_drop"],
                   o["aggregation_tolerance"], o["one_scan"], o["aggregation"])


def _run(name: str, g, **kw):
    off, idx, w = _csr(g)
    n = off.shape[0] - 1
    p = _params(name, **kw)
    labels = np.zeros(max(n, 1), dtype=np.int32)
    st = _Stats()
    rc = getattr(lib(), "oracle_" + name)(n, _p(off), _p(idx), _p(w), ct.byref(p), _p(labels),
                                          ct.byref(st))
    if rc:
        raise ValueError(f"oracle_{name} failed: {rc}")
    return labels[:n], Stats(st.iterations, st.passes, st.communities, st.edges_scanned,
                             st.moved_last)


def lpa(g, **kw):
    return _run("lpa", g, **kw)


def louvain(g, **kw):
    return _run("louvain", g, **kw)


def leiden(g, **kw):
    return _run("leiden", g, **kw)
