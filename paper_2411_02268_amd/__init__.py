"""MI355X community detection with weighted Misra-Gries sketches.

Thin ctypes binding over libmgcd.so (include/mgcd.h).  PyTorch provides device
memory and the current HIP stream; every step of the computation runs in the
library's HIP kernels.  Importing works without a GPU; calling requires the built
library and a GPU, and fails loudly otherwise (there is no CPU fallback).

    g = to_device(csr)                      # offsets int64, indices int32, weights uint32
    labels, stats = louvain(g, k=8)         # device int32 tensor, dict
    q = modularity(g, labels)
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgcd.so")

MODE_EXACT, MODE_ALG1, MODE_UNCOND, MODE_STD, MODE_BM, MODE_SMALL = 0, 1, 2, 3, 4, 5
ALGO_LPA, ALGO_LOUVAIN, ALGO_LEIDEN = 0, 1, 2
ERRORS = {-1: "E_ARG", -2: "E_GRAPH", -3: "E_OVERFLOW", -4: "E_WORKSPACE", -5: "E_HIP",
          -6: "E_UNSUPPORTED"}


class MgcdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(ct.Structure):
    _fields_ = [("mode", ct.c_int32), ("k", ct.c_int32), ("k_aggregate", ct.c_int32),
                ("max_iterations", ct.c_int32), ("max_passes", ct.c_int32),
                ("validate", ct.c_int32), ("chunk_len", ct.c_int64),
                ("tolerance", ct.c_double), ("tolerance_drop", ct.c_double),
                ("aggregation_tolerance", ct.c_double), ("row_lanes", ct.c_int32),
                ("exact_small", ct.c_int32), ("exact_lds", ct.c_int32),
                ("exact_lds_big", ct.c_int32), ("direct_launch", ct.c_int32),
                ("one_scan", ct.c_int32), ("aggregation", ct.c_int32),
                ("storage_order", ct.c_int32), ("short_rows", ct.c_int32)]


class Stats(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("passes", ct.c_int32), ("communities", ct.c_int32),
                ("reserved", ct.c_int32), ("edges_scanned", ct.c_int64),
                ("moved_last", ct.c_int64), ("ms_local_move", ct.c_float),
                ("ms_refine", ct.c_float), ("ms_aggregate", ct.c_float), ("ms_total", ct.c_float),
                ("l0_sweeps", ct.c_int32), ("reserved2", ct.c_int32),
                ("ms_l0_kernel", ct.c_float * 3), ("reserved3", ct.c_float),
                ("l0_candidates", ct.c_int64)]

    def asdict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if not f.startswith("reserved")}
        d["ms_l0_kernel"] = list(self.ms_l0_kernel)
        return d


class GraphStats(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("passes", ct.c_int32), ("communities", ct.c_int32),
                ("reserved", ct.c_int32), ("edges_scanned", ct.c_int64), ("moved_last", ct.c_int64)]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class StepStats(ct.Structure):
    _fields_ = [(f, ct.c_int64) for f in ("steps", "sweeps", "sweeps_moving", "packs", "transitions",
                                          "rows_swept", "rows_moving")] + \
               [(f, ct.c_double) for f in ("s_pack", "s_sweep", "s_phase", "s_admit")]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class CSRDesc(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("reserved", ct.c_int32), ("nnz", ct.c_int64),
                ("offsets", ct.c_void_p), ("indices", ct.c_void_p), ("weights", ct.c_void_p)]


_lib = None


def lib():
    """The loaded libmgcd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2411_02268_amd.build` (no CPU fallback exists)")
        L = ct.CDLL(LIB_PATH)
        P, i32, i64, sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_size_t
        L.mgcd_default_params.argtypes = [i32, ct.POINTER(Params)]
        L.mgcd_default_params.restype = None
        L.mgcd_workspace_bytes.argtypes = [i32, i32, i64, ct.POINTER(Params)]
        L.mgcd_workspace_bytes.restype = sz
        for name in ("lpa_run", "louvain_run", "leiden_run"):
            f = getattr(L, name)
            f.argtypes = [ct.POINTER(CSRDesc), ct.POINTER(Params), P, P, sz, ct.POINTER(Stats), P]
            f.restype = ct.c_int
        L.mgcd_modularity_workspace_bytes.argtypes = [i32, i64]
        L.mgcd_modularity_workspace_bytes.restype = sz
        L.modularity.argtypes = [ct.POINTER(CSRDesc), P, ct.POINTER(ct.c_double), P, sz, P]
        L.modularity.restype = ct.c_int
        L.modularity_noalloc.argtypes = [ct.POINTER(CSRDesc), P, ct.POINTER(ct.c_double), P]
        L.modularity_noalloc.restype = ct.c_int
        L.mgcd_move_sweep.argtypes = [ct.POINTER(CSRDesc), ct.POINTER(Params), i32, P, i32, P, P, P,
                                      P, sz, P]
        L.mgcd_move_sweep.restype = ct.c_int
        L.mgcd_refine.argtypes = [ct.POINTER(CSRDesc), ct.POINTER(Params), P, P, P, sz, P]
        L.mgcd_refine.restype = ct.c_int
        L.mgcd_aggregate.argtypes = [ct.POINTER(CSRDesc), ct.POINTER(Params), P, i32, i32, P, P, P,
                                     ct.POINTER(ct.c_int64), P, sz, P]
        L.mgcd_aggregate.restype = ct.c_int
        L.mgcd_workspace_bytes_batched.argtypes = [i32, i32, i64, i64, ct.POINTER(Params)]
        L.mgcd_workspace_bytes_batched.restype = sz
        for name in ("lpa_run_batched", "louvain_run_batched"):
            f = getattr(L, name)
            f.argtypes = [ct.POINTER(CSRDesc), i32, ct.POINTER(Params), ct.POINTER(ct.c_void_p), P,
                          sz, ct.POINTER(GraphStats), ct.POINTER(Stats), P]
            f.restype = ct.c_int
        L.mgcd_server_create.argtypes = [P, sz, i32, i32, ct.POINTER(Params), ct.POINTER(P)]
        L.mgcd_server_create.restype = ct.c_int
        L.mgcd_server_create_stepped.argtypes = [P, sz, sz, i32, i32, i32, ct.POINTER(Params), ct.POINTER(P)]
        L.mgcd_server_create_stepped.restype = ct.c_int
        L.mgcd_server_step_stats.argtypes = [P, ct.POINTER(StepStats)]
        L.mgcd_server_step_stats.restype = ct.c_int
        L.mgcd_server_submit.argtypes = [P, ct.POINTER(CSRDesc), P, ct.POINTER(i64)]
        L.mgcd_server_submit.restype = ct.c_int
        L.mgcd_server_poll.argtypes = [P, i64, ct.POINTER(i32)]
        L.mgcd_server_poll.restype = ct.c_int
        L.mgcd_server_wait.argtypes = [P, i64, ct.POINTER(Stats), ct.POINTER(ct.c_double)]
        L.mgcd_server_wait.restype = ct.c_int
        L.mgcd_server_info.argtypes = [P, ct.POINTER(i64), ct.POINTER(i64), ct.POINTER(sz),
                                       ct.POINTER(sz)]
        L.mgcd_server_info.restype = ct.c_int
        L.mgcd_server_destroy.argtypes = [P]
        L.mgcd_server_destroy.restype = ct.c_int
        L.mgcd_last_error.argtypes = []
        L.mgcd_last_error.restype = ct.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise MgcdError(rc, lib().mgcd_last_error().decode())


@dataclass
class DeviceGraph:
    """A CSR graph in device memory (torch tensors); weights stored as int32 bits."""
    offsets: "object"
    indices: "object"
    weights: "object"

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0]) - 1

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    def desc(self) -> CSRDesc:
        return CSRDesc(self.n, 0, self.nnz, self.offsets.data_ptr(),
                       self.indices.data_ptr() if self.nnz else None,
                       self.weights.data_ptr() if self.nnz else None)


def to_device(g, device: str = "cuda") -> DeviceGraph:
    """Copy a host CSR (offsets/indices/weights numpy arrays) to the GPU."""
    import torch
    off = torch.from_numpy(np.ascontiguousarray(g.offsets, dtype=np.int64)).to(device)
    idx = torch.from_numpy(np.ascontiguousarray(g.indices, dtype=np.int32)).to(device)
    w = torch.from_numpy(np.ascontiguousarray(g.weights, dtype=np.uint32).view(np.int32)).to(device)
    return DeviceGraph(off, idx, w)


def params(algo: int, **kw) -> Params:
    p = Params()
    lib().mgcd_default_params(algo, ct.byref(p))
    if "k" in kw and "k_aggregate" not in kw:
        kw["k_aggregate"] = kw["k"]
    for key, val in kw.items():
        if not hasattr(p, key):
            raise TypeError(f"unknown parameter {key}")
        setattr(p, key, val)
    return p


def _stream():
    import torch
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(algo: int, g: DeviceGraph, p: Params):
    import torch
    nbytes = lib().mgcd_workspace_bytes(algo, g.n, g.nnz, ct.byref(p))
    return torch.empty(int(nbytes), dtype=torch.uint8, device=g.offsets.device), int(nbytes)


def _run(name: str, algo: int, g: DeviceGraph, **kw):
    import torch
    p = params(algo, **kw)
    out = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.offsets.device)
    ws, nbytes = _workspace(algo, g, p)
    st = Stats()
    d = g.desc()
    _check(getattr(lib(), name)(ct.byref(d), ct.byref(p), out.data_ptr(), ws.data_ptr(), nbytes,
                                ct.byref(st), _stream()))
    return out[:g.n], st.asdict()


def lpa(g: DeviceGraph, **kw):
    """Label propagation with MG sketches.  Returns (labels, stats)."""
    return _run("lpa_run", ALGO_LPA, g, **kw)


def louvain(g: DeviceGraph, **kw):
    """Louvain with MG local moving and aggregation.  Returns (labels, stats)."""
    return _run("louvain_run", ALGO_LOUVAIN, g, **kw)


def leiden(g: DeviceGraph, **kw):
    """Leiden with MG local moving, refinement and aggregation.  Returns (labels, stats)."""
    return _run("leiden_run", ALGO_LEIDEN, g, **kw)


def modularity(g: DeviceGraph, labels) -> float:
    import torch
    nbytes = int(lib().mgcd_modularity_workspace_bytes(g.n, g.nnz))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=g.offsets.device)
    q = ct.c_double()
    d = g.desc()
    _check(lib().modularity(ct.byref(d), labels.data_ptr(), ct.byref(q), ws.data_ptr(),
                            ws.numel(), _stream()))
    return q.value


def modularity_noalloc(g: DeviceGraph, labels) -> float:
    """modularity() without a workspace: the library's own fixed device scratch
    (graphs of up to NOALLOC_MAX_VERTICES vertices; overlapping calls on one device
    race)."""
    q = ct.c_double()
    d = g.desc()
    _check(lib().modularity_noalloc(ct.byref(d), labels.data_ptr() if g.n else None,
                                    ct.byref(q), _stream()))
    return q.value


NOALLOC_MAX_VERTICES = 1 << 22


def move_sweep(g: DeviceGraph, algo: int, C, direction: int = 0, **kw):
    """One synchronous sweep.  Returns (C_new, gain, [moved, proposals, sum_gain])."""
    import torch
    p = params(ALGO_LOUVAIN if algo == ALGO_LOUVAIN else ALGO_LPA, **kw)
    Cn = torch.empty_like(C)
    gain = torch.zeros(max(g.n, 1), dtype=torch.int64, device=C.device)
    ctr = (ct.c_int64 * 3)()
    ws, nbytes = _workspace(ALGO_LPA, g, p)
    d = g.desc()
    _check(lib().mgcd_move_sweep(ct.byref(d), ct.byref(p), algo, C.data_ptr(), direction,
                                 Cn.data_ptr(), gain.data_ptr(), ctr, ws.data_ptr(), nbytes,
                                 _stream()))
    return Cn, gain[:g.n], [ctr[0], ctr[1], ctr[2]]


def refine(g: DeviceGraph, bound, **kw):
    import torch
    p = params(ALGO_LEIDEN, **kw)
    R = torch.empty_like(bound)
    ws, nbytes = _workspace(ALGO_LPA, g, p)
    d = g.desc()
    _check(lib().mgcd_refine(ct.byref(d), ct.byref(p), bound.data_ptr(), R.data_ptr(),
                             ws.data_ptr(), nbytes, _stream()))
    return R


def aggregate(g: DeviceGraph, D, m: int, symmetric: bool = False, **kw):
    """Aggregated CSR (offsets, indices, weights as uint32 numpy) under dense D."""
    import torch
    p = params(ALGO_LEIDEN if symmetric else ALGO_LOUVAIN, **kw)
    off = torch.empty(m + 1, dtype=torch.int64, device=D.device)
    idx = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=D.device)
    w = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=D.device)
    ws, nbytes = _workspace(ALGO_LEIDEN, g, p)
    nnz = ct.c_int64()
    d = g.desc()
    _check(lib().mgcd_aggregate(ct.byref(d), ct.byref(p), D.data_ptr(), m, int(symmetric),
                                off.data_ptr(), idx.data_ptr(), w.data_ptr(), ct.byref(nnz),
                                ws.data_ptr(), nbytes, _stream()))
    k = nnz.value
    return (off.cpu().numpy(), idx[:k].cpu().numpy(),
            w[:k].cpu().numpy().view(np.uint32))


def batched_workspace_bytes(algo: int, graphs, **kw) -> int:
    p = params(algo, **kw)
    return int(lib().mgcd_workspace_bytes_batched(algo, len(graphs), sum(g.n for g in graphs),
                                                  sum(g.nnz for g in graphs), ct.byref(p)))


def run_batched(algo: int, graphs, workspace=None, **kw):
    """Run LPA (ALGO_LPA) or Louvain (ALGO_LOUVAIN) on many device graphs together.
    `workspace` (optional): a device uint8 tensor of at least batched_workspace_bytes.
    Returns (labels per graph, stats per graph, total stats)."""
    import torch
    count = len(graphs)
    p = params(algo, **kw)
    dev = graphs[0].offsets.device if count else torch.device("cuda")
    outs = [torch.empty(max(g.n, 1), dtype=torch.int32, device=dev) for g in graphs]
    descs = (CSRDesc * max(count, 1))(*[g.desc() for g in graphs])
    ptrs = (ct.c_void_p * max(count, 1))(*[o.data_ptr() for o in outs])
    N = sum(g.n for g in graphs)
    E = sum(g.nnz for g in graphs)
    nbytes = int(lib().mgcd_workspace_bytes_batched(algo, count, N, E, ct.byref(p)))
    if workspace is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    else:
        ws = workspace
        nbytes = int(ws.numel())
    gst = (GraphStats * max(count, 1))()
    tot = Stats()
    name = "lpa_run_batched" if algo == ALGO_LPA else "louvain_run_batched"
    _check(getattr(lib(), name)(descs, count, ct.byref(p), ptrs, ws.data_ptr(), nbytes, gst,
                                ct.byref(tot), _stream()))
    return ([o[:g.n] for o, g in zip(outs, graphs)], [gst[i].asdict() for i in range(count)],
            tot.asdict())


class Server:
    """Continuous-batching server over the library's mgcd_server_* calls, in one device
    arena of `arena_bytes`.  stepped=False: `slots` worker streams run whole calls of
    `algo`, each in a block of the arena.  stepped=True: up to `slots` resident
    requests advance together, up to `sweeps_per_step` sweeps per step
    (mgcd_server_create_stepped; shared_bytes and sweeps_per_step as there, 0 = their
    defaults).  submit() returns a ticket; wait()
    returns (labels, stats, (t_submit, t_start, t_end)) with times in seconds since
    creation."""

    def __init__(self, algo: int, arena_bytes: int, slots: int = 4, device: str = "cuda",
                 stepped: bool = False, shared_bytes: int = 0, sweeps_per_step: int = 0, **kw):
        import torch
        self.algo = algo
        self.p = params(algo, **kw)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        self.device = self.arena.device
        self._h = ct.c_void_p()
        self._held = {}
        torch.cuda.current_stream().synchronize()  # the arena exists before the server uses it
        if stepped:
            _check(lib().mgcd_server_create_stepped(self.arena.data_ptr(), int(arena_bytes), int(shared_bytes),
                                                    int(slots), int(sweeps_per_step), algo, ct.byref(self.p),
                                                    ct.byref(self._h)))
        else:
            _check(lib().mgcd_server_create(self.arena.data_ptr(), int(arena_bytes), int(slots), algo,
                                            ct.byref(self.p), ct.byref(self._h)))

    def submit(self, g: DeviceGraph) -> int:
        import torch
        out = torch.empty(max(g.n, 1), dtype=torch.int32, device=self.device)
        torch.cuda.current_stream().synchronize()  # the graph and out exist before the server reads
        t = ct.c_int64()
        d = g.desc()
        _check(lib().mgcd_server_submit(self._h, ct.byref(d), out.data_ptr(), ct.byref(t)))
        self._held[t.value] = (g, out)
        return t.value

    def poll(self, ticket: int) -> str:
        s = ct.c_int32()
        _check(lib().mgcd_server_poll(self._h, ticket, ct.byref(s)))
        return ("waiting", "running", "done")[s.value]

    def wait(self, ticket: int):
        st = Stats()
        tm = (ct.c_double * 3)()
        rc = lib().mgcd_server_wait(self._h, ticket, ct.byref(st), tm)
        g, out = self._held.pop(ticket)
        _check(rc)
        return out[:g.n], st.asdict(), (tm[0], tm[1], tm[2])

    def info(self) -> dict:
        w, r = ct.c_int64(), ct.c_int64()
        u, pk = ct.c_size_t(), ct.c_size_t()
        _check(lib().mgcd_server_info(self._h, ct.byref(w), ct.byref(r), ct.byref(u), ct.byref(pk)))
        return {"waiting": w.value, "running": r.value, "bytes_in_use": u.value, "peak_bytes": pk.value}

    def step_stats(self) -> dict:
        st = StepStats()
        _check(lib().mgcd_server_step_stats(self._h, ct.byref(st)))
        return st.asdict()

    def close(self):
        if self._h:
            rc = lib().mgcd_server_destroy(self._h)
            self._h = ct.c_void_p()
            self._held.clear()
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
